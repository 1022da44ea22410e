"""General output modes through the C ABI against the FP64 oracle: the mirror
average with the reflected pair, the Y1 <= Y2 and fundamental domains with
full r planes, and Y1 slabs (one second scan per slab)."""
import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_BF16 = 1e-5


def _run(snap, w, y, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    dt = torch.float32 if snap.dtype == np.float32 else torch.float64
    dev = torch.from_numpy(np.ascontiguousarray(snap)).to(device="cuda", dtype=dt)
    res, prof = runner.run_slabs(dev, y, w.lx, w.lz, w.nu,
                                 dtype="f32" if snap.dtype == np.float32 else "f64", **kw)
    torch.cuda.synchronize()
    return [(p, [o.cpu().numpy() for o in out]) for p, out in res], prof


def _check(res, ref_fn, width, label, tol, expect_pairs=None):
    """res: [(pairs, maps)]; ref_fn(pairs) -> oracle [n][14][nz][nx]."""
    allp = []
    worst = np.zeros(14)
    scale = np.zeros(14)
    errs = np.zeros(14)
    for pairs, maps in res:
        allp += [tuple(p) for p in pairs]
        ref = ref_fn([tuple(p) for p in pairs])
        for t in range(14):
            r = ref[:, t, 0, 0] if t == 13 else ref[:, t, :, :width]
            g = maps[t]
            errs[t] = max(errs[t], np.abs(g - r).max())
            scale[t] = max(scale[t], np.abs(r).max())
    for t in range(14):
        worst[t] = errs[t] / (scale[t] if scale[t] > 0 else 1.0)
    print(label, " ".join(f"T{t + 1}={e:.1e}" for t, e in enumerate(worst)), flush=True)
    for t in range(14):
        assert worst[t] <= tol, f"{label}: T{t + 1} norm-wise error {worst[t]:.3e}"
    if expect_pairs is not None:
        assert allp == expect_pairs, label
    return worst


def test_mirror_fundamental_slabs_tiny():
    w = synth.workload("tiny", S=5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 31)
    ny = w.ny
    print("case mirror fundamental slab=3 tiny", flush=True)
    res, _ = _run(snap, w, y, mirror=1, domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=3, chunk=4)
    assert len(res) == 3   # rows 0..8 in slabs of 3
    expect = [(a, b) for a in range((ny - 1) // 2 + 1) for b in range(a, ny - a)]
    _check(res, lambda p: oracle.mirror_terms(snap, y, w.lx, w.lz, w.nu, p), w.nx,
           "mirror fundamental", TOL_FP64, expect)


def test_y1ley2_full_r_slabs_tiny():
    w = synth.workload("tiny", S=4)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 32)
    ny = w.ny
    print("case Y1<=Y2 full r slab=5 tiny", flush=True)
    res, _ = _run(snap, w, y, domain=gke.GKE_DOMAIN_Y1LEY2_FULLR, slab=5)
    expect = [(a, b) for a in range(ny) for b in range(a, ny)]
    _check(res, lambda p: oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, p), w.nx,
           "Y1<=Y2 full r", TOL_FP64, expect)


def test_allpairs_mirror_one_slab_tiny():
    w = synth.workload("tiny", S=3)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 33)
    ny = w.ny
    print("case all pairs half rx, mirror, one slab", flush=True)
    res, _ = _run(snap, w, y, mirror=1)
    assert len(res) == 1
    expect = [(a, b) for a in range(ny) for b in range(ny)]
    _check(res, lambda p: oracle.mirror_terms(snap, y, w.lx, w.lz, w.nu, p), w.nx // 2 + 1,
           "all pairs mirror", TOL_FP64, expect)


def test_mirror_fundamental_ragged_radix35():
    # 24 x 21 x 20: a 16-plane tile plus a 5-plane tail, radix 3 and 5
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=5, M=6, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 34)
    print("case mirror fundamental 24x21x20 slab=4 f32", flush=True)
    res, _ = _run(snap, w, y, mirror=1, domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=4,
                  chunk=2, pair_batch=50)
    _check(res, lambda p: oracle.mirror_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, p),
           w.nx, "mirror fundamental 24x21x20", TOL_FP64)


def test_mirror_fundamental_bf16x3():
    w = synth.workload("tiny", S=6, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 35)
    print("case mirror fundamental bf16x3", flush=True)
    res, _ = _run(snap, w, y, mirror=1, domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=4,
                  precision="bf16x3", chunk=4)
    _check(res, lambda p: oracle.mirror_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, p),
           w.nx, "mirror fundamental bf16x3", TOL_BF16)


def test_split_slabs_two_row_tiles():
    """Slabs of 20 rows at Ny = 65 (four column tiles): the inner slabs hold two
    row tiles, so the split rank-k works in whole 2 x 2 blocks of tile pairs with
    the operands staged in LDS; the last slab holds one row tile and takes the
    one-wave-per-pair form.  Both against the oracle."""
    w = synth.workload("tiny", ny=65, S=6, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 36)
    ny = w.ny
    print("case Y1<=Y2 full r slab=20 ny=65 bf16x3", flush=True)
    res, _ = _run(snap, w, y, domain=gke.GKE_DOMAIN_Y1LEY2_FULLR, slab=20, precision="bf16x3",
                  chunk=4)
    assert len(res) == 4
    expect = [(a, b) for a in range(ny) for b in range(a, ny)]
    _check(res, lambda p: oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, p),
           w.nx, "Y1<=Y2 full r slab=20 bf16x3", TOL_BF16, expect)


@pytest.mark.timeout(900)
def test_re200_grid_mirror_fundamental_first_slab():
    """The Re_tau=200 grid, mirror average, fundamental domain, slabs of 8 rows:
    the first slab (rows 0..7, the wall rows) against the oracle on sampled
    pairs; 12 FP64 snapshots."""
    w = synth.workload("re200", S=12)
    y = synth.y_grid(w)
    print("case re200 mirror fundamental slab 0: generating", flush=True)
    snap = synth.snapshots(w, 77)
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    dev = torch.from_numpy(snap).cuda()
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, chunk=12, mirror=1,
                      domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=8)
    assert r.slab_count() == 9
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    r.begin_stats()
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    print("case re200 mirror fundamental slab 0: GPU finalize", flush=True)
    maps = [m.cpu().numpy() for m in r.finalize(r.alloc_terms(slab=0))]
    pairs = [tuple(p) for p in r.slab_pairs(0)]
    r.close()
    ny = w.ny
    assert pairs[0] == (0, 0) and pairs[-1] == (7, ny - 8)
    pick = [0, 5, 130, len(pairs) // 2, len(pairs) - 1]
    sel = [pairs[i] for i in pick]
    print("case re200 mirror fundamental slab 0: oracle on", sel, flush=True)
    ref = oracle.mirror_terms(snap, y, w.lx, w.lz, w.nu, sel)
    for t in range(14):
        g = np.array([maps[t][i] for i in pick])
        rr = ref[:, t, 0, 0] if t == 13 else ref[:, t]
        e = np.abs(g - rr).max() / np.abs(rr).max()
        assert e <= TOL_FP64, (t, e)


@pytest.mark.timeout(900)
def test_re1000_grid_split_mirror_slab_sampled():
    """Config 5's shape: the Re_tau=1000 grid (512 x 257 x 384), FP32 inputs,
    split-BF16 update, mirror average, fundamental domain, slabs of 4 rows;
    the first slab (the wall rows) and one interior slab on sampled pairs
    against the oracle; 3 snapshots."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    w = synth.workload("re1000", S=3)
    y = synth.y_grid(w)
    print("case re1000 mirror fundamental slabs: generating", flush=True)
    snap = synth.snapshots(w, 91)
    dev = torch.from_numpy(snap).cuda()
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype="f32", precision="bf16x3",
                      chunk=4, pair_batch=1024, mirror=1,
                      domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=4)
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    r.begin_stats()
    got = {}
    for sl in (0, 20):
        if sl:
            r.begin_slab(sl)
        for s in range(w.S):
            r.accumulate_snapshot(dev[s])
        print("case re1000: finalize slab", sl, flush=True)
        maps = r.finalize(r.alloc_terms(slab=sl))
        pairs = [tuple(p) for p in r.slab_pairs(sl)]
        pick = [0, len(pairs) // 3, len(pairs) - 1]
        got[sl] = ([pairs[i] for i in pick], [m[pick].cpu().numpy() for m in maps])
        del maps
    r.close()
    for sl, (sel, maps) in got.items():
        print("case re1000: oracle on", sel, flush=True)
        ref = oracle.mirror_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, sel)
        errs = []
        for t in range(14):
            rr = ref[:, t, 0, 0] if t == 13 else ref[:, t]
            e = np.abs(maps[t] - rr).max() / np.abs(rr).max()
            errs.append(e)
        print(f"re1000 slab {sl}: " + " ".join(f"T{t + 1}={e:.1e}" for t, e in enumerate(errs)),
              flush=True)
        assert max(errs) <= TOL_BF16, (sl, errs)
