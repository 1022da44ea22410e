"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: norm-wise error max|gpu - oracle| / max|oracle| <= 1e-10 per term for
the FP64 path (inputs in FP64, or FP32 inputs read exactly by both sides).
The GPU writes the half plane rx >= 0 of every ordered pair; the oracle
computes the full periodic plane, whose columns p = 0..Nx/2 are compared.
"""
import sys

import numpy as np
import pytest

from oracle import direct, oracle
from paper_1910_06409_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(snap, w, y, **kw):
    torch = _torch()
    from paper_1910_06409_amd import runner
    dt = torch.float32 if snap.dtype == np.float32 else torch.float64
    dev = torch.from_numpy(np.ascontiguousarray(snap)).to(device="cuda", dtype=dt)
    out, prof = runner.run_snapshots(dev, y, w.lx, w.lz, w.nu,
                                     dtype="f32" if snap.dtype == np.float32 else "f64", **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy() if o is not None else None for o in out], prof


def compare(gpu_maps, ref, pairs, nx, label, tol=TOL_FP64):
    """ref: [npairs][14][nz][nx] full plane; gpu_maps[t]: [ny][ny][nz][nx/2+1]."""
    nkx = nx // 2 + 1
    worst = 0.0
    for t in range(14):
        if t == 13:
            g = np.array([[gpu_maps[13][a, b]] for (a, b) in pairs])
            r = ref[:, 13, 0, 0][:, None]
        else:
            g = np.array([gpu_maps[t][a, b] for (a, b) in pairs])
            r = ref[:, t, :, :nkx]
        m = np.abs(r).max()
        e = np.abs(g - r).max() / (m if m > 0 else 1.0)
        worst = max(worst, e)
        assert e <= tol, f"{label}: T{t + 1} norm-wise error {e:.3e} > {tol:.0e}"
    say(f"{label}: worst norm-wise error {worst:.3e}")
    return worst


def test_tiny_all_pairs_fp64(tiny):
    w, y, snap = tiny
    say("case tiny all pairs", snap.shape)
    g, prof = run_gpu(snap, w, y)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, "tiny")
    p_ref = oracle.step1(snap, y, w.lx, w.lz, w.nu)
    assert np.abs(prof - p_ref).max() <= 1e-12 * np.abs(p_ref).max()


def test_tiny_direct_sums_sampled(tiny):
    """GPU against the level-0 definitions at a few points."""
    w, y, snap = tiny
    g, _ = run_gpu(snap, w, y)
    mean, fl, S, eps, _ = direct.profiles(snap, y, w.lx, w.lz, w.nu)
    for (j1, j2, p, q) in [(0, 16, 3, 5), (7, 2, 8, 0), (11, 11, 1, 15), (4, 9, 0, 7)]:
        st = direct.point_stats(fl, mean, S, eps, j1, j2, p, q)
        for t, val in st.items():
            gv = g[t - 1][j1, j2] if t == 14 else g[t - 1][j1, j2, q, p]
            scale = np.abs(g[t - 1]).max()
            assert abs(gv - val) <= TOL_FP64 * scale, (j1, j2, p, q, t)


def test_odd_snapshots_multi_chunk():
    w = synth.workload("tiny", S=5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 21)
    say("case multi-chunk S=5 chunk=2")
    g, _ = run_gpu(snap, w, y, chunk=2)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, "chunk=2")


def test_radix_3_5_ragged_planes():
    # Nx = 24 (2^3 3), Nz = 20 (2^2 5), Ny = 21 (two plane tiles, ragged tail)
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=3, M=6)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 4)
    say("case 24x21x20")
    g, _ = run_gpu(snap, w, y, chunk=4, pair_batch=97)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, "24x21x20")


@pytest.mark.parametrize("ny,S,chunk", [
    (9, 2, 0),    # no full 16-plane tile: every pair goes to the remainder kernel
    (16, 3, 2),   # exactly one tile, no remainder plane; a last chunk of one snapshot
    (47, 1, 0),   # two tiles and the longest ragged tail (15 planes); one snapshot
    (33, 5, 2),   # one leftover plane: its pairs with the tiled planes are formed by
                  # the blocks of the last column tile; three chunks, the last partial
])
def test_plane_tiling_edge_cases(ny, S, chunk):
    w = synth.workload("tiny", ny=ny, S=S)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 100 + ny)
    say(f"case tiling Ny={ny} S={S} chunk={chunk}")
    g, _ = run_gpu(snap, w, y, chunk=chunk)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, f"Ny={ny}")


def test_fp32_inputs():
    w = synth.workload("tiny", dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 9)
    assert snap.dtype == np.float32
    say("case f32 inputs")
    g, _ = run_gpu(snap, w, y)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, "f32-in")


def test_set_means_and_refinalize():
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=6)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 13)
    prof_all = oracle.step1(snap, y, w.lx, w.lz, w.nu)
    dev = torch.from_numpy(snap).cuda()
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, chunk=4)
    r.set_means(*prof_all[:4])
    for s in range(3):
        r.accumulate_snapshot(dev[s])
    first = [t.cpu().numpy() if t is not None else None for t in r.finalize()]
    for s in range(3, 6):
        r.accumulate_snapshot(dev[s])
    second = [t.cpu().numpy() if t is not None else None for t in r.finalize()]
    r.close()
    pairs = oracle.all_pairs(w.ny)
    # profiles of the first three snapshots about the given (six-snapshot) means
    ref3 = oracle.pair_terms(snap[:3], y, w.lx, w.lz, w.nu, pairs,
                             prof=_onepoint(snap[:3], y, w, prof_all))
    compare(first, ref3, pairs, w.nx, "set_means 3 snapshots")
    ref6 = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs, prof=prof_all)
    compare(second, ref6, pairs, w.nx, "re-finalize 6 snapshots")


def test_set_means_split_path_gradient_energy():
    """Split path with the means given by the caller: the wall-normal gradient
    energy of the pseudo-dissipation then comes from the x pass's five-plane
    stencil of the fluctuations (the first scan, which otherwise sums it,
    did not run); T14 = -4 eps* and every other term against the oracle."""
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=6, dtype="f32", precision="bf16x3", noise=0.3)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 17)
    s64 = snap.astype(np.float64)
    prof_all = oracle.step1(s64, y, w.lx, w.lz, w.nu)
    dev = torch.from_numpy(snap).cuda()
    say("case split path, means from the caller")
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype="f32", precision="bf16x3",
                      chunk=4)
    r.set_means(*prof_all[:4])
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    out = [t.cpu().numpy() if t is not None else None for t in r.finalize()]
    r.close()
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(s64, y, w.lx, w.lz, w.nu, pairs, prof=prof_all)
    compare(out, ref, pairs, w.nx, "split path, set_means", tol=TOL_BF16)


def _onepoint(snap, y, w, prof_means):
    """Oracle one-point profiles of `snap` about externally given means."""
    return oracle.step1(snap, y, w.lx, w.lz, w.nu, means=prof_means[:4])


def test_scan_count_mismatch_is_refused():
    torch = _torch()
    from paper_1910_06409_amd import gke, runner
    w = synth.workload("tiny")
    y = synth.y_grid(w)
    snap = torch.from_numpy(synth.snapshots(w, 1)).cuda()
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu)
    for s in range(4):
        r.accumulate_snapshot(snap[s])
    r.begin_stats()
    for s in range(3):
        r.accumulate_snapshot(snap[s])
    with pytest.raises(gke.GkeError) as e:
        r.finalize()
    assert e.value.status == gke.GKE_ERR_STATE
    r.close()


@pytest.mark.timeout(900)
def test_re200_full_size_sampled_pairs():
    """The benchmark's workload (192 x 129 x 160, 100 FP64 snapshots, chunk 100)
    checked on sampled pairs against the oracle, and at sampled points against
    the direct sums of the definitions."""
    w = synth.workload("re200")
    y = synth.y_grid(w)
    say("case re200 full size: generating", w.S, "snapshots")
    snap = synth.snapshots(w, 2024)
    say("case re200 full size: GPU run")
    g, prof = run_gpu(snap, w, y, chunk=100)
    pairs = [(0, 0), (3, 120), (64, 64), (20, 90), (128, 5), (100, 101)]
    say("case re200 full size: oracle on", len(pairs), "pairs")
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    compare(g, ref, pairs, w.nx, "re200 sampled pairs")
    # level-0 definitions at sampled points (T1..T13 except the derivative terms)
    mean = snap.mean(axis=(0, 3, 4))
    S = direct.fd5_weights(y) @ mean[0]
    for (j1, j2, p, q) in [(2, 126, 17, 100), (60, 61, 96, 0), (33, 33, 0, 80)]:
        sel = [j1, j2]
        fl = snap[:, :, sel] - mean[None, :, sel, None, None]
        st = direct.point_stats(fl, mean[:, sel], S[sel], np.zeros(2), 0, 1, p, q)
        for t, val in st.items():
            if t == 14:
                continue
            scale = np.abs(g[t - 1]).max()   # norm-wise: the whole map
            assert abs(g[t - 1][j1, j2, q, p] - val) <= TOL_FP64 * scale, (j1, j2, p, q, t)
    say("re200 direct-sum points ok")


# ---------------------------------------------------------------------------
# split-BF16 three-term rank-k update (FP32 transforms, FP32 accumulation)
# ---------------------------------------------------------------------------
TOL_BF16 = 1e-5


def term_errors(gpu_maps, ref, pairs, nx):
    """Per-term norm-wise error max|gpu - oracle| / max|oracle| over the pairs."""
    nkx = nx // 2 + 1
    errs = []
    for t in range(14):
        if t == 13:
            g = np.array([[gpu_maps[13][a, b]] for (a, b) in pairs])
            r = ref[:, 13, 0, 0][:, None]
        else:
            g = np.array([gpu_maps[t][a, b] for (a, b) in pairs])
            r = ref[:, t, :, :nkx]
        m = np.abs(r).max()
        errs.append(float(np.abs(g - r).max() / (m if m > 0 else 1.0)))
    return errs


def check_bf16(g, ref, pairs, nx, label):
    errs = term_errors(g, ref, pairs, nx)
    say(f"{label}: per-term norm-wise error " +
        " ".join(f"T{t + 1}={e:.1e}" for t, e in enumerate(errs)))
    for t, e in enumerate(errs):
        assert e <= TOL_BF16, f"{label}: T{t + 1} norm-wise error {e:.3e} > {TOL_BF16:.0e}"
    return errs


def test_tiny_bf16x3(tiny):
    w, y, snap = tiny
    say("case tiny bf16x3")
    g, prof = run_gpu(snap, w, y, precision="bf16x3")
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    errs = check_bf16(g, ref, pairs, w.nx, "tiny bf16x3")
    # the split products are not exact: the error is above FP64 rounding
    assert max(errs) > 1e-12
    p_ref = oracle.step1(snap, y, w.lx, w.lz, w.nu)
    # means and point moments stay in FP64; eps takes its x, z part from the
    # split-product scale-energy spectra
    assert np.abs(prof[:11] - p_ref[:11]).max() <= 1e-12 * np.abs(p_ref).max()
    assert np.abs(prof[11] - p_ref[11]).max() <= TOL_BF16 * np.abs(p_ref[11]).max()


def test_bf16x3_ragged_multi_chunk_f32_inputs():
    # 24 x 21 x 20: radix 3 and 5, one full plane tile and a 5-plane tail;
    # 7 snapshots in chunks of 4 (the second chunk partly filled)
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=7, M=6, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 77)
    say("case bf16x3 24x21x20 S=7 chunk=4 f32")
    g, _ = run_gpu(snap, w, y, precision="bf16x3", chunk=4, pair_batch=61)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
    check_bf16(g, ref, pairs, w.nx, "bf16x3 24x21x20")


@pytest.mark.parametrize("S,chunk", [
    (27, 26),   # first chunk: one full group of 16 snapshots (four quads), then
                # two full quads and a quad of two snapshots; then a chunk of one
    (24, 24),   # one full group of 16 snapshots and a half group (two quads)
    (32, 32),   # exactly two full groups, no partial group or quad
])
def test_bf16x3_snapshot_quad_groups(S, chunk):
    # the split update sums 16 snapshots (four 32-byte records of four) per
    # matrix-core product; Ny = 33: two plane tiles and a remainder plane
    w = synth.workload("tiny", ny=33, S=S, M=6)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 100 + S)
    say(f"case bf16x3 quad groups Ny=33 S={S} chunk={chunk}")
    g, _ = run_gpu(snap, w, y, precision="bf16x3", chunk=chunk)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    check_bf16(g, ref, pairs, w.nx, f"bf16x3 S={S} chunk={chunk}")


@pytest.mark.timeout(600)
def test_bf16x3_512_snapshots_one_batch():
    # the split path's launch configuration at Re_tau = 200 (512 FP32
    # snapshots in one FP32-accumulated rank-k batch of 128 quads, the chunk
    # the automatic choice takes there) on a small grid, every pair: the FP32
    # sums over the longest batch stay within the split-BF16 bar
    w = synth.workload("tiny", nx=24, nz=20, ny=33, S=512, M=6, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 512)
    say("case bf16x3 Ny=33 S=512 chunk=512 f32")
    g, _ = run_gpu(snap, w, y, precision="bf16x3", chunk=512)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
    check_bf16(g, ref, pairs, w.nx, "bf16x3 S=512 chunk=512")


def test_bf16x3_remainder_only_grid():
    # Ny = 9: no full plane tile, every pair in the remainder kernel (packed
    # across wavenumbers on the split path); 3 snapshots, one partial quad
    w = synth.workload("tiny", ny=9, S=3)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 91)
    say("case bf16x3 Ny=9 S=3")
    g, _ = run_gpu(snap, w, y, precision="bf16x3")
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    check_bf16(g, ref, pairs, w.nx, "bf16x3 Ny=9")


@pytest.mark.timeout(900)
def test_re200_grid_bf16x3_sampled_pairs():
    """The Re_tau=200 grid with FP32 inputs and the split-BF16 update (64
    snapshots, the automatic chunk: one FP32-accumulated batch of 64) on
    sampled pairs against the oracle."""
    w = synth.workload("re200_bf16", S=64)
    y = synth.y_grid(w)
    say("case re200 grid bf16x3: generating", w.S, "snapshots")
    snap = synth.snapshots(w, 512)
    say("case re200 grid bf16x3: GPU run")
    g, _ = run_gpu(snap, w, y, precision="bf16x3", chunk=0)
    pairs = [(0, 0), (5, 127), (64, 64), (30, 95), (128, 1), (70, 71)]
    say("case re200 grid bf16x3: oracle on", len(pairs), "pairs")
    ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
    check_bf16(g, ref, pairs, w.nx, "re200 bf16x3 sampled pairs")
