"""Output forms of gke_finalize through the C ABI: FP32 maps (each value
assembled in FP64 and rounded once) and host maps (written to a device staging
buffer, copied to pinned host memory on the library's copy stream, two
buffers in turn so that a slab's copies overlap the next slab's scan)."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
U32 = 2.0 ** -24   # unit roundoff of FP32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _slab_run(dev, w, y, out_dtype, host):
    from paper_1910_06409_amd import runner
    res, _ = runner.run_slabs(dev, y, w.lx, w.lz, w.nu, dtype="f32", mirror=1,
                              domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=3, chunk=2,
                              out_dtype=out_dtype, host=host)
    return [(p, [m.cpu().numpy().astype(np.float64) for m in maps]) for p, maps in res]


def test_slab_outputs_fp32_and_host():
    torch = _torch()
    w = synth.workload("tiny", S=3, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 71)
    dev = torch.from_numpy(snap).cuda()
    say("case slab outputs: device FP64, host FP64, host FP32, device FP32")
    d64 = _slab_run(dev, w, y, torch.float64, False)
    h64 = _slab_run(dev, w, y, torch.float64, True)
    h32 = _slab_run(dev, w, y, torch.float32, True)
    d32 = _slab_run(dev, w, y, torch.float32, False)
    assert len(d64) == len(h64) == len(h32) == 3
    s64 = snap.astype(np.float64)
    for (pa, a), (pb, b), (_, c), (_, e) in zip(d64, h64, h32, d32):
        assert np.array_equal(pa, pb)
        ref = oracle.mirror_terms(s64, y, w.lx, w.lz, w.nu, [tuple(int(v) for v in q) for q in pa])
        for t in range(14):
            assert np.array_equal(a[t], b[t]), t          # the same values through the host
            assert np.array_equal(c[t], e[t]), t          # FP32 on the host == on the device
            # FP32 maps are the FP64 maps rounded once
            assert np.all(np.abs(c[t] - a[t]) <= U32 * np.abs(a[t]) + 1e-300), t
            r = ref[:, 13, 0, 0] if t == 13 else ref[:, t]
            m = np.abs(r).max()
            assert np.abs(a[t] - r).max() <= TOL_FP64 * (m if m > 0 else 1.0), t
    say("  host == device, FP32 == FP64 rounded once, FP64 == oracle")


def test_all_pairs_fp32_and_host_outputs():
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=3, noise=0.5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 72)
    dev = torch.from_numpy(snap).cuda()
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, chunk=2, residual=True,
                      host_staging=2)
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    r.begin_stats()
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    say("case all-pairs outputs: device FP64, host FP64, host FP32 (with the residual)")
    ra = r.alloc_residual()
    a = r.finalize(r.alloc_terms(), residual=ra)
    b = r.alloc_terms(host=True)
    rb = torch.empty(tuple(ra.shape), dtype=torch.float64, pin_memory=True)
    r.finalize(b, residual=rb)
    c = r.alloc_terms(host=True, dtype=torch.float32)
    rc = torch.empty(tuple(ra.shape), dtype=torch.float32, pin_memory=True)
    r.finalize(c, residual=rc)
    r.wait_outputs()
    torch.cuda.synchronize()
    a = [x.cpu().numpy() for x in a]
    b = [x.numpy() for x in b]
    c = [x.numpy().astype(np.float64) for x in c]
    ra, rb, rc = ra.cpu().numpy(), rb.numpy(), rc.numpy().astype(np.float64)
    r.close()
    nu = w.nu
    D = oracle.fd5_matrix(y)
    wsum = np.abs(D).sum(axis=1)
    for t in range(14):
        assert np.array_equal(a[t], b[t]), t
        if t in (5, 10):
            # formed from the rounded <du^2>: |dT| <= nu (sum |w| over both indices) u max|T1|
            bound = 2 * nu * 2 * wsum.max() * U32 * np.abs(a[0]).max() + U32 * np.abs(a[t])
            assert np.all(np.abs(c[t] - a[t]) <= bound), t
        else:
            assert np.all(np.abs(c[t] - a[t]) <= U32 * np.abs(a[t]) + 1e-300), t
    assert np.array_equal(ra, rb)
    scale = max(np.abs(a[t]).max() for t in range(14))
    assert np.abs(rc - ra).max() <= 1e-5 * scale
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    nkx = w.nx // 2 + 1
    for t in range(13):
        g = np.array([a[t][p, q] for (p, q) in pairs])
        rr = ref[:, t, :, :nkx]
        assert np.abs(g - rr).max() <= TOL_FP64 * np.abs(rr).max(), t
    say("  host == device, FP32 within the rounding bounds, FP64 == oracle")


@pytest.mark.parametrize("host", [True, False])
def test_slab_callback_sees_complete_maps(host):
    """gke_set_slab_callback: one call per finalize, in slab order, and the
    maps the callback reads (host arrays, or device maps for device outputs)
    are already the final ones.  The host case reuses two sets of host arrays
    in turn, as a streaming caller does, so a late copy would show."""
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=3, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    dev = torch.from_numpy(synth.snapshots(w, 73)).cuda()
    ref = [[m.astype(np.float64) for m in maps] for _, maps in _slab_run(dev, w, y,
                                                                          torch.float64, False)]
    say(f"case slab callback, host outputs={host}")
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype="f32", chunk=2, mirror=1,
                      domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=3, device=dev.device,
                      host_staging=2 if host else 0)
    nslab = r.slab_count()
    npairs = [len(r.slab_pairs(sl)) for sl in range(nslab)]
    big = int(np.argmax(npairs))
    sets = [r.alloc_terms(slab=big, host=host) for _ in range(2 if host else 1)]
    seen = []
    cur = {}

    def note(slab):
        # runs on a HIP runtime thread once the slab's maps are complete
        n = npairs[slab]
        maps = sets[slab % len(sets)]
        if host:
            seen.append((slab, [maps[t][:n].numpy().copy() for t in range(14)]))
        else:
            seen.append((slab, None))
        cur["last"] = slab

    r.on_slab(note)
    for s in range(w.S):
        r.accumulate_snapshot(dev[s])
    r.begin_stats()
    dev_maps = []
    for sl in range(nslab):
        if sl > 0:
            r.begin_slab(sl)
        for s in range(w.S):
            r.accumulate_snapshot(dev[s])
        outs = sets[sl % len(sets)]
        r.finalize([o[:npairs[sl]] for o in outs])
        if not host:   # finalize returns after the device maps are written
            assert cur.get("last") == sl
            dev_maps.append([outs[t][:npairs[sl]].cpu().numpy().astype(np.float64)
                             for t in range(14)])
    r.wait_outputs()
    r.on_slab(None)
    r.close()
    assert [s for s, _ in seen] == list(range(nslab))
    got = [m for _, m in seen] if host else dev_maps
    for sl in range(nslab):
        for t in range(14):
            assert np.array_equal(got[sl][t].astype(np.float64), ref[sl][t]), (sl, t)
