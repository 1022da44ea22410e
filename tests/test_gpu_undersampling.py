"""rx / rz undersampling with two thresholds (Section "Undersampling and
parallelisation") through the C ABI: the stored maps are the oracle's
full-resolution maps at the kept separations -- the derivatives (spectral
T4, T8 and the residual's r-divergence, five-point T6, T11) are taken before
the points are dropped -- in the all-pairs mode and in the mirror /
fundamental-domain slab mode."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_BF16 = 1e-5
US_X = (2, 5, 2, 3)   # rx: full below 2, every 2nd below 5, every 3rd beyond
US_Z = (3, 6, 2, 4)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _err(g, r):
    m = np.abs(r).max()
    return float(np.abs(g - r).max() / (m if m > 0 else 1.0))


@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("bf16x3", TOL_BF16)])
def test_undersampled_all_pairs_and_residual(precision, tol):
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=3, noise=0.5, dtype="f32" if precision == "bf16x3" else "f64")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 61)
    rx = oracle.sample_indices(w.nx, *US_X, True)
    rz = oracle.sample_indices(w.nz, *US_Z, False)
    assert len(rx) < w.nx // 2 + 1 and len(rz) < w.nz
    say(f"case undersampled all pairs {precision}: {len(rz)} x {len(rx)} of {w.nz} x {w.nx // 2 + 1}")
    dev = torch.from_numpy(snap).cuda()
    res = runner.run_snapshots(dev, y, w.lx, w.lz, w.nu, dtype=w.dtype, precision=precision,
                               undersample={0: US_X, 1: US_Z}, residual=precision == "fp64")
    torch.cuda.synchronize()
    out = [o.cpu().numpy() for o in res[0]]
    assert out[0].shape == (w.ny, w.ny, len(rz), len(rx))
    pairs = oracle.all_pairs(w.ny)
    s64 = snap.astype(np.float64)
    ref = oracle.pair_terms(s64, y, w.lx, w.lz, w.nu, pairs)
    ix = np.ix_(rz, rx)
    errs = []
    for t in range(14):
        if t == 13:
            g = np.array([out[13][a, b] for (a, b) in pairs])
            r = ref[:, 13, 0, 0]
        else:
            g = np.array([out[t][a, b] for (a, b) in pairs])
            r = np.array([ref[k, t][ix] for k in range(len(pairs))])
        errs.append(_err(g, r))
    say("  " + " ".join(f"T{t + 1}={e:.1e}" for t, e in enumerate(errs)))
    assert max(errs) <= tol
    if precision == "fp64":
        resid = res[2].cpu().numpy()
        rref, parts = oracle.residual(s64, y, w.lx, w.lz, w.nu, pairs, parts=True)
        g = np.array([resid[a, b] for (a, b) in pairs])
        r = np.array([rref[k][ix] for k in range(len(pairs))])
        e = np.abs(g - r).max() / max(np.abs(parts).max(), np.abs(rref).max())
        say(f"  residual {e:.1e}")
        assert e <= TOL_FP64


def test_undersampled_mirror_fundamental_slabs():
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=4, M=6, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 62)
    us_x, us_z = (3, 8, 2, 4), (2, 6, 3, 4)
    rx = oracle.sample_indices(w.nx, *us_x, False)
    rz = oracle.sample_indices(w.nz, *us_z, False)
    say(f"case undersampled mirror fundamental: {len(rz)} x {len(rx)} of {w.nz} x {w.nx}")
    dev = torch.from_numpy(snap).cuda()
    res, _ = runner.run_slabs(dev, y, w.lx, w.lz, w.nu, dtype="f32", mirror=1,
                              domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=4, chunk=2,
                              undersample={0: us_x, 1: us_z})
    torch.cuda.synchronize()
    s64 = snap.astype(np.float64)
    ix = np.ix_(rz, rx)
    err = np.zeros(14)
    scale = np.zeros(14)
    for pairs, maps in res:
        pl = [tuple(int(v) for v in p) for p in pairs]
        ref = oracle.mirror_terms(s64, y, w.lx, w.lz, w.nu, pl)
        for t in range(14):
            gm = maps[t].cpu().numpy()
            if t == 13:
                r = ref[:, 13, 0, 0]
            else:
                assert gm.shape == (len(pl), len(rz), len(rx))
                r = np.array([ref[k, t][ix] for k in range(len(pl))])
            err[t] = max(err[t], np.abs(gm - r).max())
            scale[t] = max(scale[t], np.abs(r).max())
    e = err / np.where(scale > 0, scale, 1.0)
    say("  " + " ".join(f"T{t + 1}={v:.1e}" for t, v in enumerate(e)))
    assert (e <= TOL_FP64).all()
