"""The measured launch configurations at full size, checked on sampled pairs:

* the split-BF16 path as it is benched (Re_tau=200 grid, 512 FP32 snapshots,
  the automatic chunk: one FP32-accumulated rank-k batch), per-term error
  against the 1e-5 bar, printed term by term;
* the batched FP64 path (same grid, 512 FP32 snapshots, FP64 rank-k in the
  library's automatic chunks), against the 1e-10 bar;
* the Re_tau=1000 transform lengths (512 x 384) on a few planes, both paths.

The snapshots are built on the device by the seeded generator; the planes the
oracle needs (the sampled pairs' planes and their five-point stencils) are
copied back, so that both sides read the same input values."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_BF16 = 1e-5
PAIRS = [(3, 120), (64, 65), (128, 5)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_sampled(w, seed, pairs, **kw):
    """GPU maps of `pairs` and the oracle's, for the ensemble of workload w."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    dev = torch.device("cuda", 0)
    tdt = torch.float32 if w.dtype == "f32" else torch.float64
    say(f"  generating {w.S} snapshots of {w.name} on the device")
    snaps = torch.empty((w.S, 4, w.ny, w.nz, w.nx), dtype=tdt, device=dev)
    gen = synth.DeviceSnapshots(w, seed, dev)
    for s in range(w.S):
        gen(s, out=snaps[s])
    torch.cuda.synchronize()
    del gen
    y = synth.y_grid(w)
    held = oracle.stencil_closure(y, {j for p in pairs for j in p})
    host = snaps[:, :, held].cpu().numpy().astype(np.float64)
    say(f"  GPU run ({kw})")
    out, _ = runner.run_snapshots(snaps, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                                  precision=w.precision, **kw)
    torch.cuda.synchronize()
    g = [np.array([o[a, b].cpu().numpy() for (a, b) in pairs]) for o in out]
    del out, snaps
    torch.cuda.empty_cache()
    say(f"  oracle on {len(pairs)} pairs, {len(held)} planes, {w.S} snapshots")
    ref = oracle.pair_terms(host, y, w.lx, w.lz, w.nu, pairs, held=held)
    return g, ref


def term_errors(g, ref, nx, pointwise=None):
    """Norm-wise error max|T_gpu - T_oracle| / max|T_oracle| per term; with a
    list `pointwise`, also the pointwise relative error over the points where
    |T_oracle| > 1e-3 max|T_oracle| is appended to it per term."""
    nkx = nx // 2 + 1
    errs = []
    for t in range(14):
        r = ref[:, 13, 0, 0] if t == 13 else ref[:, t, :, :nkx]
        m = np.abs(r).max()
        d = np.abs(np.asarray(g[t]) - r)
        errs.append(float(d.max() / (m if m > 0 else 1.0)))
        if pointwise is not None:
            big = np.abs(r) > 1e-3 * m
            pointwise.append(float((d[big] / np.abs(r[big])).max()) if big.any() else 0.0)
    return errs


@pytest.mark.timeout(1200)
def test_re200_bf16_benched_configuration():
    w = synth.workload("re200_bf16")
    assert (w.S, w.dtype, w.precision) == (512, "f32", "bf16x3")
    say("case re200_bf16 as benched: 512 FP32 snapshots, automatic chunk")
    g, ref = run_sampled(w, 2024, PAIRS, chunk=0)
    pw = []
    errs = term_errors(g, ref, w.nx, pw)
    say("re200_bf16 per-term norm-wise error: " +
        " ".join(f"T{t + 1}={e:.2e}" for t, e in enumerate(errs)))
    say("re200_bf16 per-term pointwise error (|T| > 1e-3 max): " +
        " ".join(f"T{t + 1}={e:.2e}" for t, e in enumerate(pw)))
    for t, e in enumerate(errs):
        assert e <= TOL_BF16, f"T{t + 1}: {e:.3e}"


@pytest.mark.timeout(1200)
def test_re200_batched_fp64_config():
    w = synth.workload("re200_batched")
    assert (w.S, w.dtype, w.precision) == (512, "f32", "fp64")
    say("case re200_batched: 512 FP32 snapshots, FP64 rank-k, automatic chunk")
    g, ref = run_sampled(w, 2025, PAIRS, chunk=0)
    errs = term_errors(g, ref, w.nx)
    say("re200_batched per-term norm-wise error: " +
        " ".join(f"T{t + 1}={e:.2e}" for t, e in enumerate(errs)))
    for t, e in enumerate(errs):
        assert e <= TOL_FP64, f"T{t + 1}: {e:.3e}"


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,dtype,tol", [("fp64", "f64", TOL_FP64),
                                                 ("bf16x3", "f32", TOL_BF16)])
def test_re1000_transform_lengths(precision, dtype, tol):
    """The x and z lengths of the Re_tau=1000 grid (512 and 384, whose plans
    are compiled into the transform and finalize kernels) on a few planes and
    snapshots, with full-band inputs so that every bin carries data."""
    w = synth.workload("re1000", ny=13, S=6, noise=0.5, dtype=dtype, precision=precision)
    say(f"case re1000 lengths: {w.nx}x{w.ny}x{w.nz}, {w.S} {dtype} snapshots, {precision}")
    pairs = [(1, 11), (6, 6), (12, 0)]
    g, ref = run_sampled(w, 77, pairs, chunk=6)
    errs = term_errors(g, ref, w.nx)
    say("re1000 lengths per-term norm-wise error: " +
        " ".join(f"T{t + 1}={e:.2e}" for t, e in enumerate(errs)))
    for t, e in enumerate(errs):
        assert e <= tol, f"T{t + 1}: {e:.3e}"
