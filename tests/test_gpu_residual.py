"""The budget residual written by gke_finalize (all-pairs mode) against the
oracle's residual (eq. GKE-conservative): spectral r_x, r_z divergence of the
scale fluxes, five-point Y1/Y2 derivatives of the r_y and Y fluxes, minus the
source; on full-band inputs, every ordered pair, and on sampled pairs of the
Re_tau=200 grid."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_BF16 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(snap, w, y, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    f32 = snap.dtype == np.float32
    dev = torch.from_numpy(np.ascontiguousarray(snap)).to(
        device="cuda", dtype=torch.float32 if f32 else torch.float64)
    out, prof, res = runner.run_snapshots(dev, y, w.lx, w.lz, w.nu,
                                          dtype="f32" if f32 else "f64", residual=True, **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], res.cpu().numpy()


def _check(res, ref, pairs, nx, label, tol):
    """ref = (residual, parts) from the oracle.  Norm-wise error of the
    residual: max|Res_gpu - Res| over the larger of max|Res| and the largest
    of the budget's parts (the residual is a difference of comparable parts;
    the paper judges it against production and dissipation)."""
    ref, parts = ref
    nkx = nx // 2 + 1
    g = np.array([res[a, b] for (a, b) in pairs])
    r = ref[:, :, :nkx]
    scale = max(np.abs(parts[..., :nkx]).max(), np.abs(r).max())
    e = np.abs(g - r).max() / scale
    say(f"{label}: residual error {e:.2e} (scale {scale:.3e}, max |Res| {np.abs(r).max():.3e})")
    assert e <= tol, f"{label}: {e:.3e}"
    return e


SIGMA_R = np.array([+1, -1, -1, -1, -1, -1, -1, -1, +1, +1, +1, +1, +1, +1], dtype=np.float64)


def full_plane_maps(maps, ny, nz, nx):
    """The GPU's all-pairs half-plane maps as full periodic planes: columns
    p > Nx/2 of pair (Y1, Y2) are those of (Y2, Y1) at -r with the sign of
    each term under the exchange; T14 is constant over the plane."""
    nkx = nx // 2 + 1
    out = np.zeros((ny, ny, 14, nz, nx))
    qm = (-np.arange(nz)) % nz
    for t in range(13):
        h = maps[t]                               # [Y1][Y2][nz][nkx]
        out[:, :, t, :, :nkx] = h
        hm = np.swapaxes(h, 0, 1)[:, :, qm, :]    # (Y2, Y1) at -rz
        for p in range(nkx, nx):
            out[:, :, t, :, p] = SIGMA_R[t] * hm[:, :, :, nx - p]
    out[:, :, 13] = maps[13][:, :, None, None]
    return out


@pytest.mark.parametrize("label,kw,chunk", [
    ("16x17x16", dict(), 0),
    ("24x21x20", dict(nx=24, nz=20, ny=21, M=6), 2),
])
def test_residual_full_band_fp64_all_pairs(label, kw, chunk):
    w = synth.workload("tiny", S=3, noise=0.5, **kw)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 51)
    say(f"case residual fp64 {label}")
    maps, res = _run(snap, w, y, chunk=chunk, pair_batch=97 if chunk else 0)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.residual(snap, y, w.lx, w.lz, w.nu, pairs, parts=True)
    _check(res, ref, pairs, w.nx, f"residual fp64 {label}", TOL_FP64)


def test_residual_band_limited_bf16x3():
    """Split-BF16 path: (1) the residual the GPU writes agrees with the oracle's
    residual operator applied to the GPU's own maps to the split bar (the
    operator itself is checked to the FP64 bar on the FP64 path above; here the
    rx < 0 half of each map is rebuilt from the exchanged pair, which the split
    update accumulates separately on the diagonal plane tiles, so the two
    halves obey the exchange symmetry only to the split precision); (2)
    against the oracle end to end the error is that of the maps (each within
    the split bar) amplified by the r and Y derivatives, held to 10x the split
    bar."""
    w = synth.workload("tiny", S=5, dtype="f32")
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 52)
    say("case residual bf16x3 tiny")
    maps, res = _run(snap, w, y, precision="bf16x3")
    pairs = oracle.all_pairs(w.ny)
    full = full_plane_maps(maps, w.ny, w.nz, w.nx)
    own = oracle.residual_of_maps(lambda p: full[p[0], p[1]], y, w.lx, w.lz, pairs, parts=True)
    _check(res, own, pairs, w.nx, "residual operator on the split maps", TOL_BF16)
    ref = oracle.residual(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs, parts=True)
    _check(res, ref, pairs, w.nx, "residual bf16x3 tiny end to end", 10 * TOL_BF16)


@pytest.mark.timeout(900)
def test_residual_re200_grid_sampled_pairs():
    w = synth.workload("re200", S=8)
    y = synth.y_grid(w)
    pairs = [(3, 120), (64, 65)]
    say("case residual re200 grid, 8 snapshots: generating")
    snap = synth.snapshots(w, 53)
    maps, res = _run(snap, w, y, chunk=8)
    held = oracle.stencil_closure(y, oracle.stencil_closure(y, {j for p in pairs for j in p}))
    say(f"  oracle on {len(held)} planes")
    ref = oracle.residual(np.ascontiguousarray(snap[:, :, held]), y, w.lx, w.lz, w.nu, pairs,
                          held=held, parts=True)
    _check(res, ref, pairs, w.nx, "residual re200 sampled", TOL_FP64)
