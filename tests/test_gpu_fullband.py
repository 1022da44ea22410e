"""Parity on full-band inputs: white noise added to every field, so that every
(kx, kz) bin of every plane, the Nyquist bins included, carries content and
every bin of every term spectrum is compared against the oracle.  This covers
what band-limited inputs leave at zero: the half-spectrum weights of eps, the
zero multipliers of the spectral r-derivatives at the Nyquist wavenumbers,
the Hermitian extension of the kx = Nx/2 bin in the inverse real transform,
and every transform, rank-k and finalize step at |k| > N/3."""
import sys

import numpy as np
import pytest

from conftest import nyquist_content
from oracle import oracle
from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_BF16 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(snap, w, y, **kw):
    torch = _torch()
    from paper_1910_06409_amd import runner
    f32 = snap.dtype == np.float32
    dev = torch.from_numpy(np.ascontiguousarray(snap)).to(
        device="cuda", dtype=torch.float32 if f32 else torch.float64)
    out, prof = runner.run_snapshots(dev, y, w.lx, w.lz, w.nu, dtype="f32" if f32 else "f64",
                                     **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], prof


def _errors(g, ref, pairs, nx):
    nkx = nx // 2 + 1
    errs = []
    for t in range(14):
        if t == 13:
            gv = np.array([[g[13][a, b]] for (a, b) in pairs])
            r = ref[:, 13, 0, 0][:, None]
        else:
            gv = np.array([g[t][a, b] for (a, b) in pairs])
            r = ref[:, t, :, :nkx]
        m = np.abs(r).max()
        errs.append(float(np.abs(gv - r).max() / (m if m > 0 else 1.0)))
    return errs


def _check(g, ref, pairs, nx, label, tol):
    errs = _errors(g, ref, pairs, nx)
    say(f"{label}: " + " ".join(f"T{t + 1}={e:.1e}" for t, e in enumerate(errs)))
    for t, e in enumerate(errs):
        assert e <= tol, f"{label}: T{t + 1} norm-wise error {e:.3e} > {tol:.0e}"


def _nyquist_maps_nonzero(g, nx, nz):
    """The term maps carry energy at the Nyquist separations' wavenumbers:
    the rz spectrum of <du^2> at kz = Nz/2 is not zero."""
    t1 = g[0]
    spec = np.fft.fft(t1 - t1.mean(axis=(-2, -1), keepdims=True), axis=-2)
    assert np.abs(spec[..., nz // 2, :]).max() > 1e-8 * np.abs(spec).max()


CASES = [
    ("16x17x16", dict(), 0),
    # radix 3 and 5, one 16-plane tile and a five-plane tail, chunks of 2,
    # pair batches in finalize
    ("24x21x20", dict(nx=24, nz=20, ny=21, M=6), 2),
]


@pytest.mark.parametrize("label,kw,chunk", CASES)
def test_full_band_fp64_all_pairs(label, kw, chunk):
    w = synth.workload("tiny", S=3, noise=0.5, **kw)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 41)
    assert nyquist_content(snap) > 0.05 / max(w.nx, w.nz)
    say(f"case full-band fp64 {label}")
    g, prof = _run(snap, w, y, chunk=chunk, pair_batch=97 if chunk else 0)
    _nyquist_maps_nonzero(g, w.nx, w.nz)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs)
    _check(g, ref, pairs, w.nx, f"full-band fp64 {label}", TOL_FP64)
    p_ref = oracle.step1(snap, y, w.lx, w.lz, w.nu)
    assert np.abs(prof - p_ref).max() <= 1e-12 * np.abs(p_ref).max()


@pytest.mark.parametrize("label,kw,chunk", CASES)
def test_full_band_bf16x3_all_pairs(label, kw, chunk):
    w = synth.workload("tiny", S=5, noise=0.5, dtype="f32", **kw)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 42)
    assert nyquist_content(snap) > 0.05 / max(w.nx, w.nz)
    say(f"case full-band bf16x3 {label}")
    g, prof = _run(snap, w, y, precision="bf16x3", chunk=chunk or 0)
    pairs = oracle.all_pairs(w.ny)
    ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
    _check(g, ref, pairs, w.nx, f"full-band bf16x3 {label}", TOL_BF16)
    p_ref = oracle.step1(snap.astype(np.float64), y, w.lx, w.lz, w.nu)
    assert np.abs(prof[:11] - p_ref[:11]).max() <= 1e-12 * np.abs(p_ref).max()
    assert np.abs(prof[11] - p_ref[11]).max() <= TOL_BF16 * np.abs(p_ref[11]).max()


def test_full_band_mirror_fundamental_slabs():
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=4, M=6, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 43)
    assert nyquist_content(snap) > 0.05 / max(w.nx, w.nz)
    say("case full-band mirror fundamental 24x21x20 slab=4")
    dev = torch.from_numpy(snap).cuda()
    res, _ = runner.run_slabs(dev, y, w.lx, w.lz, w.nu, dtype="f32", mirror=1,
                              domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=4, chunk=2,
                              pair_batch=50)
    torch.cuda.synchronize()
    s64 = snap.astype(np.float64)
    err = np.zeros(14)
    scale = np.zeros(14)
    n = 0
    for pairs, maps in res:
        pl = [tuple(int(v) for v in p) for p in pairs]
        n += len(pl)
        ref = oracle.mirror_terms(s64, y, w.lx, w.lz, w.nu, pl)
        for t in range(14):
            r = ref[:, 13, 0, 0] if t == 13 else ref[:, t]
            gm = maps[t].cpu().numpy()
            err[t] = max(err[t], np.abs(gm - r).max())
            scale[t] = max(scale[t], np.abs(r).max())
    ny = w.ny
    assert n == sum(ny - 2 * a for a in range((ny - 1) // 2 + 1))
    e = err / np.where(scale > 0, scale, 1.0)
    say("full-band mirror fundamental: " + " ".join(f"T{t + 1}={v:.1e}" for t, v in enumerate(e)))
    assert (e <= TOL_FP64).all(), e
