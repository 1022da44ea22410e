"""The seeded synthetic channel generator (no method arithmetic): shapes,
determinism, the no-slip and divergence-free structure, and agreement of the
device-side builder with the host one."""
import numpy as np
import pytest

from conftest import nyquist_content
from paper_1910_06409_amd import synth


def test_deterministic_and_seeded(tiny):
    w, _, _ = tiny
    a = synth.snapshot(w, 5, 2)
    assert a.shape == (4, w.ny, w.nz, w.nx)
    assert np.array_equal(a, synth.snapshot(w, 5, 2))
    assert not np.array_equal(a, synth.snapshot(w, 5, 3))
    assert not np.array_equal(a, synth.snapshot(w, 6, 2))


def test_no_slip_and_mean(tiny):
    w, y, _ = tiny
    a = synth.snapshot(w, 1, 0)
    U = synth.mean_profile(w, y)
    # velocities vanish at the walls; u~ carries the mean profile
    assert np.abs(a[:3, 0]).max() < 1e-12 and np.abs(a[:3, -1]).max() < 1e-12
    assert abs(a[0].mean(axis=(1, 2)) - U).max() < 0.2


def test_divergence_free_spectrally():
    # i alpha u^ + d(v^)/dy + i beta w^ = 0 per wavenumber, with the exact y
    # derivative of v^ = F (i beta psi_x - i alpha psi_z) from the expansion
    w = synth.workload("tiny", ny=33)
    y = synth.y_grid(w)
    f, fp = synth._envelope(w, y)
    T, dT = synth._cheb(w.M, y)
    alpha, beta, band, _ = synth._wavenumbers(w)
    iz, ix = np.nonzero(band)
    cm = synth._coefficients(w, 3, 0)
    co = synth._assemble(np, w, cm, T, dT, f, fp, alpha[ix][None, :], beta[iz][None, :])
    nb = iz.size
    ps = (T @ cm).reshape(w.ny, 4, nb)
    dps = (dT @ cm).reshape(w.ny, 4, nb)
    a, b = alpha[ix][None, :], beta[iz][None, :]
    F, Fp = f[:, None], fp[:, None]
    dv = 1j * b * (Fp * ps[:, 0] + F * dps[:, 0]) - 1j * a * (Fp * ps[:, 2] + F * dps[:, 2])
    div = 1j * a * co[0] + dv + 1j * b * co[2]
    assert np.abs(div).max() <= 1e-12 * np.abs(co[:3]).max() * max(alpha.max(), beta.max())


@pytest.mark.parametrize("name", ["tiny", "re200_bf16"])
def test_device_builder_matches_host(name):
    torch = pytest.importorskip("torch")
    w = synth.workload(name)
    g = synth.DeviceSnapshots(w, 11, torch.device("cpu"))
    for s in (0, 4):
        a = synth.snapshot(w, 11, s)
        b = g(s).numpy()
        assert b.dtype == a.dtype
        tol = 1e-13 if a.dtype == np.float64 else 1e-6
        assert np.abs(a.astype(np.float64) - b).max() <= tol * np.abs(a).max()



def test_band_limited_default_has_no_nyquist_content(tiny):
    w, _, snap = tiny
    assert nyquist_content(snap[:, :3, 1:-1]) < 1e-28


@pytest.mark.parametrize("kw", [dict(), dict(nx=24, nz=20, ny=21, M=6)])
def test_full_band_inputs_fill_every_bin(kw):
    w = synth.workload("tiny", noise=0.5, S=2, **kw)
    snap = synth.snapshots(w, 3)
    # every field, every plane (walls included), both Nyquist lines carry energy
    # of the order of a white spectrum's share (1/Nx and 1/Nz of the plane)
    share = min(1.0 / w.nx, 1.0 / w.nz)
    assert nyquist_content(snap) > 0.05 * share
    # every single bin is non-zero
    X = np.fft.rfft2(snap - snap.mean(axis=(-2, -1), keepdims=True), axes=(-2, -1))
    X[..., 0, 0] = 1.0
    assert np.abs(X).min() > 1e-9
    # deterministic, and noise = 0 gives back the band-limited snapshot
    assert np.array_equal(snap[1], synth.snapshot(w, 3, 1))
    w0 = synth.workload("tiny", S=2, **kw)
    assert not np.array_equal(snap[1], synth.snapshot(w0, 3, 1))
    assert np.abs(snap[1] - synth.snapshot(w0, 3, 1)).max() < 10 * w.noise * w.rms_u


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_device_drawn_generator_statistics(dtype):
    """The device-drawn generator (for ensembles regenerated per scan) has the
    host generator's plane-mean profile and, over an ensemble, its fluctuation
    rms per plane; it is seeded, and writes in the snapshot's dtype."""
    import torch
    w = synth.workload("tiny", dtype=dtype)
    cpu = torch.device("cpu")
    g = synth.FastDeviceSnapshots(w, 7, cpu)
    d = synth.DeviceSnapshots(w, 7, cpu)

    def rms(x):
        x = x.double()
        return torch.sqrt(((x - x.mean(dim=(-2, -1), keepdim=True)) ** 2).mean(dim=(-2, -1))).numpy()

    S = 12
    rf = np.mean([rms(g(s)) for s in range(S)], axis=0)[:, 1:-1]
    rd = np.mean([rms(d(s)) for s in range(S)], axis=0)[:, 1:-1]
    assert np.all(np.abs(rf.mean(axis=1) / rd.mean(axis=1) - 1) < 0.15)
    a, b = g(0), d(0)
    assert a.dtype == (torch.float32 if dtype == "f32" else torch.float64)
    tol = 1e-6 if dtype == "f32" else 1e-14
    assert float((a[0].double().mean(dim=(-2, -1)) - b[0].double().mean(dim=(-2, -1))).abs().max()) < tol
    out = torch.empty_like(a)
    g(0, out=out)
    assert torch.equal(out, a)
    assert not torch.equal(g(1), a)
