"""Seeded synthetic channel-flow snapshots.

Input generation only: this module holds none of the GKE arithmetic (no
fluctuations, products, cross-spectra or term assembly).  It is the one
module that both the HIP path's tests/benchmark and the CPU oracle draw their
inputs from.

The paper's DNS databases (Section "Computational details": Re_tau=200 with
Lx=4*pi*h, Lz=2*pi*h; Re_tau=1000 on the same box) are not available, so the
workloads below are synthetic stand-ins with the same geometry, grids
stretched towards the walls, and near-wall-peaked, divergence-free,
no-slip fluctuations:

* u' = curl(f(y) psi): psi is a random vector potential made of Fourier modes
  in (x, z) times Chebyshev polynomials T_m(y), m < M, with complex Gaussian
  coefficients scaled by (1 + alpha^2 + beta^2)^(-5/6); f = f' = 0 at the
  walls gives no-slip, and the curl makes the field solenoidal.
* Modes are band-limited to |kx| <= Nx/3, |kz| <= Nz/3 (the grid then
  resolves every quadratic product, as for dealiased DNS data) and the (0,0)
  mode is absent.
* p' has the same amplitude law and no envelope.
* A mean profile U(y) (laminar for the tiny case, a Reichardt wall law with
  U(0)=1 otherwise) is added to u.
* One RNG stream per snapshot: SeedSequence([seed, s]).
* Optional full-band content (noise > 0): seeded white noise of relative
  amplitude `noise` added to u', v', w', p' at every grid point (stream
  SeedSequence([seed, s, 1])).  It is neither divergence-free nor
  band-limited: every (kx, kz) bin of every plane carries content, the
  Nyquist bins included, so that no part of the spectrum is zero by
  construction.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, replace

import numpy as np
import scipy.fft


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    nu: float
    S: int
    grid: str            # "cgl" or "tanh"
    gamma: float         # tanh stretching
    M: int               # Chebyshev modes in y
    envelope: str        # "quartic" or "nearwall"
    mean: str            # "laminar" or "reichardt"
    re_tau: float
    dtype: str           # "f64" or "f32" input storage
    precision: str       # "fp64" or "bf16x3" rank-k arithmetic
    spectrum_scale: float = 1.0   # k -> k/spectrum_scale in the amplitude law
    rms_u: float = 0.15           # target peak rms of the velocity fluctuation
    rms_p: float = 0.10           # target peak rms of the pressure fluctuation
    noise: float = 0.0            # relative amplitude of added full-band white noise

    @property
    def nk(self) -> int:
        return (self.nx // 2 + 1) * self.nz

    @property
    def points_out(self) -> int:
        """(Y1, Y2, rx>=0, rz) points of the all-pairs half-plane output."""
        return self.ny * self.ny * (self.nx // 2 + 1) * self.nz


_PI = math.pi
WORKLOADS = {
    # Tiny channel, FP64: 16 x 17 x 16 CGL grid, 4 snapshots.
    "tiny": Workload("tiny", 16, 17, 16, 2 * _PI, _PI, 1 / 200, 4, "cgl", 0.0,
                     8, "quartic", "laminar", 0.0, "f64", "fp64", rms_u=0.1),
    # Re_tau=200-shaped grid, FP64 inputs and FP64 rank-k, 100 snapshots.
    "re200": Workload("re200", 192, 129, 160, 4 * _PI, 2 * _PI, 1 / 200, 100,
                      "tanh", 2.0, 24, "nearwall", "reichardt", 200.0, "f64", "fp64"),
    # Same grid, 512 FP32 snapshots, chunked/batched FP64 rank-k.
    "re200_batched": Workload("re200_batched", 192, 129, 160, 4 * _PI, 2 * _PI, 1 / 200,
                              512, "tanh", 2.0, 24, "nearwall", "reichardt", 200.0,
                              "f32", "fp64"),
    # Same grid, 512 FP32 snapshots, split-BF16 three-term rank-k.
    "re200_bf16": Workload("re200_bf16", 192, 129, 160, 4 * _PI, 2 * _PI, 1 / 200,
                           512, "tanh", 2.0, 24, "nearwall", "reichardt", 200.0,
                           "f32", "bf16x3"),
    # Re_tau=1000-shaped grid, 256 FP32 snapshots, spectra extended to higher k.
    "re1000": Workload("re1000", 512, 257, 384, 4 * _PI, 2 * _PI, 1 / 1000, 256,
                       "tanh", 2.5, 48, "nearwall", "reichardt", 1000.0, "f32",
                       "bf16x3", spectrum_scale=2.0),
}


def workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


# ----------------------------------------------------------------------------
# grids and profiles
# ----------------------------------------------------------------------------
def y_grid(w: Workload) -> np.ndarray:
    j = np.arange(w.ny, dtype=np.float64)
    if w.grid == "cgl":
        y = -np.cos(np.pi * j / (w.ny - 1))
    elif w.grid == "tanh":
        xi = -1.0 + 2.0 * j / (w.ny - 1)
        y = np.tanh(w.gamma * xi) / np.tanh(w.gamma)
    else:
        raise ValueError(w.grid)
    y[0], y[-1] = -1.0, 1.0
    if w.ny % 2 == 1:
        y[w.ny // 2] = 0.0
    # exact mirror symmetry of the node set
    y = 0.5 * (y - y[::-1])
    return y


def mean_profile(w: Workload, y: np.ndarray) -> np.ndarray:
    if w.mean == "laminar":
        return 1.0 - y * y
    kappa = 0.41
    yp = (1.0 - np.abs(y)) * w.re_tau
    up = (np.log1p(kappa * yp) / kappa
          + 7.8 * (1.0 - np.exp(-yp / 11.0) - (yp / 11.0) * np.exp(-yp / 3.0)))
    yc = w.re_tau
    uc = (np.log1p(kappa * yc) / kappa
          + 7.8 * (1.0 - np.exp(-yc / 11.0) - (yc / 11.0) * np.exp(-yc / 3.0)))
    return up / uc


def _envelope(w: Workload, y: np.ndarray):
    """f(y) and f'(y); f = f' = 0 at y = +-1."""
    a = 1.0 - y * y
    if w.envelope == "quartic":
        return a * a, -4.0 * y * a
    c0 = 0.001
    g = c0 + y ** 16
    f = a * a * g
    fp = -4.0 * y * a * g + a * a * 16.0 * y ** 15
    return f, fp


def _cheb(M: int, y: np.ndarray):
    """T_m(y) and T_m'(y) for m < M, shape (ny, M)."""
    ny = y.size
    T = np.zeros((ny, M))
    dT = np.zeros((ny, M))
    T[:, 0] = 1.0
    if M > 1:
        T[:, 1] = y
        dT[:, 1] = 1.0
    for m in range(2, M):
        T[:, m] = 2.0 * y * T[:, m - 1] - T[:, m - 2]
        dT[:, m] = 2.0 * T[:, m - 1] + 2.0 * y * dT[:, m - 1] - dT[:, m - 2]
    return T, dT


def _wavenumbers(w: Workload):
    nkx = w.nx // 2 + 1
    kx = np.arange(nkx)
    kz = np.fft.fftfreq(w.nz, d=1.0 / w.nz).astype(np.int64)
    alpha = 2.0 * np.pi * kx / w.lx
    beta = 2.0 * np.pi * kz / w.lz
    band = (np.abs(kz)[:, None] <= w.nz // 3) & (kx[None, :] <= w.nx // 3)
    band[0, 0] = False
    k2 = (alpha[None, :] ** 2 + beta[:, None] ** 2) / (w.spectrum_scale ** 2)
    amp = np.where(band, (1.0 + k2) ** (-5.0 / 6.0), 0.0)
    return alpha, beta, band, amp


# ----------------------------------------------------------------------------
# snapshots
# ----------------------------------------------------------------------------
_SCALE_CACHE: dict = {}


def _coefficients(w: Workload, seed: int, s: int) -> np.ndarray:
    """Seeded random stream-function and pressure coefficients [M][4 nb]
    (Chebyshev mode x (field, band wavenumber)), amplitude law applied."""
    _, _, band, amp = _wavenumbers(w)
    iz, ix = np.nonzero(band)
    nb = iz.size
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(s)]))
    c = rng.standard_normal((4, w.M, nb)) + 1j * rng.standard_normal((4, w.M, nb))
    c *= amp[iz, ix][None, None, :]
    return c.transpose(1, 0, 2).reshape(w.M, 4 * nb)


def _assemble(xp, w: Workload, cm, T, dT, f, fp, a, b):
    """Velocity (curl of the enveloped stream function) and pressure
    coefficients on the band wavenumbers, [4][ny][nb]; xp is numpy or torch."""
    nb = a.shape[-1]
    ps = (T @ cm).reshape(w.ny, 4, nb)
    dps = (dT @ cm).reshape(w.ny, 4, nb)
    F, Fp = f[:, None], fp[:, None]
    px, py, pz, pp = ps[:, 0], ps[:, 1], ps[:, 2], ps[:, 3]
    dpx, dpz = dps[:, 0], dps[:, 2]
    uh = Fp * pz + F * dpz - 1j * b * F * py
    vh = 1j * b * F * px - 1j * a * F * pz
    wh = 1j * a * F * py - Fp * px - F * dpx
    return xp.stack([uh, vh, wh, pp])


def _raw_snapshot(w: Workload, seed: int, s: int) -> np.ndarray:
    """Unscaled fluctuation fields [4][ny][nz][nx] (u', v', w', p') in float64."""
    y = y_grid(w)
    f, fp = _envelope(w, y)
    T, dT = _cheb(w.M, y)
    alpha, beta, band, amp = _wavenumbers(w)
    iz, ix = np.nonzero(band)
    cm = _coefficients(w, seed, s)
    co = _assemble(np, w, cm, T, dT, f, fp, alpha[ix][None, :], beta[iz][None, :])
    spec = np.zeros((4, w.ny, w.nz, w.nx // 2 + 1), dtype=np.complex128)
    spec[:, :, iz, ix] = co
    workers = max(1, min(16, os.cpu_count() or 1))
    phys = scipy.fft.irfft2(spec, s=(w.nz, w.nx), axes=(-2, -1), norm="forward",
                            workers=workers)
    return phys


def _scales(w: Workload, seed: int):
    key = (w.name, w.nx, w.ny, w.nz, w.M, w.spectrum_scale, int(seed))
    if key not in _SCALE_CACHE:
        r = _raw_snapshot(w, seed, 0)
        rms = np.sqrt(np.mean(r * r, axis=(-2, -1)))  # [4][ny]
        su = w.rms_u / max(rms[0].max(), 1e-300)
        sp = w.rms_p / max(rms[3].max(), 1e-300)
        _SCALE_CACHE[key] = (su, sp)
    return _SCALE_CACHE[key]


def _noise(w: Workload, seed: int, s: int) -> np.ndarray:
    """Seeded white noise [4][ny][nz][nx] scaled to noise * (rms_u, rms_p)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), int(s), 1]))
    n = rng.standard_normal((4, w.ny, w.nz, w.nx))
    n[:3] *= w.noise * w.rms_u
    n[3] *= w.noise * w.rms_p
    return n


def snapshot(w: Workload, seed: int, s: int) -> np.ndarray:
    """Full fields (u~, v~, w~, p~) of snapshot s, shape [4][ny][nz][nx].

    float64 for dtype "f64"; for dtype "f32" the fields are rounded to float32
    (the returned array is float32 and holds exactly the values the GPU reads).
    """
    su, sp = _scales(w, seed)
    r = _raw_snapshot(w, seed, s)
    r[:3] *= su
    r[3] *= sp
    if w.noise:
        r += _noise(w, seed, s)
    y = y_grid(w)
    r[0] += mean_profile(w, y)[:, None, None]
    if w.dtype == "f32":
        return r.astype(np.float32)
    return r


class DeviceSnapshots:
    """The same snapshots built on a torch device: the seeded coefficients are
    drawn on the host exactly as in `snapshot`, the Chebyshev expansion and the
    inverse transforms run on the device (for large ensembles: generation
    speed only; values agree with `snapshot` to rounding)."""

    def __init__(self, w: Workload, seed: int, device):
        import torch
        self.torch, self.w, self.seed, self.device = torch, w, int(seed), device
        y = y_grid(w)
        f, fp = _envelope(w, y)
        T, dT = _cheb(w.M, y)
        alpha, beta, band, _ = _wavenumbers(w)
        iz, ix = np.nonzero(band)
        c128 = torch.complex128
        dev = lambda x, dt=c128: torch.as_tensor(x).to(device=device, dtype=dt)
        self.T, self.dT = dev(T), dev(dT)
        self.f, self.fp = dev(f), dev(fp)
        self.a, self.b = dev(alpha[ix][None, :]), dev(beta[iz][None, :])
        self.flat = dev(iz * (w.nx // 2 + 1) + ix, torch.int64)
        self.su, self.sp = _scales(w, seed)
        self.mean = dev(mean_profile(w, y), torch.float64)[:, None, None]

    def __call__(self, s: int, out=None):
        """Snapshot s as a device tensor [4][ny][nz][nx] (written into out if given)."""
        torch, w = self.torch, self.w
        cm = torch.from_numpy(_coefficients(w, self.seed, s)).to(self.device)
        co = _assemble(torch, w, cm, self.T, self.dT, self.f, self.fp, self.a, self.b)
        nkx = w.nx // 2 + 1
        spec = torch.zeros((4, w.ny, w.nz * nkx), dtype=torch.complex128, device=self.device)
        spec[:, :, self.flat] = co
        spec = spec.view(4, w.ny, w.nz, nkx)
        r = torch.fft.irfft2(spec, s=(w.nz, w.nx), norm="forward")
        r[:3] *= self.su
        r[3] *= self.sp
        if w.noise:
            r += torch.from_numpy(_noise(w, self.seed, s)).to(self.device)
        r[0] += self.mean
        dt = torch.float32 if w.dtype == "f32" else torch.float64
        if out is None:
            return r.to(dt)
        out.copy_(r)
        return out


class FastDeviceSnapshots(DeviceSnapshots):
    """Snapshots with the same amplitude law, envelope, scaling and mean as
    DeviceSnapshots, but with the random coefficients drawn on the device
    (a torch generator seeded per snapshot), for ensembles too large to keep
    resident or to draw on the host: statistically the same fields, not the
    same values as `snapshot`.  Built in the snapshot's own precision, with the
    scales and the mean profile applied to the coefficients, so one inverse
    transform writes the snapshot."""

    def __init__(self, w: Workload, seed: int, device):
        if w.noise:
            raise ValueError("FastDeviceSnapshots draws no white-noise component")
        super().__init__(w, seed, device)
        torch = self.torch
        self.rdt = torch.float32 if w.dtype == "f32" else torch.float64
        self.cdt = torch.complex64 if w.dtype == "f32" else torch.complex128
        for k in ("T", "dT", "f", "fp", "a", "b"):
            setattr(self, k, getattr(self, k).to(self.cdt))
        _, _, band, amp = _wavenumbers(w)
        iz, ix = np.nonzero(band)
        self.amp = torch.as_tensor(amp[iz, ix]).to(device=device, dtype=self.rdt)
        self.nb = iz.size
        self.scale = torch.tensor([self.su, self.su, self.su, self.sp], device=device,
                                  dtype=self.rdt)[:, None, None]
        nkx = w.nx // 2 + 1
        # band entries are rewritten every call, the rest stay zero
        self.spec = torch.zeros((4, w.ny, w.nz * nkx), dtype=self.cdt, device=device)
        self.mean_in_band = bool(((iz == 0) & (ix == 0)).any())
        self.mean_c = self.mean[:, 0, 0].to(self.cdt)
        if not self.mean_in_band:
            self.spec[0, :, 0] = self.mean_c

    def coefficients(self, s: int):
        torch, w = self.torch, self.w
        g = torch.Generator(device=self.device)
        g.manual_seed(int(self.seed) * 1000003 + int(s))
        # unit-variance real and imaginary parts, as the host draw
        re = torch.randn((4, w.M, self.nb), generator=g, device=self.device, dtype=self.rdt)
        im = torch.randn((4, w.M, self.nb), generator=g, device=self.device, dtype=self.rdt)
        c = torch.complex(re, im) * self.amp[None, None, :]
        return c.permute(1, 0, 2).reshape(w.M, 4 * self.nb)

    def __call__(self, s: int, out=None):
        torch, w = self.torch, self.w
        co = _assemble(torch, w, self.coefficients(s), self.T, self.dT, self.f, self.fp,
                       self.a, self.b)
        self.spec[:, :, self.flat] = co * self.scale
        if self.mean_in_band:
            self.spec[0, :, 0] += self.mean_c
        nkx = w.nx // 2 + 1
        spec = self.spec.view(4, w.ny, w.nz, nkx)
        if out is None:
            return torch.fft.irfft2(spec, s=(w.nz, w.nx), norm="forward")
        if out.dtype != self.rdt or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the snapshot dtype")
        torch.fft.irfft2(spec, s=(w.nz, w.nx), norm="forward", out=out)
        return out


def snapshots(w: Workload, seed: int, S: int | None = None) -> np.ndarray:
    """Stack of S snapshots, shape [S][4][ny][nz][nx]."""
    S = w.S if S is None else S
    out = np.empty((S, 4, w.ny, w.nz, w.nx),
                   dtype=np.float32 if w.dtype == "f32" else np.float64)
    for s in range(S):
        out[s] = snapshot(w, seed, s)
    return out


def mirror(snap: np.ndarray) -> np.ndarray:
    """Reflection y -> -y of a stack [S][4][ny][nz][nx]: (u, -v, w, p)(x, -y, z).

    Used to build ensembles closed under the wall-normal inversion.
    """
    m = snap[:, :, ::-1].copy()
    m[:, 1] *= -1
    return m
