"""Level-0 oracle: the GKE terms straight from their definitions by direct sums.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's CPU leg).  No Parseval,
no correlation expansion: every statistic is the average, over snapshots and
over the Nx*Nz points of a plane (periodic wrap-around of the separation),
of the increments between x = (x, Y1, z) and x' = (x + rx, Y2, z + rz)
(Section "The Generalised Kolmogorov equation": du = u(x') - u(x),
(.)* = average of the two points).  Cost O(S Nx Nz) per output point, so it
serves tiny grids whole and large grids point by point.

Definitions used (eqs. du2, GKE, scale-flux, physical-flux, source):
  T1  <du_i du_i>             T8  -2 nu d T1/d rz  (spectral in r)
  T2  <du^2 du>               T9  <v* du^2>
  T3  <du^2 dU>               T10 2 <dp dv>         (rho = 1)
  T4  -2 nu d T1/d rx         T11 -(nu/2) d T1/d Y  = -(nu/2)(d/dY1 + d/dY2) T1
  T5  <du^2 dv>               T12 -2 <du dv> (dU/dy)*
  T6  -2 nu d T1/d ry = -nu (d/dY2 - d/dY1) T1
  T7  <du^2 dw>               T13 -2 <du v*> d(dU/dy)
                              T14 -4 <eps*>,  eps = nu <du_i/dx_j du_i/dx_j>
x and z derivatives are spectral (numpy's FFT as a library step, Nyquist
multiplier 0); y derivatives use five-point weights obtained here by solving
the Vandermonde moment conditions (exact for polynomials of degree <= 4).
"""
from __future__ import annotations

import numpy as np


def fd5_weights(y: np.ndarray) -> np.ndarray:
    """Five-point first-derivative matrix by moment conditions (np.linalg.solve)."""
    ny = y.size
    D = np.zeros((ny, ny))
    for j in range(ny):
        j0 = min(max(j - 2, 0), ny - 5)
        nodes = np.arange(j0, j0 + 5)
        h = y[nodes] - y[j]
        # sum_m w_m h_m^k = d/dy (y - y_j)^k at y_j  ->  [0, 1, 0, 0, 0]
        A = np.vstack([h ** k for k in range(5)])
        rhs = np.array([0.0, 1.0, 0.0, 0.0, 0.0])
        D[j, nodes] = np.linalg.solve(A, rhs)
    return D


def _kvec(n: int, length: float) -> np.ndarray:
    k = np.fft.fftfreq(n, d=1.0 / n)
    a = 2.0 * np.pi * k / length
    if n % 2 == 0:
        a[n // 2] = 0.0
    return a


def spectral_dx(f: np.ndarray, length: float, axis: int) -> np.ndarray:
    n = f.shape[axis]
    a = _kvec(n, length)
    shape = [1] * f.ndim
    shape[axis] = n
    F = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(1j * a.reshape(shape) * F, axis=axis))


def profiles(snap: np.ndarray, y: np.ndarray, lx: float, lz: float, nu: float):
    """Means, fluctuations, dU/dy and eps by direct averaging."""
    snap = np.asarray(snap, dtype=np.float64)
    mean = snap.mean(axis=(0, 3, 4))                       # [4][ny]
    fl = snap - mean[None, :, :, None, None]
    D = fd5_weights(y)
    S = D @ mean[0]
    g2 = np.zeros(y.size)
    for c in range(3):
        f = fl[:, c]                                        # [S][ny][nz][nx]
        dx = spectral_dx(f, lx, axis=3)
        dz = spectral_dx(f, lz, axis=2)
        dy = np.einsum("jm,smzx->sjzx", D, f)
        g2 += (dx ** 2 + dy ** 2 + dz ** 2).mean(axis=(0, 2, 3))
    eps = nu * g2
    return mean, fl, S, eps, D


def _shifted(plane: np.ndarray, p: int, q: int) -> np.ndarray:
    """plane[..., z, x] -> plane[..., z + q, x + p] (periodic)."""
    return np.roll(plane, shift=(-q, -p), axis=(-2, -1))


def point_stats(fl, mean, S, eps, j1, j2, p, q):
    """Definitions at one (Y1, Y2, rx index p, rz index q): T1 T2 T3 T5 T7 T9 T10 T12 T13 T14."""
    a = fl[:, :, j1]                                        # [S][4][nz][nx] at x
    b = _shifted(fl[:, :, j2], p, q)                        # at x'
    du = b[:, :3] - a[:, :3]
    du2 = (du * du).sum(axis=1)
    dU = mean[0, j2] - mean[0, j1]
    vstar = 0.5 * (a[:, 1] + b[:, 1])
    dp = b[:, 3] - a[:, 3]
    out = {
        1: du2.mean(),
        2: (du2 * du[:, 0]).mean(),
        3: (du2 * dU).mean(),
        5: (du2 * du[:, 1]).mean(),
        7: (du2 * du[:, 2]).mean(),
        9: (vstar * du2).mean(),
        10: 2.0 * (dp * du[:, 1]).mean(),
        12: -2.0 * (du[:, 0] * du[:, 1]).mean() * 0.5 * (S[j1] + S[j2]),
        13: -2.0 * (du[:, 0] * vstar).mean() * (S[j2] - S[j1]),
        14: -4.0 * 0.5 * (eps[j1] + eps[j2]),
    }
    return out


def pair_maps(fl, mean, S, eps, j1, j2):
    """Full [14][nz][nx] maps for one pair, except T6 and T11 (need neighbours)."""
    nz, nx = fl.shape[-2:]
    out = np.zeros((14, nz, nx))
    for q in range(nz):
        for p in range(nx):
            st = point_stats(fl, mean, S, eps, j1, j2, p, q)
            for t, v in st.items():
                out[t - 1, q, p] = v
    return out


def terms(snap, y, lx, lz, nu, pairs):
    """All 14 maps [npairs][14][nz][nx] for the listed ordered pairs, by direct sums."""
    mean, fl, S, eps, D = profiles(snap, y, lx, lz, nu)
    cache = {}

    def maps(j1, j2):
        if (j1, j2) not in cache:
            cache[(j1, j2)] = pair_maps(fl, mean, S, eps, j1, j2)
        return cache[(j1, j2)]

    res = []
    for (j1, j2) in pairs:
        o = maps(j1, j2).copy()
        t1 = o[0]
        o[3] = -2.0 * nu * spectral_dx(t1, lx, axis=1)      # d/drx along the p index
        o[7] = -2.0 * nu * spectral_dx(t1, lz, axis=0)      # d/drz along the q index
        dY1 = sum(D[j1, m] * maps(int(m), j2)[0] for m in np.nonzero(D[j1])[0])
        dY2 = sum(D[j2, m] * maps(j1, int(m))[0] for m in np.nonzero(D[j2])[0])
        o[5] = -2.0 * nu * 0.5 * (dY2 - dY1)
        o[10] = -0.5 * nu * (dY1 + dY2)
        res.append(o)
    return np.array(res)
