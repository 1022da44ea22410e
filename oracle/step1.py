"""Oracle of Step 1 upstream of the two-point statistics: the full velocity
from the wall-normal velocity and vorticity, and the pressure from the
Poisson equation, on the nonuniform y grid (Section "Step 1": the database
may hold only v and omega_y as Fourier coefficients in x and z; the pressure
is obtained by solving its Poisson equation for each velocity field).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the HIP product path.

Conventions (readings; the paper gives no formulas for this step):
  * coefficients f^(kx, kz; y) of f(x, z) = sum_k f^ e^{i(alpha x + beta z)}
    over the half spectrum kx = 0..Nx/2 (Hermitian in the rest), i.e. the
    forward transform scaled by 1/(Nx Nz); alpha = 2 pi kx/Lx, beta =
    2 pi kz_signed/Lz, both taken as 0 at the Nyquist wavenumbers (as for
    every spectral derivative of the statistics);
  * continuity i alpha u^ + D v^ + i beta w^ = 0 and omega_y = du/dz - dw/dx,
    i.e. omega^ = i beta u^ - i alpha w^, give for k^2 = alpha^2 + beta^2 > 0
        u^ = i (alpha D v^ - beta omega^) / k^2,  w^ = i (beta D v^ + alpha omega^) / k^2;
    the (0, 0) mode of u and w is the given plane-mean profile; bins whose two
    multipliers vanish otherwise carry no u, w;
  * pressure: div of the momentum equation, lap p = -d_i d_j (u_i u_j) with
    the total velocity (products formed on the grid), so per wavenumber
        (D2 - k^2) p^ = alpha^2 (uu)^ + 2 alpha beta (uw)^ + beta^2 (ww)^
                        - 2 i alpha D (uv)^ - 2 i beta D (vw)^ - D2 (vv)^
    on the interior nodes, and at the two walls the wall-normal momentum
    equation with no-slip, D p^ = nu D2 v^ (Neumann);
    the (0, 0) mode: p^ = -(vv)^ (the solution of its equation with zero
    integration constants; the mean pressure does not enter the budget), and
    other bins with k^2 = 0 (Nyquist multipliers) p^ = 0;
  * D: the five-point first derivative of the statistics; D2: the five-point
    second-derivative weights on the same windows (exact on quartics).
"""
from __future__ import annotations

import numpy as np

from . import oracle


def fd5_second_matrix(y: np.ndarray) -> np.ndarray:
    """Five-point second-derivative operator on the first-derivative windows
    (centred in the interior, the five nodes nearest a wall at the ends), by
    the moment conditions sum_m w_m (y_m - y_j)^p = d^2/dy^2 (y - y_j)^p at y_j."""
    y = np.asarray(y, dtype=np.float64)
    ny = y.size
    D2 = np.zeros((ny, ny))
    for j in range(ny):
        j0 = min(max(j - 2, 0), ny - 5)
        nodes = np.arange(j0, j0 + 5)
        h = y[nodes] - y[j]
        A = np.vstack([h ** p for p in range(5)])
        D2[j, nodes] = np.linalg.solve(A, np.array([0.0, 0.0, 2.0, 0.0, 0.0]))
    return D2


def multipliers(nx: int, nz: int, lx: float, lz: float):
    """alpha [nkx] and beta [nz] with zero multipliers at the Nyquist indices."""
    kx = np.arange(nx // 2 + 1)
    alpha = 2.0 * np.pi * kx / lx
    alpha[nx // 2] = 0.0
    kz = np.fft.fftfreq(nz, d=1.0 / nz)
    beta = 2.0 * np.pi * kz / lz
    beta[nz // 2] = 0.0
    return alpha, beta


def velocity_spectra(vhat, ohat, mean_u, mean_w, y, lx, lz):
    """u^, v^, w^ [3][ny][nz][nkx] from v^, omega^ [ny][nz][nkx] and the (0, 0)
    profiles of u and w."""
    ny, nz, nkx = vhat.shape
    nx = 2 * (nkx - 1)
    D = oracle.fd5_matrix(y)
    alpha, beta = multipliers(nx, nz, lx, lz)
    a = alpha[None, None, :]
    b = beta[None, :, None]
    k2 = a * a + b * b
    dv = np.einsum("jm,mzx->jzx", D, vhat)
    safe = np.where(k2 > 0, k2, 1.0)
    uh = np.where(k2 > 0, 1j * (a * dv - b * ohat) / safe, 0.0)
    wh = np.where(k2 > 0, 1j * (b * dv + a * ohat) / safe, 0.0)
    uh[:, 0, 0] = mean_u
    wh[:, 0, 0] = mean_w
    return np.stack([uh, vhat, wh])


def to_physical(spec, nx):
    """Physical fields [..][nz][nx] of half-spectrum coefficients (numpy's
    inverse transform as a library step; the kx = 0 and Nx/2 lines taken as
    the Hermitian part, i.e. the real map they define)."""
    return np.fft.irfft2(spec, s=(spec.shape[-2], nx), axes=(-2, -1), norm="forward")


def to_spectrum(phys):
    """Half-spectrum coefficients (forward transform / (Nx Nz))."""
    return np.fft.rfft2(phys, axes=(-2, -1), norm="forward")


def pressure_rhs(u, v, w, y, lx, lz):
    """Right-hand side of the Poisson equation per wavenumber and plane,
    [ny][nz][nkx], from the physical total velocity [ny][nz][nx]."""
    ny, nz, nx = u.shape
    D = oracle.fd5_matrix(y)
    D2 = fd5_second_matrix(y)
    alpha, beta = multipliers(nx, nz, lx, lz)
    a = alpha[None, None, :]
    b = beta[None, :, None]
    P = {k: to_spectrum(f) for k, f in (("uu", u * u), ("uw", u * w), ("ww", w * w),
                                         ("uv", u * v), ("vw", v * w), ("vv", v * v))}
    Dy = lambda f: np.einsum("jm,mzx->jzx", D, f)
    D2y = lambda f: np.einsum("jm,mzx->jzx", D2, f)
    return (a * a * P["uu"] + 2 * a * b * P["uw"] + b * b * P["ww"]
            - 2j * a * Dy(P["uv"]) - 2j * b * Dy(P["vw"]) - D2y(P["vv"])), P["vv"]


def pressure_solve(rhs, bc0, bc1, k2, y):
    """p^ on the nodes y from (D2 - k2) p^ = rhs on the interior nodes and
    D p^ = bc0 (first node), bc1 (last node): a dense solve (numpy's LU with
    partial pivoting as a library step)."""
    ny = y.size
    D = oracle.fd5_matrix(y)
    A = fd5_second_matrix(y) - k2 * np.eye(ny)
    A[0] = D[0]
    A[-1] = D[-1]
    b = np.array(rhs, dtype=np.complex128)
    b[0], b[-1] = bc0, bc1
    return np.linalg.solve(A, b)


def reconstruct(vhat, ohat, mean_u, mean_w, y, lx, lz, nu):
    """Physical u, v, w, p [4][ny][nz][nx] of one snapshot stored as v^ and
    omega_y^ (half spectra [ny][nz][nkx]) and the plane-mean u and w."""
    y = np.asarray(y, dtype=np.float64)
    ny, nz, nkx = vhat.shape
    nx = 2 * (nkx - 1)
    spec = velocity_spectra(vhat, ohat, mean_u, mean_w, y, lx, lz)
    u, v, w = to_physical(spec, nx)
    rhs, vv = pressure_rhs(u, v, w, y, lx, lz)
    D2 = fd5_second_matrix(y)
    bc = nu * np.einsum("jm,mzx->jzx", D2, spec[1])
    alpha, beta = multipliers(nx, nz, lx, lz)
    ph = np.zeros((ny, nz, nkx), dtype=np.complex128)
    for iz in range(nz):
        for ix in range(nkx):
            k2 = alpha[ix] ** 2 + beta[iz] ** 2
            if ix == 0 and iz == 0:
                ph[:, 0, 0] = -vv[:, 0, 0]
            elif k2 > 0:
                ph[:, iz, ix] = pressure_solve(rhs[:, iz, ix], bc[0, iz, ix], bc[-1, iz, ix],
                                               k2, y)
    p = to_physical(ph, nx)
    return np.stack([u, v, w, p])
