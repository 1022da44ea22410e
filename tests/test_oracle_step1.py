"""Pins of the Step-1 oracle (velocity from v and omega_y, pressure from its
Poisson equation) against what the mathematics fixes: polynomial exactness of
the five-point operators, the defining equations of the reconstruction
(continuity and the wall-normal vorticity), a hand-derived closed form of the
Poisson right-hand side, exact recovery of polynomial pressures, and
convergence to an analytic solution of the continuous Neumann problem."""
import numpy as np
import pytest

from oracle import oracle, step1
from paper_1910_06409_amd import synth

P = np.polynomial.Polynomial


def _grid(n=17):
    return -np.cos(np.pi * np.arange(n) / (n - 1))


@pytest.mark.parametrize("y", [_grid(17), synth.y_grid(synth.workload("re200"))])
def test_second_derivative_exact_on_quartics(y):
    D2 = step1.fd5_second_matrix(y)
    for k in range(5):
        f = y ** k
        d2 = k * (k - 1) * y ** (k - 2) if k >= 2 else 0 * y
        assert np.abs(D2 @ f - d2).max() < 1e-8 * max(1.0, np.abs(d2).max())
    # the windows are the first derivative's
    D = oracle.fd5_matrix(y)
    assert np.array_equal(D != 0, D2 != 0)


def _spectral_d(f, n_len, length, axis):
    """Spectral derivative along an axis of a physical field, zero Nyquist multiplier."""
    n = f.shape[axis]
    k = np.fft.fftfreq(n, d=1.0 / n)
    m = 2 * np.pi * k / length
    m[n // 2] = 0.0
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * m.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def test_velocity_reconstruction_satisfies_continuity_and_vorticity():
    nx, nz, lx, lz = 16, 12, 2 * np.pi, np.pi
    y = _grid(13)
    rng = np.random.default_rng(3)
    nkx = nx // 2 + 1
    # v^ of degree 4 in y per mode (so the five-point D v^ is exact), omega^ arbitrary
    c = rng.standard_normal((5, nz, nkx)) + 1j * rng.standard_normal((5, nz, nkx))
    vh = sum(c[p][None] * y[:, None, None] ** p for p in range(5))
    dvh = sum(p * c[p][None] * y[:, None, None] ** (p - 1) for p in range(1, 5))
    oh = rng.standard_normal((y.size, nz, nkx)) + 1j * rng.standard_normal((y.size, nz, nkx))
    # bins with both multipliers zero carry nothing (undetermined u, w)
    for iz, ix in [(0, 0), (0, nkx - 1), (nz // 2, 0), (nz // 2, nkx - 1)]:
        vh[:, iz, ix] = dvh[:, iz, ix] = oh[:, iz, ix] = 0.0
    mu, mw = 1 - y ** 2, 0.1 * y
    spec = step1.velocity_spectra(vh, oh, mu, mw, y, lx, lz)
    u, v, w = step1.to_physical(spec, nx)
    dvdy = step1.to_physical(dvh, nx)
    div = _spectral_d(u, nx, lx, 2) + dvdy + _spectral_d(w, nz, lz, 1)
    assert np.abs(div).max() < 1e-12 * np.abs(dvdy).max()
    om = _spectral_d(u, nz, lz, 1) - _spectral_d(w, nx, lx, 2)
    om_ref = step1.to_physical(oh, nx)
    # omega of the reconstruction is the input except on the lines whose z or x
    # multiplier is zero (there only the part along the other direction acts)
    sel = np.ones((nz, nkx), bool)
    sel[nz // 2, :] = sel[:, nkx - 1] = sel[0, 0] = False
    om_sel = step1.to_physical(np.where(sel[None], oh, 0), nx)
    om_rec = step1.to_physical(np.where(sel[None], step1.to_spectrum(om), 0), nx)
    assert np.abs(om_rec - om_sel).max() < 1e-12 * np.abs(om_ref).max()
    assert np.abs(u.mean(axis=(1, 2)) - mu).max() < 1e-14
    assert np.abs(w.mean(axis=(1, 2)) - mw).max() < 1e-14


def test_pressure_rhs_closed_form():
    """One harmonic per component, amplitudes of degree <= 2: by product-to-sum,
    -d_i d_j (u_i u_j) has harmonics 0 and 2 with polynomial amplitudes of
    degree <= 4, on which the five-point operators are exact."""
    nx, nz, lx, lz = 16, 12, 3.0, 2.0
    y = _grid(11)
    a, b, cc = P([0.7, 0.2, -0.3]), P([0.0, 0.5, 0.4]), P([0.3, -0.1, 0.2])
    pu, pv, pw = 0.2, 1.1, -0.7
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    a0, b0 = 2 * np.pi / lx, 2 * np.pi / lz
    th = a0 * x[None, :] + b0 * z[:, None]
    Y = y[:, None, None]
    u = a(Y) * np.cos(th + pu)
    v = b(Y) * np.cos(th + pv)
    w = cc(Y) * np.cos(th + pw)
    rhs, _ = step1.pressure_rhs(u, v, w, y, lx, lz)
    got = step1.to_physical(rhs, nx)
    C = lambda f, ph: np.cos(2 * th + ph) * f
    S = lambda f, ph: np.sin(2 * th + ph) * f
    ab, bc = a * b, b * cc
    expect = -(0.5 * a(Y) ** 2 * (-4 * a0 ** 2) * np.cos(2 * th + 2 * pu)
               + 2 * 0.5 * a(Y) * cc(Y) * (-4 * a0 * b0) * np.cos(2 * th + pu + pw)
               + 0.5 * cc(Y) ** 2 * (-4 * b0 ** 2) * np.cos(2 * th + 2 * pw)
               + 2 * 0.5 * S(ab.deriv()(Y), pu + pv) * (-2 * a0)
               + 2 * 0.5 * S(bc.deriv()(Y), pv + pw) * (-2 * b0)
               + 0.5 * (b * b).deriv(2)(Y) * (1 + np.cos(2 * th + 2 * pv)))
    del C
    assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()


def test_pressure_solve_recovers_quartics():
    y = synth.y_grid(synth.workload("re200"))
    rng = np.random.default_rng(5)
    for k2 in (0.3, 7.0, 400.0):
        c = rng.standard_normal(5) + 1j * rng.standard_normal(5)
        p = P(c.real) + 1j * P(c.imag)
        pr, pi_ = P(c.real), P(c.imag)
        val = lambda q: pr.deriv(q)(y) + 1j * pi_.deriv(q)(y) if q else pr(y) + 1j * pi_(y)
        rhs = val(2) - k2 * val(0)
        d1 = val(1)
        got = step1.pressure_solve(rhs, d1[0], d1[-1], k2, y)
        assert np.abs(got - val(0)).max() < 1e-9 * np.abs(val(0)).max(), k2
        del p


def test_pressure_solve_converges_to_the_continuous_solution():
    """p'' - k^2 p = 6 y - k^2 y^3 with p'(+-1) given has the solution
    C cosh(k y) + y^3; the discrete Neumann problem converges at >= 3rd order."""
    k = 2.5
    C = 0.7
    exact = lambda y: C * np.cosh(k * y) + y ** 3
    dexact = lambda y: C * k * np.sinh(k * y) + 3 * y ** 2
    errs = []
    for n in (33, 65, 129):
        xi = -1 + 2 * np.arange(n) / (n - 1)
        y = np.tanh(1.5 * xi) / np.tanh(1.5)
        rhs = 6 * y - k * k * y ** 3
        got = step1.pressure_solve(rhs.astype(complex), dexact(-1.0), dexact(1.0), k * k, y)
        errs.append(np.abs(got.real - exact(y)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.8), (errs, rates)


def test_reconstruct_round_trip_on_synthetic_fields():
    """The synthetic fields are solenoidal: feeding their v and omega_y (and
    plane-mean u, w) back gives u and w again, up to the five-point error of
    D v (small on the smooth fields), and the pressure is finite and real."""
    w = synth.workload("tiny", ny=33, S=1)
    y = synth.y_grid(w)
    s = synth.snapshot(w, 4, 0)
    spec = step1.to_spectrum(s[:3])
    uh, vh, wh = spec
    ohat = 1j * step1.multipliers(w.nx, w.nz, w.lx, w.lz)[1][None, :, None] * uh \
        - 1j * step1.multipliers(w.nx, w.nz, w.lx, w.lz)[0][None, None, :] * wh
    out = step1.reconstruct(vh, ohat, uh[:, 0, 0].real, wh[:, 0, 0].real, y, w.lx, w.lz, w.nu)
    assert np.isfinite(out).all()
    err = np.abs(out[:3] - s[:3]).max() / np.abs(s[1:3]).max()
    assert err < 2e-2, err
