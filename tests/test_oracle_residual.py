"""Pins of the oracle's budget residual (eq. GKE-conservative) against closed
forms derived by hand from the definitions, and an exact symmetry.

Prescribed trigonometric fields with velocity and pressure amplitudes of
degree <= 2 in y make every wall-normal flux a polynomial of degree <= 4 in
Y1 and in Y2, on which the five-point stencil is exact, so the residual
equals its analytic value; the separations' derivatives are exact spectrally
(single harmonics far from Nyquist).  Y-derivatives of the closed-form triple
terms are taken by complex-step differentiation (exact to rounding for the
polynomial-times-cosine expressions)."""
import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import synth

P = np.polynomial.Polynomial


def _snapshots(nx, nz, lx, lz, y, amps, harm, phase, Uprof, S=2):
    """u_i = U_i(y) + a_i(y) cos(n_i theta + phi_i), theta = alpha0 x + beta0 z,
    translated by 0.7 s in theta for snapshot s (statistics unchanged)."""
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    th = 2 * np.pi / lx * x[None, :] + 2 * np.pi / lz * z[:, None]
    snap = np.zeros((S, 4, y.size, nz, nx))
    for s in range(S):
        for f in range(4):
            snap[s, f] = amps[f](y)[:, None, None] * np.cos(harm[f] * (th + 0.7 * s)[None]
                                                            + phase[f])
        snap[s, 0] += Uprof(y)[:, None, None]
    return snap


def _psi(nx, nz):
    p = np.arange(nx)
    q = np.arange(nz)
    return 2 * np.pi * (p[None, :] / nx + q[:, None] / nz)   # [q][p]


def test_residual_closed_form_single_harmonic():
    """Every field on one harmonic: the turbulent fluxes vanish and
    Res = d/drx (T3 + T4) + d/drz T8 - nu (d2/dY1^2 + d2/dY2^2) <du^2>
          + (d/dY1 + d/dY2) T10 - (T12 + T13 + T14)."""
    nx, nz, lx, lz, nu = 12, 10, 3.0, 2.5, 0.03
    y = -np.cos(np.pi * np.arange(13) / 12)
    a = [P([1.0, 0.5, -0.8]), P([0.3, -0.6, 0.4]), P([0.7, 0.2, 0.0]), P([0.5, 0.1, 0.3])]
    ph = [0.4, -1.2, 2.1, 0.9]
    U = P([1.0, 0.0, -1.0])
    snap = _snapshots(nx, nz, lx, lz, y, a, [1, 1, 1, 1], ph, U)
    pairs = [(3, 9), (9, 3), (6, 6), (4, 5), (2, 10)]
    res = oracle.residual(snap, y, lx, lz, nu, pairs)
    psi = _psi(nx, nz)
    a0, b0 = 2 * np.pi / lx, 2 * np.pi / lz
    da = [ai.deriv() for ai in a]
    d2a = [ai.deriv(2) for ai in a]
    q = 0.5 * sum(ai * ai for ai in a[:3])
    S = U.deriv()
    uv = lambda Y: 0.5 * a[0](Y) * a[1](Y) * np.cos(ph[1] - ph[0])
    pv = 0.5 * a[3] * a[1] * np.cos(ph[1] - ph[3])
    eps = lambda Y: nu * sum(0.5 * a[i](Y) ** 2 * (a0 ** 2 + b0 ** 2) + 0.5 * da[i](Y) ** 2
                             for i in range(3))
    for k, (j1, j2) in enumerate(pairs):
        y1, y2 = y[j1], y[j2]
        A12 = sum(a[i](y1) * a[i](y2) for i in range(3))
        dU = U(y2) - U(y1)
        # separations: d/drx of T3 = dU T1 and of T4 = -2 nu dT1/drx, d/drz of T8
        div_h = dU * a0 * A12 * np.sin(psi) - 2 * nu * (a0 ** 2 + b0 ** 2) * A12 * np.cos(psi)
        # viscous wall-normal parts: (1/2)(d2 - d1) T6 + (d1 + d2) T11
        d11 = q.deriv(2)(y1) - sum(d2a[i](y1) * a[i](y2) for i in range(3)) * np.cos(psi)
        d22 = q.deriv(2)(y2) - sum(a[i](y1) * d2a[i](y2) for i in range(3)) * np.cos(psi)
        visc = -nu * (d11 + d22)
        # pressure flux T10 = 2 <dp dv>, C[A, B] = 1/2 A(Y1) B(Y2) cos(psi + phi_B - phi_A)
        cpv = np.cos(psi + ph[1] - ph[3])
        cvp = np.cos(psi + ph[3] - ph[1])
        dT10 = 2 * (pv.deriv()(y1) + pv.deriv()(y2)
                    - 0.5 * (da[3](y1) * a[1](y2) + a[3](y1) * da[1](y2)) * cpv
                    - 0.5 * (da[1](y1) * a[3](y2) + a[1](y1) * da[3](y2)) * cvp)
        # sources
        c = lambda fa, fb: 0.5 * a[fa](y1) * a[fb](y2) * np.cos(psi + ph[fb] - ph[fa])
        dudv = uv(y1) + uv(y2) - c(1, 0) - c(0, 1)
        duvs = 0.5 * (uv(y2) - uv(y1) + c(1, 0) - c(0, 1))
        xi = (-2 * dudv * 0.5 * (S(y1) + S(y2)) - 2 * duvs * (S(y2) - S(y1))
              - 2 * (eps(y1) + eps(y2)))
        expect = div_h + visc + dT10 - xi
        scale = max(np.abs(xi).max(), np.abs(dT10).max(), np.abs(div_h).max())
        assert np.abs(res[k] - expect).max() < 1e-11 * scale, (k, np.abs(res[k] - expect).max())
        assert np.abs(expect).max() > 1e-3 * scale


def _cstep(f, x):
    """df/dx by complex-step differentiation."""
    h = 1e-30
    return np.imag(f(x + 1j * h)) / h


def test_residual_closed_form_triple_terms():
    """u on harmonic 1 and v on harmonic 2 (w = p = 0, no mean flow): the
    r_y and Y turbulent fluxes T5 and T9 enter through their Y-derivatives."""
    nx, nz, lx, lz, nu = 16, 16, 4.0, 3.0, 0.02
    y = -np.cos(np.pi * np.arange(11) / 10)
    fa = P([0.9, 0.3])
    fb = P([0.4, 0.0, -0.5])
    zero = P([0.0])
    al, be = 0.6, -1.3
    snap = _snapshots(nx, nz, lx, lz, y, [fa, fb, zero, zero], [1, 2, 1, 1], [al, be, 0, 0],
                      zero)
    pairs = [(2, 7), (7, 2), (5, 5), (1, 9)]
    res = oracle.residual(snap, y, lx, lz, nu, pairs)
    psi = _psi(nx, nz)
    a0, b0 = 2 * np.pi / lx, 2 * np.pi / lz
    cos = np.cos

    def T5(y1, y2):
        a1, a2, b1, b2 = fa(y1), fa(y2), fb(y1), fb(y2)
        return (0.25 * a2 ** 2 * b2 * cos(be - 2 * al) - 0.25 * a2 ** 2 * b1 * cos(be - 2 * psi - 2 * al)
                - 0.5 * a1 * a2 * b2 * cos(psi + be - 2 * al) + 0.5 * a1 * a2 * b1 * cos(be - psi - 2 * al)
                + 0.25 * a1 ** 2 * b2 * cos(2 * psi + be - 2 * al) - 0.25 * a1 ** 2 * b1 * cos(be - 2 * al))

    def T9(y1, y2):
        a1, a2, b1, b2 = fa(y1), fa(y2), fb(y1), fb(y2)
        return 0.125 * (a2 ** 2 * b1 * cos(be - 2 * psi - 2 * al) - 2 * a1 * a2 * b1 * cos(be - psi - 2 * al)
                        + a1 ** 2 * b1 * cos(be - 2 * al) + a2 ** 2 * b2 * cos(be - 2 * al)
                        - 2 * a1 * a2 * b2 * cos(psi + be - 2 * al) + a1 ** 2 * b2 * cos(2 * psi + be - 2 * al))

    eps = lambda Y: nu * (0.5 * fa(Y) ** 2 * (a0 ** 2 + b0 ** 2) + 0.5 * fa.deriv()(Y) ** 2
                          + 0.5 * fb(Y) ** 2 * 4 * (a0 ** 2 + b0 ** 2) + 0.5 * fb.deriv()(Y) ** 2)
    for k, (j1, j2) in enumerate(pairs):
        y1, y2 = y[j1], y[j2]
        a1, a2, b1, b2 = fa(y1), fa(y2), fb(y1), fb(y2)
        # T1 = q1 + q2 - a1 a2 cos psi - b1 b2 cos 2 psi; T4, T8 viscous r-fluxes
        div_h = -2 * nu * (a0 ** 2 + b0 ** 2) * (a1 * a2 * cos(psi) + 4 * b1 * b2 * cos(2 * psi))
        q2d = lambda Y: fa.deriv()(Y) ** 2 + fa(Y) * fa.deriv(2)(Y) + fb.deriv()(Y) ** 2 \
            + fb(Y) * fb.deriv(2)(Y)
        d11 = q2d(y1) - fa.deriv(2)(y1) * a2 * cos(psi) - fb.deriv(2)(y1) * b2 * cos(2 * psi)
        d22 = q2d(y2) - a1 * fa.deriv(2)(y2) * cos(psi) - b1 * fb.deriv(2)(y2) * cos(2 * psi)
        visc = -nu * (d11 + d22)
        dT5_1 = _cstep(lambda t: T5(t, y2), y1)
        dT5_2 = _cstep(lambda t: T5(y1, t), y2)
        dT9_1 = _cstep(lambda t: T9(t, y2), y1)
        dT9_2 = _cstep(lambda t: T9(y1, t), y2)
        turb = 0.5 * (dT5_2 - dT5_1) + dT9_1 + dT9_2
        xi = -2 * (eps(y1) + eps(y2))
        expect = div_h + visc + turb - xi
        scale = max(np.abs(turb).max(), np.abs(visc).max(), abs(xi))
        assert np.abs(res[k] - expect).max() < 1e-11 * scale, (k, np.abs(res[k] - expect).max())
        if j1 != j2:
            assert np.abs(turb).max() > 1e-2 * scale


def test_residual_r_inversion_symmetry():
    """Every part of the residual is even under the exchange (r, Y1, Y2) ->
    (-r, Y2, Y1) (the r-divergence of odd fluxes, d/dry of an odd flux, d/dY
    of an even one, the even source), exactly for any sample."""
    w = synth.workload("tiny", S=2, noise=0.5)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 8)
    pairs = [(3, 9), (9, 3), (0, 16), (16, 0)]
    r = oracle.residual(snap, y, w.lx, w.lz, w.nu, pairs)
    neg = lambda m: np.roll(m[::-1, ::-1], shift=(1, 1), axis=(0, 1))
    for a, b in ((0, 1), (2, 3)):
        assert np.abs(r[a] - neg(r[b])).max() < 1e-12 * np.abs(r[a]).max()
    assert np.abs(r[0] - r[1]).max() > 1e-6 * np.abs(r[0]).max()   # not trivially symmetric


@pytest.mark.parametrize("dir_", ["x", "z"])
def test_residual_closed_form_homogeneous_triple_fluxes(dir_):
    """One velocity component on harmonic 2 (amplitude a) and another on
    harmonic 1 (amplitude c), the rest zero, no mean flow: with the component
    on harmonic 2 along x, T2 = <du^2 du> is the only non-zero turbulent flux
    (along z: T7 = <du^2 dw>), from <dw^2 du> (<du^2 dw>):
        T = 1/4 [c2^2 a2 cos g - c2^2 a1 cos(2 psi + g) - 2 c1 c2 a2 cos(g - psi)
                 + 2 c1 c2 a1 cos(psi + g) + c1^2 a2 cos(g - 2 psi) - c1^2 a1 cos g],
    g = 2 phi_c - phi_a (product-to-sum on the three cosines), and the
    residual gets its r derivative (alpha0 or beta0 times d/dpsi)."""
    nx, nz, lx, lz, nu = 16, 16, 4.0, 3.0, 0.02
    y = -np.cos(np.pi * np.arange(11) / 10)
    fa = P([0.5, -0.2, 0.3])   # harmonic 2
    fc = P([0.8, 0.4])         # harmonic 1
    zero = P([0.0])
    pa, pc = 0.3, -0.9
    if dir_ == "x":   # u on harmonic 2, w on harmonic 1
        amps, harm, ph, slot = [fa, zero, fc, zero], [2, 1, 1, 1], [pa, 0, pc, 0], 1
    else:             # w on harmonic 2, u on harmonic 1
        amps, harm, ph, slot = [fc, zero, fa, zero], [1, 1, 2, 1], [pc, 0, pa, 0], 6
    snap = _snapshots(nx, nz, lx, lz, y, amps, harm, ph, zero)
    pairs = [(2, 7), (7, 2), (5, 5), (1, 9)]
    terms = oracle.pair_terms(snap, y, lx, lz, nu, pairs)
    res = oracle.residual(snap, y, lx, lz, nu, pairs)
    psi = _psi(nx, nz)
    a0, b0 = 2 * np.pi / lx, 2 * np.pi / lz
    cos = np.cos
    g = 2 * pc - pa

    def T(y1, y2, ps):
        a1, a2, c1, c2 = fa(y1), fa(y2), fc(y1), fc(y2)
        return 0.25 * (c2 ** 2 * a2 * cos(g) - c2 ** 2 * a1 * cos(2 * ps + g)
                       - 2 * c1 * c2 * a2 * cos(g - ps) + 2 * c1 * c2 * a1 * cos(ps + g)
                       + c1 ** 2 * a2 * cos(g - 2 * ps) - c1 ** 2 * a1 * cos(g))

    eps = lambda Y: nu * (0.5 * fa(Y) ** 2 * 4 * (a0 ** 2 + b0 ** 2) + 0.5 * fa.deriv()(Y) ** 2
                          + 0.5 * fc(Y) ** 2 * (a0 ** 2 + b0 ** 2) + 0.5 * fc.deriv()(Y) ** 2)
    k_r = a0 if dir_ == "x" else b0
    for k, (j1, j2) in enumerate(pairs):
        y1, y2 = y[j1], y[j2]
        Tc = T(y1, y2, psi)
        # the flux itself, and the other turbulent fluxes vanish
        sc = np.abs(Tc).max() if j1 != j2 else 1e-3
        assert np.abs(terms[k, slot] - Tc).max() < 1e-12 * max(sc, 1e-3), (k, slot)
        for other in {1, 4, 6, 8} - {slot}:
            assert np.abs(terms[k, other]).max() < 1e-13, (k, other)
        a1, a2, c1, c2 = fa(y1), fa(y2), fc(y1), fc(y2)
        dT = k_r * _cstep(lambda t: T(y1, y2, t), psi)
        div_h = -2 * nu * (a0 ** 2 + b0 ** 2) * (4 * a1 * a2 * cos(2 * psi) + c1 * c2 * cos(psi))
        q2d = lambda Y: fa.deriv()(Y) ** 2 + fa(Y) * fa.deriv(2)(Y) + fc.deriv()(Y) ** 2 \
            + fc(Y) * fc.deriv(2)(Y)
        d11 = q2d(y1) - fa.deriv(2)(y1) * a2 * cos(2 * psi) - fc.deriv(2)(y1) * c2 * cos(psi)
        d22 = q2d(y2) - a1 * fa.deriv(2)(y2) * cos(2 * psi) - c1 * fc.deriv(2)(y2) * cos(psi)
        expect = dT + div_h - nu * (d11 + d22) + 2 * (eps(y1) + eps(y2))
        scale = max(np.abs(dT).max(), np.abs(div_h).max(), 2 * (eps(y1) + eps(y2)))
        assert np.abs(res[k] - expect).max() < 1e-11 * scale, (k, np.abs(res[k] - expect).max())
        if j1 != j2:
            assert np.abs(dT).max() > 1e-2 * scale
