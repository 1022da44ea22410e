"""Python front end of the FP64 CPU oracle (level 1: the paper's Parseval method).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP product path.

Steps follow the paper (Gatti et al., Section "General structure of the
program"):
  Step 1 -- means, dU/dy, one-point moments and pseudo-dissipation
            (``liboracle.or_means`` / ``or_onepoint``);
  Step 2 -- two-point correlations through the Parseval identity for each
            requested ordered pair (Y1, Y2) and assembly of the terms that
            need no wall-normal derivative (``or_pairs``);
  Step 3 -- the viscous Phi_ry and phi parts from the five-point derivative of
            <du^2> along Y1 and Y2 (Section "Step 3": d/dry = (d/dY2 - d/dY1)/2,
            d/dY = d/dY1 + d/dY2), done here.

Term slots T1..T14 (index 0..13):
  T1 <du^2>                         T8  -2 nu d<du^2>/drz
  T2 <du^2 du>                      T9  <v* du^2>
  T3 <du^2 dU>                      T10 (2/rho)<dp dv>
  T4 -2 nu d<du^2>/drx              T11 -(nu/2) d<du^2>/dY
  T5 <du^2 dv>                      T12 -2<du dv>(dU/dy)*
  T6 -2 nu d<du^2>/dry              T13 -2<du v*> d(dU/dy)
  T7 <du^2 dw>                      T14 -4<eps*>
Maps are indexed [rz index q][rx index p] over the full periodic grid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "gke_oracle.c")

NT = 14
PROFILE_ROWS = ["U", "V", "W", "P", "S", "q", "uv", "pv", "Tx", "Ty", "Tz", "eps"]
NPROF = len(PROFILE_ROWS)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (building the checker, not running it)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-fcx-limited-range",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_fft1.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = ctypes.c_int
        L.or_fd5.argtypes = [ctypes.c_int, dp, dp]
        L.or_means.argtypes = [ctypes.c_int] * 4 + [dp, dp]
        L.or_onepoint.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, ctypes.c_double,
                                                       ctypes.c_double, ctypes.c_double, ip, dp]
        L.or_pairs.argtypes = ([ctypes.c_int] * 4 + [dp, dp] + [ctypes.c_double] * 3
                               + [ctypes.c_int, ip, ip, dp, ctypes.c_int])
        for f in (L.or_fft1, L.or_fd5, L.or_means, L.or_onepoint, L.or_pairs):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the oracle; returns the count in effect."""
    return lib().or_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def fft1(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """The oracle's own unnormalised 1-D DFT with exp(sign*2*pi*i*n*k/N)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    rc = lib().or_fft1(x.size, _dp(x.view(np.float64)), _dp(out.view(np.float64)), int(sign))
    assert rc == 0
    return out


def fd5_matrix(y: np.ndarray) -> np.ndarray:
    """Dense five-point first-derivative operator on the grid y."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    D = np.zeros((y.size, y.size))
    rc = lib().or_fd5(y.size, _dp(y), _dp(D))
    if rc:
        raise ValueError("five-point stencil needs at least 5 nodes")
    return D


def _as_snap(snap: np.ndarray) -> np.ndarray:
    if snap.ndim != 5 or snap.shape[1] != 4:
        raise ValueError("snapshots must be [S][4][ny][nz][nx]")
    return np.ascontiguousarray(snap, dtype=np.float64)


def _held(snap, y, held):
    """Global plane index of each plane the snapshot array holds."""
    if held is None:
        if snap.shape[2] != y.size:
            raise ValueError("the snapshots must hold every plane of y (or pass held=)")
        return list(range(y.size))
    held = [int(j) for j in held]
    if len(held) != snap.shape[2] or sorted(set(held)) != held:
        raise ValueError("held must list the snapshot planes in increasing order")
    return held


def stencil_closure(y: np.ndarray, planes) -> list:
    """The planes plus the five-point stencil nodes of each of them: the
    planes an ensemble must hold for the terms of pairs on `planes`."""
    D = fd5_matrix(y)
    out = set(int(j) for j in planes)
    for j in list(out):
        out.update(int(m) for m in np.nonzero(D[j])[0])
    return sorted(out)


def step1(snap: np.ndarray, y: np.ndarray, lx: float, lz: float, nu: float,
          planes=None, means=None, held=None) -> np.ndarray:
    """Profiles [NPROF][ny]: U V W P S=dU/dy <q> <uv> <pv> Tx Ty Tz eps.

    planes: optional iterable of plane indices; the one-point moments are then
    computed on those planes only (the other rows of q..eps are left 0).
    means: optional [4][ny] means to use instead of the ensemble means.
    held: optional increasing global indices of the planes `snap` holds (a
    subset of the grid y); the profiles are then [NPROF][len(held)] in that
    order, `planes` and `means` refer to the held planes, and S and eps are
    valid on the planes whose five-point stencil is held.
    """
    snap = _as_snap(snap)
    ns, _, ny, nz, nx = snap.shape
    held = _held(snap, np.asarray(y), held)
    if means is None:
        means = np.zeros((4, ny))
        lib().or_means(nx, ny, nz, ns, _dp(snap), _dp(means))
    else:
        means = np.ascontiguousarray(np.asarray(means, dtype=np.float64)[:4])
    D = np.ascontiguousarray(fd5_matrix(y)[np.ix_(held, held)])
    prof = np.zeros((NPROF, ny))
    mask = None
    if planes is not None:
        mask = np.zeros(ny, dtype=np.int32)
        mask[np.asarray(list(planes), dtype=np.int64)] = 1
    rc = lib().or_onepoint(nx, ny, nz, ns, _dp(snap), _dp(means), _dp(D),
                           float(lx), float(lz), float(nu),
                           _ip(mask) if mask is not None else None, _dp(prof))
    assert rc == 0
    return prof


def _raw_pairs(snap, prof, lx, lz, nu, pairs, nthreads):
    ns, _, ny, nz, nx = snap.shape
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    y1 = np.ascontiguousarray(pairs[:, 0])
    y2 = np.ascontiguousarray(pairs[:, 1])
    out = np.zeros((len(pairs), NT, nz, nx))
    prof = np.ascontiguousarray(prof, dtype=np.float64)
    rc = lib().or_pairs(nx, ny, nz, ns, _dp(snap), _dp(prof), float(lx), float(lz), float(nu),
                        len(pairs), _ip(y1), _ip(y2), _dp(out), int(nthreads or 0))
    if rc:
        raise RuntimeError(f"or_pairs failed ({rc})")
    return out


def pair_terms(snap: np.ndarray, y: np.ndarray, lx: float, lz: float, nu: float,
               pairs, prof: np.ndarray | None = None, nthreads: int | None = None,
               held=None):
    """All 14 term maps for each ordered pair (Y1, Y2): array [npairs][14][nz][nx].

    T6 and T11 (Step 3) use T1 on the five-point stencil neighbours along Y1
    and Y2, which are computed as extra pairs.
    held: optional increasing global indices of the planes `snap` holds; pairs
    are global indices and the snapshots must hold stencil_closure of their
    planes (prof, when given, is then in held order).  The arithmetic is the
    same as with every plane held.
    """
    snap = _as_snap(snap)
    y = np.asarray(y, dtype=np.float64)
    held = _held(snap, y, held)
    loc = {g: i for i, g in enumerate(held)}
    D = fd5_matrix(y)
    pairs = [tuple(int(v) for v in p) for p in np.asarray(pairs).reshape(-1, 2)]
    missing = sorted(set(stencil_closure(y, {j for pr in pairs for j in pr})) - set(held))
    if missing:
        raise ValueError(f"the snapshots do not hold planes {missing}")
    need = list(dict.fromkeys(pairs))
    for (j1, j2) in pairs:
        for m in np.nonzero(D[j1])[0]:
            need.append((int(m), j2))
        for m in np.nonzero(D[j2])[0]:
            need.append((j1, int(m)))
    need = list(dict.fromkeys(need))
    if prof is None:
        planes = sorted({loc[j] for pr in need for j in pr})
        prof = step1(snap, y, lx, lz, nu, planes=planes, held=held)
    index = {p: i for i, p in enumerate(need)}
    raw = _raw_pairs(snap, prof, lx, lz, nu, [(loc[a], loc[b]) for (a, b) in need], nthreads)
    out = np.empty((len(pairs),) + raw.shape[1:])
    for k, (j1, j2) in enumerate(pairs):
        o = raw[index[(j1, j2)]].copy()
        d1 = sum(D[j1, m] * raw[index[(int(m), j2)], 0] for m in np.nonzero(D[j1])[0])
        d2 = sum(D[j2, m] * raw[index[(j1, int(m))], 0] for m in np.nonzero(D[j2])[0])
        o[5] = -nu * (d2 - d1)          # -2 nu * (d/dY2 - d/dY1)/2 <du^2>
        o[10] = -0.5 * nu * (d1 + d2)   # -(nu/2) (d/dY1 + d/dY2) <du^2>
        out[k] = o
    return out


# Sign of each term under the statistical reflection about the centreline,
# (u, v, w, p)(x, y, z) -> (u, -v, w, p)(x, 2h - y, z), at fixed (rx, rz):
#   T_i(Y1, Y2) = SIGMA_Y[i] * T_i(2h - Y1, 2h - Y2)
# (Section "Exploiting symmetries": every term is symmetric or antisymmetric
# under the inversion of y).  A term flips when it carries an odd number of
# wall-normal components (v, d/dy or r_y): the r_y fluxes T5, T6 and the
# Y fluxes T9, T10, T11.
SIGMA_Y = np.array([+1, +1, +1, +1, -1, -1, +1, +1, -1, -1, -1, +1, +1, +1], dtype=np.float64)


def mirror_terms(snap: np.ndarray, y: np.ndarray, lx: float, lz: float, nu: float,
                 pairs, prof: np.ndarray | None = None, nthreads: int | None = None,
                 held=None):
    """Terms of each ordered pair averaged with those of the reflected pair
    (Section "Step 2": the other half of the channel doubles the sample):
        Tbar(Y1, Y2) = (T(Y1, Y2) + SIGMA_Y * T(2h - Y1, 2h - Y2)) / 2,
    same (rx, rz).  The y grid must be symmetric about the centreline, so the
    reflected plane of index j is Ny - 1 - j.  Returns [npairs][14][nz][nx]."""
    ny = np.asarray(y).size
    pairs = [tuple(int(v) for v in p) for p in np.asarray(pairs).reshape(-1, 2)]
    refl = [(ny - 1 - a, ny - 1 - b) for (a, b) in pairs]
    t = pair_terms(snap, y, lx, lz, nu, pairs + refl, prof=prof, nthreads=nthreads, held=held)
    n = len(pairs)
    return 0.5 * (t[:n] + SIGMA_Y[None, :, None, None] * t[n:])


def _spectral_dr(f: np.ndarray, length: float, axis: int) -> np.ndarray:
    """Spectral derivative of a real periodic map along one separation axis
    (numpy's FFT as a library step), zero multiplier at the Nyquist index."""
    n = f.shape[axis]
    k = np.fft.fftfreq(n, d=1.0 / n)
    mult = 2.0 * np.pi * k / length
    if n % 2 == 0:
        mult[n // 2] = 0.0
    shape = [1] * f.ndim
    shape[axis] = n
    F = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(1j * mult.reshape(shape) * F, axis=axis))


def residual(snap: np.ndarray, y: np.ndarray, lx: float, lz: float, nu: float, pairs,
             prof: np.ndarray | None = None, nthreads: int | None = None, held=None,
             parts: bool = False):
    """Residual of the budget in conservative form (eq. GKE-conservative),
        div_r Phi + d phi / dY - xi,
    for each ordered pair (Y1, Y2): array [npairs][nz][nx] over the full
    periodic (rz, rx) plane, from the oracle's own term maps (pair_terms) of
    the pairs and of their five-point neighbour pairs, by residual_of_maps.
    With held=, the snapshots must hold the stencil closure of the stencil
    closure of the pairs' planes."""
    y = np.asarray(y, dtype=np.float64)
    ring = neighbour_pairs(y, pairs)
    T = pair_terms(snap, y, lx, lz, nu, ring, prof=prof, nthreads=nthreads, held=held)
    idx = {p: i for i, p in enumerate(ring)}
    return residual_of_maps(lambda p: T[idx[p]], y, lx, lz, pairs, parts=parts)


def neighbour_pairs(y: np.ndarray, pairs) -> list:
    """The pairs and their five-point neighbours along Y1 and along Y2."""
    D = fd5_matrix(y)
    pairs = [tuple(int(v) for v in p) for p in np.asarray(pairs).reshape(-1, 2)]
    ring = list(pairs)
    for (j1, j2) in pairs:
        ring += [(int(m), j2) for m in np.nonzero(D[j1])[0]]
        ring += [(j1, int(m)) for m in np.nonzero(D[j2])[0]]
    return list(dict.fromkeys(ring))


def residual_of_maps(maps, y: np.ndarray, lx: float, lz: float, pairs, parts: bool = False):
    """The residual operator applied to given term maps: maps(pair) returns
    the 14 full-plane maps [14][nz][nx] of an ordered pair and is called for
    the pairs and their neighbour_pairs.  Phi_rx = T2 + T3 + T4,
    Phi_ry = T5 + T6, Phi_rz = T7 + T8, phi = T9 + T10 + T11,
    xi = T12 + T13 + T14.  The r_x and r_z derivatives are spectral (Section
    "GKE and turbulence physics": the homogeneous derivatives are spectral,
    the wall-normal ones use the same finite differences as elsewhere); with
    Y1, Y2 as the variables (Section "Step 3"), d/dry = (d/dY2 - d/dY1)/2 and
    d/dY = d/dY1 + d/dY2, each d/dYk the five-point stencil applied to the
    maps of the neighbour pairs along that index.  parts=True also returns the
    four parts [npairs][4][nz][nx]: the r_x + r_z divergence, the r_y
    divergence, the Y derivative of phi, and xi (residual = the first three
    minus xi)."""
    y = np.asarray(y, dtype=np.float64)
    D = fd5_matrix(y)
    pairs = [tuple(int(v) for v in p) for p in np.asarray(pairs).reshape(-1, 2)]
    phi_ry = lambda p: maps(p)[4] + maps(p)[5]
    phi_y = lambda p: maps(p)[8] + maps(p)[9] + maps(p)[10]
    first = maps(pairs[0])
    out = np.empty((len(pairs),) + first.shape[1:])
    part = np.empty((len(pairs), 4) + first.shape[1:])
    for k, (j1, j2) in enumerate(pairs):
        t = maps((j1, j2))
        div_xz = (_spectral_dr(t[1] + t[2] + t[3], lx, axis=1)
                  + _spectral_dr(t[6] + t[7], lz, axis=0))
        d1 = lambda f: sum(D[j1, m] * f((int(m), j2)) for m in np.nonzero(D[j1])[0])
        d2 = lambda f: sum(D[j2, m] * f((j1, int(m))) for m in np.nonzero(D[j2])[0])
        div_y = 0.5 * (d2(phi_ry) - d1(phi_ry))
        dphi = d1(phi_y) + d2(phi_y)
        xi = t[11] + t[12] + t[13]
        part[k] = (div_xz, div_y, dphi, xi)
        out[k] = div_xz + div_y + dphi - xi
    return (out, part) if parts else out


def sample_indices(n: int, t1: int, t2: int, s1: int, s2: int, half: bool) -> list:
    """Grid indices of the separations kept by the two-threshold undersampling
    (Section "Undersampling and parallelisation": full resolution below the
    first threshold, one point in s1 between the thresholds, one in s2 above
    the second; readings: thresholds and steps in grid-index units, steps
    counted from zero separation, applied to |separation|).  Indices 0..n/2
    (half=True, the rx >= 0 half plane) or 0..n-1 (signed separation n - N for
    indices past N/2), increasing."""
    out = []
    for i in range(n // 2 + 1 if half else n):
        k = abs(i if i <= n // 2 else i - n)
        if k < t1 or (k < t2 and k % s1 == 0) or (k >= t2 and k % s2 == 0):
            out.append(i)
    return out


def all_pairs(ny: int):
    return [(a, b) for a in range(ny) for b in range(ny)]
