"""Thin ctypes binding of the C ABI in include/gke.h (same names, marshalling only).

Every computation happens in the HIP library ``libgke.so``; this module only
converts arguments.  Loading fails loudly when the library is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GKE_LIBRARY may name another build of the same library (other block shapes)
LIB_PATH = os.environ.get("GKE_LIBRARY") or os.path.join(_HERE, "libgke.so")

GKE_OK, GKE_ERR_ARG, GKE_ERR_STATE, GKE_ERR_OOM, GKE_ERR_HIP, GKE_ERR_UNSUPPORTED = range(6)
GKE_OPT_DTYPE, GKE_OPT_PRECISION, GKE_OPT_CHUNK, GKE_OPT_PAIR_BATCH, GKE_OPT_TIMING = 1, 2, 3, 4, 5
GKE_OPT_MIRROR, GKE_OPT_DOMAIN, GKE_OPT_SLAB, GKE_OPT_RESIDUAL = 6, 7, 8, 9
GKE_OPT_HOST_STAGING, GKE_OPT_STEP1 = 10, 11
GKE_OPT_TUNE_ZPLANES, GKE_OPT_TUNE_KZPAIRS, GKE_OPT_TUNE_KXTRANS = 12, 13, 14
GKE_OUT_F64, GKE_OUT_F32 = 0, 1
GKE_DOMAIN_ALLPAIRS_HALFRX, GKE_DOMAIN_Y1LEY2_FULLR, GKE_DOMAIN_FUNDAMENTAL_FULLR = 0, 1, 2
GKE_DTYPE_F64, GKE_DTYPE_F32 = 0, 1
GKE_PREC_FP64, GKE_PREC_BF16X3 = 0, 1
GKE_NTERMS = 14
GKE_NPROF = 12
TERM_NAMES = ["du2", "phix_t", "phix_m", "phix_v", "phiy_t", "phiy_v", "phiz_t", "phiz_v",
              "phi_t", "phi_p", "phi_v", "xi_p1", "xi_p2", "xi_d"]
PROFILE_NAMES = ["U", "V", "W", "P", "S", "q", "uv", "pv", "Tx", "Ty", "Tz", "eps"]
KERNEL_NAMES = ["plane_sums", "fluct_xfft", "zfft_pack", "rankk", "fin_kz", "fin_kx", "fd_terms",
                "small", "rankk_rem", "resid", "step1"]
GKE_NKERNELS = len(KERNEL_NAMES)


class GkeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gke status {status}: {msg}")
        self.status = status


class gke_terms(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p * GKE_NTERMS), ("on_device", ctypes.c_int),
                ("dtype", ctypes.c_int), ("residual", ctypes.c_void_p)]


_lib = None


# gke_slab_fn: void (*)(int slab, void *user)
SLAB_FN = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.c_void_p)


def lib() -> ctypes.CDLL:
    """Load libgke.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1910_06409_amd/csrc/build.py`")
    try:
        import torch  # noqa: F401  (loads the HIP runtime first)
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    vp, i32, i64, dp, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                            ctypes.POINTER(ctypes.c_double), ctypes.c_size_t)
    sig = {
        "gke_plan": ([i32, i32, i32, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                      ctypes.POINTER(vp)], i32),
        "gke_set_option": ([vp, i32, i64], i32),
        "gke_get_option": ([vp, i32, ctypes.POINTER(i64)], i32),
        "gke_workspace_size": ([vp, ctypes.POINTER(sz)], i32),
        "gke_set_workspace": ([vp, vp, sz], i32),
        "gke_set_static_workspace": ([vp], i32),
        "gke_set_undersampling": ([vp, i32, i32, i32, i32, i32], i32),
        "gke_sample_indices": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "gke_set_stream": ([vp, vp], i32),
        "gke_accumulate": ([vp, vp, vp, vp, vp], i32),
        "gke_accumulate_batch": ([vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), ctypes.POINTER(vp)], i32),
        "gke_begin_stats": ([vp], i32),
        "gke_set_means": ([vp, dp, dp, dp, dp], i32),
        "gke_finalize": ([vp, ctypes.POINTER(gke_terms)], i32),
        "gke_wait_outputs": ([vp], i32),
        "gke_set_slab_callback": ([vp, SLAB_FN, vp], i32),
        "gke_state_size": ([vp, ctypes.POINTER(sz)], i32),
        "gke_save_state": ([vp, vp, sz], i32),
        "gke_load_state": ([vp, vp, sz], i32),
        "gke_reconstruct": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "gke_get_profiles": ([vp, dp], i32),
        "gke_slab_count": ([vp, ctypes.POINTER(i32)], i32),
        "gke_slab_pairs": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "gke_begin_slab": ([vp, i32], i32),
        "gke_reset": ([vp], i32),
        "gke_timings": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                         i32], i32),
        "gke_destroy": ([vp], None),
        "gke_last_error": ([vp], ctypes.c_char_p),
        "gke_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int, plan) -> None:
    if status != GKE_OK:
        raise GkeError(status, gke_last_error(plan))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gke_last_error(plan) -> str:
    s = lib().gke_last_error(plan)
    return s.decode() if s else ""


def gke_version() -> str:
    return lib().gke_version().decode()


def gke_plan(Nx: int, Ny: int, Nz: int, y, Lx: float, Lz: float, nu: float):
    y = np.ascontiguousarray(y, dtype=np.float64)
    if y.size != Ny:
        raise ValueError("y must have Ny entries")
    out = ctypes.c_void_p()
    _check(lib().gke_plan(Nx, Ny, Nz, _dp(y), Lx, Lz, nu, ctypes.byref(out)), None)
    return out


def gke_set_option(plan, key: int, value: int) -> None:
    _check(lib().gke_set_option(plan, key, value), plan)


def gke_get_option(plan, key: int) -> int:
    v = ctypes.c_int64()
    _check(lib().gke_get_option(plan, key, ctypes.byref(v)), plan)
    return v.value


def gke_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(lib().gke_workspace_size(plan, ctypes.byref(n)), plan)
    return n.value


def gke_set_workspace(plan, device_ptr: int, nbytes: int) -> None:
    _check(lib().gke_set_workspace(plan, device_ptr, nbytes), plan)


def gke_set_static_workspace(plan) -> None:
    _check(lib().gke_set_static_workspace(plan), plan)


GKE_STATIC_WORKSPACE_BYTES = 64 << 20


def gke_set_undersampling(plan, dir_: int, t1: int, t2: int, s1: int, s2: int) -> None:
    _check(lib().gke_set_undersampling(plan, dir_, t1, t2, s1, s2), plan)


def gke_sample_indices(plan, dir_: int) -> np.ndarray:
    """Kept output indices along rx (dir 0) or rz (dir 1)."""
    n = ctypes.c_int()
    _check(lib().gke_sample_indices(plan, dir_, ctypes.byref(n), None), plan)
    out = np.zeros(max(n.value, 1), dtype=np.int32)
    _check(lib().gke_sample_indices(plan, dir_, ctypes.byref(n),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), plan)
    return out[:n.value]


def gke_set_stream(plan, stream_ptr: int) -> None:
    _check(lib().gke_set_stream(plan, stream_ptr), plan)


def gke_accumulate(plan, u: int, v: int, w: int, p: int) -> None:
    _check(lib().gke_accumulate(plan, u, v, w, p), plan)


def gke_reconstruct(plan, vhat: int, ohat: int, mean_u: int, mean_w: int, u: int, v: int,
                    w: int, p: int) -> None:
    """Device pointers (int): see include/gke.h."""
    _check(lib().gke_reconstruct(plan, vhat, ohat, mean_u, mean_w, u, v, w, p), plan)


def gke_accumulate_batch(plan, u, v, w, p) -> None:
    """u, v, w, p: sequences of n device pointers (int)."""
    n = len(u)
    arr = [(ctypes.c_void_p * n)(*[int(x) for x in a]) for a in (u, v, w, p)]
    _check(lib().gke_accumulate_batch(plan, n, *arr), plan)


def gke_begin_stats(plan) -> None:
    _check(lib().gke_begin_stats(plan), plan)


def gke_set_means(plan, U, V, W, P) -> None:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (U, V, W, P)]
    _check(lib().gke_set_means(plan, *[_dp(a) for a in arrs]), plan)


def gke_finalize(plan, ptrs, residual: int = 0, on_device: int = 1,
                 dtype: int = GKE_OUT_F64) -> None:
    """ptrs: sequence of 14 pointers (int) or None for terms to skip;
    residual: pointer of the budget residual map, or 0."""
    t = gke_terms()
    for i in range(GKE_NTERMS):
        t.t[i] = ptrs[i] if ptrs[i] else None
    t.on_device = int(on_device)
    t.dtype = int(dtype)
    t.residual = residual if residual else None
    _check(lib().gke_finalize(plan, ctypes.byref(t)), plan)


def gke_wait_outputs(plan) -> None:
    _check(lib().gke_wait_outputs(plan), plan)


def gke_state_size(plan) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().gke_state_size(plan, ctypes.byref(n)), plan)
    return n.value


def gke_save_state(plan, host_ptr: int, nbytes: int) -> None:
    """Flush the current chunk and copy the scan state into host memory."""
    _check(lib().gke_save_state(plan, host_ptr, nbytes), plan)


def gke_load_state(plan, host_ptr: int, nbytes: int) -> None:
    _check(lib().gke_load_state(plan, host_ptr, nbytes), plan)


def gke_set_slab_callback(plan, fn):
    """Call fn(slab) once per gke_finalize when its maps are complete (on a HIP
    runtime thread; fn must not call HIP or the library); fn=None removes it.
    Returns the ctypes callback, which the caller keeps alive while it is set."""
    cb = SLAB_FN(lambda slab, _user: fn(int(slab))) if fn is not None else SLAB_FN()
    _check(lib().gke_set_slab_callback(plan, cb, None), plan)
    return cb


def gke_get_profiles(plan, ny: int) -> np.ndarray:
    out = np.zeros((GKE_NPROF, ny))
    _check(lib().gke_get_profiles(plan, _dp(out)), plan)
    return out


def gke_slab_count(plan) -> int:
    n = ctypes.c_int()
    _check(lib().gke_slab_count(plan, ctypes.byref(n)), plan)
    return n.value


def gke_slab_pairs(plan, slab: int) -> np.ndarray:
    """Output pairs of a slab in layout order, int array [n][2] of (Y1, Y2)."""
    n = ctypes.c_int()
    _check(lib().gke_slab_pairs(plan, slab, ctypes.byref(n), None), plan)
    out = np.zeros((n.value, 2), dtype=np.int32)
    _check(lib().gke_slab_pairs(plan, slab, ctypes.byref(n),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), plan)
    return out


def gke_begin_slab(plan, slab: int) -> None:
    _check(lib().gke_begin_slab(plan, slab), plan)


def gke_reset(plan) -> None:
    _check(lib().gke_reset(plan), plan)


def gke_timings(plan, reset: bool = False):
    """{kernel family: (total ms, launches)} since the last counter reset."""
    ms = (ctypes.c_double * GKE_NKERNELS)()
    n = (ctypes.c_int64 * GKE_NKERNELS)()
    _check(lib().gke_timings(plan, ms, n, 1 if reset else 0), plan)
    return {KERNEL_NAMES[i]: (ms[i], n[i]) for i in range(GKE_NKERNELS)}


def gke_destroy(plan) -> None:
    lib().gke_destroy(plan)
