"""Device-memory plumbing around the C ABI: torch allocates the workspace and
the output maps and supplies the stream; the HIP library does the work.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gke


class GkeRun:
    """One plan with its torch-owned workspace.

    Usage: r = GkeRun(nx, ny, nz, y, lx, lz, nu, dtype=..., chunk=...);
    r.scan1(snapshots); r.scan2(snapshots); maps = r.finalize().
    """

    def __init__(self, nx, ny, nz, y, lx, lz, nu, *, dtype="f64", precision="fp64",
                 chunk=64, pair_batch=0, mirror=0, domain=0, slab=0, device="cuda",
                 stream=None, static_workspace=False, residual=False, undersample=None,
                 host_staging=0, step1=False, shapes=None):
        self.nx, self.ny, self.nz = nx, ny, nz
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.plan = gke.gke_plan(nx, ny, nz, y, lx, lz, nu)
        gke.gke_set_option(self.plan, gke.GKE_OPT_DTYPE,
                           gke.GKE_DTYPE_F32 if dtype == "f32" else gke.GKE_DTYPE_F64)
        gke.gke_set_option(self.plan, gke.GKE_OPT_PRECISION,
                           gke.GKE_PREC_BF16X3 if precision == "bf16x3" else gke.GKE_PREC_FP64)
        gke.gke_set_option(self.plan, gke.GKE_OPT_CHUNK, int(chunk))
        gke.gke_set_option(self.plan, gke.GKE_OPT_PAIR_BATCH, int(pair_batch))
        gke.gke_set_option(self.plan, gke.GKE_OPT_MIRROR, int(mirror))
        gke.gke_set_option(self.plan, gke.GKE_OPT_DOMAIN, int(domain))
        gke.gke_set_option(self.plan, gke.GKE_OPT_SLAB, int(slab))
        gke.gke_set_option(self.plan, gke.GKE_OPT_RESIDUAL, 1 if residual else 0)
        gke.gke_set_option(self.plan, gke.GKE_OPT_HOST_STAGING, int(host_staging))
        gke.gke_set_option(self.plan, gke.GKE_OPT_STEP1, 1 if step1 else 0)
        # block shapes from the autotuner: {"zplanes": n, "kzpairs": n, "kxtrans": n}
        keys = {"zplanes": gke.GKE_OPT_TUNE_ZPLANES, "kzpairs": gke.GKE_OPT_TUNE_KZPAIRS,
                "kxtrans": gke.GKE_OPT_TUNE_KXTRANS}
        for k, v in (shapes or {}).items():
            gke.gke_set_option(self.plan, keys[k], int(v))
        # undersampling: {0: (t1, t2, s1, s2) for rx, 1: (...) for rz}
        for d_, u in (undersample or {}).items():
            gke.gke_set_undersampling(self.plan, int(d_), *[int(v) for v in u])
        self.domain = int(domain)
        self.general = bool(mirror or domain or slab)
        gke.gke_set_stream(self.plan, self.stream.cuda_stream)
        if static_workspace:
            # the library's own device workspace: nothing allocated here
            self.workspace = None
            with torch.cuda.device(self.device):
                gke.gke_set_static_workspace(self.plan)
        else:
            nbytes = gke.gke_workspace_size(self.plan)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            gke.gke_set_workspace(self.plan, aligned, nbytes)
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.rx_kept = gke.gke_sample_indices(self.plan, 0)
        self.rz_kept = gke.gke_sample_indices(self.plan, 1)

    def accumulate(self, u, v, w, p):
        for t in (u, v, w, p):
            if t.dtype != self.tdtype or not t.is_contiguous() or t.device != self.device:
                raise ValueError("fields must be contiguous device tensors of the plan dtype")
            if tuple(t.shape) != (self.ny, self.nz, self.nx):
                raise ValueError("fields must be [ny][nz][nx]")
        gke.gke_accumulate(self.plan, u.data_ptr(), v.data_ptr(), w.data_ptr(), p.data_ptr())

    def accumulate_snapshot(self, snap):
        """snap: device tensor [4][ny][nz][nx]."""
        self.accumulate(snap[0], snap[1], snap[2], snap[3])

    def accumulate_batch(self, snaps):
        """snaps: device tensor [n][4][ny][nz][nx], accumulated as one graph."""
        if snaps.dtype != self.tdtype or not snaps.is_contiguous() or snaps.device != self.device:
            raise ValueError("snapshots must be a contiguous device tensor of the plan dtype")
        if tuple(snaps.shape[1:]) != (4, self.ny, self.nz, self.nx):
            raise ValueError("snapshots must be [n][4][ny][nz][nx]")
        ptr = [[snaps[i, f].data_ptr() for i in range(snaps.shape[0])] for f in range(4)]
        gke.gke_accumulate_batch(self.plan, *ptr)

    def begin_stats(self):
        gke.gke_begin_stats(self.plan)

    def set_means(self, U, V, W, P):
        gke.gke_set_means(self.plan, U, V, W, P)

    def alloc_terms(self, which=None, slab=0, dtype=torch.float64, host=False):
        """Output maps for gke_finalize (of `slab` in the general modes); host=True:
        pinned host arrays (for a plan with host staging)."""
        which = range(gke.GKE_NTERMS) if which is None else which
        kw = dict(dtype=dtype, pin_memory=True) if host else dict(dtype=dtype, device=self.device)
        nq, npx = len(self.rz_kept), len(self.rx_kept)
        if self.general:
            n = len(gke.gke_slab_pairs(self.plan, slab))
            shape, s14 = (n, nq, npx), (n,)
        else:
            shape, s14 = (self.ny, self.ny, nq, npx), (self.ny, self.ny)
        out = [None] * gke.GKE_NTERMS
        for i in which:
            out[i] = torch.empty(s14 if i == 13 else shape, **kw)
        return out

    def chunk(self) -> int:
        """Snapshots per cross-spectral batch in effect (resolves chunk 0)."""
        return gke.gke_get_option(self.plan, gke.GKE_OPT_CHUNK)

    def slab_count(self) -> int:
        return gke.gke_slab_count(self.plan)

    def slab_pairs(self, slab: int) -> np.ndarray:
        return gke.gke_slab_pairs(self.plan, slab)

    def begin_slab(self, slab: int):
        gke.gke_begin_slab(self.plan, slab)

    def alloc_residual(self):
        """A map for the budget residual, laid out like the all-pairs term maps."""
        return torch.empty((self.ny, self.ny, len(self.rz_kept), len(self.rx_kept)),
                           dtype=torch.float64, device=self.device)

    def finalize(self, out=None, residual=None):
        """Write the maps into `out` (device or pinned host tensors, all FP64 or
        all FP32); host maps are complete after wait_outputs()."""
        if out is None:
            out = self.alloc_terms()
        ts = [t for t in out if t is not None]
        host = not ts[0].is_cuda
        f32 = ts[0].dtype == torch.float32
        for t in ts + ([residual] if residual is not None else []):
            if t.is_cuda == host or (t.dtype == torch.float32) != f32 or not t.is_contiguous():
                raise ValueError("output maps must share one placement and one dtype")
        gke.gke_finalize(self.plan, [t.data_ptr() if t is not None else 0 for t in out],
                         residual=residual.data_ptr() if residual is not None else 0,
                         on_device=0 if host else 1,
                         dtype=gke.GKE_OUT_F32 if f32 else gke.GKE_OUT_F64)
        return out

    def wait_outputs(self):
        gke.gke_wait_outputs(self.plan)

    def save_state(self) -> torch.Tensor:
        """The scan state (flushing the current chunk) as a host uint8 tensor."""
        n = gke.gke_state_size(self.plan)
        buf = torch.empty(n, dtype=torch.uint8)
        gke.gke_save_state(self.plan, buf.data_ptr(), n)
        return buf

    def load_state(self, buf: torch.Tensor):
        if buf.device.type != "cpu" or buf.dtype != torch.uint8 or not buf.is_contiguous():
            raise ValueError("state must be a contiguous host uint8 tensor")
        gke.gke_load_state(self.plan, buf.data_ptr(), buf.numel())

    def on_slab(self, fn):
        """fn(slab) once per finalize when its maps are complete (None: off)."""
        self._slab_cb = gke.gke_set_slab_callback(self.plan, fn)

    def reset(self):
        gke.gke_reset(self.plan)

    def set_timing(self, on: bool):
        gke.gke_set_option(self.plan, gke.GKE_OPT_TIMING, 1 if on else 0)

    def timings(self, reset=False):
        return gke.gke_timings(self.plan, reset)

    def profiles(self) -> np.ndarray:
        return gke.gke_get_profiles(self.plan, self.ny)

    def close(self):
        if self.plan is not None:
            gke.gke_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_snapshots(snaps_dev, y, lx, lz, nu, *, dtype="f64", precision="fp64", chunk=64,
                  pair_batch=0, which=None, residual=False, undersample=None):
    """Both scans over a device tensor [S][4][ny][nz][nx]; returns (maps,
    profiles), or (maps, profiles, residual map) with residual=True."""
    S, _, ny, nz, nx = snaps_dev.shape
    r = GkeRun(nx, ny, nz, y, lx, lz, nu, dtype=dtype, precision=precision, chunk=chunk,
               pair_batch=pair_batch, device=snaps_dev.device, residual=residual,
               undersample=undersample)
    for s in range(S):
        r.accumulate_snapshot(snaps_dev[s])
    r.begin_stats()
    for s in range(S):
        r.accumulate_snapshot(snaps_dev[s])
    res = r.alloc_residual() if residual else None
    out = r.finalize(r.alloc_terms(which), residual=res)
    prof = r.profiles()
    r.close()
    return (out, prof, res) if residual else (out, prof)


def run_slabs(snaps_dev, y, lx, lz, nu, *, dtype="f64", precision="fp64", chunk=64,
              pair_batch=0, mirror=0, domain=0, slab=0, which=None, undersample=None,
              out_dtype=None, host=False):
    """Both scans, then one second scan and finalize per slab.  Returns
    ([(pairs [n][2], maps of the slab)], profiles); maps as gke_finalize lays
    them out for the general modes, of torch dtype out_dtype (FP64 default),
    on the device or (host=True) in pinned host memory streamed per slab."""
    S, _, ny, nz, nx = snaps_dev.shape
    r = GkeRun(nx, ny, nz, y, lx, lz, nu, dtype=dtype, precision=precision, chunk=chunk,
               pair_batch=pair_batch, mirror=mirror, domain=domain, slab=slab,
               device=snaps_dev.device, undersample=undersample, host_staging=2 if host else 0)
    for s in range(S):
        r.accumulate_snapshot(snaps_dev[s])
    r.begin_stats()
    res = []
    for sl in range(r.slab_count()):
        if sl > 0:
            r.begin_slab(sl)
        for s in range(S):
            r.accumulate_snapshot(snaps_dev[s])
        out = r.finalize(r.alloc_terms(which, slab=sl, dtype=out_dtype or torch.float64,
                                       host=host))
        res.append((r.slab_pairs(sl), out))
    r.wait_outputs()
    prof = r.profiles()
    r.close()
    return res, prof
