#!/usr/bin/env python3
"""Throughput of the GKE two-point-statistics hot path on one MI355X.

A step is one pass of the whole path over one ensemble of synthetic
snapshots already resident in HBM: the first scan (plane sums -> means),
the second scan (fluctuations, products, forward transforms, cross-spectral
rank-k accumulation) and finalize (inverse transforms, FP64 assembly of the
14 term maps, five-point Y derivatives).

value = P_out * S / T_step   [(Y1, Y2, rx, rz) points x snapshots per second]
with P_out = Ny^2 (Nx/2 + 1) Nz points per term (all ordered pairs, rx >= 0).

Also reported: per-kernel device time from HIP events on the plan's stream,
the roofline of the dominant kernel, and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKE (y1,y2,rx,rz) term-map points/s; split-BF16 vs FP64 at stated rel. err"
UNIT = "point-snapshots/s"
# MI355X published peaks: dense MFMA (TFLOP/s), FP64 vector (TFLOP/s), HBM (GB/s)
PEAK = {"fp64_mfma": 78.6, "bf16_mfma": 2500.0, "fp64_vector": 78.6, "hbm": 8000.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_work(w, chunk):
    """Algorithmic work per launch of each kernel family (flops or bytes)."""
    ny, nx, nz, nkx, nk = w.ny, w.nx, w.nz, w.nx // 2 + 1, w.nk
    b_in = 8 if w.dtype == "f64" else 4
    n_pts = nx * ny * nz
    c16 = 16  # complex FP64
    c8 = 8 if w.precision == "bf16x3" else 16  # x-transformed values and spectra
    npair_u = ny * (ny + 1) // 2
    n16 = 16 * (ny // 16)                 # planes in full 16-plane tiles
    pairs_tiles = n16 * (n16 + 1) // 2    # unordered pairs within them
    # 27 complex MACs (216 flops) per (snapshot, wavenumber, unordered pair
    # Y1 <= Y2); the split-BF16 form takes three real products for each one
    fl = 216.0 * (3 if w.precision == "bf16x3" else 1)
    return {
        "rankk": ("flop", fl * chunk * nk * pairs_tiles),
        # pairs with a plane of the last Ny mod 16 (FP64 vector arithmetic)
        "rankk_rem": ("flop", 216.0 * chunk * nk * (npair_u - pairs_tiles)),
        # read the 4 input fields once, write the 10 x-transformed fields
        "fluct_xfft": ("byte", 4.0 * n_pts * b_in + 10.0 * ny * nkx * nz * c8),
        # read the x-transformed fields, write the 10 spectra (the split path
        # transforms the four snapshots of a quad per launch)
        "zfft_pack": ("byte", 2 * 10.0 * ny * nkx * nz * c8 * (4 if w.precision == "bf16x3" else 1)),
        "plane_sums": ("byte", 4.0 * n_pts * b_in),
        # read 8 term spectra of every unordered pair, write 9 kz-transformed
        # maps (i alpha R is formed from R in the kx pass)
        "fin_kz": ("byte", (8 + 9) * float(nk) * npair_u * c16),
        # read the 9 maps, write 12 FP64 term maps for both orientations
        "fin_kx": ("byte", 9.0 * nk * npair_u * c16 + 12.0 * ny * ny * nkx * nz * 8),
        # read <du^2>, write two maps
        "fd_terms": ("byte", 3.0 * ny * ny * nkx * nz * 8),
    }


def s8d_work(w, chunk):
    """Algorithmic work per launch on the basis of the measurement contract:
    124 real flops per (snapshot, wavenumber, ordered plane pair) for the
    cross-spectral update (15.5 complex MACs of the needed correlation set;
    three times that for the split-BF16 form), and for the HBM-bound stages
    the inputs read once and the spectra written once per snapshot (4 N b +
    10 Ny nk c bytes), and the accumulators read once plus the 14 output maps
    written once per finalize."""
    ny, nx, nz, nkx, nk = w.ny, w.nx, w.nz, w.nx // 2 + 1, w.nk
    n16 = 16 * (ny // 16)
    b_in = 8 if w.dtype == "f64" else 4
    c = 8 if w.precision == "bf16x3" else 16
    mult = 3 if w.precision == "bf16x3" else 1
    npair_u = ny * (ny + 1) // 2
    return {
        "rankk": 124.0 * mult * chunk * nk * n16 * n16,
        "rankk_rem": 124.0 * chunk * nk * (ny * ny - n16 * n16),
        # per snapshot (the two transform kernels together)
        "transforms": 4.0 * nx * ny * nz * b_in + 10.0 * ny * nk * c,
        # per finalize: 8 accumulated term spectra of every unordered pair read
        # once, 13 maps [Y1][Y2][rz][rx <= Nx/2] and T14 [Y1][Y2] written once
        "finalize": 8.0 * nk * npair_u * 16 + 13.0 * ny * ny * nkx * nz * 8 + ny * ny * 8.0,
    }


def host_info():
    """Host CPU facts recorded with the CPU baseline."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    mem = 0.0
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = float(line.split()[1]) / 2**20
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cores": avail, "cpu_model": model,
            "mem_gib": round(mem, 1), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, y, seed, threads, s_sample, j1, nb=8, s_single=2, nb_single=2):
    """The oracle on a bounded sample: S_sample snapshots, the nb x nb block of
    ordered pairs with Y1, Y2 in [j1, j1 + nb), on `threads` threads; and a
    smaller sample on one thread (the analogue of a serial run)."""
    import numpy as np

    from oracle import oracle
    from paper_1910_06409_amd import synth

    pts_pair = (w.nx // 2 + 1) * w.nz
    planes = list(range(max(0, j1 - 2), min(w.ny, j1 + nb + 2)))
    snap = np.stack([synth.snapshot(w, seed, s)[:, planes] for s in range(s_sample)])
    snap = snap.astype(np.float64)
    pairs = [(a, b) for a in range(j1, j1 + nb) for b in range(j1, j1 + nb)]
    used = oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.pair_terms(snap, y, w.lx, w.lz, w.nu, pairs, nthreads=threads, held=planes)
    dt = time.perf_counter() - t0
    p1 = pairs[:nb_single * nb_single]
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.pair_terms(np.ascontiguousarray(snap[:s_single]), y, w.lx, w.lz, w.nu,
                      [(j1 + a, j1 + b) for a in range(nb_single) for b in range(nb_single)],
                      nthreads=1, held=planes)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(used)
    res = {"value": len(pairs) * pts_pair * s_sample / dt, "unit": UNIT, "cores": used,
           "kind": "oracle", "seconds": dt,
           "sample": f"{w.name}: first {s_sample} snapshots, the {nb}x{nb} block of ordered "
                     f"pairs Y1, Y2 in [{j1}, {j1 + nb}) (plus the five-point neighbour pairs "
                     f"the oracle needs), whole oracle path incl. Step 1 on the touched "
                     f"planes; value = pairs*(Nx/2+1)*Nz*S_sample/seconds"}
    res.update(host_info())
    res["single_thread"] = {
        "value": len(p1) * pts_pair * s_single / dt1, "seconds": dt1, "cores": 1,
        "sample": f"first {s_single} snapshots, the {nb_single}x{nb_single} block of pairs "
                  f"from [{j1}, {j1 + nb_single})"}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="re200")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--chunk", type=int, default=0, help="0: one chunk for the ensemble")
    ap.add_argument("--snapshots", type=int, default=0, help="override S (0: workload's)")
    ap.add_argument("--pair-batch", type=int, default=0,
                    help="pairs per finalize batch (0: all pairs at once)")
    ap.add_argument("--precision", default="", choices=["", "fp64", "bf16x3"],
                    help="override the rank-k arithmetic of the workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (0: every core this job may use)")
    ap.add_argument("--slab-rows", type=int, default=0,
                    help="config-5 path: mirror average, fundamental domain, Y1 slabs of this "
                         "many rows (one timed pass over all slabs)")
    ap.add_argument("--host-out", action="store_true",
                    help="config-5 path: stream every slab's maps to pinned host memory")
    ap.add_argument("--also", default="re200_bf16,re200_batched",
                    help="comma-separated workloads measured after the main one (speed-up per "
                         "snapshot reported under 'extra'); empty for none")
    ap.add_argument("--also-steps", type=int, default=2)
    ap.add_argument("--graph", default="off", choices=["on", "off"],
                    help="on: the timed steps feed each scan's snapshots as one captured HIP "
                         "graph (gke_accumulate_batch) and the per-kernel times come from "
                         "extra event-timed steps; off: one gke_accumulate per snapshot with "
                         "HIP events over the timed region, and a few graph steps after it "
                         "(graph_ms_per_step)")
    ap.add_argument("--tuned", default="auto", choices=["auto", "off"],
                    help="auto: use the autotuner's cached chunk and block shapes for the "
                         "workload's shape when present (paper_1910_06409_amd/tuned.json)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device-to-device copy of MIB MiB three times "
                         "(the known-size reference for HBM traffic counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); "
              "the multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_06409_amd import profiling, runner, synth, tune

    def load_workload(name, snapshots=0, precision=""):
        w = synth.workload(name)
        if snapshots:
            w = synth.workload(name, S=snapshots)
        if precision:
            w = synth.workload(name, S=w.S, precision=precision)
        return w

    dev = torch.device("cuda", 0)

    def measure(w, steps, warmup, chunk_arg, calibrate=0):
        """Time `steps` whole-path steps of workload w; returns a result dict."""
        S = w.S
        # one batch for the whole ensemble when it is small, else the library's
        # automatic chunk (largest batch whose spectra fit its memory budget);
        # the autotuner's cached choice for this shape when there is one
        chunk = chunk_arg if chunk_arg else (S + (S & 1) if S <= 128 else 0)
        tuned = tune.load(w) if args.tuned == "auto" and S == synth.workload(w.name).S else None
        shapes = {}
        if tuned:
            if not chunk_arg:
                chunk = int(tuned["chunk"])
            shapes = {k: int(tuned[k]) for k in tune.SHAPE_KEYS if k in tuned}
            log(f"[bench] autotuned for {tune.key_of(w)}: chunk {chunk}, {shapes}")
        y = synth.y_grid(w)
        tdt = torch.float64 if w.dtype == "f64" else torch.float32
        log(f"[bench] generating {S} snapshots of {w.name} ({w.nx}x{w.ny}x{w.nz}, {w.dtype})")
        t0 = time.perf_counter()
        snaps = torch.empty((S, 4, w.ny, w.nz, w.nx), dtype=tdt, device=dev)
        gen = synth.DeviceSnapshots(w, args.seed, dev)
        for s in range(S):
            gen(s, out=snaps[s])
            if (s + 1) % 100 == 0:
                log(f"[bench]   {s + 1}/{S} snapshots resident ({time.perf_counter() - t0:.0f} s)")
        torch.cuda.synchronize()
        del gen
        r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                          precision=w.precision, chunk=chunk, pair_batch=args.pair_batch,
                          device=dev, shapes=shapes)
        chunk_used = r.chunk()
        outs = r.alloc_terms()
        log(f"[bench] workspace {r.workspace.numel() / 2**30:.1f} GiB, outputs "
            f"{sum(o.numel() for o in outs) * 8 / 2**30:.1f} GiB, chunk {chunk_used}")
        if calibrate:
            nb = calibrate << 20
            src = torch.ones(nb, dtype=torch.uint8, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"[bench] calibration copy of {nb} bytes done")
            del src, dst

        def step(graph, marks=None):
            """marks: two events recorded around the second scan and finalize
            (the span of the contract's T, from the first Step-2 accumulate to
            the return of finalize)."""
            r.reset()
            if graph:
                r.accumulate_batch(snaps)
                r.begin_stats()
                r.accumulate_batch(snaps)
            else:
                for s in range(S):
                    r.accumulate_snapshot(snaps[s])
                r.begin_stats()
                if marks:
                    marks[0].record()
                for s in range(S):
                    r.accumulate_snapshot(snaps[s])
            r.finalize(outs)
            if marks:
                marks[1].record()

        graph = args.graph == "on"
        for i in range(warmup):
            step(graph)
            log(f"[bench] warmup step {i + 1}/{warmup} done")
        # graph off: HIP events around every launch over the timed region;
        # graph on: the timed steps run the captured graphs without events and
        # the per-kernel device times come from extra event-timed steps
        r.set_timing(not graph)
        r.timings(reset=True)
        marks = [] if graph else [(torch.cuda.Event(enable_timing=True),
                                   torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(graph, marks[i] if marks else None)
            log(f"[bench] timed step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # second scan + finalize (T of the contract; pass 1 apart), per step
        t_pass2 = (sum(a.elapsed_time(b) for a, b in marks) / 1e3 / steps) if marks else None
        ksteps = steps
        if graph:
            r.set_timing(True)
            ksteps = max(1, min(steps, 3))
            for i in range(ksteps):
                step(False)
        tm = r.timings(reset=True)
        r.set_timing(False)
        graph_ms = None
        if not graph:   # the same steps as captured graphs, for comparison
            gsteps = max(1, min(steps, 3))
            step(True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for i in range(gsteps):
                step(True)
            torch.cuda.synchronize()
            graph_ms = 1e3 * (time.perf_counter() - t1) / gsteps
        r.close()
        del outs, snaps, r
        torch.cuda.empty_cache()

        t_step = elapsed / steps
        steps_k = ksteps   # the per-kernel figures below are per event-timed step
        work = kernel_work(w, chunk_used)
        s8 = s8d_work(w, chunk_used)
        kernels = {}
        for name, (ms, n) in tm.items():
            if n == 0:
                continue
            avg = ms / n
            k = {"ms_per_step": ms / steps_k, "launches_per_step": n / steps_k, "avg_launch_ms": avg}
            if name in work:
                kind, amount = work[name]
                if name in ("rankk", "rankk_rem"):
                    # the last launch of a step may hold fewer snapshots: use the mean
                    amount = amount * (S / chunk_used) / (n / steps_k)
                    k["achieved_tflops"] = (s8[name] * (S / chunk_used) / (n / steps_k)
                                            / (avg * 1e-3) / 1e12)
                    k["achieved_tflops_own_basis"] = amount / (avg * 1e-3) / 1e12
                elif kind == "flop":
                    k["achieved_tflops"] = amount / (avg * 1e-3) / 1e12
                else:
                    k["achieved_gbs"] = amount / (avg * 1e-3) / 1e9
            kernels[name] = k
        # stage rates on the contract's algorithmic bytes
        ms_of = lambda *names: sum(kernels[n]["ms_per_step"] for n in names if n in kernels)
        stages = {}
        t_tr = ms_of("fluct_xfft", "zfft_pack")
        if t_tr:
            gbs = s8["transforms"] * S / (t_tr * 1e-3) / 1e9
            stages["transforms"] = {"ms_per_step": t_tr, "bytes_per_step": s8["transforms"] * S,
                                    "achieved_gbs": gbs, "frac_hbm": gbs / PEAK["hbm"]}
        t_fin = ms_of("fin_kz", "fin_kx", "fd_terms")
        if t_fin:
            gbs = s8["finalize"] / (t_fin * 1e-3) / 1e9
            stages["finalize"] = {"ms_per_step": t_fin, "bytes_per_step": s8["finalize"],
                                  "achieved_gbs": gbs, "frac_hbm": gbs / PEAK["hbm"]}
        dom = max(kernels, key=lambda n: kernels[n]["ms_per_step"])
        dk = kernels[dom]
        extra_roof = {}
        if dom == "rankk_rem":
            # FP64 vector arithmetic: the fp64 vector peak of the chip
            ach, peak, unit, bound = dk["achieved_tflops"], PEAK["fp64_vector"], "TFLOP/s", "alu"
        elif "achieved_tflops" in dk:
            peak = PEAK["bf16_mfma" if w.precision == "bf16x3" else "fp64_mfma"]
            ach, unit, bound = dk["achieved_tflops"], "TFLOP/s", "mfma"
            extra_roof = {
                "basis": "124 flops per (snapshot, wavenumber, ordered plane pair)"
                         + (" x 3 split products" if w.precision == "bf16x3" else ""),
                "achieved_own_basis": dk.get("achieved_tflops_own_basis"),
                "own_basis": "216 flops per (snapshot, wavenumber, unordered pair): the 27 "
                             "complex products the kernel forms"
                             + (", x 3 split products" if w.precision == "bf16x3" else ""),
            }
            # matrix-core busy fraction and clock from the committed counter run
            mf = profiling.read_summary_if_current(
                os.path.join(ROOT, "profiles", f"mfma_rankk_{w.name}_{w.precision}.txt"),
                "rankk")
            if mf:
                extra_roof["mfma_busy_fraction"] = float(mf["mfma_busy_fraction"])
                extra_roof["mfma_clock_ghz"] = float(mf["clock_ghz"])
        else:
            ach, peak, unit, bound = dk.get("achieved_gbs", 0.0), PEAK["hbm"], "GB/s", "hbm"
        # HBM bytes per launch of that kernel from the committed counter summary,
        # provided its sources are unchanged since the counters were taken
        traffic = profiling.traffic_if_current(
            os.path.join(ROOT, "profiles", f"traffic_{dom}_{w.name}_{w.precision}.txt"), dom,
            w.precision) if S == synth.workload(w.name).S and chunk_arg == 0 else None
        roof = {"kernel": profiling.symbol(dom, w.precision) if dom in profiling.KERNELS else dom,
                "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                "frac": ach / peak, "traffic": traffic}
        roof.update(extra_roof)
        return {"w": w, "S": S, "chunk": chunk_used, "t_step": t_step, "kernels": kernels,
                "roofline": roof, "stages": stages, "value": w.points_out * S / t_step,
                "tuned": ({"chunk": chunk_used, **shapes} if tuned else None),
                "graph_ms_per_step": graph_ms, "t_pass2": t_pass2}

    def measure_slabs(w, slab_rows, chunk, pair_batch):
        """The config-5 path: mirror average, fundamental domain, Y1 slabs (one
        second scan per slab), every slab's maps streamed to pinned host
        memory (double-buffered device staging, copies on the library's own
        stream).  When the ensemble does not fit in HBM beside the workspace,
        every scan regenerates the snapshots on the device (the paper's
        wall-normal slices each read the whole database); the generation is
        timed apart from the library's device time."""
        S = w.S
        y = synth.y_grid(w)
        tdt = torch.float64 if w.dtype == "f64" else torch.float32
        from paper_1910_06409_amd import gke
        r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                          precision=w.precision, chunk=chunk, pair_batch=pair_batch,
                          mirror=1, domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=slab_rows,
                          device=dev, host_staging=2 if args.host_out else 0)
        nslab = r.slab_count()
        npairs = [len(r.slab_pairs(sl)) for sl in range(nslab)]
        big = int(np.argmax(npairs))
        snap_bytes = 4 * w.ny * w.nz * w.nx * (4 if w.dtype == "f32" else 8)
        free = torch.cuda.mem_get_info(dev)[0]
        out_dev = 0 if args.host_out else 14 * npairs[big] * w.nz * w.nx * 8
        resident = S * snap_bytes + out_dev < free - (8 << 30)
        log(f"[bench] workspace {r.workspace.numel() / 2**30:.1f} GiB, {nslab} slabs, chunk "
            f"{r.chunk()}, {S} snapshots {'resident' if resident else 'regenerated per scan'}")
        if resident:
            snaps = torch.empty((S, 4, w.ny, w.nz, w.nx), dtype=tdt, device=dev)
            g0 = synth.DeviceSnapshots(w, args.seed, dev)
            for s in range(S):
                g0(s, out=snaps[s])
            del g0
            gen = None
        else:
            snaps = torch.empty((2, 4, w.ny, w.nz, w.nx), dtype=tdt, device=dev)
            gen = synth.FastDeviceSnapshots(w, args.seed, dev)
        if args.host_out:   # two sets of pinned host maps, one per staging buffer
            outs = [r.alloc_terms(slab=big, host=True) for _ in range(2)]
        else:
            outs = [r.alloc_terms(slab=big)]
        per_pair_bytes = sum(o.numel() for o in outs[0] if o is not None) * 8 // npairs[big]
        log(f"[bench] slab outputs {per_pair_bytes * npairs[big] / 2**30:.1f} GiB "
            f"{'(pinned host, x2)' if args.host_out else '(device)'}")
        gen_ev = []

        def snapshot(s):
            if gen is None:
                return snaps[s]
            buf = snaps[s & 1]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            gen(s, out=buf)
            e1.record()
            gen_ev.append((e0, e1))
            return buf

        def views(sl):
            n = npairs[sl]
            return [o[:n] if o is not None else None for o in outs[sl % len(outs)]]

        torch.cuda.synchronize()
        r.set_timing(True)
        r.timings(reset=True)
        t0 = time.perf_counter()
        for s in range(S):
            r.accumulate_snapshot(snapshot(s))
        r.begin_stats()
        for sl in range(nslab):
            if sl > 0:
                r.begin_slab(sl)
            for s in range(S):
                r.accumulate_snapshot(snapshot(s))
            r.finalize(views(sl))
            log(f"[bench] slab {sl + 1}/{nslab} done ({time.perf_counter() - t0:.1f} s)")
        t_fin = time.perf_counter()
        r.wait_outputs()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tail = time.perf_counter() - t_fin
        tm = r.timings(reset=True)
        gen_s = sum(a.elapsed_time(b) for a, b in gen_ev) / 1e3
        r.close()
        del outs, snaps, r, gen
        torch.cuda.empty_cache()
        p_out = sum(npairs) * w.nz * w.nx
        lib_s = sum(v[0] for v in tm.values()) / 1e3
        return {"w": w, "S": S, "t": elapsed, "nslab": nslab, "p_out": p_out,
                "value": p_out * S / elapsed, "resident": resident,
                "generation_s": gen_s, "library_device_s": lib_s,
                "copy_tail_s": tail, "host_maps_bytes": (sum(npairs) * per_pair_bytes
                                                         if args.host_out else 0),
                "kernels_ms": {k: v[0] for k, v in tm.items() if v[1]}}

    w = load_workload(args.workload, args.snapshots, args.precision)
    if args.slab_rows:
        sr = measure_slabs(w, args.slab_rows, args.chunk or 8, args.pair_batch or 1024)
        res = {
            "metric": METRIC, "value": sr["value"], "unit": UNIT, "n_gpus": 1, "steps": 1,
            "warmup": 0, "ms_per_step": 1e3 * sr["t"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if w.precision == "fp64" else "bf16x3", "data": "synthetic",
            "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} channel grid, {sr['S']} "
                                   f"{w.dtype} snapshots, mirror average, fundamental domain "
                                   f"(full r), {sr['nslab']} Y1 slabs of {args.slab_rows} rows, "
                                   f"14 term maps"
                                   + (" streamed to pinned host memory per slab"
                                      if args.host_out else ""),
                       "points_out": sr["p_out"],
                       "snapshots_resident": sr["resident"]},
            "library_device_s": sr["library_device_s"], "generation_s": sr["generation_s"],
            "copy_tail_s": sr["copy_tail_s"], "host_maps_bytes": sr["host_maps_bytes"],
            "kernels_ms": sr["kernels_ms"],
        }
        print(json.dumps(res), flush=True)
        return
    main_res = measure(w, args.steps, args.warmup, args.chunk, args.calibrate_copy)
    S = w.S

    extra = {}
    for name in [n for n in args.also.split(",") if n]:
        we = load_workload(name)
        er = measure(we, args.also_steps, 1, 0)
        per_snap_main = main_res["t_step"] / S
        per_snap = er["t_step"] / we.S
        extra[name] = {
            "value": er["value"], "unit": UNIT, "ms_per_step": 1e3 * er["t_step"],
            "snapshots": we.S, "chunk": er["chunk"], "dtype": we.dtype,
            "precision": we.precision, "steps": args.also_steps,
            "speedup_per_snapshot_vs_main": per_snap_main / per_snap,
            "roofline": er["roofline"], "stages": er["stages"], "tuned": er["tuned"],
            "graph_ms_per_step": er["graph_ms_per_step"],
            "pass2_ms_per_step": 1e3 * er["t_pass2"] if er["t_pass2"] else None,
            "kernels_ms_per_step": {k: v["ms_per_step"] for k, v in er["kernels"].items()},
        }
        stated = profiling.stated_error(
            os.path.join(ROOT, "profiles", f"error_{we.name}_{we.precision}.txt"))
        if stated:
            extra[name]["stated_error"] = stated
        log(f"[bench] {name}: {1e3 * er['t_step']:.1f} ms/step, "
            f"{per_snap_main / per_snap:.2f}x per snapshot vs {w.name}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or \
            host_info()["affinity_cores"]
        cpu = cpu_baseline(w, synth.y_grid(w), args.seed, threads, s_sample=min(100, S),
                           j1=w.ny // 2 - 8, nb=16)
        log(f"[bench] oracle sample took {cpu['seconds']:.1f} s")

    t_step = main_res["t_step"]
    res = {
        "metric": METRIC, "value": main_res["value"], "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} channel grid, {S} "
                               f"{w.dtype} snapshots, all (Y1,Y2) pairs, rx>=0 half plane, "
                               f"14 term maps", "grid": [w.nx, w.ny, w.nz], "snapshots": S,
                   "precision": w.precision, "chunk": main_res["chunk"],
                   "points_out": w.points_out, "tuned": main_res["tuned"], "seed": args.seed},
        "points_per_s": w.points_out / t_step,
        # the contract's T (first second-scan accumulate to the return of
        # finalize) and the throughput over it; the first scan apart
        "pass2": ({"ms_per_step": 1e3 * main_res["t_pass2"],
                   "value": w.points_out * S / main_res["t_pass2"],
                   "pass1_ms_per_step": 1e3 * (t_step - main_res["t_pass2"])}
                  if main_res["t_pass2"] else None),
        "graph": {"timed_steps_as_graphs": args.graph == "on",
                  "graph_ms_per_step": main_res["graph_ms_per_step"]},
        "roofline": main_res["roofline"],
        "stages": main_res["stages"],
        "cpu_baseline": cpu,
        "kernels": main_res["kernels"],
        "extra": extra,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
