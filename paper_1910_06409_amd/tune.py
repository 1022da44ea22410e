"""Autotuner of the batching and the block shapes.

Tuned per (grid, rank-k precision, input dtype), in this order, each with the
previous choices in place:
  * chunk   -- snapshots per cross-spectral batch (one rank-k launch per
               batch): the whole step's time per snapshot;
  * zplanes -- planes per z-transform block: the z pass's device time;
  * kzpairs -- pairs per kz-finalize block: that kernel's device time;
  * kxtrans -- packed transforms per kx-finalize block: that kernel's time.
Every candidate is run on the device through the C ABI on seeded synthetic
snapshots resident in HBM and timed with the library's HIP events around
each launch (gke_timings); candidates whose workspace exceeds the memory
budget or that the library refuses are skipped.  The choices are cached in a
JSON file keyed by "NxxNyxNz/precision/dtype" (tuned.json next to this module
unless a path is given).

Command line (on a GPU):
  python -m paper_1910_06409_amd.tune --workload re200 [--snapshots S] [--cache PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")
SHAPE_KEYS = ("zplanes", "kzpairs", "kxtrans")


def key_of(w) -> str:
    return f"{w.nx}x{w.ny}x{w.nz}/{w.precision}/{w.dtype}"


def load(w, path: str = CACHE) -> dict | None:
    """The cached choice for workload w's shape, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(key_of(w))


def save(w, entry: dict, path: str = CACHE) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key_of(w)] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def _log(*a):
    print("[tune]", *a, file=sys.stderr, flush=True)


def tune(w, snapshots: int = 0, seed: int = 2024, steps: int = 2,
         budget_bytes: float = 200e9, path: str | None = CACHE) -> dict:
    """Measure the candidates for workload w; returns (and caches) the choice."""
    import torch

    from . import gke, runner, synth

    S = snapshots or w.S
    dev = torch.device("cuda", 0)
    y = synth.y_grid(w)
    tdt = torch.float32 if w.dtype == "f32" else torch.float64
    _log(f"{key_of(w)}: generating {S} snapshots")
    snaps = torch.empty((S, 4, w.ny, w.nz, w.nx), dtype=tdt, device=dev)
    gen = synth.DeviceSnapshots(w, seed, dev)
    for s in range(S):
        gen(s, out=snaps[s])
    torch.cuda.synchronize()
    del gen

    def workspace(chunk, shapes):
        p = gke.gke_plan(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu)
        try:
            gke.gke_set_option(p, gke.GKE_OPT_PRECISION,
                               gke.GKE_PREC_BF16X3 if w.precision == "bf16x3" else gke.GKE_PREC_FP64)
            gke.gke_set_option(p, gke.GKE_OPT_CHUNK, int(chunk))
            return gke.gke_workspace_size(p)
        finally:
            gke.gke_destroy(p)

    def run(chunk, shapes):
        """Device time per family (ms per step) and the wall time per step."""
        r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                          precision=w.precision, chunk=chunk, shapes=shapes, device=dev)
        outs = r.alloc_terms()

        def step():
            r.reset()
            for s in range(S):
                r.accumulate_snapshot(snaps[s])
            r.begin_stats()
            for s in range(S):
                r.accumulate_snapshot(snaps[s])
            r.finalize(outs)

        step()
        r.set_timing(True)
        r.timings(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        tm = {k: v[0] / steps for k, v in r.timings(reset=True).items() if v[1]}
        r.close()
        del outs, r
        torch.cuda.empty_cache()
        return wall, tm

    shapes: dict = {}
    log: dict = {}
    # defaults first (the built-in rule), for the record
    wall0, tm0 = run(0 if S > 128 else S + (S & 1), {})
    log["default"] = {"ms_per_step": 1e3 * wall0, "kernels_ms": tm0}
    # chunk: the whole step per snapshot
    cands = sorted({c for c in (8, 16, 32, 64, 128, 256, 512, S + (S & 1)) if c <= S + (S & 1)})
    best = None
    log["chunk"] = {}
    for c in cands:
        if workspace(c, shapes) > budget_bytes:
            log["chunk"][c] = "over the memory budget"
            continue
        wall, _ = run(c, shapes)
        log["chunk"][c] = 1e3 * wall
        _log(f"chunk {c}: {1e3 * wall:.2f} ms per step")
        if best is None or wall < best[1]:
            best = (c, wall)
    chunk = best[0]
    # block shapes, each by the device time of its own kernel family
    for name, family, cands_ in (
            ("zplanes", "zfft_pack", (4, 6, 8, 12, 16, 24, 32, 43, 64)),
            ("kzpairs", "fin_kz", (2, 4, 8, 12, 16)),
            ("kxtrans", "fin_kx", (2, 4, 6, 8, 10, 12, 16))):
        log[name] = {}
        bestv = None
        for v in cands_:
            try:
                _, tm = run(chunk, dict(shapes, **{name: v}))
            except gke.GkeError as e:   # outside this grid's limits
                log[name][v] = f"refused: {e}"
                continue
            log[name][v] = tm.get(family)
            _log(f"{name} {v}: {family} {tm.get(family):.3f} ms per step")
            if bestv is None or tm[family] < bestv[1]:
                bestv = (v, tm[family])
        if bestv is not None:
            shapes[name] = bestv[0]
    wall1, tm1 = run(chunk, shapes)
    entry = {"chunk": chunk, **shapes,
             "measured": {"snapshots": S, "steps": steps, "default_ms_per_step": 1e3 * wall0,
                          "tuned_ms_per_step": 1e3 * wall1, "tuned_kernels_ms": tm1,
                          "candidates": log},
             "device": torch.cuda.get_device_name(0)}
    _log(f"{key_of(w)}: chunk {chunk} {shapes}: {1e3 * wall0:.2f} -> {1e3 * wall1:.2f} ms per step")
    if path:
        save(w, entry, path)
    del snaps
    torch.cuda.empty_cache()
    return entry


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="re200")
    ap.add_argument("--snapshots", type=int, default=0)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from . import synth
    w = synth.workload(args.workload)
    entry = tune(w, args.snapshots, steps=args.steps, path=args.cache)
    print(json.dumps({key_of(w): entry}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
