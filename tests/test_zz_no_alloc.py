"""The allocation-free entry point gke_set_static_workspace (the library's own
static device workspace) against gke_set_workspace with a caller buffer: two
plans in a row through the C ABI, the second on a smaller grid, each compared
element by element with the caller-workspace run of the same inputs."""
import sys

import numpy as np
import pytest

from paper_1910_06409_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(snap, w, y, static, **kw):
    import torch
    from paper_1910_06409_amd import runner
    dev = torch.from_numpy(np.ascontiguousarray(snap)).to("cuda")
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, static_workspace=static, **kw)
    for s in range(snap.shape[0]):
        r.accumulate_snapshot(dev[s])
    r.begin_stats()
    for s in range(snap.shape[0]):
        r.accumulate_snapshot(dev[s])
    out = r.finalize()
    torch.cuda.synchronize()
    prof = r.profiles()
    r.close()
    return [o.cpu().numpy() for o in out], prof


def test_static_workspace_matches_caller_workspace():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import gke
    cases = [
        # radix 3 and 5, a ragged plane tail, three snapshots in chunks of 2
        (synth.workload("tiny", nx=24, nz=20, ny=21, S=3, M=6), 4, dict(chunk=2)),
        # then a smaller grid on the same static workspace
        (synth.workload("tiny", S=2), 5, dict(chunk=2)),
    ]
    for w, seed, kw in cases:
        y = synth.y_grid(w)
        snap = synth.snapshots(w, seed)
        say(f"case static workspace {w.nx}x{w.ny}x{w.nz} S={w.S}")
        got, pg = _run(snap, w, y, True, **kw)
        ref, pr = _run(snap, w, y, False, **kw)
        for t in range(14):
            m = np.abs(ref[t]).max()
            e = np.abs(got[t] - ref[t]).max() / (m if m > 0 else 1.0)
            assert e <= TOL_FP64, f"T{t + 1}: {e:.3e}"
        assert np.abs(pg - pr).max() <= 1e-12 * np.abs(pr).max()
        say(f"  static == caller workspace on all 14 maps")
    # a plan whose workspace exceeds the static size is refused before any work
    w = synth.workload("re200")
    plan = gke.gke_plan(w.nx, w.ny, w.nz, synth.y_grid(w), w.lx, w.lz, w.nu)
    try:
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_static_workspace(plan)
        assert e.value.status == gke.GKE_ERR_OOM
    finally:
        gke.gke_destroy(plan)
