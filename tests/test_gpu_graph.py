"""gke_accumulate_batch (the launches of a batch of snapshots as one HIP
graph) against gke_accumulate one by one: identical maps, over several
replays of the same graph with eager work and synchronisations between them,
a batch with other pointers (the graph updated in place) and a partial chunk."""
import sys

import numpy as np
import pytest

from paper_1910_06409_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,dtype", [("fp64", "f64"), ("bf16x3", "f32")])
def test_graph_batches_equal_eager(precision, dtype):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", nx=24, nz=20, ny=21, S=6, M=6, dtype=dtype, noise=0.3)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 91)
    dev = torch.from_numpy(snap).cuda()
    other = torch.from_numpy(snap[::-1].copy()).cuda()   # the same snapshots, other buffers
    say(f"case graph batches {precision}")
    r = runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype=dtype, precision=precision,
                      chunk=4)

    def eager(src):
        r.reset()
        for s in range(w.S):
            r.accumulate_snapshot(src[s])
        r.begin_stats()
        for s in range(w.S):
            r.accumulate_snapshot(src[s])
        out = r.finalize()
        torch.cuda.synchronize()
        return [o.cpu().numpy() for o in out]

    def batched(src, split=None):
        r.reset()
        r.accumulate_batch(src)
        r.begin_stats()
        if split:   # two batches: a partial chunk, then the rest
            r.accumulate_batch(src[:split])
            r.accumulate_batch(src[split:])
        else:
            r.accumulate_batch(src)
        out = r.finalize()
        torch.cuda.synchronize()
        return [o.cpu().numpy() for o in out]

    ref = eager(dev)
    for rep in range(3):   # capture, then replays
        got = batched(dev)
        for t in range(14):
            assert np.array_equal(got[t], ref[t]), (rep, t)
    ref_o = eager(other)
    got_o = batched(other)          # other pointers: captured again, graph updated
    for t in range(14):
        assert np.array_equal(got_o[t], ref_o[t]), t
    got_s = batched(dev, split=3)   # other batch sizes and chunk positions
    for t in range(14):
        assert np.array_equal(got_s[t], ref[t]), t
    got = batched(dev)              # the first graph again
    for t in range(14):
        assert np.array_equal(got[t], ref[t]), t
    r.close()
    say("  graph == eager on every replay")
