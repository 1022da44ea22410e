"""Bit reproducibility: every reduction of the library has a fixed order (the
plane sums, the moment partials, the rank-k accumulation over snapshots and
chunks, the finalize), so the same inputs with the same plan options give the
same bits in every map and profile, run after run and plan after plan, on
both rank-k paths and in the slab mode."""
import sys

import numpy as np
import pytest

from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(snaps, w, y, **kw):
    from paper_1910_06409_amd import runner
    out, prof = runner.run_snapshots(snaps, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                                     precision=w.precision, **kw)
    return [o.cpu().numpy() for o in out], np.array(prof)


@pytest.mark.parametrize("name,kw", [("tiny", dict(S=6, noise=0.5)),
                                     ("tiny", dict(S=9, dtype="f32", precision="bf16x3")),
                                     ("re200", dict(ny=33, S=8, noise=0.2))])
def test_same_inputs_same_bits(name, kw):
    torch = _torch()
    w = synth.workload(name, **kw)
    y = synth.y_grid(w)
    snaps = torch.from_numpy(synth.snapshots(w, 5)).cuda()
    say(f"case {name} {kw}: three runs, chunk 4, fresh plan each")
    runs = [_run(snaps, w, y, chunk=4) for _ in range(3)]
    for out, prof in runs[1:]:
        assert np.array_equal(prof, runs[0][1])
        for t in range(14):
            assert np.array_equal(out[t], runs[0][0][t]), f"T{t + 1}"


def test_slab_mode_same_bits():
    torch = _torch()
    from paper_1910_06409_amd import runner
    w = synth.workload("tiny", S=5, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    snaps = torch.from_numpy(synth.snapshots(w, 9)).cuda()
    say("case slab mode: mirror, fundamental domain, slabs of 3, two runs")
    res = []
    for _ in range(2):
        r, _ = runner.run_slabs(snaps, y, w.lx, w.lz, w.nu, dtype="f32", mirror=1,
                                domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=3, chunk=2)
        res.append([(p, [m.cpu().numpy() for m in maps]) for p, maps in r])
    for (pa, a), (pb, b) in zip(res[0], res[1]):
        assert np.array_equal(pa, pb)
        for t in range(14):
            assert np.array_equal(a[t], b[t]), f"T{t + 1}"
