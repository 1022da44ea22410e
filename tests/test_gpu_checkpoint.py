"""Checkpoint and resume through the C ABI (gke_state_size, gke_save_state,
gke_load_state): a run saved part-way (in the first scan, in the second, in a
slab's scan) and continued in a fresh plan gives the maps and profiles of the
uninterrupted run with the same chunk boundaries bit for bit (saving flushes
the current chunk, so the uninterrupted run saves too and goes on); the maps
agree with the oracle; a state from a plan of another shape is refused."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1910_06409_amd import gke, synth

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(w, y, dev, **kw):
    from paper_1910_06409_amd import runner
    return runner.GkeRun(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu, dtype=w.dtype,
                         precision=w.precision, device=dev.device, **kw)


def _maps(out):
    return [o.cpu().numpy() if o is not None else None for o in out]


@pytest.mark.parametrize("name,kw,save_at", [
    ("tiny", dict(S=7), ("scan2", 5)),
    ("tiny", dict(S=7), ("scan1", 3)),
    ("tiny", dict(S=9, dtype="f32", precision="bf16x3", noise=0.3), ("scan2", 6)),
])
def test_resume_equals_uninterrupted(name, kw, save_at):
    torch = _torch()
    w = synth.workload(name, **kw)
    y = synth.y_grid(w)
    snap = synth.snapshots(w, 31)
    dev = torch.from_numpy(snap).cuda()
    where, at = save_at
    say(f"case {name} {kw}: save in the {where} after {at} snapshots, resume in a new plan")

    def scan(r, lo, hi):
        for s in range(lo, hi):
            r.accumulate_snapshot(dev[s])

    # uninterrupted (it saves at the same point, which flushes the chunk, and goes on)
    a = _plan(w, y, dev, chunk=4)
    if where == "scan1":
        scan(a, 0, at)
        state = a.save_state()
        scan(a, at, w.S)
        a.begin_stats()
        scan(a, 0, w.S)
    else:
        scan(a, 0, w.S)
        a.begin_stats()
        scan(a, 0, at)
        state = a.save_state()
        scan(a, at, w.S)
    maps_a, prof_a = _maps(a.finalize()), a.profiles()
    a.close()
    say(f"  state {state.numel()} bytes")
    # resumed in a fresh plan
    b = _plan(w, y, dev, chunk=4)
    b.load_state(state)
    if where == "scan1":
        scan(b, at, w.S)
        b.begin_stats()
        scan(b, 0, w.S)
    else:
        scan(b, at, w.S)
    maps_b, prof_b = _maps(b.finalize()), b.profiles()
    b.close()
    assert np.array_equal(prof_a, prof_b)
    for t in range(14):
        assert np.array_equal(maps_a[t], maps_b[t]), f"T{t + 1}"
    if w.precision == "fp64":
        pairs = [(0, 16), (5, 5), (11, 3)]
        ref = oracle.pair_terms(snap.astype(np.float64), y, w.lx, w.lz, w.nu, pairs)
        nkx = w.nx // 2 + 1
        for t in range(13):
            g = np.array([maps_a[t][p, q] for (p, q) in pairs])
            r = ref[:, t, :, :nkx]
            assert np.abs(g - r).max() <= TOL_FP64 * np.abs(r).max(), f"T{t + 1}"


def test_resume_inside_a_slab():
    torch = _torch()
    w = synth.workload("tiny", S=5, dtype="f32", noise=0.5)
    y = synth.y_grid(w)
    dev = torch.from_numpy(synth.snapshots(w, 37)).cuda()
    kw = dict(chunk=2, mirror=1, domain=gke.GKE_DOMAIN_FUNDAMENTAL_FULLR, slab=3)
    say("case slab mode: save in the second slab's scan, resume in a new plan")
    a = _plan(w, y, dev, **kw)
    for s in range(w.S):
        a.accumulate_snapshot(dev[s])
    a.begin_stats()
    for s in range(w.S):
        a.accumulate_snapshot(dev[s])
    a.finalize(a.alloc_terms(slab=0))
    a.begin_slab(1)
    for s in range(3):
        a.accumulate_snapshot(dev[s])
    state = a.save_state()
    for s in range(3, w.S):
        a.accumulate_snapshot(dev[s])
    out_a = _maps(a.finalize(a.alloc_terms(slab=1)))
    a.close()
    b = _plan(w, y, dev, **kw)
    b.load_state(state)
    for s in range(3, w.S):
        b.accumulate_snapshot(dev[s])
    out_b = _maps(b.finalize(b.alloc_terms(slab=1)))
    b.close()
    for t in range(14):
        assert np.array_equal(out_a[t], out_b[t]), f"T{t + 1}"


def test_state_of_another_shape_is_refused():
    torch = _torch()
    w = synth.workload("tiny", S=3)
    y = synth.y_grid(w)
    dev = torch.from_numpy(synth.snapshots(w, 41)).cuda()
    a = _plan(w, y, dev, chunk=4)
    for s in range(w.S):
        a.accumulate_snapshot(dev[s])
    state = a.save_state()
    a.close()
    w2 = synth.workload("tiny", S=3, nz=20)
    b = _plan(w2, y, torch.from_numpy(synth.snapshots(w2, 41)).cuda(), chunk=4)
    with pytest.raises(gke.GkeError) as e:
        b.load_state(state)
    assert e.value.status == gke.GKE_ERR_ARG
    with pytest.raises(gke.GkeError) as e:
        b.load_state(state[:64].contiguous())
    assert e.value.status == gke.GKE_ERR_ARG
    b.close()
