"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/gke.h declares, and validates arguments before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_06409_amd import gke

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gke.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gke_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gke.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in gke.gke_version()


def test_plan_argument_validation():
    y = np.linspace(-1, 1, 17)
    bad = [
        dict(Nx=15, Ny=17, Nz=16),   # odd
        dict(Nx=14, Ny=17, Nz=16),   # factor 7
        dict(Nx=16, Ny=4, Nz=16),    # too few planes
        dict(Nx=16, Ny=17, Nz=2),    # too short
    ]
    for b in bad:
        yy = np.linspace(-1, 1, b["Ny"])
        with pytest.raises(gke.GkeError) as e:
            gke.gke_plan(b["Nx"], b["Ny"], b["Nz"], yy, 1.0, 1.0, 0.01)
        assert e.value.status == gke.GKE_ERR_ARG
    with pytest.raises(gke.GkeError):
        gke.gke_plan(16, 17, 16, y[::-1].copy(), 1.0, 1.0, 0.01)   # not increasing
    with pytest.raises(gke.GkeError):
        gke.gke_plan(16, 17, 16, y, -1.0, 1.0, 0.01)
    with pytest.raises(gke.GkeError):
        gke.gke_plan(16, 17, 16, y, 1.0, 1.0, 0.0)


def test_options_and_state_errors():
    y = np.linspace(-1, 1, 17)
    p = gke.gke_plan(16, 17, 16, y, 2 * np.pi, np.pi, 0.005)
    try:
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 3)
        assert e.value.status == gke.GKE_ERR_ARG
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_option(p, 99, 1)
        assert e.value.status == gke.GKE_ERR_ARG
        n64 = gke.gke_workspace_size(p)
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 8)
        n8 = gke.gke_workspace_size(p)
        assert n64 > n8 > 0
        assert gke.gke_get_option(p, gke.GKE_OPT_CHUNK) == 8
        # chunk 0: the library picks the largest batch within its memory budget
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 0)
        gke.gke_workspace_size(p)
        assert gke.gke_get_option(p, gke.GKE_OPT_CHUNK) == 512
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 64)
        # no workspace yet: every device step is refused with a state error
        with pytest.raises(gke.GkeError) as e:
            gke.gke_accumulate(p, 1, 1, 1, 1)
        assert e.value.status == gke.GKE_ERR_STATE
        with pytest.raises(gke.GkeError) as e:
            gke.gke_begin_stats(p)
        assert e.value.status == gke.GKE_ERR_STATE
        with pytest.raises(gke.GkeError) as e:
            gke.gke_finalize(p, [0] * 14)
        assert e.value.status == gke.GKE_ERR_STATE
        # checkpoints need the workspace too; NULL buffers are argument errors
        for call in (lambda: gke.gke_state_size(p),
                     lambda: gke.gke_save_state(p, 4096, 1 << 20),
                     lambda: gke.gke_load_state(p, 4096, 1 << 20)):
            with pytest.raises(gke.GkeError) as e:
                call()
            assert e.value.status == gke.GKE_ERR_STATE
        for call in (lambda: gke.gke_save_state(p, 0, 1 << 20),
                     lambda: gke.gke_load_state(p, 0, 1 << 20)):
            with pytest.raises(gke.GkeError) as e:
                call()
            assert e.value.status == gke.GKE_ERR_ARG
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_workspace(p, 0, 1 << 20)
        assert e.value.status == gke.GKE_ERR_ARG
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_workspace(p, 256, 16)
        assert e.value.status == gke.GKE_ERR_OOM
        assert "workspace" in gke.gke_last_error(p)
    finally:
        gke.gke_destroy(p)


def test_general_mode_options():
    y = np.linspace(-1, 1, 17)
    p = gke.gke_plan(16, 17, 16, y, 2 * np.pi, np.pi, 0.005)
    try:
        n_all = gke.gke_workspace_size(p)
        for key, bad in [(gke.GKE_OPT_MIRROR, 2), (gke.GKE_OPT_DOMAIN, 5), (gke.GKE_OPT_SLAB, -1)]:
            with pytest.raises(gke.GkeError) as e:
                gke.gke_set_option(p, key, bad)
            assert e.value.status == gke.GKE_ERR_ARG
        # the fundamental domain needs the mirror average
        gke.gke_set_option(p, gke.GKE_OPT_DOMAIN, gke.GKE_DOMAIN_FUNDAMENTAL_FULLR)
        with pytest.raises(gke.GkeError) as e:
            gke.gke_workspace_size(p)
        assert e.value.status == gke.GKE_ERR_ARG
        gke.gke_set_option(p, gke.GKE_OPT_MIRROR, 1)
        gke.gke_set_option(p, gke.GKE_OPT_SLAB, 2)
        n_slab = gke.gke_workspace_size(p)
        assert 0 < n_slab
        with pytest.raises(gke.GkeError) as e:   # slab queries need the workspace
            gke.gke_slab_count(p)
        assert e.value.status == gke.GKE_ERR_STATE
        del n_all
    finally:
        gke.gke_destroy(p)
    # a grid that is not symmetric about its centre refuses the mirror average
    ya = np.linspace(-1, 1, 17) ** 3 + 0.01 * np.linspace(-1, 1, 17) ** 2
    p = gke.gke_plan(16, 17, 16, ya, 1.0, 1.0, 0.01)
    try:
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_option(p, gke.GKE_OPT_MIRROR, 1)
        assert e.value.status == gke.GKE_ERR_ARG
        assert "symmetric" in gke.gke_last_error(p)
    finally:
        gke.gke_destroy(p)


def test_workspace_scales_with_grid():
    from paper_1910_06409_amd import synth
    w = synth.workload("re200")
    p = gke.gke_plan(w.nx, w.ny, w.nz, synth.y_grid(w), w.lx, w.lz, w.nu)
    try:
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 100)
        n = gke.gke_workspace_size(p)
        # spectra: nk * 10 fields * chunk * planes * 16 B; accumulators: 8 spectra
        # per compact pair (36 tile pairs of 256 + 129 pairs of the last plane)
        spec = w.nk * 10 * 100 * 129 * 16
        acc = 8 * w.nk * (36 * 256 + 129) * 16
        assert spec + acc < n < 2 * (spec + acc)
        assert n < 200 * 2 ** 30
    finally:
        gke.gke_destroy(p)


def test_split_records_and_long_nz():
    """Split path: the spectra take 32-byte records of four snapshots (a chunk
    rounded up to whole quads, plane slots rounded up to 16), and a z length
    whose four-snapshot transform batch exceeds one block is refused."""
    from paper_1910_06409_amd import synth
    w = synth.workload("re200")
    p = gke.gke_plan(w.nx, w.ny, w.nz, synth.y_grid(w), w.lx, w.lz, w.nu)
    try:
        gke.gke_set_option(p, gke.GKE_OPT_PRECISION, gke.GKE_PREC_BF16X3)
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 26)
        n26 = gke.gke_workspace_size(p)
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 28)
        n28 = gke.gke_workspace_size(p)
        assert n26 == n28                      # 26 and 28 snapshots: seven quads
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 32)
        n32 = gke.gke_workspace_size(p)
        assert n32 - n28 == w.nk * 10 * 144 * 32   # one more quad of records
    finally:
        gke.gke_destroy(p)
    y = np.linspace(-1, 1, 17)
    p = gke.gke_plan(16, 17, 1000, y, 2 * np.pi, np.pi, 0.005)
    try:
        assert gke.gke_workspace_size(p) > 0   # FP64: one transform per block
        gke.gke_set_option(p, gke.GKE_OPT_PRECISION, gke.GKE_PREC_BF16X3)
        with pytest.raises(gke.GkeError) as e:
            gke.gke_workspace_size(p)
        assert e.value.status == gke.GKE_ERR_UNSUPPORTED
    finally:
        gke.gke_destroy(p)


def test_static_workspace_refuses_a_plan_larger_than_it():
    """gke_set_static_workspace checks the plan's size before any device work."""
    from paper_1910_06409_amd import synth
    w = synth.workload("re200")
    p = gke.gke_plan(w.nx, w.ny, w.nz, synth.y_grid(w), w.lx, w.lz, w.nu)
    try:
        assert gke.gke_workspace_size(p) > gke.GKE_STATIC_WORKSPACE_BYTES
        with pytest.raises(gke.GkeError) as e:
            gke.gke_set_static_workspace(p)
        assert e.value.status == gke.GKE_ERR_OOM
        assert str(gke.GKE_STATIC_WORKSPACE_BYTES) in str(e.value)
    finally:
        gke.gke_destroy(p)
    # the tiny channel fits it (the size the GPU test runs)
    w = synth.workload("tiny")
    p = gke.gke_plan(w.nx, w.ny, w.nz, synth.y_grid(w), w.lx, w.lz, w.nu)
    try:
        gke.gke_set_option(p, gke.GKE_OPT_CHUNK, 2)
        assert gke.gke_workspace_size(p) <= gke.GKE_STATIC_WORKSPACE_BYTES
    finally:
        gke.gke_destroy(p)


def test_undersampling_indices_match_the_oracle_rule():
    """The kept rx / rz separations the library reports follow the two-threshold
    rule of the oracle (full resolution below t1, every s1-th index below t2,
    every s2-th beyond), for the half-plane and the full-r domains."""
    from oracle import oracle
    from paper_1910_06409_amd import synth
    # a hand-written case: n = 32, thresholds 4 and 10, steps 2 and 4
    assert oracle.sample_indices(32, 4, 10, 2, 4, True) == [0, 1, 2, 3, 4, 6, 8, 12, 16]
    assert oracle.sample_indices(8, 0, 0, 1, 1, False) == list(range(8))
    full = oracle.sample_indices(32, 4, 10, 2, 4, False)
    assert full == [0, 1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 26, 28, 29, 30, 31]
    w = synth.workload("re1000")
    y = synth.y_grid(w)
    cases = [(0, (0, 0, 1, 1)), (0, (8, 20, 4, 8)), (1, (12, 30, 4, 8)), (1, (3, 3, 5, 5)),
             (0, (5, 100, 3, 7))]
    for domain in (gke.GKE_DOMAIN_ALLPAIRS_HALFRX, gke.GKE_DOMAIN_Y1LEY2_FULLR):
        for d, u in cases:
            p = gke.gke_plan(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu)
            try:
                gke.gke_set_option(p, gke.GKE_OPT_DOMAIN, domain)
                gke.gke_set_undersampling(p, d, *u)
                n = w.nx if d == 0 else w.nz
                half = d == 0 and domain == gke.GKE_DOMAIN_ALLPAIRS_HALFRX
                got = list(gke.gke_sample_indices(p, d))
                assert got == oracle.sample_indices(n, *u, half), (domain, d, u)
                # the other direction keeps everything
                o = 1 - d
                assert len(gke.gke_sample_indices(p, o)) == (
                    (w.nx // 2 + 1 if domain == 0 else w.nx) if o == 0 else w.nz)
            finally:
                gke.gke_destroy(p)
    p = gke.gke_plan(w.nx, w.ny, w.nz, y, w.lx, w.lz, w.nu)
    try:
        for bad in [(2, 0, 0, 1, 1), (0, 5, 4, 1, 1), (0, 0, 0, 0, 1), (1, -1, 2, 1, 1)]:
            with pytest.raises(gke.GkeError) as e:
                gke.gke_set_undersampling(p, *bad)
            assert e.value.status == gke.GKE_ERR_ARG
    finally:
        gke.gke_destroy(p)


def test_tuned_cache_round_trip(tmp_path):
    """The autotuner's cache: one entry per (grid, precision, dtype) key."""
    from paper_1910_06409_amd import synth, tune
    path = str(tmp_path / "tuned.json")
    a, b = synth.workload("re200"), synth.workload("re200_bf16")
    assert tune.key_of(a) == "192x129x160/fp64/f64"
    assert tune.load(a, path) is None
    tune.save(a, {"chunk": 100, "zplanes": 12}, path)
    tune.save(b, {"chunk": 512, "kxtrans": 8}, path)
    assert tune.load(a, path)["zplanes"] == 12
    assert tune.load(b, path)["chunk"] == 512
    assert tune.load(synth.workload("tiny"), path) is None


def test_accumulate_batch_argument_checks():
    y = np.linspace(-1, 1, 17)
    p = gke.gke_plan(16, 17, 16, y, 2 * np.pi, np.pi, 0.005)
    try:
        with pytest.raises(gke.GkeError) as e:
            gke.gke_accumulate_batch(p, [1], [1], [1], [1])
        assert e.value.status == gke.GKE_ERR_STATE     # no workspace yet
        with pytest.raises(gke.GkeError) as e:
            gke.gke_accumulate_batch(p, [], [], [], [])
        assert e.value.status == gke.GKE_ERR_ARG
    finally:
        gke.gke_destroy(p)
