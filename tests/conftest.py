import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def tiny():
    from paper_1910_06409_amd import synth
    w = synth.workload("tiny")
    return w, synth.y_grid(w), synth.snapshots(w, 7)


def nyquist_content(snap):
    """Smallest, over snapshots, fields and planes, of the energy fraction in
    the kx = Nx/2 column and in the kz = Nz/2 row of each plane's spectrum
    (relative to the plane's fluctuation energy)."""
    import numpy as np
    s = np.asarray(snap, dtype=np.float64)
    s = s - s.mean(axis=(-2, -1), keepdims=True)
    X = np.fft.rfft2(s, axes=(-2, -1))
    nz = s.shape[-2]
    tot = (np.abs(X) ** 2).sum(axis=(-2, -1))
    ex = (np.abs(X[..., -1]) ** 2).sum(axis=-1) / tot
    ez = (np.abs(X[..., nz // 2, :]) ** 2).sum(axis=-1) / tot
    return float(min(ex.min(), ez.min()))
