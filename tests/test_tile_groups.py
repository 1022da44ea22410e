"""The grouping of tile pairs for the split-BF16 rank-k workgroups (host
logic, CPU only): compiled with g++ from the library's header and run over
the all-pairs triangles and slab rectangles up to 17 tiles."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1910_06409_amd", "csrc")


@pytest.fixture(scope="module")
def groups(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("tg") / "tile_groups_check")
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "tile_groups_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    out = {}
    for line in r.stdout.splitlines():
        kind, *v = line.split()
        out[(kind,) + tuple(int(x) for x in v[:-2])] = (int(v[-2]), int(v[-1]))
    return out


def test_every_pair_once(groups):
    # the program checks coverage and slot consistency itself; both layouts ran
    assert ("triangle", 17) in groups and ("rectangle", 6, 17) in groups


def test_triangles_fill_every_wave(groups):
    # 8 tiles (Ny = 129 .. 143): 36 pairs in 9 groups; 16 tiles (Ny = 257): 136 in 34
    assert groups[("triangle", 8)] == (9, 0)
    assert groups[("triangle", 16)] == (34, 0)
    for nt in range(18):
        ng, idle = groups[("triangle", nt)]
        assert 4 * ng - idle == nt * (nt + 1) // 2


def test_rectangles(groups):
    # two row tiles or more: whole 2 x 2 blocks; one row tile: three pairs per group
    assert groups[("rectangle", 2, 16)] == (8, 0)
    assert groups[("rectangle", 1, 16)] == (6, 8)
    for (kind, *dims), (ng, idle) in groups.items():
        if kind == "rectangle":
            assert 4 * ng - idle == dims[0] * dims[1]
