"""Halo coverage of the LDS tiles of the fused Q-side kernels, checked on the
host: tests/hostcheck/tile_halo.cpp stages a plane with the kernels' own
index maps (tiles.h) into an array prefilled with NaN, as the kernels'
HLB_DEBUG_NAN_LDS mode does to their LDS, and reads every value the stencils
read.  With the maps as built nothing reads NaN or a wrong site and every
point of the halo-1 plane is evaluated by exactly one thread (the tile sites
by their own threads); a staging that misses a halo column or row (planted in
the checker, not in the library) surfaces as NaN reads, and a loader that
takes the wrong component for some elements as wrong values."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("tile") / "tile_halo")
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(HERE, "hostcheck", "tile_halo.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def run(exe, drop):
    """(nan, bad, cover) for each tile shape: FP32's, then FP64's."""
    out = subprocess.run([exe, str(drop)], capture_output=True, text=True, check=True).stdout
    rows = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(rows) == 2
    return rows


def test_tile_maps_cover_every_halo_read(checker):
    for nan, bad, cover in run(checker, 0):
        assert (nan, bad, cover) == (0, 0, 0)


@pytest.mark.parametrize("drop", [1, 2])
def test_missed_halo_surfaces_as_nan(checker, drop):
    for nan, bad, cover in run(checker, drop):
        assert nan > 0 and bad == 0


def test_wrong_component_split_surfaces_as_wrong_values(checker):
    for nan, bad, cover in run(checker, 3):
        assert bad > 0 and cover == 0
