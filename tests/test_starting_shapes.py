"""The shapes a context or a batch starts with, by share size (host logic
only: the starting-shape rule is compiled from the library's own header into
a small host program that makes no HIP call).  Shapes: level tiles of the
edge, cell and vertex kernels (0 = whole columns), the column and vertex
block sizes, the column's waves per SIMD and the column build (0 streaming,
1 level-parallel)."""
import os
import shutil
import subprocess

import pytest

from paper_2511_02021_amd import _build

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("shapes") / "shapes_probe")
    csrc = os.path.join(os.path.dirname(_build.NHDC_SO), "csrc")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", csrc, "-I", _build.INCLUDE,
                    os.path.join(HERE, "shapes_probe.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)

    def run(*args):
        out = subprocess.run([exe] + [str(a) for a in args], check=True, capture_output=True, text=True)
        return tuple(int(v) for v in out.stdout.split())
    return run


def _grid(k, n_lev):
    """(cells, edges, vertices, levels) of the bisection grid R2Bk."""
    nc = 20 * 4 ** (k + 1)
    return nc, nc * 3 // 2, nc // 2 + 2, n_lev


@pytest.mark.parametrize("k,n_lev,want", [
    (3, 90, (4, 4, 4, 256, 64, 3, 1)),     # 5120 cells: tiles of 4, level-parallel column
    (4, 20, (4, 4, 4, 256, 64, 3, 1)),
    (4, 90, (8, 4, 8, 256, 64, 3, 1)),
    (5, 90, (32, 16, 48, 64, 64, 3, 0)),   # streaming column in blocks of 64
    (6, 90, (0, 0, 0, 256, 64, 3, 0)),     # whole columns from R2B6 on
    (7, 90, (0, 0, 0, 256, 64, 3, 0)),
    (8, 90, (0, 0, 0, 256, 64, 3, 0)),
])
def test_starting_shapes_by_share(probe, k, n_lev, want):
    assert probe(*_grid(k, n_lev)) == want


def test_a_batch_starts_by_its_total_share(probe):
    one = probe(*_grid(3, 90))
    many = probe(*(_grid(3, 90) * 16))  # 16 x 5120 cells: more blocks, larger tiles
    assert one[6] == 1 and many[6] == 0   # 81 920 cells: past the level-parallel share
    assert all(m == 0 or m > o for m, o in zip(many[:3], one[:3]))
    assert probe(*(_grid(3, 90) * 8))[6] == 1  # 40 960 cells: still level-parallel


def test_level_parallel_columns_per_block(probe):
    # six arrays of (N + 1) rows of (C + 1) doubles within 160 KiB of LDS
    assert probe("w", 163840, 2, 90, 199, 200, 256) == (16, 16, 16, 8, 8)
    assert probe("w", 65536, 90) == (8,)
    assert probe("w", 65536, 256) == (4,)
