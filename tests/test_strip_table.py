"""The strip table of the row-sweep kernels (host code, built here with g++):
every fluid node of every active capillary is swept exactly once, strips stay
inside their lattice, wide strips start on 32-column boundaries (whole
128-byte lines), chunks start an even number of rows into their column (the
kernels' row loops are unrolled by two), the table never outgrows the capacity
the library allocates (at any chunking, for one capillary or a batch), and the solid walls of the tube are not swept (beyond
one wall row and the rounding of the cut to 32 columns where the tube enters or
leaves a strip)."""
import os
import shutil
import subprocess

import pytest

from paper_0911_0459_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (nx, ny, x_in, tube_len, tube_h, y0): inlets on and off 32-column boundaries,
# tubes that reach the right edge or end inside the lattice, odd and even
# heights and walls, no tube, the smallest lattice, a tube over every column
# (no strip holds both ends of a tube)
EDGE_CASES = [
    (700, 45, 250, 450, 17, 14), (150, 37, 53, 97, 13, 11), (300, 61, 120, 180, 23, 19),
    (520, 41, 150, 280, 15, 13), (520, 41, 150, 280, 15, 0), (520, 41, 150, 280, 28, 13),
    (400, 30, 10, 380, 9, 10), (256, 64, 128, 128, 20, 22), (4096, 256, 1024, 3072, 100, 78),
    (1000, 50, 0, 400, 20, 15), (1000, 50, 600, 400, 20, 15), (5, 3, 0, 0, 0, 0), (96, 40, 0, 0, 0, 0),
    (3, 12, 0, 3, 10, 1), (210, 48, 100, 110, 16, 16),
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("strips") / "strip_table_check")
    subprocess.run([gxx, "-std=c++17", "-O2", "-D_GLIBCXX_ASSERTIONS", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_0911_0459_amd", "csrc"),
                    os.path.join(ROOT, "tests", "strip_table_check.cpp"), "-o", exe], check=True)
    return exe


def run(exe, geoms, alone=False):
    """Check one strip table of all `geoms` (or, with alone, one table per geometry)."""
    text = f"{len(geoms)} {int(alone)}\n" + "".join(" ".join(str(v) for v in g) + "\n" for g in geoms)
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=600, check=True)
    return {k: int(v) for k, v in (line.split() for line in r.stdout.splitlines())}


def expect_clean(res):
    assert res == dict(bad_bounds=0, bad_align32=0, twice=0, missed=0, inactive=0, bad_parity=0, bad_xcd=0,
                       over_capacity=0, max_extra_solid=res["max_extra_solid"]), res
    assert res["max_extra_solid"] <= 0, res


def test_edge_geometries(checker):
    expect_clean(run(checker, [(*g, 1) for g in EDGE_CASES]))


def test_each_geometry_alone(checker):
    """One capillary per table (as the sequential runs and the autotuner of a
    single lattice build it): every column of an XCD run may end in a tail."""
    sweep = [(w.geom.nx, w.geom.ny, w.geom.x_in, w.geom.tube_len, w.geom.tube_h, w.geom.y0)
             for w in I.sweep_batch()]
    expect_clean(run(checker, [(*g, 1) for g in EDGE_CASES + sweep], alone=True))


def test_sweep_batch_with_retired_capillaries(checker):
    """The 256 capillaries of the sweep, every third one retired."""
    geoms = [(w.geom.nx, w.geom.ny, w.geom.x_in, w.geom.tube_len, w.geom.tube_h, w.geom.y0, int(k % 3 != 0))
             for k, w in enumerate(I.sweep_batch())]
    expect_clean(run(checker, geoms))
