"""CPU checks of the tile orders (paper_1412_1498_amd/csrc/tile_order.hpp),
compiled for the host from the very header the kernels include: for
lattices of several shapes and tile sizes, the order that pick_slab_order
chooses (2-d column blocks where a z plane is a whole number of tiles, 1-d
blocks otherwise) and the plain 1-d column blocks must visit every tile
exactly once after the XCD-contiguous mapping, whatever the number of
tiles (whole time slices or not). The F/theta kernel's choice on the
benchmark lattice is pinned: 3 tiles along a z plane by 6 planes."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_1498_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tile_order") / "check")
    src = os.path.join(ROOT, "tests", "tile_order", "check.cpp")
    r = subprocess.run(["hipcc", "-I" + CSRC, "-O1", "-x", "hip", src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run(exe, cases):
    inp = "".join(" ".join(map(str, c)) + "\n" for c in cases)
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    return [tuple(int(v) for v in line.split()) for line in r.stdout.splitlines()]


def test_benchmark_lattice_orders(checker):
    # F/theta tiles (128 half indices, both parities) of the 48^4 lattice:
    # float 18-, 12-, 8-real links and double 18-real
    out = run(checker, [(48, 48, 48, 48, 128, 256 * 4 * 9 * 8), (48, 48, 48, 48, 128, 256 * 4 * 6 * 8),
                        (48, 48, 48, 48, 128, 256 * 4 * 4 * 8), (48, 48, 48, 48, 128, 256 * 4 * 9 * 16)])
    S, nrow, B, P, w, ok, ok1 = out[0]
    assert (S, nrow, B, P, w) == (432, 48, 18, 9, 3)
    for row in out:
        assert row[5] == 1 and row[6] == 1, row
        assert row[3] == 9 and row[2] % row[4] == 0 and 48 % (row[2] // row[4]) == 0, row


def test_orders_are_bijections(checker):
    cases = [(32, 32, 32, 32, 128, 73728), (24, 24, 24, 24, 128, 73728), (16, 16, 16, 16, 128, 73728),
             (48, 48, 48, 96, 128, 73728), (48, 48, 48, 12, 128, 147456), (6, 4, 4, 2, 128, 1000),
             (10, 6, 14, 6, 128, 5000), (12, 12, 12, 12, 64, 20000), (8, 8, 8, 8, 128, 73728),
             (16, 16, 8, 14, 128, 147456), (2, 2, 2, 2, 128, 100)]
    rng = random.Random(7)
    for _ in range(40):
        d = [2 * rng.randint(1, 20) for _ in range(4)]
        cases.append((*d, rng.choice([32, 64, 128]), rng.choice([4096, 32768, 73728, 147456, 1 << 20])))
    for case, row in zip(cases, run(checker, cases)):
        assert row[5] == 1 and row[6] == 1, (case, row)
        if row[3]:  # 2-d blocks: whole planes of tiles, blocks of whole planes
            nx, ny, nz, nt, th, _ = case
            assert (nx // 2 * ny) % th == 0 and row[3] == nx // 2 * ny // th
            assert row[3] % row[4] == 0 and nz % (row[2] // row[4]) == 0
