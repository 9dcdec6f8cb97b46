"""CPU check of the windows of the K-step kernel with half-way walls
(k_step_tb, csrc/d2q9_temporal.hpp), for every (K, TX, TY) the library
launches for a single cavity, on lattices from 3 x 3 up with ragged edge
tiles.

Model: a block owns a TX x TY tile and a (TX + 2K) x (TY + 2K) region
around it; step 1 pulls from the state f*(t) in global memory over region
sites [1, RW - 1) x [1, RH - 1); step s updates [s, RW - s) x [s, RH - s);
sites outside the lattice are skipped.  A site pulls each link from the
neighbour it streams from when that neighbour is in the lattice and
reflects (its own opposite population) otherwise.  Checked: every
neighbour pulled was valid after the previous step and lies in the region
(LDS index in range), the last window is exactly the tile, and every site
is stored once.
"""
import itertools
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2211_05009_amd", "csrc", "lbm.hip")
with open(SRC) as fh:
    SHAPES = sorted(set((int(k), int(a), int(b)) for k, a, b in re.findall(
        r"launch_tb_t<T, S, (\d+), (\d+), (\d+), \d+", fh.read())))
LINKS = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _check(nx, ny, K, TX, TY):
    RW, RH = TX + 2 * K, TY + 2 * K
    stored = set()
    for tx, ty in itertools.product(range(-(-nx // TX)), range(-(-ny // TY))):
        X0, Y0 = tx * TX - K, ty * TY - K
        valid = None   # step 1 reads global memory
        for s in range(1, K + 1):
            new = set()
            for lx, ly in itertools.product(range(s, RW - s), range(s, RH - s)):
                x, y = X0 + lx, Y0 + ly
                if not (0 <= x < nx and 0 <= y < ny):
                    continue
                for cx, cy in LINKS:
                    xs, ys = x - cx, y - cy
                    if not (0 <= xs < nx and 0 <= ys < ny):
                        continue   # reflected: the site's own value
                    assert 0 <= xs - X0 < RW and 0 <= ys - Y0 < RH
                    assert valid is None or (xs, ys) in valid, (nx, ny, K, TX, TY, s, x, y)
                new.add((x, y))
            valid = new
        tile = {(x, y) for x in range(tx * TX, min(tx * TX + TX, nx))
                for y in range(ty * TY, min(ty * TY + TY, ny))}
        assert valid == tile
        assert not (valid & stored)
        stored |= valid
    assert len(stored) == nx * ny


def test_shapes_read_from_the_source():
    assert len(SHAPES) >= 8 and all(k >= 2 for k, _, _ in SHAPES)


@pytest.mark.parametrize("nx,ny", list(itertools.product((3, 5, 31, 33, 65, 97), (3, 4, 17, 49))))
def test_tb_windows(nx, ny):
    for K, TX, TY in SHAPES:
        _check(nx, ny, K, TX, TY)
