"""CPU check of the windows of the K-step kernel with the paper's on-node
walls (k_step_nee_tb, csrc/d2q9_nee_tb.hpp, Sec. 2.2 (ii)), for every
(K, TX, TY) the library launches, on lattices that leave tiles one node wide
or high at the right and top walls.

Modelled step by step: step 1 pulls from the state f*(t) in global memory
(every lattice node valid) over region sites [1, RW - 1) x [1, RH - 1);
step s over [s, RW - s) x [s, RH - s); the last step over the tile alone.
A node pulls the 3 x 3 neighbourhood of its reference node (itself, or one
node inward for a wall node).  Checked: every such node was valid after the
previous step and lies in the region (LDS index in range), and the nodes
stored are exactly the lattice, each once.
"""
import itertools
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2211_05009_amd", "csrc", "lbm.hip")
with open(SRC) as fh:
    SHAPES = sorted(set((int(k), int(a), int(b)) for k, a, b in re.findall(
        r"launch_nee_tb_t<T, S, (\d+), (\d+), (\d+), \d+>", fh.read())))


def _ref(x, n):
    return min(max(x, 1), n - 2)


def _pulls_ok(x, y, nx, ny, valid, X0, Y0, RW, RH):
    xr, yr = _ref(x, nx), _ref(y, ny)
    for dx, dy in itertools.product((-1, 0, 1), repeat=2):
        q = (xr + dx, yr + dy)
        if valid is not None and q not in valid:
            return False
        if not (0 <= q[0] - X0 < RW and 0 <= q[1] - Y0 < RH):
            return False
    return True


def _check(nx, ny, K, TX, TY):
    RW, RH = TX + 2 * K + 1, TY + 2 * K + 1
    stored = set()
    for tx, ty in itertools.product(range(-(-nx // TX)), range(-(-ny // TY))):
        X0, Y0 = tx * TX - K - 1, ty * TY - K - 1
        tile = {(x, y) for x in range(tx * TX, min(tx * TX + TX, nx))
                for y in range(ty * TY, min(ty * TY + TY, ny))}
        valid = None   # step 1 reads global memory
        for s in range(1, K + 1):
            lo = K + 1 if s == K else s
            xs = range(X0 + lo, X0 + lo + TX) if s == K else range(X0 + s, X0 + RW - s)
            ys = range(Y0 + lo, Y0 + lo + TY) if s == K else range(Y0 + s, Y0 + RH - s)
            new = set()
            for x, y in itertools.product(xs, ys):
                if not (0 <= x < nx and 0 <= y < ny):
                    continue
                assert _pulls_ok(x, y, nx, ny, valid, X0, Y0, RW, RH), \
                    (nx, ny, K, TX, TY, tx, ty, s, x, y)
                new.add((x, y))
            valid = new
        assert valid == tile, (nx, ny, K, TX, TY, tx, ty)
        assert not (valid & stored)
        stored |= valid
    assert len(stored) == nx * ny


def test_shapes_read_from_the_source():
    assert len(SHAPES) >= 4 and all(k >= 2 for k, _, _ in SHAPES)


@pytest.mark.parametrize("ny", (3, 4, 17, 33, 65))
def test_nee_windows(ny):
    for (K, TX, TY), nx in itertools.product(SHAPES, (3, 4, 5, 17, 33, 34, 66, 97)):
        _check(nx, ny, K, TX, TY)
