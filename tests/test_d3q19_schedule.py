"""CPU check of the LDS schedule of the z-marching D3Q19 kernel (k_step3_zs2,
csrc/d3q19_tb2.hpp): a plane-by-plane model of one block's step-1 writes
and step-2 reads, run for every tile shape the library launches.

The model follows the kernel: step 1 on plane z1 writes each window site's
19 post-collision values to pop(i, z1); after the barrier, step 2 on plane
z1 - 1 reads, for a link from inside the box, pop(i, z - c_z) at the
neighbouring site, and otherwise (reflection) pop(opp(i), z) at its own
site; a second barrier separates it from the next step 1.  pop() keeps the
-z populations two planes deep, the in-plane ones two and the +z ones three
(43 values per window site).  Checked: every LDS index lies in the array,
every step-2 read finds the value step 1 computed for that population,
site and plane (nothing overwrote it in between), and every site of the box
is stored exactly once per launch, for chunks of 1, 2, 3, 5 and all planes
per block.  The velocity tables, the population order inside each c_z
group and the tile shapes are read from the sources.
"""
import itertools
import os
import re

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2211_05009_amd", "csrc")


def _read(name):
    with open(os.path.join(CSRC, name)) as fh:
        return fh.read()


def _table(src, fn):
    m = re.search(fn + r"\(int i\) \{\s*constexpr int v\[19\] = \{([^}]*)\}", src)
    return [int(t) for t in m.group(1).split(",")]


STEP = _read("d3q19_step.hpp")
CX, CY, CZ = (_table(STEP, f) for f in ("cx19", "cy19", "cz19"))
KZ = _table(_read("d3q19_tb2.hpp"), "kz19")
SHAPES = sorted(set((int(a), int(b), int(c)) for a, b, c in re.findall(
    r"launch3_zs2_t<T, S, (\d+), (\d+), (\d+)>", _read("lbm3d.hip"))))


def _opp(i):
    return 0 if i == 0 else (i + 1 if i % 2 else i - 1)


def _schedule(nx, ny, nz, tx_, ty_, nt, zc):
    wx_, wy_ = tx_ + 2, ty_ + 2
    wp, tp = wx_ * wy_, tx_ * ty_
    dn, mid = 0, 2 * 5 * wp
    up = mid + 2 * 9 * wp
    ring = up + 3 * 5 * wp
    assert nt >= wp

    def pop(i, z):
        assert z >= -1
        if CZ[i] < 0:
            return dn + ((z + 2) & 1) * 5 * wp + KZ[i] * wp
        if CZ[i] == 0:
            return mid + ((z + 2) & 1) * 9 * wp + KZ[i] * wp
        return up + ((z + 3) % 3) * 5 * wp + KZ[i] * wp

    tiles_x, tiles_y = -(-nx // tx_), -(-ny // ty_)
    cols = tiles_x * tiles_y
    chunks = -(-nz // zc)
    stored = set()
    for b in range(cols * chunks):
        c, r = divmod(b, cols)
        ty, tx = divmod(r, tiles_x)
        x0, y0 = tx * tx_ - 1, ty * ty_ - 1
        zb, ze = c * zc, min(c * zc + zc, nz)
        lds = [None] * ring
        for z1 in range(zb - 1, ze + 1):
            for q in range(min(nt, wp)):                        # step 1
                x, y = x0 + q % wx_, y0 + q // wx_
                if 0 <= x < nx and 0 <= y < ny and 0 <= z1 < nz:
                    for i in range(19):
                        a = pop(i, z1) + q
                        assert 0 <= a < ring
                        lds[a] = (i, x, y, z1)
            z2 = z1 - 1                                         # step 2
            if z2 < zb:
                continue
            for q in range(tp):
                x, y = x0 + 1 + q % tx_, y0 + 1 + q // tx_
                if x >= nx or y >= ny:
                    continue
                sl = (1 + q // tx_) * wx_ + 1 + q % tx_
                for i in range(19):
                    xs, ys, zs = x - CX[i], y - CY[i], z2 - CZ[i]
                    if 0 <= xs < nx and 0 <= ys < ny and 0 <= zs < nz:
                        a = pop(i, zs) + sl - CX[i] - CY[i] * wx_
                        want = (i, xs, ys, zs)
                    else:
                        a = pop(_opp(i), z2) + sl
                        want = (_opp(i), x, y, z2)
                    assert 0 <= a < ring and lds[a] == want, (b, z2, q, i)
                assert (x, y, z2) not in stored
                stored.add((x, y, z2))
    assert len(stored) == nx * ny * nz


def test_tables_read_from_the_sources():
    assert len(SHAPES) >= 4
    for i in range(19):   # kz19 numbers each c_z group 0, 1, ... in index order
        group = [j for j in range(19) if CZ[j] == CZ[i]]
        assert KZ[i] == group.index(i)
        assert (CX[_opp(i)], CY[_opp(i)], CZ[_opp(i)]) == (-CX[i], -CY[i], -CZ[i])


@pytest.mark.parametrize("box", [(37, 23, 13), (3, 3, 3), (2, 66, 4), (67, 9, 5)])
def test_z_marching_schedule(box):
    # any chunk length (planes per block) the launcher may choose
    for (tx_, ty_, nt), zc in itertools.product(SHAPES, sorted({1, 2, 3, 5, box[2]})):
        _schedule(*box, tx_, ty_, nt, zc)
