"""GPU vortex extraction (lbm_vortex_extrema, lbm_vortex_centres,
lbm_bottom_vortex_count) against the oracle's definitions, and the steady
square cavity against Table 1.

The library's Psi is checked against the oracle elsewhere; here the oracle's
vortex functions run on the library's own Psi (lbm_stream_function), so the
extrema, the centre lists and the counts must agree exactly.
"""
import numpy as np
import pytest

from cavity_inputs import U_LID, random_fields
from oracle import d2q9, monitors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2211_05009_amd import lbm as m
    return m


def _check_against_oracle(c, min_abs):
    psi = c.stream_function()
    want = monitors.vortex_centres(psi, min_abs)
    got, n = c.vortex_centres(min_abs, cap=len(want) + 7)
    assert n == len(want)
    assert [v.as_tuple() for v in got] == want
    for v in got:
        assert v.x == (v.ix + 0.5) / c.nx and v.y == (v.iy + 0.5) / c.nx
    ext = monitors.vortex_extrema(psi, c.nx)
    gext = c.vortex_extrema()
    for name, v in zip(("primary", "lower_left", "lower_right"), gext):
        assert (v.psi, v.x, v.y) == ext[name], name
    assert c.bottom_vortex_count(min_abs) == monitors.bottom_vortex_count(psi, min_abs)
    return want


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_vortices_of_a_developing_cavity(lbm, dtype):
    c = lbm.Cavity(150, 180, re=1000.0, u_lid=U_LID, dtype=dtype)
    c.step(30000)
    for thr in (0.0, 1e-6, 1e-3):
        want = _check_against_oracle(c, thr)
    assert len(want) >= 1
    c.close()


def test_many_centres_and_caps(lbm):
    """A random velocity field has thousands of local extrema of Psi: more
    than the library's first scan holds, so it scans again."""
    nx, ny = 300, 260
    drho, ux, uy = random_fields(nx, ny, seed=11)
    c = lbm.Cavity(nx, ny, re=500.0, u_lid=U_LID, dtype="f64")
    c.init_fields(1.0 + drho, ux, uy)
    want = _check_against_oracle(c, 0.0)
    assert len(want) > 4096
    got, n = c.vortex_centres(0.0, cap=10)
    assert n == len(want) and [v.as_tuple() for v in got] == want[:10]
    got, n = c.vortex_centres(0.0, cap=0)
    assert got == [] and n == len(want)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_vortex_centres(c.h, -1.0, 5)
    c.close()


@pytest.mark.parametrize("shape", [(2, 2), (2, 9), (9, 2), (3, 3), (5, 4)])
def test_tiny_lattices(lbm, shape):
    nx, ny = shape
    c = lbm.Cavity(nx, ny, re=10.0, u_lid=U_LID, dtype="f64")
    c.step(37)
    _check_against_oracle(c, 0.0)
    c.close()


def test_oracle_cavity_gives_the_same_vortices(lbm):
    """Both sides from their own arithmetic (FP64): the same centres, values
    within 1e-12 of max |Psi|."""
    nx, ny, re, steps = 64, 80, 400.0, 3000
    ref = d2q9.Cavity(nx, ny, re=re, u_lid=U_LID).step(steps)
    _, ux0, _ = ref.moments()
    psi0 = monitors.stream_function(ux0)
    c = lbm.Cavity(nx, ny, re=re, u_lid=U_LID, dtype="f64")
    c.step(steps)
    tol = 1e-12 * np.abs(psi0).max()
    want = monitors.vortex_centres(psi0, 1e-9)
    got, n = c.vortex_centres(1e-9)
    assert [v.as_tuple()[:3] for v in got] == [w[:3] for w in want]
    assert all(abs(v.psi - w[3]) <= tol for v, w in zip(got, want))
    ext = monitors.vortex_extrema(psi0, nx)
    for name, v in zip(("primary", "lower_left", "lower_right"), c.vortex_extrema()):
        assert abs(v.psi - ext[name][0]) <= tol and (v.x, v.y) == ext[name][1:]
    c.close()


# Table 1, row a (Ghia et al.), 256 x 256: Psi / (U L), centre (x, y) / L.
TABLE1_A = {
    400.0: {"primary": (0.1139, 0.5547, 0.6055), "lower_left": (-1.42e-5, 0.0508, 0.0469),
            "lower_right": (-6.42e-4, 0.8906, 0.1250)},
    1000.0: {"primary": (0.1179, 0.5313, 0.5625), "lower_left": (-2.31e-4, 0.0859, 0.0781),
             "lower_right": (-1.75e-3, 0.8594, 0.1094)},
}


@pytest.mark.parametrize("re", sorted(TABLE1_A))
def test_square_cavity_against_table1(lbm, re):
    """Physical sanity check, not parity: the steady 256 x 256 cavity (FP64,
    Eq. 6 < 1e-10) with half-way bounce-back walls against the values of
    Table 1 row a.  Psi of the primary vortex within 2 %, of the corner
    vortices within 15 %; centres within 0.01 L (primary) and 0.015 L
    (corners): about two and four lattice spacings."""
    n = 256
    c = lbm.Cavity(n, n, re=re, u_lid=U_LID, dtype="f64")
    for _ in range(400):
        c.step(5000)
        if c.residual()[0] < 1e-10:
            break
    assert c.residual()[0] < 1e-10
    scale = U_LID * n
    got = dict(zip(("primary", "lower_left", "lower_right"), c.vortex_extrema()))
    for name, (psi, x, y) in TABLE1_A[re].items():
        v = got[name]
        print(f"Re {re:.0f} {name}: Psi/(UL) {v.psi / scale:.5g} (table {psi:.5g}), "
              f"x {v.x:.4f} ({x}), y {v.y:.4f} ({y})")
    for name, (psi, x, y) in TABLE1_A[re].items():
        v = got[name]
        rel, pos = (0.02, 0.01) if name == "primary" else (0.15, 0.015)
        assert abs(v.psi / scale - psi) <= rel * abs(psi), name
        assert abs(v.x - x) <= pos and abs(v.y - y) <= pos, name
    # both corner vortices are vortex centres below the primary one
    centres, _ = c.vortex_centres(1e-9 * scale)
    print("centres below the primary:",
          [(v.iy, v.ix, v.kind, f"{v.psi / scale:.3g}") for v in centres if v.iy < got["primary"].iy])
    for name in ("lower_left", "lower_right"):
        assert (got[name].iy, got[name].ix, -1) in [(v.iy, v.ix, v.kind) for v in centres]
    assert c.bottom_vortex_count(1e-9 * scale) >= 2
    c.close()
