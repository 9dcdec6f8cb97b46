"""Pins of the non-equilibrium extrapolation oracle (oracle/nee.py), the
paper's wall scheme (Sec. 2.2 (ii)), and mutations they must catch."""
import math
import os
import types

import numpy as np
import pytest

from cavity_inputs import random_shift
from oracle import nee
from oracle.d2q9 import W, collide, equilibrium, macroscopic
from oracle.naive import naive_steps_nee

U = 0.1


def _brute_force_gap(mod, nx, ny, re, steps, seed=None):
    c = mod.CavityNEE(nx, ny, re=re, u_lid=U)
    if seed is not None:
        c.set_state(c.f + random_shift(nx, ny, seed))
    f0 = c.f.copy()
    c.step(steps)
    return np.abs(np.array(naive_steps_nee(f0, c.tau, U, steps)) - c.f).max()


@pytest.mark.parametrize("shape", [(3, 3), (5, 4), (6, 7), (4, 9)])
def test_matches_the_push_form_twin(shape):
    """The vectorised oracle against the pure-Python push-form twin (a
    separate implementation of the same definition), with and without a
    random perturbation of every distribution."""
    nx, ny = shape
    assert _brute_force_gap(nee, nx, ny, 20.0, 60) <= 2e-15
    assert _brute_force_gap(nee, nx, ny, 20.0, 30, seed=nx * ny) <= 2e-15


def test_tau_uses_the_distance_between_the_walls():
    # 257 nodes = 256 spacings: Re = 400 gives nu = 0.064, tau = 0.692
    assert math.isclose(nee.relaxation_time(257, 400.0, U), 0.692, rel_tol=1e-14)
    assert math.isclose(nee.relaxation_time(501, 8000.0, U), 0.51875, rel_tol=1e-14)


def test_rest_is_a_fixed_point():
    c = nee.CavityNEE(7, 6, tau=0.8, u_lid=0.0)
    f0 = c.f.copy()
    assert np.array_equal(f0, np.broadcast_to(W[:, None, None], f0.shape))
    c.step(25)
    # sum_i w_i rounds to 1 + O(1e-16) in FP64, so f^eq(rho, 0) = rho w moves
    # the rest state by a few ulps at most
    assert np.abs(c.f - f0).max() <= 2e-16


def test_initial_state_moves_the_whole_top_row():
    c = nee.CavityNEE(8, 6, re=100.0, u_lid=U)
    rho, ux, uy = c.moments()
    assert np.allclose(rho, 1.0, rtol=0, atol=1e-15)
    assert np.allclose(ux[-1], U, rtol=0, atol=1e-16) and np.all(ux[:-1] == 0)
    assert np.all(uy == 0)


def test_first_step_closed_form():
    """From the initial state, the row below the lid pulls f_4, f_7, f_8
    from the moving top row (f^eq(1, U)) and rest values elsewhere:
    rho = 1 + (1/9)(-3U^2/2) + (1/36)(6 U^2) = 1, rho u_x = f_8 - f_7 = U/6,
    rho u_y = 0.  The corner nodes move with the lid, so the end nodes of that
    row agree too.  Rows further down stay at rest; wall nodes carry their
    reference node's density and the wall velocity."""
    nx, ny = 9, 7
    c = nee.CavityNEE(nx, ny, re=100.0, u_lid=U).step(1)
    rho, ux, uy = c.moments()
    assert np.allclose(rho[ny - 2, 1:-1], 1.0, rtol=0, atol=1e-15)
    assert np.allclose(ux[ny - 2, 1:-1], U / 6, rtol=0, atol=1e-16)
    assert np.allclose(uy[ny - 2, 1:-1], 0.0, rtol=0, atol=1e-16)
    assert np.abs(rho[:ny - 2] - 1).max() <= 1e-15 and np.abs(ux[:ny - 2]).max() == 0
    assert np.allclose(ux[ny - 1], U, rtol=0, atol=1e-16)
    assert np.allclose(rho[ny - 1, 1:-1], rho[ny - 2, 1:-1], rtol=0, atol=1e-15)


def test_wall_nodes_carry_reference_density_and_wall_velocity():
    nx, ny = 12, 10
    c = nee.CavityNEE(nx, ny, re=200.0, u_lid=U)
    c.set_state(c.f + random_shift(nx, ny, 3))
    c.step(40)
    rho, ux, uy = c.moments()
    ys, xs, yr, xr = nee.wall_nodes(nx, ny)
    assert np.allclose(rho[ys, xs], rho[yr, xr], rtol=0, atol=2e-15)
    assert np.allclose(ux[ys, xs], np.where(ys == ny - 1, U, 0.0), rtol=0, atol=2e-16)
    assert np.allclose(uy[ys, xs], 0.0, rtol=0, atol=2e-16)
    # corners refer to their diagonal fluid neighbour
    k = list(zip(ys, xs)).index((0, 0))
    assert (yr[k], xr[k]) == (1, 1)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_couette_flow_is_linear_between_on_node_walls(tau):
    """Channel between the moving top row and the resting bottom row (x
    periodic): the steady profile is u_x = U y / (Ny - 1), u_y = 0, rho = 1,
    exactly (the extrapolated non-equilibrium part of a linear profile is
    the same on every row)."""
    ny = 7
    c = nee.CavityNEE(4, ny, tau=tau, u_lid=U, periodic_x=True).step(5000)
    rho, ux, uy = c.moments()
    y = np.arange(ny)[:, None]
    assert np.abs(ux - U * y / (ny - 1)).max() <= 1e-13
    assert np.abs(uy).max() <= 1e-15
    assert np.abs(rho - 1).max() <= 1e-12


def test_mirror_symmetry():
    """x -> Nx - 1 - x with U -> -U maps solutions onto solutions."""
    nx, ny = 10, 8
    a = nee.CavityNEE(nx, ny, tau=0.7, u_lid=U).step(50)
    b = nee.CavityNEE(nx, ny, tau=0.7, u_lid=-U).step(50)
    ra, uxa, uya = a.moments()
    rb, uxb, uyb = b.moments()
    # equal up to the order of the sums (a few ulps)
    assert np.allclose(ra, rb[:, ::-1], rtol=0, atol=2e-15)
    assert np.allclose(uxa, -uxb[:, ::-1], rtol=0, atol=5e-16)
    assert np.allclose(uya, uyb[:, ::-1], rtol=0, atol=5e-16)


def test_post_collision_of_a_wall_node():
    """The stored (post-collision) value of a wall node is
    f^eq(rho_f, u_w) + (1 - 1/tau)(f_f - f^eq_f): the form a fused kernel
    computes from the streamed reference node alone; and that equals the
    BGK update of f_f plus f^eq(rho_f, u_w) - f^eq_f, the form in which the
    library runs wall nodes through the fluid nodes' collision."""
    nx, ny = 9, 8
    c = nee.CavityNEE(nx, ny, re=120.0, u_lid=U)
    c.set_state(c.f + random_shift(nx, ny, 5))
    c.step(7)
    fs = c.post_collision()
    rho, ux, uy = macroscopic(c.f)
    for (y, x) in [(ny - 1, 0), (ny - 1, 4), (0, 0), (3, nx - 1), (0, 5)]:
        yr, xr = min(max(y, 1), ny - 2), min(max(x, 1), nx - 2)
        ff = c.f[:, yr, xr]
        feq_f = equilibrium(rho[yr, xr], ux[yr, xr], uy[yr, xr])
        feq_w = equilibrium(rho[yr, xr], U if y == ny - 1 else 0.0, 0.0)
        want = feq_w + (1 - 1 / c.tau) * (ff - feq_f)
        assert np.allclose(fs[:, y, x], want, rtol=0, atol=5e-16)
        via_bgk = collide(ff, c.tau) + (feq_w - feq_f)
        assert np.allclose(fs[:, y, x], via_bgk, rtol=0, atol=5e-16)


# -- mutations -------------------------------------------------------------
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "nee.py")

MUTATIONS = {
    "non-equilibrium part dropped": ("f[:, ys, xs] = feq_w + f[:, yr, xr] - feq_f",
                                     "f[:, ys, xs] = feq_w"),
    "wall node extrapolates from itself": ("yr = np.clip(ys, 1, ny - 2)", "yr = ys"),
    "corners belong to the side walls": ("uw = np.where(ys == ny - 1, u_lid, 0.0)",
                                         "uw = np.where((ys == ny - 1) & (xs > 0) & (xs < nx - 1), "
                                         "u_lid, 0.0)"),
    "wall density taken as 1": ("feq_w = equilibrium(rf, uw", "feq_w = equilibrium(1.0 + 0 * rf, uw"),
    "L counted in nodes": ("u_lid * (nx - 1) / re", "u_lid * nx / re"),
    "streaming from the wrong side": ("src_x = np.mod(xs - cx, nx) if periodic_x else xs - cx",
                                      "src_x = np.mod(xs + cx, nx) if periodic_x else xs + cx"),
}


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle.mutated_nee")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "mutated_nee", "exec"), mod.__dict__)
    return mod


def _battery(m):
    failed = []
    if not math.isclose(m.relaxation_time(257, 400.0, U), 0.692, rel_tol=1e-14):
        failed.append("tau")
    if _brute_force_gap(m, 5, 4, 20.0, 20) > 2e-15 or _brute_force_gap(m, 6, 7, 20.0, 10, 1) > 2e-15:
        failed.append("twin")
    c = m.CavityNEE(9, 7, re=100.0, u_lid=U).step(1)
    rho, ux, _ = c.moments()
    if not (np.allclose(ux[5, 1:-1], U / 6, rtol=0, atol=1e-16)
            and np.allclose(rho[5, 1:-1], 1, rtol=0, atol=1e-15)):
        failed.append("first step")
    c = m.CavityNEE(4, 7, tau=0.8, u_lid=U, periodic_x=True).step(2000)
    _, ux, _ = c.moments()
    if np.abs(ux - U * np.arange(7)[:, None] / 6).max() > 1e-10:
        failed.append("couette")
    return failed


def test_unmodified_nee_oracle_passes_the_battery():
    assert _battery(_mutant("import numpy as np", "import numpy as np")) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_battery_rejects_mutation(name):
    assert _battery(_mutant(*MUTATIONS[name])), f"mutation '{name}' was not caught"
