"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
exact invariant, a special case, a textbook solution, or an independently
written brute-force twin (arXiv 2211.05009, Sec. 2.1 Eqs. 1-3 and 5).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from cavity_inputs import random_shift
from oracle import d2q9
from oracle.d2q9 import C, OPP, W, Cavity, equilibrium, relaxation_time
from oracle.naive import naive_steps


# ---------------------------------------------------------------- lattice ---
def test_lattice_isotropy_closed_forms():
    """D2Q9 weights (Sec. 2.1): sum w = 1, sum w c = 0, sum w c c = c_s^2 I,
    fourth-order isotropy sum w cx^2 cy^2 = c_s^4 and sum w cx^4 = 3 c_s^4."""
    assert math.isclose(W.sum(), 1.0, rel_tol=0, abs_tol=2e-16)
    assert np.all(np.abs(W @ C) < 1e-17)
    M2 = np.einsum("i,ia,ib->ab", W, C.astype(float), C.astype(float))
    assert np.allclose(M2, np.eye(2) / 3.0, atol=1e-16, rtol=0)
    cx, cy = C[:, 0].astype(float), C[:, 1].astype(float)
    assert math.isclose(W @ (cx**2 * cy**2), 1 / 9, rel_tol=1e-15)
    assert math.isclose(W @ cx**4, 3 / 9, rel_tol=1e-15)
    for i in range(9):
        assert np.all(C[OPP[i]] == -C[i])
        assert W[OPP[i]] == W[i]


def test_relaxation_time_values():
    """Eq. 5 with nu = U L / Re (Sec. 1), lattice units (Sec. 3)."""
    assert math.isclose(relaxation_time(64, 100, 0.1), 0.692, rel_tol=1e-15)
    assert math.isclose(relaxation_time(500, 8000, 0.1), 0.51875, rel_tol=1e-15)
    assert math.isclose(relaxation_time(500, 1000, 0.1), 0.65, rel_tol=1e-15)
    assert math.isclose(relaxation_time(4096, 1e4, 0.1), 0.62288, rel_tol=1e-15)
    with pytest.raises(ValueError):
        Cavity(8, 8, tau=0.5)


def test_equilibrium_moments_closed_form():
    """Eq. 2 reproduces rho, rho u (Eq. 3) and the Euler stress
    rho c_s^2 I + rho u u exactly."""
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.9, 1.1, 500)
    ux = rng.uniform(-0.14, 0.14, 500)
    uy = rng.uniform(-0.14, 0.14, 500)
    feq = equilibrium(rho, ux, uy)
    cx, cy = C[:, 0].astype(float), C[:, 1].astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=1e-15, atol=0)
    assert np.allclose(cx @ feq, rho * ux, rtol=0, atol=1e-16)
    assert np.allclose(cy @ feq, rho * uy, rtol=0, atol=1e-16)
    assert np.allclose((cx * cx) @ feq, rho / 3 + rho * ux * ux, rtol=1e-15, atol=0)
    assert np.allclose((cy * cy) @ feq, rho / 3 + rho * uy * uy, rtol=1e-15, atol=0)
    assert np.allclose((cx * cy) @ feq, rho * ux * uy, rtol=0, atol=1e-16)
    # the rest state is the weights themselves
    assert np.array_equal(equilibrium(np.ones(1), np.zeros(1), np.zeros(1))[:, 0], W)


# ---------------------------------------------------- special cases, BB ---
def test_rest_state_is_a_fixed_point():
    """U = 0: f = w stays f = w (collision of an equilibrium is the identity,
    every wall reflection is a plain reversal)."""
    c = Cavity(9, 7, tau=0.6, u_lid=0.0)
    c.step(50)
    assert np.max(np.abs(c.f - W[:, None, None])) <= 2e-16


def test_first_step_from_rest_closed_form():
    """One application of Eq. 1 from rest: only the lid-row populations 7 and
    8 change, by -U/6 and +U/6 (moving-wall term -6 w rho_w c.u_w with
    w = 1/36), corners included; every site keeps rho = 1 and the lid row
    gets u_x = U/3."""
    U = 0.1
    c = Cavity(6, 5, tau=0.7, u_lid=U)
    c.step(1)
    exp = np.broadcast_to(W[:, None, None], c.f.shape).copy()
    exp[7, -1, :] -= U / 6
    exp[8, -1, :] += U / 6
    assert np.max(np.abs(c.f - exp)) <= 5e-16      # a few ulps of 4/9
    rho, ux, uy = c.moments()
    assert np.max(np.abs(rho - 1)) <= 4.5e-16
    assert np.allclose(ux[-1], U / 3, atol=1e-16, rtol=0)
    assert np.max(np.abs(ux[:-1])) == 0 and np.max(np.abs(uy)) <= 3e-17


def test_mirror_symmetry():
    """Reflecting x -> Nx-1-x and reversing the lid maps the solution onto
    itself with u_x -> -u_x (populations 1<->3, 5<->6, 7<->8)."""
    a = Cavity(12, 9, tau=0.56, u_lid=0.1).step(1000)
    b = Cavity(12, 9, tau=0.56, u_lid=-0.1).step(1000)
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    fb = b.f[perm][:, :, ::-1]
    assert np.max(np.abs(a.f - fb)) <= 1e-14
    ra, uxa, uya = a.moments()
    assert np.max(np.abs(uxa)) > 1e-3          # the flow is not trivial


def test_stream_is_a_permutation_without_lid_motion():
    """With U = 0 the streaming + reflection step only moves numbers: the
    multiset of values is preserved bit for bit."""
    fs = W[:, None, None] + random_shift(7, 5, seed=3)
    out = d2q9.stream(fs, u_lid=0.0)
    assert np.array_equal(np.sort(out.ravel()), np.sort(fs.ravel()))


def test_exact_mass_conservation_rational():
    """In exact rational arithmetic, collision conserves mass and momentum
    and streaming with bounce-back conserves mass exactly, moving lid
    included (the two lid corrections of each lid-row site cancel)."""
    w = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    for nx, ny in ((3, 3), (4, 3)):
        f0 = [[[w[i] + Fraction((7 * i + 3 * y + 5 * x) % 11 - 5, 2000)
                for x in range(nx)] for y in range(ny)] for i in range(9)]
        m0 = sum(f0[i][y][x] for i in range(9) for y in range(ny) for x in range(nx))
        f3 = naive_steps(f0, Fraction(3, 5), Fraction(1, 10), 3, num=Fraction)
        m3 = sum(f3[i][y][x] for i in range(9) for y in range(ny) for x in range(nx))
        assert m3 == m0


def test_mass_drift_is_rounding_only():
    """FP64 mass over 20,000 steps of a driven cavity.  In exact arithmetic it
    is constant (previous test); in FP64 the only change is rounding, which
    has no preferred sign once the weights are applied exactly (measured
    6.9e-15 of the mass; with FP64-rounded weights every collision would
    remove ~1e-16 and the drift would reach ~1e-12).  A wrong reflection or
    an uncancelled lid term would change it by ~U/6 per lid site per step."""
    c = Cavity(16, 16, tau=0.55, u_lid=0.1)
    m0 = d2q9.mass(c.f)
    c.step(20000)
    assert abs(d2q9.mass(c.f) - m0) / m0 <= 1e-13
    # one collision conserves the site mass and momentum to rounding: the
    # site masses are near 1 (ulp 2.2e-16) and the two nine-term sums and the
    # nine relaxed populations each round, so allow three ulps
    f = W[:, None, None] + random_shift(5, 4, seed=4)
    fs = d2q9.collide(f, 0.53)
    assert np.max(np.abs(fs.sum(0) - f.sum(0))) <= 3 * 2.0 ** -52
    jx0, jy0 = d2q9.momentum(f)
    jx1, jy1 = d2q9.momentum(fs)
    assert np.max(np.abs(jx1 - jx0)) <= 4e-16 and np.max(np.abs(jy1 - jy0)) <= 4e-16


def test_collision_rounds_without_bias():
    """Eq. 2's weights are exact rationals (4/9, 1/9, 1/36).  Rounded to FP64
    constants they would all lie 5.6e-17 (relative) low, and every collision
    would take ~1e-16 of a site's mass away (8e-17 to 1.1e-16 measured at these
    two tau), the same way each step: over the 1e5-step relaxation of a steady
    cavity that drift moves u = j / rho by ~1.5e-12 U.  With the weights
    applied exactly, the mean change over 60,000 random sites is rounding
    noise that averages out (a few 1e-19)."""
    f = W[:, None, None] + random_shift(300, 200, seed=5)
    for tau in (0.51875, 0.692):
        dm = d2q9.collide(f, tau).sum(0) - f.sum(0)
        assert abs(np.mean(dm)) <= 1e-17, tau


# ------------------------------------------------------- closed forms -----
@pytest.mark.parametrize("tau", [0.6, 0.8, 1.5])
def test_couette_closed_form(tau):
    """Periodic in x, bottom at rest, lid at U: the half-way bounce-back
    steady state is exactly u_x = U (y + 1/2) / H, u_y = 0, rho = 1, for any
    tau (walls at y = -1/2 and y = H - 1/2)."""
    H, U = 8, 0.1
    nu = (tau - 0.5) / 3
    c = Cavity(4, H, tau=tau, u_lid=U, periodic_x=True)
    c.step(int(40 * H * H / (math.pi ** 2 * nu)))
    rho, ux, uy = c.moments()
    exact = U * (np.arange(H) + 0.5) / H
    assert np.max(np.abs(ux - exact[:, None])) <= 1e-12 * U
    assert np.max(np.abs(uy)) <= 1e-13
    assert np.max(np.abs(rho - 1)) <= 1e-12


@pytest.mark.parametrize("tau", [0.6, 0.8, 0.5 + math.sqrt(3) / 4, 1.2])
def test_poiseuille_closed_form(tau):
    """Periodic channel, both walls at rest, Guo body force g: the BGK
    half-way bounce-back steady state is the parabola through the half-way
    walls plus a uniform slip g (16 L - 3) / (24 nu), L = (tau - 1/2)^2,
    which vanishes at tau = 1/2 + sqrt(3)/4."""
    H = 8
    nu = (tau - 0.5) / 3
    g = 0.01 * 8 * nu / H ** 2                      # centre-line speed ~0.01
    c = Cavity(4, H, tau=tau, u_lid=0.0, periodic_x=True, force=(g, 0.0))
    c.step(int(45 * H * H / (math.pi ** 2 * nu)))
    rho, ux, uy = c.moments()
    y = np.arange(H)
    lam = (tau - 0.5) ** 2
    exact = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y) + g * (16 * lam - 3) / (24 * nu)
    assert np.max(np.abs(ux - exact[:, None])) <= 1e-12 * np.max(exact)


def _taylor_green_nu_error(N, tau, U0=0.01):
    k = 2 * math.pi / N
    nu = (tau - 0.5) / 3
    x = np.arange(N, dtype=float)
    X, Y = np.meshgrid(x, x)                       # [y, x]
    ux = -U0 * np.cos(k * X) * np.sin(k * Y)
    uy = U0 * np.sin(k * X) * np.cos(k * Y)
    rho = 1 + 3 * (-U0 ** 2 / 4) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    c = Cavity(N, N, tau=tau, u_lid=0.0, periodic_x=True, periodic_y=True)
    c.set_state(equilibrium(rho, ux, uy))
    T = int(round(0.5 / (2 * nu * k * k)))
    c.step(T)
    a1 = np.abs(c.moments()[1]).max()
    c.step(T)
    a2 = np.abs(c.moments()[1]).max()
    return math.log(a1 / a2) / T / (2 * k * k) / nu - 1


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_taylor_green_viscosity(tau):
    """Fully periodic Taylor-Green vortex: u decays as exp(-2 nu k^2 t) with
    nu = (tau - 1/2)/3 (Eq. 5); the lattice error is second order in k."""
    e16 = _taylor_green_nu_error(16, tau)
    e32 = _taylor_green_nu_error(32, tau)
    e64 = _taylor_green_nu_error(64, tau)
    assert abs(e32) < 1e-2 and abs(e64) < 2e-3
    assert 3.5 < e16 / e32 < 4.5 and 3.5 < e32 / e64 < 4.5


# ------------------------------------------------------- brute force ------
@pytest.mark.parametrize("nx,ny,tau,u", [(3, 3, 0.6, 0.1), (4, 6, 0.52, 0.1),
                                         (5, 5, 1.3, -0.05), (7, 4, 0.75, 0.2)])
def test_vectorised_matches_naive_twin(nx, ny, tau, u):
    """The vectorised oracle (pull form) against the pure-Python push-form
    twin, from a random state, for 200 steps.  Both apply the weights
    exactly, so they differ only in the order of their roundings: measured
    at most 8.9e-16 (16 ulps of the largest population)."""
    f0 = W[:, None, None] + random_shift(nx, ny, seed=nx * 10 + ny)
    c = Cavity(nx, ny, tau=tau, u_lid=u)
    c.set_state(f0)
    c.step(200)
    ref = np.array(naive_steps(f0, tau, u, 200))
    assert np.max(np.abs(c.f - ref)) <= 1e-15


# ------------------------------------------- period-two invariants -------
@pytest.mark.parametrize("nx,ny", [(8, 6), (7, 5)])
def test_staggered_momenta_alternate_exactly(nx, ny):
    """Collision keeps j per site; links and reflections flip the column (or
    row) parity of every population with c_x (c_y) != 0: P_x, P_y change
    sign each step, P_x gains u/3 per step from the lid term when Nx is odd."""
    U = 0.1
    c = Cavity(nx, ny, tau=0.6, u_lid=U)
    c.set_state(W[:, None, None] + random_shift(nx, ny, 3))
    for _ in range(5):
        px, py = d2q9.staggered_momenta(c.f)
        c.step(1)
        qx, qy = d2q9.staggered_momenta(c.f)
        assert abs(qx + px - (U / 3 if nx % 2 else 0.0)) < 1e-14
        assert abs(qy + py) < 1e-14


def test_steady_state_is_set_by_mass_and_staggered_momenta():
    """A start from a random field converges to the cold-start steady state
    only once its staggered momenta are removed (both have P = 0)."""
    nx, ny, re = 16, 12, 40.0
    rng = np.random.default_rng(0)
    rho = 1 + 0.01 * rng.standard_normal((ny, nx))
    rho *= nx * ny / rho.sum()
    ux = 0.02 * rng.standard_normal((ny, nx))
    uy = 0.02 * rng.standard_normal((ny, nx))
    cold = Cavity(nx, ny, re=re)
    raw = Cavity(nx, ny, re=re)
    raw.set_state(equilibrium(rho, ux, uy))
    fixed = Cavity(nx, ny, re=re)
    vx, vy = d2q9.destaggered_velocity(rho, ux, uy)
    fixed.set_state(equilibrium(rho, vx, vy))
    assert max(abs(v) for v in d2q9.staggered_momenta(fixed.f)) < 1e-14
    for c in (cold, raw, fixed):
        c.step(12000)
    _, u0, v0 = cold.moments()
    _, u1, v1 = raw.moments()
    _, u2, v2 = fixed.moments()
    assert np.max(np.abs(u2 - u0)) < 1e-11 and np.max(np.abs(v2 - v0)) < 1e-11
    assert np.max(np.abs(u1 - u0)) > 1e-5
