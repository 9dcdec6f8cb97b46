"""Pins of the D3Q19 lid-driven cube oracle (oracle/d3q19.py), the 3-D
extension Sec. 4 names as future work."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import d2q9, d3q19 as D
from oracle.naive import naive_steps_3d

U = 0.1


def test_velocity_set_and_weights():
    assert len(D.C) == 19 and math.isclose(D.W.sum(), 1.0, rel_tol=1e-15)
    assert np.all(D.C[D.OPP] == -D.C)
    cc = np.einsum("i,ia,ib->ab", D.W, D.C.astype(float), D.C.astype(float))
    assert np.allclose(cc, np.eye(3) / 3, rtol=0, atol=3e-16)       # isotropy, c_s^2 = 1/3
    c4 = np.einsum("i,ia,ib,ic,id->abcd", D.W, *(D.C.astype(float),) * 4)
    d = np.eye(3)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(c4, want, rtol=0, atol=3e-16)                 # fourth-order isotropy


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho, ux, uy, uz = rng.uniform(0.9, 1.1, 40), *rng.uniform(-0.1, 0.1, (3, 40))
    feq = D.equilibrium(rho, ux, uy, uz)
    c = D.C.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=1e-14, atol=0)
    for a, u in enumerate((ux, uy, uz)):
        assert np.allclose(c[:, a] @ feq, rho * u, rtol=0, atol=1e-15)
    u = (ux, uy, uz)
    for a in range(3):
        for b in range(3):
            want = rho * u[a] * u[b] + (rho / 3 if a == b else 0.0)
            assert np.allclose((c[:, a] * c[:, b]) @ feq, want, rtol=0, atol=1e-15)


def test_z_invariant_flow_is_the_two_dimensional_cavity():
    """Summed over c_z the D3Q19 weights are the D2Q9 weights and the
    equilibrium at u_z = 0 is the D2Q9 one, so a z-periodic, z-invariant
    state evolves exactly as the 2-D cavity (walls included)."""
    nx, ny, nz = 12, 9, 3
    c3 = D.Cube(nx, ny, nz, re=50.0, u_lid=U, periodic_z=True).step(200)
    c2 = d2q9.Cavity(nx, ny, re=50.0, u_lid=U).step(200)
    r3, u3, v3, w3 = c3.moments()
    r2, u2, v2 = c2.moments()
    assert np.abs(r3 - r2[None]).max() <= 5e-15
    assert max(np.abs(u3 - u2[None]).max(), np.abs(v3 - v2[None]).max()) <= 5e-15
    assert np.abs(w3).max() <= 1e-15


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 3, 2), (2, 5, 3)])
def test_matches_the_push_form_twin(shape):
    nx, ny, nz = shape
    c = D.Cube(nx, ny, nz, re=10.0, u_lid=U)
    rng = np.random.default_rng(nx * ny * nz)
    c.set_state(c.f + rng.uniform(-4e-3, 4e-3, c.f.shape))
    f0 = c.f.copy()
    c.step(8)
    assert np.abs(np.array(naive_steps_3d(f0, c.tau, U, 8)) - c.f).max() <= 2e-15


def test_mass_is_conserved_exactly():
    """In rational arithmetic the closed box keeps its mass exactly (the lid
    term moves momentum between a link and its reverse at the same site)."""
    nx, ny, nz = 3, 3, 2
    f0 = D.equilibrium(np.ones((nz, ny, nx)), np.zeros((nz, ny, nx)),
                       np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)))
    fr = [[[[Fraction(f0[i, z, y, x]).limit_denominator(10 ** 6) for x in range(nx)]
            for y in range(ny)] for z in range(nz)] for i in range(19)]
    m0 = sum(v for a in fr for b in a for c in b for v in c)
    out = naive_steps_3d(fr, Fraction(4, 5), Fraction(1, 10), 2, num=Fraction)
    assert sum(v for a in out for b in a for c in b for v in c) == m0


def test_collision_rounds_without_bias():
    """The weights 1/3, 1/18, 1/36 enter as whole 36ths: one collision changes
    the mass only by rounding noise that averages out over many sites (with
    the weights rounded to FP64 constants every collision would remove ~1e-16
    of each site's mass, the same way every step)."""
    rng = np.random.default_rng(5)
    shape = (8, 40, 50)
    f = D.equilibrium(np.ones(shape), np.zeros(shape), np.zeros(shape), np.zeros(shape))
    f = f + rng.uniform(-4e-3, 4e-3, f.shape)
    for tau in (0.51875, 0.692):
        dm = D.collide(f, tau).sum(0) - f.sum(0)
        assert abs(np.mean(dm)) <= 1e-17, tau


def test_first_step_closed_form_and_rest():
    """From rest the only change after one step is the lid term on the top
    row: f_9 (c = (1,-1,0)) gains U/6 and f_8 (c = (-1,-1,0)) loses U/6 at
    every top site, the three other downward links are unchanged, so the top
    row carries rho u_x = 2 U / 6 = U / 3 and nothing else moves."""
    nx, ny, nz = 5, 4, 3
    c = D.Cube(nx, ny, nz, re=30.0, u_lid=U)
    f0 = c.f.copy()
    c.step(1)
    d = c.f - f0
    assert np.allclose(d[9, :, ny - 1, :], U / 6, rtol=0, atol=1e-16)
    assert np.allclose(d[8, :, ny - 1, :], -U / 6, rtol=0, atol=1e-16)
    d[9, :, ny - 1, :] = 0
    d[8, :, ny - 1, :] = 0
    # sum_i w_i rounds to 1 + O(1e-16), so rest values move by an ulp or two
    assert np.abs(d).max() <= 3e-16
    rest = D.Cube(nx, ny, nz, tau=0.8, u_lid=0.0)
    g0 = rest.f.copy()
    assert np.abs(rest.step(20).f - g0).max() <= 3e-16


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_couette_between_the_lid_and_the_bottom(tau):
    """x and z periodic: steady u_x = U (y + 1/2) / Ny, as in two dimensions."""
    ny = 6
    c = D.Cube(2, ny, 2, tau=tau, u_lid=U, periodic_x=True, periodic_z=True).step(3000)
    _, ux, uy, uz = c.moments()
    y = (np.arange(ny) + 0.5)[None, :, None]
    assert np.abs(ux - U * y / ny).max() <= 1e-12
    assert max(np.abs(uy).max(), np.abs(uz).max()) <= 1e-14


def test_mirror_symmetry_in_z():
    """The lid moves along x, so z -> Nz - 1 - z maps the box onto itself:
    u_x, u_y even and u_z odd in z."""
    c = D.Cube(6, 5, 4, re=20.0, u_lid=U).step(60)
    r, ux, uy, uz = c.moments()
    assert np.abs(ux - ux[::-1]).max() <= 5e-16 and np.abs(uy - uy[::-1]).max() <= 5e-16
    assert np.abs(uz + uz[::-1]).max() <= 5e-16 and np.abs(r - r[::-1]).max() <= 2e-15
