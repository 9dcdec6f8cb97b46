"""Pins of the oracle's monitors (Eq. 6 residual, probes, stream function)."""
import math

import numpy as np

from oracle import monitors


def test_residual_definition():
    """Eq. 6: relative L2 change of (u_x, u_y) over 100 steps, denominator at
    the earlier time."""
    ux0 = np.full((3, 4), 0.2)
    uy0 = np.zeros((3, 4))
    assert math.isclose(monitors.residual(1.1 * ux0, uy0, ux0, uy0), 0.1, rel_tol=1e-14)
    # a pure rotation of every vector by 90 degrees: |du|^2 = 2 |u|^2
    assert math.isclose(monitors.residual(-uy0, ux0, ux0, uy0), math.sqrt(2), rel_tol=1e-14)
    assert monitors.residual(ux0, uy0, np.zeros((3, 4)), uy0) == math.inf
    assert monitors.residual(ux0, uy0, ux0, uy0) == 0.0


def test_stream_function_of_uniform_and_couette_flow():
    """Psi = 0 on the bottom wall, dPsi/dy = -u_x, midpoint rule on site
    centres: uniform u_x = a gives Psi = -a (y + 1/2); the Couette profile
    u_x = U (y + 1/2)/H gives Psi = -U/H ((y + 1/2)^2/2 + 1/8)."""
    ny, nx = 7, 3
    y = np.arange(ny)[:, None] + np.zeros((1, nx))
    psi = monitors.stream_function(np.full((ny, nx), 0.3))
    assert np.allclose(psi, -0.3 * (y + 0.5), atol=1e-15, rtol=0)
    U, H = 0.1, ny
    psi = monitors.stream_function(U * (y + 0.5) / H)
    assert np.allclose(psi, -U / H * ((y + 0.5) ** 2 / 2 + 1 / 8), atol=1e-15, rtol=0)


def test_vortex_extrema_locates_planted_extrema():
    """Primary = global max of Psi; lower-left / lower-right = min over the
    bottom quarter on each side; positions are site centres in units of L."""
    nx, ny = 20, 24
    psi = np.zeros((ny, nx))
    psi[15, 11] = 0.12
    psi[2, 1] = -1e-4
    psi[3, 17] = -2e-3
    psi[20, 3] = -5.0      # above the bottom quarter: not a corner vortex
    ext = monitors.vortex_extrema(psi, nx)
    assert ext["primary"] == (0.12, 11.5 / nx, 15.5 / nx)
    assert ext["lower_left"] == (-1e-4, 1.5 / nx, 2.5 / nx)
    assert ext["lower_right"] == (-2e-3, 17.5 / nx, 3.5 / nx)


def test_probe_is_exact_on_linear_fields_and_on_site_centres():
    """Bilinear interpolation over site centres reproduces a linear field
    exactly inside the centre hull, returns the site value at a centre, and
    clamps to the outermost centres outside it."""
    nx, ny = 10, 6
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    field = 0.3 + 0.02 * X - 0.05 * Y
    pts = [(0.37, 0.21), (0.5, 0.3), (0.91, 0.52)]
    out = monitors.probe(field, field, 2 * field, pts)
    for (px, py), row in zip(pts, out):
        exp = 0.3 + 0.02 * px * nx - 0.05 * py * nx
        assert math.isclose(row[0], exp, rel_tol=1e-14)
        assert math.isclose(row[2], 2 * exp, rel_tol=1e-14)
    rnd = np.random.default_rng(0).uniform(size=(ny, nx))
    val = monitors.probe(rnd, rnd, rnd, [((3 + 0.5) / nx, (2 + 0.5) / nx)])[0, 0]
    assert val == rnd[2, 3]
    corner = monitors.probe(rnd, rnd, rnd, [(0.0, 0.0), (1.0, 5.0)])
    assert corner[0, 0] == rnd[0, 0] and corner[1, 0] == rnd[-1, -1]


def test_centreline_even_and_odd():
    ux = np.arange(12.0).reshape(3, 4)
    uy = np.arange(12.0).reshape(3, 4) * 2
    u, v = monitors.centreline(ux, uy)
    assert np.array_equal(u, 0.5 * (ux[:, 1] + ux[:, 2]))
    assert np.array_equal(v, uy[1])


def _cells(P=7, Q=9, a=3, b=2, ramp=0.1):
    """Psi = sin(pi (x + 1/2) / P) sin(pi (y + 1/2) / Q) (1 + ramp y / Ny) on
    a P x Q-cell checkerboard: odd P and Q put each cell's extremum exactly
    on a site, with both neighbours in each direction strictly lower."""
    nx, ny = a * P, b * Q
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    psi = np.sin(np.pi * (x + 0.5) / P) * np.sin(np.pi * (y + 0.5) / Q) * (1 + ramp * y / ny)
    return psi, P, Q, a, b


def test_vortex_centres_of_a_checkerboard():
    psi, P, Q, a, b = _cells()
    got = monitors.vortex_centres(psi)
    want = []
    for cb in range(b):
        for ca in range(a):
            j, i = cb * Q + (Q - 1) // 2, ca * P + (P - 1) // 2
            want.append((j, i, 1 if (ca + cb) % 2 == 0 else -1, psi[j, i]))
    assert got == want
    # the threshold drops the weaker bottom row: |Psi| = 1 + ramp * 4/18 there
    thr = 0.5 * (abs(psi[4, 3]) + abs(psi[13, 3]))
    assert [c[:2] for c in monitors.vortex_centres(psi, thr)] == [(13, 3), (13, 10), (13, 17)]
    assert monitors.vortex_centres(psi, 10.0) == []


def test_vortex_centres_need_a_strict_extremum():
    y, x = np.mgrid[0:21, 0:21].astype(np.float64)
    assert monitors.vortex_centres((x - 10) ** 2 - (y - 10) ** 2) == []      # saddle
    assert monitors.vortex_centres(np.full((9, 9), 0.25)) == []             # plateau
    assert monitors.vortex_centres(monitors.stream_function(0.01 * y)) == []  # shear flow
    bump = -((x - 10) ** 2 + (y - 10) ** 2)
    assert monitors.vortex_centres(bump) == [(10, 10, 1, 0.0)]
    bump[10, 11] = 0.0                        # a tie with a neighbour: not strict
    assert monitors.vortex_centres(bump) == []
    # above its four axis neighbours but below a diagonal one: not a centre
    assert monitors.vortex_centres((x + y) - 3 * (x - y) ** 2) == []
    # the outer ring is never a candidate
    edge = np.zeros((5, 5))
    edge[0, 2] = edge[2, 0] = 1.0
    assert monitors.vortex_centres(edge) == []
    assert monitors.vortex_centres(np.zeros((2, 7))) == []


def test_bottom_vortex_count():
    psi, *_ = _cells()
    # the ramp makes the top row of cells stronger: the primary is the top
    # row's first maximum, and the three centres of the bottom row lie below it
    assert monitors.bottom_vortex_count(psi) == 3
    assert monitors.bottom_vortex_count(psi[::-1].copy()) == 0
    psi3, *_ = _cells(b=3)
    assert monitors.bottom_vortex_count(psi3) == 6


def test_node_stream_function_closed_forms():
    """Trapezoid rule from the bottom wall row: exact for uniform and linear
    (Couette) profiles on nodes y = 0 ... Ny - 1."""
    ny, nx, U = 9, 4, 0.1
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    assert np.allclose(monitors.stream_function_nodes(np.full((ny, nx), 0.03)), -0.03 * y,
                       rtol=0, atol=1e-16)
    psi = monitors.stream_function_nodes(U * y / (ny - 1))
    assert np.allclose(psi, -U * y ** 2 / (2 * (ny - 1)), rtol=0, atol=1e-16)
    assert np.all(psi[0] == 0)


def test_on_node_positions():
    nx = 11
    psi = np.zeros((8, nx))
    psi[5, 3] = 2.0
    psi[1, 2] = -1.0
    psi[2, 8] = -0.5
    ext = monitors.vortex_extrema(psi, nx, on_node=True)
    assert ext["primary"] == (2.0, 0.3, 0.5)
    assert ext["lower_left"] == (-1.0, 0.2, 0.1)
    assert ext["lower_right"] == (-0.5, 0.8, 0.2)
    # probe at nodes and between them (node i at i / (nx - 1))
    yy, xx = np.mgrid[0:8, 0:nx].astype(np.float64)
    f = 3.0 + 0.5 * xx - 0.25 * yy
    got = monitors.probe(f, f, f, [(0.3, 0.5), (0.35, 0.05)], on_node=True)
    assert np.allclose(got[:, 0], [3.0 + 1.5 - 1.25, 3.0 + 1.75 - 0.125], rtol=0, atol=1e-15)
