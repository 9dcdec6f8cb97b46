"""Monitors of the cavity run (oracle; test infrastructure only).

* ``residual``        -- Sec. 2.2 (iii), Eq. 6: relative L2 change of the
                         velocity field over 100 steps, denominator at the
                         earlier time; +inf when that denominator is zero.
* ``stream_function`` -- Psi with Psi = 0 on the bottom wall and
                         dPsi/dy = -u_x (so the clockwise primary vortex has
                         Psi > 0, the sign of Tables 1-2), midpoint rule on
                         site centres, lattice units.
* ``probe``           -- velocity at an observing point (Sec. 3.3) given in
                         units of the cavity width L, bilinear over site
                         centres ((i + 1/2) / Nx), clamped to the outermost
                         centres.
* ``centreline``      -- u_x on the vertical line x = L/2 and u_y on the
                         horizontal line y = H/2 (Figs. 1-2), averaging the two
                         central columns / rows when the count is even.
* ``vortex_extrema``  -- the primary vortex (max Psi) and the two bottom
                         corner vortices (min Psi in each bottom quadrant), with
                         centre positions in units of L, as in Tables 1-2.
* ``vortex_centres``  -- every vortex centre: an interior site where Psi is a
                         strict extremum of its 3 x 3 neighbourhood.
* ``stream_function_nodes`` -- Psi on a lattice whose walls lie on the
                         outermost nodes (the paper's own wall scheme): Psi = 0
                         on the bottom row, trapezoid rule up each column.

``probe`` and ``vortex_extrema`` take ``on_node=True`` for such lattices: node
i then sits at i / (Nx - 1) in units of L.
* ``bottom_vortex_count`` -- the vortex centres below the primary vortex
                         (the count of Table 2's last column).
"""
from __future__ import annotations

import math

import numpy as np


def mass(rho):
    """Sum of rho over all sites, exactly rounded (math.fsum)."""
    return math.fsum(np.asarray(rho, dtype=np.float64).ravel().tolist())


def residual(ux_new, uy_new, ux_old, uy_old):
    """Eq. 6 with (u_x, u_y)(t) = *_old and (u_x, u_y)(t + 100) = *_new."""
    num = math.fsum(((np.asarray(ux_new) - ux_old) ** 2
                     + (np.asarray(uy_new) - uy_old) ** 2).ravel().tolist())
    den = math.fsum((np.asarray(ux_old) ** 2
                     + np.asarray(uy_old) ** 2).ravel().tolist())
    if den == 0.0:
        return math.inf
    return math.sqrt(num / den)


def stream_function(ux):
    """Psi[y, x] = -(sum_{y' < y} u_x[y', x] + u_x[y, x] / 2) (lattice units)."""
    ux = np.asarray(ux, dtype=np.float64)
    below = np.zeros_like(ux)
    below[1:] = np.cumsum(ux, axis=0)[:-1]
    return -(below + 0.5 * ux)


def stream_function_nodes(ux):
    """Psi[0, x] = 0, Psi[y, x] = Psi[y-1, x] - (u_x[y-1, x] + u_x[y, x]) / 2."""
    ux = np.asarray(ux, dtype=np.float64)
    psi = np.zeros_like(ux)
    for y in range(1, ux.shape[0]):
        psi[y] = psi[y - 1] - 0.5 * (ux[y - 1] + ux[y])
    return psi


def _bilinear(field, X, Y):
    ny, nx = field.shape
    X = min(max(X, 0.0), nx - 1.0)
    Y = min(max(Y, 0.0), ny - 1.0)
    i0 = min(int(math.floor(X)), max(nx - 2, 0))
    j0 = min(int(math.floor(Y)), max(ny - 2, 0))
    i1 = min(i0 + 1, nx - 1)
    j1 = min(j0 + 1, ny - 1)
    tx = X - i0
    ty = Y - j0
    return ((1 - tx) * (1 - ty) * field[j0, i0] + tx * (1 - ty) * field[j0, i1]
            + (1 - tx) * ty * field[j1, i0] + tx * ty * field[j1, i1])


def probe(rho, ux, uy, points, on_node=False):
    """(rho, u_x, u_y) at each point (x, y), coordinates in units of L = Nx.

    Site (i, j) has its centre at ((i + 1/2)/Nx, (j + 1/2)/Nx); with
    on_node, node (i, j) sits at (i, j)/(Nx - 1) and L = Nx - 1."""
    nx = np.asarray(rho).shape[1]
    out = []
    for (px, py) in points:
        if on_node:
            X = px * (nx - 1)
            Y = py * (nx - 1)
        else:
            X = px * nx - 0.5
            Y = py * nx - 0.5
        out.append([_bilinear(np.asarray(rho), X, Y),
                    _bilinear(np.asarray(ux), X, Y),
                    _bilinear(np.asarray(uy), X, Y)])
    return np.array(out, dtype=np.float64)


def centreline(ux, uy):
    """(u_x along x = L/2 as a function of y, u_y along y = H/2 as a function
    of x); central two columns/rows averaged for even counts."""
    ux = np.asarray(ux)
    uy = np.asarray(uy)
    ny, nx = ux.shape
    if nx % 2 == 0:
        u_vert = 0.5 * (ux[:, nx // 2 - 1] + ux[:, nx // 2])
    else:
        u_vert = ux[:, nx // 2].copy()
    if ny % 2 == 0:
        v_horz = 0.5 * (uy[ny // 2 - 1, :] + uy[ny // 2, :])
    else:
        v_horz = uy[ny // 2, :].copy()
    return u_vert, v_horz


def vortex_extrema(psi, nx, on_node=False):
    """Primary vortex = global max of Psi; lower-left / lower-right vortices =
    min of Psi over the bottom-left / bottom-right quarter (x < W/2 or
    x >= W/2, y < W/2, W = Nx sites or nodes).  Positions are site centres in
    units of L = Nx (on_node: node positions i / (Nx - 1)).  Returns a dict of
    (value, x, y)."""
    psi = np.asarray(psi)
    ny = psi.shape[0]

    def pos(i):
        return i / (nx - 1) if on_node else (i + 0.5) / nx

    res = {}
    j, i = np.unravel_index(int(np.argmax(psi)), psi.shape)
    res["primary"] = (float(psi[j, i]), pos(i), pos(j))
    hy = min(ny, nx // 2)
    for name, xs in (("lower_left", slice(0, nx // 2)),
                     ("lower_right", slice(nx // 2, nx))):
        sub = psi[:hy, xs]
        jj, ii = np.unravel_index(int(np.argmin(sub)), sub.shape)
        ii += xs.start
        res[name] = (float(psi[jj, ii]), pos(ii), pos(jj))
    return res


def vortex_centres(psi, min_abs=0.0):
    """Sites (iy, ix) with 1 <= ix <= Nx-2 and 1 <= iy <= Ny-2 where Psi is
    strictly greater (kind +1) or strictly smaller (kind -1) than at all
    eight neighbours, and |Psi| >= min_abs.  Returns (iy, ix, kind, psi)
    tuples in row-major order."""
    psi = np.asarray(psi, dtype=np.float64)
    ny, nx = psi.shape
    if nx < 3 or ny < 3:
        return []
    c = psi[1:-1, 1:-1]
    is_max = np.ones(c.shape, dtype=bool)
    is_min = np.ones(c.shape, dtype=bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = psi[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
            is_max &= c > nb
            is_min &= c < nb
    keep = np.abs(c) >= min_abs
    out = []
    for j, i in zip(*np.nonzero((is_max | is_min) & keep)):
        out.append((int(j) + 1, int(i) + 1, 1 if is_max[j, i] else -1, float(c[j, i])))
    return out


def bottom_vortex_count(psi, min_abs=0.0):
    """Number of vortex centres strictly below the primary vortex's centre
    (the first site of maximal Psi in row-major order)."""
    psi = np.asarray(psi, dtype=np.float64)
    jp, _ = np.unravel_index(int(np.argmax(psi)), psi.shape)
    return sum(1 for (j, _, _, _) in vortex_centres(psi, min_abs) if j < jp)
