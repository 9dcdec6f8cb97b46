"""Cavity with non-equilibrium extrapolation walls (oracle; test
infrastructure only).

This is the wall scheme the paper itself uses (Sec. 2.2 (ii), after Guo, Zheng
and Shi): the walls lie on the outermost lattice nodes, and the distribution
at a wall node b is rebuilt every step from a fluid node f next to it,

    f_i(b) = f_i^eq(rho(f), u_w(b)) + [f_i(f) - f_i^eq(rho(f), u(f))],

i.e. the equilibrium of the wall velocity at the neighbour's density plus the
neighbour's non-equilibrium part.  The bulk update is Eq. 1 as in
``oracle.d2q9`` (same equilibrium, moments and collision functions).

Geometry (the readings this oracle fixes):

* Nodes (x, y), x in [0, Nx), y in [0, Ny); the wall nodes are the rows
  y = 0, y = Ny - 1 and the columns x = 0, x = Nx - 1; the rest are fluid.
  The walls are Nx - 1 spacings apart, so L = Nx - 1 and nu = U (Nx - 1)/Re;
  node x sits at x/(Nx - 1) in units of L.
* The lid is the top row, its two corner nodes included (the "nodes at the
  top wall" of Sec. 2.2 (i)): u_w = (U, 0) there, 0 on every other wall node.
* The reference node of wall node (x, y) is the nearest fluid node,
  (clamp(x, 1, Nx-2), clamp(y, 1, Ny-2)): the neighbour along the wall's
  normal, the diagonal neighbour for a corner.
* Initial state (Sec. 2.2 (i)): f = f^eq(1, u0) with u0 = (U, 0) on the top
  row and 0 elsewhere.
* One step: collide every node (Eq. 1 right-hand side), stream into the fluid
  nodes (every source is a node), then rebuild every wall node by the
  extrapolation above from the streamed fluid nodes.

Test-only switch: ``periodic_x`` removes the side walls (x wraps), leaving a
channel between the lid and the bottom wall (Couette flow).
"""
from __future__ import annotations

import numpy as np

from .d2q9 import C, CS2, collide, equilibrium, macroscopic


def relaxation_time(nx: int, re: float, u_lid: float) -> float:
    """tau from Eq. 5 with Re = U L / nu and L = Nx - 1 spacings."""
    return u_lid * (nx - 1) / re / CS2 + 0.5


def wall_nodes(nx, ny, periodic_x=False):
    """(ys, xs) of the wall nodes, (yr, xr) of their reference nodes, and the
    x velocity of each wall node."""
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    wall = (yy == 0) | (yy == ny - 1)
    if not periodic_x:
        wall |= (xx == 0) | (xx == nx - 1)
    ys, xs = yy[wall], xx[wall]
    yr = np.clip(ys, 1, ny - 2)
    xr = xs if periodic_x else np.clip(xs, 1, nx - 2)
    return ys, xs, yr, xr


def extrapolate_walls(f, u_lid, periodic_x=False):
    """Rebuild every wall node of f (pre-collision distributions) in place."""
    _, ny, nx = f.shape
    ys, xs, yr, xr = wall_nodes(nx, ny, periodic_x)
    rho, ux, uy = macroscopic(f)
    rf = rho[yr, xr]
    uw = np.where(ys == ny - 1, u_lid, 0.0)
    feq_w = equilibrium(rf, uw, np.zeros_like(uw))
    feq_f = equilibrium(rf, ux[yr, xr], uy[yr, xr])
    f[:, ys, xs] = feq_w + f[:, yr, xr] - feq_f
    return f


def stream_fluid(fs, periodic_x=False):
    """Pull streaming into the fluid nodes: f_i(x) = fs_i(x - c_i).  Wall
    nodes are left as they are (they are rebuilt afterwards)."""
    _, ny, nx = fs.shape
    out = fs.copy()
    x0, x1 = (0, nx) if periodic_x else (1, nx - 1)
    xs = np.arange(x0, x1)
    for i in range(9):
        cx, cy = int(C[i, 0]), int(C[i, 1])
        src_x = np.mod(xs - cx, nx) if periodic_x else xs - cx
        out[i, 1:ny - 1, x0:x1] = fs[i][1 - cy:ny - 1 - cy][:, src_x]
    return out


class CavityNEE:
    """Lid-driven cavity of Nx x Ny nodes with on-node walls (see above).

    ``f`` holds f(x, t) before the collision of step t, at every node (wall
    nodes already extrapolated); ``post_collision()`` is the right-hand side
    of Eq. 1, the state the GPU library stores."""

    def __init__(self, nx, ny, re=None, u_lid=0.1, tau=None, periodic_x=False):
        if nx < 3 or ny < 3:
            raise ValueError("on-node walls need at least 3 x 3 nodes")
        if tau is None:
            if re is None:
                raise ValueError("give re or tau")
            tau = relaxation_time(nx, re, u_lid)
        if not tau > 0.5:
            raise ValueError("tau must exceed 1/2 (positive viscosity)")
        self.nx, self.ny = int(nx), int(ny)
        self.tau = float(tau)
        self.u_lid = float(u_lid)
        self.periodic_x = bool(periodic_x)
        self.t = 0
        ux0 = np.zeros((ny, nx))
        ux0[ny - 1, :] = u_lid
        self.f = equilibrium(np.ones((ny, nx)), ux0, np.zeros((ny, nx)))

    def set_state(self, f, t=0):
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self.f = f.copy()
        self.t = int(t)

    def post_collision(self):
        return collide(self.f, self.tau)

    def moments(self):
        return macroscopic(self.f)

    def step(self, n=1):
        for _ in range(int(n)):
            f = stream_fluid(self.post_collision(), self.periodic_x)
            self.f = extrapolate_walls(f, self.u_lid, self.periodic_x)
            self.t += 1
        return self
