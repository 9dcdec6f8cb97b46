"""Vectorised FP64 D3Q19 lattice-BGK lid-driven cube (oracle; test
infrastructure only).

The three-dimensional extension that Sec. 4 names as future work, built from
the same equations as the two-dimensional oracle (Sec. 2.1): the BGK update
of Eq. 1, the second-order equilibrium of Eq. 2 with c_s^2 = 1/3 (now with
the D3Q19 velocity set and weights 1/3, 1/18, 1/36), the moments of Eq. 3,
tau = 3 nu + 1/2 (Eq. 5) and Re = U L / nu with L = Nx (Sec. 1).

Walls: half-way bounce-back on all six faces, the lid being the face above
the top row y = Ny - 1, moving with (U, 0, 0); a reflected link picks up
-6 w rho_w (c . u_w), rho_w = 1, and every link that crosses the lid plane
belongs to the lid (as in two dimensions).  Test-only switches make x and / or
z periodic.

Site (x, y, z), arrays f[i, z, y, x].  Velocity order:
  0: (0,0,0)
  1: (1,0,0)  2: (-1,0,0)  3: (0,1,0)  4: (0,-1,0)  5: (0,0,1)  6: (0,0,-1)
  7: (1,1,0)  8: (-1,-1,0) 9: (1,-1,0) 10: (-1,1,0)
  11: (1,0,1) 12: (-1,0,-1) 13: (1,0,-1) 14: (-1,0,1)
  15: (0,1,1) 16: (0,-1,-1) 17: (0,1,-1) 18: (0,-1,1)
(each odd index followed by its opposite).  ``Cube.f`` holds f(t) before the
collision; ``post_collision()`` is the right-hand side of Eq. 1.
"""
from __future__ import annotations

import numpy as np

C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
# The weights as whole 36ths, w_i = K36[i] / 36: Eq. 2 multiplies by K36[i]
# and divides by 36 once, with 1/cs2 = 3, 1/(2 cs2^2) = 9/2, 1/(2 cs2) = 3/2
# exact, so no rounded weight biases every collision the same way (as in the
# two-dimensional oracle).
K36 = np.array([12] + [2] * 6 + [1] * 12, dtype=np.int64)
OPP = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17],
               dtype=np.int64)
CS2 = 1.0 / 3.0


def relaxation_time(nx, re, u_lid):
    """Eq. 5 with nu = U Nx / Re."""
    return u_lid * nx / re / CS2 + 0.5


def equilibrium(rho, ux, uy, uz):
    """Eq. 2 on the D3Q19 set, cs2 = 1/3 substituted:
    w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u], w_i = K36[i] / 36."""
    rho, ux, uy, uz = (np.asarray(a, dtype=np.float64) for a in (rho, ux, uy, uz))
    uu = ux * ux + uy * uy + uz * uz
    feq = np.empty((19,) + rho.shape)
    for i in range(19):
        cu = C[i, 0] * ux + C[i, 1] * uy + C[i, 2] * uz
        feq[i] = K36[i] * (rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)) / 36.0
    return feq


def macroscopic(f):
    """Eq. 3: rho and u = sum_i c_i f_i / rho."""
    rho = f.sum(axis=0)
    j = [np.tensordot(C[:, a].astype(np.float64), f, axes=(0, 0)) for a in range(3)]
    return rho, j[0] / rho, j[1] / rho, j[2] / rho


def collide(f, tau):
    rho, ux, uy, uz = macroscopic(f)
    return f - (f - equilibrium(rho, ux, uy, uz)) / tau


def stream(fs, u_lid, periodic_x=False, periodic_z=False):
    """Pull streaming with the wall reflections (see the module text)."""
    _, nz, ny, nx = fs.shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty_like(fs)
    for i in range(19):
        cx, cy, cz = (int(v) for v in C[i])
        xs, ys, zs = xx - cx, yy - cy, zz - cz
        if periodic_x:
            xs = np.mod(xs, nx)
        if periodic_z:
            zs = np.mod(zs, nz)
        inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny) & (zs >= 0) & (zs < nz)
        out[i][inside] = fs[i][zs[inside], ys[inside], xs[inside]]
        wall = ~inside
        if not np.any(wall):
            continue
        j = OPP[i]
        uwx = np.where(wall & (ys >= ny), u_lid, 0.0)       # lid links first
        out[i][wall] = fs[j][wall] - (K36[j] * (C[j, 0] * uwx[wall])) / 6.0  # 6 w_j = K36[j]/6
    return out


class Cube:
    """Lid-driven box of nx x ny x nz sites at rest (rho = 1, u = 0)."""

    def __init__(self, nx, ny, nz, re=None, u_lid=0.1, tau=None, periodic_x=False,
                 periodic_z=False):
        if tau is None:
            tau = relaxation_time(nx, re, u_lid)
        if not tau > 0.5:
            raise ValueError("tau must exceed 1/2")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.tau, self.u_lid = float(tau), float(u_lid)
        self.periodic_x, self.periodic_z = bool(periodic_x), bool(periodic_z)
        shape = (nz, ny, nx)
        self.f = equilibrium(np.ones(shape), np.zeros(shape), np.zeros(shape), np.zeros(shape))
        self.t = 0

    def set_state(self, f, t=0):
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == (19, self.nz, self.ny, self.nx)
        self.f = f.copy()
        self.t = int(t)

    def post_collision(self):
        return collide(self.f, self.tau)

    def moments(self):
        return macroscopic(self.f)

    def step(self, n=1):
        for _ in range(int(n)):
            self.f = stream(self.post_collision(), self.u_lid, self.periodic_x, self.periodic_z)
            self.t += 1
        return self
