"""Vectorised FP64 D2Q9 lattice-BGK solver (oracle; test infrastructure only).

Every function below follows the method of arXiv 2211.05009, Sec. 2.1:

* Eq. 1  -- the BGK evolution: collide with relaxation time tau, then move each
            population one lattice link along its velocity.
* Eq. 2  -- the second-order equilibrium with c_s^2 = 1/3 (lattice units,
            c = dx/dt = 1, Sec. 3 opening paragraph).
* Eq. 3  -- density and momentum as the zeroth and first moments.
* Eq. 5  -- nu = c_s^2 (tau - 1/2), hence tau = 3 nu + 1/2.
* Sec. 1 -- Re = U L / nu with L the cavity *width*; so nu = U Nx / Re.

Wall treatment (half-way bounce-back with the moving-wall momentum term).  The
paper itself uses non-equilibrium extrapolation (Sec. 2.2 (ii), implemented
separately in ``oracle.nee``); the bounce-back variant here is the one the GPU
library implements.  Walls sit half a link outside the outermost sites.  A
population that would leave the lattice through a wall is reflected back into
the site it left, reversed, and picks up -6 w rho_w (c . u_w) for the wall's
velocity u_w (rho_w = 1).  A link that crosses the lid row counts as a lid link
even when it also crosses a side wall (the two top corners).

Site (x, y): x in [0, Nx) along the lid, y in [0, Ny), y = 0 at the bottom and
y = Ny - 1 just below the lid.  Arrays are indexed ``f[i, y, x]``.

Velocity order: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
7:(-1,-1) 8:(1,-1).  Weights 4/9, 1/9 (axis), 1/36 (diagonal) per Sec. 2.1.

Time-level convention: ``Cavity.f`` holds f(x, t), the distribution *before*
the collision of Eq. 1 at time t.  ``post_collision()`` gives the right-hand
side of Eq. 1 at time t.  ``step(n)`` applies Eq. 1 n times.
"""
from __future__ import annotations

import math

import numpy as np

# D2Q9 velocity set and weights (Sec. 2.1, below Eq. 2).
C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
              [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
W = np.array([4.0 / 9.0,
              1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0])
# The same weights as whole 36ths, w_i = K36[i] / 36.  Eq. 2 is evaluated
# with these (an exact integer multiple, then one correctly rounded division)
# and with c_s^2 = 1/3 substituted (1/cs2 = 3, 1/(2 cs2^2) = 9/2, 1/(2 cs2) =
# 3/2, all exact).  Multiplying by W itself would round every collision's
# equilibrium the same way (the FP64 values of 4/9, 1/9 and 1/36 all lie
# 5.6e-17 below the exact weights, relative), and over the 1e5-step
# relaxation of a steady cavity that same-signed error adds up to ~1.5e-12 U.
K36 = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1], dtype=np.int64)
# OPP[i] is the index of -c_i.
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6], dtype=np.int64)
CS2 = 1.0 / 3.0   # c_s^2 = c^2 / 3 with c = 1


def viscosity(nx: int, re: float, u_lid: float) -> float:
    """nu = U L / Re with L = Nx lattice spacings (Sec. 1 definition of Re)."""
    return u_lid * nx / re


def relaxation_time(nx: int, re: float, u_lid: float) -> float:
    """tau from Eq. 5: nu = c_s^2 (tau - 1/2) dt, dt = 1."""
    return viscosity(nx, re, u_lid) / CS2 + 0.5


def equilibrium(rho, ux, uy):
    """Eq. 2: f_i^eq = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)],
    with cs2 = 1/3: w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u], w_i = K36[i]/36."""
    rho = np.asarray(rho, dtype=np.float64)
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    uu = ux * ux + uy * uy
    feq = np.empty((9,) + rho.shape)
    for i in range(9):
        cu = C[i, 0] * ux + C[i, 1] * uy
        feq[i] = K36[i] * (rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)) / 36.0
    return feq


def density(f):
    """Eq. 3, zeroth moment."""
    return np.sum(f, axis=0)


def momentum(f):
    """Eq. 3, first moment: (sum_i c_ix f_i, sum_i c_iy f_i)."""
    jx = np.tensordot(C[:, 0].astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(C[:, 1].astype(np.float64), f, axes=(0, 0))
    return jx, jy


def macroscopic(f, force=(0.0, 0.0)):
    """rho and u of Eq. 3.  With a body force F (test-only), the velocity is
    (sum_i c_i f_i + F/2) / rho, the second-order-accurate definition that goes
    with Guo's forcing term."""
    rho = density(f)
    jx, jy = momentum(f)
    ux = (jx + 0.5 * force[0]) / rho
    uy = (jy + 0.5 * force[1]) / rho
    return rho, ux, uy


def collide(f, tau, force=(0.0, 0.0)):
    """Right-hand side of Eq. 1: f - (f - f^eq)/tau.

    With a body force F (test-only switch, not part of the paper's cavity) the
    Guo source (1 - 1/(2 tau)) w_i [(c_i - u)/cs2 + (c_i.u) c_i / cs2^2] . F is
    added."""
    rho, ux, uy = macroscopic(f, force)
    feq = equilibrium(rho, ux, uy)
    fs = f - (f - feq) / tau
    if force[0] != 0.0 or force[1] != 0.0:
        fx, fy = force
        for i in range(9):
            cx, cy = float(C[i, 0]), float(C[i, 1])
            cu = cx * ux + cy * uy
            src = ((cx - ux) / CS2 + cu * cx / (CS2 * CS2)) * fx \
                + ((cy - uy) / CS2 + cu * cy / (CS2 * CS2)) * fy
            fs[i] = fs[i] + (1.0 - 0.5 / tau) * W[i] * src
    return fs


def _links(nx, ny, periodic_x, periodic_y):
    """For each direction i: where each destination's population comes from.

    Returns a list of (inside, ys_in, xs_in, wall, ys, xs) with ``inside``
    the destinations whose source (x - c_ix, y - c_iy) is a lattice site
    (after periodic wrapping), ``ys_in, xs_in`` those sources, ``wall`` the
    destinations whose link crosses a wall, and ``ys, xs`` the source row and
    column of every link (row >= ny: the lid, < 0: the bottom)."""
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    links = []
    for i in range(9):
        xs = xx - C[i, 0]
        ys = yy - C[i, 1]
        if periodic_x:
            xs = np.mod(xs, nx)
        if periodic_y:
            ys = np.mod(ys, ny)
        inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny)
        links.append((inside, ys[inside], xs[inside], ~inside, ys, xs))
    return links


def stream(fs, u_lid=0.0, periodic_x=False, periodic_y=False, u_bottom=0.0,
           links=None):
    """Streaming half of Eq. 1 plus the wall treatment.

    Destination (x, y) receives population i from (x - c_ix, y - c_iy).  If
    that source lies outside the lattice (and the axis is not periodic), the
    population instead comes from the reflection at the wall crossed by the
    link: f_i(x) = fs_opp(i)(x) - 6 w_opp rho_w (c_opp . u_w), rho_w = 1.
    The lid is at y = Ny (velocity (u_lid, 0)); the bottom at y = -1
    (velocity (u_bottom, 0), zero for the cavity); side walls at x = -1 and
    x = Nx are at rest.  The lid is tested first, so the top corner links
    belong to the lid."""
    _, ny, nx = fs.shape
    if links is None:
        links = _links(nx, ny, periodic_x, periodic_y)
    out = np.empty_like(fs)
    for i in range(9):
        inside, ys_in, xs_in, wall, ys, xs = links[i]
        out[i][inside] = fs[i][ys_in, xs_in]
        if not np.any(wall):
            continue
        j = OPP[i]
        # wall velocity for each crossed link: lid, else bottom, else side (0)
        uwx = np.zeros((ny, nx))
        uwx[wall & (ys >= ny)] = u_lid
        uwx[wall & (ys < 0)] = u_bottom
        # c_opp . u_w, with u_w = (uwx, 0)
        cu = C[j, 0] * uwx
        out[i][wall] = fs[j][wall] - (K36[j] * 1.0 * cu[wall]) / 6.0   # 6 w_j = K36[j] / 6
    return out


class Cavity:
    """Lid-driven cavity (default) or a test channel.

    Parameters
    ----------
    nx, ny : number of fluid sites across (along the lid) and up.
    re, u_lid : Reynolds number and lid speed; tau = 3 U Nx / Re + 1/2.
    tau : give the relaxation time directly instead of ``re``.
    periodic_x, periodic_y : test-only switches (Couette, Poiseuille,
        Taylor-Green); with periodic_y there are no top/bottom walls.
    force : test-only uniform body force density (Guo forcing).
    """

    def __init__(self, nx, ny, re=None, u_lid=0.1, tau=None,
                 periodic_x=False, periodic_y=False, force=(0.0, 0.0),
                 u_bottom=0.0):
        if tau is None:
            if re is None:
                raise ValueError("give re or tau")
            tau = relaxation_time(nx, re, u_lid)
        if not tau > 0.5:
            raise ValueError("tau must exceed 1/2 (positive viscosity)")
        self.nx, self.ny = int(nx), int(ny)
        self.tau = float(tau)
        self.u_lid = float(u_lid)
        self.u_bottom = float(u_bottom)
        self.periodic_x = bool(periodic_x)
        self.periodic_y = bool(periodic_y)
        self.force = (float(force[0]), float(force[1]))
        self.t = 0
        self._links = None
        # Initial state (Sec. 2.2 (i)): rho = 1, u = 0, f = f^eq.  With walls
        # half a link outside the lattice there are no wall sites, so every
        # site starts at rest; the lid acts through the wall treatment.
        self.f = equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)),
                             np.zeros((ny, nx)))

    # -- state access -----------------------------------------------------
    def set_state(self, f, t=0):
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self.f = f.copy()
        self.t = int(t)

    def post_collision(self):
        """RHS of Eq. 1 at the current time."""
        return collide(self.f, self.tau, self.force)

    def moments(self):
        """(rho, ux, uy), each [ny, nx] (Eq. 3)."""
        return macroscopic(self.f, self.force)

    # -- time stepping ----------------------------------------------------
    def stream(self, fs):
        if self._links is None:
            self._links = _links(self.nx, self.ny, self.periodic_x, self.periodic_y)
        return stream(fs, self.u_lid, self.periodic_x, self.periodic_y,
                      self.u_bottom, self._links)

    def step(self, n=1):
        """Apply Eq. 1 (collide, then stream with the wall treatment) n times."""
        for _ in range(int(n)):
            self.f = self.stream(self.post_collision())
            self.t += 1
        return self


def staggered_momenta(f):
    """P_x = sum (-1)^x j_x and P_y = sum (-1)^y j_y (j = sum_i c_i f_i).

    Collision keeps every site's j; streaming moves each population with
    c_x != 0 to a column of the other parity, and a wall reflection reverses
    c at the same site.  Hence one application of Eq. 1 maps P_y -> -P_y and
    P_x -> -P_x, plus u_lid/3 from the lid term when Nx is odd: two
    invariants of period two besides the mass."""
    _, ny, nx = f.shape
    jx, jy = momentum(f)
    sx = (-1.0) ** np.arange(nx)[None, :]
    sy = (-1.0) ** np.arange(ny)[:, None]
    return float((sx * jx).sum()), float((sy * jy).sum())


def destaggered_velocity(rho, ux, uy):
    """Velocity with the staggered momenta of rho u removed by a uniform
    (-1)^x (resp. (-1)^y) momentum: sum (-1)^x rho u_x = sum (-1)^y rho u_y
    = 0 afterwards."""
    ny, nx = rho.shape
    n = nx * ny
    sx = (-1.0) ** np.arange(nx)[None, :]
    sy = (-1.0) ** np.arange(ny)[:, None]
    px = (sx * rho * ux).sum() / n
    py = (sy * rho * uy).sum() / n
    return ux - px * sx / rho, uy - py * sy / rho


def mass(f):
    """Total mass sum_x rho(x), summed exactly (math.fsum) so that the oracle's
    own rounding does not mask a conservation error."""
    return math.fsum(np.asarray(f, dtype=np.float64).ravel().tolist())
