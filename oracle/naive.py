"""Brute-force twin of ``oracle.d2q9`` (test infrastructure only).

Pure-Python loops over sites and directions, written in *push* form from the
same definitions (arXiv 2211.05009, Sec. 2.1 Eqs. 1-3 and 5): every site
collides its own populations, then sends each one along its link; a population
whose link would end outside the cavity is reflected by the wall it meets
(half-way bounce-back, moving-wall term -6 w_i rho_w c_i.u_w with rho_w = 1;
the lid owns links through the top corners).  It shares no code with the
vectorised oracle on purpose: the two are compared on tiny lattices.

Only for lattices of a few dozen sites.
"""
from __future__ import annotations

# Written out independently of oracle.d2q9 (no import from it).
_VEL = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
        (1, 1), (-1, 1), (-1, -1), (1, -1))
_WGT_NUM = (4, 1, 1, 1, 1, 1, 1, 1, 1)
_WGT_DEN = (9, 9, 9, 9, 9, 36, 36, 36, 36)


def _reverse(i):
    cx, cy = _VEL[i]
    return _VEL.index((-cx, -cy))


def _feq_site(rho, ux, uy, one):
    """Eq. 2 at one site; each weight a / b enters as a times the bracket,
    divided by b (exact in rationals; in FP64 no rounded weight)."""
    out = []
    three = 3 * one
    for (cx, cy), a, b in zip(_VEL, _WGT_NUM, _WGT_DEN):
        cu = cx * ux + cy * uy
        out.append(a * (rho * (one + three * cu + (9 * one / 2) * cu * cu
                               - (three / 2) * (ux * ux + uy * uy))) / b)
    return out


def naive_steps(f, tau, u_lid, nsteps, num=float):
    """Advance ``f`` (nested lists or array, [9][ny][nx]) by ``nsteps``
    applications of Eq. 1 in the closed cavity; returns nested lists.

    ``num`` is the number type every quantity is converted to: ``float`` for
    IEEE FP64, or ``fractions.Fraction`` for exact rational arithmetic (then
    ``f``, ``tau`` and ``u_lid`` should be given as exact values)."""
    ny = len(f[0])
    nx = len(f[0][0])
    one = num(1)
    tau = num(tau)
    u_lid = num(u_lid)
    cur = [[[num(f[i][y][x]) for x in range(nx)] for y in range(ny)]
           for i in range(9)]
    for _ in range(nsteps):
        nxt = [[[None] * nx for _ in range(ny)] for _ in range(9)]
        for y in range(ny):
            for x in range(nx):
                # collision at (x, y)
                pops = [cur[i][y][x] for i in range(9)]
                rho = num(0)
                jx = num(0)
                jy = num(0)
                for i in range(9):
                    rho += pops[i]
                    jx += _VEL[i][0] * pops[i]
                    jy += _VEL[i][1] * pops[i]
                ux = jx / rho
                uy = jy / rho
                eq = _feq_site(rho, ux, uy, one)
                post = [pops[i] - (pops[i] - eq[i]) / tau for i in range(9)]
                # push every population along its link
                for i in range(9):
                    cx, cy = _VEL[i]
                    tx, ty = x + cx, y + cy
                    if 0 <= tx < nx and 0 <= ty < ny:
                        nxt[i][ty][tx] = post[i]
                        continue
                    # reflected back into (x, y) as the reverse direction
                    if ty >= ny:
                        wall_u = u_lid        # lid first: corners belong to it
                    else:
                        wall_u = num(0)       # bottom and side walls at rest
                    r = _reverse(i)
                    # 6 w_i = 6 a / b
                    nxt[r][y][x] = post[i] - 6 * _WGT_NUM[i] * one * (cx * wall_u) / _WGT_DEN[i]
        cur = nxt
    return cur


def naive_steps_nee(f, tau, u_lid, nsteps, num=float):
    """Push-form twin of ``oracle.nee``: walls on the outermost nodes, rebuilt
    after every step from the nearest fluid node by non-equilibrium
    extrapolation (Sec. 2.2 (ii)); the top row, corners included, moves
    with (u_lid, 0).  ``f`` is [9][ny][nx] with ny, nx >= 3."""
    ny = len(f[0])
    nx = len(f[0][0])
    one = num(1)
    tau = num(tau)
    u_lid = num(u_lid)
    cur = [[[num(f[i][y][x]) for x in range(nx)] for y in range(ny)]
           for i in range(9)]

    def moments(pops):
        rho = sum(pops, num(0))
        jx = sum((_VEL[i][0] * pops[i] for i in range(9)), num(0))
        jy = sum((_VEL[i][1] * pops[i] for i in range(9)), num(0))
        return rho, jx / rho, jy / rho

    def fluid(x, y):
        return 0 < x < nx - 1 and 0 < y < ny - 1

    for _ in range(nsteps):
        nxt = [[[None] * nx for _ in range(ny)] for _ in range(9)]
        for y in range(ny):
            for x in range(nx):
                pops = [cur[i][y][x] for i in range(9)]
                rho, ux, uy = moments(pops)
                eq = _feq_site(rho, ux, uy, one)
                for i in range(9):
                    tx, ty = x + _VEL[i][0], y + _VEL[i][1]
                    if fluid(tx, ty):
                        nxt[i][ty][tx] = pops[i] - (pops[i] - eq[i]) / tau
        for y in range(ny):
            for x in range(nx):
                if fluid(x, y):
                    continue
                xr = min(max(x, 1), nx - 2)
                yr = min(max(y, 1), ny - 2)
                ref = [nxt[i][yr][xr] for i in range(9)]
                rho, ux, uy = moments(ref)
                eq_ref = _feq_site(rho, ux, uy, one)
                eq_wall = _feq_site(rho, u_lid if y == ny - 1 else num(0), num(0), one)
                for i in range(9):
                    nxt[i][y][x] = eq_wall[i] + ref[i] - eq_ref[i]
        cur = nxt
    return cur


# D3Q19 set and weights, written out again (no import from oracle.d3q19).
_VEL3 = [(0, 0, 0)] + [v for a in range(3) for v in
                       (tuple(1 if k == a else 0 for k in range(3)),
                        tuple(-1 if k == a else 0 for k in range(3)))]
_VEL3 += [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
          (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def naive_steps_3d(f, tau, u_lid, nsteps, num=float):
    """Push-form twin of ``oracle.d3q19`` for a closed box (all six faces
    half-way bounce-back, lid above y = ny - 1 moving with (u_lid, 0, 0) and
    owning every link through its plane).  ``f`` is [19][nz][ny][nx]."""
    nz, ny, nx = len(f[0]), len(f[0][0]), len(f[0][0][0])
    one = num(1)
    den = [3] + [18] * 6 + [36] * 12          # weights 1/3, 1/18, 1/36
    tau, u_lid = num(tau), num(u_lid)
    cur = [[[[num(f[i][z][y][x]) for x in range(nx)] for y in range(ny)] for z in range(nz)]
           for i in range(19)]
    for _ in range(nsteps):
        nxt = [[[[None] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(19)]
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    pops = [cur[i][z][y][x] for i in range(19)]
                    rho = sum(pops, num(0))
                    u = [sum((_VEL3[i][a] * pops[i] for i in range(19)), num(0)) / rho
                         for a in range(3)]
                    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
                    for i in range(19):
                        c = _VEL3[i]
                        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
                        eq = (rho * (one + 3 * cu + (9 * one / 2) * cu * cu
                                     - (3 * one / 2) * uu)) / den[i]
                        post = pops[i] - (pops[i] - eq) / tau
                        tx, ty, tz = x + c[0], y + c[1], z + c[2]
                        if 0 <= tx < nx and 0 <= ty < ny and 0 <= tz < nz:
                            nxt[i][tz][ty][tx] = post
                        else:
                            wall_u = u_lid if ty >= ny else num(0)
                            r = _VEL3.index((-c[0], -c[1], -c[2]))
                            nxt[r][z][y][x] = post - 6 * one * (c[0] * wall_u) / den[i]
        cur = nxt
    return cur
