"""Writes the stored expected values of the 64 x 64, Re = 100 cavity run.

Calls only the CPU oracle.  Run from the repository root:

    python tests/golden/make_golden.py

Workload: lid-driven square cavity, 64 x 64 sites, Re = 100, lid speed 0.1,
tau = 3 * 0.1 * 64 / 100 + 1/2 = 0.692, half-way bounce-back walls, started
from rest, 20,000 applications of Eq. 1 (arXiv 2211.05009, Sec. 2).
Stored: centre-line profiles (u_x on x = L/2, u_y on y = H/2), total mass
every 1,000 steps, and the Eq. 6 residual at the last 100-step pair.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import monitors            # noqa: E402
from oracle.d2q9 import Cavity, mass   # noqa: E402


def main():
    c = Cavity(64, 64, re=100.0, u_lid=0.1)
    masses = [mass(c.f)]
    prev = None
    for k in range(20):
        c.step(1000 - (100 if k == 19 else 0))
        if k == 19:
            _, ux0, uy0 = c.moments()
            c.step(100)
            _, ux1, uy1 = c.moments()
            prev = monitors.residual(ux1, uy1, ux0, uy0)
        masses.append(mass(c.f))
    rho, ux, uy = c.moments()
    u_vert, v_horz = monitors.centreline(ux, uy)
    psi = monitors.stream_function(ux)
    ext = monitors.vortex_extrema(psi / (0.1 * 64), 64)
    out = dict(workload="cavity 64x64 Re=100 U=0.1 tau=0.692, 20000 steps from rest",
               steps=c.t, u_centre=u_vert.tolist(), v_centre=v_horz.tolist(),
               mass_every_1000=masses, residual_eq6=prev,
               psi_primary=ext["primary"])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "cavity64_re100_20000.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
