"""The oracle's pins have teeth: plant plausible mistakes in a copy of the
oracle source (on the CPU) and check that the pin battery rejects every one,
while the unmodified source passes it."""
import math
import os
import types

import numpy as np
import pytest

from cavity_inputs import random_shift
from oracle.naive import naive_steps

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "d2q9.py")

MUTATIONS = {
    "second-order equilibrium term dropped":
        ("4.5 * cu * cu", "0.0 * cu"),
    "velocity term sign flipped":
        ("1.0 + 3.0 * cu", "1.0 - 3.0 * cu"),
    "lid momentum term sign flipped":
        ("fs[j][wall] - (K36[j]", "fs[j][wall] + (K36[j]"),
    "reflection keeps the direction":
        ("out[i][wall] = fs[j][wall]", "out[i][wall] = fs[i][wall]"),
    "streaming pulls from the wrong side":
        ("xs = xx - C[i, 0]", "xs = xx + C[i, 0]"),
    "side walls own the top corners":
        ("uwx[wall & (ys >= ny)] = u_lid", "uwx[wall & (ys >= ny) & (xs >= 0) & (xs < nx)] = u_lid"),
    "viscosity relation off by a factor":
        ("return viscosity(nx, re, u_lid) / CS2 + 0.5", "return viscosity(nx, re, u_lid) / 2 + 0.5"),
    "relaxation applied as multiply by tau":
        ("fs = f - (f - feq) / tau", "fs = f - (f - feq) * (2.0 - 1.0 / tau)"),
    "transposed moment axes":
        ("jx = np.tensordot(C[:, 0]", "jx = np.tensordot(C[:, 1]"),
    "weights rounded to FP64 constants":
        ("K36[i] * (rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)) / 36.0",
         "W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)"),
}


def _load(src):
    mod = types.ModuleType("mutated_d2q9")
    exec(compile(src, "mutated_d2q9", "exec"), mod.__dict__)
    return mod


def _battery(m):
    """Fast versions of the pins; returns the list of failed pin names."""
    failed = []
    W, C = m.W, m.C
    # Eq. 2 moment identities
    rng = np.random.default_rng(1)
    rho, ux, uy = rng.uniform(0.9, 1.1, 50), rng.uniform(-.1, .1, 50), rng.uniform(-.1, .1, 50)
    feq = m.equilibrium(rho, ux, uy)
    cx = C[:, 0].astype(float)
    if not (np.allclose(feq.sum(0), rho, rtol=1e-14, atol=0)
            and np.allclose(cx @ feq, rho * ux, atol=1e-15, rtol=0)
            and np.allclose((cx * cx) @ feq, rho / 3 + rho * ux * ux, rtol=1e-14, atol=0)):
        failed.append("equilibrium")
    # no same-signed rounding of the mass in a collision (weights exact)
    f = W[:, None, None] + random_shift(300, 200, seed=5)
    if abs(np.mean(m.collide(f, 0.51875).sum(0) - f.sum(0))) > 1e-17:
        failed.append("mass bias")
    # Eq. 5 value
    if not math.isclose(m.relaxation_time(500, 8000, 0.1), 0.51875, rel_tol=1e-14):
        failed.append("tau")
    # first step from rest
    c = m.Cavity(6, 5, tau=0.7, u_lid=0.1)
    c.step(1)
    exp = np.broadcast_to(W[:, None, None], c.f.shape).copy()
    exp[7, -1, :] -= 0.1 / 6
    exp[8, -1, :] += 0.1 / 6
    if np.max(np.abs(c.f - exp)) > 5e-16:
        failed.append("first step")
    # brute-force twin
    f0 = W[:, None, None] + random_shift(4, 6, seed=46)
    c = m.Cavity(4, 6, tau=0.6, u_lid=0.1)
    c.set_state(f0)
    c.step(30)
    if np.max(np.abs(c.f - np.array(naive_steps(f0, 0.6, 0.1, 30)))) > 1e-14:
        failed.append("naive twin")
    # Couette
    H, tau = 8, 1.5
    c = m.Cavity(4, H, tau=tau, u_lid=0.1, periodic_x=True)
    c.step(int(40 * H * H / (math.pi ** 2 * (tau - 0.5) / 3)))
    if np.max(np.abs(c.moments()[1] - (0.1 * (np.arange(H) + 0.5) / H)[:, None])) > 1e-12:
        failed.append("couette")
    return failed


def test_unmodified_oracle_passes_battery():
    assert _battery(_load(open(SRC).read())) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, f"mutation target missing: {old!r}"
    assert _battery(_load(src.replace(old, new))) != []
