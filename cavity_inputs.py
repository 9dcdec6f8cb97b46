"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module draws random numbers and lists workload shapes.  It holds none of
the method's arithmetic (no equilibrium, no moments, no weights): callers turn
what it returns into lattice states with their own code.

The cavity workloads follow arXiv 2211.05009: lattices of Nx = 500 sites
across and Ny = 500 * Ar up (Sec. 3.2 opening paragraph), Re = 4000-8000 and
Ar = 0.4-2.0 (Sec. 1 last paragraph), a 256 x 256 validation lattice
(Sec. 3.1), lid speed 0.1 (Sec. 3 opening paragraph).
"""
from __future__ import annotations

import numpy as np

U_LID = 0.1

# Small lattice used for the multi-step comparison runs.
SMALL = dict(nx=64, ny=64, re=100.0)

# The paper's production lattices: 500 x (500 Ar) at the aspect ratios and
# Reynolds numbers of the single-cavity study.
PAPER_AR = (0.4, 1.0, 2.0)
PAPER_RE = (1000.0, 4000.0, 8000.0)

# The Re x Ar sweep advanced as one batch (25 uneven cavities).
SWEEP_AR = (0.4, 0.8, 1.2, 1.6, 2.0)
SWEEP_RE = (4000.0, 5000.0, 6000.0, 7000.0, 8000.0)


def ny_for(nx: int, ar: float) -> int:
    """Number of sites up the cavity for width ``nx`` and aspect ratio ``ar``
    (round half to even when nx * ar is not an integer)."""
    return int(np.round(nx * ar))


def paper_cases(nx: int = 500):
    """(nx, ny, re) for every Ar x Re pair of the single-cavity study."""
    return [(nx, ny_for(nx, ar), re) for ar in PAPER_AR for re in PAPER_RE]


def sweep_cases(nx: int = 500):
    """(nx, ny, re) of the 25-cavity sweep, Ar-major order."""
    return [(nx, ny_for(nx, ar), re) for ar in SWEEP_AR for re in SWEEP_RE]


def random_shift(nx: int, ny: int, seed: int, amp: float = 4e-3):
    """Random perturbation g[9, ny, nx] (float64), uniform in [-amp, amp].

    Added to the lattice weights it gives a positive, low-Mach population
    field that exercises every branch of a step from its first application."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(9, ny, nx))


def random_fields(nx: int, ny: int, seed: int, drho: float = 2e-3,
                  du: float = 0.05):
    """Random (rho - 1, u_x, u_y) fields, each [ny, nx] float64."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(-drho, drho, size=(ny, nx)),
            rng.uniform(-du, du, size=(ny, nx)),
            rng.uniform(-du, du, size=(ny, nx)))


def random_points(n: int, ar: float, seed: int):
    """n observing points (x, y) in units of the width L, inside [0,1]x[0,Ar]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.0, 1.0, n), rng.uniform(0.0, ar, n)], axis=1)


def normal_draws(n: int, seed: int):
    """n standard normal draws (float32), e.g. for network weight init."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n).astype(np.float32)
