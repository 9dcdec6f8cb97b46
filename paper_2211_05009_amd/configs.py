"""Command-line runs of the five reference workloads of this library.

    python -m paper_2211_05009_amd.configs 1      # 64 x 64, Re 100, 20,000 steps
    python -m paper_2211_05009_amd.configs 2      # 500 x (500 Ar) single cavities
    python -m paper_2211_05009_amd.configs 3      # 25-cavity Re x Ar sweep, one batch
    python -m paper_2211_05009_amd.configs 4      # learned warm start, steps to 1e-8
    python -m paper_2211_05009_amd.configs 5      # long unsteady run with probes; 4096^2

Each prints one JSON object.  Orchestration only: the work runs in the
library's kernels (include/lbm.h).
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import lbm


def _inputs():
    """The repository's seeded-input module (cavity_inputs.py beside the
    package), found from this file's location, so the runner works from any
    working directory."""
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "cavity_inputs.py")
    spec = importlib.util.spec_from_file_location("cavity_inputs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod

U = 0.1


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def config1(dtype="f64"):
    """64 x 64, Re 100 (tau = 0.692), 20,000 steps from rest: u_x along the
    vertical centre line and u_y along the horizontal one (central two
    columns / rows averaged), total mass at 0, 10,000 and 20,000 steps."""
    c = lbm.Cavity(64, 64, re=100.0, u_lid=U, dtype=dtype)
    mass = [c.mass()]
    for _ in range(2):
        c.step(10000)
        mass.append(c.mass())
    _, ux, uy = c.moments()
    u_line = 0.5 * (ux[:, 31] + ux[:, 32])
    v_line = 0.5 * (uy[31, :] + uy[32, :])
    res, at = c.residual()
    c.close()
    return {"config": 1, "lattice": "64 x 64", "re": 100.0, "tau": 0.692, "steps": 20000,
            "storage": dtype, "y": ((np.arange(64) + 0.5) / 64).tolist(),
            "u_x_centre_over_U": (u_line / U).tolist(), "u_y_centre_over_U": (v_line / U).tolist(),
            "mass": mass, "residual": res, "residual_step": at}


def config2(steps=200_000):
    """500 x (500 Ar), Ar 0.4 / 1.0 / 2.0, Re 1000 / 4000 / 8000, FP32 f - w
    and FP64, from rest: MLUPS of each."""
    rows = []
    for ar in (0.4, 1.0, 2.0):
        for re in (1000.0, 4000.0, 8000.0):
            for dt in ("f32s", "f64"):
                ny = int(round(500 * ar))
                c = lbm.Cavity(500, ny, re=re, u_lid=U, dtype=dt)
                c.autotune(chunks=4)
                _, sec = _timed(lambda: c.step(steps))
                rows.append({"nx": 500, "ny": ny, "re": re, "storage": dt, "steps": steps,
                             "MLUPS": round(500 * ny * steps / sec / 1e6, 1),
                             "residual": c.residual()[0], "mass": c.mass()})
                c.close()
    return {"config": 2, "cases": rows}


def config3(steps=500_000):
    """The 25-cavity sweep (Ar 0.4 ... 2.0 x Re 4000 ... 8000, 500 wide) as
    one batch, 1000-step graphs: aggregate MLUPS."""
    ars = (0.4, 0.8, 1.2, 1.6, 2.0)
    res = (4000.0, 5000.0, 6000.0, 7000.0, 8000.0)
    nx = [500] * 25
    ny = [int(round(500 * a)) for a in ars for _ in res]
    re = [r for _ in ars for r in res]
    b = lbm.Batch(nx, ny, re, u_lid=U, dtype="f32s")
    b.autotune(chunks=2)
    _, sec = _timed(lambda: b.step(steps))
    sites = sum(a * c for a, c in zip(nx, ny))
    out = {"config": 3, "cavities": 25, "sites": sites, "steps": steps,
           "MLUPS": round(sites * steps / sec / 1e6, 1), "residuals": b.residuals().tolist()}
    b.close()
    return out


def config4(threshold=1e-8):
    """Learned warm start: train on 200 solver fields, then steps to Eq. 6 <
    threshold for the steady sweep (FP64 storage), cold and warm-started."""
    from . import warmstart
    npar = lbm.Surrogate(1).num_params
    return {"config": 4, **warmstart.steady_sweep_study(
        _inputs().normal_draws(npar, seed=0), threshold=threshold, dtype="f64",
        modes=("batch-cold", "batch-warm", "batch-warm-fallback"))}


def config5():
    """Ar 1.5, Re 8000, 500 x 750, FP32, 2 M steps with 5 probes every 100
    steps (classified); 4096 x 4096, Re 1e4, 10,000 steps, FP32 and FP64."""
    from . import flowmap
    out = {"config": 5, "long": flowmap.long_unsteady()}
    big = []
    for dt in ("f32s", "f64"):
        c = lbm.Cavity(4096, 4096, re=1e4, u_lid=U, dtype=dt)
        c.autotune(chunks=2)
        _, sec = _timed(lambda: c.step(10000))
        big.append({"storage": dt, "MLUPS": round(4096 * 4096 * 10000 / sec / 1e6, 1),
                    "mass": c.mass()})
        c.close()
    out["large"] = big
    return out


RUNS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 1 or not argv[0].isdigit() or int(argv[0]) not in RUNS:
        print(__doc__, file=sys.stderr)
        return 2
    print(json.dumps(RUNS[int(argv[0])]()), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
