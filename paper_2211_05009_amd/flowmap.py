"""Flow-state map of the Re x Ar plane (Sec. 3.3 and Fig. 17; periods as in
Table 3), run as one batch with probe series classified on the device.

Orchestration only: the lattice updates, the probe records and the
classification run in the library's kernels (include/lbm.h); this module
picks the cavities and the observing points and formats the results.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm

U_LID = 0.1

# The sweep of Fig. 17: Re 4000 ... 8000 in steps of 500, Ar 0.4 ... 2.0 in
# steps of 0.1.
FIG17_RE = tuple(4000.0 + 500.0 * i for i in range(9))
FIG17_AR = tuple(round(0.4 + 0.1 * i, 1) for i in range(17))


def observing_point(ar):
    """The observing point of Sec. 3.3 in units of L: (0.5, 0.2) for
    Ar = 0.4, (0.5, 0.3) for Ar = 0.5 and 0.6, (0.5, 0.5) otherwise."""
    if ar < 0.45:
        return (0.5, 0.2)
    if ar < 0.65:
        return (0.5, 0.3)
    return (0.5, 0.5)


def state_map(cases, nx=500, steps=3_000_000, window=10_000, dtype="f32s",
              steady_tol=1e-4 * U_LID, periodic_tol=0.05, chunk=100_000, log=None):
    """Run every (Re, Ar) of `cases` from rest on nx x round(nx Ar) lattices
    for `steps` steps in one batch, recording u at the observing point every
    100 steps, and classify u_x over the last `window` records.

    Returns a list of dicts: re, ar, nx, ny, state, period_steps (period x
    100), cycle_steps and cycle_mismatch, amplitude and mean of u_x over the
    window (units of U), mismatch;
    plus the run's wall time and aggregate MLUPS as a second value.  The
    dominant cycle (cycle_steps) is the first return of the lag mismatch,
    also for modulated or aperiodic flows."""
    nxs = [nx] * len(cases)
    nys = [int(round(nx * ar)) for _, ar in cases]
    res = [re for re, _ in cases]
    b = lbm.Batch(nxs, nys, res, u_lid=U_LID, dtype=dtype)
    pts = np.array([[observing_point(ar)] for _, ar in cases])
    b.probe_config(pts, capacity=window)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        b.step(k)
        done += k
        if log:
            log(f"state map: {done} of {steps} steps, {time.perf_counter() - t0:.0f} s")
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    states = b.probe_classify(1, window, steady_tol, periodic_tol)
    out = []
    for (re, ar), ny, st in zip(cases, nys, states):
        s = st[0]
        out.append({"re": re, "ar": ar, "nx": nx, "ny": ny, "state": s["state"],
                    "period_steps": round(100.0 * s["period"], 1),
                    "cycle_steps": round(100.0 * s["cycle"], 1),
                    "cycle_mismatch": s["cycle_mismatch"],
                    "amplitude_U": s["amplitude"] / U_LID, "mean_U": s["mean"] / U_LID,
                    "mismatch": s["mismatch"]})
    sites = sum(a * c for a, c in zip(nxs, nys))
    b.close()
    return out, {"seconds": round(seconds, 2), "steps": steps,
                 "MLUPS": round(sites * steps / seconds / 1e6, 1)}


# Probes of the long unsteady run, in units of L: the paper's three
# observing points (0.5, 0.5), (0.5, 0.3), (0.5, 0.2) (Sec. 3.3) and two
# points near the bottom corner eddies.
LONG_PROBES = ((0.5, 0.5), (0.5, 0.3), (0.5, 0.2), (0.1, 0.1), (0.9, 0.1))


def long_unsteady(nx=500, ar=1.5, re=8000.0, steps=2_000_000, dtype="f32s", window=10_000,
                  points=LONG_PROBES, steady_tol=1e-4 * U_LID, periodic_tol=0.05, log=None):
    """One long unsteady cavity with probes every 100 steps (FP64-interpolated
    moments), timed with the probes inside the run, then classified."""
    import torch
    ny = int(round(nx * ar))
    c = lbm.Cavity(nx, ny, re=re, u_lid=U_LID, dtype=dtype)
    c.autotune(chunks=5)
    c.probe_config(np.array(points), every=100, capacity=window)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(200_000, steps - done)
        c.step(k)
        done += k
        if log:
            log(f"long run: {done} of {steps} steps")
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    states = c.probe_classify(1, min(window, steps // 100), steady_tol, periodic_tol)
    c.close()
    return {"workload": f"{nx} x {ny}, Ar {ar}, Re {re:g}, {dtype}, {steps} steps, "
                        f"{len(points)} probes every 100 steps",
            "seconds": round(seconds, 2), "MLUPS": round(nx * ny * steps / seconds / 1e6, 1),
            "probes": [{"xy": list(p), "state": s["state"],
                        "period_steps": round(100.0 * s["period"], 1),
                        "amplitude_U": s["amplitude"] / U_LID} for p, s in zip(points, states)]}
