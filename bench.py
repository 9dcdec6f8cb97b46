"""Throughput of the fused D2Q9 BGK step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--ar 1.0] [--re 8000] [--dtype f32s]

Workload: lid-driven cavity of 500 x (500 Ar) sites (the production lattice
of arXiv 2211.05009, Sec. 3.2-3.3), lid speed 0.1, Re = 8000, populations
stored as f - w in FP32, started from rest.  A "step" is one application of
Eq. 1 to every site (one fused stream + bounce-back + collide launch) with the
FP64 mass / Eq. 6 monitors every 100 steps, exactly as lbm_step runs them.
The lattice is resident in device memory before timing starts.

Prints one JSON line: MLUPS (million lattice-site updates per second), the
HBM roofline of the step kernel (72 B per site update in FP32, 144 B in FP64:
nine populations read and nine written), per-case figures for the other
aspect ratios and FP64 storage, and the CPU oracle timed on a bounded sample.

``--copy-probe BYTES`` instead runs a plain device copy of BYTES bytes ten
times (used to calibrate the rocprofv3 FETCH_SIZE / WRITE_SIZE counters).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 MLUPS & % HBM roofline at 500×500·Ar; sweep time-to-steady vs plain"
HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E, published
BYTES_PER_SITE = {"f32s": 72, "f64": 144}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--nx", type=int, default=500)
    ap.add_argument("--ar", type=float, default=1.0)
    ap.add_argument("--re", type=float, default=8000.0)
    ap.add_argument("--dtype", default="f32s", choices=["f32s", "f64"])
    ap.add_argument("--cases", type=int, default=1,
                    help="also time Ar 0.4/1.0/2.0 in both storage types (0: skip)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--variant", type=int, default=-1, help="step tile shape (-1: default)")
    ap.add_argument("--copy-probe", type=int, default=0)
    return ap.parse_args()


def time_case(lbm, torch, nx, ny, re, dtype, steps, warmup, variant=-1):
    """Returns (seconds for `steps` steps, launches) with HIP events recorded on
    the stream the library launches on."""
    stream = torch.cuda.Stream()
    c = lbm.Cavity(nx, ny, re=re, u_lid=0.1, dtype=dtype)
    c.set_stream(stream)
    if variant >= 0:
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, variant)
    c.step(warmup)
    t_start = c.steps_done
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        ev0.record(stream)
        c.step(steps)
        ev1.record(stream)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3
    assert c.steps_done == t_start + steps
    mass = c.mass()
    c.close()
    return sec, mass


def cpu_baseline(nx, ny, re, steps):
    """The CPU oracle, untouched, on a bounded sample of the same workload."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:            # pragma: no cover
        threadpool_limits = None
    from oracle import d2q9
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        o = d2q9.Cavity(nx, ny, re=re, u_lid=0.1)
        o.step(10)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": round(nx * ny * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} steps of the {nx}x{ny} Re={re:g} cavity after 10 warm-up "
                      f"steps, NumPy FP64, one thread ({dt:.1f} s)"}


def copy_probe(nbytes):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 10}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the lattice of one cavity fits one "
              "MI355X; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from paper_2211_05009_amd import lbm
    nx = args.nx
    ny = int(round(nx * args.ar))
    sites = nx * ny

    sec, mass = time_case(lbm, torch, nx, ny, args.re, args.dtype, args.steps,
                          args.warmup, args.variant)
    mlups = sites * args.steps / sec / 1e6
    per_launch = sec / args.steps
    bpl = BYTES_PER_SITE[args.dtype] * sites            # algorithmic bytes per launch
    achieved = bpl / per_launch / 1e9
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(per_launch * 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32s" else "f64", "data": "synthetic",
        "config": {"workload": f"lid-driven cavity {nx}x{ny} (Ar={args.ar:g}), Re={args.re:g}, "
                               f"U=0.1, D2Q9 BGK, half-way bounce-back walls, "
                               f"{'FP32 f-w' if args.dtype == 'f32s' else 'FP64'} populations, "
                               f"from rest", "nx": nx, "ny": ny, "re": args.re,
                   "storage": args.dtype, "monitors_every": 100},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "lbm::k_step (fused pull stream + bounce-back + BGK)",
                     "bytes_per_launch": bpl,
                     "note": "per-launch time = HIP-event time of the timed region / steps "
                             "(includes the monitor kernels every 100 steps and launch gaps)"},
        "final_mass": mass,
    }
    if args.cases:
        cases = []
        for ar in (0.4, 1.0, 2.0):
            for dt in ("f32s", "f64"):
                nyc = int(round(nx * ar))
                k = max(2000, args.steps // 5)
                s, _ = time_case(lbm, torch, nx, nyc, args.re, dt, k, 1000)
                ml = nx * nyc * k / s / 1e6
                gbs = ml * BYTES_PER_SITE[dt] / 1e3
                cases.append({"nx": nx, "ny": nyc, "storage": dt, "steps": k,
                              "MLUPS": round(ml, 1), "GB/s": round(gbs, 1),
                              "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
        out["cases"] = cases
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, ny, args.re, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
