"""Throughput of the fused D2Q9 BGK update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--ar 1.0] [--re 8000] [--dtype f32s]

Workload: lid-driven cavity of 500 x (500 Ar) sites (the production lattice
of arXiv 2211.05009, Sec. 3.2-3.3), lid speed 0.1, Re = 8000, populations
stored as f - w in FP32, started from rest.  A "step" is one application of
Eq. 1 to every site (pull streaming, half-way / moving-wall bounce-back, BGK
collision) with the FP64 mass and Eq. 6 monitors every 100 steps, exactly as
lbm_step runs them.  The kernel tile shape is picked by the library's
autotuner before timing.  The lattice is resident in device memory before
timing starts.

One JSON line: MLUPS (million lattice-site updates per second); the HBM
roofline of the step kernel (72 B per site update in FP32, 144 B in FP64:
nine populations read and nine written; a multi-step launch counts K
updates); per-case figures for the other aspect ratios and FP64 storage; the
25-cavity Re x Ar sweep advanced as one batch against the same 25 cavities
run one after another; the time to steady state (Eq. 6 residual below
--tts-threshold, 1e-6 by default) of a steady 25-cavity sweep (Re 1000-3000
x Ar 0.4-2.0 at 500 x (500 Ar)) batched and warm-started by the learned
surrogate against plain cold single runs, with the batched-cold and
single-warm ablations and the surrogate's MFMA throughput; a plain device
copy's bandwidth on the same GPU; and the CPU oracle timed on a bounded
sample.

``--copy-probe BYTES`` instead runs a plain device copy of BYTES bytes ten
times (used to calibrate the rocprofv3 FETCH_SIZE / WRITE_SIZE counters).
Other single-purpose modes, each printing one JSON line: ``--flowmap`` (the
Fig. 17 flow-state map as one batch), ``--precision`` (FP32 f - w against
FP64 on the nine 500 x (500 Ar) cavities), ``--aux`` (kernels off the
metric: the paper's wall scheme, vortex extraction, surrogate, classifier).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 MLUPS & % HBM roofline at 500×500·Ar; sweep time-to-steady vs plain"
HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E, published
BYTES_PER_SITE = {"f32s": 72, "f64": 144}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--nx", type=int, default=500)
    ap.add_argument("--ar", type=float, default=1.0)
    ap.add_argument("--re", type=float, default=8000.0)
    ap.add_argument("--dtype", default="f32s", choices=["f32s", "f64"])
    ap.add_argument("--variant", type=int, default=-1,
                    help="step kernel shape (-1: autotune)")
    ap.add_argument("--cases", type=int, default=1,
                    help="also time Ar 0.4/1.0/2.0 in both storage types (0: skip)")
    ap.add_argument("--sweep", type=int, default=1,
                    help="also time the 25-cavity batch against sequential runs (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=50000)
    ap.add_argument("--sweep-sequential", type=int, default=1,
                    help="also time the same 25 cavities one after another (0: the batch only)")
    ap.add_argument("--tts", type=int, default=1,
                    help="time-to-steady of the steady sweep, batched + warm-started vs "
                         "plain (0: skip)")
    ap.add_argument("--tts-epochs", type=int, default=150)
    ap.add_argument("--tts-modes",
                    default="single-cold,batch-warm,batch-cold,single-warm,batch-warm-fallback",
                    help="time-to-steady arms: plain (single-cold), treatment (batch-warm), "
                         "the two ablations and the treatment with the cold-start fallback "
                         "(calibrated on held-out cavities)")
    ap.add_argument("--tts-strict", type=int, default=1,
                    help="also the FP64 Eq. 6 < 1e-8 study (warm vs cold, batched) on nine "
                         "cavities of the steady sweep (0: skip)")
    ap.add_argument("--tts-dtype", default="f32s", choices=["f32s", "f64"],
                    help="storage of the time-to-steady runs")
    ap.add_argument("--tts-threshold", type=float, default=1e-6,
                    help="Eq. 6 residual that counts as steady")
    ap.add_argument("--long", type=int, default=1,
                    help="also run the long unsteady cavity (500 x 750, Re 8000, 2 M steps, "
                         "5 probes) and classify its probe series (0: skip)")
    ap.add_argument("--flowmap", default="",
                    help="run a flow-state map instead: 'fig17' (153 cavities) or "
                         "'Re1,Re2,...:Ar1,Ar2,...'; prints one JSON line")
    ap.add_argument("--flowmap-steps", type=int, default=3_000_000)
    ap.add_argument("--large", type=int, default=1,
                    help="also time the 4096 x 4096 Re = 1e4 cavity, FP32 and FP64, "
                         "10,000 steps each (0: skip)")
    ap.add_argument("--cube", type=int, default=1,
                    help="also time the D3Q19 box: 256^3 FP32 and 192^3 FP64 (0: skip)")
    ap.add_argument("--aux", type=int, default=0,
                    help="instead time the kernels off the metric (non-equilibrium-"
                         "extrapolation step, vortex extraction, surrogate convolutions, "
                         "series classifier; 2: the surrogate alone; 3: the "
                         "non-equilibrium-extrapolation step alone); prints one JSON line")
    ap.add_argument("--precision", type=int, default=0,
                    help="instead compare FP32 f - w storage with FP64 on the nine "
                         "500 x (500 Ar) cavities (Ar 0.4/1.0/2.0 x Re 1000/4000/8000) after "
                         "1000 and 200,000 steps; prints one JSON line")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=500)
    ap.add_argument("--cpu-sweep-steps", type=int, default=150)
    ap.add_argument("--copy-probe", type=int, default=0)
    return ap.parse_args()


# Sources of the single-cavity step kernels (the shape each variant number
# launches is fixed by the library's variant table).
STEP_SOURCES = ("d2q9_step.hpp", "d2q9_temporal.hpp")


def source_hash():
    """Fingerprint of the step kernels' sources (decides whether stored
    counters still apply)."""
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        p = os.path.join(ROOT, "paper_2211_05009_amd", "csrc", name)
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def progress(*a):
    """Progress lines go to stderr; stdout carries only the result line."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_single(lbm, torch, nx, ny, re, dtype, steps, warmup, variant=-1, record=None,
                sync=None):
    """Seconds for `steps` steps (HIP events on the library's stream), the
    shape used and its steps per launch.  The timed lbm_step call runs with
    LBM_OPT_SYNC 0: a call with no monitor point returns once its launches
    are issued, and the region ends when the device is synchronised (calls
    that reach a monitor point finish before returning either way).
    `record`, a dict, receives what the timed call launched
    (lbm_last_launches); `sync`, a dict, receives the seconds of the same
    call from the same place on the 100-step grid with LBM_OPT_SYNC 1 (the
    call returning after its work has finished: its host wake-up and the
    event record after it fall inside the region)."""
    stream = torch.cuda.Stream()
    c = lbm.Cavity(nx, ny, re=re, u_lid=0.1, dtype=dtype)
    c.set_stream(stream)
    c.step(warmup - warmup % 100)
    if variant >= 0:
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, variant)
    else:
        c.autotune(chunks=4, use_cache=False)
    v = c.get_option(lbm.LBM_OPT_STEP_VARIANT)
    k = c.get_option(lbm.LBM_OPT_STEPS_PER_LAUNCH)
    c.step(1000)
    # warm-up calls of the timed call's length off a chunk boundary, from
    # both start buffers, so that graphs the library captures on first use
    # exist before timing; then back onto the chunk grid
    w = steps % 100
    if w:
        for _ in range(2):
            c.step(w)
            c.step(100 - w)
    t_start = c.steps_done
    e0, e1 = events(torch)

    def timed_call(sync_calls):
        c.set_option(lbm.LBM_OPT_SYNC, sync_calls)
        torch.cuda.synchronize()
        e0.record(stream)
        c.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        c.set_option(lbm.LBM_OPT_SYNC, 1)
        return e0.elapsed_time(e1) / 1e3

    sec = timed_call(0)
    assert c.steps_done == t_start + steps
    if record is not None:
        record.update(c.last_launches())
    if sync is not None:
        c.step((100 - steps % 100) % 100)    # back onto the 100-step grid
        sync["seconds"] = timed_call(1)
    mass = c.mass()
    c.close()
    return sec, (v, k), mass


def kernel_of(variant, k):
    """Kernel name of a single-cavity shape."""
    if k > 1:
        return "lbm::k_step_tb (K steps per launch, tile in LDS)"
    if variant >= 8:
        return "lbm::k_step_vec (16-byte loads)"
    return "lbm::k_step"


def roofline(rec, sec, sites, dtype, nx, ny):
    """Roofline block of the timed region from what it launched (rec:
    lbm_last_launches of the timed call).  The dominant kernel is the step
    kernel that applied most of the steps; its launch time is the region's
    HIP-event time over its launches when the region ran nothing else,
    otherwise the region's time per K steps (an upper bound)."""
    multi = rec["multi_launches"] * rec["steps_per_launch"]
    if multi >= rec["single_launches"]:
        v, k, launches = rec["multi_variant"], rec["steps_per_launch"], rec["multi_launches"]
        others = rec["single_launches"]
    else:
        v, k, launches = rec["single_variant"], 1, rec["single_launches"]
        others = rec["multi_launches"]
    pure = (others == 0 and rec["monitor_passes"] == 0 and rec["multi_monitor_launches"] == 0
            and rec["probe_launches"] == 0)
    bpl = BYTES_PER_SITE[dtype] * sites * k               # algorithmic bytes per launch
    launch_s = sec / launches if pure else sec * k / rec["steps"]
    achieved = bpl / launch_s / 1e9
    traffic = stored_traffic(v, 0, nx, ny, dtype) if pure else None
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": kernel_of(v, k), "variant": v, "steps_per_launch": k,
           "launches": launches, "bytes_per_launch": bpl,
           "launch_us": round(launch_s * 1e6, 3), "region_launches": rec,
           "note": ("launch time = HIP-event time of the timed region / its launches "
                    "(launch gaps included); the region ran only these launches"
                    if pure else
                    "launch time = HIP-event time of the timed region per K steps: the "
                    "region also ran other launches (region_launches)") +
                   "; algorithmic bytes count 72 B (FP32) / 144 B (FP64) per site update, "
                   "so a K-step launch can exceed the HBM peak; traffic = rocprofv3 "
                   "FETCH_SIZE + WRITE_SIZE per launch of this kernel, calibrated on a "
                   "plain copy"}
    if traffic:
        out["traffic_GBs"] = round(traffic / launch_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    return out


def time_sweep(lbm, torch, re_cases, dtype, steps, sequential=True):
    """25-cavity sweep: one batch vs the same cavities one after another."""
    nx, ny, re = zip(*re_cases)
    sites = sum(a * b for a, b in zip(nx, ny))
    stream = torch.cuda.Stream()
    b = lbm.Batch(nx, ny, re, u_lid=0.1, dtype=dtype)
    b.set_stream(stream)
    b.step(1000)
    bv, _ = b.autotune(chunks=2, use_cache=False)
    b.step(1000)
    e0, e1 = events(torch)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    b.close()
    out = {"cavities": len(re_cases), "sites": sites, "steps": steps, "storage": dtype,
           "batch_variant": bv,
           "batch_MLUPS": round(sites * steps / t_batch / 1e6, 1),
           "batch_GBs_effective": round(sites * steps * BYTES_PER_SITE[dtype] / t_batch / 1e9, 1)}
    if not sequential:
        return out
    t_seq = 0.0
    for (x, y, r) in re_cases:
        s, _, _ = time_single(lbm, torch, x, y, r, dtype, steps, 1000)
        t_seq += s
    out["sequential_MLUPS"] = round(sites * steps / t_seq / 1e6, 1)
    out["speedup"] = round(t_seq / t_batch, 3)
    return out


def time_cube(lbm, torch, n, dtype, steps):
    """D3Q19 lid-driven box of n^3 sites (Re 1000): MLUPS and the
    algorithmic bytes at 19 populations read and written per site update
    (152 B in FP32, 304 B in FP64; a two-step launch counts two updates),
    timed with HIP events on the handle's stream."""
    c = lbm.Cube(n, n, n, re=1000.0, u_lid=0.1, dtype=dtype)
    stream = torch.cuda.Stream()
    lbm.lbm3d_set_stream(c.h, stream)
    best, _ = c.autotune(2)
    k = c.get_option(lbm.LBM_OPT_STEPS_PER_LAUNCH)
    c.step(200)
    e0, e1 = events(torch)
    torch.cuda.synchronize()
    e0.record(stream)
    c.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    c.close()
    mlups = n ** 3 * steps / sec / 1e6
    bps = 152 if dtype == "f32s" else 304
    return {"sites": f"{n}^3", "storage": dtype, "steps": steps, "variant": best,
            "steps_per_launch": k, "MLUPS": round(mlups, 1), "GB/s": round(mlups * bps / 1e3, 1),
            "frac_hbm": round(mlups * bps / 1e3 / HBM_PEAK_GBS, 4)}


def copy_bandwidth(torch, nbytes=1 << 30):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = events(torch)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    return round(2 * nbytes * 10 / sec / 1e9, 1)


def host_cpu():
    """Model name of the host CPU and the CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def _oracle_run(args):
    """One oracle cavity (one process, one thread): site updates and seconds."""
    nx, ny, re, steps = args
    from threadpoolctl import threadpool_limits
    from oracle import d2q9
    with threadpool_limits(limits=1):
        o = d2q9.Cavity(nx, ny, re=re, u_lid=0.1)
        o.step(2)
        t0 = time.perf_counter()
        o.step(steps)
        return nx * ny * steps, time.perf_counter() - t0


def cpu_baseline(nx, ny, re, steps, sweep, sweep_steps):
    """The CPU oracle, untouched, on bounded samples of the workloads: the
    headline lattice in one process and one thread, and the 25-cavity sweep
    with one cavity per process over the CPUs available (at most 16: the
    host's share of one GPU).  Runs before anything touches the GPU, so the
    worker processes are plain forks."""
    import multiprocessing as mp
    model, nproc, avail = host_cpu()
    upd, dt = _oracle_run((nx, ny, re, steps))
    out = {"value": round(upd / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "sample": f"{steps} steps of the {nx}x{ny} Re={re:g} cavity after 2 warm-up "
                     f"steps, NumPy FP64, one process, one thread ({dt:.1f} s)",
           "cpu_model": model, "nproc": nproc, "cpus_available": avail}
    if sweep:
        workers = max(1, min(16, avail))
        jobs = [(x, y, r, sweep_steps) for (x, y, r) in sweep]
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_run, jobs, chunksize=1)
        wall = time.perf_counter() - t0
        total = sum(u for u, _ in res)
        out["sweep_aggregate"] = {
            "value": round(total / wall / 1e6, 3), "unit": "MLUPS", "cores": workers,
            "sample": f"the {len(jobs)} sweep cavities, {sweep_steps} steps each after 2 "
                      f"warm-up steps, one cavity per process, {workers} processes of one "
                      f"thread; aggregate = site updates / wall time of the pool "
                      f"({wall:.1f} s)",
            "per_process_MLUPS_mean": round(float(sum(u / t for u, t in res)) / len(res)
                                            / 1e6, 3)}
    return out


def copy_probe(nbytes):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 10}), flush=True)


def stored_traffic(variant, mon, nx, ny, dtype):
    """Per-launch HBM traffic (calibrated FETCH_SIZE + WRITE_SIZE bytes)
    measured by rocprofv3 for exactly this kernel source, shape, monitor
    form (0: plain launch) and lattice, else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entries = json.load(fh)["entries"]
    except (OSError, ValueError, KeyError, TypeError):
        return None
    for t in entries:
        if (t.get("source_hash") == source_hash() and t.get("variant") == variant
                and t.get("mon") == mon and t.get("nx") == nx and t.get("ny") == ny
                and t.get("storage") == dtype):
            return t.get("bytes_per_launch")
    return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the lattice of one cavity fits one "
              "MI355X; multi-GPU runs are not implemented", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if (args.cpu_baseline and not (args.flowmap or args.aux or args.precision
                                   or args.copy_probe)):
        # the oracle first: its worker processes are forked before the GPU is touched
        from cavity_inputs import sweep_cases
        progress("CPU oracle baseline")
        ny0 = int(round(args.nx * args.ar))
        cpu = cpu_baseline(args.nx, ny0, args.re, args.cpu_steps,
                           sweep_cases(args.nx) if args.sweep else None, args.cpu_sweep_steps)
    import torch
    if args.flowmap:
        return run_flowmap(args)
    if args.aux:
        return run_aux(surrogate_only=args.aux == 2, nee_only=args.aux == 3)
    if args.precision:
        return run_precision()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from paper_2211_05009_amd import lbm
    from cavity_inputs import sweep_cases
    nx = args.nx
    ny = int(round(nx * args.ar))
    sites = nx * ny

    progress(f"headline {nx}x{ny} {args.dtype}, {args.steps} steps")
    rec, sync = {}, {}
    sec, (variant, k), mass = time_single(lbm, torch, nx, ny, args.re, args.dtype, args.steps,
                                          args.warmup, args.variant, record=rec, sync=sync)
    mlups = sites * args.steps / sec / 1e6
    per_step = sec / args.steps
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(per_step * 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32s" else "f64", "data": "synthetic",
        "config": {"workload": f"lid-driven cavity {nx}x{ny} (Ar={args.ar:g}), Re={args.re:g}, "
                               f"U=0.1, D2Q9 BGK, half-way bounce-back walls, "
                               f"{'FP32 f-w' if args.dtype == 'f32s' else 'FP64'} populations, "
                               f"from rest", "nx": nx, "ny": ny, "re": args.re,
                   "storage": args.dtype, "monitors_every": 100},
        "roofline": roofline(rec, sec, sites, args.dtype, nx, ny),
        # the same call with LBM_OPT_SYNC 1 (returning after its work has
        # finished), from the same place on the 100-step grid
        "sync_call": {"value": round(sites * args.steps / sync["seconds"] / 1e6, 2),
                      "ms_per_step": round(sync["seconds"] / args.steps * 1e3, 6)},
        "final_mass": mass,
        "source_hash": source_hash(),
    }
    if args.cases:
        cases = []
        for ar in (0.4, 1.0, 2.0):
            for dt in ("f32s", "f64"):
                nyc = int(round(nx * ar))
                kk = max(10000, args.steps // 10)
                progress(f"case {nx}x{nyc} {dt}")
                s, (v, _), _ = time_single(lbm, torch, nx, nyc, args.re, dt, kk, 1000)
                ml = nx * nyc * kk / s / 1e6
                gbs = ml * BYTES_PER_SITE[dt] / 1e3
                cases.append({"nx": nx, "ny": nyc, "storage": dt, "steps": kk, "variant": v,
                              "MLUPS": round(ml, 1), "GB/s": round(gbs, 1),
                              "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
        out["cases"] = cases
    if args.sweep:
        progress("25-cavity sweep: batch vs sequential")
        out["sweep"] = time_sweep(lbm, torch, sweep_cases(nx), "f32s", args.sweep_steps,
                                  sequential=bool(args.sweep_sequential))
    if args.tts:
        from paper_2211_05009_amd import warmstart
        from cavity_inputs import normal_draws
        from paper_2211_05009_amd.lbm import lbm_sur_num_params, Surrogate
        probe = Surrogate(max_batch=1)
        npar = lbm_sur_num_params(probe.s)
        probe.close()
        progress("time to steady: training data, training, plain and warm-started sweeps")
        out["sweep_time_to_steady"] = warmstart.steady_sweep_study(
            normal_draws(npar, seed=0), threshold=args.tts_threshold, epochs=args.tts_epochs,
            modes=tuple(args.tts_modes.split(",")), dtype=args.tts_dtype, log=progress,
            strict=({"threshold": 1e-8, "dtype": "f64",
                     "modes": ("batch-cold", "batch-warm", "batch-warm-fallback")}
                    if args.tts_strict else None))
    if args.large:
        large = []
        for dt in ("f32s", "f64"):
            progress(f"4096 x 4096 {dt}")
            sec, (v, k), _ = time_single(lbm, torch, 4096, 4096, 1e4, dt, 10000, 1000)
            ml = 4096 * 4096 * 10000 / sec / 1e6
            gbs = ml * BYTES_PER_SITE[dt] / 1e3
            large.append({"nx": 4096, "ny": 4096, "re": 1e4, "storage": dt, "steps": 10000,
                          "variant": v, "steps_per_launch": k, "MLUPS": round(ml, 1),
                          "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
        out["large"] = large
    if args.cube:
        progress("D3Q19 box")
        out["cube"] = [time_cube(lbm, torch, n, dt, k) for n, dt, k in
                       ((256, "f32s", 2000), (192, "f64", 1000))]
    if args.long:
        from paper_2211_05009_amd import flowmap
        progress("long unsteady cavity with probes")
        out["long_unsteady"] = flowmap.long_unsteady(log=progress)
    out["copy_GBs"] = copy_bandwidth(torch)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def run_precision():
    """Error of the FP32 f - w storage against FP64 for each reported result
    (velocity field, mass, Eq. 6 residual, Psi maximum, the observing point's
    velocity), on the nine 500 x (500 Ar) cavities.  The FP64 path matches
    the CPU oracle to 1e-12 (the parity tests), so it stands in for it at
    these sizes.  Beyond about a thousand steps the unsteady cavities
    (Re >= 4500) amplify any rounding difference, so their 200 k-step figures
    measure trajectory divergence, not accuracy."""
    import numpy as np
    from paper_2211_05009_amd import lbm
    from paper_2211_05009_amd.flowmap import observing_point
    rows = []
    for ar in (0.4, 1.0, 2.0):
        for re in (1000.0, 4000.0, 8000.0):
            nx, ny = 500, int(round(500 * ar))
            progress(f"precision {nx}x{ny} Re {re:g}")
            h = {dt: lbm.Cavity(nx, ny, re=re, u_lid=0.1, dtype=dt) for dt in ("f64", "f32s")}
            pt = np.array([observing_point(ar)])
            done = 0
            for horizon in (1000, 200000):
                for c in h.values():
                    c.step(horizon - done)
                done = horizon
                m = {dt: c.moments() for dt, c in h.items()}
                du = max(np.abs(m["f32s"][1] - m["f64"][1]).max(),
                         np.abs(m["f32s"][2] - m["f64"][2]).max())
                psi = {dt: c.stream_function().max() for dt, c in h.items()}
                pr = {dt: c.probe(pt)[0] for dt, c in h.items()}
                res = {dt: c.residual()[0] for dt, c in h.items()}
                rows.append({"nx": nx, "ny": ny, "re": re, "steps": horizon,
                             "max_du_over_U": float(du / 0.1),
                             "max_drho": float(np.abs(m["f32s"][0] - m["f64"][0]).max()),
                             "mass_rel": float(abs(h["f32s"].mass() - h["f64"].mass())
                                               / (nx * ny)),
                             "residual": [float(res["f64"]), float(res["f32s"])],
                             "psi_max_rel": float(abs(psi["f32s"] - psi["f64"]) / psi["f64"]),
                             "probe_du_over_U": float(np.abs(pr["f32s"][1:] - pr["f64"][1:]).max()
                                                      / 0.1)})
            for c in h.values():
                c.close()
    print(json.dumps({"precision": rows}), flush=True)


def run_aux(surrogate_only=False, nee_only=False):
    """Timings of the kernels off the metric, for profiling (one JSON line)."""
    import torch
    import numpy as np
    from paper_2211_05009_amd import lbm, warmstart
    from cavity_inputs import normal_draws
    out = {}
    if surrogate_only:
        sur = warmstart.make_surrogate(normal_draws(lbm.Surrogate(1).num_params, seed=0))
        out["surrogate"] = warmstart.surrogate_throughput(sur)
        sur.close()
        print(json.dumps({"aux": out}), flush=True)
        return
    # the paper's walls: the 256 x 256 validation lattice and a 500 x 500 one
    for n, steps in ((257, 20000), (501, 10000)):
        for dt in ("f64", "f32s"):
            c = lbm.Cavity(n, n, re=1000.0, u_lid=0.1, dtype=dt, wall="nee")
            c.autotune(chunks=5)
            c.step(2000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.step(steps)
            sec = time.perf_counter() - t0
            out[f"nee_{n}_{dt}"] = {"MLUPS": round(n * n * steps / sec / 1e6, 1),
                                    "variant": c.get_option(lbm.LBM_OPT_STEP_VARIANT)}
            c.close()
    if nee_only:
        print(json.dumps({"aux": out}), flush=True)
        return
    progress("vortex extraction")
    c = lbm.Cavity(500, 600, re=6000.0, u_lid=0.1, dtype="f32s")
    c.step(20000)
    t0 = time.perf_counter()
    for _ in range(10):
        c.vortex_extrema()
        n = c.vortex_centres(1e-9 * 50)[1]
    out["vortex_500x600_ms"] = round((time.perf_counter() - t0) / 10 * 1e3, 3)
    out["vortex_centres"] = n
    c.close()
    progress("surrogate throughput")
    sur = warmstart.make_surrogate(normal_draws(lbm.Surrogate(1).num_params, seed=0))
    out["surrogate"] = warmstart.surrogate_throughput(sur)
    sur.close()
    progress("series classifier")
    k = np.arange(10000, dtype=np.float64)
    rng = np.random.default_rng(0)
    ser = np.stack([np.sin(2 * np.pi * k / (80 + i)) + 1e-3 * rng.normal(size=k.size)
                    for i in range(153)])
    dev = torch.tensor(ser, dtype=torch.float64, device="cuda")
    lbm.lbm_classify_series(dev, 1e-6, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = lbm.lbm_classify_series(dev, 1e-6, 0.05)
    out["classify_153x10000_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    out["classify_periodic"] = sum(r["state"] == "periodic" for r in res)
    print(json.dumps({"aux": out}), flush=True)


def run_flowmap(args):
    """Flow-state map (Sec. 3.3, Fig. 17) as one batch; one JSON line."""
    from paper_2211_05009_amd import flowmap
    if args.flowmap == "fig17":
        res, ars = flowmap.FIG17_RE, flowmap.FIG17_AR
    else:
        a, b = args.flowmap.split(":")
        res = [float(v) for v in a.split(",")]
        ars = [float(v) for v in b.split(",")]
    cases = [(re, ar) for ar in ars for re in res]
    progress(f"flow-state map: {len(cases)} cavities, {args.flowmap_steps} steps")
    rows, run = flowmap.state_map(cases, steps=args.flowmap_steps, log=progress)
    print(json.dumps({"flowmap": rows, "run": run, "cavities": len(cases)}), flush=True)


if __name__ == "__main__":
    main()
