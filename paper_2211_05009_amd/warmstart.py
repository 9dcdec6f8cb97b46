"""Learned warm start: training data from the solver, training, and the
time-to-steady comparison of warm-started batches against cold single runs.

Orchestration only: the lattice updates, monitors, the network's forward and
backward passes, the optimiser and the mapping of a prediction onto a lattice
all run in the library's HIP kernels (include/lbm.h); this module chooses
cases, moves fields between device buffers and keeps the clock.

Steady state is Eq. 6 of arXiv 2211.05009 (Sec. 2.2 (iii)): the relative
change of the velocity field over 100 steps below a threshold (the paper
uses 1e-6).
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm

CANVAS_H, CANVAS_W = 256, 128
U_LID = 0.1
RHO_SCALE = 100.0      # network channel 0 = 100 (rho - 1)


# (level, ci, co) of the network's 15 convolutions as the kernels run them
# (padded channel counts); level l works on (256 >> l) x (128 >> l) pixels.
CONV_SHAPES = ((0, 32, 32), (0, 32, 32), (1, 32, 64), (1, 64, 64), (2, 64, 128),
               (2, 128, 128), (3, 128, 256), (3, 256, 256), (2, 384, 128), (2, 128, 128),
               (1, 192, 64), (1, 64, 64), (0, 96, 32), (0, 32, 32), (0, 32, 32))


def conv_flops(backward=False):
    """Multiply-add work (2 flops each) of the 3 x 3 convolutions for one
    sample: the forward pass, or the backward pass (weight gradients of every
    layer, input gradients of every layer but the first)."""
    fwd = [2 * 9 * ci * co * (CANVAS_H >> l) * (CANVAS_W >> l) for l, ci, co in CONV_SHAPES]
    return sum(fwd) + sum(fwd[1:]) if backward else sum(fwd)


def surrogate_throughput(sur, n=8, reps=20, seed=0):
    """MFMA throughput of the surrogate: TFLOP/s of the forward pass and of a
    whole training step (forward + backward + Adam) at batch n, timed over
    `reps` repetitions after one warm-up."""
    import torch
    rng = np.random.default_rng(seed)
    re, ar = rng.uniform(100.0, 3000.0, n), rng.uniform(0.4, 2.0, n)
    out = torch.empty((n, CANVAS_H, CANVAS_W, 3), dtype=torch.float32, device="cuda")
    mask = torch.ones((n, CANVAS_H, CANVAS_W), dtype=torch.float32, device="cuda")
    sur.forward(re, ar, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sur.forward(re, ar, out)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    target = out.clone()
    sur.train_step(re, ar, target, mask, 0.0, apply_update=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sur.train_step(re, ar, target, mask, 0.0, apply_update=False)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    f_fwd, f_bwd = conv_flops(), conv_flops(backward=True)
    return {"batch": n, "forward_ms": round(t_fwd * 1e3, 3),
            "forward_TFLOPs": round(n * f_fwd / t_fwd / 1e12, 2),
            "train_step_ms": round(t_train * 1e3, 3),
            "train_step_TFLOPs": round(n * (f_fwd + f_bwd) / t_train / 1e12, 2),
            "gflop_per_sample_fwd": round(f_fwd / 1e9, 3),
            "gflop_per_sample_fwd_bwd": round((f_fwd + f_bwd) / 1e9, 3)}


def sample_cases(n, seed, re_range=(100.0, 3000.0), ar_range=(0.4, 2.0)):
    """(Re, Ar) pairs uniform in the given ranges (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return rng.uniform(*re_range, size=n), rng.uniform(*ar_range, size=n)


def solve_steady(nx, ny, re, threshold, max_steps, dtype="f32s", chunk=10000,
                 warm=None, log=None, log_every=30.0, warm_mask=None):
    """Run a batch of cavities (lists nx, ny, re) from rest (or warm-started
    by `warm`, a Surrogate: every cavity, or those whose `warm_mask` entry is
    true) until every Eq. 6 residual is below `threshold` or `max_steps` is
    reached.  Returns the batch (kept alive) and a list of per-cavity dicts
    with the steps taken and the final residual.  With `log`, reports the
    number of running cavities every `log_every` s."""
    b = lbm.Batch(nx, ny, re, u_lid=U_LID, dtype=dtype)
    if warm is not None:
        for k in range(len(nx)):
            if warm_mask is None or warm_mask[k]:
                warm.warm_start_batch(b, k)
    b.set_threshold(threshold)
    done = 0
    t_log = time.perf_counter()
    while done < max_steps:
        step = min(chunk, max_steps - done)
        b.step(step)
        done += step
        active = sum(b.status(k)["active"] for k in range(len(nx)))
        if not active:
            break
        if log and time.perf_counter() - t_log > log_every:
            log(f"step {done}: {active} of {len(nx)} cavities running")
            t_log = time.perf_counter()
    return b, [b.status(k) for k in range(len(nx))]


def training_data(n, seed, nx=200, threshold=1e-6, max_steps=2_000_000, dtype="f32s"):
    """Steady fields of n random cavities on nx x round(nx Ar) lattices,
    resampled onto the network canvas on the GPU (lbm_batch_canvas).

    The lattice is finer than the 128-pixel canvas because BGK stays stable
    in the driven cavity only up to a lattice Reynolds number U / nu = Re / nx
    of about 16 (the paper's 500-site runs at Re = 8000 sit at 16): nx = 200
    covers Re = 3000.  Ar is returned as the lattice's ny / nx.  Returns a
    dict with re, ar, target [n, 256, 128, 3] and mask [n, 256, 128] as
    device tensors, steps, residual, seconds."""
    import torch
    re, ar = sample_cases(n, seed)
    nxs = [nx] * n
    nys = [int(np.rint(nx * a)) for a in ar]
    ar = np.array([y / nx for y in nys])
    t0 = time.perf_counter()
    b, st = solve_steady(nxs, nys, re, threshold, max_steps, dtype)
    target = torch.empty((n, CANVAS_H, CANVAS_W, 3), dtype=torch.float32, device="cuda")
    mask = torch.empty((n, CANVAS_H, CANVAS_W), dtype=torch.float32, device="cuda")
    for k in range(n):
        b.canvas(k, target[k], mask[k])
    b.close()
    return {"re": re, "ar": ar, "target": target, "mask": mask,
            "steps": [s["steps_done"] for s in st],
            "residual": [s["residual"] for s in st],
            "seconds": time.perf_counter() - t0}


def train(sur, data, epochs, batch=8, lr=1e-3, lr_final=1e-5, seed=0, log_every=0,
          log=print):
    """Adam over shuffled minibatches with a cosine learning-rate decay.
    Returns the per-epoch mean loss."""
    import torch
    n = len(data["re"])
    rng = np.random.default_rng(seed)
    tgt, msk = data["target"], data["mask"]
    hist = []
    total = epochs * ((n + batch - 1) // batch)
    it = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        losses = []
        for i in range(0, n, batch):
            idx = np.sort(perm[i:i + batch])
            t = it / max(total - 1, 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * t))
            ti = torch.as_tensor(idx, device="cuda")
            losses.append(sur.train_step(data["re"][idx], data["ar"][idx],
                                         tgt.index_select(0, ti).contiguous(),
                                         msk.index_select(0, ti).contiguous(), rate))
            it += 1
        hist.append(float(np.mean(losses)))
        if log_every and (ep + 1) % log_every == 0:
            log(f"epoch {ep + 1}: loss {hist[-1]:.5f}")
    return hist


def evaluate(sur, data):
    """Masked mean-squared error of the predictions on a data set."""
    import torch
    n = len(data["re"])
    out = torch.empty((n, CANVAS_H, CANVAS_W, 3), dtype=torch.float32, device="cuda")
    for i in range(0, n, sur.max_batch):
        j = min(i + sur.max_batch, n)
        sur.forward(data["re"][i:j], data["ar"][i:j], out[i:j])
    m = data["mask"][..., None]
    return float((((out - data["target"]) ** 2) * m).sum() / data["mask"].sum())


def time_to_steady(cases, threshold, max_steps, mode, sur=None, dtype="f32s", log=None,
                   ar_cut=None):
    """Wall time and steps to reach Eq. 6 residual < threshold for every
    cavity in `cases` ((nx, ny, re) list).

    mode: "single-cold" (one cavity after another, from rest: the plain
    method), "single-warm", "batch-cold", "batch-warm", "batch-warm-fallback"
    (warm start only for cavities with Ny / Nx >= ar_cut, the others from
    rest).  Warm starts include the surrogate inference and the mapping onto
    the lattice in the time.  `log` receives a progress line per cavity
    (single modes) or every 30 s (batch modes)."""
    import torch
    if mode not in TTS_MODES:
        raise ValueError(f"unknown mode {mode!r}: one of {TTS_MODES}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    if mode.startswith("single"):
        for (nx, ny, re) in cases:
            c = lbm.Cavity(nx, ny, re=re, u_lid=U_LID, dtype=dtype)
            if mode == "single-warm":
                sur.warm_start(c)
            done, res = 0, np.inf
            while done < max_steps:
                c.step(1000)
                done += 1000
                res = c.residual()[0]
                if res < threshold:
                    break
            steps.append(done)
            c.close()
            if log:
                log(f"{mode} {len(steps)}/{len(cases)}: {nx} x {ny}, Re {re:g}: {done} steps")
    else:
        nx, ny, re = zip(*cases)
        mask = None
        if mode == "batch-warm-fallback":
            mask = [y / x >= ar_cut for x, y in zip(nx, ny)]
        b, st = solve_steady(list(nx), list(ny), list(re), threshold, max_steps, dtype,
                             chunk=1000, warm=sur if mode.startswith("batch-warm") else None,
                             log=log, warm_mask=mask)
        steps = [s["steps_done"] for s in st]
        b.close()
    torch.cuda.synchronize()
    return {"mode": mode, "seconds": time.perf_counter() - t0, "steps": steps,
            "max_steps_hit": int(sum(s >= max_steps for s in steps))}



STEADY_RE = (1000.0, 1500.0, 2000.0, 2500.0, 3000.0)
STEADY_AR = (0.4, 0.8, 1.2, 1.6, 2.0)


def steady_sweep_cases(nx=500):
    """The steady Re x Ar sweep on the paper's 500 x (500 Ar) lattices."""
    return [(nx, int(round(nx * ar)), re) for ar in STEADY_AR for re in STEADY_RE]


def make_surrogate(normals, max_batch=8):
    """A surrogate with He-normal weights drawn from `normals` (a float array
    of lbm_sur_num_params standard normal draws)."""
    sur = lbm.Surrogate(max_batch=max_batch)
    lbm.lbm_sur_init_params(sur.s, normals)
    return sur


TTS_MODES = ("single-cold", "batch-warm", "batch-cold", "single-warm", "batch-warm-fallback")


def calibrate_fallback(sur, held, threshold, max_steps=2_000_000, dtype="f32s"):
    """The aspect ratio below which the warm start is not used, chosen on the
    held-out cavities (never on the cavities it is then applied to): their
    cold step counts come with `held` (training_data), their warm ones from a
    batched warm-started run; the cut a (one of their Ar values, or 0: warm
    everywhere) minimises the total steps of 'cold where Ar < a, warm
    elsewhere' on them (the smallest such a on ties)."""
    nx = 200
    nys = [int(round(nx * a)) for a in held["ar"]]
    b, st = solve_steady([nx] * len(nys), nys, list(held["re"]), threshold, max_steps, dtype,
                         warm=sur)
    b.close()
    warm = [s["steps_done"] for s in st]
    cold = list(held["steps"])
    ars = [y / nx for y in nys]
    best_cut, best = 0.0, sum(warm)
    for a in sorted(set(ars)):
        tot = sum(c if r < a else w for r, c, w in zip(ars, cold, warm))
        if tot < best:
            best_cut, best = a, tot
    return {"ar_cut": best_cut, "held_cold_total": int(sum(cold)),
            "held_warm_total": int(sum(warm)), "held_fallback_total": int(best),
            "held_cases": len(ars)}


STRICT_RE = (1000.0, 2000.0, 3000.0)
STRICT_AR = (0.4, 0.8, 1.2)


def strict_subset_cases(nx=500):
    """The nine cavities of the bounded FP64 Eq. 6 < 1e-8 study: Re 1000,
    2000, 3000 x Ar 0.4, 0.8, 1.2 of the steady sweep (the Ar 1.6 and 2.0
    cavities take most of the full sweep's time at this threshold)."""
    return [(nx, int(round(nx * ar)), re) for ar in STRICT_AR for re in STRICT_RE]


def _study_modes(cases, threshold, max_steps, modes, sur, dtype, log, ar_cut):
    res = {}
    for m in modes:
        r = time_to_steady(cases, threshold, max_steps, m, sur=sur, dtype=dtype, log=log,
                           ar_cut=ar_cut)
        res[m] = {"seconds": round(r["seconds"], 3), "steps_total": int(sum(r["steps"])),
                  "steps_median": float(np.median(r["steps"])),
                  "max_steps_hit": r["max_steps_hit"], "steps": [int(v) for v in r["steps"]]}
        if log:
            log(m, {k: v for k, v in res[m].items() if k != "steps"})
    return res


def steady_sweep_study(normals, threshold=1e-6, ntrain=200, epochs=150, nx=500,
                       max_steps=5_000_000, modes=TTS_MODES, dtype="f32s",
                       data_threshold=1e-6, log=None, strict=None):
    """Time-to-steady of the steady sweep (25 cavities, Re 1000-3000 x Ar
    0.4-2.0 at nx x (nx Ar)): plain = single cavities one after another from
    rest; treatment = one batch, every cavity warm-started by the surrogate
    (inference, mapping and mass renormalisation inside the timed region);
    batch-cold and single-warm are the two ablations.  Per-cavity step counts
    do not depend on batching (a batched cavity evolves bit for bit as it
    does alone, and both check Eq. 6 every 1000 steps).
    The one-off surrogate cost (training data and training) is reported
    separately.  `dtype` is the storage of the timed runs; the training data
    are FP32 runs to `data_threshold` (or the FP32 residual floor) whatever
    the timed storage."""
    t0 = time.perf_counter()
    data = training_data(ntrain, seed=0, threshold=data_threshold)
    t_data = time.perf_counter() - t0
    if log:
        log(f"training data: {ntrain} fields in {t_data:.1f} s")
    sur = make_surrogate(normals)
    t1 = time.perf_counter()
    hist = train(sur, data, epochs, log_every=25 if log else 0, log=log or print)
    t_train = time.perf_counter() - t1
    if log:
        log(f"trained {epochs} epochs in {t_train:.1f} s, loss {hist[-1]:.5f}")
    held = training_data(20, seed=1, threshold=data_threshold)
    perf = surrogate_throughput(sur)
    fallback = calibrate_fallback(sur, held, data_threshold)
    if log:
        log(f"cold-start fallback below Ar {fallback['ar_cut']:g} (held-out calibration)")
    cases = steady_sweep_cases(nx)
    res = _study_modes(cases, threshold, max_steps, modes, sur, dtype, log, fallback["ar_cut"])
    out = {"cases": len(cases), "lattice": f"{nx} x ({nx} Ar)", "threshold_eq6": threshold,
           "storage": dtype, "modes": res, "fallback": fallback,
           "case_list": [[x, y, r] for x, y, r in cases],
           "speedup": (round(res["single-cold"]["seconds"] / res["batch-warm"]["seconds"], 3)
                       if "single-cold" in res and "batch-warm" in res else None),
           "speedup_with_fallback": (round(res["single-cold"]["seconds"]
                                           / res["batch-warm-fallback"]["seconds"], 3)
                                     if "single-cold" in res and "batch-warm-fallback" in res
                                     else None),
           "surrogate": {"train_samples": ntrain, "epochs": epochs,
                         "data_seconds": round(t_data, 2), "train_seconds": round(t_train, 2),
                         "final_train_loss": round(hist[-1], 6),
                         "heldout_mse": round(evaluate(sur, held), 6), **perf}}
    if strict:
        # the same surrogate, a second threshold and storage (e.g. FP64 to 1e-8)
        sc = strict.get("cases") or strict_subset_cases(nx)
        sres = _study_modes(sc, strict["threshold"], strict.get("max_steps", max_steps),
                            strict["modes"], sur, strict["dtype"], log, fallback["ar_cut"])
        cold, warm = sres.get("batch-cold"), sres.get("batch-warm")
        out["strict"] = {"cases": len(sc), "case_list": [[x, y, r] for x, y, r in sc],
                         "threshold_eq6": strict["threshold"], "storage": strict["dtype"],
                         "modes": sres,
                         "steps_saved_warm": (round(1 - warm["steps_total"]
                                                    / cold["steps_total"], 4)
                                              if cold and warm else None),
                         "speedup_warm_vs_cold": (round(cold["seconds"] / warm["seconds"], 3)
                                                  if cold and warm else None)}
        fb = sres.get("batch-warm-fallback")
        if cold and fb:
            out["strict"]["speedup_fallback_vs_cold"] = round(cold["seconds"] / fb["seconds"], 3)
    sur.close()
    return out
