"""GPU parity: the HIP step against the CPU FP64 oracle, element by element.

Bars (written in each test):
  * FP64 storage: max |d rho| and max |d u| / U <= 1e-12 after up to 1000
    steps; populations to 1e-12 as well.
  * FP32 f - w storage: max |d u| <= 1e-5 U over a 1000-step horizon.
Sizes span several 64-wide tiles and ragged tails; the full 500 x (500 Ar)
lattices are checked one launch at a time (the oracle applies one step to the
GPU's own state) and over 1000 steps at Ar = 0.4, Re = 8000.
"""
import math

import numpy as np
import pytest

from cavity_inputs import U_LID, random_shift
from oracle import d2q9
from oracle.d2q9 import W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_UTOL = 1e-5 * U_LID


@pytest.fixture(scope="module")
def lbm():
    from paper_2211_05009_amd import lbm as mod
    return mod


def oracle_from(f0, tau, u=U_LID):
    ny, nx = f0.shape[1:]
    o = d2q9.Cavity(nx, ny, tau=tau, u_lid=u)
    o.set_state(f0)
    return o


def compare(gpu, orc, dtype, what=""):
    """gpu, orc: Cavity objects at the same step."""
    rg, uxg, uyg = gpu.moments()
    ro, uxo, uyo = orc.moments()
    du = max(np.max(np.abs(uxg - uxo)), np.max(np.abs(uyg - uyo)))
    dr = np.max(np.abs(rg - ro))
    if dtype == "f64":
        assert dr <= F64_TOL, f"{what} rho {dr}"
        assert du / U_LID <= F64_TOL, f"{what} u {du}"
        fg = gpu.get_populations()
        fo = orc.post_collision()
        assert np.max(np.abs(fg - fo)) <= F64_TOL, what
    else:
        assert du <= F32_UTOL, f"{what} u {du}"
        assert dr <= 1e-5, f"{what} rho {dr}"
    return dr, du


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_first_step_from_rest_matches_closed_form(lbm, dtype):
    """One step from rest: lid-row populations 7, 8 become 1/36 -+ U/6, all
    else stays w (Eq. 1 with the moving-wall term); checked through the
    stored post-collision state."""
    c = lbm.Cavity(37, 29, tau=0.7, u_lid=U_LID, dtype=dtype)
    c.step(1)
    o = d2q9.Cavity(37, 29, tau=0.7, u_lid=U_LID).step(1)
    tol = 1e-15 if dtype == "f64" else 2e-8
    assert np.max(np.abs(c.get_populations() - o.post_collision())) <= tol
    rho, ux, uy = c.moments()
    assert np.max(np.abs(ux[-1] - U_LID / 3)) <= (1e-16 if dtype == "f64" else 1e-8)
    assert np.max(np.abs(ux[:-1])) == 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_parity_from_rest_64(lbm, dtype):
    """64 x 64 cavity, Re = 100, 1000 steps from rest (graph chunks)."""
    c = lbm.Cavity(64, 64, re=100.0, u_lid=U_LID, dtype=dtype)
    o = d2q9.Cavity(64, 64, re=100.0, u_lid=U_LID)
    for k in range(4):
        c.step(250)
        o.step(250)
        compare(c, o, dtype, f"t={o.t}")


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
@pytest.mark.parametrize("nx,ny,tau,seed", [(2, 2, 0.8, 1), (3, 70, 0.6, 2),
                                            (65, 3, 0.9, 3), (130, 67, 0.51875, 4),
                                            (200, 129, 1.2, 5), (64, 64, 0.55, 6)])
def test_parity_random_state(lbm, dtype, nx, ny, tau, seed):
    """Random low-Mach state, ragged lattices, 257 steps (two graph chunks and
    57 single launches), several relaxation times."""
    f0 = W[:, None, None] + random_shift(nx, ny, seed)
    c = lbm.Cavity(nx, ny, tau=tau, u_lid=U_LID, dtype=dtype)
    c.set_populations(f0)
    o = oracle_from(f0, tau)
    compare(c, o, dtype, "t=0")
    c.step(257)
    o.step(257)
    compare(c, o, dtype, "t=257")


def interior_tiles(nx, ny, tx, ty, k):
    """Tiles of a K-step shape whose region (the tile plus K sites on every
    side) lies inside the cavity: the ones that take the wall-free pull."""
    n = 0
    for by in range((ny + ty - 1) // ty):
        for bx in range((nx + tx - 1) // tx):
            x0, y0 = bx * tx - k, by * ty - k
            n += x0 >= 0 and x0 + tx + 2 * k <= nx and y0 >= 0 and y0 + ty + 2 * k <= ny
    return n


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
@pytest.mark.parametrize("nx,ny", [(131, 77), (260, 150)])
def test_variants_graph_and_direct_launch_agree_bitwise(lbm, dtype, nx, ny):
    """Every tile shape and both launch paths compute the same per-site
    arithmetic, so their results agree bit for bit.  On 260 x 150 every
    multi-step shape has tiles away from the walls (the wall-free pull) as
    well as wall tiles and ragged edge tiles; 230 steps are two chunks and a
    30-step span off the chunk grid."""
    f0 = W[:, None, None] + random_shift(nx, ny, 7)
    ref = None
    c = lbm.Cavity(nx, ny, tau=0.56, u_lid=U_LID, dtype=dtype)
    nvar = c.get_option(lbm.LBM_OPT_NUM_VARIANTS)
    for v in range(nvar):
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        k = c.get_option(lbm.LBM_OPT_STEPS_PER_LAUNCH)
        tx, ty = c.get_option(lbm.LBM_OPT_TILE_X), c.get_option(lbm.LBM_OPT_TILE_Y)
        if k > 1 and nx >= 260:
            assert interior_tiles(nx, ny, tx, ty, k) > 0, (v, tx, ty, k)
            assert nx % tx and ny % ty, "ragged edge tiles"
        for graph in (1, 0):
            c.set_option(lbm.LBM_OPT_USE_GRAPH, graph)
            c.set_populations(f0)
            c.step(230)
            rec = c.last_launches()
            if k > 1:   # the 30-step span: 30 // K launches of K steps, the rest single
                assert rec["multi_variant"] == v and rec["single_launches"] == 30 % k, rec
                assert rec["multi_launches"] * k + rec["single_launches"] == 230, rec
            f = c.get_populations()
            if ref is None:
                ref = f
            assert np.array_equal(f, ref), (v, graph)


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_calls_that_return_once_issued(lbm, dtype):
    """LBM_OPT_SYNC 0: calls without a monitor point return once their
    launches are issued; after a device synchronisation the populations
    equal those of synchronous calls bit for bit, calls that reach a
    monitor point still return the same monitors, and the launch record is
    the same."""
    import torch
    nx, ny, tau = 131, 77, 0.56
    f0 = W[:, None, None] + random_shift(nx, ny, 37)
    calls = [20, 37, 43, 100, 45, 5, 250]
    runs = {}
    for sync in (1, 0):
        c = lbm.Cavity(nx, ny, tau=tau, u_lid=U_LID, dtype=dtype)
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, 24 if dtype == "f32s" else 22)
        c.set_populations(f0)
        c.set_option(lbm.LBM_OPT_SYNC, sync)
        assert c.get_option(lbm.LBM_OPT_SYNC) == sync
        states, mons, recs = [], [], []
        for n in calls:
            c.step(n)
            recs.append(c.last_launches())
            torch.cuda.synchronize()
            states.append(c.get_populations())
            mons.append((c.mass(), *c.residual()))
        runs[sync] = (states, mons, recs)
        c.close()
    for a, b in zip(runs[1][0], runs[0][0]):
        assert np.array_equal(a, b)
    for a, b in zip(runs[1][1], runs[0][1]):
        assert a[2] == b[2] and (a[1] == b[1] or (math.isinf(a[1]) and math.isinf(b[1])))
        assert a[0] == b[0]
    assert runs[1][2] == runs[0][2]


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
@pytest.mark.parametrize("variant", [22, 12, 20, 14])
def test_short_and_unaligned_calls(lbm, dtype, variant):
    """Calls shorter than or off the 100-step chunk grid run the multi-step
    shape's K-step launches wherever t is a multiple of K and K steps remain
    (one-step launches otherwise), and give the same populations, bit for
    bit, as one-step launches of shape 0; monitors land on the same steps
    and agree to 1e-12 relative; probe records every 10 steps (a multiple of
    K = 2, 5, 10; not of K = 4, which falls back to one-step launches) are
    identical.  FP64 is checked against the oracle at the end."""
    nx, ny, tau = 131, 77, 0.56
    f0 = W[:, None, None] + random_shift(nx, ny, 31)
    calls = [20, 37, 3, 140, 45, 7, 250, 1, 99]
    pts = np.array([[0.5, 0.5], [0.1, 0.55], [0.9, 0.1]])
    runs = {}
    for v in (0, variant):
        c = lbm.Cavity(nx, ny, tau=tau, u_lid=U_LID, dtype=dtype)
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        c.set_populations(f0)
        c.probe_config(pts, 10, 1000)
        k = c.get_option(lbm.LBM_OPT_STEPS_PER_LAUNCH)
        states, mons, recs = [], [], []
        for n in calls:
            t0 = c.steps_done
            c.step(n)
            rec = c.last_launches()
            assert rec["steps"] == n
            assert rec["single_launches"] + k * rec["multi_launches"] == n, rec
            recs.append(rec)
            states.append(c.get_populations())
            mons.append((c.mass(), *c.residual()))
            if v == variant and k > 1 and 10 % k == 0 and t0 % k == 0 and n % k == 0:
                assert rec["single_launches"] == 0, (t0, n, rec)
        runs[v] = (states, mons, recs, c.probe_read(1000), k)
        c.close()
    s0, m0, _, p0, _ = runs[0]
    s1, m1, r1, p1, k = runs[variant]
    for a, b, n in zip(s0, s1, calls):
        assert np.array_equal(a, b), n
    for (ma, ra, ta), (mb, rb, tb) in zip(m0, m1):
        assert ta == tb
        assert abs(ma - mb) <= 1e-12 * nx * ny
        assert (math.isinf(ra) and math.isinf(rb)) or abs(ra - rb) <= 1e-12 * abs(ra)
    assert np.array_equal(p0, p1)
    # the first call (20 steps from t = 0) is K-step launches only when K
    # divides both 20 and the probe cadence
    if 10 % k == 0:
        assert r1[0]["multi_launches"] == 20 // k and r1[0]["single_launches"] == 0
        assert r1[0]["multi_variant"] == variant
    else:
        assert r1[0]["multi_launches"] == 0 and r1[0]["single_launches"] == 20
    if dtype == "f64":
        o = oracle_from(f0, tau).step(sum(calls))
        fo = o.post_collision()
        assert np.max(np.abs(s1[-1] - fo)) <= F64_TOL


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
@pytest.mark.parametrize("ar", [0.4, 1.0, 2.0])
def test_full_size_single_launch(lbm, dtype, ar):
    """500 x (500 Ar): one launch of the step, as timed by the benchmark
    (after a 100-step graph chunk), against one oracle step applied to the
    GPU's own stored state."""
    nx, ny = 500, int(round(500 * ar))
    tau = d2q9.relaxation_time(nx, 8000.0, U_LID)
    c = lbm.Cavity(nx, ny, re=8000.0, u_lid=U_LID, dtype=dtype)
    c.set_populations(W[:, None, None] + random_shift(nx, ny, 11))
    c.step(100)                                   # one captured chunk
    fs = c.get_populations()                      # f*(100)
    c.step(1)                                     # one direct launch
    o = d2q9.Cavity(nx, ny, tau=tau, u_lid=U_LID)
    f101 = o.stream(fs)
    o.set_state(f101, t=101)
    ref = o.post_collision()
    got = c.get_populations()
    if dtype == "f64":
        assert np.max(np.abs(got - ref)) <= 1e-15
    else:
        # one FP32 step from an exactly representable state: each stored
        # value passes through ~10 FP32 operations on numbers no larger than
        # the largest shift |f - w|, so the bound is 16 ulps of that shift
        gmax = np.max(np.abs(ref - W[:, None, None]))
        assert np.max(np.abs(got - ref)) <= 16 * 2.0 ** -24 * gmax


def _light_cone_check(f_start, f_end, tau, n, width, dtype, what):
    """Compare the GPU's f*(t + n) with the oracle on windows of the lattice.

    In n steps information moves at most n sites, so the oracle can evolve a
    width x width window cut out of the GPU's f*(t): where a window edge is
    not a wall of the cavity the oracle's wall there is wrong, but its effect
    reaches at most n sites in.  Sites further than n + 1 from such an edge
    come out exactly as on the whole lattice.  Windows: the four corners
    (two walls and, at the top, the lid) and the centre."""
    _, ny, nx = f_start.shape
    m = n + 1
    xs = sorted({0, (nx - width) // 2, nx - width})
    ys = sorted({0, (ny - width) // 2, ny - width})
    wins = [(x0, y0) for x0 in xs for y0 in ys
            if (x0, y0) in {(xs[0], ys[0]), (xs[0], ys[-1]), (xs[-1], ys[0]),
                            (xs[-1], ys[-1]), (xs[1], ys[1])}]
    worst = 0.0
    for x0, y0 in wins:
        x1, y1 = x0 + width, y0 + width
        o = d2q9.Cavity(width, width, tau=tau, u_lid=U_LID)
        o.set_state(o.stream(f_start[:, y0:y1, x0:x1]), t=1)
        o.step(n - 1)
        ref = o.post_collision()
        # exact region: n + 1 sites away from window edges that are not walls
        ex0 = 0 if x0 == 0 else m
        ex1 = width if x1 == nx else width - m
        ey0 = 0 if y0 == 0 else m
        ey1 = width if y1 == ny else width - m
        got = f_end[:, y0 + ey0:y0 + ey1, x0 + ex0:x0 + ex1]
        want = ref[:, ey0:ey1, ex0:ex1]
        assert got.size > 0
        if dtype == "f64":
            d = np.max(np.abs(got - want))
            assert d <= F64_TOL, (what, x0, y0, d)
        else:
            rg, ug, vg = d2q9.macroscopic(got)
            rw, uw, vw = d2q9.macroscopic(want)
            d = max(np.abs(ug - uw).max(), np.abs(vg - vw).max())
            assert d <= F32_UTOL, (what, x0, y0, d)
        worst = max(worst, d)
    return worst


@pytest.mark.parametrize("dtype,nx,ny,variant", [
    ("f32s", 500, 500, 22), ("f64", 500, 500, 22), ("f32s", 500, 1000, 21),
    ("f64", 500, 1000, 19), ("f32s", 4096, 4096, 22), ("f64", 4096, 4096, 19),
    ("f32s", 4096, 4096, 16), ("f32s", 4096, 4096, 18), ("f32s", 4096, 4096, 23),
    ("f64", 4096, 4096, 16), ("f64", 4096, 4096, 18), ("f64", 4096, 4096, 23)])
def test_full_size_chunk_in_the_timed_shape(lbm, dtype, nx, ny, variant):
    """A 100-step chunk as the benchmark runs it (graph replay, the
    multi-step shape the autotuner picks for this lattice and storage, the
    Eq. 6 monitor inside the chunk's first two launches) on the full
    lattices of the single-cavity and long-run workloads, from a random
    low-Mach state, checked against the oracle on light-cone windows.  Bars:
    FP64 populations <= 1e-12, FP32 velocity <= 1e-5 U."""
    tau = d2q9.relaxation_time(nx, 8000.0 if nx == 500 else 1e4, U_LID)
    c = lbm.Cavity(nx, ny, tau=tau, u_lid=U_LID, dtype=dtype)
    c.set_option(lbm.LBM_OPT_STEP_VARIANT, variant)
    c.set_populations(W[:, None, None] + random_shift(nx, ny, 23))
    c.step(100)
    f_start = c.get_populations()                 # f*(100)
    c.step(100)                                   # one graph chunk
    f_end = c.get_populations()                   # f*(200)
    assert c.residual()[1] == 200
    c.close()
    worst = _light_cone_check(f_start, f_end, tau, 100, 234, dtype, f"{nx}x{ny} {dtype}")
    print(f"{nx}x{ny} {dtype} shape {variant}: worst window difference {worst:.3e}")


@pytest.fixture(scope="module")
def re8000_oracle():
    """Oracle run: 500 x 200 (Ar = 0.4), Re = 8000, 1000 steps from rest."""
    o = d2q9.Cavity(500, 200, re=8000.0, u_lid=U_LID)
    o.step(1000)
    return o


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_full_size_1000_steps_re8000(lbm, dtype, re8000_oracle):
    c = lbm.Cavity(500, 200, re=8000.0, u_lid=U_LID, dtype=dtype)
    c.step(1000)
    dr, du = compare(c, re8000_oracle, dtype, "500x200 Re=8000 t=1000")
    print(f"{dtype}: max|drho| {dr:.3e}  max|du|/U {du / U_LID:.3e}")


@pytest.mark.parametrize("ar", [0.4, 1.0, 2.0])
@pytest.mark.parametrize("re", [1000.0, 4000.0, 8000.0])
def test_full_size_fp32_against_fp64_1000_steps(lbm, re, ar):
    """The nine 500 x (500 Ar) cavities of the single-cavity workload, 1000
    steps from rest: FP32 f - w storage against FP64 storage, which is held
    to the oracle at 1e-12 by the tests above (one launch at every size, 1000
    steps at Ar = 0.4, Re = 8000).  Bar: 1e-5 U in velocity.  The largest
    error sits along the lid at Re = 8000, where the collision relaxes
    fastest (omega near 2)."""
    nx, ny = 500, int(round(500 * ar))
    out = {}
    for dtype in ("f64", "f32s"):
        c = lbm.Cavity(nx, ny, re=re, u_lid=U_LID, dtype=dtype)
        c.step(1000)
        out[dtype] = c.moments()
        c.close()
    (r0, u0, v0), (r1, u1, v1) = out["f64"], out["f32s"]
    du = max(np.abs(u1 - u0).max(), np.abs(v1 - v0).max())
    dr = np.abs(r1 - r0).max()
    print(f"{nx}x{ny} Re {re:g}: max|du|/U {du / U_LID:.3e}  max|drho| {dr:.3e}")
    assert du <= F32_UTOL
    assert dr <= 1e-5


@pytest.mark.parametrize("ny,steps", [(200, 400_000), (500, 1_600_000)])
def test_full_size_fp32_at_steady_state(lbm, ny, steps):
    """Steady cavities at full size (500 x 200 and 500 x 500, Re 1000) run
    from rest until FP64 has settled to its rounding floor (Eq. 6 below
    1e-10): the FP32 f - w field against the FP64 one (held to the oracle at
    1e-12).  Bar: 1e-5 U at steady state; measured 3.2e-6 U and 1.9e-6 U.
    During the slow final approach the two fields sit at slightly different
    points of the slowest decaying mode, so the gap passes through a larger
    value on the way (500 x 500: 2.1e-5 U at 600 k steps, where FP64's Eq. 6
    is still 3e-8) before it settles.  Rounded weights in the collision once
    left 1e-4 to 3e-4 U already at 200 k steps."""
    out = {}
    for dtype in ("f64", "f32s"):
        c = lbm.Cavity(500, ny, re=1000.0, u_lid=U_LID, dtype=dtype)
        c.step(steps)
        out[dtype] = (c.moments(), c.residual()[0])
        c.close()
    (r0, u0, v0), res64 = out["f64"]
    (r1, u1, v1), res32 = out["f32s"]
    du = max(np.abs(u1 - u0).max(), np.abs(v1 - v0).max())
    print(f"500x{ny} Re 1000, {steps} steps: Eq. 6 FP64 {res64:.2e} FP32 {res32:.2e}, "
          f"max|du|/U {du / U_LID:.3e}")
    assert res64 < 1e-10
    assert du <= F32_UTOL


def test_fp32_gap_at_the_paper_steady_criterion(lbm):
    """The FP32 f - w field against the FP64 one at the paper's own steady
    criterion (Sec. 2.2 (iii): Eq. 6 below 1e-6): 500 x 500, Re 1000, from
    rest, FP64 monitored every 100 steps until its Eq. 6 first drops below
    1e-6, FP32 run the same number of steps.  A KNOWN EXCEEDANCE of the
    1e-5 U bar: during the slow final approach the two fields sit at slightly
    different points of the slowest decaying mode (a smooth difference, not
    a checkerboard), which peaks near 2.1e-5 U around 600 k steps and
    settles at 2-3e-6 U once FP64 reaches its rounding floor
    (test_full_size_fp32_at_steady_state).  Measured 1.006e-5 U after
    370,100 steps (FP64 monitored every 100 steps); asserted <= 2e-5 U so
    that a regression shows."""
    c64 = lbm.Cavity(500, 500, re=1000.0, u_lid=U_LID, dtype="f64")
    steps = 0
    while True:
        c64.step(100)
        steps += 100
        res, at = c64.residual()
        assert at == steps
        if res < 1e-6:
            break
        assert steps < 2_000_000, "FP64 never reached Eq. 6 < 1e-6"
    c32 = lbm.Cavity(500, 500, re=1000.0, u_lid=U_LID, dtype="f32s")
    c32.step(steps)
    (r0, u0, v0), (r1, u1, v1) = c64.moments(), c32.moments()
    res32 = c32.residual()[0]
    c64.close()
    c32.close()
    du = max(np.abs(u1 - u0).max(), np.abs(v1 - v0).max())
    print(f"500x500 Re 1000: FP64 Eq. 6 < 1e-6 after {steps} steps (FP32 Eq. 6 {res32:.2e}); "
          f"max|du|/U {du / U_LID:.3e}")
    assert 300_000 <= steps <= 600_000
    assert du <= 2e-5 * U_LID


def test_mass_conservation_long_run(lbm):
    """20,000 steps of the 64 x 64, Re = 100 cavity.  The collision applies
    the weights exactly, so its rounding has no preferred sign: FP64 storage
    drifts by 4.4e-16 of the mass (measured; bound 1e-13).  FP32 f - w
    storage conserves mass only to its own rounding: at steady state the same
    roundings of the stored shifts repeat every step and add up (measured
    5.2e-10 after 20,000 steps; bound 1e-8)."""
    for dtype, tol in (("f64", 1e-13), ("f32s", 1e-8)):
        c = lbm.Cavity(64, 64, re=100.0, u_lid=U_LID, dtype=dtype)
        m0 = c.mass()
        assert abs(m0 - 64 * 64) <= 1e-12 * 64 * 64     # sum of the nine rounded w
        c.step(20000)
        drift = abs(c.mass() - m0) / m0
        print(f"{dtype}: relative mass drift after 20000 steps {drift:.3e}")
        assert drift <= tol, dtype
