"""GPU D3Q19 lid-driven box (lbm3d_*) against the D3Q19 oracle
(oracle/d3q19.py): populations and moments after hundreds of steps, every
tile shape bit-identical, monitors, symmetry."""
import math

import numpy as np
import pytest

from oracle import d3q19 as D

pytestmark = pytest.mark.gpu
U = 0.1


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2211_05009_amd import lbm as m
    return m


def _pair(lbm, shape, re, dtype, seed):
    nx, ny, nz = shape
    ref = D.Cube(nx, ny, nz, re=re, u_lid=U)
    c = lbm.Cube(nx, ny, nz, re=re, u_lid=U, dtype=dtype)
    if seed is not None:
        rng = np.random.default_rng(seed)
        ref.set_state(ref.f + rng.uniform(-4e-3, 4e-3, ref.f.shape))
        c.set_populations(ref.f)
    return ref, c


@pytest.mark.parametrize("shape,re,steps,seed", [((67, 9, 5), 60.0, 300, None),
                                                 ((3, 3, 3), 5.0, 250, 1),
                                                 ((20, 17, 11), 100.0, 200, 2),
                                                 ((2, 66, 4), 20.0, 150, 3)])
def test_fp64_parity_and_shapes(lbm, shape, re, steps, seed):
    ref, c = _pair(lbm, shape, re, "f64", seed)
    f0 = ref.f.copy()
    ref.step(steps)
    r0, u0, v0, w0 = ref.moments()
    fs0 = ref.post_collision()
    outs = []
    for v in range(c.get_option(lbm.LBM_OPT_NUM_VARIANTS)):
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        c.set_populations(f0)
        c.step(steps)
        r, u, vv, w = c.moments()
        assert np.abs(r - r0).max() <= 1e-12
        assert max(np.abs(u - u0).max(), np.abs(vv - v0).max(), np.abs(w - w0).max()) <= 1e-12 * U
        outs.append(c.get_populations())
        assert np.abs(outs[-1] - fs0).max() <= 1e-12
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    c.close()


def test_fp32_parity(lbm):
    """FP32 f - w storage in every tile shape against the FP64 oracle."""
    ref, c = _pair(lbm, (33, 20, 7), 200.0, "f32s", 4)
    f0 = ref.f.copy()
    ref.step(300)
    _, u0, v0, w0 = ref.moments()
    for v in range(c.get_option(lbm.LBM_OPT_NUM_VARIANTS)):
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        c.set_populations(f0)
        c.step(300)
        _, u, vv, w = c.moments()
        d = max(np.abs(u - u0).max(), np.abs(vv - v0).max(), np.abs(w - w0).max())
        assert d <= 1e-5 * U, (v, d)
    c.close()


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_graph_direct_and_monitors(lbm, dtype):
    """Graph replay and direct launches agree bit for bit; mass and the
    Eq. 6 residual equal their definitions on the library's own moments."""
    nx, ny, nz = 40, 30, 12
    a = lbm.Cube(nx, ny, nz, re=400.0, u_lid=U, dtype=dtype)
    b = lbm.Cube(nx, ny, nz, re=400.0, u_lid=U, dtype=dtype)
    b.set_option(lbm.LBM_OPT_USE_GRAPH, 0)
    a.step(1900)
    b.step(1900)
    assert np.array_equal(a.get_populations(), b.get_populations())
    _, u1, v1, w1 = a.moments()
    a.step(100)
    b.step(37)
    b.step(63)
    assert a.residual() == b.residual()
    r2, u2, v2, w2 = a.moments()
    num = math.fsum(((u2 - u1) ** 2 + (v2 - v1) ** 2 + (w2 - w1) ** 2).ravel().tolist())
    den = math.fsum((u1 ** 2 + v1 ** 2 + w1 ** 2).ravel().tolist())
    res, at = a.residual()
    assert at == 2000 and abs(res - math.sqrt(num / den)) <= 1e-12 * res
    assert abs(a.mass() - math.fsum(r2.ravel().tolist())) <= 1e-12 * nx * ny * nz
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32s"])
def test_two_step_shapes_agree_bitwise(lbm, dtype):
    """The two-step shapes against a one-step one, bit for bit, on a box
    ragged for every tile: 137 steps (a graph or direct 100-step chunk, then
    18 two-step launches and one single step), and the Eq. 6 monitor."""
    nx, ny, nz = 37, 23, 13
    rng = np.random.default_rng(31)
    f0 = D.W[:, None, None, None] + rng.uniform(-4e-3, 4e-3, (19, nz, ny, nx))
    c = lbm.Cube(nx, ny, nz, re=200.0, u_lid=U, dtype=dtype)
    c.set_option(lbm.LBM_OPT_STEP_VARIANT, 0)
    c.set_populations(f0)
    c.step(137)
    ref, ref_res = c.get_populations(), c.residual()
    for v in range(3, c.get_option(lbm.LBM_OPT_NUM_VARIANTS)):
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        assert c.get_option(lbm.LBM_OPT_STEPS_PER_LAUNCH) == 2
        for graph in (1, 0):
            c.set_option(lbm.LBM_OPT_USE_GRAPH, graph)
            c.set_populations(f0)
            c.step(137)
            assert np.array_equal(c.get_populations(), ref), (v, graph)
            assert c.residual() == ref_res
    c.close()


def test_fp64_z_marching_beyond_buffer_range(lbm):
    """FP64 z-marching shapes read and write states below 2^31 bytes as raw
    buffers and larger ones through pointers: a 128 x 130 x 864 box (2.19 GB
    of populations) takes the pointer path; 101 steps from rest (a graph
    chunk and a single step) equal a one-step shape's bit for bit."""
    nx, ny, nz = 128, 130, 864
    assert 19 * nx * ny * nz * 8 > 2 ** 31
    out = []
    for v in (1, 4):
        c = lbm.Cube(nx, ny, nz, re=400.0, u_lid=U, dtype="f64")
        c.set_option(lbm.LBM_OPT_STEP_VARIANT, v)
        c.step(101)
        out.append((c.get_populations(), c.residual()))
        c.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_mirror_symmetry_in_z(lbm):
    c = lbm.Cube(24, 20, 9, re=300.0, u_lid=U, dtype="f64")
    c.step(1500)
    r, u, v, w = c.moments()
    assert np.abs(u - u[::-1]).max() <= 1e-14 and np.abs(w + w[::-1]).max() <= 1e-14
    c.close()


def test_autotune_keeps_the_state(lbm):
    c = lbm.Cube(64, 48, 32, re=500.0, u_lid=U, dtype="f32s")
    c.step(200)
    f = c.get_populations()
    best, ms = c.autotune(2)
    assert 0 <= best < c.get_option(lbm.LBM_OPT_NUM_VARIANTS) and ms > 0
    assert c.steps_done() == 200
    assert np.array_equal(c.get_populations(), f)
    c.close()


def test_errors(lbm):
    for args in ((1, 4, 4, 100.0, U, "f64"), (4, 4, 4, -1.0, U, "f64"), (4, 4, 4, 100.0, 0.7, "f64"),
                 (4, 4, 4, 100.0, U, 9)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm3d_create(*args)
        assert e.value.code == lbm.LBM_EINVAL


@pytest.mark.parametrize("dtype,n,variant", [("f32s", 256, 2), ("f64", 192, 1),
                                             ("f32s", 256, 3), ("f32s", 256, 6),
                                             ("f64", 192, 4)])
def test_full_size_box_light_cone(lbm, dtype, n, variant):
    """The boxes the benchmark times (256^3 FP32, 192^3 FP64, in a one-step
    shape, a 3-D two-step tile and a z-marching one) from a random state: one 100-step graph chunk,
    then ten steps of direct launches, checked against the oracle on 42^3
    windows cut from the
    GPU's state.  In ten steps information moves at most ten sites, so sites
    more than eleven sites from a cut face are exact.  Windows: the lid
    corner at x = z = 0, the opposite bottom corner, the centre.  Bars: FP64
    populations <= 1e-12, FP32 velocity <= 1e-5 U."""
    steps, w = 10, 42
    m = steps + 1
    tau = D.relaxation_time(n, 1000.0, U)
    c = lbm.Cube(n, n, n, re=1000.0, u_lid=U, dtype=dtype)
    c.set_option(lbm.LBM_OPT_STEP_VARIANT, variant)
    rng = np.random.default_rng(29)
    f0 = rng.uniform(-4e-3, 4e-3, (19, n, n, n))
    f0 += D.W[:, None, None, None]
    c.set_populations(f0)
    del f0
    c.step(100)
    f_start = c.get_populations()
    c.set_option(lbm.LBM_OPT_USE_GRAPH, 0)
    c.step(steps)
    f_end = c.get_populations()
    c.close()
    worst = 0.0
    for x0, y0, z0 in ((0, n - w, 0), (n - w, 0, n - w), ((n - w) // 2,) * 3):
        o = D.Cube(w, w, w, tau=tau, u_lid=U)
        o.set_state(D.stream(f_start[:, z0:z0 + w, y0:y0 + w, x0:x0 + w], U), t=1)
        o.step(steps - 1)
        ref = o.post_collision()
        lo = [0 if a == 0 else m for a in (z0, y0, x0)]
        hi = [w if a + w == n else w - m for a in (z0, y0, x0)]
        sl = (slice(None), slice(lo[0], hi[0]), slice(lo[1], hi[1]), slice(lo[2], hi[2]))
        got = f_end[:, z0:z0 + w, y0:y0 + w, x0:x0 + w][sl]
        want = ref[sl]
        if dtype == "f64":
            d = np.abs(got - want).max()
            assert d <= 1e-12, (x0, y0, z0, d)
        else:
            _, ug, vg, wg = D.macroscopic(got)
            _, uw, vw, ww = D.macroscopic(want)
            d = max(np.abs(ug - uw).max(), np.abs(vg - vw).max(), np.abs(wg - ww).max())
            assert d <= 1e-5 * U, (x0, y0, z0, d)
        worst = max(worst, d)
    print(f"{n}^3 {dtype} shape {variant}: worst window difference {worst:.3e}")

