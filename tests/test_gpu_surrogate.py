"""GPU tests of the BF16 MFMA surrogate kernels and driver against the FP64
reference (oracle/surrogate.py).

Inputs are rounded to bfloat16 first and the reference runs on exactly those
values, so the only differences are FP32 accumulation order (~1e-6) and the
rounding of each kernel's bf16 output (half an ulp: 2^-9 relative).
"""
import math

import numpy as np
import pytest

from oracle import surrogate as S

pytestmark = pytest.mark.gpu
BF_REL = 2.0 ** -8


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2211_05009_amd import lbm
    return torch, lbm


def bf16(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def f64(t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 12, 8, 32, 32), (1, 10, 7, 96, 96),
                                         (2, 8, 8, 64, 160), (3, 29, 17, 32, 32),
                                         (2, 23, 19, 32, 64), (1, 21, 13, 64, 128),
                                         (2, 9, 11, 128, 256), (8, 128, 128, 32, 32),
                                         (4, 128, 128, 32, 64), (4, 64, 64, 64, 128),
                                         (16, 64, 64, 64, 128), (2, 4, 128, 96, 32),
                                         (2, 6, 64, 192, 64), (2, 8, 32, 64, 128),
                                         (3, 8, 16, 128, 256), (2, 12, 16, 96, 32),
                                         (2, 16, 16, 128, 256), (3, 20, 16, 96, 32),
                                         (2, 9, 32, 64, 128)])
def test_conv_forward_dgrad_wgrad(env, n, h, w, ci, co):
    """Each pass against the FP64 reference on bf16-rounded inputs.  The
    shapes cover every kernel of the forward / input-gradient passes: the
    direct convolution from an LDS patch on 128-, 64-, 32- and 16-wide images
    (32- and 64-channel tiles, one and several 32-channel chunks) and the
    implicit
    GEMM elsewhere (256 x 32, 128 x 32, 128 x 64, 64 x 64, 64 x 128,
    128 x 128 tiles, chosen by channel count and pixel count), ragged pixel
    tails, and slices of wider tensors."""
    torch, lbm = env
    rng = np.random.default_rng(n * 1000 + ci + co)
    xs, xo = ci + 32, 32                       # input is a slice of a wider tensor
    xfull = bf16(torch, rng.normal(size=(n, h, w, xs)))
    wt = bf16(torch, rng.normal(0, 1 / math.sqrt(9 * ci), size=(9, ci, co)))
    bias = torch.tensor(rng.normal(size=co), dtype=torch.float32).cuda()
    x = f64(xfull)[..., xo:xo + ci]
    W = f64(wt)
    # forward into a slice, ReLU
    os_, oo = co + 64, 32
    out = bf16(torch, np.full((n, h, w, os_), 7.0))
    lbm.lbm_nn_conv3x3(0, n, h, w, ci, co, xfull, xs, xo, None, 0, 0, wt, bias, 1, out, os_, oo)
    torch.cuda.synchronize()
    ref = np.maximum(S.conv3x3(x, W, f64(bias)), 0)
    got = f64(out)
    assert np.all(got[..., :oo] == 7.0) and np.all(got[..., oo + co:] == 7.0)
    err = np.abs(got[..., oo:oo + co] - ref)
    assert np.all(err <= BF_REL * np.abs(ref) + 1e-4 * np.abs(ref).max())
    # dgrad: gradient w.r.t. the input, added to an existing slice
    gy = bf16(torch, rng.normal(size=(n, h, w, co)))
    gx0 = rng.normal(size=(n, h, w, ci))
    gx = bf16(torch, np.concatenate([np.zeros((n, h, w, 32)), gx0], axis=-1))
    gx0 = f64(gx)[..., 32:]
    lbm.lbm_nn_conv3x3(1, n, h, w, ci, co, gy, co, 0, None, 0, 0, wt, None, 0, gx, ci + 32, 32,
                       accumulate=True)
    torch.cuda.synchronize()
    rgx, rgw, rgb = S.conv3x3_backward(x, W, f64(gy))
    ref = gx0 + rgx
    got = f64(gx)[..., 32:]
    assert np.all(np.abs(got - ref) <= BF_REL * np.abs(ref) + 1e-4 * np.abs(ref).max())
    assert np.all(f64(gx)[..., :32] == 0)
    # wgrad: FP32 [9][ci][co], accumulated
    gw = torch.zeros((9, ci, co), dtype=torch.float32, device="cuda")
    lbm.lbm_nn_conv3x3(2, n, h, w, ci, co, xfull, xs, xo, gy, co, 0, None, None, 0, gw, 0, 0)
    gb = torch.zeros(co, dtype=torch.float32, device="cuda")
    lbm.lbm_nn_bias_grad(n * h * w, co, gy, co, 0, gb)
    torch.cuda.synchronize()
    assert np.max(np.abs(gw.cpu().numpy() - rgw)) <= 1e-5 * np.abs(rgw).max()
    assert np.max(np.abs(gb.cpu().numpy() - rgb)) <= 1e-5 * np.abs(rgb).max()


def test_pool_and_upsample(env):
    torch, lbm = env
    rng = np.random.default_rng(9)
    n, h, w, c = 2, 8, 6, 32
    xf = bf16(torch, rng.normal(size=(n, h, w, c + 32)))     # slice at offset 32
    y = torch.zeros((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    lbm.lbm_nn_pool2(0, n, h, w, c, xf, c + 32, 32, y, c, 0)
    torch.cuda.synchronize()
    ref = S.pool2(f64(xf)[..., 32:])
    assert np.all(np.abs(f64(y) - ref) <= BF_REL * np.abs(ref))
    gy = bf16(torch, rng.normal(size=(n, h // 2, w // 2, c)))
    gx = bf16(torch, np.ones((n, h, w, c + 32)))
    lbm.lbm_nn_pool2(1, n, h, w, c, gy, c, 0, gx, c + 32, 32, accumulate=True)
    torch.cuda.synchronize()
    ref = 1.0 + S.pool2_backward(f64(gy))
    assert np.all(np.abs(f64(gx)[..., 32:] - ref) <= BF_REL * np.abs(ref))
    # upsampling into a slice and its adjoint
    lo = bf16(torch, rng.normal(size=(n, h // 2, w // 2, c)))
    hi = torch.zeros((n, h, w, 2 * c), dtype=torch.bfloat16, device="cuda")
    lbm.lbm_nn_up2(0, n, h // 2, w // 2, c, lo, c, 0, hi, 2 * c, 0)
    torch.cuda.synchronize()
    assert np.array_equal(f64(hi)[..., :c], S.up2(f64(lo)))
    g = torch.zeros((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    gh = bf16(torch, rng.normal(size=(n, h, w, 2 * c)))
    lbm.lbm_nn_up2(1, n, h // 2, w // 2, c, gh, 2 * c, c, g, c, 0)
    torch.cuda.synchronize()
    ref = S.up2_backward(f64(gh)[..., c:])
    assert np.all(np.abs(f64(g) - ref) <= BF_REL * np.abs(ref) + 1e-6)


def _bf16_round(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


def test_network_forward_and_gradients(env):
    """Whole U-Net on the 256 x 128 canvas, two samples: forward output and
    per-layer gradients against the FP64 reference run with the same
    bf16-rounded weights.  BF16 activations are rounded after every layer
    (15 convolutions deep); measured <= 1e-2, bound 2e-2."""
    torch, lbm = env
    p = S.he_init(0)
    rng = np.random.default_rng(3)
    p = p + (p != 0) * rng.normal(0, 0.01, size=p.shape).astype(np.float32)
    sur = lbm.Surrogate(max_batch=4)
    assert sur.num_params == S.n_params()
    sur.set_params(p)
    re, ar = np.array([1200.0, 400.0]), np.array([1.2, 0.6])
    x = S.encode(re, ar)
    mask = x[..., 0]
    target = rng.normal(0, 0.5, size=(2, 256, 128, 3))
    pr = _bf16_round(torch, p).astype(np.float64)
    # bias stays FP32 in the library
    for (w, b), (wr, br) in zip(S.split_params(p.astype(np.float64)), S.split_params(pr)):
        br[...] = b
    xr = _bf16_round(torch, x).astype(np.float64)
    y_ref, st = S.forward(pr, xr)
    loss_ref, gy = S.loss_and_grad_output(y_ref, target, mask)
    g_ref = S.backward(pr, st, gy)
    out = torch.empty((2, 256, 128, 3), dtype=torch.float32, device="cuda")
    sur.forward(re, ar, out)
    y = out.cpu().numpy()
    ferr = np.linalg.norm(y - y_ref[..., :3]) / np.linalg.norm(y_ref[..., :3])
    tgt = torch.tensor(target, dtype=torch.float32).cuda()
    msk = torch.tensor(mask, dtype=torch.float32).cuda()
    loss = sur.train_step(re, ar, tgt, msk, lr=0.0, apply_update=False)
    _, g = sur.get_params(with_grads=True)
    offs = np.cumsum([0] + [9 * ci * co + co for ci, co, _ in S.CONVS])
    errs = []
    for li in range(15):
        a, b = g[offs[li]:offs[li + 1]], g_ref[offs[li]:offs[li + 1]]
        errs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"forward rel err {ferr:.3e}, loss {loss:.6f} vs {loss_ref:.6f}, "
          f"grad rel errs {np.round(errs, 4).tolist()}")
    assert ferr <= 2e-2
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref
    assert max(errs) <= 2e-2


def test_training_reduces_loss(env):
    torch, lbm = env
    sur = lbm.Surrogate(max_batch=4)
    sur.set_params(S.he_init(1))
    re, ar = np.array([300.0, 2000.0, 900.0, 1500.0]), np.array([0.5, 1.0, 1.5, 2.0])
    x = S.encode(re, ar)
    mask = torch.tensor(x[..., 0], dtype=torch.float32).cuda()
    yy = x[..., 2:3]
    target = np.concatenate([0.1 * yy, np.sin(3 * yy), x[..., 1:2] * yy], axis=-1)
    tgt = torch.tensor(target, dtype=torch.float32).cuda()
    losses = [sur.train_step(re, ar, tgt, mask, lr=1e-3) for _ in range(60)]
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    assert all(math.isfinite(v) for v in losses)


def test_training_is_bit_reproducible(env):
    """Every reduction of a training step (weight and bias gradients split
    over pixel chunks, the loss over blocks) adds its partials in a fixed
    order, so two networks trained from the same weights on the same data
    end with the same weights, bit for bit."""
    torch, lbm = env
    re, ar = np.array([300.0, 2000.0, 900.0, 1500.0]), np.array([0.5, 1.0, 1.5, 2.0])
    x = S.encode(re, ar)
    mask = torch.tensor(x[..., 0], dtype=torch.float32).cuda()
    yy = x[..., 2:3]
    tgt = torch.tensor(np.concatenate([0.1 * yy, np.sin(3 * yy), x[..., 1:2] * yy], axis=-1),
                       dtype=torch.float32).cuda()
    out = []
    for _ in range(2):
        sur = lbm.Surrogate(max_batch=4)
        sur.set_params(S.he_init(2))
        losses = [sur.train_step(re, ar, tgt, mask, lr=1e-3) for _ in range(8)]
        out.append((np.array(losses), sur.get_params()))
        sur.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_training_on_a_caller_stream_matches_the_own_stream(env):
    """The weight gradients run on a second stream of the handle, forked
    from and joined back into the stream the caller set: training on a
    caller's stream, with unrelated work queued on it, gives the same
    losses, weights and gradients, bit for bit, as on the handle's own."""
    torch, lbm = env
    re, ar = np.array([400.0, 2500.0, 1200.0]), np.array([0.6, 1.2, 1.8])
    x = S.encode(re, ar)
    mask = torch.tensor(x[..., 0], dtype=torch.float32).cuda()
    yy = x[..., 2:3]
    tgt = torch.tensor(np.concatenate([0.2 * yy, np.cos(2 * yy), x[..., 1:2]], axis=-1),
                       dtype=torch.float32).cuda()
    torch.cuda.synchronize()
    out = []
    for own in (True, False):
        sur = lbm.Surrogate(max_batch=3)
        sur.set_params(S.he_init(5))
        st = None
        if not own:
            st = torch.cuda.Stream()
            sur.set_stream(st)
        losses = []
        for _ in range(4):
            if st is not None:   # work of the caller's own ahead of each step
                with torch.cuda.stream(st):
                    big = torch.ones(1 << 22, device="cuda")
                    big.mul_(2.0).add_(1.0)
            losses.append(sur.train_step(re, ar, tgt, mask, lr=1e-3))
        params, grads = sur.get_params(with_grads=True)
        out.append((np.array(losses), params, grads))
        sur.close()
        torch.cuda.synchronize()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_warm_start_maps_prediction_onto_the_lattice(env):
    """lbm_sur_warm_start = bilinear map of the prediction onto site
    centres, mass renormalised, staggered momenta removed, f = f^eq
    (checked through the moments)."""
    torch, lbm = env
    sur = lbm.Surrogate(max_batch=1)
    sur.set_params(S.he_init(2))
    nx, ny, re = 200, 160, 900.0
    c = lbm.Cavity(nx, ny, re=re, u_lid=0.1, dtype="f64")
    sur.warm_start(c)
    out = torch.empty((1, 256, 128, 3), dtype=torch.float32, device="cuda")
    sur.forward([re], [ny / nx], out)
    p3 = out.cpu().numpy()[0].astype(np.float64)
    nyc = int(np.rint(128 * ny / nx))
    X = np.clip((np.arange(nx) + 0.5) * 128 / nx - 0.5, 0, 127)
    Y = np.clip((np.arange(ny) + 0.5) * 128 / nx - 0.5, 0, nyc - 1)
    x0 = np.minimum(np.floor(X).astype(int), 126)
    y0 = np.minimum(np.floor(Y).astype(int), nyc - 2)
    tx, ty = X - x0, Y - y0
    ref = ((1 - ty)[:, None, None] * (1 - tx)[None, :, None] * p3[y0][:, x0]
           + (1 - ty)[:, None, None] * tx[None, :, None] * p3[y0][:, x0 + 1]
           + ty[:, None, None] * (1 - tx)[None, :, None] * p3[y0 + 1][:, x0]
           + ty[:, None, None] * tx[None, :, None] * p3[y0 + 1][:, x0 + 1])
    rho = 1 + ref[..., 0] / 100
    rho *= nx * ny / math.fsum(rho.ravel().tolist())
    from oracle.d2q9 import destaggered_velocity
    vx, vy = destaggered_velocity(rho, 0.1 * ref[..., 1], 0.1 * ref[..., 2])
    r, ux, uy = c.moments()
    assert np.max(np.abs(r - rho)) <= 1e-12
    assert np.max(np.abs(ux - vx)) <= 1e-12
    assert np.max(np.abs(uy - vy)) <= 1e-12
    assert abs(c.mass() - nx * ny) <= 1e-9 * nx * ny


def test_init_params_he_normal_layout(env):
    torch, lbm = env
    from cavity_inputs import normal_draws
    sur = lbm.Surrogate(max_batch=1)
    z = normal_draws(sur.num_params, seed=7)
    lbm.lbm_sur_init_params(sur.s, z)
    p = sur.get_params().astype(np.float64)
    parts = S.split_params(p)
    zp = S.split_params(z.astype(np.float64))
    for li, ((w, b), (zw, _)) in enumerate(zip(parts, zp)):
        ci, co, _ = S.CONVS[li]
        cr = S.N_IN if li == 0 else ci
        orr = S.N_OUT if li == 14 else co
        sd = math.sqrt(2.0 / (9 * cr))
        assert np.allclose(w[:, :cr, :orr], sd * zw[:, :cr, :orr], rtol=1e-6, atol=0)
        assert np.all(w[:, cr:, :] == 0) and np.all(w[:, :, orr:] == 0) and np.all(b == 0)


def test_warm_start_converges_to_the_cold_steady_state_and_saves_steps(env):
    """Train a small surrogate on solver fields (200-wide lattices, 40 random
    cavities with Re 100-2500 plus the three test cavities, FP32 runs of up
    to 600 k steps: Eq. 6 < 1e-6 or the FP32 residual floor),
    then for the test cavities: (1) each warm start reaches Eq. 6 < 1e-6 in
    no more steps than the cold start, and in at least 15 % fewer steps in
    total (measured 27 %), (2) warm and cold starts converge to the same
    steady field (FP64, Eq. 6 < 1e-10: max |du| <= 1e-4 U).  The gain on
    unseen cavities is measured by bench.py's steady-sweep study."""
    import time
    torch, lbm = env
    from cavity_inputs import normal_draws
    from paper_2211_05009_amd import warmstart as W
    t0 = time.perf_counter()
    cases = [(200, 160, 700.0), (200, 120, 300.0), (200, 200, 2500.0)]
    re, ar = W.sample_cases(40, 0, re_range=(100.0, 2500.0))
    re = np.concatenate([re, [c[2] for c in cases]])
    nys = [int(round(200 * a)) for a in ar] + [c[1] for c in cases]
    n = len(re)
    b, st = W.solve_steady([200] * n, nys, re, 1e-6, 600_000)
    tgt = torch.empty((n, 256, 128, 3), dtype=torch.float32, device="cuda")
    msk = torch.empty((n, 256, 128), dtype=torch.float32, device="cuda")
    for k in range(n):
        b.canvas(k, tgt[k], msk[k])
    b.close()
    data = {"re": re, "ar": np.array(nys) / 200.0, "target": tgt, "mask": msk}
    t1 = time.perf_counter()
    sur = W.make_surrogate(normal_draws(lbm.Surrogate(1).num_params, seed=0))
    hist = W.train(sur, data, epochs=150)
    assert hist[-1] < 0.01 * hist[0]
    t2 = time.perf_counter()
    cold = W.time_to_steady(cases, 1e-6, 2_000_000, "single-cold")
    warm = W.time_to_steady(cases, 1e-6, 2_000_000, "single-warm", sur=sur)
    print(f"data {t1 - t0:.1f} s, training {t2 - t1:.1f} s, loss {hist[0]:.4f} -> "
          f"{hist[-1]:.6f}, steps cold {cold['steps']} warm {warm['steps']}")
    assert all(w <= c for w, c in zip(warm["steps"], cold["steps"]))
    assert sum(warm["steps"]) <= 0.85 * sum(cold["steps"])
    nx, ny, re1 = cases[1]
    a = lbm.Cavity(nx, ny, re=re1, u_lid=0.1, dtype="f64")
    w = lbm.Cavity(nx, ny, re=re1, u_lid=0.1, dtype="f64")
    sur.warm_start(w)
    for c in (a, w):
        for _ in range(3000):
            c.step(1000)
            if c.residual()[0] < 1e-10:
                break
        assert c.residual()[0] < 1e-10
    _, ua, va = a.moments()
    _, uw, vw = w.moments()
    print(f"converged fields: max |du| {max(np.max(np.abs(ua - uw)), np.max(np.abs(va - vw))):.3e}")
    assert max(np.max(np.abs(ua - uw)), np.max(np.abs(va - vw))) <= 1e-4 * 0.1
