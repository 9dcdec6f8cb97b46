"""FP64 reference of the warm-start surrogate network (test infrastructure
only): forward and backward of every layer and of the whole U-Net, in NumPy.

The network is the one the library documents (include/lbm.h, "Learned warm
start"): NHWC tensors, 3 x 3 zero-padded convolutions with weights
[9][ci][co] (tap t = 3 dy + dx reads the input at offset (dy - 1, dx - 1)),
bias and ReLU, 2 x 2 average pooling, nearest 2x upsampling, skip
concatenation (upsampled channels first, then the skip), a linear head, and a
masked mean-squared-error loss.  Parameters are one flat vector: for each
convolution, weights then bias.  The canvas size is a parameter so the
finite-difference pins can run on a small one.
"""
from __future__ import annotations

import numpy as np

# (ci, co, relu) of the 15 convolutions, with the first layer's 5 inputs and
# the head's 3 outputs padded to 32 channels.
CONVS = [(32, 32, 1), (32, 32, 1), (32, 64, 1), (64, 64, 1), (64, 128, 1), (128, 128, 1),
         (128, 256, 1), (256, 256, 1), (384, 128, 1), (128, 128, 1), (192, 64, 1),
         (64, 64, 1), (96, 32, 1), (32, 32, 1), (32, 32, 0)]
N_IN, N_OUT = 5, 3


def n_params():
    return sum(9 * ci * co + co for ci, co, _ in CONVS)


def split_params(p):
    """Flat vector -> list of (w [9, ci, co], b [co]) views."""
    out, k = [], 0
    for ci, co, _ in CONVS:
        w = p[k:k + 9 * ci * co].reshape(9, ci, co)
        k += 9 * ci * co
        b = p[k:k + co]
        k += co
        out.append((w, b))
    return out


def he_init(seed=0):
    """He-normal weights (std sqrt(2 / (9 ci_real))), zero biases, zero
    padding entries; FP32 like the library's master weights."""
    rng = np.random.default_rng(seed)
    p = np.zeros(n_params(), dtype=np.float64)
    for li, (w, b) in enumerate(split_params(p)):
        ci, co, _ = CONVS[li]
        ci_real = N_IN if li == 0 else ci
        co_real = N_OUT if li == len(CONVS) - 1 else co
        w[:, :ci_real, :co_real] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci_real)),
                                              size=(9, ci_real, co_real))
    return p.astype(np.float32)


# ------------------------------------------------------------------ layers
def conv3x3(x, w, b):
    """y[n, i, j, o] = sum_{t, c} x[n, i + dy - 1, j + dx - 1, c] w[t, c, o] + b[o]."""
    n, h, wd, ci = x.shape
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, h, wd, w.shape[2]))
    for t in range(9):
        dy, dx = divmod(t, 3)
        y += xp[:, dy:dy + h, dx:dx + wd, :] @ w[t]
    return y + b


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 w.r.t. x, w, b given the output gradient gy."""
    n, h, wd, ci = x.shape
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    g2 = gy.reshape(-1, gy.shape[-1])
    for t in range(9):
        dy, dx = divmod(t, 3)
        gw[t] = xp[:, dy:dy + h, dx:dx + wd, :].reshape(-1, ci).T @ g2
        gxp[:, dy:dy + h, dx:dx + wd, :] += gy @ w[t].T
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(0, 1, 2))


def pool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(gy):
    n, h, w, c = gy.shape
    return gy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


# ------------------------------------------------------------------ network
def encode(re, ar, H=256, W=128):
    """Input canvas [n, H, W, 32]: mask (rows y < round(128 Ar) -- scaled to
    H/2 for smaller canvases), (x + 1/2)/128, (y + 1/2)/128, Re/3000, Ar/2."""
    re = np.asarray(re, dtype=np.float64)
    ar = np.asarray(ar, dtype=np.float64)
    n = len(re)
    x = np.zeros((n, H, W, 32))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for b in range(n):
        ny = int(np.rint(W * ar[b]))
        x[b, :, :, 0] = (yy < ny)
        x[b, :, :, 1] = (xx + 0.5) / W
        x[b, :, :, 2] = (yy + 0.5) / W
        x[b, :, :, 3] = re[b] / 3000.0
        x[b, :, :, 4] = ar[b] / 2.0
    return x


def forward(params, x):
    """Returns the head output [n, H, W, 32] and the saved activations."""
    P = split_params(np.asarray(params, dtype=np.float64))
    relu = lambda v: np.maximum(v, 0.0)   # noqa: E731
    s = {"x": x}
    s["a0"] = relu(conv3x3(x, *P[0]))
    s["s0"] = relu(conv3x3(s["a0"], *P[1]))
    s["p0"] = pool2(s["s0"])
    s["a1"] = relu(conv3x3(s["p0"], *P[2]))
    s["s1"] = relu(conv3x3(s["a1"], *P[3]))
    s["p1"] = pool2(s["s1"])
    s["a2"] = relu(conv3x3(s["p1"], *P[4]))
    s["s2"] = relu(conv3x3(s["a2"], *P[5]))
    s["p2"] = pool2(s["s2"])
    s["b0"] = relu(conv3x3(s["p2"], *P[6]))
    s["b1"] = relu(conv3x3(s["b0"], *P[7]))
    s["c2"] = np.concatenate([up2(s["b1"]), s["s2"]], axis=-1)
    s["d2a"] = relu(conv3x3(s["c2"], *P[8]))
    s["d2b"] = relu(conv3x3(s["d2a"], *P[9]))
    s["c1"] = np.concatenate([up2(s["d2b"]), s["s1"]], axis=-1)
    s["d1a"] = relu(conv3x3(s["c1"], *P[10]))
    s["d1b"] = relu(conv3x3(s["d1a"], *P[11]))
    s["c0"] = np.concatenate([up2(s["d1b"]), s["s0"]], axis=-1)
    s["d0a"] = relu(conv3x3(s["c0"], *P[12]))
    s["d0b"] = relu(conv3x3(s["d0a"], *P[13]))
    s["y"] = conv3x3(s["d0b"], *P[14])
    return s["y"], s


def loss_and_grad_output(y, target, mask):
    """Masked MSE over the first three channels: sum mask (y - t)^2 /
    sum mask; returns (loss, dL/dy)."""
    cnt = mask.sum()
    d = (y[..., :N_OUT] - target) * mask[..., None]
    loss = float((d * (y[..., :N_OUT] - target)).sum() / cnt)
    gy = np.zeros_like(y)
    gy[..., :N_OUT] = 2.0 * d / cnt
    return loss, gy


def backward(params, s, gy):
    """Gradient of the loss w.r.t. the flat parameter vector."""
    P = split_params(np.asarray(params, dtype=np.float64))
    g = np.zeros(n_params())
    G = split_params(g)

    def conv_b(li, xin, yout, gout, relu=True):
        if relu:
            gout = gout * (yout > 0)
        gx, gw, gb = conv3x3_backward(xin, P[li][0], gout)
        G[li][0][...] = gw
        G[li][1][...] = gb
        return gx

    g_d0b = conv_b(14, s["d0b"], s["y"], gy, relu=False)
    g_d0a = conv_b(13, s["d0a"], s["d0b"], g_d0b)
    g_c0 = conv_b(12, s["c0"], s["d0a"], g_d0a)
    c_up = s["d1b"].shape[-1]
    g_d1b = up2_backward(g_c0[..., :c_up])
    g_s0 = g_c0[..., c_up:]
    g_d1a = conv_b(11, s["d1a"], s["d1b"], g_d1b)
    g_c1 = conv_b(10, s["c1"], s["d1a"], g_d1a)
    c_up = s["d2b"].shape[-1]
    g_d2b = up2_backward(g_c1[..., :c_up])
    g_s1 = g_c1[..., c_up:]
    g_d2a = conv_b(9, s["d2a"], s["d2b"], g_d2b)
    g_c2 = conv_b(8, s["c2"], s["d2a"], g_d2a)
    c_up = s["b1"].shape[-1]
    g_b1 = up2_backward(g_c2[..., :c_up])
    g_s2 = g_c2[..., c_up:]
    g_b0 = conv_b(7, s["b0"], s["b1"], g_b1)
    g_p2 = conv_b(6, s["p2"], s["b0"], g_b0)
    g_s2 = g_s2 + pool2_backward(g_p2)
    g_a2 = conv_b(5, s["a2"], s["s2"], g_s2)
    g_p1 = conv_b(4, s["p1"], s["a2"], g_a2)
    g_s1 = g_s1 + pool2_backward(g_p1)
    g_a1 = conv_b(3, s["a1"], s["s1"], g_s1)
    g_p0 = conv_b(2, s["p0"], s["a1"], g_a1)
    g_s0 = g_s0 + pool2_backward(g_p0)
    g_a0 = conv_b(1, s["a0"], s["s0"], g_s0)
    conv_b(0, s["x"], s["a0"], g_a0)
    return g


def loss_and_grad(params, re, ar, target, mask, H=256, W=128):
    x = encode(re, ar, H, W)
    y, s = forward(params, x)
    loss, gy = loss_and_grad_output(y, target, mask)
    return loss, backward(params, s, gy), y
