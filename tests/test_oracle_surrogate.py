"""Pins of the FP64 surrogate reference (oracle/surrogate.py): each layer
against brute force or the definition of its adjoint, the whole network's
gradient against central finite differences."""
import numpy as np
import pytest

from oracle import surrogate as S


def test_parameter_count_and_layout():
    assert S.n_params() == 1_964_448
    p = S.he_init(0)
    parts = S.split_params(p)
    assert len(parts) == 15
    w0, b0 = parts[0]
    assert np.all(w0[:, S.N_IN:, :] == 0)          # padded input channels
    wl, bl = parts[-1]
    assert np.all(wl[:, :, S.N_OUT:] == 0)         # padded output channels
    assert np.all(p[S.n_params() - 32:] == 0)      # head bias


def test_conv3x3_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(9, 3, 2))
    b = rng.normal(size=2)
    y = S.conv3x3(x, w, b)
    ref = np.zeros_like(y)
    for n in range(2):
        for i in range(4):
            for j in range(5):
                for o in range(2):
                    s = b[o]
                    for dy in range(3):
                        for dx in range(3):
                            ii, jj = i + dy - 1, j + dx - 1
                            if 0 <= ii < 4 and 0 <= jj < 5:
                                s += x[n, ii, jj, :] @ w[3 * dy + dx, :, o]
                    ref[n, i, j, o] = s
    assert np.allclose(y, ref, atol=1e-12, rtol=0)


def test_conv3x3_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 3, 4, 2))
    w = rng.normal(size=(9, 2, 3))
    b = rng.normal(size=3)
    gy = rng.normal(size=(1, 3, 4, 3))
    gx, gw, gb = S.conv3x3_backward(x, w, gy)
    f = lambda x_, w_, b_: float((S.conv3x3(x_, w_, b_) * gy).sum())   # noqa: E731
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 3, 1), (0, 1, 2, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0), (4, 1, 2), (8, 1, 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - gw[idx]) < 1e-7
    assert np.allclose(gb, gy.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_adjoints():
    """<A x, y> = <x, A^T y> for the pooling and upsampling pairs, and pooling
    undoes upsampling."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 6, 4, 3))
    y = rng.normal(size=(2, 3, 2, 3))
    assert np.isclose((S.pool2(x) * y).sum(), (x * S.pool2_backward(y)).sum(), rtol=1e-13)
    assert np.isclose((S.up2(y) * x).sum(), (y * S.up2_backward(x)).sum(), rtol=1e-13)
    assert np.allclose(S.pool2(S.up2(y)), y, atol=1e-15)


def test_network_gradient_finite_differences():
    """Whole U-Net on a 16 x 8 canvas, FP64: backward pass against central
    differences of the loss for parameters in every layer."""
    H, W = 16, 8
    rng = np.random.default_rng(4)
    p = S.he_init(5).astype(np.float64)
    p += rng.normal(0.0, 0.01, size=p.shape)      # non-zero biases, no exact ties
    re, ar = [1500.0, 600.0], [1.6, 0.8]
    target = rng.normal(size=(2, H, W, 3))
    mask = S.encode(re, ar, H, W)[..., 0]
    loss, g, _ = S.loss_and_grad(p, re, ar, target, mask, H, W)
    offs = np.cumsum([0] + [9 * ci * co + co for ci, co, _ in S.CONVS])
    h = 1e-6
    for li in range(15):
        for k in range(2):
            i = int(rng.integers(offs[li], offs[li + 1]))
            if g[i] == 0 and li in (0, 14):
                continue                          # padding entries
            e = np.zeros_like(p)
            e[i] = h
            lp = S.loss_and_grad(p + e, re, ar, target, mask, H, W)[0]
            lm = S.loss_and_grad(p - e, re, ar, target, mask, H, W)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (li, i, fd, g[i])


def test_flop_table_matches_the_network():
    """The throughput report counts the convolutions the library runs: its
    shape table gives the same channel list and parameter count as the
    reference network."""
    from paper_2211_05009_amd import warmstart as W
    assert [(ci, co) for _, ci, co in W.CONV_SHAPES] == [(ci, co) for ci, co, _ in S.CONVS]
    assert sum(9 * ci * co + co for _, ci, co in W.CONV_SHAPES) == S.n_params()
    # levels: 2 convs per encoder level, the bottleneck pair, 2 per decoder level + head
    assert [l for l, _, _ in W.CONV_SHAPES] == [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0]
    fwd = W.conv_flops()
    assert fwd == sum(2 * 9 * ci * co * (256 >> l) * (128 >> l) for l, ci, co in W.CONV_SHAPES)
    assert W.conv_flops(backward=True) == 2 * fwd - 2 * 9 * 32 * 32 * 256 * 128
