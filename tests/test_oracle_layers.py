"""Pins of the oracle's layer primitives against brute-force loops, library operators, adjoint
identities and closed forms.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import layers as L


def brute_conv(x, w, s, p, groups):
    B, C, H, W = x.shape
    Co, Cg, k, _ = w.shape
    Ho = (H + 2 * p - k) // s + 1
    Wo = (W + 2 * p - k) // s + 1
    og = Co // groups
    out = np.zeros((B, Co, Ho, Wo))
    for b in range(B):
        for o in range(Co):
            g = o // og
            for y in range(Ho):
                for xx in range(Wo):
                    acc = 0.0
                    for c in range(Cg):
                        for ky in range(k):
                            for kx in range(k):
                                iy, ix = s * y - p + ky, s * xx - p + kx
                                if 0 <= iy < H and 0 <= ix < W:
                                    acc += w[o, c, ky, kx] * x[b, g * Cg + c, iy, ix]
                    out[b, o, y, xx] = acc
    return out


def brute_deconv(x, w, s, p, groups):
    B, C, H, W = x.shape
    Ci, Og, k, _ = w.shape
    cg = C // groups
    Ho = (H - 1) * s - 2 * p + k
    Wo = (W - 1) * s - 2 * p + k
    out = np.zeros((B, Og * groups, Ho, Wo))
    for b in range(B):
        for c in range(C):
            g = c // cg
            for i in range(H):
                for j in range(W):
                    for o in range(Og):
                        for ky in range(k):
                            for kx in range(k):
                                y, xx = s * i - p + ky, s * j - p + kx
                                if 0 <= y < Ho and 0 <= xx < Wo:
                                    out[b, g * Og + o, y, xx] += x[b, c, i, j] * w[c, o, ky, kx]
    return out


CONV_CASES = [  # (C, Co, k, stride, pad, groups, H, W)
    (3, 4, 3, 1, 1, 1, 5, 6),
    (4, 8, 3, 2, 1, 1, 9, 8),
    (4, 8, 3, 2, 1, 1, 8, 6),
    (4, 4, 1, 1, 0, 1, 5, 7),
    (4, 4, 3, 1, 1, 4, 6, 5),
]
DECONV_CASES = [  # (C, Co, k, stride, pad, groups, H, W)
    (4, 2, 4, 2, 1, 1, 3, 4),
    (4, 4, 1, 1, 0, 1, 5, 3),
    (4, 4, 3, 1, 1, 4, 4, 5),
    (2, 3, 3, 2, 1, 1, 3, 3),
]


@pytest.mark.parametrize('case', CONV_CASES)
def test_conv_brute_and_library(case):
    C, Co, k, s, p, g, H, W = case
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, C, H, W))
    w = rng.standard_normal((Co, C // g, k, k))
    out = L.conv2d(x, w, s, p, g)
    np.testing.assert_allclose(out, brute_conv(x, w, s, p, g), rtol=1e-12, atol=1e-12)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(w), stride=s, padding=p, groups=g).numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize('case', DECONV_CASES)
def test_deconv_brute_and_library(case):
    C, Co, k, s, p, g, H, W = case
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, C, H, W))
    w = rng.standard_normal((C, Co // g, k, k))
    out = L.deconv2d(x, w, s, p, g)
    np.testing.assert_allclose(out, brute_deconv(x, w, s, p, g), rtol=1e-12, atol=1e-12)
    ref = F.conv_transpose2d(torch.from_numpy(x), torch.from_numpy(w), stride=s, padding=p,
                             groups=g).numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize('case', CONV_CASES)
def test_conv_adjoint_identities(case):
    """<conv(x), y> = <x, conv^T(y)> and, conv being linear in w, <conv(x; w), y> = <w, dW>."""
    C, Co, k, s, p, g, H, W = case
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, C, H, W))
    w = rng.standard_normal((Co, C // g, k, k))
    y = rng.standard_normal(L.conv2d(x, w, s, p, g).shape)
    lhs = (L.conv2d(x, w, s, p, g) * y).sum()
    dx = L.conv2d_grad_input(y, w, x.shape, s, p, g)
    dw = L.conv2d_grad_weight(x, y, w.shape, s, p, g)
    assert abs(lhs - (x * dx).sum()) <= 1e-12 * max(1.0, abs(lhs)) * 10
    assert abs(lhs - (w * dw).sum()) <= 1e-12 * max(1.0, abs(lhs)) * 10


@pytest.mark.parametrize('case', DECONV_CASES)
def test_deconv_adjoint_identities(case):
    C, Co, k, s, p, g, H, W = case
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, C, H, W))
    w = rng.standard_normal((C, Co // g, k, k))
    y = rng.standard_normal(L.deconv2d(x, w, s, p, g).shape)
    lhs = (L.deconv2d(x, w, s, p, g) * y).sum()
    dx = L.deconv2d_grad_input(y, w, x.shape, s, p, g)
    dw = L.deconv2d_grad_weight(x, y, w.shape, s, p, g)
    assert abs(lhs - (x * dx).sum()) <= 1e-11 * max(1.0, abs(lhs))
    assert abs(lhs - (w * dw).sum()) <= 1e-11 * max(1.0, abs(lhs))


def test_conv_deconv_same_weight_are_adjoint():
    """A stride-2 convolution and the transposed convolution with the same weight are adjoint
    once the transposed output is cropped to the convolution's input size."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 3, 8, 6))
    w = rng.standard_normal((5, 3, 3, 3))
    y = rng.standard_normal((1, 5, 4, 3))
    lhs = (L.conv2d(x, w, 2, 1) * y).sum()
    # conv weight [Co, C, k, k] read as a deconv weight [Cin=Co, Cout=C, k, k]; the uncropped
    # scatter has (4-1)*2 + 3 = 9 rows, of which rows 1..8 line up with the conv input
    full = L.deconv2d(y, w, 2, 0)
    t8 = full[:, :, 1:9, 1:7]
    assert abs(lhs - (x * t8).sum()) < 1e-12 * 100


def test_depthwise_deconv_is_flipped_conv():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 4, 5, 6))
    w = rng.standard_normal((4, 1, 3, 3))
    a = L.deconv2d(x, w, 1, 1, 4)
    b = L.conv2d(x, w[:, :, ::-1, ::-1].copy(), 1, 1, 4)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13)


def test_linearity():
    rng = np.random.default_rng(7)
    x1, x2 = rng.standard_normal((2, 2, 4, 8, 8))
    w = rng.standard_normal((4, 2, 4, 4))
    np.testing.assert_allclose(L.deconv2d(2 * x1 - 3 * x2, w, 2, 1),
                               2 * L.deconv2d(x1, w, 2, 1) - 3 * L.deconv2d(x2, w, 2, 1), atol=1e-12)


def test_bn_train_moments_and_library():
    rng = np.random.default_rng(8)
    x = 3.0 + 2.0 * rng.standard_normal((4, 5, 6, 7))
    gamma = rng.uniform(0.5, 2.0, 5)
    beta = rng.standard_normal(5)
    out, cache = L.bn_forward(x, gamma, beta, 'train')
    var = x.var(axis=(0, 2, 3))
    np.testing.assert_allclose(out.mean(axis=(0, 2, 3)), beta, atol=1e-12)
    np.testing.assert_allclose(out.var(axis=(0, 2, 3)), gamma ** 2 * var / (var + L.BN_EPS), rtol=1e-12)
    rm, rv = np.zeros(5), np.ones(5)
    nm, nv = L.bn_running_update(rm, rv, cache)
    trm, trv = torch.zeros(5, dtype=torch.float64), torch.ones(5, dtype=torch.float64)
    ref = F.batch_norm(torch.from_numpy(x), trm, trv, torch.from_numpy(gamma), torch.from_numpy(beta),
                       training=True, momentum=0.1, eps=1e-5).numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(nm, trm.numpy(), rtol=1e-12)
    np.testing.assert_allclose(nv, trv.numpy(), rtol=1e-12)


@pytest.mark.parametrize('mode', ['train', 'eval'])
def test_bn_backward_finite_difference(mode):
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 3, 4, 5))
    gamma = rng.uniform(0.5, 2.0, 3)
    beta = rng.standard_normal(3)
    rm, rv = rng.standard_normal(3), rng.uniform(0.5, 2, 3)
    y = rng.standard_normal(x.shape)
    f = lambda xx, gg, bb: (L.bn_forward(xx, gg, bb, mode, rm, rv)[0] * y).sum()
    _, cache = L.bn_forward(x, gamma, beta, mode, rm, rv)
    dx, dg, db = L.bn_backward(y, cache)
    h = 1e-6
    for arr, grad, idx in ((x, dx, (1, 2, 3, 4)), (x, dx, (0, 0, 0, 0)), (gamma, dg, (1,)), (beta, db, (2,))):
        ap, am = arr.copy(), arr.copy()
        ap[idx] += h
        am[idx] -= h
        args_p = [ap if arr is v else v for v in (x, gamma, beta)]
        args_m = [am if arr is v else v for v in (x, gamma, beta)]
        fd = (f(*args_p) - f(*args_m)) / (2 * h)
        assert abs(fd - grad[idx]) < 1e-7 * max(1, abs(fd))


def test_eca_constant_and_one_hot():
    rng = np.random.default_rng(10)
    w = rng.standard_normal(3)
    y = np.ones((1, 6, 4, 5)) * np.arange(1, 7)[None, :, None, None]
    _, cache = L.eca_forward(y, w)
    np.testing.assert_allclose(cache['g'][0], np.arange(1, 7), rtol=1e-15)
    # a one-hot GAP at channel 3 moves exactly channels 2, 3, 4 by sigma(w_k) - 1/2
    y = np.zeros((1, 6, 4, 4))
    y[0, 3] = 1.0
    _, cache = L.eca_forward(y, w)
    a = cache['a'][0]
    expect = np.full(6, 0.5)
    expect[2] = 1 / (1 + np.exp(-w[2]))      # s[2] = w2 g[3]
    expect[3] = 1 / (1 + np.exp(-w[1]))
    expect[4] = 1 / (1 + np.exp(-w[0]))      # s[4] = w0 g[3]
    np.testing.assert_allclose(a, expect, rtol=1e-14)


def test_eca_backward_finite_difference():
    rng = np.random.default_rng(11)
    y = rng.standard_normal((2, 5, 3, 4))
    w = rng.standard_normal(3)
    d = rng.standard_normal(y.shape)
    out, cache = L.eca_forward(y, w)
    dy, dw = L.eca_backward(d, w, cache)
    f = lambda yy, ww: (L.eca_forward(yy, ww)[0] * d).sum()
    h = 1e-6
    for idx in ((0, 0, 0, 0), (1, 4, 2, 3), (0, 2, 1, 1)):
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        assert abs((f(yp, w) - f(ym, w)) / (2 * h) - dy[idx]) < 1e-8
    for k in range(3):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        assert abs((f(y, wp) - f(y, wm)) / (2 * h) - dw[k]) < 1e-8


def test_deconv_output_padding_and_adjoint():
    """DeConv3x3-s2-p1 with output padding 1 (the alternative decoder residual): equals the
    library's ConvTranspose, doubles the map, and is the adjoint of Conv3x3-s2-p1 with the same
    weight (an inner-product identity)."""
    rng = np.random.default_rng(12)
    x = rng.standard_normal((2, 4, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    out = L.deconv2d(x, w, stride=2, pad=1, out_pad=1)
    assert out.shape == (2, 3, 10, 12)
    ref = torch.nn.functional.conv_transpose2d(torch.from_numpy(x), torch.from_numpy(w), stride=2, padding=1,
                                               output_padding=1).numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    yb = rng.standard_normal((2, 3, 10, 12))
    # <deconv(x), y> = <x, conv(y)> with conv weights [Cout=4, Cin=3] = w itself
    lhs = (out * yb).sum()
    rhs = (x * L.conv2d(yb, w, stride=2, pad=1)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    dout = rng.standard_normal(out.shape)
    gx = L.deconv2d_grad_input(dout, w, x.shape, stride=2, pad=1, out_pad=1)
    gw = L.deconv2d_grad_weight(x, dout, w.shape, stride=2, pad=1, out_pad=1)
    np.testing.assert_allclose(gx, L.conv2d(dout, w, stride=2, pad=1), rtol=1e-12, atol=1e-12)
    eps = 1e-6
    e = np.zeros_like(w)
    e[1, 2, 0, 2] = eps
    fd = ((L.deconv2d(x, w + e, 2, 1, out_pad=1) - L.deconv2d(x, w - e, 2, 1, out_pad=1)) * dout).sum() / (2 * eps)
    assert abs(fd - gw[1, 2, 0, 2]) <= 1e-7 * max(1.0, abs(fd))
