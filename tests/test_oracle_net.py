"""Pins of the oracle network: parameter count, zero input, an independent torch.nn.functional
re-expression (forward, running statistics, autograd gradient), FP64 central finite
differences, the loss closed form, and the EVAL-mode re-parameterisation identity.  CPU only."""
import os

import numpy as np
import pytest
import torch

from oracle import layers as L
from oracle import net
from paper_2307_09063_amd import inputs
from tests import torch_ref


def _setup(B=2, H=16, W=16, seed=0):
    specs = net.param_specs()
    w = inputs.make_weights(specs).astype(np.float64)
    r = inputs.make_running([c for _, c in net.bn_specs()]).astype(np.float64)
    rng = np.random.default_rng(seed)
    x = rng.random((B, 3, H, W))
    y = rng.random((B, 1, H, W))
    return w, r, x, y


def _torch_params(w, r):
    P = {k: torch.tensor(v, requires_grad=True) for k, v in net.unflatten(w).items()}
    R = {k: (torch.tensor(v[0]), torch.tensor(v[1])) for k, v in net.unflatten_running(r).items()}
    return P, R


def test_param_count_matches_paper_scale():
    # 0.14 M parameters (Table 7); this reading gives 137,469
    assert net.param_count() == 137469
    assert net.running_count() == 2 * 592


@pytest.mark.parametrize('mode', ['train', 'eval'])
def test_zero_input_gives_head_bias(mode):
    w, r, _, _ = _setup()
    P = net.unflatten(w.copy())
    P['head.conv.b'][0] = 0.37
    x = np.zeros((2, 3, 16, 16))
    z, _, _ = net.forward(P, r, x, mode)
    np.testing.assert_array_equal(z, np.full_like(z, 0.37))


@pytest.mark.parametrize('mode', ['train', 'eval'])
def test_forward_matches_torch_functional(mode):
    w, r, x, _ = _setup(B=2, H=16, W=12)
    rng = np.random.default_rng(5)
    w = w + 0.1 * rng.standard_normal(w.shape)          # move BN affine off (1, 0)
    r = r + 0.2 * rng.random(r.shape)
    z, newr, _ = net.forward(w, r, x, mode)
    P, R = _torch_params(w, r)
    zt, newR = torch_ref.forward(P, R, torch.from_numpy(x), train=(mode == 'train'))
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-11, atol=1e-12)
    rt = net.flatten_running({k: (v[0].numpy(), v[1].numpy()) for k, v in newR.items()})
    np.testing.assert_allclose(newr, rt, rtol=1e-12, atol=1e-14)


def test_backward_matches_torch_autograd():
    w, r, x, y = _setup(B=2, H=16, W=12)
    rng = np.random.default_rng(6)
    w = w + 0.1 * rng.standard_normal(w.shape)
    loss, g, dx, _, _ = net.loss_and_grad(w, r, x, y, want_dx=True)
    P, R = _torch_params(w, r)
    xt = torch.tensor(x, requires_grad=True)
    zt, _ = torch_ref.forward(P, R, xt, train=True)
    lt = ((zt - torch.from_numpy(y)) ** 2).mean()
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12 * abs(loss)
    gt = net.flatten({k: v.grad.numpy() for k, v in P.items()})
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-14 * np.abs(gt).max())
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-9, atol=1e-14 * np.abs(dx).max())


def _kinks(w, r, x):
    """Signs of every ReLU input, to reject finite-difference steps that cross a kink."""
    _, _, cache = net.forward(w, r, x, 'train')
    a = cache['acts']
    return np.concatenate([(a[k] > 0).ravel() for k in sorted(a) if k.endswith('.x1') or k.endswith('.m')]
                          + [(a['s0'] > 0).ravel()])


def _fd_coordinates(args):
    """Central differences of the loss along single coordinates (worker of the FD test): for each
    index, (True, None) if a step flips a ReLU, else (False, relative error against g)."""
    w, r, x, y, g, idx, h = args
    f = lambda ww: net.mse_loss(net.forward(ww, r, x, 'train')[0], y)[0]
    base = _kinks(w, r, x)
    out = []
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        if not (np.array_equal(base, _kinks(w + e, r, x)) and np.array_equal(base, _kinks(w - e, r, x))):
            out.append((True, None))
            continue
        fd = (f(w + e) - f(w - e)) / (2 * h)
        out.append((False, abs(fd - g[i]) / max(abs(fd), 1e-3 * np.abs(g).max())))
    return out


def test_gradient_central_finite_differences():
    """One 3 x 16 x 16 clip (B = 2 for non-degenerate batch statistics), h = 1e-6: a random
    direction over all parameters plus 2,000 sampled coordinates and one in every parameter tensor
    (BN, ECA and the head bias included); steps that flip a ReLU are counted and skipped.  The
    coordinates are spread over worker processes."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    w, r, x, y = _setup(B=2, H=16, W=16, seed=33)
    loss, g, _, _, _ = net.loss_and_grad(w, r, x, y)
    f = lambda ww: net.mse_loss(net.forward(ww, r, x, 'train')[0], y)[0]
    h = 1e-6
    rng = np.random.default_rng(33)
    v = rng.standard_normal(w.shape)
    v /= np.linalg.norm(v)
    base = _kinks(w, r, x)
    assert np.array_equal(base, _kinks(w + h * v, r, x)) and np.array_equal(base, _kinks(w - h * v, r, x))
    fd = (f(w + h * v) - f(w - h * v)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-6 * abs(fd)
    idx = rng.choice(w.size, 2000, replace=False)
    offs, o = [], 0
    for _, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        offs.append(o + n // 2)
        o += n
    idx = np.unique(np.concatenate([idx, offs]))
    workers = max(1, min(8, os.cpu_count() or 1))
    chunks = [(w, r, x, y, g, c, h) for c in np.array_split(idx, 4 * workers)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context('spawn')) as ex:
        res = [t for part in ex.map(_fd_coordinates, chunks) for t in part]
    flips = sum(1 for fl, _ in res if fl)
    errs = [e for fl, e in res if not fl]
    assert len(idx) >= 2000
    assert flips < len(idx) // 10
    assert max(errs) < 1e-5


def test_loss_closed_form():
    rng = np.random.default_rng(1)
    z = rng.random((2, 1, 4, 4))
    loss, dz = net.mse_loss(z, z)
    assert loss == 0.0 and not dz.any()
    y = rng.random(z.shape)
    loss, dz = net.mse_loss(z, y)
    assert abs(loss - ((z - y) ** 2).sum() / 32) < 1e-15
    np.testing.assert_allclose(dz, (z - y) / 16, rtol=1e-15)


def test_sgd_step():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.1, 0.2, -0.3])
    np.testing.assert_allclose(net.sgd_step(w, g, 0.01, 5e-4),
                               [1 - 0.01 * (0.1 + 5e-4), -2 - 0.01 * (0.2 - 1e-3), 0.5 - 0.01 * (-0.3 + 2.5e-4)])


def test_eval_stage1_reparameterisation():
    """In EVAL mode the three branches of stage 1 fold into one depthwise 3x3 plus a pointwise
    1x1 plus a bias (the MobileOne-style inference form); the folded form must reproduce the sum."""
    rng = np.random.default_rng(12)
    c = 8
    x = rng.standard_normal((2, c, 7, 6))
    wp = rng.standard_normal((c, c, 1, 1))
    wd = rng.standard_normal((c, 1, 3, 3))
    bns = [(rng.uniform(0.5, 2, c), rng.standard_normal(c), rng.standard_normal(c), rng.uniform(0.5, 2, c))
           for _ in range(3)]
    outs = [L.bn_forward(t, g, b, 'eval', m, v)[0] for t, (g, b, m, v) in
            zip((L.conv2d(x, wp), L.conv2d(x, wd, 1, 1, c), x), bns)]
    u = sum(outs)
    sc = [g / np.sqrt(v + L.BN_EPS) for g, b, m, v in bns]
    bias = sum(b - m * s for (g, b, m, v), s in zip(bns, sc))
    wp2 = wp * sc[0][:, None, None, None]
    wp2[np.arange(c), np.arange(c), 0, 0] += sc[2]
    wd2 = wd * sc[1][:, None, None, None]
    folded = L.conv2d(x, wp2) + L.conv2d(x, wd2, 1, 1, c) + bias[None, :, None, None]
    np.testing.assert_allclose(u, folded, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------- architecture ablations
ARCHS = [(3, 'identity', 'dense'), (4, 'sigmoid', 'dense'), (3, 'sigmoid', 'dense'), (4, 'identity', 'depthwise'),
         (3, 'sigmoid', 'depthwise')]


@pytest.fixture()
def arch():
    yield
    net.set_arch()


@pytest.mark.parametrize('res_k,head,pw', ARCHS)
def test_ablation_param_count(arch, res_k, head, pw):
    net.set_arch(res_k, head, pw)
    # a 3 x 3 decoder residual has 7 of 16 taps fewer: (64*32 + 32*16) * 7 weights fewer; a
    # depthwise 1x1 branch keeps C of the C^2 weights of each of the four blocks
    fewer = (res_k == 3) * (64 * 32 + 32 * 16) * 7 + (pw == 'depthwise') * sum(c * c - c for c in (16, 32, 64, 32))
    assert net.param_count() == 137469 - fewer


@pytest.mark.parametrize('res_k,head,pw', ARCHS)
def test_ablation_forward_and_gradient_match_torch(arch, res_k, head, pw):
    net.set_arch(res_k, head, pw)
    w, r, x, y = _setup(B=2, H=16, W=12)
    rng = np.random.default_rng(7)
    w = w + 0.1 * rng.standard_normal(w.shape)
    z, _, _ = net.forward(w, r, x, 'train')
    P, R = _torch_params(w, r)
    xt = torch.tensor(x, requires_grad=True)
    zt, _ = torch_ref.forward(P, R, xt, train=True, res_k=res_k, head=head, pw=pw)
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-11, atol=1e-12)
    loss, g, dx, _, _ = net.loss_and_grad(w, r, x, y, want_dx=True)
    lt = ((zt - torch.from_numpy(y)) ** 2).mean()
    lt.backward()
    gt = net.flatten({k: v.grad.numpy() for k, v in P.items()})
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-14 * np.abs(gt).max())
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-9, atol=1e-14 * np.abs(dx).max())


@pytest.mark.parametrize('res_k,head,pw', ARCHS)
def test_ablation_directional_finite_difference(arch, res_k, head, pw):
    net.set_arch(res_k, head, pw)
    w, r, x, y = _setup(B=2, H=16, W=16, seed=34)
    _, g, _, _, _ = net.loss_and_grad(w, r, x, y)
    f = lambda ww: net.mse_loss(net.forward(ww, r, x, 'train')[0], y)[0]
    h = 1e-6
    v = np.random.default_rng(34).standard_normal(w.shape)
    v /= np.linalg.norm(v)
    base = _kinks(w, r, x)
    assert np.array_equal(base, _kinks(w + h * v, r, x)) and np.array_equal(base, _kinks(w - h * v, r, x))
    fd = (f(w + h * v) - f(w - h * v)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-6 * abs(fd)


def test_depthwise_pointwise_is_the_diagonal_of_the_dense_one(arch):
    """A depthwise 1x1 branch is the dense one with a diagonal weight: the same output in both
    modes, and its gradient is the diagonal of the dense gradient."""
    net.set_arch(pw='depthwise')
    w_dw, r, x, y = _setup(B=2, H=16, W=12, seed=5)
    specs_dw = net.param_specs()
    net.set_arch()
    specs = net.param_specs()
    blocks = ('enc0', 'enc1', 'dec0', 'dec1')
    # build the dense vector: the diagonal from the depthwise weights, zeros elsewhere
    parts, off_dw, src = [], 0, {}
    for name, shape, _ in specs_dw:
        n = int(np.prod(shape))
        src[name] = w_dw[off_dw:off_dw + n].reshape(shape)
        off_dw += n
    for name, shape, _ in specs:
        if name.endswith('.s1.pw.w'):
            c = shape[0]
            d = np.zeros(shape)
            d[np.arange(c), np.arange(c), 0, 0] = src[name][:, 0, 0, 0]
            parts.append(d.ravel())
        else:
            parts.append(src[name].ravel())
    w_dense = np.concatenate(parts)
    for mode in ('train', 'eval'):
        z_dense, r_dense, _ = net.forward(w_dense, r, x, mode)
        net.set_arch(pw='depthwise')
        z_dw, r_dw, _ = net.forward(w_dw, r, x, mode)
        net.set_arch()
        np.testing.assert_allclose(z_dw, z_dense, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(r_dw, r_dense, rtol=1e-13, atol=1e-13)
    _, g_dense, dx_dense, _, _ = net.loss_and_grad(w_dense, r, x, y, want_dx=True)
    net.set_arch(pw='depthwise')
    _, g_dw, dx_dw, _, _ = net.loss_and_grad(w_dw, r, x, y, want_dx=True)
    np.testing.assert_allclose(dx_dw, dx_dense, rtol=1e-12, atol=1e-15 * np.abs(dx_dense).max())
    off, off_dw = 0, 0
    for (name, shape, _), (_, shape_dw, _) in zip(specs, specs_dw):
        n, n_dw = int(np.prod(shape)), int(np.prod(shape_dw))
        gd, gw = g_dense[off:off + n].reshape(shape), g_dw[off_dw:off_dw + n_dw].reshape(shape_dw)
        if name.endswith('.s1.pw.w'):
            c = shape[0]
            gd = gd[np.arange(c), np.arange(c), 0, 0].reshape(shape_dw)
        np.testing.assert_allclose(gw, gd, rtol=1e-10, atol=1e-13 * np.abs(g_dense).max(), err_msg=name)
        off, off_dw = off + n, off_dw + n_dw
    assert set(blocks) == {k.split('.')[0] for k, s, _ in specs if k.endswith('.s1.pw.w')}
