"""GPU-vs-oracle parity of the FP32 path, through the C ABI: forward (EVAL and TRAIN), running
statistics, loss, backward (every parameter gradient and dx), SGD, the autograd wrapper,
uneven segments, edge shapes, determinism.  Gate: rel-L2 <= 1e-4 per tensor (FP32).

Inputs are screened so that no ReLU pre-activation lies within a relative 1e-5 of its kink:
there FP32 and FP64 may legitimately take different decisions, and one flipped decision moves a
batch-norm shift gradient (a sum of n terms of random sign) by about 1/sqrt(n)."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TOL = 1e-4
SHAPES = [(2, 16, 16), (3, 32, 24), (1, 64, 64), (2, 8, 12), (2, 40, 36)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


def _run_forward(S, x, w, r, mode, dtype=0):
    B, _, H, W = x.shape
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, dtype, mode)
    saved = S.alloc_bytes(sv) if mode == S.TRAIN else None
    ws = S.alloc_bytes(wsb)
    xd, wd, rd = U.dev(x), U.dev(w), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, dtype, mode)
    torch.cuda.synchronize()
    return z.cpu().numpy(), rd.cpu().numpy(), (segs, xd, wd, saved, ws)


@pytest.mark.parametrize('shape', SHAPES)
def test_forward_eval(S, shape):
    B, H, W = shape
    _say('forward eval', shape)
    x, _ = U.maps(B, H, W, seed=H * 7 + W)
    w, r = U.weights(), U.running()
    z, r_out, _ = _run_forward(S, x, w, r, S.EVAL)
    zr, _, _ = net.forward(w, r, x, 'eval')
    assert U.rel_l2(z, zr) < TOL
    np.testing.assert_array_equal(r_out, r)      # EVAL leaves the running buffer alone


@pytest.mark.parametrize('shape', SHAPES)
def test_forward_train_and_running(S, shape):
    B, H, W = shape
    _say('forward train', shape)
    x, _ = U.maps(B, H, W, seed=H * 5 + W)
    w, r = U.weights(), U.running()
    z, r_out, _ = _run_forward(S, x, w, r, S.TRAIN)
    zr, rr, _ = net.forward(w, r, x, 'train')
    assert U.rel_l2(z, zr) < TOL
    assert U.rel_l2(r_out, rr) < TOL


@pytest.mark.parametrize('shape', SHAPES)
def test_backward(S, shape):
    B, H, W = shape
    _say('backward', shape)
    w, r = U.weights(), U.running()
    x, y = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, H * 3 + W)
    z, _, (segs, xd, wd, saved, ws) = _run_forward(S, x, w, r, S.TRAIN)
    # loss and dz on the GPU
    zd = U.dev(z)
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    dz = torch.empty_like(zd)
    S.mse_loss(segs, zd, U.dev(y), loss, dz, ws)
    torch.cuda.synchronize()
    lr_, dzr = net.mse_loss(z.astype(np.float64), y)
    assert abs(loss.item() - lr_) <= 1e-12 * abs(lr_) + 1e-300
    assert U.rel_l2(dz.cpu().numpy(), dzr) < 1e-6
    # the adjoint itself, on the same dz for both sides
    rng = np.random.default_rng(B * H * W)
    g = rng.standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    dw = torch.full((net.param_count(),), float('nan'), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws)
    torch.cuda.synchronize()
    _, _, cache = net.forward(w, r, x, 'train')
    gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    errs = U.per_tensor_errors(dw.cpu().numpy(), gr)
    bad = {k: v for k, v in errs.items() if not v < TOL}
    assert not bad, bad
    assert U.rel_l2(dx.cpu().numpy(), dxr) < TOL


def test_sgd(S):
    _say('sgd')
    rng = np.random.default_rng(0)
    w = rng.standard_normal(net.param_count()).astype(np.float32)
    g = rng.standard_normal(net.param_count()).astype(np.float32)
    wd, gd = U.dev(w), U.dev(g)
    wb = torch.empty(w.size, dtype=torch.int16, device='cuda')
    S.sgd_step(wd, gd, 1e-3, 5e-4, wb)
    torch.cuda.synchronize()
    ref = net.sgd_step(w, g, 1e-3, 5e-4)
    assert np.abs(wd.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref).max()
    # the BF16 copy is the round-to-nearest-even of the new master
    bits = wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    back = bits.view(np.float32)
    assert np.all(np.abs(back - wd.cpu().numpy()) <= np.abs(wd.cpu().numpy()) * 2.0 ** -8)


def test_autograd_function(S):
    _say('autograd')
    B, H, W = 2, 16, 16
    w, r = U.weights(), U.running()
    x, y = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, 11)
    xd = U.dev(x).requires_grad_(True)
    wd = U.dev(w).requires_grad_(True)
    rd = U.dev(r.copy())
    z = S.stda(xd, wd, rd)
    loss = ((z - U.dev(y)) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    lr_, gr, dxr, zr, _ = net.loss_and_grad(w, r, x, y, want_dx=True)
    assert U.rel_l2(z.detach().cpu().numpy(), zr) < TOL
    errs = U.per_tensor_errors(wd.grad.cpu().numpy(), gr)
    assert max(errs.values()) < TOL, errs
    assert U.rel_l2(xd.grad.cpu().numpy(), dxr) < TOL


def test_uneven_segments(S):
    """Two map sizes in one call: each segment has its own batch statistics, the loss is the
    sum of the per-segment means, and dw is the sum of the per-segment gradients."""
    _say('uneven segments')
    parts = [(2, 16, 16), (3, 32, 24)]
    w, r = U.weights(), U.running()
    xs, ys = zip(*(U.maps(n, H, W, seed=n * H) for n, H, W in parts))
    segs = S.packed_segments(parts)
    xd = U.dev(np.concatenate([a.ravel() for a in xs]))
    yd = U.dev(np.concatenate([a.ravel() for a in ys]))
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    rd = U.dev(r.copy())
    z = torch.empty(yd.shape, device='cuda')
    wd = U.dev(w)
    S.forward(segs, xd, wd, rd, z, saved, ws, S.FP32, S.TRAIN)
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    dz = torch.empty_like(z)
    S.mse_loss(segs, z, yd, loss, dz, ws)
    dw = torch.empty(net.param_count(), device='cuda')
    S.backward(segs, xd, dz, wd, saved, dw, None, ws)
    torch.cuda.synchronize()
    zc = z.cpu().numpy()
    off, lsum, gsum, rcur = 0, 0.0, 0.0, r.astype(np.float64)
    for (n, H, W), x, y in zip(parts, xs, ys):
        zr, rcur, cache = net.forward(w, rcur, x, 'train')
        assert U.rel_l2(zc[off:off + n * H * W], zr.ravel()) < TOL
        l, d = net.mse_loss(zr, y)
        g, _ = net.backward(d, cache)
        lsum += l
        gsum = gsum + g
        off += n * H * W
    assert abs(loss.item() - lsum) < 1e-5 * lsum
    assert U.rel_l2(rd.cpu().numpy(), rcur) < TOL
    errs = U.per_tensor_errors(dw.cpu().numpy(), gsum)
    assert max(errs.values()) < TOL, errs


def test_deterministic(S):
    _say('determinism')
    B, H, W = 2, 32, 24
    x, y = U.maps(B, H, W, seed=5)
    w, r = U.weights(), U.running()
    outs = []
    for _ in range(2):
        z, _, (segs, xd, wd, saved, ws) = _run_forward(S, x, w, r, S.TRAIN)
        dw = torch.empty(net.param_count(), device='cuda')
        S.backward(segs, xd, U.dev(z - y), wd, saved, dw, None, ws)
        torch.cuda.synchronize()
        outs.append((z, dw.cpu().numpy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
