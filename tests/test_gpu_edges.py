"""Edge cases of the network path on the GPU against the FP64 oracle, through the C ABI.

* Maximum map extent on one axis (4096 x 8 and 8 x 4096; H and W may reach 4096): forward in EVAL
  and TRAIN (z and the running statistics) at the FP32 gate, and the adjoint's dx.  Parameter
  gradients are gated on the smaller shapes of the other parity tests: at 32k pixels some ReLU
  pre-activation always lies within FP32 rounding of its kink, and one decision taken differently
  moves a batch-norm shift gradient (a sum over all pixels) by about 1/sqrt(n), while dx changes
  only next to that pixel.
* Zero input, the method's degenerate case: every batch-norm input has zero variance, ECA sees a
  zero average, and with the initial affine (gamma 1, beta 0) and running statistics (0, 1) the
  output is exactly the output-module bias, in TRAIN and EVAL, FP32 and BF16; the adjoint stays
  finite and matches the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from paper_2307_09063_amd import inputs
from tests import gpu_util as U

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


def _forward(S, x, w, r, mode, dtype=0):
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


@pytest.mark.parametrize('shape', [(1, 4096, 8), (1, 8, 4096)], ids=['4096x8', '8x4096'])
def test_maximum_extent(S, shape):
    B, H, W = shape
    _say('maximum extent', shape)
    x, _ = U.maps(B, H, W, seed=H + 3 * W)
    w, r = U.weights(), U.running()
    z, r_out, _ = _forward(S, x, w, r, S.EVAL)
    zr, _, _ = net.forward(w, r, x, 'eval')
    U.assert_close(z, zr, TOL, what='z')
    z, r_out, (segs, xd, wd, saved, ws) = _forward(S, x, w, r, S.TRAIN)
    zr, rr, cache = net.forward(w, r, x, 'train')
    U.assert_close(z, zr, TOL, what='z')
    U.assert_close(r_out, rr, TOL, what='running')
    g = np.random.default_rng(H * W).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    dw = torch.empty(net.param_count(), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws)
    torch.cuda.synchronize()
    _, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    U.assert_close(dx.cpu().numpy(), dxr, TOL, what='dx')
    assert np.isfinite(dw.cpu().numpy()).all()


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
@pytest.mark.parametrize('mode', ['eval', 'train'])
def test_zero_input_gives_head_bias(S, mode, dtype):
    _say('zero input', mode, dtype)
    B, H, W = 2, 24, 16
    w = inputs.make_weights(net.param_specs(), 1234)
    off = {n: o for n, o in zip([s[0] for s in net.param_specs()],
                                np.cumsum([0] + [int(np.prod(s[1])) for s in net.param_specs()]))}
    w[off['head.conv.b']] = 0.37
    r = inputs.make_running([c for _, c in net.bn_specs()])
    x = np.zeros((B, 3, H, W), dtype=np.float32)
    m = S.TRAIN if mode == 'train' else S.EVAL
    z, _, state = _forward(S, x, w, r, m, dtype)
    np.testing.assert_array_equal(z, np.full_like(z, np.float32(0.37)))
    if mode == 'train':
        segs, xd, wd, saved, ws = state
        g = np.random.default_rng(1).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
        dw = torch.full((net.param_count(),), float('nan'), device='cuda')
        dx = torch.empty_like(xd)
        S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, dtype)
        torch.cuda.synchronize()
        got = dw.cpu().numpy()
        assert np.isfinite(got).all() and np.isfinite(dx.cpu().numpy()).all()
        if dtype == 0:
            _, _, cache = net.forward(w, r, x, 'train')
            gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
            bad = U.grad_failures(got, gr, TOL)
            assert not bad, bad
            U.assert_close(dx.cpu().numpy(), dxr, TOL, what='dx')
