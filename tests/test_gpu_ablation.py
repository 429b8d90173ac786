"""GPU-vs-oracle parity of the architecture readings selected by stda_set_arch: the decoder long
residual as DeConv3x3-s2-p1 with output padding 1, the logistic-sigmoid output, and a depthwise
stage-1 1x1 branch (Sec. IV-C leaves all three open).  Forward in EVAL and TRAIN (with the
running statistics), and the adjoint (every parameter gradient and dx), FP32, with and without
block recomputation, on shapes with ragged tiles.  Gate: rel-L2 <= 1e-4 per tensor, as for the
default network.  Inputs are screened for ReLU decisions near their kink as in the default parity
tests.

Depthwise 1x1 branch: batch norm makes BN(w x) independent of the size of a per-channel weight w
except through its epsilon, so in TRAIN mode dL/dw is the epsilon-sized remainder of a sum whose
terms cancel; its FP32 value carries the rounding of those terms, not of the remainder.  That
gradient is therefore gated where it is well conditioned: weights with w^2 var(x) below epsilon,
where the branch is nearly linear in w.  At the default weights every other tensor is gated."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TOL = 1e-4
ARCHS = [(3, 'identity', 'dense'), (4, 'sigmoid', 'dense'), (3, 'sigmoid', 'dense'), (4, 'identity', 'depthwise'),
         (3, 'sigmoid', 'depthwise')]
SHAPES = [(2, 16, 16), (2, 40, 36)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _select(param):
    from paper_2307_09063_amd import stda
    res_k, head, pw = param
    stda.set_arch(res_k, head, pw)
    net.set_arch(res_k, head, pw)
    yield stda, res_k, head, pw
    stda.set_arch()
    net.set_arch()


def _arch_id(a):
    return f'res{a[0]}-{a[1]}-{a[2]}'


@pytest.fixture(params=ARCHS, ids=_arch_id)
def arch(request):
    yield from _select(request.param)


@pytest.fixture(params=[a for a in ARCHS if a[2] == 'depthwise'], ids=_arch_id)
def arch_dw(request):
    yield from _select(request.param)


def _conditioned(w):
    """The same weights with every depthwise 1x1 weight scaled to |w| <= 3e-4."""
    w = w.copy()
    off = 0
    for name, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        if name.endswith('.s1.pw.w'):
            w[off:off + n] *= 3e-4 / np.abs(w[off:off + n]).max()
        off += n
    return w


@pytest.mark.parametrize('shape', SHAPES)
def test_forward(arch, shape):
    S, res_k, head, pw = arch
    B, H, W = shape
    _say('ablation forward', res_k, head, pw, shape)
    assert S.param_count() == net.param_count()
    x, _ = U.maps(B, H, W, seed=H * 7 + W + res_k)
    w, r = U.weights(), U.running()
    segs = S.uniform_segments(B, H, W)
    for mode in (S.EVAL, S.TRAIN):
        sv, wsb = S.workspace_size(segs, S.FP32, mode)
        saved = S.alloc_bytes(sv) if mode == S.TRAIN else None
        ws = S.alloc_bytes(wsb)
        rd = U.dev(r.copy())
        z = torch.empty((B, 1, H, W), device='cuda')
        S.forward(segs, U.dev(x), U.dev(w), rd, z, saved, ws, S.FP32, mode)
        torch.cuda.synchronize()
        zr, rr, _ = net.forward(w, r, x, 'train' if mode == S.TRAIN else 'eval')
        U.assert_close(z.cpu().numpy(), zr, TOL, what=f'z mode {mode}')
        U.assert_close(rd.cpu().numpy(), rr if mode == S.TRAIN else r, TOL, what=f'running mode {mode}')
        if head == 'sigmoid':
            zz = z.cpu().numpy()
            assert zz.min() > 0 and zz.max() < 1


@pytest.mark.parametrize('recompute', [0, 1])
@pytest.mark.parametrize('shape', SHAPES)
def test_backward(arch, shape, recompute):
    _backward(arch, shape, recompute, False)


@pytest.mark.parametrize('recompute', [0, 1])
@pytest.mark.parametrize('shape', SHAPES)
def test_backward_depthwise_conditioned(arch_dw, shape, recompute):
    _backward(arch_dw, shape, recompute, True)


def _backward(arch, shape, recompute, conditioned):
    S, res_k, head, pw = arch
    B, H, W = shape
    _say('ablation backward', res_k, head, pw, shape, recompute, conditioned)
    w, r = U.weights(), U.running()
    if conditioned:
        w = _conditioned(w)
    x, _ = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, H * 3 + W + res_k)
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN, recompute)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, wd = U.dev(x), U.dev(w)
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, U.dev(r.copy()), z, saved, ws, S.FP32, S.TRAIN, recompute)
    rng = np.random.default_rng(B * H * W + res_k)
    g = rng.standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    dw = torch.full((net.param_count(),), float('nan'), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, S.FP32, recompute)
    torch.cuda.synchronize()
    _, _, cache = net.forward(w, r, x, 'train')
    gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    skip = ('.s1.pw.w',) if pw == 'depthwise' and not conditioned else ()
    bad = U.grad_failures(dw.cpu().numpy(), gr, TOL, skip=skip)
    assert not bad, bad
    U.assert_close(dx.cpu().numpy(), dxr, TOL, what='dx')


def test_train_step_graph(arch):
    """A captured training step (forward, loss, backward, SGD) under the reading, replayed with
    eager work in between, against the same step run eagerly."""
    S, res_k, head, pw = arch
    _say('ablation graph', res_k, head, pw)
    B, H, W = 2, 32, 24
    x, y = U.maps(B, H, W, seed=5 + res_k)
    w0, r0 = U.weights(), U.running()
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
    n = S.param_count()

    def bufs():
        return dict(w=U.dev(w0.copy()), running=U.dev(r0.copy()), z=torch.empty((B, 1, H, W), device='cuda'),
                    loss=torch.zeros(1, dtype=torch.float64, device='cuda'), dz=torch.empty((B, 1, H, W), device='cuda'),
                    dw=torch.empty(n, device='cuda'), saved=S.alloc_bytes(sv), ws=S.alloc_bytes(wsb))

    xd, yd = U.dev(x), U.dev(y)
    e = bufs()
    eager = []
    for _ in range(3):
        S.forward(segs, xd, e['w'], e['running'], e['z'], e['saved'], e['ws'], S.FP32, S.TRAIN)
        S.mse_loss(segs, e['z'], yd, e['loss'], e['dz'], e['ws'])
        S.backward(segs, xd, e['dz'], e['w'], e['saved'], e['dw'], None, e['ws'], S.FP32)
        S.sgd_step(e['w'], e['dw'], 1e-2, 5e-4)
        torch.cuda.synchronize()
        eager.append(e['w'].cpu().numpy())
    gbuf = bufs()
    graph = S.TrainStepGraph(segs, xd, yd, gbuf['w'], gbuf['running'], gbuf['z'], gbuf['loss'], gbuf['dz'],
                             gbuf['dw'], gbuf['saved'], gbuf['ws'], lr=1e-2, weight_decay=5e-4)
    torch.cuda.synchronize()
    try:
        for k in range(3):
            graph.launch()
            torch.cuda.synchronize()
            junk = torch.randn(1 << 16, device='cuda').sum()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(gbuf['w'].cpu().numpy(), eager[k])
            del junk
    finally:
        graph.close()
