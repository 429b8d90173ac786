"""FP32 forward and backward parity on the multi-tile paths of the tiled kernels.

At the benchmark's sizes each workgroup of a tiled kernel walks several tiles and carries its
accumulators (batch-norm partial sums, the stage-2 weight-gradient products, the stage-1
pointwise and depthwise weight-gradient sums) from one tile to the next, under the
XCD-contiguous schedule when the grid is a multiple of 8 and the plain grid stride otherwise.
Here the grid is bounded (stda_set_grid_cap) so that the small, oracle-checkable maps take the
same paths: 8 and 24 workgroups keep the XCD-contiguous schedule with several tiles per
workgroup, 13 the plain stride.  Inputs are screened for ReLU decisions within 1e-5 of their
kink, as in the other FP32 gradient tests.  Gates: rel-L2 < 1e-4 and max-rel <= 1e-3 per tensor.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TOL = 1e-4
CAPS = [8, 24, 13]
SHAPES = [(2, 40, 36), (1, 72, 88)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture()
def S():
    from paper_2307_09063_amd import stda
    yield stda
    stda.set_grid_cap(0)
    for dt in (stda.FP32, stda.BF16):
        for kind in stda.TUNE_KINDS:
            for b in range(4):
                stda.tune_set(kind, dt, b, 0)


def _fwd_bwd(S, x, w, r, g, recompute):
    B, _, H, W = x.shape
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN, recompute)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, wd, rd = U.dev(x), U.dev(w), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, S.FP32, S.TRAIN, recompute)
    dw = torch.full((net.param_count(),), float('nan'), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, S.FP32, recompute)
    torch.cuda.synchronize()
    return z.cpu().numpy(), rd.cpu().numpy(), dw.cpu().numpy(), dx.cpu().numpy()


def _check(S, shape, cap, recompute=0, seed=0):
    B, H, W = shape
    w, r = U.weights(), U.running()
    x, _ = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, 500 + H + W + seed)
    g = np.random.default_rng(B * H * W + cap).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    S.set_grid_cap(cap)
    assert S.get_grid_cap() == cap
    z, rd, dw, dx = _fwd_bwd(S, x, w, r, g, recompute)
    zr, rr, cache = net.forward(w, r, x, 'train')
    gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    U.assert_close(z, zr, TOL, what='z')
    U.assert_close(rd, rr, TOL, what='running')
    bad = U.grad_failures(dw, gr, TOL)
    assert not bad, bad
    U.assert_close(dx, dxr, TOL, what='dx')


@pytest.mark.parametrize('cap', CAPS)
@pytest.mark.parametrize('shape', SHAPES, ids=lambda s: 'x'.join(map(str, s)))
def test_capped_grid_fp32(S, shape, cap):
    _say('multi-tile fp32', shape, 'cap', cap)
    _check(S, shape, cap)


@pytest.mark.parametrize('v', [1, 2, 3])
def test_capped_grid_variants(S, v):
    """Every tiling variant of the stage-2 layers, their weight gradients and the stage-1 adjoint
    under an 8-workgroup grid."""
    _say('multi-tile variant', v)
    for kind in S.TUNE_KINDS:
        for b in range(4):
            S.tune_set(kind, S.FP32, b, v)
    _check(S, SHAPES[0], 8, seed=v)


def test_capped_grid_recompute(S):
    _say('multi-tile recompute')
    _check(S, SHAPES[1], 24, recompute=1)


def test_capped_grid_eval(S):
    """EVAL forward (running statistics; the ECA pooling sums still take the capped per-clip
    tiling) under each bound, against the oracle."""
    B, H, W = SHAPES[1]
    x, _ = U.maps(B, H, W, seed=3)
    w, r = U.weights(), U.running()
    segs = S.uniform_segments(B, H, W)
    _, wsb = S.workspace_size(segs, S.FP32, S.EVAL)
    ws = S.alloc_bytes(wsb)
    zr, _, _ = net.forward(w, r, x, 'eval')
    for cap in CAPS:
        _say('multi-tile eval', cap)
        S.set_grid_cap(cap)
        z = torch.empty((B, 1, H, W), device='cuda')
        S.forward(segs, U.dev(x), U.dev(w), U.dev(r.copy()), z, None, ws, S.FP32, S.EVAL)
        torch.cuda.synchronize()
        U.assert_close(z.cpu().numpy(), zr, TOL, what=f'z cap {cap}')
