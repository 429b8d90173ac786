"""BF16 on the multi-tile paths of the tiled kernels.

At the BF16 training workload's size every workgroup of the tiled kernels walks several tiles,
fetching the next tile's input into LDS while it processes the current one (stage-1 forward,
backward statistics and fused adjoint, input and output modules).  At the sizes the oracle and
the BF16 storage model handle in seconds a workgroup gets one tile, so here the grid is bounded
(stda_set_grid_cap): 8 workgroups keep the XCD-contiguous schedule, 13 the plain stride, both
with several tiles per workgroup, including workgroups whose last tile has no successor.

EVAL: every tile is computed as with the full grid, so z is bit-identical to the uncapped run.
TRAIN: the batch-norm partials merge in another order, and BF16 storage turns those FP32
rounding differences into occasional full BF16 steps (see the format envelope in
tests/test_gpu_bf16.py), so the capped step meets the BF16 training gates of that file: z
against the FP64 oracle, and z, every parameter-gradient tensor, the whole gradient and dx
against the BF16 storage model within the envelope of its jittered runs."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U
from tests.test_gpu_bf16 import TOL, _envelope

pytestmark = pytest.mark.gpu

CAPS = [8, 13]
SHAPES = [(2, 40, 36), (1, 72, 88)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture()
def S():
    from paper_2307_09063_amd import stda
    yield stda
    stda.set_grid_cap(0)


def _eval(S, x, w, r, cap):
    B, _, H, W = x.shape
    segs = S.uniform_segments(B, H, W)
    _, wsb = S.workspace_size(segs, S.BF16, S.EVAL)
    S.set_grid_cap(cap)
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, U.dev(x), U.dev(w), U.dev(r.copy()), z, None, S.alloc_bytes(wsb), S.BF16, S.EVAL)
    torch.cuda.synchronize()
    return z.cpu().numpy()


@pytest.mark.parametrize('shape', SHAPES, ids=lambda s: 'x'.join(map(str, s)))
def test_bf16_capped_eval_bitwise(S, shape):
    B, H, W = shape
    x, _ = U.maps(B, H, W, seed=11)
    w, r = U.weights(), U.running()
    z0 = _eval(S, x, w, r, 0)
    for cap in CAPS:
        _say('bf16 multi-tile eval', shape, 'cap', cap)
        np.testing.assert_array_equal(_eval(S, x, w, r, cap), z0)


@pytest.mark.parametrize('rec', [0, 1])
@pytest.mark.parametrize('cap', CAPS)
@pytest.mark.parametrize('shape', SHAPES, ids=lambda s: 'x'.join(map(str, s)))
def test_bf16_capped_train_within_envelope(S, shape, cap, rec):
    B, H, W = shape
    _say('bf16 multi-tile train', shape, 'cap', cap, 'recompute', rec)
    x, _ = U.maps(B, H, W, seed=11)
    w, r = U.weights(), U.running()
    g = np.random.default_rng(B * H * W).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.BF16, S.TRAIN, rec)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, wd, rd = U.dev(x), U.dev(w), U.dev(r.copy())
    S.set_grid_cap(cap)
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, S.BF16, S.TRAIN, rec)
    dw = torch.full((net.param_count(),), float('nan'), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, S.BF16, rec)
    torch.cuda.synchronize()
    zc, dwc, dxc = z.cpu().numpy(), dw.cpu().numpy(), dx.cpu().numpy()
    zr, _, _ = net.forward(w, r, x, 'train')
    env, (zm, _, gm, dxm) = _envelope(w, r, x, g.astype(np.float64), (1, 2, 3))
    em = U.per_tensor_errors(dwc, gm)
    _say(f'  z vs oracle {U.rel_l2(zc, zr):.2e}; vs storage model z {U.rel_l2(zc, zm):.2e} (envelope {env["z"]:.2e}), '
         f'grad {U.rel_l2(dwc, gm):.2e} ({env["flat"]:.2e}), dx {U.rel_l2(dxc, dxm):.2e} ({env["dx"]:.2e})')
    assert np.isfinite(dwc).all()
    assert U.rel_l2(zc, zr) < TOL
    assert U.rel_l2(zc, zm) <= 3 * env['z']
    bad = {k: (v, env[k]) for k, v in em.items() if v > TOL + 2 * env[k]}
    assert not bad, bad
    assert U.rel_l2(dwc, gm) <= TOL + 2 * env['flat']
    assert U.rel_l2(dxc, dxm) <= TOL + 2 * env['dx']
