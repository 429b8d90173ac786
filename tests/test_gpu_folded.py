"""Folded-weight EVAL inference (stda_eval_fold + stda_forward_folded) against the FP64 oracle's
EVAL forward, through the C ABI: batch norm folded into the weights (Sec. IV-C), stage 2 as one
launch.  FP32 gate as the unfolded forward: rel-L2 <= 1e-4 and max |a - b| / max |b| <= 1e-3;
BF16 within 2e-2.  Also: the captured folded graph replays to the eager result bit for bit, the
sigmoid output reading."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TOL = 1e-4
SHAPES = [(1, 128, 64), (1, 64, 64), (2, 40, 36), (3, 32, 24), (2, 8, 12), (4, 256, 128)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


def _folded(S, x, w, r, dtype=0):
    B, _, H, W = x.shape
    segs = S.uniform_segments(B, H, W)
    fb = S.alloc_bytes(S.eval_fold_size(dtype))
    wd, rd = U.dev(w), U.dev(r)
    S.eval_fold(wd, rd, fb, dtype)
    _, wsb = S.workspace_size(segs, dtype, S.EVAL)
    ws = S.alloc_bytes(wsb)
    xd = U.dev(x)
    z = torch.full((B, 1, H, W), float('nan'), device='cuda')
    S.forward_folded(segs, xd, fb, z, ws, dtype)
    torch.cuda.synchronize()
    return z, (segs, xd, fb, ws)


@pytest.mark.parametrize('shape', SHAPES)
def test_folded_eval_fp32(S, shape):
    B, H, W = shape
    _say('folded eval', shape)
    x, _ = U.maps(B, H, W, seed=H * 11 + W)
    w, r = U.weights(), U.running()
    z, _ = _folded(S, x, w, r)
    zr, _, _ = net.forward(w, r, x, 'eval')
    U.assert_close(z.cpu().numpy(), zr, TOL, what='z')


def test_folded_eval_bf16(S):
    B, H, W = 2, 64, 32
    x, _ = U.maps(B, H, W, seed=9)
    w, r = U.weights(), U.running()
    z, _ = _folded(S, x, w, r, dtype=1)
    zr, _, _ = net.forward(w, r, x, 'eval')
    e = U.rel_l2(z.cpu().numpy(), zr)
    _say(f'folded bf16: z rel-L2 {e:.2e}')
    assert e < 2e-2


def test_folded_graph_replays(S):
    B, H, W = 1, 128, 64
    x, _ = U.maps(B, H, W, seed=3)
    w, r = U.weights(), U.running()
    z, (segs, xd, fb, ws) = _folded(S, x, w, r)
    ref = z.clone()
    zg = torch.full_like(z, float('nan'))
    g = S.FoldedForwardGraph(segs, xd, fb, zg, ws)
    try:
        for k in range(4):
            zg.fill_(float('nan'))
            torch.cuda.synchronize()
            g.launch()
            g.stream.synchronize()
            assert torch.equal(zg, ref), k
            S.forward_folded(segs, xd, fb, z, ws)   # eager work between the replays
            torch.cuda.synchronize()
    finally:
        g.close()


def test_folded_sigmoid_output(S):
    B, H, W = 2, 32, 24
    x, _ = U.maps(B, H, W, seed=21)
    w, r = U.weights(), U.running()
    S.set_arch(head='sigmoid')
    net.set_arch(head='sigmoid')
    try:
        z, _ = _folded(S, x, w, r)
        zr, _, _ = net.forward(w, r, x, 'eval')
    finally:
        S.set_arch()
        net.set_arch()
    U.assert_close(z.cpu().numpy(), zr, TOL, what='z')
