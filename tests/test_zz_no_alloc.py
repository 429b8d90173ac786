"""The no-allocation EVAL forward (stda_forward_noalloc, scratch in a static device array) against
stda_forward with a caller workspace, through the C ABI: several calls in a row on the shared
array, each smaller than the one before, in FP32 and BF16; every output bit-identical to the
workspace entry point's (the same kernels on the same inputs), and the FP32 outputs within the
FP32 gate of the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

# the largest 256 x 128 batch whose EVAL workspace fits the static array, then smaller ones
# (several tiles with ragged edges, then a map smaller than one tile in width)
SEQ = [(1, 256, 128), (2, 64, 48), (1, 24, 20)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


def _with_ws(S, segs, xd, wd, rd, dtype):
    B, _, H, W = xd.shape
    _, wsb = S.workspace_size(segs, dtype, S.EVAL)
    ws = S.alloc_bytes(wsb)
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, None, ws, dtype, S.EVAL)
    return z


@pytest.mark.parametrize('dtype', [0, 1])
def test_noalloc_matches_workspace_forward(S, dtype):
    w, r = U.weights(), U.running()
    wd, rd = U.dev(w), U.dev(r)
    runs = []
    for B, H, W in SEQ:
        segs = S.uniform_segments(B, H, W)
        assert S.workspace_size(segs, dtype, S.EVAL)[1] <= S.NOALLOC_WS_MAX
        x, _ = U.maps(B, H, W, seed=B * 1000 + H + W)
        xd = U.dev(x)
        z = torch.full((B, 1, H, W), float('nan'), device='cuda')
        _say('noalloc forward', 'bf16' if dtype else 'fp32', (B, H, W))
        S.forward_noalloc(segs, xd, wd, rd, z, dtype)
        runs.append((segs, x, xd, z))
    torch.cuda.synchronize()
    for segs, x, xd, z in runs:
        ref = _with_ws(S, segs, xd, wd, rd, dtype)
        torch.cuda.synchronize()
        assert torch.equal(z, ref), f'{tuple(xd.shape)}: max |diff| {float((z - ref).abs().max()):.3e}'
        if dtype == 0:
            zr, _, _ = net.forward(w, r, x, 'eval')
            U.assert_close(z.cpu().numpy(), zr, 1e-4, what=f'z {tuple(xd.shape)}')
    np.testing.assert_array_equal(rd.cpu().numpy(), r)  # EVAL leaves the running statistics alone


def test_noalloc_refuses_oversized_batch(S):
    w, r = U.dev(U.weights()), U.dev(U.running())
    segs = S.uniform_segments(2, 256, 128)
    assert S.workspace_size(segs, 0, S.EVAL)[1] > S.NOALLOC_WS_MAX
    x = torch.zeros((2, 3, 256, 128), device='cuda')
    z = torch.zeros((2, 1, 256, 128), device='cuda')
    with pytest.raises(S.StdaError, match='workspace'):
        S.forward_noalloc(segs, x, w, r, z, 0)
