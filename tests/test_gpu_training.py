"""A short training run of the whole FP32 path on the GPU (TRAIN forward with running-statistics
updates, MSE loss, hand-written backward, SGD) against the same run of the FP64 oracle: the loss
of every step, and after the last step the accumulated weight update and the running statistics.
Differences of the two precisions compound over the steps, so the gates are those of one step
(rel-L2 1e-4) applied to what the run accumulated.  The input is screened for ReLU decisions near
their kink at the first step, as in the single-step parity tests."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize('shape', [(2, 16, 16), (3, 24, 20)])
def test_sgd_run_tracks_oracle(shape):
    from paper_2307_09063_amd import stda as S
    B, H, W = shape
    steps, lr, wd = 8, 1e-2, 5e-4
    _say('training run', shape)
    w0, r0 = U.weights(), U.running()
    x, y = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w0, r0, 17 + H)
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, yd, wd_, rd = U.dev(x), U.dev(y), U.dev(w0.copy()), U.dev(r0.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    dz = torch.empty_like(z)
    dw = torch.empty(net.param_count(), device='cuda')
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    losses = []
    for _ in range(steps):
        S.forward(segs, xd, wd_, rd, z, saved, ws, S.FP32, S.TRAIN)
        S.mse_loss(segs, z, yd, loss, dz, ws)
        S.backward(segs, xd, dz, wd_, saved, dw, None, ws, S.FP32)
        S.sgd_step(wd_, dw, lr, wd)
        torch.cuda.synchronize()
        losses.append(loss.item())
    w, r = w0.astype(np.float64), r0.astype(np.float64)
    ref = []
    for _ in range(steps):
        lv, g, _, _, r = net.loss_and_grad(w, r, x, y)
        w = net.sgd_step(w, g, lr, wd)
        ref.append(lv)
    np.testing.assert_allclose(losses, ref, rtol=1e-5)
    assert ref[-1] < ref[0]   # the run trains
    got = wd_.cpu().numpy().astype(np.float64)
    U.assert_close(got - w0, w - w0, 1e-4, what='accumulated update')
    U.assert_close(rd.cpu().numpy(), r, 1e-4, what='running')
