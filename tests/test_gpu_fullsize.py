"""Parity at the benchmark's map size (3 x 256 x 128) and launch configurations.

* rd_synth for the whole B = 32 batch of the forward configuration; sampled clips against the
  oracle (clips are independent).
* EVAL forward at B = 32 (the forward configuration's launch): sampled clips against the oracle
  (in EVAL mode every clip is independent of the others).
* TRAIN forward at B = 4: z and the running statistics against the oracle over the whole batch
  (batch statistics couple the clips, so the oracle needs the whole batch).
* TRAIN loss at B = 64 (the training configuration's launch): the FP64 loss equals the mean of
  squares recomputed on the host from the returned z, and dz = 2 (z - y) / n.
Gradients at this size are not compared element-wise: a network of 256 x 128 maps has about
2.6 million ReLU sites per clip, some within FP32 rounding of their kink, where FP32 and FP64
legitimately decide differently (see the parity tests for the screened comparison)."""
import sys

import numpy as np
import pytest
import torch

from oracle import net, rdsynth
from paper_2307_09063_amd import inputs
from tests import gpu_util as U

pytestmark = pytest.mark.gpu
N, M = 256, 128


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope='module')
def batch32():
    from paper_2307_09063_amd import stda
    rc = inputs.WORKLOADS['cfg2_fwd_256x128']
    tab, meta = inputs.make_scenes(rc['B'], N, M, rc['seed'], targets=rc['targets'], intf=rc['intf'], inr=rc['inr'],
                                   clutter=rc['clutter'])
    _say('rd_synth B=32 256x128')
    x, clean = stda.synthesize(tab, meta)
    torch.cuda.synchronize()
    return tab, meta, x, clean


def test_rd_synth_full_batch_sampled(batch32):
    tab, meta, x, clean = batch32
    sc = inputs.scene_dict(tab, meta)
    for b in (0, 17, 31):
        xr, cr = rdsynth.synth_clip(sc, b)
        assert np.abs(x[b].cpu().numpy() - xr).max() <= 2e-3
        assert np.abs(clean[b].cpu().numpy() - cr).max() <= 2e-3


def test_eval_forward_b32_sampled(batch32):
    from paper_2307_09063_amd import stda
    _, _, x, _ = batch32
    w, r = U.weights(), U.running()
    segs = stda.uniform_segments(32, N, M)
    _, wsb = stda.workspace_size(segs, stda.FP32, stda.EVAL)
    z = torch.empty((32, 1, N, M), device='cuda')
    _say('eval forward B=32 256x128')
    stda.forward(segs, x.contiguous(), U.dev(w), U.dev(r.copy()), z, None, stda.alloc_bytes(wsb), stda.FP32,
                 stda.EVAL)
    torch.cuda.synchronize()
    xc = x.cpu().numpy()
    for b in (0, 9, 31):
        zr, _, _ = net.forward(w, r, xc[b:b + 1], 'eval')
        U.assert_close(z[b:b + 1].cpu().numpy(), zr, 1e-4, what=f'z clip {b}')


def test_train_forward_b4_full_batch(batch32):
    from paper_2307_09063_amd import stda
    _, _, x, _ = batch32
    xb = x[:4].contiguous()
    w, r = U.weights(), U.running()
    segs = stda.uniform_segments(4, N, M)
    sv, wsb = stda.workspace_size(segs, stda.FP32, stda.TRAIN)
    rd = U.dev(r.copy())
    z = torch.empty((4, 1, N, M), device='cuda')
    _say('train forward B=4 256x128')
    stda.forward(segs, xb, U.dev(w), rd, z, stda.alloc_bytes(sv), stda.alloc_bytes(wsb), stda.FP32, stda.TRAIN)
    torch.cuda.synchronize()
    zr, rr, _ = net.forward(w, r, xb.cpu().numpy(), 'train')
    U.assert_close(z.cpu().numpy(), zr, 1e-4, what='z')
    U.assert_close(rd.cpu().numpy(), rr, 1e-4, what='running')


def test_train_loss_b64_launch():
    from paper_2307_09063_amd import stda
    rc = inputs.WORKLOADS['cfg3_train_256x128']
    B = rc['B']
    tab, meta = inputs.make_scenes(B, N, M, rc['seed'], targets=rc['targets'], intf=rc['intf'], inr=rc['inr'],
                                   clutter=rc['clutter'])
    _say('train step B=64 256x128')
    x, y = stda.synthesize(tab, meta)
    w, r = U.weights(), U.running()
    segs = stda.uniform_segments(B, N, M)
    sv, wsb = stda.workspace_size(segs, stda.FP32, stda.TRAIN)
    saved, ws = stda.alloc_bytes(sv), stda.alloc_bytes(wsb)
    z = torch.empty((B, 1, N, M), device='cuda')
    stda.forward(segs, x, U.dev(w), U.dev(r.copy()), z, saved, ws, stda.FP32, stda.TRAIN)
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    dz = torch.empty_like(z)
    stda.mse_loss(segs, z, y, loss, dz, ws)
    dw = torch.empty(net.param_count(), device='cuda')
    stda.backward(segs, x, dz, U.dev(w), saved, dw, None, ws)
    torch.cuda.synchronize()
    zc, yc = z.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    lr_, dzr = net.mse_loss(zc, yc)
    assert abs(loss.item() - lr_) <= 1e-12 * lr_
    U.assert_close(dz.cpu().numpy(), dzr, 1e-6, what='dz')
    assert np.isfinite(dw.cpu().numpy()).all()
