"""Uneven batching in BF16 against the per-size FP32 path: one captured training step (forward,
loss, backward) over clips of the three map sizes of the uneven workload (128 x 64, 256 x 128,
512 x 256), each size its own batch-norm segment, against the FP32 path run on each size alone,
in the same order, on the same weights and running buffer.  z, the loss (the sum of the
per-segment means) and the running statistics agree within the BF16 gate (rel-L2 2e-2).  The
gradient (the sum of the per-segment gradients) is gated as in the BF16 parity tests, against
the BF16 storage model's gradient of the same step: rel-L2 <= 2e-2 + 2 x the spread of a
jittered run of the model (the format's own floor; see tests/test_gpu_bf16.py)."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import bf16_model as M
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def test_uneven_bf16_graph_matches_per_size_fp32():
    from paper_2307_09063_amd import stda as S
    print('uneven bf16 vs per-size fp32', file=sys.stderr, flush=True)
    parts = [(2, 128, 64), (1, 256, 128), (1, 512, 256)]
    xs, ys = zip(*(U.maps(n, H, W, seed=5 * n + H + W) for n, H, W in parts))
    w0, r0 = U.weights(), U.running()
    # the per-size FP32 path, size by size
    rd = U.dev(r0.copy())
    wd = U.dev(w0.copy())
    zs, loss_sum, dw_sum = [], 0.0, np.zeros(net.param_count())
    for (n, H, W), x, y in zip(parts, xs, ys):
        segs = S.uniform_segments(n, H, W)
        sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
        saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
        xd, yd = U.dev(x), U.dev(y)
        z = torch.empty((n, 1, H, W), device='cuda')
        dz = torch.empty_like(z)
        loss = torch.zeros(1, dtype=torch.float64, device='cuda')
        dw = torch.empty(net.param_count(), device='cuda')
        S.forward(segs, xd, wd, rd, z, saved, ws, S.FP32, S.TRAIN)
        S.mse_loss(segs, z, yd, loss, dz, ws)
        S.backward(segs, xd, dz, wd, saved, dw, None, ws, S.FP32)
        torch.cuda.synchronize()
        zs.append(z.cpu().numpy().ravel())
        loss_sum += loss.item()
        dw_sum += dw.cpu().numpy()
    r_ref = rd.cpu().numpy()
    # one captured BF16 step over the packed batch (learning rate 0: the weights stay as they are)
    segs = S.packed_segments(parts)
    x = U.dev(np.concatenate([a.ravel() for a in xs]))
    y = U.dev(np.concatenate([a.ravel() for a in ys]))
    sv, wsb = S.workspace_size(segs, S.BF16, S.TRAIN)
    nz = y.numel()
    b = dict(w=U.dev(w0.copy()), running=U.dev(r0.copy()), z=torch.empty(nz, device='cuda'),
             loss=torch.zeros(1, dtype=torch.float64, device='cuda'), dz=torch.empty(nz, device='cuda'),
             dw=torch.empty(net.param_count(), device='cuda'), saved=S.alloc_bytes(sv), ws=S.alloc_bytes(wsb))
    wb = torch.empty(net.param_count(), dtype=torch.int16, device='cuda')
    graph = S.TrainStepGraph(segs, x, y, b['w'], b['running'], b['z'], b['loss'], b['dz'], b['dw'], b['saved'],
                             b['ws'], dtype=S.BF16, lr=0.0, weight_decay=0.0, w_bf16=wb)
    torch.cuda.synchronize()
    graph.launch()
    graph.stream.synchronize()
    graph.close()
    z = b['z'].cpu().numpy()
    off = 0
    for (n, H, W), zr in zip(parts, zs):
        assert U.rel_l2(z[off:off + n * H * W], zr) < 2e-2, (n, H, W)
        off += n * H * W
    assert abs(b['loss'].item() - loss_sum) <= 2e-2 * abs(loss_sum)
    assert U.rel_l2(b['running'].cpu().numpy(), r_ref) < 2e-2
    np.testing.assert_array_equal(b['w'].cpu().numpy(), w0)   # lr 0, no decay
    # the storage model's step (segments in order, each its own statistics) and a jittered run
    gm, gj = np.zeros(net.param_count()), np.zeros(net.param_count())
    for x_, y_ in zip(xs, ys):
        for jit, acc in ((None, gm), ((1, 2.0 ** -20), gj)):
            zm, cm = M.forward(w0, r0, x_, 'train', jitter=jit)
            _, dzm = net.mse_loss(zm, y_)
            acc += net.backward(dzm, cm)[0]
    dwc = b['dw'].cpu().numpy()
    env = U.rel_l2(gj, gm)
    print(f'  gradient rel-L2 vs storage model {U.rel_l2(dwc, gm):.2e} (envelope {env:.2e}), vs per-size FP32 '
          f'{U.rel_l2(dwc, dw_sum):.2e} (model vs FP32 {U.rel_l2(gm, dw_sum):.2e})', file=sys.stderr, flush=True)
    assert U.rel_l2(dwc, gm) <= 2e-2 + 2 * env
