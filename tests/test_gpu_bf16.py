"""BF16 path (BF16 activations, gradients and convolution weights, FP32 accumulation, FP32
master weights) against the FP64 oracle run on the FP32 master weights.

Gates: rel-L2 <= 2e-2 for z and the running statistics; mean |delta SINR| <= 0.05 dB over an
8-clip batch on z, with the target and noise cells of the scene that produced the input.  Gradients: with activations
rounded to 8 significant bits, ReLU pre-activations within about 2^-9 of their layer's scale of
the kink take the other decision than in FP64 (a few per thousand sites); each flip moves a
batch-norm shift gradient (a sum of n terms of random sign) by about 1/sqrt(n), so per-tensor
gradient errors of several percent against the FP64 oracle are the expected cost of the format.
They are reported; the gate on the whole gradient vector is rel-L2 <= 0.25."""
import sys

import numpy as np
import pytest
import torch

from oracle import net, rdsynth
from paper_2307_09063_amd import inputs
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TOL = 2e-2
CASES = [(2, 32, 24, False), (2, 40, 36, False), (2, 64, 64, True), (4, 128, 64, True)]


@pytest.mark.parametrize('case', CASES, ids=lambda c: f'{c[0]}x{c[1]}x{c[2]}')
def test_bf16_train_forward_backward(case):
    from paper_2307_09063_amd import stda
    B, H, W, rd = case
    print('bf16', case, file=sys.stderr, flush=True)
    if rd:
        x, y, tab, meta = U.rd_maps(B, H, W, seed=H + W, intf=(1, 2))
    else:
        x, y = U.maps(B, H, W, seed=3)
    w, r = U.weights(), U.running()
    segs = stda.uniform_segments(B, H, W)
    sv, wsb = stda.workspace_size(segs, stda.BF16, stda.TRAIN)
    saved, ws = stda.alloc_bytes(sv), stda.alloc_bytes(wsb)
    xd, wd, rd_ = U.dev(x), U.dev(w), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    stda.forward(segs, xd, wd, rd_, z, saved, ws, stda.BF16, stda.TRAIN)
    g = np.random.default_rng(1).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    dw = torch.empty(net.param_count(), device='cuda')
    dx = torch.empty_like(xd)
    stda.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, stda.BF16)
    torch.cuda.synchronize()
    zr, rr, cache = net.forward(w, r, x, 'train')
    gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    zc = z.cpu().numpy()
    assert U.rel_l2(zc, zr) < TOL
    assert U.rel_l2(rd_.cpu().numpy(), rr) < TOL
    errs = U.per_tensor_errors(dw.cpu().numpy(), gr)
    flat = U.rel_l2(dw.cpu().numpy(), gr)
    print(f'bf16 {case}: z rel-L2 {U.rel_l2(zc, zr):.2e} max-abs {_maxabs(zc, zr):.2e}; grad flat {flat:.2e} '
          f'dx {U.rel_l2(dx.cpu().numpy(), dxr):.2e} '
          f'worst ' + ' '.join(f'{k}:{v:.1e}' for k, v in sorted(errs.items(), key=lambda t: -t[1])[:4]),
          file=sys.stderr, flush=True)
    assert flat < 0.25


def _maxabs(a, b):
    """max |a - b| / max |b| (reported next to rel-L2)."""
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def _sinr_deltas(zc, zr, meta, H, W):
    ds = []
    for b in range(zc.shape[0]):
        o, n = inputs.sinr_masks(meta['peaks'][b], H, W)
        ds.append(rdsynth.sinr_db(zc[b, 0], o, n) - rdsynth.sinr_db(zr[b, 0], o, n))
    return np.array(ds)


@pytest.mark.parametrize('mode', ['eval', 'train'])
def test_bf16_sinr_delta(mode):
    """Mean |delta SINR| over 8 clips of the paper's map shape (128 range x 64 Doppler bins).
    The O set is one cell per target, so one clip's delta is the error of 1-3 cells of a
    random-weight output; the SINR of the paper is a mean over its test clips."""
    from paper_2307_09063_amd import stda
    B, H, W = 8, 128, 64
    print('bf16 sinr', mode, file=sys.stderr, flush=True)
    x, _, tab, meta = U.rd_maps(B, H, W, seed=77, intf=(1, 2))
    w, r = U.weights(), U.running()
    m = stda.TRAIN if mode == 'train' else stda.EVAL
    segs = stda.uniform_segments(B, H, W)
    sv, wsb = stda.workspace_size(segs, stda.BF16, m)
    saved = stda.alloc_bytes(sv) if m == stda.TRAIN else None
    z = torch.empty((B, 1, H, W), device='cuda')
    stda.forward(segs, U.dev(x), U.dev(w), U.dev(r.copy()), z, saved, stda.alloc_bytes(wsb), stda.BF16, m)
    torch.cuda.synchronize()
    zr, _, _ = net.forward(w, r, x, mode)
    zc = z.cpu().numpy()
    ds = _sinr_deltas(zc, zr, meta, H, W)
    print(f'bf16 {mode}: z rel-L2 {U.rel_l2(zc, zr):.2e} max-abs {_maxabs(zc, zr):.2e}; mean |delta SINR| '
          f'{np.mean(np.abs(ds)):.4f} dB; per clip ' + ' '.join(f'{d:+.4f}' for d in ds),
          file=sys.stderr, flush=True)
    assert U.rel_l2(zc, zr) < TOL
    assert np.mean(np.abs(ds)) <= 0.05, ds


def test_bf16_eval_forward():
    from paper_2307_09063_amd import stda
    B, H, W = 2, 64, 32
    x, _ = U.maps(B, H, W, seed=8)
    w, r = U.weights(), U.running()
    segs = stda.uniform_segments(B, H, W)
    _, wsb = stda.workspace_size(segs, stda.BF16, stda.EVAL)
    z = torch.empty((B, 1, H, W), device='cuda')
    stda.forward(segs, U.dev(x), U.dev(w), U.dev(r.copy()), z, None, stda.alloc_bytes(wsb), stda.BF16, stda.EVAL)
    torch.cuda.synchronize()
    zr, _, _ = net.forward(w, r, x, 'eval')
    assert U.rel_l2(z.cpu().numpy(), zr) < TOL
