"""Batch-norm statistics of inputs far from zero mean: the TRAIN forward with BN inputs whose
|mean| / std reaches tens (maps offset by 100, every BN shift at +100 so that every ReLU passes
its input and the following layers see large-mean inputs too).  A one-pass variance
E[x^2] - E[x]^2 of FP32 partial sums loses about (mean/std)^2 of its precision there.  The
initial running variances are tiny, so the updated running variance is one tenth of the batch
variance (unbiased) and shows its error at full relative size: every channel of every layer is
gated element-wise, beside z and the whole running buffer at the FP32 gate."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


def _offset_weights():
    w = U.weights().astype(np.float64)
    off = 0
    for name, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        if name.endswith('.beta'):
            w[off:off + n] += 100.0
        off += n
    return w.astype(np.float32)


@pytest.mark.parametrize('B,H,W', [(2, 256, 128), (3, 40, 36)])
def test_train_forward_large_mean(S, B, H, W):
    print('bn offset', (B, H, W), file=sys.stderr, flush=True)
    x, _ = U.maps(B, H, W, seed=H + W + 5)
    x = (x + 100.0).astype(np.float32)
    w, r = _offset_weights(), U.running(perturb=False)
    r = r.copy()
    off = 0
    for _, c in net.bn_specs():
        r[off + c:off + 2 * c] = 1e-6  # running variances
        off += 2 * c
    zr, rr, cache = net.forward(w, r, x, 'train')
    ratios = {}
    for name, _ in net.bn_specs():
        c = cache['caches'][name]
        ok = c['var'] > 0  # (a channel can be constant: its ratio is unbounded)
        ratios[name] = float(np.max(np.abs(c['mu'][ok]) / np.sqrt(c['var'][ok])))
    # every layer's largest |mean| / std is above 1, and at least four layers reach 30
    assert min(ratios.values()) > 1 and sum(v >= 30 for v in ratios.values()) >= 4, ratios
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, wd, rd = U.dev(x), U.dev(w), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, S.FP32, S.TRAIN)
    torch.cuda.synchronize()
    print('  median |mean|/std %.1f, min %.1f; z rel-L2 %.2e, running rel-L2 %.2e' % (
        np.median(list(ratios.values())), min(ratios.values()), U.rel_l2(z.cpu().numpy(), zr),
        U.rel_l2(rd.cpu().numpy(), rr)), file=sys.stderr, flush=True)
    rg = rd.cpu().numpy().astype(np.float64)
    # per channel: relative error of the running variance in units of 2^-24 (1 + |mean| / std).
    # A variance computed from FP32 values cannot do better than about one such unit (the values
    # themselves carry that error after normalisations of large-mean inputs); a one-pass
    # E[x^2] - E[x]^2 of FP32 partial sums misses by (mean / std)^2 units.  The input module and the
    # encoder blocks, whose inputs come straight from large-mean layers, are gated at 4 units; the
    # decoder blocks, whose inputs have passed through every earlier normalisation, at 1e-4
    # relative (their FP32 inputs already differ from the oracle's by about that much).
    units, worst, off = {}, {}, 0
    for name, c in net.bn_specs():
        cc = cache['caches'][name]
        ratio = np.abs(cc['mu']) / np.sqrt(np.maximum(cc['var'], 1e-300))
        vg, vr = rg[off + c:off + 2 * c], rr[off + c:off + 2 * c]
        e = np.abs(vg - vr) / vr
        worst[name] = float(e.max())
        units[name] = float(np.max(e / (2.0 ** -24 * (1.0 + ratio))))
        off += 2 * c
    print('  running variance: worst relative error %.2e (%s); worst %.1f units of 2^-24 (1 + |mean|/std) (%s)' % (
        max(worst.values()), max(worst, key=worst.get), max(units.values()), max(units, key=units.get)),
        file=sys.stderr, flush=True)
    U.assert_close(z.cpu().numpy(), zr, 1e-4, what='z')
    U.assert_close(rg, rr, 1e-4, what='running')
    enc = {k: v for k, v in units.items() if not k.startswith('dec')}
    assert max(enc.values()) <= 4.0, enc
    assert max(worst.values()) <= 1e-4, worst
