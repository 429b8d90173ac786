"""The tiling variants of the stage-2 dense layers, of their weight gradients and of the fused
stage-1 adjoint (the autotuner's candidates), through the C ABI.

* EVAL forward: every variant gives bit-identical z (each output element sums its taps and
  channels in the same order whatever the tiling), on shapes whose maps leave ragged tiles at
  every level.
* FP32 TRAIN forward + backward of every variant against the FP64 oracle (inputs screened for
  ReLU decisions within 1e-5 of their kink, as in the other FP32 parity tests).
* BF16 TRAIN forward of every variant against the oracle at the BF16 gate.
* The autotuner: its choice is one of the candidates, it leaves the master weights untouched,
  and the network still matches the oracle afterwards."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu
SHAPES = [(2, 40, 36), (1, 72, 88)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture()
def S():
    from paper_2307_09063_amd import stda
    yield stda
    for dt in (stda.FP32, stda.BF16):
        for kind in stda.TUNE_KINDS:
            for b in range(4):
                stda.tune_set(kind, dt, b, 0)


def _set_all(S, dtype, v):
    for kind in S.TUNE_KINDS:
        for b in range(4):
            S.tune_set(kind, dtype, b, v)


def _forward(S, x, w, r, mode, dtype):
    B, _, H, W = x.shape
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, dtype, mode)
    saved = S.alloc_bytes(sv) if mode == S.TRAIN else None
    ws = S.alloc_bytes(wsb)
    xd, wd, rd = U.dev(x), U.dev(w), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, dtype, mode)
    torch.cuda.synchronize()
    return z, rd, (segs, xd, wd, saved, ws)


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
@pytest.mark.parametrize('shape', SHAPES)
def test_variants_eval_bitwise(S, dtype, shape):
    B, H, W = shape
    x, _ = U.maps(B, H, W, seed=H + W)
    w, r = U.weights(), U.running()
    outs = []
    for v in range(S.tune_count(S.TUNE_FWD)):
        _say('variant eval', dtype, shape, v)
        _set_all(S, dtype, v)
        z, _, _ = _forward(S, x, w, r, S.EVAL, dtype)
        outs.append(z.cpu().numpy())
    for v in range(1, len(outs)):
        np.testing.assert_array_equal(outs[v], outs[0])
    zr, _, _ = net.forward(w, r, x, 'eval')
    if dtype == 0:
        U.assert_close(outs[0], zr, 1e-4, what='z')
    else:
        assert U.rel_l2(outs[0], zr) < 2e-2


@pytest.mark.parametrize('v', [0, 1, 2, 3])
def test_variant_fp32_train_backward(S, v):
    B, H, W = SHAPES[0]
    _say('variant train fp32', v)
    _set_all(S, S.FP32, v)
    w, r = U.weights(), U.running()
    x, _ = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, 77)
    z, rd, (segs, xd, wd, saved, ws) = _forward(S, x, w, r, S.TRAIN, S.FP32)
    zr, rr, cache = net.forward(w, r, x, 'train')
    U.assert_close(z.cpu().numpy(), zr, 1e-4, what='z')
    U.assert_close(rd.cpu().numpy(), rr, 1e-4, what='running')
    g = np.random.default_rng(v).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    dw = torch.full((net.param_count(),), float('nan'), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws)
    torch.cuda.synchronize()
    gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
    bad = U.grad_failures(dw.cpu().numpy(), gr, 1e-4)
    assert not bad, bad
    U.assert_close(dx.cpu().numpy(), dxr, 1e-4, what='dx')


@pytest.mark.parametrize('v', [0, 1, 2, 3])
def test_variant_bf16_train_forward(S, v):
    B, H, W = SHAPES[1]
    _say('variant train bf16', v)
    _set_all(S, S.BF16, v)
    x, _ = U.maps(B, H, W, seed=5)
    w, r = U.weights(), U.running()
    z, rd, _ = _forward(S, x, w, r, S.TRAIN, S.BF16)
    zr, rr, _ = net.forward(w, r, x, 'train')
    assert U.rel_l2(z.cpu().numpy(), zr) < 2e-2
    assert U.rel_l2(rd.cpu().numpy(), rr) < 2e-2


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
def test_autotune(S, dtype):
    B, H, W = 2, 32, 24
    _say('autotune', dtype)
    w0, r = U.weights(), U.running()
    x, y = U.maps(B, H, W, seed=9)
    segs = S.uniform_segments(B, H, W)
    sv, wsb = S.workspace_size(segs, dtype, S.TRAIN)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    xd, yd, wd, rs = U.dev(x), U.dev(y), U.dev(w0), U.dev(r.copy())
    z = torch.empty((B, 1, H, W), device='cuda')
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    dz, dw = torch.empty_like(z), torch.empty(net.param_count(), device='cuda')
    res = S.autotune(segs, xd, yd, wd, rs, z, loss, dz, dw, saved, ws, dtype, reps=2)
    torch.cuda.synchronize()
    n = S.tune_count(S.TUNE_FWD)
    assert sorted(res) == [(k, b) for k in S.TUNE_KINDS for b in range(4)]
    for (kind, b), (choice, ms) in res.items():
        assert 0 <= choice < n and len(ms) == n and all(t > 0 for t in ms)
        # the fastest, except that the default stays unless another is 3 % faster
        # (times are printed to 1e-6 ms, hence the slack)
        assert ms[choice] == min(ms) or (choice == 0 and min(ms) >= 0.97 * ms[0] - 1e-6)
        assert choice == 0 or ms[choice] <= 0.97 * ms[0] + 1e-6
        assert S.tune_get(kind, dtype, b) == choice
    np.testing.assert_array_equal(wd.cpu().numpy(), w0)
    zt, _, _ = _forward(S, x, w0, r, S.EVAL, dtype)
    zr, _, _ = net.forward(w0, r, x, 'eval')
    assert U.rel_l2(zt.cpu().numpy(), zr) < (1e-4 if dtype == 0 else 2e-2)


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
def test_wgrad_variants_agree(S, dtype):
    """Only the weight-gradient tiling changes: forward, dx and every gradient that does not come
    from a stage-2 weight are bit-identical, and the stage-2 weight gradients differ only by the
    order of their FP32 pixel sums."""
    B, H, W = SHAPES[1]
    x, y = U.maps(B, H, W, seed=31)
    w, r = U.weights(), U.running()
    g = np.random.default_rng(3).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    res = []
    for v in range(S.tune_count(S.TUNE_WGRAD)):
        _say('wgrad variant', dtype, v)
        for b in range(4):
            S.tune_set(S.TUNE_WGRAD, dtype, b, v)
        z, _, (segs, xd, wd, saved, ws) = _forward(S, x, w, r, S.TRAIN, dtype)
        dw = torch.full((net.param_count(),), float('nan'), device='cuda')
        dx = torch.empty_like(xd)
        S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, dtype)
        torch.cuda.synchronize()
        res.append((z.cpu().numpy(), dw.cpu().numpy(), dx.cpu().numpy()))
    stage2 = {f'{k}.s2.{m}.w' for k in ('enc0', 'enc1', 'dec0', 'dec1') for m in ('main', 'res')}
    for v in range(1, len(res)):
        np.testing.assert_array_equal(res[v][0], res[0][0])
        np.testing.assert_array_equal(res[v][2], res[0][2])
        off = 0
        for name, shape, _ in net.param_specs():
            n = int(np.prod(shape))
            a, b = res[v][1][off:off + n], res[0][1][off:off + n]
            if name in stage2:
                assert U.rel_l2(a, b) < 1e-5, (name, v)
            else:
                np.testing.assert_array_equal(a, b)
            off += n


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
def test_stage1_adjoint_variants_agree(S, dtype):
    """Only the stage-1 adjoint tiling changes.  Each pixel's input gradient is the same expression
    in every variant, but each instantiation is compiled on its own (tile shape, register budget)
    and may fuse its multiply-adds differently, so dx and the gradients upstream of it agree to
    FP32 rounding rather than bitwise; the stage-1 weight gradients (summed per tile) also differ
    by the order of their pixel sums (in BF16, where the adjoint stores its outputs in BF16, those
    FP32 differences can move single elements by a BF16 step).  Each variant also meets the oracle
    gate (test_variant_fp32_train_backward)."""
    B, H, W = SHAPES[1]
    x, _ = U.maps(B, H, W, seed=41)
    w, r = U.weights(), U.running()
    g = np.random.default_rng(4).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    res = []
    for v in range(S.tune_count(S.TUNE_S1_BWD)):
        _say('stage-1 adjoint variant', dtype, v)
        for b in range(4):
            S.tune_set(S.TUNE_S1_BWD, dtype, b, v)
        z, _, (segs, xd, wd, saved, ws) = _forward(S, x, w, r, S.TRAIN, dtype)
        dw = torch.full((net.param_count(),), float('nan'), device='cuda')
        dx = torch.empty_like(xd)
        S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, dtype)
        torch.cuda.synchronize()
        res.append((dw.cpu().numpy(), dx.cpu().numpy()))
    # FP32: agreement to FP32 rounding.  BF16: the adjoint's outputs are stored in BF16, so an FP32
    # difference that straddles a BF16 rounding boundary moves that element by a full BF16 step
    # (2^-8 relative); a few such elements per ten thousand give rel-L2 of order 1e-4.
    tol_dx, tol_w = (1e-6, 1e-5) if dtype == 0 else (2e-3, 2e-3)
    for v in range(1, len(res)):
        assert U.rel_l2(res[v][1], res[0][1]) < tol_dx, v
        bad = {k: e for k, e in U.per_tensor_errors(res[v][0], res[0][0]).items() if not e < tol_w}
        assert not bad, (v, bad)
