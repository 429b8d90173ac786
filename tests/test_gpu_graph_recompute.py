"""Recompute mode and the hipGraph-captured training step, through the C ABI.

Recompute re-runs each block's forward kernels (with the saved batch statistics) right before
its adjoint, so its gradients must equal the stored-activation path bit for bit; it is also
checked against the FP64 oracle.  The captured step (forward, loss, backward, SGD) is replayed
several times, with eager work and synchronisation between replays, and every replay must equal
the same step run eagerly, bit for bit (all reductions are in a fixed order)."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _fwd_bwd(S, segs, xd, wd, r, g, dtype, rec):
    sv, wsb = S.workspace_size(segs, dtype, S.TRAIN, rec)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    rd = U.dev(r.copy())
    z = torch.empty(g.shape, device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, dtype, S.TRAIN, rec)
    dw = torch.empty(net.param_count(), device='cuda')
    dx = torch.empty_like(xd)
    S.backward(segs, xd, U.dev(g), wd, saved, dw, dx, ws, dtype, rec)
    torch.cuda.synchronize()
    return z.cpu().numpy(), rd.cpu().numpy(), dw.cpu().numpy(), dx.cpu().numpy()


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
def test_recompute_bitwise_and_oracle(dtype):
    from paper_2307_09063_amd import stda as S
    B, H, W = 3, 32, 24
    _say('recompute', dtype)
    w, r = U.weights(), U.running()
    x, _ = U.unambiguous(lambda s: U.maps(B, H, W, seed=s), w, r, 21)
    g = np.random.default_rng(2).standard_normal((B, 1, H, W)).astype(np.float32) / (B * H * W)
    segs = S.uniform_segments(B, H, W)
    xd, wd = U.dev(x), U.dev(w)
    a = _fwd_bwd(S, segs, xd, wd, r, g, dtype, 0)
    b = _fwd_bwd(S, segs, xd, wd, r, g, dtype, 1)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    if dtype == 0:
        _, _, cache = net.forward(w, r, x, 'train')
        gr, dxr = net.backward(g.astype(np.float64), cache, want_dx=True)
        bad = U.grad_failures(b[2], gr, 1e-4)
        assert not bad, bad
        U.assert_close(b[3], dxr, 1e-4, what='dx')


@pytest.mark.parametrize('case', ['uniform', 'uneven'])
def test_graph_replay_matches_eager(case):
    from paper_2307_09063_amd import stda as S
    _say('graph', case)
    parts = [(2, 32, 24)] if case == 'uniform' else [(2, 16, 16), (3, 32, 24)]
    segs = S.packed_segments(parts)
    xs, ys = zip(*(U.maps(n, H, W, seed=n * H + W) for n, H, W in parts))
    x = U.dev(np.concatenate([a.ravel() for a in xs]))
    y = U.dev(np.concatenate([a.ravel() for a in ys]))
    w0, r0 = U.weights(), U.running()
    sv, wsb = S.workspace_size(segs, S.FP32, S.TRAIN)
    nz = y.numel()

    def buffers():
        return dict(w=U.dev(w0.copy()), running=U.dev(r0.copy()), z=torch.empty(nz, device='cuda'),
                    loss=torch.zeros(1, dtype=torch.float64, device='cuda'), dz=torch.empty(nz, device='cuda'),
                    dw=torch.empty(net.param_count(), device='cuda'), saved=S.alloc_bytes(sv), ws=S.alloc_bytes(wsb))

    steps = 3
    eb = buffers()
    eager = []
    for _ in range(steps):
        S.forward(segs, x, eb['w'], eb['running'], eb['z'], eb['saved'], eb['ws'], S.FP32, S.TRAIN)
        S.mse_loss(segs, eb['z'], y, eb['loss'], eb['dz'], eb['ws'])
        S.backward(segs, x, eb['dz'], eb['w'], eb['saved'], eb['dw'], None, eb['ws'])
        S.sgd_step(eb['w'], eb['dw'], 1e-3, 5e-4)
        torch.cuda.synchronize()
        eager.append((eb['w'].cpu().numpy(), eb['running'].cpu().numpy(), eb['loss'].item()))
    gb = buffers()
    graph = S.TrainStepGraph(segs, x, y, gb['w'], gb['running'], gb['z'], gb['loss'], gb['dz'], gb['dw'],
                             gb['saved'], gb['ws'])
    torch.cuda.synchronize()
    # capturing ran nothing: the master weights are untouched
    np.testing.assert_array_equal(gb['w'].cpu().numpy(), w0)
    for k in range(steps):
        graph.launch()
        graph.stream.synchronize()
        junk = torch.randn(1 << 16, device='cuda').sum()   # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gb['w'].cpu().numpy(), eager[k][0])
        np.testing.assert_array_equal(gb['running'].cpu().numpy(), eager[k][1])
        assert gb['loss'].item() == eager[k][2]
        del junk
    graph.close()


@pytest.mark.parametrize('dtype', [0, 1], ids=['fp32', 'bf16'])
def test_forward_graph_replays(dtype):
    """A captured EVAL forward replays bit-identically to the eager call, and reads the bound
    input buffer afresh on every replay."""
    from paper_2307_09063_amd import stda as S
    B, H, W = 1, 128, 64
    _say('forward graph', dtype)
    w, r = U.weights(), U.running()
    segs = S.uniform_segments(B, H, W)
    _, wsb = S.workspace_size(segs, dtype, S.EVAL)
    xs = [U.maps(B, H, W, seed=40 + k)[0] for k in range(3)]
    xd, wd, rd = U.dev(xs[0]), U.dev(w), U.dev(r.copy())
    z_e = torch.empty((B, 1, H, W), device='cuda')
    z_g = torch.empty_like(z_e)
    ws_e, ws_g = S.alloc_bytes(wsb), S.alloc_bytes(wsb)
    graph = S.ForwardGraph(segs, xd, wd, rd, z_g, ws_g, dtype)
    for k in range(3):
        xd.copy_(U.dev(xs[k]))
        S.forward(segs, xd, wd, rd, z_e, None, ws_e, dtype, S.EVAL)
        torch.cuda.synchronize()
        graph.launch()
        graph.stream.synchronize()
        junk = torch.randn(1 << 16, device='cuda').sum()   # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(z_g.cpu().numpy(), z_e.cpu().numpy())
        del junk
    np.testing.assert_array_equal(rd.cpu().numpy(), r)
    graph.close()
