"""One launch per kernel kind over segments of uneven map sizes, against the same path run on each
size alone.

A packed batch of the uneven workload's three map sizes (128 x 64, 256 x 128, 512 x 256; each
size its own batch-norm segment) runs every layer as one launch whose workgroups walk the tile
lists of all three segments.  Per segment the kernels, tilings and grids are those of a call on
that segment alone, so the forward output, the batch statistics and the running buffer (one
momentum update per segment, in segment order) are bit-identical to three calls made size by
size in that order.  Parameter gradients are the per-segment gradients summed: the packed call
sums the partial rows of all segments in FP64 and rounds once, the per-size calls round each
segment's sum before they are added, so they agree to FP32 rounding (rel-L2 <= 1e-6 FP32,
2e-6 BF16).  Covered in TRAIN (with and without recomputation), EVAL and folded EVAL, FP32 and
BF16, and with a grid cap that makes every workgroup walk several tiles.  The packed call issues
as many launches as a call on one size."""
import sys

import numpy as np
import pytest
import torch

from oracle import net
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

PARTS = [(2, 128, 64), (1, 256, 128), (1, 512, 256)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _inputs():
    xs, ys = zip(*(U.maps(n, H, W, seed=7 * n + H + W) for n, H, W in PARTS))
    return xs, ys


def _train(S, segs, x, y, w, r, dtype, rec):
    sv, wsb = S.workspace_size(segs, dtype, S.TRAIN, rec)
    saved, ws = S.alloc_bytes(sv), S.alloc_bytes(wsb)
    nz = y.size
    xd, yd = U.dev(x.ravel()), U.dev(y.ravel())
    rd, wd = U.dev(r.copy()), U.dev(w)
    z, dz = torch.empty(nz, device='cuda'), torch.empty(nz, device='cuda')
    loss = torch.zeros(1, dtype=torch.float64, device='cuda')
    dw = torch.empty(net.param_count(), device='cuda')
    dx = torch.empty(x.size, device='cuda')
    S.forward(segs, xd, wd, rd, z, saved, ws, dtype, S.TRAIN, rec)
    S.mse_loss(segs, z, yd, loss, dz, ws)
    S.backward(segs, xd, dz, wd, saved, dw, dx, ws, dtype, rec)
    torch.cuda.synchronize()
    return z.cpu().numpy(), rd.cpu().numpy(), dw.cpu().numpy(), dx.cpu().numpy(), dz.cpu().numpy()


def _per_size_train(S, xs, ys, w, r, dtype, rec):
    """Each size alone, in order, the running buffer carried from one call to the next."""
    zs, dws, dxs = [], np.zeros(net.param_count()), []
    run = r.copy()
    for (n, H, W), x, y in zip(PARTS, xs, ys):
        z, run, dw, dx, _ = _train(S, S.uniform_segments(n, H, W), x, y, w, run, dtype, rec)
        zs.append(z)
        dws += dw
        dxs.append(dx)
    return np.concatenate(zs), run, dws, np.concatenate(dxs)


@pytest.mark.parametrize('dtype,rec,cap', [('fp32', 0, 0), ('fp32', 1, 0), ('fp32', 0, 24), ('bf16', 1, 0)])
def test_packed_train_step_equals_per_size(dtype, rec, cap):
    from paper_2307_09063_amd import stda as S
    dt = S.FP32 if dtype == 'fp32' else S.BF16
    _say('multiseg train', dtype, 'recompute', rec, 'grid cap', cap)
    xs, ys = _inputs()
    w, r = U.weights(), U.running()
    S.set_grid_cap(cap)
    try:
        zr, rr, dwr, dxr = _per_size_train(S, xs, ys, w, r, dt, rec)
        segs = S.packed_segments(PARTS)
        x = np.concatenate([a.ravel() for a in xs])
        y = np.concatenate([a.ravel() for a in ys])
        z, run, dw, dx, _ = _train(S, segs, x, y, w, r, dt, rec)
    finally:
        S.set_grid_cap(0)
    gate = 1e-6 if dt == S.FP32 else 2e-6
    _say(f'  z max |diff| {np.abs(z - zr).max():.3e}, running {np.abs(run - rr).max():.3e}, '
         f'dw rel-L2 {U.rel_l2(dw, dwr):.2e} max-rel {U.max_rel(dw, dwr):.2e}, dx {U.rel_l2(dx, dxr):.2e}')
    np.testing.assert_array_equal(z, zr)
    np.testing.assert_array_equal(run, rr)
    np.testing.assert_array_equal(dx, dxr)   # per clip: no sum across segments
    bad = U.grad_failures(dw, dwr, gate, elem=10 * gate)
    assert not bad, bad


@pytest.mark.parametrize('dtype', ['fp32', 'bf16'])
def test_packed_eval_and_folded_equal_per_size(dtype):
    from paper_2307_09063_amd import stda as S
    dt = S.FP32 if dtype == 'fp32' else S.BF16
    _say('multiseg eval / folded', dtype)
    xs, _ = _inputs()
    w, r = U.weights(), U.running()
    fb = S.eval_fold_size(dt)
    folded = S.alloc_bytes(fb)
    S.eval_fold(U.dev(w), U.dev(r), folded, dt)

    def run(segs, x, folded_path):
        _, wsb = S.workspace_size(segs, dt, S.EVAL)
        ws = S.alloc_bytes(wsb)
        z = torch.empty(x.size // 3, device='cuda')
        if folded_path:
            S.forward_folded(segs, U.dev(x.ravel()), folded, z, ws, dt)
        else:
            S.forward(segs, U.dev(x.ravel()), U.dev(w), U.dev(r.copy()), z, None, ws, dt, S.EVAL)
        torch.cuda.synchronize()
        return z.cpu().numpy()

    for folded_path in (False, True):
        zr = np.concatenate([run(S.uniform_segments(n, H, W), x, folded_path) for (n, H, W), x in zip(PARTS, xs)])
        z = run(S.packed_segments(PARTS), np.concatenate([a.ravel() for a in xs]), folded_path)
        _say(f'  folded {folded_path}: max |diff| {np.abs(z - zr).max():.3e}')
        np.testing.assert_array_equal(z, zr)


def test_eight_small_segments_equal_per_size():
    """The most segments a launch takes (8), of small and ragged sizes whose grids are not
    multiples of 8 (so later segments start after idle workgroup slots): a TRAIN step against the
    sizes run one at a time, as above."""
    from paper_2307_09063_amd import stda as S
    parts = [(1, 8, 8), (2, 12, 16), (1, 16, 8), (1, 20, 28), (2, 8, 32), (1, 36, 12), (1, 24, 24), (1, 16, 40)]
    _say('multiseg 8 segments')
    xs, ys = zip(*(U.maps(n, H, W, seed=3 * n + H + 5 * W) for n, H, W in parts))
    w, r = U.weights(), U.running()
    zs, dwr, dxs, run = [], np.zeros(net.param_count()), [], r.copy()
    for (n, H, W), x, y in zip(parts, xs, ys):
        z, run, dw, dx, _ = _train(S, S.uniform_segments(n, H, W), x, y, w, run, S.FP32, 0)
        zs.append(z)
        dwr += dw
        dxs.append(dx)
    z, rp, dw, dx, _ = _train(S, S.packed_segments(parts), np.concatenate([a.ravel() for a in xs]),
                              np.concatenate([a.ravel() for a in ys]), w, r, S.FP32, 0)
    np.testing.assert_array_equal(z, np.concatenate(zs))
    np.testing.assert_array_equal(rp, run)
    np.testing.assert_array_equal(dx, np.concatenate(dxs))
    bad = U.grad_failures(dw, dwr, 1e-6, elem=1e-5)
    assert not bad, bad


def test_packed_launch_count_equals_one_size():
    """The packed three-size step issues as many launches as a step on one size."""
    from paper_2307_09063_amd import stda as S
    _say('multiseg launch count')
    xs, ys = _inputs()
    w, r = U.weights(), U.running()
    counts = {}
    for name, segs, x, y in (('one size', S.uniform_segments(*PARTS[0]), xs[0], ys[0]),
                             ('packed', S.packed_segments(PARTS), np.concatenate([a.ravel() for a in xs]),
                              np.concatenate([a.ravel() for a in ys]))):
        for rec in (0, 1):
            _train(S, segs, x, y, w, r, S.BF16, rec)  # warm: the library's first call sets up events
            S.profile_select('*')
            try:
                _train(S, segs, x, y, w, r, S.BF16, rec)
                counts[(name, rec)] = sum(n for n, _ in S.profile_report().values())
            finally:
                S.profile_select(None)
    _say('  launches', counts)
    for rec in (0, 1):
        assert counts[('packed', rec)] == counts[('one size', rec)] > 0
