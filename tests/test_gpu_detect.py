"""GPU detection step against the oracle: CA-CFAR masks and counts (tests/ ... oracle/detect.py),
EVM (oracle/rdsynth.py).  CFAR decisions are compared cell by cell except where the oracle's own
decision margin |p - threshold| is below 1e-9 of the threshold: there FP64 sums taken in another
order may legitimately decide the other way (none were met in these inputs in practice; the
test reports how many were excluded)."""
import sys

import numpy as np
import pytest
import torch

from oracle import detect, rdsynth
from paper_2307_09063_amd import inputs
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_cfar(S, maps, params, o_mask=None):
    n, H, W = maps.shape
    md = U.dev(maps.astype(np.float32))
    det = torch.empty((n, H, W), dtype=torch.uint8, device='cuda')
    counts = torch.empty((n, 2), dtype=torch.int32, device='cuda')
    om = U.dev(o_mask.astype(np.uint8)) if o_mask is not None else None
    S.cfar(md, det, *params, o_mask=om, counts=counts)
    torch.cuda.synchronize()
    g = det.cpu().numpy().astype(bool)
    ref, margin = detect.cfar(maps.astype(np.float32).astype(np.float64), *params)
    thr = (maps.astype(np.float32).astype(np.float64) ** 2) - margin
    ambiguous = np.abs(margin) <= 1e-9 * np.maximum(np.abs(thr), 1e-300)
    assert np.array_equal(g[~ambiguous], ref[~ambiguous])
    c = counts.cpu().numpy()
    np.testing.assert_array_equal(c[:, 0], g.sum(axis=(1, 2)))
    if o_mask is not None:
        np.testing.assert_array_equal(c[:, 1], (g & o_mask).sum(axis=(1, 2)))
    else:
        assert not c[:, 1].any()
    return g, int(ambiguous.sum())


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import stda
    return stda


@pytest.mark.parametrize('params', [(2, 2, 4, 4, 1e-3), (0, 1, 3, 2, 1e-2), (1, 0, 0, 5, 1e-4), (3, 3, 5, 5, 1e-3)])
def test_cfar_exponential_fields(S, params):
    _say('cfar exp', params)
    rng = np.random.default_rng(7)
    maps = np.sqrt(rng.exponential(1.0, size=(3, 40, 36)))
    g, amb = _check_cfar(S, maps, params)
    _say('  detections', int(g.sum()), 'ambiguous', amb)


def test_cfar_rd_maps_and_peak_hits(S):
    B, N, M = 4, 128, 64
    _say('cfar rd maps')
    x, clean, tab, meta = U.rd_maps(B, N, M, seed=41, intf=(1, 2))
    o = np.stack([inputs.sinr_masks(meta['peaks'][b], N, M)[0] for b in range(B)])
    for maps in (x[:, 0], clean[:, 0]):
        g, amb = _check_cfar(S, maps, (2, 2, 4, 4, 1e-3), o_mask=o)
        _say('  hits', (g & o).sum(axis=(1, 2)), 'of', o.sum(axis=(1, 2)), 'ambiguous', amb)


@pytest.mark.parametrize('shape', [(1, 17, 17), (2, 64, 128), (1, 257, 70)])
def test_cfar_edges_and_window_fit(S, shape):
    _say('cfar edges', shape)
    rng = np.random.default_rng(shape[1])
    maps = rng.random(shape)
    maps[:, 0, 0] = 5.0
    maps[:, -1, -1] = 5.0
    _check_cfar(S, maps, (2, 2, 6, 6, 1e-3))   # 17 x 17 window: fits the smallest map exactly


def test_evm(S):
    B, N, M = 3, 64, 64
    _say('evm')
    x, clean, tab, meta = U.rd_maps(B, N, M, seed=42)
    o = np.stack([inputs.sinr_masks(meta['peaks'][b], N, M)[0] for b in range(B)])
    o[2] = False   # a map without reference cells gives 0
    out = torch.empty(B, dtype=torch.float64, device='cuda')
    S.evm(U.dev(x[:, 0]), U.dev(clean[:, 0]), U.dev(o.astype(np.uint8)), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b in range(2):
        ref = rdsynth.evm(clean[b, 0].astype(np.float64), x[b, 0].astype(np.float64), o[b])
        assert abs(got[b] - ref) <= 1e-12 * abs(ref)
    assert got[2] == 0.0
