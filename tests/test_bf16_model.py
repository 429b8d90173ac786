"""CPU pins of the BF16 storage model (tests/bf16_model.py): its rounding is round-to-nearest-even
to 8 significant bits, and with the rounding removed its forward, running statistics and (through
the oracle's adjoint on its cache) gradient are exactly the FP64 oracle's."""
import numpy as np

from oracle import net
from tests import bf16_model as M
from tests import gpu_util as U


def test_bf16_rounding():
    e = 2.0 ** -7  # BF16 spacing in [1, 2)
    v = np.array([1.0, 1.0 + e / 2, 1.0 + 1.5 * e, 1.0 + 0.49 * e, 1.0 + 0.51 * e, -3.0 - 0.51 * 2 * e, 0.0, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1.0 + 2 * e, 1.0, 1.0 + e, -3.0 - 2 * e, 0.0, 2.0 ** -130])
    np.testing.assert_array_equal(M.bf16(v), want)
    r = np.random.default_rng(0).standard_normal(10000)
    q = M.bf16(r)
    assert np.all(np.abs(q - r) <= np.abs(r) * 2.0 ** -8)                  # half a spacing
    assert np.all((q.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)    # 8 significant bits


def test_model_without_rounding_is_the_oracle(monkeypatch):
    monkeypatch.setattr(M, '_bf16', lambda a: np.asarray(a, np.float64))
    x, _ = U.maps(2, 16, 12, seed=5)
    w, r = U.weights(), U.running()
    g = np.random.default_rng(7).standard_normal((2, 1, 16, 12))
    for mode in ('train', 'eval'):
        z, rr, cache = net.forward(w, r, x, mode)
        zm, cm = M.forward(w, r, x, mode)
        assert np.abs(zm - z).max() <= 1e-12 * np.abs(z).max()
        assert np.abs(cm['running'] - rr).max() <= 1e-12 * np.abs(rr).max()
        if mode == 'train':
            gr, dxr = net.backward(g, cache, want_dx=True)
            gm, dxm = net.backward(g, cm, want_dx=True)
            assert np.abs(gm - gr).max() <= 1e-10 * np.abs(gr).max()
            assert np.abs(dxm - dxr).max() <= 1e-10 * np.abs(dxr).max()


def test_model_rounding_error_is_bf16_sized():
    x, _ = U.maps(2, 32, 24, seed=6)
    w, r = U.weights(), U.running()
    z, _, _ = net.forward(w, r, x, 'train')
    e = U.rel_l2(M.forward(w, r, x, 'train')[0], z)
    assert 1e-4 < e < 2e-2
