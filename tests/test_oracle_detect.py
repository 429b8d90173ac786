"""Pins of the CA-CFAR oracle (oracle/detect.py) against what the definition and the
statistics fix: the exact false-alarm probability on exponential noise, the threshold factor's
closed form, edge rules (circular Doppler, truncated range), and the per-cell definition."""
import numpy as np
import pytest

from oracle import detect

GR, GD, TR, TD = 2, 2, 4, 4


def test_alpha_gives_pfa_for_exponential_noise_closed_form():
    # P(X > alpha * mean of N exponentials) = (1 + alpha / N)^-N for unit-mean exponentials
    for n in (8, 24, 64, 264):
        for pfa in (1e-2, 1e-3, 1e-6):
            a = detect.cfar_alpha(n, pfa)
            assert abs((1.0 + a / n) ** (-n) - pfa) <= 1e-12 * pfa


def test_false_alarm_rate_on_exponential_noise():
    rng = np.random.default_rng(0)
    pfa = 1e-2
    p = rng.exponential(1.0, size=(16, 96, 96))
    det, _ = detect.cfar(np.sqrt(p), GR, GD, TR, TD, pfa)
    cells = det.size
    rate = det.sum() / cells
    # the cells are not independent (shared training cells), so allow ~6 binomial sigmas
    sigma = np.sqrt(pfa * (1 - pfa) / cells)
    assert abs(rate - pfa) < 6 * sigma + 0.05 * pfa, (rate, pfa)


def test_vectorised_equals_per_cell_definition():
    rng = np.random.default_rng(1)
    m = rng.random((2, 12, 10))
    det, margin = detect.cfar(m, 1, 1, 2, 3, 1e-3)
    for k in range(2):
        p = m[k] ** 2
        for y in range(12):
            for x in range(10):
                s, n = detect.cfar_training(p, y, x, 1, 1, 2, 3)
                thr = detect.cfar_alpha(n, 1e-3) * s / n
                assert det[k, y, x] == (p[y, x] > thr)
                assert abs(margin[k, y, x] - (p[y, x] - thr)) < 1e-12


def test_constant_map_has_no_detections():
    det, _ = detect.cfar(np.full((1, 32, 32), 0.7), GR, GD, TR, TD, 1e-3)
    assert not det.any()


def test_doppler_axis_is_circular():
    H, W = 33, 40
    pfa = 1e-3
    n_full = (2 * (GR + TR) + 1) * (2 * (GD + TD) + 1) - (2 * GR + 1) * (2 * GD + 1)
    c = 1.0
    m = np.full((1, H, W), np.sqrt(c))
    y0 = 16
    # target at Doppler column W - 4; a strong cell at column 1 lies in its training window only
    # through the wrap (offset +5 > guard 2, <= guard + train 6)
    t2 = 0.9 * detect.cfar_alpha(n_full, pfa) * c + 0.1 * 1e6  # above threshold without the spike
    m[0, y0, W - 4] = np.sqrt(t2)
    det, _ = detect.cfar(m, GR, GD, TR, TD, pfa)
    assert det[0, y0, W - 4]
    m[0, y0, 1] = np.sqrt(1e6 * n_full)  # raises the target's training mean by > 1e6
    det, _ = detect.cfar(m, GR, GD, TR, TD, pfa)
    assert not det[0, y0, W - 4]


def test_range_edge_uses_only_rows_inside_the_map():
    H, W = 40, 32
    pfa = 1e-3
    rows_edge = GR + TR + 1          # rows 0 .. GR+TR inside the window of row 0
    n_edge = rows_edge * (2 * (GD + TD) + 1) - (GR + 1) * (2 * GD + 1)
    n_full = (2 * (GR + TR) + 1) * (2 * (GD + TD) + 1) - (2 * GR + 1) * (2 * GD + 1)
    a_edge, a_full = detect.cfar_alpha(n_edge, pfa), detect.cfar_alpha(n_full, pfa)
    assert a_edge > a_full
    amp2 = 0.5 * (a_edge + a_full)   # between the two thresholds (background power 1)
    m = np.ones((1, H, W))
    m[0, 0, 5] = np.sqrt(amp2)
    m[0, 20, 5] = np.sqrt(amp2)
    det, _ = detect.cfar(m, GR, GD, TR, TD, pfa)
    assert det[0, 20, 5] and not det[0, 0, 5]


def test_isolated_peak_on_zero_background():
    m = np.zeros((1, 24, 24))
    m[0, 10, 7] = 0.5
    det, _ = detect.cfar(m, GR, GD, TR, TD, 1e-3)
    assert det.sum() == 1 and det[0, 10, 7]


def test_detected_fraction():
    det = np.zeros((2, 8, 8), dtype=bool)
    o = np.zeros((2, 8, 8), dtype=bool)
    o[0, 1, 1] = o[0, 2, 2] = o[0, 3, 3] = True
    det[0, 1, 1] = det[0, 3, 3] = det[0, 5, 5] = True
    o[1, 4, 4] = True
    np.testing.assert_allclose(detect.detected_fraction(det, o), [2 / 3, 0.0])


@pytest.mark.parametrize('pfa', [1e-2, 1e-4])
def test_more_permissive_pfa_detects_superset(pfa):
    rng = np.random.default_rng(5)
    m = rng.random((1, 40, 48))
    d1, _ = detect.cfar(m, GR, GD, TR, TD, pfa)
    d2, _ = detect.cfar(m, GR, GD, TR, TD, pfa / 10)
    assert np.all(d1 | ~d2)
