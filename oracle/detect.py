"""FP64 reference of the detection step applied to the restored RD maps: CA-CFAR peak detection
and the fraction of reference peaks it finds (Radar-STDA, arXiv 2307.09063, Sec. V-B).

Test infrastructure only: the product library never imports or calls it.

The paper names the detector (cell-averaging CFAR, Sec. V-B) and the ratio it reports
(correctly detected peaks over reference peaks, Eq. (21)) but no detector parameters, so the
following is a reading:
  * square-law detector: the statistic of a cell is |m|^2 of the map value m (the SINR of
    Eq. (19) is also taken on |m|^2);
  * the training cells of the cell under test (y, x) are the cells of the
    (2(Gr+Tr)+1) x (2(Gd+Td)+1) window centred on it that lie outside the (2Gr+1) x (2Gd+1)
    guard window; the Doppler axis is circular (DFT bins wrap), the range axis is not (rows
    outside the map do not count);
  * with N training cells of mean power P, the cell is a detection when |m|^2 > alpha(N) P,
    alpha(N) = N (Pfa^(-1/N) - 1): for N independent exponentially distributed training cells
    and an exponentially distributed cell under test of the same mean this gives a false-alarm
    probability of exactly Pfa, since P(X > alpha mean) = (1 + alpha / N)^(-N);
  * a reference peak counts as correctly detected when the detector fires at its cell (no
    clustering step: the clustering and labelling of the paper need its dataset).
"""
import numpy as np


def cfar_alpha(n, pfa):
    """Threshold factor of CA-CFAR with n training cells for false-alarm probability pfa."""
    n = np.asarray(n, dtype=np.float64)
    return n * (pfa ** (-1.0 / n) - 1.0)


def cfar_training(power, y, x, gr, gd, tr, td):
    """(sum, count) of the training cells of cell (y, x) of one H x W power map, by definition."""
    H, W = power.shape
    s, n = 0.0, 0
    for dy in range(-(gr + tr), gr + tr + 1):
        yy = y + dy
        if yy < 0 or yy >= H:
            continue
        for dx in range(-(gd + td), gd + td + 1):
            if abs(dy) <= gr and abs(dx) <= gd:
                continue
            s += power[yy, (x + dx) % W]
            n += 1
    return s, n


def cfar(maps, gr, gd, tr, td, pfa):
    """Detection mask (bool, same shape as maps [..., H, W]) and the decision margin
    |m|^2 - alpha N^-1 sum, both from the definition, vectorised over whole rows of offsets."""
    m = np.asarray(maps, dtype=np.float64)
    lead = m.shape[:-2]
    H, W = m.shape[-2:]
    p = (m * m).reshape(-1, H, W)
    det = np.zeros_like(p, dtype=bool)
    margin = np.zeros_like(p)
    rows = np.arange(H)
    for k in range(p.shape[0]):
        tot = np.zeros((H, W))
        cnt = np.zeros((H, 1))
        for dy in range(-(gr + tr), gr + tr + 1):
            src = rows + dy
            ok = (src >= 0) & (src < H)
            for dx in range(-(gd + td), gd + td + 1):
                if abs(dy) <= gr and abs(dx) <= gd:
                    continue
                shifted = np.zeros((H, W))
                shifted[ok] = np.roll(p[k], -dx, axis=1)[src[ok]]
                tot += shifted
                cnt[ok, 0] += 1
        thr = cfar_alpha(cnt, pfa) * tot / cnt
        det[k] = p[k] > thr
        margin[k] = p[k] - thr
    return det.reshape(lead + (H, W)), margin.reshape(lead + (H, W))


def detected_fraction(det, o_mask):
    """Eq. (21) without the percent: detected reference peaks over reference peaks, per map."""
    det = np.asarray(det, dtype=bool)
    o = np.asarray(o_mask, dtype=bool)
    n_o = o.sum(axis=(-2, -1))
    return (det & o).sum(axis=(-2, -1)) / np.maximum(n_o, 1)
