"""FP64 reference of the range-Doppler map synthesizer and of the SINR / EVM metrics.

Test infrastructure only: the product library never imports or calls it.

Signal model (Radar-STDA, arXiv 2307.09063, Sec. III-A): the corrupted IF signal is the sum of
target beat tones, interferer terms and complex white Gaussian noise, Eq. (IF signal); a target
term is a 2-D complex tone in fast time n and slow time m, Eq. (discrete signal).  RD processing
(Sec. III-B): a DFT over fast time, Eq. (column transform), then over slow time,
Eq. (row transform).

Normalised encoding of a scene (the scene table the generator hands over; see the field list in
`synth_clip`):
  * tone k of a frame: s(n, m) = a * exp(j 2 pi u / 2^32), u = (fr*n + fd*m + ph) mod 2^32,
    with fr, fd, ph unsigned 32-bit fixed-point cycles (per sample, per chirp, absolute).
  * interferer i of a frame: start beat frequency of chirp m g(m) = f0 + m*dl, or, when
    wrap > 0, g(m) = f0 + ((s0 + m*dl) mod wrap) (the aggressor's own ramp seen at each victim
    chirp start: a sawtooth of span wrap); instantaneous beat frequency F(n, m) = 2*q*n + g(m)
    (signed fixed point, 2^-32 cycles/sample); the term a * exp(j 2 pi P / 2^32) with
    P = g(m)*n + q*n^2 + phi_m mod 2^32 is kept only while |F| < 2^31 (an ideal IF low-pass at
    half the sampling rate after dechirping); phi_m is word 0 of
    Philox4x32-10(counter=(m, i, frame, 1), key=(seed, clip)), or ph0 + m*phd mod 2^32 when
    the record is marked coherent.
  * noise: Philox4x32-10(counter=(n, m, frame, 0), key=(seed, clip)) words 0, 1 -> two
    uniforms -> Box-Muller -> re, im, each scaled by sigma/sqrt(2).
  * periodic Hann window on both axes, 2-D DFT (0-based index; a 1-based index only rotates the
    phase), the zero Doppler bin moved to column M/2, 20*log10|Y|, values below (max - 80 dB)
    raised to that floor, then min-max scaled to [0, 1].
Output channel order: frame t, t-1, t-2; the clean map is frame t without interferers.
"""
import numpy as np

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
FLOOR_DB = 80.0


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round multiplies
    words 0 and 2 by the two round constants, swaps the high halves in with the key, and the
    key is bumped by the Weyl constants between rounds.  Arguments are uint64 arrays (or
    ints) holding 32-bit values; returns four uint64 arrays of 32-bit values."""
    c = [np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    sh = np.uint64(32)
    mk = np.uint64(MASK32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mk
            k1 = (k1 + np.uint64(PHILOX_W1)) & mk
        p0 = m0 * c[0]            # < 2^64, exact in uint64
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> sh, p0 & mk
        hi1, lo1 = p1 >> sh, p1 & mk
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform_open(x):
    """32-bit word -> uniform in (0, 1): top 23 bits, centred in their cell (exact in FP32)."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def uniform_half_open(x):
    """32-bit word -> uniform in [0, 1): top 24 bits."""
    return (np.asarray(x, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def box_muller(u1, u2):
    """Two independent standard normals from u1 in (0, 1] and u2 in [0, 1)."""
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    return r * np.cos(th), r * np.sin(th)


def phase_to_unit(u32):
    """exp(j 2 pi u / 2^32) for 32-bit fixed-point phases u."""
    s = (np.asarray(u32, dtype=np.uint64) & np.uint64(MASK32)).astype(np.int64)
    s = np.where(s >= 2 ** 31, s - 2 ** 32, s)          # signed cycles in [-1/2, 1/2)
    return np.exp(2j * np.pi * (s.astype(np.float64) / 2.0 ** 32))


def hann_periodic(n):
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * np.arange(n) / n))


def beat_signal(scene, clip, frame, with_interference=True):
    """Complex N x M IF signal s(n, m) of one frame of one clip (Eq. (IF signal))."""
    N, M = scene['N'], scene['M']
    n = np.arange(N, dtype=np.uint64)[:, None]
    m = np.arange(M, dtype=np.uint64)[None, :]
    s = np.zeros((N, M), dtype=np.complex128)
    for k in range(int(scene['n_tones'][clip, frame])):
        fr = np.uint64(int(scene['tone_fr'][clip, frame, k]))
        fd = np.uint64(int(scene['tone_fd'][clip, frame, k]))
        ph = np.uint64(int(scene['tone_ph'][clip, frame, k]))
        u = (fr * n + fd * m + ph) & np.uint64(MASK32)
        s += float(scene['tone_amp'][clip, frame, k]) * phase_to_unit(u)
    if with_interference:
        seed = int(scene['seed'])
        for i in range(int(scene['n_intf'][clip, frame])):
            q = int(scene['intf_q'][clip, frame, i])
            f0 = int(scene['intf_f0'][clip, frame, i])
            dl = int(scene['intf_dl'][clip, frame, i])
            wrap = int(scene['intf_wrap'][clip, frame, i]) if 'intf_wrap' in scene else 0
            s0 = int(scene['intf_s0'][clip, frame, i]) if 'intf_s0' in scene else 0
            coherent = int(scene['intf_coherent'][clip, frame, i]) if 'intf_coherent' in scene else 0
            amp = float(scene['intf_amp'][clip, frame, i])
            mm = np.arange(M, dtype=np.int64)
            # start beat frequency of each victim chirp, exact integers (the aggressor's ramp
            # sampled at the chirp starts is a sawtooth of span `wrap` when wrap > 0)
            g = np.array([f0 + m * dl if wrap == 0 else f0 + (s0 + m * dl) % wrap for m in range(M)],
                         dtype=np.int64)
            if coherent:
                ph0 = int(scene['intf_ph0'][clip, frame, i])
                phd = int(scene['intf_phd'][clip, frame, i])
                phi = np.array([(ph0 + m * phd) % 2 ** 32 for m in range(M)], dtype=np.uint64)
            else:
                phi = philox4x32_10(mm.astype(np.uint64), i, frame, 1, seed, clip)[0]
            nn = np.arange(N, dtype=np.int64)[:, None]
            fi = 2 * q * nn + g[None, :]                            # exact int64
            keep = np.abs(fi) < 2 ** 31
            # phase mod 2^32: two's-complement uint64 arithmetic wraps mod 2^64, whose low
            # 32 bits are the value mod 2^32
            u64 = lambda v: np.uint64(v % 2 ** 64)
            nu = np.arange(N, dtype=np.uint64)[:, None]
            gu = g.astype(np.uint64)[None, :]                      # two's complement: g mod 2^64
            with np.errstate(over='ignore'):
                P = (gu * nu + u64(q) * (nu * nu) + phi[None, :]) & np.uint64(MASK32)
            s += np.where(keep, amp * phase_to_unit(P), 0.0)
    seed = int(scene['seed'])
    nn = np.broadcast_to(np.arange(N, dtype=np.uint64)[:, None], (N, M))
    mm = np.broadcast_to(np.arange(M, dtype=np.uint64)[None, :], (N, M))
    w = philox4x32_10(nn, mm, frame, 0, seed, clip)
    g0, g1 = box_muller(uniform_open(w[0]), uniform_half_open(w[1]))
    sig = float(scene['noise_sigma']) / np.sqrt(2.0)
    s += sig * (g0 + 1j * g1)
    return s


def rd_spectrum(s, window=True):
    """Hann-windowed 2-D DFT (fast time then slow time), zero Doppler moved to column M/2."""
    N, M = s.shape
    sw = s * hann_periodic(N)[:, None] * hann_periodic(M)[None, :] if window else s
    y = np.fft.fft(sw, axis=0)          # Eq. (column transform): over n for every chirp m
    y = np.fft.fft(y, axis=1)           # Eq. (row transform): over m for every range bin p
    return np.roll(y, M // 2, axis=1)


def normalise_db(Y):
    """20 log10 |Y|, floored at (max - 80 dB), min-max scaled to [0, 1]."""
    mag = np.abs(Y)
    if not np.any(mag > 0):
        return np.zeros(Y.shape)
    with np.errstate(divide='ignore'):
        db = 20.0 * np.log10(mag)
    mx = db.max()
    v = np.maximum(db, mx - FLOOR_DB)
    mn = v.min()
    if mx == mn:
        return np.zeros(Y.shape)
    return (v - mn) / (mx - mn)


def synth_clip(scene, clip):
    """Returns (x [3, N, M] interfered maps t, t-1, t-2, clean [1, N, M] frame t)."""
    x = np.stack([normalise_db(rd_spectrum(beat_signal(scene, clip, f))) for f in range(3)])
    clean = normalise_db(rd_spectrum(beat_signal(scene, clip, 0, with_interference=False)))[None]
    return x, clean


def synth(scene):
    """All clips of a scene table: (x [B, 3, N, M], clean [B, 1, N, M])."""
    xs, cs = zip(*(synth_clip(scene, b) for b in range(scene['n_tones'].shape[0])))
    return np.stack(xs), np.stack(cs)


# --------------------------------------------------------------------- metrics
def sinr_db(z, o_mask, n_mask):
    """SINR of a map (Sec. V-B): 10 log10 of the mean squared value on the target-peak cells O
    over the mean squared value on the noise cells N."""
    z = np.asarray(z, dtype=np.float64)
    po = (z[o_mask] ** 2).mean()
    pn = (z[n_mask] ** 2).mean()
    return 10.0 * np.log10(po / pn)


def evm(clean, est, o_mask):
    """EVM (Sec. V-B): mean over O of |clean - est| / |clean|."""
    c = np.asarray(clean, dtype=np.float64)[o_mask]
    e = np.asarray(est, dtype=np.float64)[o_mask]
    return float((np.abs(c - e) / np.abs(c)).mean())
