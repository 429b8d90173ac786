"""Seeded synthetic inputs: scene tables for the RD-map synthesizer, initial weights, running
statistics, SINR cell sets and clip-size mixes.

This module draws random numbers and encodes them; it performs none of the method's
arithmetic (no beat-signal synthesis, no transform, no network step).  Both the GPU path and
the test oracle consume what it produces.

Physical constants of the victim radar (Radar-STDA, arXiv 2307.09063, Table 3): sweep
bandwidth 153.6 MHz over a 5.12 us ADC window sampled at 12.5 MHz (kappa_s = B/f_s = 12.288
cycles of sweep per chirp), frame rate 30 fps, maximum range 62.45 m, maximum velocity
23.02 m/s; the chirp repetition interval of 42.24 us (two TDM transmitters of 21.12 us each)
gives T_frame / T_chirp = 789.1.

Normalised scene model:
  * target: range r = D / R_max in U[0.1, 0.9] cycles/sample, v / v_max in U[-0.8, 0.8],
    Doppler d = v / (2 v_max) cycles/chirp, RCS ~ lognormal(0, 1), amplitude
    sigma_n * sqrt(SNR * RCS).  Frame t-k: r - k (v / v_max) kappa_f with
    kappa_f = v_max T_frame / R_max, phase - 2 pi d k T_frame / T_chirp.
  * clutter: N/16 stationary scatterers (d = 0) at r in U[0, 1), each 20 dB above the
    post-transform noise floor (per-sample amplitude 10 sigma_n / sqrt(N M)).
  * interferer with slope ratio rho: chirp-rate difference (1 - rho) kappa_s / N
    cycles/sample^2, start frequency f0 in U[-kappa_s/2, kappa_s/2], chirp-to-chirp step
    delta in U[-0.05, 0.05], INR gives the amplitude sigma_n 10^(INR/20); redrawn per frame
    except rho and INR.
Every frequency and phase is encoded in 32-bit fixed point (cycles * 2^32).
"""
import numpy as np

KAPPA_S = 153.6e6 / 12.5e6          # sweep cycles per chirp (B_SW / f_s)
R_MAX = 62.45
V_MAX = 23.02
T_FRAME = 1.0 / 30.0
T_CHIRP = 42.24e-6
KAPPA_F = V_MAX * T_FRAME / R_MAX
FRAME_CHIRPS = T_FRAME / T_CHIRP

RD_MAX_TONES = 48
RD_MAX_INTF = 4

TONE_DTYPE = np.dtype([('fr', '<u4'), ('fd', '<u4'), ('ph', '<u4'), ('amp', '<f4')], align=True)
INTF_DTYPE = np.dtype([('q', '<i8'), ('f0', '<i8'), ('dl', '<i8'), ('s0', '<i8'), ('wrap', '<i8'),
                       ('ph0', '<u4'), ('phd', '<u4'), ('amp', '<f4'), ('coherent', '<u4')], align=True)
SCENE_DTYPE = np.dtype([('n_tones', '<i4', (3,)), ('n_intf', '<i4', (3,)),
                        ('tone', TONE_DTYPE, (3, RD_MAX_TONES)),
                        ('intf', INTF_DTYPE, (3, RD_MAX_INTF))], align=True)

# Workload recipes: scene parameters of the benchmark configurations.
WORKLOADS = {
    'cfg1_fwd_64x64': dict(B=1, sizes=[(64, 64)], targets=(1, 3), intf=(1, 1), inr=(20.0, 20.0),
                           clutter=False, seed=1),
    'cfg2_fwd_256x128': dict(B=32, sizes=[(256, 128)], targets=(1, 5), intf=(0, 3),
                             inr=(10.0, 30.0), clutter=True, seed=2),
    'cfg3_train_256x128': dict(B=64, sizes=[(256, 128)], targets=(1, 5), intf=(0, 3),
                               inr=(10.0, 30.0), clutter=True, seed=3),
    'cfg4_bf16_train_256x128': dict(B=256, sizes=[(256, 128)], targets=(1, 5), intf=(0, 3),
                                    inr=(10.0, 30.0), clutter=True, seed=4),
    'cfg5_uneven_bf16_train': dict(B=512, sizes=[(128, 64), (256, 128), (512, 256)],
                                   targets=(1, 8), intf=(0, 4), inr=(10.0, 30.0), clutter=True,
                                   seed=5),
}
WEIGHT_SEED = 1234


def _fx(v):
    """Cycles -> unsigned 32-bit fixed point (mod 1 cycle)."""
    return np.uint32(int(np.round(float(v) * 2.0 ** 32)) % 2 ** 32)


def _fx_signed(v):
    return int(np.round(float(v) * 2.0 ** 32))


def make_scenes(n_clips, N, M, seed, targets=(1, 3), intf=(1, 1), inr=(20.0, 20.0),
                clutter=False, snr_db=10.0, rho=(0.5, 1.5), noise_sigma=1.0):
    """Draw n_clips scenes of N samples x M chirps.

    Returns (table, meta): `table` is a numpy array of SCENE_DTYPE (the layout of `rd_scene`);
    `meta` holds the seed, noise sigma, sizes and, per clip, the frame-t target peak bins.
    """
    rng = np.random.default_rng(seed)
    tab = np.zeros(n_clips, dtype=SCENE_DTYPE)
    peaks = []
    for b in range(n_clips):
        nt = int(rng.integers(targets[0], targets[1] + 1))
        ni = int(rng.integers(intf[0], intf[1] + 1))
        r = rng.uniform(0.1, 0.9, nt)
        vr = rng.uniform(-0.8, 0.8, nt)
        rcs = rng.lognormal(0.0, 1.0, nt)
        ph0 = rng.uniform(0.0, 1.0, nt)
        amp = np.float32(noise_sigma) * np.sqrt(10.0 ** (snr_db / 10.0) * rcs)
        d = 0.5 * vr
        ncl = N // 16 if clutter else 0
        cr = rng.uniform(0.0, 1.0, ncl)
        cph = rng.uniform(0.0, 1.0, ncl)
        camp = 10.0 * noise_sigma / np.sqrt(N * M)
        assert nt + ncl <= RD_MAX_TONES and ni <= RD_MAX_INTF
        rhos = rng.uniform(rho[0], rho[1], ni)
        inrs = rng.uniform(inr[0], inr[1], ni)
        for f in range(3):
            k = 0
            for o in range(nt):
                t = tab[b]['tone'][f, k]
                t['fr'] = _fx(r[o] - f * vr[o] * KAPPA_F)
                t['fd'] = _fx(d[o])
                t['ph'] = _fx(ph0[o] - d[o] * f * FRAME_CHIRPS)
                t['amp'] = np.float32(amp[o])
                k += 1
            for o in range(ncl):
                t = tab[b]['tone'][f, k]
                t['fr'] = _fx(cr[o])
                t['fd'] = 0
                t['ph'] = _fx(cph[o])
                t['amp'] = np.float32(camp)
                k += 1
            tab[b]['n_tones'][f] = k
            for i in range(ni):
                e = tab[b]['intf'][f, i]
                e['q'] = _fx_signed(0.5 * (1.0 - rhos[i]) * KAPPA_S / N)
                e['f0'] = _fx_signed(rng.uniform(-KAPPA_S / 2, KAPPA_S / 2))
                e['dl'] = _fx_signed(rng.uniform(-0.05, 0.05))
                e['amp'] = np.float32(noise_sigma * 10.0 ** (inrs[i] / 20.0))
            tab[b]['n_intf'][f] = ni
        peaks.append([(int(np.round(ro * N)) % N, (M // 2 + int(np.round(do * M))) % M)
                      for ro, do in zip(r, d)])
    meta = {'seed': np.uint32(seed & 0xFFFFFFFF), 'noise_sigma': float(noise_sigma), 'N': N,
            'M': M, 'peaks': peaks}
    return tab, meta


# --------------------------------------------------------------- physical-units interferers
# Victim ramp (Table 3): 153.6 MHz swept over the N-sample ADC window at 12.5 MHz (30 MHz/us at
# N = 64), carrier 77 GHz, one victim chirp every T_CHIRP.  An aggressor (Table 4, or the
# ratio scenarios of Table 2) with carrier fc_i, sweep bandwidth B_i over duration T_i (ramps
# back to back), one-way radial velocity v (negative: approaching) and a random ramp timing
# t_off gives, per victim chirp m, the beat frequency (received minus victim, cycles/sample)
#   F(n, m) = (fc_i - fc_v + f_D) / f_s + (S_i u_m) / f_s + (S_i - S_v) n / f_s^2,
#   u_m = (m T_CHIRP - t_off) mod T_i,  S = sweep slope,  f_D = -v fc_i / c,
# i.e. q = (S_i - S_v) / (2 f_s^2), f0 = (fc_i - fc_v + f_D) / f_s, dl = S_i T_CHIRP / f_s,
# s0 = -S_i t_off / f_s, wrap = B_i / f_s, and the two carriers stay coherent from chirp to
# chirp: the relative phase advances by (fc_i - fc_v + f_D) T_CHIRP cycles per victim chirp.
# The aggressor's ramp is taken as continuing through the victim's sampling window (no reset
# inside it).  The amplitude follows the signal-to-interference ratio per sample, relative to
# the mean power of the clip's targets.
F_S = 12.5e6
B_VICTIM = 153.6e6
FC_VICTIM = 77e9
C_LIGHT = 299792458.0
TABLE2 = {  # scenario: (ratio of sweep bandwidth, ratio of sweep duration, carrier offset in Hz)
    1: (1.0, 1.0, 0.0), 2: (1.0, 1.1, 0.0), 3: (1.0, 2.0, 0.0), 4: (2.0, 1.0, 0.0),
    5: (1.0, 1.0, -20e6), 6: (2.0, 1.1, 0.0), 7: (2.0, 2.0, 0.0),
}
T_SWEEP_VICTIM = 21.12e-6   # victim sweep duration (Table 3), the unit of the Table 2 ratios


def aggressor_record(e, N, fc_i, b_i, t_i, v, t_off, ph0, amp):
    """Fill one interferer record from physical aggressor parameters (SI units)."""
    s_v = B_VICTIM * F_S / N
    s_i = b_i / t_i
    f_d = -v * fc_i / C_LIGHT
    base = (fc_i - FC_VICTIM + f_d) / F_S
    wrap = b_i / F_S
    e['q'] = _fx_signed(0.5 * (s_i - s_v) / F_S ** 2)
    e['f0'] = _fx_signed(base)
    e['dl'] = _fx_signed(s_i * T_CHIRP / F_S)
    e['wrap'] = _fx_signed(wrap)
    e['s0'] = _fx_signed((-s_i * t_off / F_S) % wrap)
    e['ph0'] = _fx(ph0)
    e['phd'] = _fx((fc_i - FC_VICTIM + f_d) * T_CHIRP)
    e['coherent'] = 1
    e['amp'] = np.float32(amp)


def make_scenes_table4(n_clips, N, M, seed, targets=(1, 3), clutter=False, snr_db=10.0, noise_sigma=1.0):
    """Scenes with one aggressor per clip drawn from the intervals of Table 4: SIR level
    U{-5, 0, ..., 25} dB, carrier U{76.8, 76.9, ..., 77.2} GHz, sweep bandwidth U[120, 400] MHz,
    sweep duration U[4, 30] us, distance U[2, 63] m (recorded), radial velocity U[-23.05, 0] m/s;
    the ramp timing is redrawn per frame.  Targets and clutter as in make_scenes.  meta['aggressor']
    lists the draws."""
    tab, meta = make_scenes(n_clips, N, M, seed, targets=targets, intf=(0, 0), clutter=clutter, snr_db=snr_db,
                            noise_sigma=noise_sigma)
    rng = np.random.default_rng([seed, 4])
    draws = []
    for b in range(n_clips):
        sir = float(rng.choice(np.arange(-5, 30, 5)))
        fc_i = 76.8e9 + 0.1e9 * int(rng.integers(0, 5))
        b_i = rng.uniform(120e6, 400e6)
        t_i = rng.uniform(4e-6, 30e-6)
        dist = rng.uniform(2.0, 63.0)
        v = rng.uniform(-23.05, 0.0)
        nt = int(tab[b]['n_tones'][0])
        p_sig = float(np.mean(tab[b]['tone'][0, :nt]['amp'].astype(np.float64) ** 2)) if nt else noise_sigma ** 2
        amp = np.sqrt(p_sig / 10.0 ** (sir / 10.0))
        for f in range(3):
            aggressor_record(tab[b]['intf'][f, 0], N, fc_i, b_i, t_i, v, rng.uniform(0.0, t_i), rng.random(), amp)
            tab[b]['n_intf'][f] = 1
        draws.append(dict(sir_db=sir, fc=fc_i, bandwidth=b_i, duration=t_i, distance=dist, velocity=v))
    meta['aggressor'] = draws
    return tab, meta


def table2_scene(scenario, N, M, seed, amp=3.0, beat0=None, noise_sigma=1.0):
    """One clip with one target and the aggressor of Table 2 scenario 1..7 (ratios of sweep
    bandwidth and duration to the victim's, carrier offset), stationary, every frame the same;
    amp is the aggressor's amplitude per sample.
    The ramp timing is random, or chosen so that the aggressor's ramp offset at the victim's chirp
    start is beat0 cycles/sample (beat0 = s(0), the sawtooth value of chirp 0)."""
    rb, rt, dfc = TABLE2[scenario]
    t_i = rt * T_SWEEP_VICTIM
    s_i = rb / rt * (B_VICTIM * F_S / N)    # the victim's slope times the ratio of slopes
    b_i = s_i * t_i
    wrap = b_i / F_S
    tab, meta = make_scenes(1, N, M, seed, targets=(1, 1), intf=(0, 0), noise_sigma=noise_sigma)
    rng = np.random.default_rng([seed, 2])
    t_off = rng.uniform(0.0, t_i) if beat0 is None else ((wrap - beat0) % wrap) * F_S / s_i
    for f in range(3):
        aggressor_record(tab[0]["intf"][f, 0], N, FC_VICTIM + dfc, b_i, t_i, 0.0, t_off, 0.0, amp)
        tab[0]['n_intf'][f] = 1
    meta['aggressor'] = [dict(scenario=scenario, bandwidth=b_i, duration=t_i, t_off=t_off)]
    return tab, meta


def scene_dict(tab, meta):
    """The scene table as plain arrays (the form the oracle reads)."""
    return {
        'N': meta['N'], 'M': meta['M'], 'seed': int(meta['seed']),
        'noise_sigma': meta['noise_sigma'],
        'n_tones': tab['n_tones'], 'n_intf': tab['n_intf'],
        'tone_fr': tab['tone']['fr'], 'tone_fd': tab['tone']['fd'], 'tone_ph': tab['tone']['ph'],
        'tone_amp': tab['tone']['amp'].astype(np.float64),
        'intf_q': tab['intf']['q'], 'intf_f0': tab['intf']['f0'], 'intf_dl': tab['intf']['dl'],
        'intf_s0': tab['intf']['s0'], 'intf_wrap': tab['intf']['wrap'], 'intf_ph0': tab['intf']['ph0'],
        'intf_phd': tab['intf']['phd'], 'intf_coherent': tab['intf']['coherent'],
        'intf_amp': tab['intf']['amp'].astype(np.float64),
    }


def sinr_masks(peaks, N, M, guard=2):
    """SINR cell sets of one clip: O = the frame-t peak bin of every target; N = every cell
    further than `guard` bins from all targets and outside the zero-Doppler columns M/2 +- 1."""
    o = np.zeros((N, M), dtype=bool)
    n = np.ones((N, M), dtype=bool)
    for p, q in peaks:
        o[p, q] = True
        for dp in range(-guard, guard + 1):
            for dq in range(-guard, guard + 1):
                n[(p + dp) % N, (q + dq) % M] = False
    n[:, M // 2 - 1:M // 2 + 2] = False
    return o, n


def make_weights(specs, seed=WEIGHT_SEED):
    """Kaiming-uniform initial weights U(+-sqrt(6 / fan_in)); BN gamma = 1, beta = 0; biases 0.

    specs: ordered (name, shape, fan_in).  Returns a float32 flat vector."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape, fan_in in specs:
        n = int(np.prod(shape))
        if name.endswith('.gamma'):
            out.append(np.ones(n))
        elif name.endswith('.beta') or name.endswith('.b'):
            out.append(np.zeros(n))
        else:
            bound = np.sqrt(6.0 / fan_in)
            out.append(rng.uniform(-bound, bound, n))
    return np.concatenate(out).astype(np.float32)


def make_running(bn_channels):
    """Initial running statistics: per BN layer, C zeros (mean) then C ones (variance)."""
    return np.concatenate([np.concatenate([np.zeros(c), np.ones(c)]) for c in bn_channels]
                          ).astype(np.float32)


def random_maps(shape, seed):
    """Plain uniform [0, 1) maps of a given shape (for shape sweeps that need no scene)."""
    return np.random.default_rng(seed).random(shape).astype(np.float32)


def uneven_sizes(n_clips, sizes, seed):
    """Clip sizes drawn uniformly from `sizes` (a list of (N, M))."""
    rng = np.random.default_rng(seed + 7919)
    idx = rng.integers(0, len(sizes), n_clips)
    return [sizes[i] for i in idx]
