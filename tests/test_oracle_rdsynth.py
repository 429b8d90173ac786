"""Pins of the oracle RD-map synthesizer and metrics: Philox known answers, Box-Muller moments,
Parseval, closed-form Hann tone spectra, brute-force DFT, analytic peak positions and their motion
over the three frames, the physical beat frequency of a converted aggressor record, the ghost case
of identical chirps, the IF gate, and the SINR / EVM closed forms.  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import rdsynth as R
from paper_2307_09063_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def _empty_scene(B, N, M, sigma=0.0, seed=7):
    tab = np.zeros(B, dtype=inputs.SCENE_DTYPE)
    meta = {'seed': np.uint32(seed), 'noise_sigma': sigma, 'N': N, 'M': M, 'peaks': [[]] * B}
    return tab, meta


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, 'philox4x32_10_kat.json')) as f:
        kat = json.load(f)
    for case in kat['cases']:
        c = [int(v, 16) for v in case['ctr']]
        k = [int(v, 16) for v in case['key']]
        out = R.philox4x32_10(*c, *k)
        assert [int(v) for v in out] == [int(v, 16) for v in case['out']]


def test_noise_moments():
    tab, meta = _empty_scene(1, 64, 64, sigma=2.0)
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 1)
    n = s.size
    assert abs(s.mean()) < 5 * 2.0 / np.sqrt(n)
    assert abs((np.abs(s) ** 2).mean() / 4.0 - 1.0) < 5 * np.sqrt(2.0 / n) * 2
    assert abs((s.real ** 2).mean() - (s.imag ** 2).mean()) < 0.1 * 2.0
    assert abs((s.real * s.imag).mean()) < 0.05 * 4.0
    # Gaussian fourth moment of a real component: 3 sigma^4
    k4 = (s.real ** 4).mean() / (s.real ** 2).mean() ** 2
    assert abs(k4 - 3.0) < 0.3
    # a different frame uses a different counter
    s2 = R.beat_signal(inputs.scene_dict(tab, meta), 0, 2)
    assert abs(np.vdot(s, s2)) / n < 0.2


def test_parseval():
    tab, meta = inputs.make_scenes(2, 32, 16, seed=3, intf=(1, 2))
    sc = inputs.scene_dict(tab, meta)
    for b in range(2):
        s = R.beat_signal(sc, b, 0)
        Y = R.rd_spectrum(s)
        sw = s * R.hann_periodic(32)[:, None] * R.hann_periodic(16)[None, :]
        assert abs((np.abs(Y) ** 2).sum() - 32 * 16 * (np.abs(sw) ** 2).sum()) < 1e-9 * (np.abs(Y) ** 2).sum()


@pytest.mark.parametrize('N,M,p0,q0', [(16, 8, 3, 2), (32, 32, 0, 31), (64, 16, 17, 5)])
def test_unit_tone_hann_closed_form(N, M, p0, q0):
    tab, meta = _empty_scene(1, N, M)
    t = tab[0]['tone'][0, 0]
    t['fr'] = p0 * (2 ** 32 // N)
    t['fd'] = q0 * (2 ** 32 // M)
    t['amp'] = 1.0
    tab[0]['n_tones'][0] = 1
    Y = R.rd_spectrum(R.beat_signal(inputs.scene_dict(tab, meta), 0, 0))
    expect = np.zeros((N, M), dtype=complex)
    wn = {0: N / 2, 1: -N / 4, -1: -N / 4}
    wm = {0: M / 2, 1: -M / 4, -1: -M / 4}
    for a, va in wn.items():
        for b, vb in wm.items():
            expect[(p0 + a) % N, (q0 + b + M // 2) % M] += va * vb
    np.testing.assert_allclose(Y, expect, atol=1e-9 * N * M)
    # rectangular window: a single bin of amplitude N*M
    Yr = R.rd_spectrum(R.beat_signal(inputs.scene_dict(tab, meta), 0, 0), window=False)
    er = np.zeros((N, M), dtype=complex)
    er[p0, (q0 + M // 2) % M] = N * M
    np.testing.assert_allclose(Yr, er, atol=1e-9 * N * M)


def test_fft_equals_brute_dft():
    tab, meta = inputs.make_scenes(1, 8, 8, seed=4, intf=(1, 1))
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 0)
    sw = s * R.hann_periodic(8)[:, None] * R.hann_periodic(8)[None, :]
    Y = np.zeros((8, 8), dtype=complex)
    for p in range(8):
        for q in range(8):
            for n in range(8):
                for m in range(8):
                    Y[p, q] += sw[n, m] * np.exp(-2j * np.pi * (n * p / 8 + m * q / 8))
    np.testing.assert_allclose(R.rd_spectrum(s), np.roll(Y, 4, axis=1), atol=1e-10)
    # a 1-based index (as printed) changes the phase only
    Y1 = np.zeros((8, 8), dtype=complex)
    for p in range(8):
        for q in range(8):
            for n in range(8):
                for m in range(8):
                    Y1[p, q] += sw[n, m] * np.exp(-2j * np.pi * ((n + 1) * p / 8 + (m + 1) * q / 8))
    np.testing.assert_allclose(np.abs(Y1), np.abs(Y), atol=1e-10)


def test_normalisation_range_and_floor():
    tab, meta = inputs.make_scenes(1, 64, 32, seed=5)
    x, clean = R.synth_clip(inputs.scene_dict(tab, meta), 0)
    for m in list(x) + list(clean):
        assert m.max() == 1.0 and m.min() == 0.0
    Y = np.zeros((4, 4), dtype=complex)
    Y[1, 2] = 10.0
    out = R.normalise_db(Y)              # zeros sit on the floor, the peak at 1
    assert out[1, 2] == 1.0 and out.sum() == 1.0
    assert not R.normalise_db(np.zeros((4, 4))).any()


def test_target_peak_positions():
    """Noise-free single targets peak at (round(r N), M/2 + round(d M)) in frame t."""
    rng = np.random.default_rng(9)
    for trial in range(6):
        tab, meta = inputs.make_scenes(1, 64, 32, seed=100 + trial, targets=(1, 1), intf=(0, 0))
        sc = inputs.scene_dict(tab, meta)
        sc['noise_sigma'] = 0.0
        Y = np.abs(R.rd_spectrum(R.beat_signal(sc, 0, 0)))
        p, q = np.unravel_index(np.argmax(Y), Y.shape)
        ep, eq = meta['peaks'][0][0]
        assert abs(((p - ep + 32) % 64) - 32) <= 1 and abs(((q - eq + 16) % 32) - 16) <= 1


def test_target_motion_across_frames():
    """A target of radial velocity v (in units of v_max, the sign of its Doppler bin offset) moves
    v kappa_f range units per frame, kappa_f = v_max T_frame / R_max (Sec. V-A): the RD peak of
    frame t - f sits at the range bin nearest (r - f v kappa_f) N, r = the frame-t range read back
    from the tone table as f_r / 2^32 and v = 2 f_d / 2^32, and at the same Doppler bin in all
    three frames.  At N = 256
    a target at the velocity limit moves 2.5 bins a frame, so a dropped or reversed frame term
    moves the peak by 2 bins or more."""
    N, M = 256, 32
    moved = 0
    for trial in range(8):
        tab, meta = inputs.make_scenes(1, N, M, seed=300 + trial, targets=(1, 1), intf=(0, 0))
        sc = inputs.scene_dict(tab, meta)
        sc['noise_sigma'] = 0.0
        r = int(tab[0]['tone']['fr'][0, 0]) / 2.0 ** 32
        fd = int(tab[0]['tone']['fd'][0, 0])
        v = 2.0 * (fd - 2 ** 32 if fd >= 2 ** 31 else fd) / 2.0 ** 32
        qs = set()
        for f in range(3):
            Y = np.abs(R.rd_spectrum(R.beat_signal(sc, 0, f)))
            p, q = np.unravel_index(np.argmax(Y), Y.shape)
            ep = (r - f * v * inputs.KAPPA_F) * N
            assert abs(((p - ep + N / 2) % N) - N / 2) <= 0.5 + 1e-9, (trial, f, p, ep)
            qs.add(int(q))
        assert len(qs) == 1 and abs(((qs.pop() - meta['peaks'][0][0][1] + M // 2) % M) - M // 2) <= 1
        moved += abs(v) * inputs.KAPPA_F * N > 1.0
    assert moved >= 3


def test_ghost_identical_chirps():
    """Identical chirp slopes (q = 0) with no chirp-to-chirp step give a constant beat tone at
    f0 in every chirp: after the range transform all energy sits in range bin round(f0 N)."""
    N, M = 32, 16
    tab, meta = _empty_scene(1, N, M)
    e = tab[0]['intf'][0, 0]
    e['q'], e['dl'], e['f0'], e['amp'] = 0, 0, int(round(0.3125 * 2 ** 32)), 1.0
    tab[0]['n_intf'][0] = 1
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 0)
    prof = (np.abs(np.fft.fft(s, axis=0)) ** 2).sum(axis=1)
    assert np.argmax(prof) == 10 and prof[10] > 0.999 * prof.sum()
    # a frequency outside the IF band is gated out entirely
    e['f0'] = int(round(0.75 * 2 ** 32))
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 0)
    assert not s.any()


def test_interferer_phase_exact_integers():
    """The vectorised wrap-around phase equals the phase computed with unbounded integers."""
    N, M = 16, 8
    tab, meta = _empty_scene(1, N, M, seed=11)
    e = tab[0]['intf'][0, 0]
    e['q'], e['f0'], e['dl'], e['amp'] = -123456789, -987654321, 55555555, 1.0
    tab[0]['n_intf'][0] = 1
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 0)
    phi = R.philox4x32_10(np.arange(M), 0, 0, 1, 11, 0)[0]
    for n in range(N):
        for m in range(M):
            F = 2 * e['q'] * n + e['f0'] + m * e['dl']
            if abs(int(F)) >= 2 ** 31:
                assert s[n, m] == 0
                continue
            P = (int(e['f0']) + m * int(e['dl'])) * n + int(e['q']) * n * n + int(phi[m])
            P %= 2 ** 32
            ang = 2 * np.pi * ((P - 2 ** 32 if P >= 2 ** 31 else P) / 2 ** 32)
            assert abs(s[n, m] - np.exp(1j * ang)) < 1e-12


def test_sinr_and_evm_closed_form():
    z = np.full((8, 8), 0.1)
    o = np.zeros((8, 8), dtype=bool)
    o[2, 3] = o[5, 6] = True
    z[o] = 0.8
    n = ~o
    assert abs(R.sinr_db(z, o, n) - 20 * np.log10(8.0)) < 1e-12
    clean = np.ones((8, 8))
    assert abs(R.evm(clean, z, o) - 0.2) < 1e-12


# ------------------------------------------------ physical-units aggressors (Tables 2 and 4)
def _aggressor_only(scenario, N, M, beat0):
    tab, meta = inputs.table2_scene(scenario, N, M, seed=5, amp=1.0, beat0=beat0, noise_sigma=0.0)
    tab[0]['tone']['amp'] = 0.0
    sc = inputs.scene_dict(tab, meta)
    s = R.beat_signal(sc, 0, 0)
    Y = np.abs(R.rd_spectrum(s)) ** 2
    return s, Y


def test_sawtooth_and_coherent_phase_exact_integers():
    """Sawtooth start frequency and coherent phase against unbounded-integer arithmetic."""
    N, M = 16, 12
    tab, meta = _empty_scene(1, N, M, seed=3)
    e = tab[0]['intf'][0, 0]
    e['q'], e['f0'], e['dl'] = -12345678, -3 * 2 ** 31, 7 * 2 ** 32 + 123457
    e['s0'], e['wrap'] = 2 ** 32 + 99, 5 * 2 ** 31 + 17
    e['ph0'], e['phd'], e['coherent'], e['amp'] = 4000000000, 3000000001, 1, 1.0
    tab[0]['n_intf'][0] = 1
    s = R.beat_signal(inputs.scene_dict(tab, meta), 0, 0)
    hit = 0
    for m in range(M):
        g = int(e['f0']) + (int(e['s0']) + m * int(e['dl'])) % int(e['wrap'])
        for n in range(N):
            F = 2 * int(e['q']) * n + g
            if abs(F) >= 2 ** 31:
                assert s[n, m] == 0
                continue
            hit += 1
            P = (g * n + int(e['q']) * n * n + int(e['ph0']) + m * int(e['phd'])) % 2 ** 32
            ang = 2 * np.pi * ((P - 2 ** 32 if P >= 2 ** 31 else P) / 2 ** 32)
            assert abs(s[n, m] - np.exp(1j * ang)) < 1e-12
    assert 0 < hit < N * M


@pytest.mark.parametrize('scenario', [1, 7])
def test_table2_equal_slopes_give_a_zero_doppler_ghost(scenario):
    # equal slopes with a sweep period that divides the chirp period: the same beat every chirp
    N, M = 64, 32
    _, Y = _aggressor_only(scenario, N, M, beat0=0.3125)
    p0 = int(round(0.3125 * N))
    assert Y[p0 - 1:p0 + 2, M // 2 - 1:M // 2 + 2].sum() > 0.99 * Y.sum()


@pytest.mark.parametrize('scenario', [3, 4])
def test_table2_repeated_sweep_gives_a_ridge(scenario):
    # different slopes, the same crossing in every chirp: a ridge along range at zero Doppler
    N, M = 64, 32
    # falling beat (scenario 3) enters the band from above, rising beat (4) must start inside it
    _, Y = _aggressor_only(scenario, N, M, beat0=0.45 if scenario == 3 else 0.1)
    assert Y[:, M // 2 - 1:M // 2 + 2].sum() > 0.99 * Y.sum()
    prof = Y.sum(axis=1)
    assert prof.max() < 0.5 * prof.sum() and (prof > 0.01 * prof.max()).sum() >= N // 8


@pytest.mark.parametrize('scenario', [2, 6])
def test_table2_detuned_period_raises_the_floor(scenario):
    # the crossing moves from chirp to chirp: energy leaves the zero-Doppler columns
    N, M = 64, 128
    s, Y = _aggressor_only(scenario, N, M, beat0=0.45 if scenario == 2 else 0.1)
    assert Y.sum() > 0
    assert Y[:, M // 2 - 1:M // 2 + 2].sum() < 0.5 * Y.sum()


def test_table2_carrier_offset_moves_the_beat_out_of_band():
    # scenario 5 with the ramp timing of the in-band ghost of scenario 1: the 20 MHz carrier
    # offset (1.6 cycles/sample at 12.5 MHz) puts the beat outside the IF band at every sample
    s1, _ = _aggressor_only(1, 64, 32, beat0=0.3125)
    s5, _ = _aggressor_only(5, 64, 32, beat0=0.3125)
    assert s1.any() and not s5.any()


def test_table4_draws_and_amplitude():
    tab, meta = inputs.make_scenes_table4(16, 64, 128, seed=9)
    for b, a in enumerate(meta['aggressor']):
        assert a['sir_db'] in range(-5, 30, 5)
        assert 76.8e9 - 1 <= a['fc'] <= 77.2e9 + 1 and round((a['fc'] - 76.8e9) / 0.1e9, 6).is_integer()
        assert 120e6 <= a['bandwidth'] <= 400e6 and 4e-6 <= a['duration'] <= 30e-6
        assert 2 <= a['distance'] <= 63 and -23.05 <= a['velocity'] <= 0
        nt = tab[b]['n_tones'][0]
        p_sig = np.mean(tab[b]['tone'][0, :nt]['amp'].astype(np.float64) ** 2)
        amp = float(tab[b]['intf'][0, 0]['amp'])
        assert abs(amp ** 2 - p_sig / 10 ** (a['sir_db'] / 10)) <= 1e-6 * amp ** 2
        e = tab[b]['intf'][0, 0]
        assert e['coherent'] == 1 and abs(e['wrap'] / 2 ** 32 - a['bandwidth'] / inputs.F_S) < 1e-8


def test_aggressor_record_matches_the_physical_beat_frequency():
    """The interferer record built from an aggressor's physical parameters (carrier, sweep
    bandwidth and duration, radial velocity, ramp timing; Sec. III-A's beat of the aggressor ramp
    against the victim ramp) against the beat frequency evaluated from first principles: at victim
    sample n of chirp m (time m T_chirp + n / f_s) the aggressor sits at f_c,i + f_D + S_i ((t -
    t_off) mod T_i), the victim at f_c + S_v n / f_s, S_v = B f_s / N, f_D = -v f_c,i / c.  Checked
    (1) on the record's integer fields as the synthesizer reads them (2 q n + f0 + (s0 + m dl) mod
    wrap), and (2) on the oracle's synthesized interference itself, whose phase advances between
    samples n and n + 1 by the physical beat at n + 1/2; wherever the aggressor ramp does not
    restart inside the chirp."""
    rng = np.random.default_rng(21)
    N, M = 256, 16
    checked = recs = 0
    for trial in range(6):
        fc_i = inputs.FC_VICTIM + rng.uniform(-1.5e6, 1.5e6)
        t_i = rng.uniform(30e-6, 60e-6)          # longer than a chirp: at most one restart in it
        b_i = rng.uniform(0.8, 1.2) * inputs.B_VICTIM * inputs.F_S / N * t_i   # slope near the victim's
        v = rng.uniform(-23.0, 23.0)
        t_off = rng.uniform(0.0, t_i)
        tab, meta = inputs.make_scenes(1, N, M, seed=40 + trial, targets=(1, 1), intf=(0, 0))
        for f in range(3):
            tab[0]['n_tones'][f] = 0
            tab[0]['n_intf'][f] = 1
            inputs.aggressor_record(tab[0]['intf'][f, 0], N, fc_i, b_i, t_i, v, t_off, rng.random(), 1.0)
        e = tab[0]['intf'][0, 0]
        q, f0, dl, s0, wrap = (int(e[k]) for k in ('q', 'f0', 'dl', 's0', 'wrap'))
        n = np.arange(N)
        s_v = inputs.B_VICTIM * inputs.F_S / N
        f_d = -v * fc_i / inputs.C_LIGHT
        sc = inputs.scene_dict(tab, meta)
        sc['noise_sigma'] = 0.0
        s = R.beat_signal(sc, 0, 0)
        for m in range(M):
            tm = m * inputs.T_CHIRP + n / inputs.F_S
            ramp = (tm - t_off) % t_i
            beat = (fc_i + f_d + b_i / t_i * ramp - inputs.FC_VICTIM - s_v * n / inputs.F_S) / inputs.F_S
            no_restart = ((m * inputs.T_CHIRP - t_off) % t_i) + n / inputs.F_S < t_i
            rec = (2 * q * n + f0 + (s0 + m * dl) % wrap) / 2.0 ** 32
            assert np.abs(rec - beat)[no_restart].max() < 1e-6, (trial, m)
            recs += int(no_restart.sum())
            # the synthesized signal: phase step between n and n + 1 = beat at n + 1/2 (mod 1)
            mid = (beat[:-1] + beat[1:]) / 2
            ok = no_restart[:-1] & no_restart[1:] & (np.abs(rec[:-1]) < 0.5) & (np.abs(rec[1:]) < 0.5)
            with np.errstate(divide='ignore', invalid='ignore'):
                step = np.angle(s[1:, m] / s[:-1, m]) / (2 * np.pi)
            d = (step - mid + 0.5) % 1.0 - 0.5
            assert np.abs(d[ok]).max() < 1e-6 if ok.any() else True, (trial, m)
            checked += int(ok.sum())
    assert recs > 5000 and checked > 100, (recs, checked)
