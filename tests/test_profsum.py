"""Host logic of the rocprofv3 summariser on small synthetic databases (no GPU)."""
import os
import sqlite3

import pytest

from paper_2307_09063_amd import profsum


def _counter_db(d, rows):
    os.makedirs(d, exist_ok=True)
    con = sqlite3.connect(os.path.join(d, 'run_results.db'))
    con.execute('create table counters_collection (kernel_name text, dispatch_id int, counter_name text, '
                'value real, duration real)')
    con.executemany('insert into counters_collection values (?, ?, ?, ?, ?)', rows)
    con.commit()
    con.close()


def _rows(counters):
    """Two dispatches of kernel A, one of kernel B; each counter value is per (kernel, dispatch)."""
    out = []
    for disp, name, dur in ((1, 'void stda::k_a<float>(float*)', 2000.0), (2, 'void stda::k_a<float>(float*)', 4000.0),
                            (3, 'stda::k_b(int)', 1000.0)):
        for cn, val in counters(name, disp).items():
            out.append((name, disp, cn, val, dur))
    return out


def test_counter_sums_and_per_dispatch(tmp_path):
    d = str(tmp_path / 'a')
    _counter_db(d, _rows(lambda n, disp: {'SQ_WAVES': 10.0 * disp, 'SQ_INSTS_VALU': 100.0 * disp,
                                          'FETCH_SIZE': 7.0 + disp}))
    sums = profsum.counter_sums(d)
    c, n, t = sums['void k_a<float>']
    assert n == 2 and t == pytest.approx(6000.0)
    assert c['SQ_WAVES'] == pytest.approx(30.0) and c['SQ_INSTS_VALU'] == pytest.approx(300.0)
    cb, nb, tb = sums['k_b']
    assert nb == 1 and cb['SQ_WAVES'] == pytest.approx(30.0) and tb == pytest.approx(1000.0)
    mean, cnt = profsum.counter_per_dispatch(d, 'FETCH_SIZE', 'void k_a<float>')
    assert cnt == 2 and mean == pytest.approx((8.0 + 9.0) / 2)
    with pytest.raises(SystemExit):
        profsum.counter_per_dispatch(d, 'FETCH_SIZE', 'k_missing')


def test_counters_table(tmp_path, capsys):
    a, b = str(tmp_path / 'A'), str(tmp_path / 'B')
    _counter_db(a, _rows(lambda n, disp: {'SQ_WAVES': 4.0, 'SQ_INSTS_VALU': 40.0, 'SQ_INSTS_MFMA': 8.0,
                                          'SQ_INSTS_LDS': 12.0, 'SQ_INSTS_VMEM_RD': 2.0, 'SQ_WAVE_CYCLES': 1000.0}))
    _counter_db(b, _rows(lambda n, disp: {'SQ_WAIT_ANY': 500.0, 'SQ_WAIT_INST_LDS': 100.0,
                                          'SQ_ACTIVE_INST_VALU': 250.0}))
    profsum.main(['counters', '--a', a, '--b', b])
    lines = [l for l in capsys.readouterr().out.splitlines() if l.startswith('void k_a')]
    f = lines[0].split()
    # n, us, VALU, MFMA, LDS, VMEM per wave (sums over both dispatches / 8 waves), then the shares
    assert f[-9:] == ['2', '3.0', '10', '2', '3', '0', '50.0', '10.0', '25.0']


def test_trace_rows(tmp_path):
    d = str(tmp_path / 't')
    os.makedirs(d)
    con = sqlite3.connect(os.path.join(d, 'run_results.db'))
    con.execute('create table kernels (name text, duration real, vgpr_count int, lds_size int)')
    con.executemany('insert into kernels values (?, ?, ?, ?)',
                    [('stda::k_x(int)', 10.0, 32, 0), ('stda::k_x(int)', 30.0, 40, 0), ('k_y', 5.0, 8, 1024)])
    con.commit()
    con.close()
    rows = profsum.trace_rows(d)
    assert rows[0] == ('k_x', 2, 40.0, 20.0, 40, 0) and rows[1][0] == 'k_y'


def test_kernel_tag_mapping():
    """Kernel names as rocprofv3 prints them map to bench.py's profiling tags (the block follows
    from the template's channel counts), so per-kernel counters meet the algorithmic work."""
    cases = {
        'void k_s2_tile<float, 3, 32, 64, 16, 8, 8, false, 4>': 'dense_dgrad_main.dec0',
        'void k_s2_tile<bf16, 0, 16, 32, 32, 8, 32, true, 4>': 'dense_fwd_main.enc0',
        'void k_dense_mfma<float, 1, 64, 32, 4, true>': 'dense_fwd_main.dec0',
        'void k_s2_wgrad_v<bf16, true, 32, 16, 8, 16>': 'wgrad_main.dec1',
        'void k_s2_wgrad<float, false, 64, 32, 8, 8>': 'wgrad_main.enc1',
        'void k_s1_bwd_fused<float, 16, false, true, 8, 16, 2>': 's1_bwd_fused.enc0',
        'void k_s1_bwd_stats_tile<bf16, 64, true>': 's1_bwd_stats.dec0',
        'void k_s1_tile<float, 32, true, 0>': 's1_stats.dec1',
        'void k_s1_tile<float, 32, false, 1>': 's1_apply.enc1',
        'void k_eca_next<float, 32, true>': 'eca_next.dec0',
        'void k_eca_next<float, 32, false>': 'eca_next.enc0',
        'void k_s2_bwd_apply<float, 16>': 's2_bwd_apply.dec1',
        'void k_stem_tile<float, 2>': 'stem_bwd_stats',
        'void k_head_fwd_tile<float, false>': 'head_fwd',
        'k_bn_stats_reduce': None,
    }
    for name, tag in cases.items():
        assert profsum.kernel_tag(name) == tag, name
