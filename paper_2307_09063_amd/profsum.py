"""Summaries of rocprofv3 output databases (SQLite, ``-d DIR``).

    python -m paper_2307_09063_amd.profsum trace DIR [--top N]
        per-kernel dispatch count, total and average duration, VGPRs and LDS of a
        ``--kernel-trace`` run
    python -m paper_2307_09063_amd.profsum traffic --fetch DIR --write DIR \
            --copy-fetch DIR --copy-write DIR --copy-bytes N --kernel NAME --tag TAG --workload NAME \
            --bench-log FETCH_LOG --bench-log WRITE_LOG [--out FILE]
        HBM bytes per dispatch of one kernel from a ``--pmc FETCH_SIZE`` run and a
        ``--pmc WRITE_SIZE`` run, each scaled by the factor that makes the same counter read
        exactly N bytes for a plain device copy of N bytes (``bench.py --copy-calib``)

    python -m paper_2307_09063_amd.profsum layers --fetch DIR --write DIR --trace DIR \
            --copy-fetch DIR --copy-write DIR --copy-bytes N --workload NAME [--top N]
        per network kernel of a training step: algorithmic bytes (bench.py's table), HBM bytes
        per dispatch from FETCH_SIZE / WRITE_SIZE (calibrated on a device copy as above), the
        bandwidth they give over the trace run's mean duration, and the matrix-core busy share
        (the derived counter MfmaUtil, taken in the FETCH_SIZE run)

    python -m paper_2307_09063_amd.profsum counters --a DIR --b DIR [--top N]
        per-kernel instruction mix and stall shares from two ``--pmc`` runs of the same command:
        A = SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_MFMA SQ_INSTS_SALU
            SQ_WAVE_CYCLES SQ_BUSY_CYCLES,
        B = SQ_WAIT_INST_LDS SQ_WAIT_INST_ANY SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VALU
            SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE SQ_INST_LEVEL_VMEM SQ_WAIT_ANY

The traffic summary carries the SHA-256 of the library sources it was taken on and the tiling
variant the autotuner chose for the kernel; bench.py reports it only while both still hold."""
import argparse
import glob
import json
import os
import re
import sqlite3
import sys


def _db(d):
    found = sorted(glob.glob(os.path.join(d, '**', '*.db'), recursive=True))
    if not found:
        raise SystemExit(f'no rocprofv3 database under {d}')
    return sqlite3.connect(found[0])


def short_name(name):
    s = re.sub(r'\(.*', '', name)
    return s.replace('stda::', '').replace('(anonymous namespace)::', '').strip()


def trace_rows(d):
    con = _db(d)
    q = ('select name, count(*), sum(duration), avg(duration), max(vgpr_count), max(lds_size) '
         'from kernels group by name order by sum(duration) desc')
    return [(short_name(n), c, s, a, v, l) for n, c, s, a, v, l in con.execute(q).fetchall()]


def counter_per_dispatch(d, counter, match):
    """Mean over dispatches of `counter` (KiB) for kernels whose short name equals `match`."""
    con = _db(d)
    rows = con.execute('select kernel_name, dispatch_id, value from counters_collection where counter_name = ?',
                       (counter,)).fetchall()
    per = {}
    for name, disp, v in rows:
        if short_name(name) == match:
            per[disp] = per.get(disp, 0.0) + v
    if not per:
        raise SystemExit(f'{counter}: no dispatch of {match!r} in {d}')
    return sum(per.values()) / len(per), len(per)


def cmd_trace(a):
    rows = trace_rows(a.dir)
    tot = sum(r[2] for r in rows)
    print(f'total kernel time {tot / 1e6:.3f} ms over {sum(r[1] for r in rows)} dispatches')
    print(f'{"share":>6} {"calls":>6} {"avg_us":>9} {"vgpr":>5} {"lds_B":>6}  kernel')
    for n, c, s, av, v, l in rows[:a.top]:
        print(f'{100 * s / tot:5.1f}% {c:6d} {av / 1e3:9.1f} {v:5d} {l:6d}  {n}')


def cmd_traffic(a):
    fetch, nf = counter_per_dispatch(a.fetch, 'FETCH_SIZE', a.kernel)
    write, nw = counter_per_dispatch(a.write, 'WRITE_SIZE', a.kernel)
    cf, _ = counter_per_dispatch(a.copy_fetch, 'FETCH_SIZE', a.copy_kernel)
    cw, _ = counter_per_dispatch(a.copy_write, 'WRITE_SIZE', a.copy_kernel)
    f_fac = a.copy_bytes / (cf * 1024.0)
    w_fac = a.copy_bytes / (cw * 1024.0)
    hbm = fetch * 1024.0 * f_fac + write * 1024.0 * w_fac
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    # the tiling the autotuner chose for this kernel in the counter runs (their bench.py logs)
    key = bench.tile_key(a.tag)
    chosen = set()
    for log in a.bench_log:
        with open(log) as f:
            lines = [ln for ln in f if ln.startswith('{')]
        if not lines:
            raise SystemExit(f'no bench.py result line in {log}')
        chosen.add((json.loads(lines[-1])['config'].get('tiles') or {}).get(key, 0))
    if len(chosen) != 1:
        raise SystemExit(f'the counter runs chose different tilings for {key}: {sorted(chosen)}')
    out = {'kernel_tag': a.tag, 'workload': a.workload, 'kernel': a.kernel, 'source_sha256': bench.source_hash(),
           'tile_key': key, 'tile_variant': chosen.pop(),
           'fetch_kib_per_dispatch': round(fetch, 1), 'write_kib_per_dispatch': round(write, 1),
           'dispatches': [nf, nw], 'copy_bytes': a.copy_bytes,
           'copy_fetch_kib': round(cf, 1), 'copy_write_kib': round(cw, 1),
           'fetch_factor': round(f_fac, 5), 'write_factor': round(w_fac, 5),
           'hbm_read_bytes_per_launch': round(fetch * 1024.0 * f_fac),
           'hbm_write_bytes_per_launch': round(write * 1024.0 * w_fac),
           'hbm_bytes_per_launch': round(hbm)}
    text = json.dumps(out, indent=1)
    if a.out:
        with open(a.out, 'w') as f:
            f.write(text + '\n')
    print(text)


_BLK = ('enc0', 'enc1', 'dec0', 'dec1')
# (OP, K, N) of the stage-2 GEMM kernels -> block (OP 0/1: forward of encoder / decoder, 2/3:
# their input gradients)
_S2 = {(0, 16, 32): ('dense_fwd', 'enc0'), (0, 32, 64): ('dense_fwd', 'enc1'),
       (1, 64, 32): ('dense_fwd', 'dec0'), (1, 32, 16): ('dense_fwd', 'dec1'),
       (2, 32, 16): ('dense_dgrad', 'enc0'), (2, 64, 32): ('dense_dgrad', 'enc1'),
       (3, 32, 64): ('dense_dgrad', 'dec0'), (3, 16, 32): ('dense_dgrad', 'dec1')}


def kernel_tag(name):
    """bench.py profiling tag (kind.block) of a network kernel's short name, or None.  Launches
    that differ only in their data (main and residual convolutions) share the main one's tag;
    per-level kernels whose width occurs at two blocks of one level take the first."""
    m = re.match(r'(?:void )?(\w+)<(.*)>$', name)
    if not m:
        return {'k_head_fwd_tile': 'head_fwd', 'k_head_bwd_tile': 'head_bwd'}.get(name.replace('void ', ''))
    k, args = m.group(1), [x.strip() for x in m.group(2).split(',')]
    tb = lambda c, dec: {(16, 'false'): 'enc0', (32, 'false'): 'enc1', (64, 'true'): 'dec0',
                         (32, 'true'): 'dec1'}.get((c, dec))
    if k in ('k_s2_tile', 'k_dense_mfma'):
        kind_blk = _S2.get((int(args[1]), int(args[2]), int(args[3])))
        return f'{kind_blk[0]}_main.{kind_blk[1]}' if kind_blk else None
    if k in ('k_s2_wgrad_v', 'k_s2_wgrad'):
        dec, cl, ch = args[1], int(args[2]), int(args[3])
        blk = {('false', 32, 16): 'enc0', ('false', 64, 32): 'enc1', ('true', 64, 32): 'dec0',
               ('true', 32, 16): 'dec1'}.get((dec, cl, ch))
        return f'wgrad_main.{blk}' if blk else None
    if k == 'k_s1_tile':
        blk = tb(int(args[1]), args[2])
        return f'{("s1_stats", "s1_apply")[int(args[3])]}.{blk}' if blk else None
    if k in ('k_s1_bwd_stats_tile', 'k_s1_bwd_fused'):
        blk = tb(int(args[1]), args[2])
        return f'{"s1_bwd_stats" if k == "k_s1_bwd_stats_tile" else "s1_bwd_fused"}.{blk}' if blk else None
    if k == 'k_eca_next':  # the decoder blocks add a skip
        blk = {(32, 'false'): 'enc0', (64, 'false'): 'enc1', (32, 'true'): 'dec0', (16, 'true'): 'dec1'}.get(
            (int(args[1]), args[2]))
        return f'eca_next.{blk}' if blk else None
    if k in ('k_s2_apply', 'k_eca_bwd_part', 'k_s2_bwd_stats', 'k_s2_bwd_apply'):
        blk = {32: 'enc0', 64: 'enc1', 16: 'dec1'}.get(int(args[1]))
        kind = {'k_s2_apply': 's2_apply', 'k_eca_bwd_part': 'eca_bwd', 'k_s2_bwd_stats': 's2_bwd_stats',
                'k_s2_bwd_apply': 's2_bwd_apply'}[k]
        return f'{kind}.{blk}' if blk else None
    if k == 'k_stem_tile':
        return ('stem_stats', 'stem_apply', 'stem_bwd_stats', 'stem_bwd_apply')[int(args[1])]
    if k in ('k_head_fwd_tile', 'k_head_bwd_tile'):
        return 'head_fwd' if k == 'k_head_fwd_tile' else 'head_bwd'
    return None


def per_dispatch(d, counters):
    """{short kernel name: {counter: mean over dispatches of its per-dispatch value}}."""
    con = _db(d)
    acc = {}
    for name, disp, cn, v in con.execute('select kernel_name, dispatch_id, counter_name, value from counters_collection'):
        if cn in counters:
            acc.setdefault(short_name(name), {}).setdefault(cn, {})
            acc[short_name(name)][cn][disp] = acc[short_name(name)][cn].get(disp, 0.0) + v
    return {k: {cn: sum(dv.values()) / len(dv) for cn, dv in cs.items()} for k, cs in acc.items()}


def cmd_layers(a):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    from paper_2307_09063_amd import inputs
    recipe, dt, _ = bench.WORKLOADS[a.workload]
    rc = inputs.WORKLOADS[recipe]
    if len(rc['sizes']) != 1:
        raise SystemExit('layers: a workload of one map size')
    B, (H, W), es = rc['B'], rc['sizes'][0], 2 if dt == 'bf16' else 4
    F = per_dispatch(a.fetch, ('FETCH_SIZE', 'MfmaUtil'))
    Wr = per_dispatch(a.write, ('WRITE_SIZE',))
    cf = per_dispatch(a.copy_fetch, ('FETCH_SIZE',))[a.copy_kernel]['FETCH_SIZE']
    cw = per_dispatch(a.copy_write, ('WRITE_SIZE',))[a.copy_kernel]['WRITE_SIZE']
    f_fac, w_fac = a.copy_bytes / (cf * 1024.0), a.copy_bytes / (cw * 1024.0)
    rows = trace_rows(a.trace)
    print(f'{a.workload}: B = {B}, {H} x {W}, {dt}; HBM bytes = FETCH_SIZE x {f_fac:.3f} + WRITE_SIZE x {w_fac:.3f} '
          f'(factors from a {a.copy_bytes >> 20} MiB device copy); peak HBM {bench.PEAK["hbm"]:.0f} GB/s')
    print(f'{"kernel":58s} {"tag":22s} {"n":>3s} {"us":>7s} {"alg MB":>7s} {"hbm MB":>7s} {"hbm/alg":>7s} '
          f'{"GB/s":>6s} {"of pk":>5s} {"alg of pk":>9s} {"MFMA%":>6s}')
    shown = 0
    for n, c, s_, av, v, l in rows:
        tag = kernel_tag(n)
        if tag is None or n not in F or n not in Wr:
            continue
        work = bench.kernel_work(tag, B, H, W, es)
        if work is None:
            continue
        alg = work[1]
        hbm = F[n]['FETCH_SIZE'] * 1024.0 * f_fac + Wr[n]['WRITE_SIZE'] * 1024.0 * w_fac
        us = av / 1e3
        gbs = hbm / (us * 1e3)
        rl = bench.roofline(tag, us / 1e3, B, H, W, dt == 'bf16')
        mf = F[n].get('MfmaUtil')
        print(f'{n[:58]:58s} {tag:22s} {c:3d} {us:7.1f} {alg / 1e6:7.1f} {hbm / 1e6:7.1f} {hbm / alg:7.2f} '
              f'{gbs:6.0f} {gbs / bench.PEAK["hbm"]:5.2f} {rl["frac"]:5.2f} {rl["bound"]:>4s} '
              f'{"" if mf is None else f"{mf:6.1f}"}')
        shown += 1
        if shown >= a.top:
            break


def counter_sums(d):
    """{short kernel name: ({counter: sum over dispatches}, dispatches, summed duration ns)}."""
    con = _db(d)
    out, seen = {}, set()
    for name, disp, cn, v, dur in con.execute(
            'select kernel_name, dispatch_id, counter_name, value, duration from counters_collection'):
        k = short_name(name)
        c, n, t = out.get(k, ({}, 0, 0.0))
        c[cn] = c.get(cn, 0.0) + v
        if disp not in seen:
            seen.add(disp)
            n, t = n + 1, t + dur
        out[k] = (c, n, t)
    return out


def cmd_counters(a):
    A, B = counter_sums(a.a), counter_sums(a.b)
    names = sorted(A, key=lambda k: -A[k][2])[:a.top]
    print('per wave: instructions issued; wait / VALU: share of the wave-cycles (SQ_WAVE_CYCLES) spent '
          'waiting on anything (SQ_WAIT_ANY), waiting on LDS (SQ_WAIT_INST_LDS) and issuing VALU '
          '(SQ_ACTIVE_INST_VALU); us: mean dispatch duration in the counter run')
    print(f'{"kernel":60s} {"n":>4s} {"us":>8s} {"VALU":>7s} {"MFMA":>6s} {"LDS":>6s} {"VMEM":>6s} '
          f'{"wait%":>6s} {"wLDS%":>6s} {"VALU%":>6s}')
    for k in names:
        ca, n, t = A[k]
        cb = B.get(k, ({}, 0, 0.0))[0]
        w = max(ca.get('SQ_WAVES', 0.0), 1.0)
        wc = max(ca.get('SQ_WAVE_CYCLES', 0.0), 1.0)
        print(f'{k[:60]:60s} {n:4d} {t / n / 1e3:8.1f} {ca.get("SQ_INSTS_VALU", 0) / w:7.0f} '
              f'{ca.get("SQ_INSTS_MFMA", 0) / w:6.0f} {ca.get("SQ_INSTS_LDS", 0) / w:6.0f} '
              f'{ca.get("SQ_INSTS_VMEM_RD", 0) / w:6.0f} {100 * cb.get("SQ_WAIT_ANY", 0) / wc:6.1f} '
              f'{100 * cb.get("SQ_WAIT_INST_LDS", 0) / wc:6.1f} {100 * cb.get("SQ_ACTIVE_INST_VALU", 0) / wc:6.1f}')


def main(argv=None):
    ap = argparse.ArgumentParser(prog='profsum')
    sub = ap.add_subparsers(dest='cmd', required=True)
    t = sub.add_parser('trace')
    t.add_argument('dir')
    t.add_argument('--top', type=int, default=40)
    t.set_defaults(fn=cmd_trace)
    r = sub.add_parser('traffic')
    for k in ('fetch', 'write', 'copy_fetch', 'copy_write'):
        r.add_argument('--' + k.replace('_', '-'), dest=k, required=True)
    r.add_argument('--copy-bytes', type=int, required=True)
    r.add_argument('--copy-kernel', default='__amd_rocclr_copyBuffer')
    r.add_argument('--kernel', required=True, help='short kernel name as the trace summary prints it')
    r.add_argument('--tag', required=True, help='the profiling tag bench.py uses for that kernel')
    r.add_argument('--workload', required=True, help='bench.py workload the counters were taken on')
    r.add_argument('--bench-log', action='append', required=True,
                   help='output of a bench.py counter run (give both); their tiling choice is recorded')
    r.add_argument('--out', default=None)
    r.set_defaults(fn=cmd_traffic)
    y = sub.add_parser('layers')
    for k in ('fetch', 'write', 'trace', 'copy_fetch', 'copy_write'):
        y.add_argument('--' + k.replace('_', '-'), dest=k, required=True)
    y.add_argument('--copy-bytes', type=int, required=True)
    y.add_argument('--copy-kernel', default='__amd_rocclr_copyBuffer')
    y.add_argument('--workload', required=True)
    y.add_argument('--top', type=int, default=60)
    y.set_defaults(fn=cmd_layers)
    q = sub.add_parser('counters')
    q.add_argument('--a', required=True, help='directory of the instruction-count run')
    q.add_argument('--b', required=True, help='directory of the stall run')
    q.add_argument('--top', type=int, default=30)
    q.set_defaults(fn=cmd_counters)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == '__main__':
    main()
