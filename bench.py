"""Benchmark of the Radar-STDA hot path on one MI355X.

One step = one pass of the whole path over one batch already resident in HBM: TRAIN forward
(batch statistics, running-statistics update), reconstruction loss, hand-written backward,
SGD update.  The RD maps come from the library's rd_synth (timed separately) before the timed
region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--dtype fp32|bf16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (inputs recipe, dtype, recompute)
    'train_fp32_b64_256x128': ('cfg3_train_256x128', 'fp32', 0),
    'train_bf16_b256_256x128': ('cfg4_bf16_train_256x128', 'bf16', 1),
    'train_uneven_bf16_512': ('cfg5_uneven_bf16_train', 'bf16', 0),
}
DEFAULT = 'train_fp32_b64_256x128'


# ---------------------------------------------------------------- algorithmic work per kernel
BLOCKS = {'enc0': (16, 32, False, 0, 1), 'enc1': (32, 64, False, 1, 2),
          'dec0': (64, 32, True, 2, 1), 'dec1': (32, 16, True, 1, 0)}
PEAK = {'hbm': 8000.0, 'mfma_f32': 157.3, 'mfma_bf16': 2500.0, 'alu_f32': 157.3}


def kernel_work(tag, B, H, W, es):
    """(FLOPs, HBM bytes, engine) of one launch of the tagged kernel, counting each input read
    once and each output written once, and every kernel tap as a multiply-add."""
    kind, _, blk = tag.partition('.')
    hw0 = H * W
    if blk in BLOCKS:
        cin, cout, dec, lin, lout = BLOCKS[blk]
        hin, hout = hw0 // 4 ** lin, hw0 // 4 ** lout
        s1_flops = 2.0 * B * hin * (cin * cin + 9 * cin)
        dense_macs = B * hout * (4 if dec else 9) * cin * cout
        skip = 1 if blk in ('dec0', 'dec1') else 0      # decoder outputs add an encoder feature
        skip_g = 1 - skip                                # encoder inputs receive its gradient back
        table = {
            'dense_fwd_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_fwd_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_dgrad_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_dgrad_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'wgrad_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'wgrad_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            's1_stats': (s1_flops, B * cin * hin * es, 'alu'),
            # writes x1 and, in TRAIN, its ReLU decisions (1 bit per element)
            's1_apply': (s1_flops, 2.0 * B * cin * hin * es + B * cin * hin / 8.0, 'alu'),
            's2_apply': (4.0 * B * hout * cout, B * hout * cout * (3 * es + 0.25), 'alu'),
            'eca_next': (2.0 * B * hout * cout, B * hout * cout * es * (2 + skip), 'alu'),
            'eca_bwd': (2.0 * B * hout * cout, 2.0 * B * hout * cout * es, 'alu'),
            's2_bwd_stats': (8.0 * B * hout * cout, B * hout * cout * (2 * es + 0.25), 'alu'),
            's2_bwd_apply': (10.0 * B * hout * cout, B * hout * cout * (4 * es + 0.25), 'alu'),
            # reads x, dx1 and the 1-bit ReLU decisions of x1
            's1_bwd_stats': (s1_flops, B * cin * hin * (2 * es + 1 / 8.0), 'alu'),
            # three pointwise products (recompute, transpose, weight gradient) and three depthwise
            # ones (recompute, transpose, weight gradient); reads x, the 1-bit ReLU decisions of
            # x1, dx1, dxr (+ the skip gradient in the encoder), writes dx
            's1_bwd_fused': (2.0 * B * hin * (3 * cin * cin + 27 * cin),
                             B * cin * hin * ((4 + skip_g) * es + 1 / 8.0), 'alu'),
        }
        return table.get(kind)
    table = {
        'stem_stats': (864.0 * B * hw0, 12.0 * B * hw0, 'alu'),
        'stem_apply': (864.0 * B * hw0, B * hw0 * (12 + 16 * es), 'alu'),
        'head_fwd': (288.0 * B * hw0, B * hw0 * (16 * es + 4), 'alu'),
        'head_bwd': (576.0 * B * hw0, B * hw0 * (4 + 32 * es), 'alu'),
        'stem_bwd_stats': (864.0 * B * hw0, B * hw0 * (32 * es + 12), 'alu'),
        'stem_bwd_apply': (1728.0 * B * hw0, B * hw0 * (32 * es + 12), 'alu'),
    }
    return table.get(kind)


def stage2_layers(per_tag, groups, bf16):
    """Roofline of every stage-2 dense launch (the layers holding most of the arithmetic) from one
    profiled step, {tag: {us, bound, frac}}; for a batch of several map sizes a launch covers every
    segment (us: mean per launch)."""
    out = {}
    for t, (cnt, tms) in sorted(per_tag.items()):
        if t.split('.')[0] in ('dense_fwd_main', 'dense_fwd_res', 'dense_dgrad_main', 'dense_dgrad_res', 'wgrad_main',
                               'wgrad_res'):
            rl = roofline_groups(t, tms, cnt, groups, bf16)
            if rl:
                out[t] = {'us': round(tms * 1e3 / cnt, 2), 'bound': rl['bound'], 'frac': rl['frac']}
    return out or None


def roofline(tag, avg_ms, B, H, W, dtype_bf16):
    return roofline_groups(tag, avg_ms, 1, [(B, H, W)], dtype_bf16)


def roofline_groups(tag, total_ms, launches, groups, dtype_bf16):
    """Roofline of `launches` launches of the tagged kernel taking total_ms together, each over all
    the segments `groups` [(clips, H, W)] (one launch walks the tiles of every segment): algorithmic
    work of all of them over their total time, against the engine's peak or HBM, whichever binds."""
    es = 2 if dtype_bf16 else 4
    per = launches
    flops = nbytes = 0.0
    engine = None
    for B, H, W in groups:
        w = kernel_work(tag, B, H, W, es)
        if w is None:
            return None
        flops += w[0] * per
        nbytes += w[1] * per
        engine = w[2]
    if total_ms <= 0:
        return None
    peak_c = PEAK['mfma_bf16' if dtype_bf16 else 'mfma_f32'] if engine == 'mfma' else PEAK['alu_f32']
    t_c = flops / (peak_c * 1e12)
    t_b = nbytes / (PEAK['hbm'] * 1e9)
    sec = total_ms / 1e3
    avg_us = round(total_ms * 1e3 / launches, 2)
    if t_c >= t_b:
        achieved = flops / sec / 1e12
        return {'bound': engine, 'achieved': round(achieved, 2), 'peak': peak_c, 'unit': 'TFLOP/s',
                'frac': round(achieved / peak_c, 4), 'traffic': None, 'kernel': tag,
                'avg_us': avg_us, 'algorithmic_flops': flops / launches, 'algorithmic_bytes': nbytes / launches}
    achieved = nbytes / sec / 1e9
    return {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': PEAK['hbm'], 'unit': 'GB/s',
            'frac': round(achieved / PEAK['hbm'], 4), 'traffic': None, 'kernel': tag,
            'avg_us': avg_us, 'algorithmic_flops': flops / launches, 'algorithmic_bytes': nbytes / launches}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--workload', default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-sample-clips', type=int, default=8)
    ap.add_argument('--train-only', action='store_true', help='only the chosen training workload')
    ap.add_argument('--no-graph', action='store_true', help='time eager steps instead of the captured step')
    ap.add_argument('--copy-calib', action='store_true',
                    help='only run a plain 256 MiB device copy 5 times (counter calibration) and exit')
    ap.add_argument('--no-tune', action='store_true', help='keep the default tilings (skip the autotuner)')
    ap.add_argument('--kernel', default=None, help='tag of the kernel for the roofline (default: the dominant one)')
    return ap.parse_args()


def make_batch(stda, inputs, torch, recipe_name, dev, rd_time=False):
    """Segments and resident inputs of a workload: RD maps from rd_synth on the GPU."""
    rc = inputs.WORKLOADS[recipe_name]
    B = rc['B']
    if len(rc['sizes']) == 1:
        groups = [(B,) + tuple(rc['sizes'][0])]
    else:
        sizes = inputs.uneven_sizes(B, rc['sizes'], rc['seed'])
        groups = [(sum(1 for q in sizes if q == sz),) + tuple(sz) for sz in rc['sizes']]
        groups = [g for g in groups if g[0] > 0]
    segs = stda.packed_segments(groups)
    nx = sum(3 * n * H * W for n, H, W in groups)
    x = torch.empty(nx, device=dev)
    y = torch.empty(nx // 3, device=dev)
    rd_ms = 0.0
    xo = yo = 0
    metas = []
    for gi, (n, H, W) in enumerate(groups):
        tab, meta = inputs.make_scenes(n, H, W, rc['seed'] + 101 * gi, targets=rc['targets'], intf=rc['intf'],
                                       inr=rc['inr'], clutter=rc['clutter'])
        metas.append(meta)
        scenes = stda.upload_scenes(tab, dev)
        rws = stda.alloc_bytes(stda.rd_synth_workspace_size(n, H, W), dev)
        xv = x[xo:xo + 3 * n * H * W]
        yv = y[yo:yo + n * H * W]
        stda.rd_synth(scenes, n, H, W, meta['seed'], meta['noise_sigma'], xv, yv, rws)
        if rd_time:
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                stda.rd_synth(scenes, n, H, W, meta['seed'], meta['noise_sigma'], xv, yv, rws)
            e1.record()
            torch.cuda.synchronize()
            rd_ms += e0.elapsed_time(e1) / 5
        xo += 3 * n * H * W
        yo += n * H * W
    torch.cuda.synchronize()
    make_batch.metas = metas  # per-group scene records (target peak cells), for the accuracy check
    return segs, groups, x, y, rd_ms


class Trainer:
    """Buffers of one training workload; eager steps and the captured step graph."""

    def __init__(self, stda, inputs, torch, segs, x, y, dtype, recompute, dev):
        self.stda, self.torch, self.segs, self.x, self.y = stda, torch, segs, x, y
        self.dtype, self.recompute = dtype, recompute
        self.w = torch.from_numpy(inputs.make_weights(stda.param_specs())).to(dev)
        self.running = torch.from_numpy(inputs.make_running(stda.bn_channels())).to(dev)
        sv_b, ws_b = stda.workspace_size(segs, dtype, stda.TRAIN, recompute)
        self.saved, self.ws = stda.alloc_bytes(sv_b, dev), stda.alloc_bytes(ws_b, dev)
        self.z = torch.empty_like(y)
        self.dz = torch.empty_like(y)
        self.dw = torch.empty_like(self.w)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.wb = torch.empty(self.w.numel(), dtype=torch.int16, device=dev) if dtype == stda.BF16 else None
        self.graph = None
        self.stream = torch.cuda.Stream()

    def step(self):
        s = self.stda
        s.forward(self.segs, self.x, self.w, self.running, self.z, self.saved, self.ws, self.dtype, s.TRAIN,
                  self.recompute)
        s.mse_loss(self.segs, self.z, self.y, self.loss, self.dz, self.ws)
        s.backward(self.segs, self.x, self.dz, self.w, self.saved, self.dw, None, self.ws, self.dtype,
                   self.recompute)
        s.sgd_step(self.w, self.dw, 1e-3, 5e-4, self.wb)

    def autotune(self, reps=2):
        """The library's autotuner on this workload's buffers (running statistics on a scratch copy);
        returns the chosen tiling variant of every tunable launch."""
        scratch = self.running.clone()
        res = self.stda.autotune(self.segs, self.x, self.y, self.w, scratch, self.z, self.loss, self.dz, self.dw,
                                 self.saved, self.ws, self.dtype, self.recompute, reps)
        self.torch.cuda.synchronize()
        names = {0: 'fwd', 1: 'dgrad', 2: 'wgrad', 3: 's1_bwd'}
        return {f'{names[k]}.{("enc0", "enc1", "dec0", "dec1")[b]}': v[0] for (k, b), v in sorted(res.items())}

    def capture(self):
        self.torch.cuda.synchronize()
        self.graph = self.stda.TrainStepGraph(self.segs, self.x, self.y, self.w, self.running, self.z, self.loss,
                                              self.dz, self.dw, self.saved, self.ws, self.dtype, self.recompute,
                                              1e-3, 5e-4, self.wb, self.stream)

    def timed(self, steps, graph):
        """ms per step over `steps` steps, bracketed by synchronisations, timed with HIP events on the
        stream the work runs on."""
        torch = self.torch
        torch.cuda.synchronize()
        st = self.stream if graph else torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            if graph:
                self.graph.launch()
            else:
                self.step()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps


def source_hash():
    """SHA-256 over the library sources: a committed counter summary applies only to this hash."""
    import hashlib
    d = os.path.join(ROOT, 'paper_2307_09063_amd', 'csrc')
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith(('.h', '.hip')):
            with open(os.path.join(d, f), 'rb') as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()


def tile_key(tag):
    """Key of config.tiles that selects the tiling of the tagged launch, or None if untuned."""
    kind, _, blk = tag.partition('.')
    k = {'dense_fwd_main': 'fwd', 'dense_fwd_res': 'fwd', 'dense_dgrad_main': 'dgrad', 'dense_dgrad_res': 'dgrad',
         'wgrad_main': 'wgrad', 'wgrad_res': 'wgrad', 's1_bwd_fused': 's1_bwd'}.get(kind)
    return f'{k}.{blk}' if k else None


def measured_traffic(kernel, workload, tiles):
    """HBM bytes per launch of `kernel` in `workload` from the committed counter summary, or
    None when the summary is missing, covers another kernel, workload or tiling, or was taken on
    different sources."""
    path = os.path.join(ROOT, 'profiles', 'traffic.json')
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get('source_sha256') != source_hash() or t.get('kernel_tag') != kernel or t.get('workload') != workload:
        return None
    key = tile_key(kernel)
    if key is not None and (tiles or {}).get(key, 0) != t.get('tile_variant'):
        return None
    return t.get('hbm_bytes_per_launch')


def main():
    args = parse()
    if args.copy_calib:
        import torch
        src = torch.ones(64 << 20, device='cuda')
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({'copy_bytes_read': src.numel() * 4, 'copy_bytes_written': dst.numel() * 4}))
        return
    if args.gpus != 1:
        print(f'bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is '
              'described, not built', file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2307_09063_amd import inputs, stda

    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    recipe_name, dt_name, recompute = WORKLOADS[args.workload]
    dtype = stda.BF16 if dt_name == 'bf16' else stda.FP32
    segs, groups, x, y, rd_ms = make_batch(stda, inputs, torch, recipe_name, dev, rd_time=not args.train_only)
    B = sum(g[0] for g in groups)
    N, M = groups[0][1], groups[0][2]
    tr = Trainer(stda, inputs, torch, segs, x, y, dtype, recompute, dev)
    tiles = None if args.no_tune else tr.autotune()
    if tiles:
        print(f'bench: autotuned tilings {tiles}', file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    # dominant kernel: one step with every tagged launch timed
    stda.profile_select('*')
    tr.step()
    torch.cuda.synchronize()
    per_tag = stda.profile_report()
    stda.profile_select(None)
    dominant = args.kernel or max(per_tag, key=lambda t: per_tag[t][1])
    # roofline of every stage-2 dense launch (the layers that hold most of the arithmetic), from the
    # same profiled step; algorithmic work as in kernel_work
    layers = stage2_layers(per_tag, groups, stda.BF16 == dtype)
    tot_tagged = sum(v[1] for v in per_tag.values())
    for t, (n, tms) in sorted(per_tag.items(), key=lambda kv: -kv[1][1])[:40]:
        print(f'bench:   {t:28s} {n:3d} launches {tms:8.3f} ms ({100 * tms / tot_tagged:4.1f}%)', file=sys.stderr)
    print(f'bench: dominant kernel {dominant}', file=sys.stderr, flush=True)
    # headline: the captured step, replayed
    use_graph = not args.no_graph
    if use_graph:
        tr.capture()
        tr.timed(2, True)
    print(f'bench: timing {args.steps} steps ({"graph" if use_graph else "eager"})', file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ms = tr.timed(args.steps, use_graph)
    wall = time.perf_counter() - t0
    clips_s = B / (ms / 1e3)
    # roofline: the same steps eagerly, the dominant kernel's launches bracketed by HIP events
    stda.profile_select(dominant)
    ms_eager = tr.timed(args.steps, False)
    k_total, k_count = stda.profile_read()
    stda.profile_select(None)
    roof = roofline_groups(dominant, k_total, max(k_count, 1), groups, dtype == stda.BF16)
    if roof is not None and len(groups) == 1:
        roof['traffic'] = measured_traffic(dominant, args.workload, tiles)
    print(f'bench: {ms:.3f} ms/step ({clips_s:.0f} clips/s), eager {ms_eager:.3f} ms, wall {wall:.2f}s, '
          f'loss {tr.loss.item():.5f}', file=sys.stderr, flush=True)

    extra = {}
    bf16_batches = {}
    if dtype == stda.BF16:
        bf16_batches[args.workload] = (segs, groups, x, make_batch.metas, tr.w, tr.running)
    if not args.train_only:
        fwd_ms, Bf, det = eval_forward(stda, inputs, torch, tr.w, tr.running, dev)
        extra['fwd_eval_fp32_b32_256x128'] = {'ms': round(fwd_ms, 4), 'clips_per_s': round(Bf / (fwd_ms / 1e3), 1)}
        extra['detect_b32_256x128'] = det
        extra['rd_synth_table4_b256_64x128'] = rd_synth_table4(stda, inputs, torch, dev)
        extra['fwd_eval_fp32_b1_64x64'] = latency_b1(stda, inputs, torch, tr.w, tr.running, dev, 64, 64)
        extra['fwd_eval_fp32_b1_128x64'] = latency_b1(stda, inputs, torch, tr.w, tr.running, dev, 128, 64)
        for other in ('train_bf16_b256_256x128', 'train_uneven_bf16_512'):
            if other == args.workload:
                continue
            rn, dn, rec = WORKLOADS[other]
            sg, gr, xo, yo, _ = make_batch(stda, inputs, torch, rn, dev)
            t2 = Trainer(stda, inputs, torch, sg, xo, yo, stda.BF16 if dn == 'bf16' else stda.FP32, rec, dev)
            tiles2 = None if args.no_tune else t2.autotune()
            t2.step()
            torch.cuda.synchronize()
            stda.profile_select('*')
            t2.step()
            torch.cuda.synchronize()
            pt2 = stda.profile_report()
            layers2 = stage2_layers(pt2, gr, dn == 'bf16')
            stda.profile_select(None)
            dom2 = max(pt2, key=lambda t: pt2[t][1])
            roof2 = roofline_groups(dom2, pt2[dom2][1], pt2[dom2][0], gr, dn == 'bf16')
            t2.capture()
            t2.timed(2, True)
            m2 = t2.timed(max(3, args.steps // 2), True)
            n2 = sum(g[0] for g in gr)
            bf16_batches[other] = (sg, gr, xo, make_batch.metas, t2.w, t2.running)
            extra[other] = {'ms_per_step': round(m2, 4), 'clips_per_s': round(n2 / (m2 / 1e3), 1), 'dtype': dn,
                            'recompute': rec, 'segments': [list(g) for g in gr], 'tiles': tiles2,
                            'roofline': roof2, 'roofline_stage2_layers': layers2}
            print(f'bench: {other}: {m2:.3f} ms/step ({n2 / (m2 / 1e3):.0f} clips/s)', file=sys.stderr, flush=True)
            t2.graph.close()
            del t2, yo
            torch.cuda.empty_cache()

    cpu = main_err = None
    if not args.no_cpu_baseline:
        k = args.cpu_sample_clips
        cpu = cpu_baseline(k, N, M, x[:3 * k * N * M].view(k, 3, N, M).cpu().numpy(),
                           y[:k * N * M].view(k, 1, N, M).cpu().numpy(), tr.w.cpu().numpy(),
                           tr.running.cpu().numpy())
        # the oracle leg also checks the BF16 workloads' forward on sampled clips
        for name, b in bf16_batches.items():
            acc = bf16_error_vs_oracle(stda, torch, *b, dev)
            if name == args.workload:
                main_err = acc
            else:
                extra[name]['error_vs_oracle'] = acc
            print(f'bench: {name}: BF16 error on sampled clips: max z rel-L2 {acc["max_z_rel_l2"]:.2e}, '
                  f'max |delta SINR| {acc["max_abs_delta_sinr_db"]:.4f} dB', file=sys.stderr, flush=True)
    bf16_batches.clear()

    out = {
        'metric': '3-frame RD clips/s, fwd+bwd training step',
        'value': round(clips_s, 1),
        'unit': 'clips/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': round(ms, 4),
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'bf16' if dtype == stda.BF16 else 'f32',
        'data': 'synthetic (seeded FMCW scenes -> rd_synth on the GPU)',
        'config': {'workload': args.workload, 'clips': B, 'frames': 3, 'segments': [list(g) for g in groups],
                   'step': 'TRAIN forward + MSE + backward + SGD', 'recompute': recompute,
                   'launch': 'one hipGraph launch per step' if use_graph else 'eager', 'tiles': tiles},
        'ms_per_step_eager': round(ms_eager, 4),
        'rd_synth_ms': round(rd_ms, 4),
        'roofline': roof,
        'roofline_stage2_layers': layers or None,
        'cpu_baseline': cpu,
    }
    if main_err is not None:
        out['error_vs_oracle'] = main_err
    out.update(extra)
    print(json.dumps(out), flush=True)


def bf16_error_vs_oracle(stda, torch, segs, groups, x, metas, w, running, dev, per_group=2):
    """Accuracy of a BF16 workload's forward on sampled clips (part of the oracle leg: run only
    with the CPU baseline).  The workload's batch goes through the BF16 EVAL forward (per-clip
    results are independent in EVAL); `per_group` clips of each map size are compared with the
    FP64 oracle's EVAL forward of the same clips: rel-L2 and max |a - b| / max |b| of z, and the
    SINR delta of Sec. V-B Eq. (19) per clip on the scene's target and noise cells."""
    import numpy as np

    from oracle import net, rdsynth
    from paper_2307_09063_amd import inputs
    _, wsb = stda.workspace_size(segs, stda.BF16, stda.EVAL)
    z = torch.empty(sum(n * H * W for n, H, W in groups), device=dev)
    stda.forward(segs, x, w, running, z, None, stda.alloc_bytes(wsb, dev), stda.BF16, stda.EVAL)
    torch.cuda.synchronize()
    wn, rn = w.cpu().numpy(), running.cpu().numpy()
    res, xo, zo = [], 0, 0
    for (n, H, W), meta in zip(groups, metas):
        for c in np.linspace(0, n - 1, per_group).round().astype(int)[:n]:
            xc = x[xo + 3 * c * H * W: xo + 3 * (c + 1) * H * W].view(1, 3, H, W).cpu().numpy()
            zc = z[zo + c * H * W: zo + (c + 1) * H * W].view(1, 1, H, W).cpu().numpy().astype(np.float64)
            zr, _, _ = net.forward(wn, rn, xc, 'eval')
            o, nm = inputs.sinr_masks(meta['peaks'][c], H, W)
            res.append({'map': [H, W], 'clip': int(c),
                        'z_rel_l2': float(np.linalg.norm(zc - zr) / np.linalg.norm(zr)),
                        'z_max_abs_rel': float(np.abs(zc - zr).max() / np.abs(zr).max()),
                        'delta_sinr_db': float(rdsynth.sinr_db(zc[0, 0], o, nm) - rdsynth.sinr_db(zr[0, 0], o, nm))})
        xo += 3 * n * H * W
        zo += n * H * W
    return {'mode': 'eval', 'clips': res,
            'max_z_rel_l2': max(r['z_rel_l2'] for r in res),
            'max_abs_delta_sinr_db': max(abs(r['delta_sinr_db']) for r in res)}


def latency_b1(stda, inputs, torch, w, running, dev, N=64, M=64):
    """EVAL forward of one clip of 3 x N x M (64 x 64: the small configuration; 128 x 64: the
    paper's own FPS setting, Table 7): per-clip time of back-to-back calls, eager and as a replayed
    graph, and the wall time of one synchronised graph replay (host-measured, median of 50); the
    same for the folded-weight EVAL forward (stda_forward_folded, its graph), with the number of
    tagged launches of one call of each."""
    rc = inputs.WORKLOADS['cfg1_fwd_64x64']
    tab, meta = inputs.make_scenes(1, N, M, rc['seed'], targets=rc['targets'], intf=rc['intf'], inr=rc['inr'],
                                   clutter=rc['clutter'])
    x1, _ = stda.synthesize(tab, meta, dev, with_clean=False)
    segs = stda.uniform_segments(1, N, M)
    _, wsb = stda.workspace_size(segs, stda.FP32, stda.EVAL)
    ws = stda.alloc_bytes(wsb, dev)
    z = torch.empty((1, 1, N, M), device=dev)
    for _ in range(5):
        stda.forward(segs, x1, w, running, z, None, ws, stda.FP32, stda.EVAL)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        stda.forward(segs, x1, w, running, z, None, ws, stda.FP32, stda.EVAL)
    e1.record()
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / 50
    g = stda.ForwardGraph(segs, x1, w, running, z, ws)
    for _ in range(5):
        g.launch()
    torch.cuda.synchronize()
    e0.record(g.stream)
    for _ in range(50):
        g.launch()
    e1.record(g.stream)
    torch.cuda.synchronize()
    graph = e0.elapsed_time(e1) / 50
    walls = []
    for _ in range(50):
        t0 = time.perf_counter()
        g.launch()
        g.stream.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    g.close()
    wall = sorted(walls)[len(walls) // 2]
    # the folded-weight EVAL forward (batch norm folded into the weights once, stage 2 in one launch)
    fb = stda.alloc_bytes(stda.eval_fold_size(stda.FP32), dev)
    stda.eval_fold(w, running, fb, stda.FP32)
    zf = torch.empty_like(z)
    gf = stda.FoldedForwardGraph(segs, x1, fb, zf, ws)
    for _ in range(5):
        gf.launch()
    torch.cuda.synchronize()
    e0.record(gf.stream)
    for _ in range(50):
        gf.launch()
    e1.record(gf.stream)
    torch.cuda.synchronize()
    graph_f = e0.elapsed_time(e1) / 50
    walls = []
    for _ in range(50):
        t0 = time.perf_counter()
        gf.launch()
        gf.stream.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    gf.close()
    wall_f = sorted(walls)[len(walls) // 2]
    # launches per forward call, unfolded and folded (every tagged launch of one call)
    stda.profile_select('*')
    stda.forward(segs, x1, w, running, z, None, ws, stda.FP32, stda.EVAL)
    torch.cuda.synchronize()
    n_unf = sum(v[0] for v in stda.profile_report().values())
    stda.profile_select('*')
    stda.forward_folded(segs, x1, fb, zf, ws)
    torch.cuda.synchronize()
    n_fold = sum(v[0] for v in stda.profile_report().values())
    stda.profile_select(None)
    return {'ms_eager': round(eager, 4), 'ms_graph': round(graph, 4), 'ms_graph_sync_wall': round(wall, 4),
            'fps_graph_sync': round(1e3 / wall, 1), 'tagged_launches': n_unf,
            'folded': {'ms_graph': round(graph_f, 4), 'ms_graph_sync_wall': round(wall_f, 4),
                       'fps_graph_sync': round(1e3 / wall_f, 1), 'tagged_launches': n_fold}}


def eval_forward(stda, inputs, torch, w, running, dev):
    """Forward-only EVAL at the forward configuration (B = 32 clips of 3 x 256 x 128, its own seeded
    scenes), ms per call; then the detection step on the restored maps (CA-CFAR with the
    reference-peak hit count, EVM and SINR against the interference-free maps), ms per call."""
    import numpy as np
    rc = inputs.WORKLOADS['cfg2_fwd_256x128']
    Bf = rc['B']
    N, M = rc['sizes'][0]
    tab, meta = inputs.make_scenes(Bf, N, M, rc['seed'], targets=rc['targets'], intf=rc['intf'],
                                   inr=rc['inr'], clutter=rc['clutter'])
    x, clean = stda.synthesize(tab, meta, dev)
    xf = x.reshape(-1).contiguous()
    segs_f = stda.uniform_segments(Bf, N, M)
    _, ws_f = stda.workspace_size(segs_f, stda.FP32, stda.EVAL)
    wsf = stda.alloc_bytes(ws_f, dev)
    zf = torch.empty((Bf, 1, N, M), device=dev)
    for _ in range(3):
        stda.forward(segs_f, xf, w, running, zf, None, wsf, stda.FP32, stda.EVAL)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        stda.forward(segs_f, xf, w, running, zf, None, wsf, stda.FP32, stda.EVAL)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    masks = [inputs.sinr_masks(meta['peaks'][b], N, M) for b in range(Bf)]
    om = torch.from_numpy(np.stack([m[0] for m in masks]).astype(np.uint8)).to(dev)
    nm = torch.from_numpy(np.stack([m[1] for m in masks]).astype(np.uint8)).to(dev)
    det = torch.empty((Bf, N, M), dtype=torch.uint8, device=dev)
    counts = torch.empty((Bf, 2), dtype=torch.int32, device=dev)
    ev = torch.empty(Bf, dtype=torch.float64, device=dev)
    sn = torch.empty(Bf, dtype=torch.float64, device=dev)

    def detect_step():
        stda.cfar(zf, det, **stda.CFAR_DEFAULT, o_mask=om, counts=counts)
        stda.evm(zf, clean, om, ev)
        stda.sinr(zf, om, nm, sn)

    for _ in range(3):
        detect_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        detect_step()
    e1.record()
    torch.cuda.synchronize()
    det_ms = e0.elapsed_time(e1) / 10
    c = counts.cpu().numpy()
    return fwd_ms, Bf, {'ms': round(det_ms, 4), 'maps_per_s': round(Bf / (det_ms / 1e3), 1),
                        'cfar': dict(stda.CFAR_DEFAULT), 'peaks_hit': int(c[:, 1].sum()),
                        'peaks': int(om.sum().item()), 'detections': int(c[:, 0].sum()),
                        'note': 'random-init weights: detection quality is not meaningful, only timing'}


def rd_synth_table4(stda, inputs, torch, dev, n=256, N=64, M=128):
    """rd_synth of the physical-units aggressor family (Table 4 intervals, one aggressor per clip)
    at the paper's map size (64 range x 128 Doppler), ms per call for n clips (4 maps each)."""
    tab, meta = inputs.make_scenes_table4(n, N, M, seed=44, clutter=True)
    scenes = stda.upload_scenes(tab, dev)
    rws = stda.alloc_bytes(stda.rd_synth_workspace_size(n, N, M), dev)
    x = torch.empty((n, 3, N, M), device=dev)
    y = torch.empty((n, 1, N, M), device=dev)
    for _ in range(2):
        stda.rd_synth(scenes, n, N, M, meta['seed'], meta['noise_sigma'], x, y, rws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        stda.rd_synth(scenes, n, N, M, meta['seed'], meta['noise_sigma'], x, y, rws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    return {'ms': round(ms, 4), 'clips_per_s': round(n / (ms / 1e3), 1), 'clips': n, 'map': [N, M]}


def _oracle_step_worker(args):
    """One FP64 oracle training step (forward, MSE, backward, SGD) on the sample; returns the
    wall-clock interval of the step itself (process start-up and imports excluded)."""
    x, y, w, r = args
    import numpy as np

    from oracle import net
    t0 = time.time()
    _, g, _, _, _ = net.loss_and_grad(w.astype(np.float64), r.astype(np.float64), x, y)
    net.sgd_step(w, g, 1e-3, 5e-4)
    return t0, time.time()


def host_cpu():
    """(usable cores, CPU model name) of this host."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline(nclips, N, M, x, y, w, r, max_workers=16):
    """The FP64 oracle's training step timed on the host's cores: one single-threaded worker
    process per core (at most max_workers, the host share of one GPU), each running the same
    bounded sample, started together; throughput = all workers' clips over the span from the
    first step's start to the last one's end.  The single-worker rate is reported beside it."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    cores, model = host_cpu()
    workers = max(1, min(cores, max_workers))
    env_keys = ('OMP_NUM_THREADS', 'OPENBLAS_NUM_THREADS', 'MKL_NUM_THREADS')
    old = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:
        os.environ[k] = '1'  # one thread per worker: the workers are the parallelism
    try:
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context('spawn')) as ex:
            spans = list(ex.map(_oracle_step_worker, [(x, y, w, r)] * workers))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    span = max(e for _, e in spans) - min(s for s, _ in spans)
    one = sum(e - s for s, e in spans) / len(spans)
    return {'value': round(workers * nclips / span, 4), 'unit': 'clips/s', 'cores': workers, 'kind': 'oracle',
            'value_per_core': round(nclips / one, 4), 'host_cores': cores, 'cpu_model': model,
            'sample': f'{workers} single-threaded workers, each one FP64 training step (forward, MSE, backward, '
                      f'SGD) on the same {nclips} clips of 3x{N}x{M}; {span:.1f} s span, {one:.1f} s per step'}


if __name__ == '__main__':
    main()
