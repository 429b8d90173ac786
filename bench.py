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
        skip = 1 if blk in ('dec0', 'dec1') else 0
        table = {
            'dense_fwd_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_fwd_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_dgrad_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'dense_dgrad_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'wgrad_main': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'wgrad_res': (2.0 * dense_macs, B * (cin * hin + cout * hout) * es, 'mfma'),
            'wgrad_pw': (2.0 * B * hin * cin * cin, 2.0 * B * cin * hin * es, 'mfma'),
            'wgrad_dw': (2.0 * B * hin * 9 * cin, 2.0 * B * cin * hin * es, 'alu'),
            's1_stats': (s1_flops, B * cin * hin * es, 'alu'),
            's1_apply': (s1_flops, 2.0 * B * cin * hin * es, 'alu'),
            's2_apply': (4.0 * B * hout * cout, B * hout * cout * (3 * es + 0.25), 'alu'),
            'eca_next': (2.0 * B * hout * cout, B * hout * cout * es * (2 + skip), 'alu'),
            'eca_bwd': (2.0 * B * hout * cout, 2.0 * B * hout * cout * es, 'alu'),
            's2_bwd_stats': (8.0 * B * hout * cout, B * hout * cout * (2 * es + 0.25), 'alu'),
            's2_bwd_apply': (10.0 * B * hout * cout, B * hout * cout * (4 * es + 0.25), 'alu'),
            's1_bwd_stats': (s1_flops, 3.0 * B * cin * hin * es, 'alu'),
            's1_bwd_apply': (s1_flops, 7.0 * B * cin * hin * es, 'alu'),
            's1_bwd_dx': (s1_flops, (4 + skip) * B * cin * hin * es, 'alu'),
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


def roofline(tag, avg_ms, B, H, W, dtype_bf16):
    es = 2 if dtype_bf16 else 4
    w = kernel_work(tag, B, H, W, es)
    if w is None or avg_ms <= 0:
        return None
    flops, nbytes, engine = w
    peak_c = PEAK['mfma_bf16' if dtype_bf16 else 'mfma_f32'] if engine == 'mfma' else PEAK['alu_f32']
    t_c = flops / (peak_c * 1e12)
    t_b = nbytes / (PEAK['hbm'] * 1e9)
    sec = avg_ms / 1e3
    if t_c >= t_b:
        achieved = flops / sec / 1e12
        return {'bound': engine, 'achieved': round(achieved, 2), 'peak': peak_c, 'unit': 'TFLOP/s',
                'frac': round(achieved / peak_c, 4), 'traffic': None, 'kernel': tag,
                'avg_us': round(avg_ms * 1e3, 2), 'algorithmic_flops': flops, 'algorithmic_bytes': nbytes}
    achieved = nbytes / sec / 1e9
    return {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': PEAK['hbm'], 'unit': 'GB/s',
            'frac': round(achieved / PEAK['hbm'], 4), 'traffic': None, 'kernel': tag,
            'avg_us': round(avg_ms * 1e3, 2), 'algorithmic_flops': flops, 'algorithmic_bytes': nbytes}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--workload', default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-sample-clips', type=int, default=4)
    ap.add_argument('--train-only', action='store_true', help='skip the EVAL-forward and rd_synth timings')
    ap.add_argument('--kernel', default=None, help='tag of the kernel for the roofline (default: the dominant one)')
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f'bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is '
              'described, not built', file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2307_09063_amd import inputs, stda

    recipe_name, dt_name, recompute = WORKLOADS[args.workload]
    recipe = inputs.WORKLOADS[recipe_name]
    dtype = stda.BF16 if dt_name == 'bf16' else stda.FP32
    B = recipe['B']
    N, M = recipe['sizes'][0]
    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)

    # ---- inputs: synthetic RD maps of the paper's workload shape, on the GPU
    tab, meta = inputs.make_scenes(B, N, M, recipe['seed'], targets=recipe['targets'], intf=recipe['intf'],
                                   inr=recipe['inr'], clutter=recipe['clutter'])
    scenes = stda.upload_scenes(tab, dev)
    x = torch.empty((B, 3, N, M), device=dev)
    y = torch.empty((B, 1, N, M), device=dev)
    rws = stda.alloc_bytes(stda.rd_synth_workspace_size(B, N, M), dev)
    stda.rd_synth(scenes, B, N, M, meta['seed'], meta['noise_sigma'], x, y, rws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        stda.rd_synth(scenes, B, N, M, meta['seed'], meta['noise_sigma'], x, y, rws)
    e1.record()
    torch.cuda.synchronize()
    rd_ms = e0.elapsed_time(e1) / 5

    w = torch.from_numpy(inputs.make_weights(stda.param_specs())).to(dev)
    running = torch.from_numpy(inputs.make_running(stda.bn_channels())).to(dev)
    segs = stda.uniform_segments(B, N, M)
    sv_b, ws_b = stda.workspace_size(segs, dtype, stda.TRAIN, recompute)
    saved, ws = stda.alloc_bytes(sv_b, dev), stda.alloc_bytes(ws_b, dev)
    z = torch.empty((B, 1, N, M), device=dev)
    dz = torch.empty_like(z)
    dw = torch.empty_like(w)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    wb = torch.empty(w.numel(), dtype=torch.int16, device=dev) if dtype == stda.BF16 else None

    def step():
        stda.forward(segs, x, w, running, z, saved, ws, dtype, stda.TRAIN, recompute)
        stda.mse_loss(segs, z, y, loss, dz, ws)
        stda.backward(segs, x, dz, w, saved, dw, None, ws, dtype, recompute)
        stda.sgd_step(w, dw, 1e-3, 5e-4, wb)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # dominant kernel: one step with every tagged launch timed
    stda.profile_select('*')
    step()
    torch.cuda.synchronize()
    per_tag = stda.profile_report()
    dominant = args.kernel or max(per_tag, key=lambda t: per_tag[t][1])
    tot_tagged = sum(v[1] for v in per_tag.values())
    for t, (n, tms) in sorted(per_tag.items(), key=lambda kv: -kv[1][1])[:40]:
        print(f'bench:   {t:28s} {n:3d} launches {tms:8.3f} ms ({100 * tms / tot_tagged:4.1f}%)', file=sys.stderr)
    print(f'bench: dominant kernel {dominant} ({per_tag.get(dominant, (0, 0))[1]:.3f} ms of one step)',
          file=sys.stderr, flush=True)
    # timed region; the dominant kernel's launches are bracketed by HIP events on their stream
    stda.profile_select(dominant)
    print(f'bench: warmup done, timing {args.steps} steps', file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_total, k_count = stda.profile_read()
    stda.profile_select(None)
    ms = e0.elapsed_time(e1) / args.steps
    clips_s = B / (ms / 1e3)
    roof = roofline(dominant, k_total / max(k_count, 1), B, N, M, dtype == stda.BF16)
    print(f'bench: {ms:.3f} ms/step ({clips_s:.0f} clips/s), wall {wall:.2f}s, loss {loss.item():.5f}',
          file=sys.stderr, flush=True)

    fwd_ms = None
    if args.train_only:
        Bf = 0
    else:
        fwd_ms, Bf = eval_forward(stda, inputs, torch, x, w, running, N, M, dev, e0, e1)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample_clips, N, M, x[:args.cpu_sample_clips].cpu().numpy(),
                           y[:args.cpu_sample_clips].cpu().numpy(), w.cpu().numpy(), running.cpu().numpy())

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
        'config': {'workload': args.workload, 'clips': B, 'frames': 3, 'range_bins': N, 'doppler_bins': M,
                   'step': 'TRAIN forward + MSE + backward + SGD', 'recompute': recompute},
        'fwd_eval_fp32_b32': None if fwd_ms is None else {'ms': round(fwd_ms, 4),
                                                           'clips_per_s': round(Bf / (fwd_ms / 1e3), 1)},
        'rd_synth': {'ms': round(rd_ms, 4), 'clips_per_s': round(B / (rd_ms / 1e3), 1), 'maps_per_clip': 4},
        'roofline': roof,
        'cpu_baseline': cpu,
    }
    print(json.dumps(out), flush=True)


def eval_forward(stda, inputs, torch, x, w, running, N, M, dev, e0, e1):
    """Forward-only EVAL at the forward configuration (B = 32) on the same maps."""
    fw = inputs.WORKLOADS['cfg2_fwd_256x128']
    Bf = fw['B']
    segs_f = stda.uniform_segments(Bf, N, M)
    _, ws_f = stda.workspace_size(segs_f, stda.FP32, stda.EVAL)
    wsf = stda.alloc_bytes(ws_f, dev)
    xf, zf = x[:Bf].contiguous(), torch.empty((Bf, 1, N, M), device=dev)
    for _ in range(3):
        stda.forward(segs_f, xf, w, running, zf, None, wsf, stda.FP32, stda.EVAL)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        stda.forward(segs_f, xf, w, running, zf, None, wsf, stda.FP32, stda.EVAL)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    return fwd_ms, Bf


def cpu_baseline(nclips, N, M, x, y, w, r):
    """The FP64 oracle's training step (forward, loss, backward, SGD) timed on the host."""
    import numpy as np
    import resource

    from oracle import net
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    loss, g, _, _, _ = net.loss_and_grad(w.astype(np.float64), r.astype(np.float64), x, y)
    net.sgd_step(w, g, 1e-3, 5e-4)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu_s = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {'value': round(nclips / wall, 4), 'unit': 'clips/s', 'cores': max(1, round(cpu_s / wall)),
            'kind': 'oracle',
            'sample': f'{nclips} clips of 3x{N}x{M}, one FP64 training step (forward, MSE, backward, SGD), '
                      f'{wall:.1f} s wall'}


if __name__ == '__main__':
    main()
