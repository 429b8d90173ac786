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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--workload', default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-sample-clips', type=int, default=4)
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
    print(f'bench: warmup done, timing {args.steps} steps', file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    clips_s = B / (ms / 1e3)
    print(f'bench: {ms:.3f} ms/step ({clips_s:.0f} clips/s), wall {wall:.2f}s, loss {loss.item():.5f}',
          file=sys.stderr, flush=True)

    # ---- forward-only EVAL at the forward configuration (B = 32), same kernels
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
        'fwd_eval_fp32_b32': {'ms': round(fwd_ms, 4), 'clips_per_s': round(Bf / (fwd_ms / 1e3), 1)},
        'rd_synth': {'ms': round(rd_ms, 4), 'clips_per_s': round(B / (rd_ms / 1e3), 1),
                     'maps_per_clip': 4},
        'roofline': None,
        'cpu_baseline': cpu,
    }
    print(json.dumps(out), flush=True)


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
