"""AdamW with step annealing on the GPU (stda_adamw_step) against the FP64 oracle
(oracle/optim.py): several steps over the full parameter vector with an annealing boundary in
between, the BF16 shadow copy, and replays of a captured step (the step counter and learning
rate live in device memory, so each replay is the next step)."""
import sys

import numpy as np
import pytest
import torch

from oracle import net, optim
from tests import gpu_util as U

pytestmark = pytest.mark.gpu
N = net.param_count()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _grads(k):
    rng = np.random.default_rng(11)
    return [(rng.standard_normal(N) * 10.0 ** rng.uniform(-4, 0, N)).astype(np.float32) for _ in range(k)]


def test_adamw_steps_match_oracle():
    from paper_2307_09063_amd import stda
    _say('adamw steps')
    lr0, gamma, step_size = 1e-2, 0.5, 2
    w0 = U.weights()
    grads = _grads(5)
    opt = stda.AdamW(N, lr=lr0, gamma=gamma, step_size=step_size)
    wd = U.dev(w0.copy())
    wb = torch.empty(N, dtype=torch.int16, device='cuda')
    w, m, v = w0.astype(np.float64), np.zeros(N), np.zeros(N)
    for t in range(1, 6):
        opt.step(wd, U.dev(grads[t - 1]), wb)
        w, m, v = optim.adamw_step(w, grads[t - 1], m, v, t, optim.step_lr(lr0, gamma, step_size, t))
    torch.cuda.synchronize()
    assert opt.t == 5
    assert U.rel_l2(opt.m.cpu().numpy(), m) < 1e-6
    assert U.rel_l2(opt.v.cpu().numpy(), v) < 1e-6
    got = wd.cpu().numpy()
    assert U.rel_l2(got - w0, w - w0) < 1e-5          # the accumulated update itself
    assert np.abs(got - w).max() <= 1e-6 * np.abs(w).max() + 1e-7
    bits = wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    back = bits.view(np.float32)
    assert np.all(np.abs(back - got) <= np.abs(got) * 2.0 ** -8)


def test_adamw_graph_replays_are_consecutive_steps():
    from paper_2307_09063_amd import stda
    _say('adamw graph')
    grads = _grads(1)
    g = U.dev(grads[0])
    w0 = U.weights()
    ea, ew = stda.AdamW(N, lr=1e-2, gamma=0.5, step_size=2), U.dev(w0.copy())
    eager = []
    for _ in range(4):
        ea.step(ew, g)
        torch.cuda.synchronize()
        eager.append(ew.cpu().numpy())
    ga, gw = stda.AdamW(N, lr=1e-2, gamma=0.5, step_size=2), U.dev(w0.copy())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ga.step(gw, g)
    torch.cuda.synchronize()
    assert ga.t == 0   # capturing ran nothing
    for k in range(4):
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device='cuda').sum()   # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gw.cpu().numpy(), eager[k])
        del junk
    assert ga.t == 4
