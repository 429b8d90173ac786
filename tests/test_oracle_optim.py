"""Pins of the AdamW / step-annealing oracle (oracle/optim.py): closed forms of the first steps
and of a constant gradient, and PyTorch's own AdamW and StepLR run in FP64 on the CPU."""
import numpy as np
import torch

from oracle import optim


def test_first_step_closed_form():
    rng = np.random.default_rng(0)
    w, g = rng.standard_normal(50), rng.standard_normal(50)
    lr, wd, eps = 1e-3, 5e-4, 1e-8
    w1, m1, v1 = optim.adamw_step(w, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps, weight_decay=wd)
    # mhat = g and vhat = g^2 on the first step
    np.testing.assert_allclose(w1, w * (1 - lr * wd) - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_constant_gradient_moves_lr_per_step():
    # with a constant gradient the bias corrections make mhat = g and vhat = g^2 at every step
    g = np.array([0.5, -2.0, 3e-3])
    w = np.zeros(3)
    m = v = np.zeros(3)
    for t in range(1, 8):
        w, m, v = optim.adamw_step(w, g, m, v, t, 1e-2, eps=0.0, weight_decay=0.0)
    np.testing.assert_allclose(w, -7 * 1e-2 * np.sign(g), rtol=1e-12)


def test_matches_torch_adamw_with_steplr():
    rng = np.random.default_rng(3)
    n, steps, lr0, gamma, step_size = 40, 12, 1e-2, 0.5, 5
    w0 = rng.standard_normal(n)
    grads = rng.standard_normal((steps, n))
    p = torch.nn.Parameter(torch.tensor(w0, dtype=torch.float64))
    opt = torch.optim.AdamW([p], lr=lr0, betas=(0.9, 0.999), eps=1e-8, weight_decay=5e-4)
    sch = torch.optim.lr_scheduler.StepLR(opt, step_size=step_size, gamma=gamma)
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, steps + 1):
        p.grad = torch.tensor(grads[t - 1], dtype=torch.float64)
        opt.step()
        sch.step()
        w, m, v = optim.adamw_step(w, grads[t - 1], m, v, t, optim.step_lr(lr0, gamma, step_size, t))
        np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_step_lr():
    assert optim.step_lr(1e-3, 0.1, 0, 1000) == 1e-3
    assert [optim.step_lr(1.0, 0.5, 3, t) for t in range(1, 8)] == [1, 1, 1, .5, .5, .5, .25]
