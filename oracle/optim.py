"""FP64 reference of the paper's optimizer: AdamW with decoupled weight decay and a step-annealed
learning rate (Radar-STDA, arXiv 2307.09063, Table 5; AdamW of Loshchilov and Hutter).

Test infrastructure only: the product library never imports or calls it.

Table 5 names the optimizer, the initial learning rate, the weight decay and "step annealing",
but no moment coefficients, epsilon or annealing period, so these are readings:
  * the common deep-learning form of AdamW, in which the decoupled decay is scaled by the
    learning rate: w <- w (1 - lr_t lambda) - lr_t mhat / (sqrt(vhat) + eps), with
    m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, mhat = m / (1 - b1^t),
    vhat = v / (1 - b2^t), t = 1, 2, ... ; b1 = 0.9, b2 = 0.999, eps = 1e-8 by default;
  * step annealing counted in optimizer steps: lr_t = lr0 gamma^floor((t - 1) / step_size)
    (constant when step_size is 0).
"""
import numpy as np


def step_lr(lr0, gamma, step_size, t):
    """Learning rate of optimizer step t (1-based)."""
    if step_size <= 0:
        return float(lr0)
    return float(lr0) * float(gamma) ** ((t - 1) // step_size)


def adamw_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=5e-4):
    """One AdamW step t (1-based) at learning rate lr; returns (w, m, v) in FP64."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    w = w * (1.0 - lr * weight_decay) - lr * mhat / (np.sqrt(vhat) + eps)
    return w, m, v
