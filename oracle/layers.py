"""FP64 layer primitives of Radar-STDA and their hand-written adjoints.

Test infrastructure only: nothing in the product library imports this module.
Tensors are numpy float64 arrays in planar [B, C, H, W] order.  Every function
follows the textbook definition of its operation literally: a convolution is a
sum over kernel taps of shifted input slices, a transposed convolution is the
scatter definition, batch normalisation is the per-channel affine
normalisation.  No blocking, fusion or reordering beyond that.

Paper passages (Radar-STDA, arXiv 2307.09063):
  * mobile encoder block, stage 1 / stage 2 -- Sec. IV-C, Eq. (mobile_encoder_stage1),
    Eq. (mobile_encoder_stage2)
  * mobile decoder block -- Sec. IV-C, Eq. (mobile_decoder_stage1),
    Eq. (mobile_decoder_stage2); convolutions replaced by de-convolutions
  * efficient channel attention -- Sec. IV-C, Eq. (eca_process_equation)

Weight layouts (PyTorch convention):
  conv   w[Cout, Cin/g, k, k];   out[o, y, x] += w[o, c, ky, kx] * xpad[c, s*y+ky, s*x+kx]
  deconv w[Cin,  Cout/g, k, k];  out[o, s*i-p+ky, s*j-p+kx] += x[c, i, j] * w[c, o, ky, kx]
"""
import numpy as np

BN_EPS = 1e-5
BN_MOMENTUM = 0.1


# ---------------------------------------------------------------- convolution
def _pad(x, p):
    if p == 0:
        return x
    return np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))


def conv2d(x, w, stride=1, pad=0, groups=1):
    """Direct 2-D cross-correlation (zero padding), sum over taps."""
    B, C, H, W = x.shape
    Co, Cg, k, _ = w.shape
    assert C == Cg * groups and Co % groups == 0
    Ho = (H + 2 * pad - k) // stride + 1
    Wo = (W + 2 * pad - k) // stride + 1
    xp = _pad(x, pad)
    out = np.zeros((B, Co, Ho, Wo))
    og = Co // groups
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, :, ky:ky + stride * (Ho - 1) + 1:stride,
                       kx:kx + stride * (Wo - 1) + 1:stride]
            for g in range(groups):
                wt = w[g * og:(g + 1) * og, :, ky, kx]            # [og, Cg]
                pt = patch[:, g * Cg:(g + 1) * Cg]                # [B, Cg, Ho, Wo]
                out[:, g * og:(g + 1) * og] += np.einsum('oc,bcyx->boyx', wt, pt)
    return out


def conv2d_grad_input(dout, w, in_shape, stride=1, pad=0, groups=1):
    """Adjoint of conv2d with respect to its input: scatter dout back through every tap."""
    B, C, H, W = in_shape
    Co, Cg, k, _ = w.shape
    _, _, Ho, Wo = dout.shape
    og = Co // groups
    dxp = np.zeros((B, C, H + 2 * pad, W + 2 * pad))
    for ky in range(k):
        for kx in range(k):
            for g in range(groups):
                wt = w[g * og:(g + 1) * og, :, ky, kx]            # [og, Cg]
                contrib = np.einsum('oc,boyx->bcyx', wt, dout[:, g * og:(g + 1) * og])
                dxp[:, g * Cg:(g + 1) * Cg, ky:ky + stride * (Ho - 1) + 1:stride,
                    kx:kx + stride * (Wo - 1) + 1:stride] += contrib
    return dxp[:, :, pad:pad + H, pad:pad + W]


def conv2d_grad_weight(x, dout, w_shape, stride=1, pad=0, groups=1):
    """Adjoint of conv2d with respect to its weight: correlate input with dout."""
    Co, Cg, k, _ = w_shape
    _, _, Ho, Wo = dout.shape
    og = Co // groups
    xp = _pad(x, pad)
    dw = np.zeros(w_shape)
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, :, ky:ky + stride * (Ho - 1) + 1:stride,
                       kx:kx + stride * (Wo - 1) + 1:stride]
            for g in range(groups):
                dw[g * og:(g + 1) * og, :, ky, kx] = np.einsum(
                    'boyx,bcyx->oc', dout[:, g * og:(g + 1) * og], patch[:, g * Cg:(g + 1) * Cg])
    return dw


def deconv2d(x, w, stride=1, pad=0, groups=1, out_pad=0):
    """Transposed convolution by its scatter definition, then crop `pad` on each side; out_pad
    extra rows and columns are kept at the far end (zero where the scatter does not reach)."""
    B, C, H, W = x.shape
    Ci, Og, k, _ = w.shape
    assert Ci == C and C % groups == 0
    cg = C // groups
    Co = Og * groups
    Hf = (H - 1) * stride + k + out_pad
    Wf = (W - 1) * stride + k + out_pad
    full = np.zeros((B, Co, Hf, Wf))
    for ky in range(k):
        for kx in range(k):
            for g in range(groups):
                wt = w[g * cg:(g + 1) * cg, :, ky, kx]            # [cg, Og]
                full[:, g * Og:(g + 1) * Og, ky:ky + stride * (H - 1) + 1:stride,
                     kx:kx + stride * (W - 1) + 1:stride] += np.einsum(
                         'co,bcij->boij', wt, x[:, g * cg:(g + 1) * cg])
    Ho = (H - 1) * stride - 2 * pad + k + out_pad
    Wo = (W - 1) * stride - 2 * pad + k + out_pad
    return full[:, :, pad:pad + Ho, pad:pad + Wo]


def deconv2d_grad_input(dout, w, in_shape, stride=1, pad=0, groups=1, out_pad=0):
    """Adjoint of deconv2d w.r.t. its input: gather dout (zero-extended by the crop) at every tap."""
    B, C, H, W = in_shape
    Ci, Og, k, _ = w.shape
    cg = C // groups
    Hf = (H - 1) * stride + k + out_pad
    Wf = (W - 1) * stride + k + out_pad
    full = np.zeros((B, dout.shape[1], Hf, Wf))
    full[:, :, pad:pad + dout.shape[2], pad:pad + dout.shape[3]] = dout
    dx = np.zeros(in_shape)
    for ky in range(k):
        for kx in range(k):
            sl = full[:, :, ky:ky + stride * (H - 1) + 1:stride, kx:kx + stride * (W - 1) + 1:stride]
            for g in range(groups):
                wt = w[g * cg:(g + 1) * cg, :, ky, kx]
                dx[:, g * cg:(g + 1) * cg] += np.einsum('co,boij->bcij', wt, sl[:, g * Og:(g + 1) * Og])
    return dx


def deconv2d_grad_weight(x, dout, w_shape, stride=1, pad=0, groups=1, out_pad=0):
    """Adjoint of deconv2d w.r.t. its weight."""
    B, C, H, W = x.shape
    Ci, Og, k, _ = w_shape
    cg = C // groups
    Hf = (H - 1) * stride + k + out_pad
    Wf = (W - 1) * stride + k + out_pad
    full = np.zeros((B, dout.shape[1], Hf, Wf))
    full[:, :, pad:pad + dout.shape[2], pad:pad + dout.shape[3]] = dout
    dw = np.zeros(w_shape)
    for ky in range(k):
        for kx in range(k):
            sl = full[:, :, ky:ky + stride * (H - 1) + 1:stride, kx:kx + stride * (W - 1) + 1:stride]
            for g in range(groups):
                dw[g * cg:(g + 1) * cg, :, ky, kx] = np.einsum(
                    'bcij,boij->co', x[:, g * cg:(g + 1) * cg], sl[:, g * Og:(g + 1) * Og])
    return dw


# ---------------------------------------------------------- batch normalisation
def bn_forward(x, gamma, beta, mode, running_mean=None, running_var=None):
    """Per-channel batch normalisation.

    TRAIN: statistics over (batch, h, w), biased variance for the normalisation.
    EVAL: the running statistics.
    Returns (out, cache); cache holds what the adjoint needs.
    """
    if mode == 'train':
        mu = x.mean(axis=(0, 2, 3))
        var = ((x - mu[None, :, None, None]) ** 2).mean(axis=(0, 2, 3))
    else:
        mu = running_mean
        var = running_var
    inv = 1.0 / np.sqrt(var + BN_EPS)
    xhat = (x - mu[None, :, None, None]) * inv[None, :, None, None]
    out = gamma[None, :, None, None] * xhat + beta[None, :, None, None]
    return out, {'xhat': xhat, 'inv': inv, 'mu': mu, 'var': var, 'mode': mode,
                 'gamma': gamma, 'n': x.shape[0] * x.shape[2] * x.shape[3]}


def bn_running_update(running_mean, running_var, cache):
    """Exponential running-statistics update; the running variance takes the unbiased estimate."""
    n = cache['n']
    unbiased = cache['var'] * n / (n - 1) if n > 1 else cache['var']
    new_mean = (1 - BN_MOMENTUM) * running_mean + BN_MOMENTUM * cache['mu']
    new_var = (1 - BN_MOMENTUM) * running_var + BN_MOMENTUM * unbiased
    return new_mean, new_var


def bn_backward(dout, cache):
    """Adjoint of bn_forward.  Returns (dx, dgamma, dbeta)."""
    xhat, inv, gamma = cache['xhat'], cache['inv'], cache['gamma']
    dbeta = dout.sum(axis=(0, 2, 3))
    dgamma = (dout * xhat).sum(axis=(0, 2, 3))
    if cache['mode'] == 'train':
        n = cache['n']
        dx = (gamma * inv)[None, :, None, None] * (
            dout - dbeta[None, :, None, None] / n - xhat * dgamma[None, :, None, None] / n)
    else:
        dx = (gamma * inv)[None, :, None, None] * dout
    return dx, dgamma, dbeta


# ----------------------------------------------------------------- activations
def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(dout, out):
    """ReLU adjoint given the ReLU output (derivative 0 at the kink)."""
    return dout * (out > 0)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


# ------------------------------------------------- efficient channel attention
def eca_forward(y, w):
    """GAP over (h, w) per clip and channel, a 1-D cross-correlation of width 3 over the
    channel axis with zero padding and no bias, a logistic sigmoid, and a channel scale."""
    g = y.mean(axis=(2, 3))                                        # [B, C]
    gp = np.pad(g, ((0, 0), (1, 1)))
    s = w[0] * gp[:, :-2] + w[1] * gp[:, 1:-1] + w[2] * gp[:, 2:]   # [B, C]
    a = sigmoid(s)
    return a[:, :, None, None] * y, {'g': g, 'a': a, 'y': y}


def eca_backward(dout, w, cache):
    """Adjoint of eca_forward.  Returns (dy, dw)."""
    y, a, g = cache['y'], cache['a'], cache['g']
    hw = y.shape[2] * y.shape[3]
    da = (dout * y).sum(axis=(2, 3))                               # [B, C]
    ds = da * a * (1.0 - a)
    gp = np.pad(g, ((0, 0), (1, 1)))
    dw = np.array([(ds * gp[:, :-2]).sum(), (ds * gp[:, 1:-1]).sum(), (ds * gp[:, 2:]).sum()])
    # s[c] = w0 g[c-1] + w1 g[c] + w2 g[c+1]  =>  dg[c] = w0 ds[c+1] + w1 ds[c] + w2 ds[c-1]
    dsp = np.pad(ds, ((0, 0), (1, 1)))
    dg = w[0] * dsp[:, 2:] + w[1] * dsp[:, 1:-1] + w[2] * dsp[:, :-2]
    dy = a[:, :, None, None] * dout + (dg / hw)[:, :, None, None]
    return dy, dw
