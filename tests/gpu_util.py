"""Helpers of the GPU parity tests: seeded inputs, oracle runs, error metrics."""
import numpy as np
import torch

from oracle import net, rdsynth
from paper_2307_09063_amd import inputs


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def weights(seed=1234, perturb=0.1):
    """Kaiming-uniform weights with the BN affine moved off (1, 0) so every term is exercised."""
    w = inputs.make_weights(net.param_specs(), seed)
    rng = np.random.default_rng(seed + 1)
    out = w.astype(np.float64)
    off = 0
    for name, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        if name.endswith('.gamma') or name.endswith('.beta') or name.endswith('.b'):
            out[off:off + n] += perturb * rng.standard_normal(n)
        off += n
    return out.astype(np.float32)


def running(seed=7, perturb=True):
    r = inputs.make_running([c for _, c in net.bn_specs()]).astype(np.float64)
    if perturb:
        rng = np.random.default_rng(seed)
        off = 0
        for _, c in net.bn_specs():
            r[off:off + c] = 0.2 * rng.standard_normal(c)
            r[off + c:off + 2 * c] = rng.uniform(0.3, 2.0, c)
            off += 2 * c
    return r.astype(np.float32)


def maps(B, H, W, seed):
    return inputs.random_maps((B, 3, H, W), seed), inputs.random_maps((B, 1, H, W), seed + 100)


def rd_maps(B, N, M, seed, **kw):
    tab, meta = inputs.make_scenes(B, N, M, seed, **kw)
    x, clean = rdsynth.synth(inputs.scene_dict(tab, meta))
    return x.astype(np.float32), clean.astype(np.float32), tab, meta


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def per_tensor_errors(g_gpu, g_ref):
    """rel-L2 of every parameter tensor."""
    out = {}
    off = 0
    for name, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        out[name] = rel_l2(g_gpu[off:off + n], g_ref[off:off + n])
        off += n
    return out
