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


def relu_margin(cache):
    """Smallest |pre-activation| / rms(pre-activation of its layer) over every ReLU of the
    network.  Where this is below the FP32 rounding of the pre-activation, FP32 and FP64 may take
    different ReLU decisions, and either decision is a correct gradient at that precision."""
    P, C = cache['P'], cache['caches']

    def pre(name):
        c = C[name]
        return P[name + '.gamma'][None, :, None, None] * c['xhat'] + P[name + '.beta'][None, :, None, None]

    sites = [pre('stem.bn')] + [pre(f'{k}.s2.main_bn') for k in ('enc0', 'enc1', 'dec0', 'dec1')]
    sites += [pre(f'{k}.s1.pw_bn') + pre(f'{k}.s1.dw_bn') + pre(f'{k}.s1.id_bn') for k in ('enc0', 'enc1', 'dec0', 'dec1')]
    return min(float(np.abs(u).min() / np.sqrt((u * u).mean())) for u in sites)


def unambiguous(make, w, r, seed, margin=1e-5, tries=100):
    """First seed >= `seed` whose input (from make(seed)) keeps every ReLU decision at least
    `margin` (relative) away from its kink in TRAIN mode."""
    for k in range(tries):
        inp = make(seed + 1000 * k)
        _, _, cache = net.forward(w, r, inp[0], 'train')
        if relu_margin(cache) >= margin:
            return inp
    raise RuntimeError('no input with unambiguous ReLU decisions found')


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


def max_rel(a, b):
    """max |a - b| / max |b|: the largest element error on the tensor's own scale (an error
    confined to a few elements, e.g. tile borders, shows here long before it moves rel-L2)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0


def elem_tol(rel):
    """Element-wise gate that goes with a rel-L2 gate of `rel`."""
    return 10.0 * rel


def assert_close(a, b, rel, elem=None, what=''):
    """rel-L2(a, b) < rel and max_rel(a, b) <= elem (default elem_tol(rel))."""
    elem = elem_tol(rel) if elem is None else elem
    e1, e2 = rel_l2(a, b), max_rel(a, b)
    assert e1 < rel and e2 <= elem, f'{what} rel-L2 {e1:.3e} (gate {rel:.1e}), max-rel {e2:.3e} (gate {elem:.1e})'


def grad_failures(g_gpu, g_ref, rel, elem=None, skip=()):
    """{tensor: (rel-L2, max-rel)} of every parameter tensor that misses either gate."""
    elem = elem_tol(rel) if elem is None else elem
    bad = {}
    off = 0
    for name, shape, _ in net.param_specs():
        n = int(np.prod(shape))
        a, b = g_gpu[off:off + n], g_ref[off:off + n]
        off += n
        if name in skip or any(name.endswith(s) for s in skip):
            continue
        e1, e2 = rel_l2(a, b), max_rel(a, b)
        if not (e1 < rel and e2 <= elem):
            bad[name] = (e1, e2)
    return bad
