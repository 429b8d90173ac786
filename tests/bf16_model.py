"""BF16 storage model of the Radar-STDA forward (test infrastructure, built on the FP64 oracle's
layers): the network of oracle/net.py computed in FP64, with every tensor that the BF16 path
stores rounded to BF16 (round to nearest even) where it is stored:
  the input-module output s0; per block the stage-1 output x1, the stage-2 main convolution
  output T (its batch statistics taken before rounding), the residual convolution output R, the
  block output Y = ReLU(BN(T)) + R (the ECA average taken over the stored Y), and the block
  output after ECA and skip; the stage-2 convolution weights (main and residual).
Everything else (the input maps, batch-norm and ECA parameters, stage-1 and output-module
weights, all arithmetic) stays FP64.  The model isolates what the storage format alone costs:
its distance to the FP64 oracle is the format's error at those storage points, and a BF16 kernel
path that rounds at the same points should track it clip by clip."""
import numpy as np

from oracle import layers as L
from oracle import net


def _bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, running, x, mode='train', jitter=None):
    """(z [B, 1, H, W], cache) of the network with BF16 storage at the points listed above (the
    main architecture reading of oracle/net.py).  The cache has the layout of oracle/net.py's, so
    that net.backward differentiates this forward: its ReLU decisions, batch-norm inputs and ECA
    values are the model's stored ones, the rounding itself passing gradients unchanged.
    jitter = (seed, eps): every stored value is first multiplied by 1 + eps u, u uniform in
    [-1, 1) (seeded), which stands for the rounding of FP32 arithmetic ahead of a store (eps about
    2^-23); two such runs show how far two equally valid BF16 computations drift apart."""
    rng = np.random.default_rng(jitter[0]) if jitter else None

    def bf16(a):
        if rng is not None:
            a = a * (1.0 + jitter[1] * rng.uniform(-1.0, 1.0, np.shape(a)))
        return _bf16(a)

    assert net.ARCH == {'res_k': 4, 'head': 'identity', 'pw': 'dense'}
    P = dict(net.unflatten(params))
    for name in ('enc0', 'enc1', 'dec0', 'dec1'):
        for k in ('.s2.main.w', '.s2.res.w'):
            P[name + k] = _bf16(P[name + k])
    R = net.unflatten_running(running)
    newR = {k: (v[0].copy(), v[1].copy()) for k, v in R.items()}
    caches = {}
    x = np.asarray(x, np.float64)
    acts = {'x': x}
    t = L.conv2d(x, P['stem.conv.w'], stride=1, pad=1)
    s0 = bf16(L.relu(net._bn('stem.bn', t, P, R, mode, newR, caches)))
    acts['s0'] = s0
    h = s0
    for name, dec in (('enc0', False), ('enc1', False), ('dec0', True), ('dec1', True)):
        acts[name + '.in'] = h
        c = h.shape[1]
        conv = L.deconv2d if dec else L.conv2d
        p = conv(h, P[name + '.s1.pw.w'])
        d = conv(h, P[name + '.s1.dw.w'], stride=1, pad=1, groups=c)
        u = (net._bn(name + '.s1.pw_bn', p, P, R, mode, newR, caches)
             + net._bn(name + '.s1.dw_bn', d, P, R, mode, newR, caches)
             + net._bn(name + '.s1.id_bn', h, P, R, mode, newR, caches))
        x1 = bf16(L.relu(u))
        acts[name + '.x1'] = x1
        t = conv(x1, P[name + '.s2.main.w'], stride=2, pad=1)
        r = bf16(conv(h, P[name + '.s2.res.w'], stride=2, pad=1))
        bn = name + '.s2.main_bn'
        g, b = P[bn + '.gamma'], P[bn + '.beta']
        if mode == 'train':   # statistics of the unrounded output, as in the oracle
            mu = t.mean(axis=(0, 2, 3))
            var = ((t - mu[None, :, None, None]) ** 2).mean(axis=(0, 2, 3))
            newR[bn] = L.bn_running_update(R[bn][0], R[bn][1], {'mu': mu, 'var': var, 'n': t.shape[0] * t.shape[2] * t.shape[3]})
        else:
            mu, var = R[bn]
        inv = 1.0 / np.sqrt(var + L.BN_EPS)
        xhat = (bf16(t) - mu[None, :, None, None]) * inv[None, :, None, None]   # the stored T, normalised
        caches[bn] = {'xhat': xhat, 'inv': inv, 'mu': mu, 'var': var, 'mode': mode, 'gamma': g,
                      'n': t.shape[0] * t.shape[2] * t.shape[3]}
        m = L.relu(g[None, :, None, None] * xhat + b[None, :, None, None])
        acts[name + '.m'] = m
        y = bf16(m + r)
        e, caches[name + '.eca'] = L.eca_forward(y, P[name + '.eca.w'])
        if name == 'dec0':
            e = e + acts['enc0.out']
        elif name == 'dec1':
            e = e + s0
        h = bf16(e)
        acts[name + '.out'] = h
    z = L.conv2d(h, P['head.conv.w'], stride=1, pad=1) + P['head.conv.b'][0]
    acts['z'] = z
    return z, {'P': P, 'caches': caches, 'acts': acts, 'mode': mode, 'arch': dict(net.ARCH),
               'running': net.flatten_running(newR)}


bf16 = _bf16
