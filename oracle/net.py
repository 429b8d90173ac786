"""FP64 reference of the Radar-STDA network: forward (TRAIN / EVAL), hand-written backward,
reconstruction loss and the SGD update.

Test infrastructure only: the product library never imports or calls it.

Architecture (Radar-STDA, arXiv 2307.09063, Sec. IV):
  * input module: the three RD maps concatenated on the channel axis, frame t first
    (Sec. IV-B, Eq. (concat_operation)), then Conv3x3 3->16, BN, ReLU (Sec. IV-A names an
    input module; its content is a reading).
  * encoder h(.): two mobile encoder blocks 16->32 and 32->64 (Sec. IV-C,
    Eq. (mobile_encoder_stage1), Eq. (mobile_encoder_stage2)), each followed by ECA
    (Eq. (eca_process_equation)).
  * decoder f(.): two mobile decoder blocks 64->32 and 32->16 (Eq. (mobile_decoder_stage1),
    Eq. (mobile_decoder_stage2)), each followed by ECA; the two skip connections of Sec. IV-D
    add the same-size encoder feature (e0 after decoder block 0, the input-module output
    after decoder block 1).
  * output module: Conv3x3 16->1 with bias, no activation.
Stage 1 of a block: BN(PW1x1(x)) + BN(DW3x3(x)) + BN(x), ReLU; the 3x3 branch is depthwise
(the paper attributes the model's speed to depthwise separable convolution, Sec. VI-C) and the
1x1 branch dense (ablation: depthwise too, see ARCH).
Stage 2: ReLU(BN(Conv3x3-s2(x'))) + Conv3x3-s2(x) in the encoder; in the decoder both are
DeConv4x4-s2-p1 (the printed decoder residual cannot produce the stated output size).
Loss: mean squared error against the interference-free frame-t map (the paper names none).
"""
import numpy as np

from . import layers as L

C0 = 16
ENC_IN = (16, 32)      # encoder block input widths
DEC_IN = (64, 32)      # decoder block input widths

# Architecture readings (the main reading by default; the alternatives are ablations):
#   res_k : kernel of the decoder long residual, 4 (DeConv4x4-s2-p1) or 3 (DeConv3x3-s2-p1 with
#           one row and column of output padding, so that it also doubles the map)
#   head  : 'identity' (z = Conv3x3(d1) + b) or 'sigmoid' (z = sigmoid of that)
#   pw    : stage-1 1x1 branch 'dense' (C x C) or 'depthwise' (one weight per channel, groups = C)
ARCH = {'res_k': 4, 'head': 'identity', 'pw': 'dense'}


def set_arch(res_k=4, head='identity', pw='dense'):
    assert res_k in (3, 4) and head in ('identity', 'sigmoid') and pw in ('dense', 'depthwise')
    ARCH['res_k'], ARCH['head'], ARCH['pw'] = res_k, head, pw


def param_specs():
    """Ordered (name, shape, fan_in) of every parameter of the flat FP32 master buffer."""
    specs = [('stem.conv.w', (16, 3, 3, 3), 27),
             ('stem.bn.gamma', (16,), 0), ('stem.bn.beta', (16,), 0)]

    def block(name, c, co, dec):
        s = []
        if ARCH['pw'] == 'depthwise':
            s.append((f'{name}.s1.pw.w', (c, 1, 1, 1), 1))
        else:
            s.append((f'{name}.s1.pw.w', (c, c, 1, 1), c))
        s.append((f'{name}.s1.pw_bn.gamma', (c,), 0))
        s.append((f'{name}.s1.pw_bn.beta', (c,), 0))
        s.append((f'{name}.s1.dw.w', (c, 1, 3, 3), 9))
        s.append((f'{name}.s1.dw_bn.gamma', (c,), 0))
        s.append((f'{name}.s1.dw_bn.beta', (c,), 0))
        s.append((f'{name}.s1.id_bn.gamma', (c,), 0))
        s.append((f'{name}.s1.id_bn.beta', (c,), 0))
        if dec:
            s.append((f'{name}.s2.main.w', (c, co, 4, 4), c * 16))
        else:
            s.append((f'{name}.s2.main.w', (co, c, 3, 3), c * 9))
        s.append((f'{name}.s2.main_bn.gamma', (co,), 0))
        s.append((f'{name}.s2.main_bn.beta', (co,), 0))
        if dec:
            k = ARCH['res_k']
            s.append((f'{name}.s2.res.w', (c, co, k, k), c * k * k))
        else:
            s.append((f'{name}.s2.res.w', (co, c, 3, 3), c * 9))
        s.append((f'{name}.eca.w', (3,), 3))
        return s

    specs += block('enc0', 16, 32, False)
    specs += block('enc1', 32, 64, False)
    specs += block('dec0', 64, 32, True)
    specs += block('dec1', 32, 16, True)
    specs += [('head.conv.w', (1, 16, 3, 3), 144), ('head.conv.b', (1,), 0)]
    return specs


def bn_specs():
    """Ordered (name, channels) of every batch-norm layer; the running buffer holds, per layer,
    the running mean of its channels followed by the running variance."""
    out = [('stem.bn', 16)]
    for name, c, co in (('enc0', 16, 32), ('enc1', 32, 64), ('dec0', 64, 32), ('dec1', 32, 16)):
        out += [(f'{name}.s1.pw_bn', c), (f'{name}.s1.dw_bn', c), (f'{name}.s1.id_bn', c),
                (f'{name}.s2.main_bn', co)]
    return out


def param_count():
    return sum(int(np.prod(s)) for _, s, _ in param_specs())


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shape, _ in param_specs():
        n = int(np.prod(shape))
        out[name] = flat[off:off + n].reshape(shape)
        off += n
    assert off == flat.size
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel()
                           for name, _, _ in param_specs()])


def unflatten_running(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, c in bn_specs():
        out[name] = (flat[off:off + c].copy(), flat[off + c:off + 2 * c].copy())
        off += 2 * c
    assert off == flat.size
    return out


def flatten_running(d):
    return np.concatenate([np.concatenate([d[name][0], d[name][1]]) for name, _ in bn_specs()])


def running_count():
    return 2 * sum(c for _, c in bn_specs())


# --------------------------------------------------------------------- forward
def _bn(name, x, P, R, mode, newR, caches):
    out, c = L.bn_forward(x, P[name + '.gamma'], P[name + '.beta'], mode, *R[name])
    if mode == 'train':
        newR[name] = L.bn_running_update(R[name][0], R[name][1], c)
    caches[name] = c
    return out


def _stage1(name, x, P, R, mode, newR, caches, dec):
    c = x.shape[1]
    gp = c if ARCH['pw'] == 'depthwise' else 1
    if dec:
        p = L.deconv2d(x, P[name + '.s1.pw.w'], groups=gp)
        d = L.deconv2d(x, P[name + '.s1.dw.w'], stride=1, pad=1, groups=c)
    else:
        p = L.conv2d(x, P[name + '.s1.pw.w'], groups=gp)
        d = L.conv2d(x, P[name + '.s1.dw.w'], stride=1, pad=1, groups=c)
    u = (_bn(name + '.s1.pw_bn', p, P, R, mode, newR, caches)
         + _bn(name + '.s1.dw_bn', d, P, R, mode, newR, caches)
         + _bn(name + '.s1.id_bn', x, P, R, mode, newR, caches))
    return L.relu(u)


def _stage2(name, x, x1, P, R, mode, newR, caches, dec):
    if dec:
        t = L.deconv2d(x1, P[name + '.s2.main.w'], stride=2, pad=1)
        r = L.deconv2d(x, P[name + '.s2.res.w'], stride=2, pad=1, out_pad=4 - ARCH['res_k'])
    else:
        t = L.conv2d(x1, P[name + '.s2.main.w'], stride=2, pad=1)
        r = L.conv2d(x, P[name + '.s2.res.w'], stride=2, pad=1)
    m = L.relu(_bn(name + '.s2.main_bn', t, P, R, mode, newR, caches))
    return m + r, m


def forward(params, running, x, mode='train'):
    """Radar-STDA forward.

    params  : flat parameter vector (param_specs order) or dict.
    running : flat running-statistics vector (bn_specs order) or dict.
    x       : [B, 3, H, W], channel 0 = frame t, 1 = t-1, 2 = t-2.
    mode    : 'train' (batch statistics, running stats updated) or 'eval'.
    Returns (z [B, 1, H, W], new_running (flat), cache).
    """
    P = params if isinstance(params, dict) else unflatten(params)
    R = running if isinstance(running, dict) else unflatten_running(running)
    x = np.asarray(x, dtype=np.float64)
    B, F, H, W = x.shape
    assert F == 3 and H % 4 == 0 and W % 4 == 0
    newR = {k: (v[0].copy(), v[1].copy()) for k, v in R.items()}
    caches, acts = {}, {'x': x}

    t = L.conv2d(x, P['stem.conv.w'], stride=1, pad=1)
    s0 = L.relu(_bn('stem.bn', t, P, R, mode, newR, caches))
    acts['s0'] = s0
    h = s0
    for name in ('enc0', 'enc1'):
        acts[name + '.in'] = h
        x1 = _stage1(name, h, P, R, mode, newR, caches, dec=False)
        acts[name + '.x1'] = x1
        y, m = _stage2(name, h, x1, P, R, mode, newR, caches, dec=False)
        acts[name + '.m'] = m
        h, caches[name + '.eca'] = L.eca_forward(y, P[name + '.eca.w'])
        acts[name + '.out'] = h
    skips = {'dec0': acts['enc0.out'], 'dec1': s0}
    for name in ('dec0', 'dec1'):
        acts[name + '.in'] = h
        x1 = _stage1(name, h, P, R, mode, newR, caches, dec=True)
        acts[name + '.x1'] = x1
        y, m = _stage2(name, h, x1, P, R, mode, newR, caches, dec=True)
        acts[name + '.m'] = m
        e, caches[name + '.eca'] = L.eca_forward(y, P[name + '.eca.w'])
        h = e + skips[name]
        acts[name + '.out'] = h
    z = L.conv2d(h, P['head.conv.w'], stride=1, pad=1) + P['head.conv.b'][0]
    if ARCH['head'] == 'sigmoid':
        z = L.sigmoid(z)
    acts['z'] = z
    cache = {'P': P, 'caches': caches, 'acts': acts, 'mode': mode, 'arch': dict(ARCH)}
    return z, flatten_running(newR), cache


# -------------------------------------------------------------------- backward
def _stage2_backward(name, dy, x, x1, P, caches, acts, G, dec):
    m = acts[name + '.m']
    dbn = L.relu_backward(dy, m)
    dt, G[name + '.s2.main_bn.gamma'], G[name + '.s2.main_bn.beta'] = \
        L.bn_backward(dbn, caches[name + '.s2.main_bn'])
    wm, wr = P[name + '.s2.main.w'], P[name + '.s2.res.w']
    if dec:
        dx1 = L.deconv2d_grad_input(dt, wm, x1.shape, stride=2, pad=1)
        G[name + '.s2.main.w'] = L.deconv2d_grad_weight(x1, dt, wm.shape, stride=2, pad=1)
        op = 4 - wr.shape[2]   # output padding of the DeConv3x3-s2 residual reading
        dx = L.deconv2d_grad_input(dy, wr, x.shape, stride=2, pad=1, out_pad=op)
        G[name + '.s2.res.w'] = L.deconv2d_grad_weight(x, dy, wr.shape, stride=2, pad=1, out_pad=op)
    else:
        dx1 = L.conv2d_grad_input(dt, wm, x1.shape, stride=2, pad=1)
        G[name + '.s2.main.w'] = L.conv2d_grad_weight(x1, dt, wm.shape, stride=2, pad=1)
        dx = L.conv2d_grad_input(dy, wr, x.shape, stride=2, pad=1)
        G[name + '.s2.res.w'] = L.conv2d_grad_weight(x, dy, wr.shape, stride=2, pad=1)
    return dx1, dx


def _stage1_backward(name, dx1, x, x1, P, caches, G, dec):
    c = x.shape[1]
    du = L.relu_backward(dx1, x1)
    dp, G[name + '.s1.pw_bn.gamma'], G[name + '.s1.pw_bn.beta'] = \
        L.bn_backward(du, caches[name + '.s1.pw_bn'])
    dd, G[name + '.s1.dw_bn.gamma'], G[name + '.s1.dw_bn.beta'] = \
        L.bn_backward(du, caches[name + '.s1.dw_bn'])
    dx, G[name + '.s1.id_bn.gamma'], G[name + '.s1.id_bn.beta'] = \
        L.bn_backward(du, caches[name + '.s1.id_bn'])
    wp, wd = P[name + '.s1.pw.w'], P[name + '.s1.dw.w']
    gp = c if wp.shape[1] == 1 and c > 1 else 1      # depthwise 1x1 reading
    if dec:
        dx = dx + L.deconv2d_grad_input(dp, wp, x.shape, groups=gp)
        G[name + '.s1.pw.w'] = L.deconv2d_grad_weight(x, dp, wp.shape, groups=gp)
        dx = dx + L.deconv2d_grad_input(dd, wd, x.shape, stride=1, pad=1, groups=c)
        G[name + '.s1.dw.w'] = L.deconv2d_grad_weight(x, dd, wd.shape, stride=1, pad=1, groups=c)
    else:
        dx = dx + L.conv2d_grad_input(dp, wp, x.shape, groups=gp)
        G[name + '.s1.pw.w'] = L.conv2d_grad_weight(x, dp, wp.shape, groups=gp)
        dx = dx + L.conv2d_grad_input(dd, wd, x.shape, stride=1, pad=1, groups=c)
        G[name + '.s1.dw.w'] = L.conv2d_grad_weight(x, dd, wd.shape, stride=1, pad=1, groups=c)
    return dx


def backward(dz, cache, want_dx=False):
    """Exact adjoint of forward() (TRAIN mode statistics are differentiated through).

    dz : [B, 1, H, W] gradient of the loss w.r.t. z.
    Returns (flat gradient in param_specs order, dx [B, 3, H, W] or None).
    """
    P, caches, acts = cache['P'], cache['caches'], cache['acts']
    G = {}
    dz = np.asarray(dz, dtype=np.float64)
    if cache['arch']['head'] == 'sigmoid':
        z = acts['z']
        dz = dz * z * (1.0 - z)
    h = acts['dec1.out']
    G['head.conv.b'] = np.array([dz.sum()])
    G['head.conv.w'] = L.conv2d_grad_weight(h, dz, P['head.conv.w'].shape, stride=1, pad=1)
    dh = L.conv2d_grad_input(dz, P['head.conv.w'], h.shape, stride=1, pad=1)

    skip_grad = {}
    for name, skip in (('dec1', 's0'), ('dec0', 'enc0.out')):
        skip_grad[skip] = dh                        # d(out) flows unchanged into the skip
        dy, G[name + '.eca.w'] = L.eca_backward(dh, P[name + '.eca.w'], caches[name + '.eca'])
        x, x1 = acts[name + '.in'], acts[name + '.x1']
        dx1, dxr = _stage2_backward(name, dy, x, x1, P, caches, acts, G, dec=True)
        dh = _stage1_backward(name, dx1, x, x1, P, caches, G, dec=True) + dxr
    for name in ('enc1', 'enc0'):
        if name + '.out' in skip_grad:
            dh = dh + skip_grad[name + '.out']
        dy, G[name + '.eca.w'] = L.eca_backward(dh, P[name + '.eca.w'], caches[name + '.eca'])
        x, x1 = acts[name + '.in'], acts[name + '.x1']
        dx1, dxr = _stage2_backward(name, dy, x, x1, P, caches, acts, G, dec=False)
        dh = _stage1_backward(name, dx1, x, x1, P, caches, G, dec=False) + dxr
    ds0 = dh + skip_grad['s0']
    dt = L.relu_backward(ds0, acts['s0'])
    dt, G['stem.bn.gamma'], G['stem.bn.beta'] = L.bn_backward(dt, caches['stem.bn'])
    G['stem.conv.w'] = L.conv2d_grad_weight(acts['x'], dt, P['stem.conv.w'].shape, stride=1, pad=1)
    dx = None
    if want_dx:
        dx = L.conv2d_grad_input(dt, P['stem.conv.w'], acts['x'].shape, stride=1, pad=1)
    return flatten(G), dx


# ----------------------------------------------------------------- loss / SGD
def mse_loss(z, y):
    """Mean squared error over every element, and its gradient 2(z - y)/n."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = z.size
    d = z - y
    return float((d * d).sum() / n), 2.0 * d / n


def sgd_step(w, g, lr, weight_decay):
    """Plain SGD with L2 weight decay over the flat master buffer."""
    w = np.asarray(w, dtype=np.float64)
    return w - lr * (np.asarray(g, dtype=np.float64) + weight_decay * w)


def loss_and_grad(params, running, x, y, want_dx=False):
    """One TRAIN forward, the MSE against y, and the backward.  Returns
    (loss, flat grad, dx, z, new_running)."""
    z, new_running, cache = forward(params, running, x, 'train')
    loss, dz = mse_loss(z, y)
    g, dx = backward(dz, cache, want_dx)
    return loss, g, dx, z, new_running
