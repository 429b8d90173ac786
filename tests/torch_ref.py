"""The same network re-expressed with torch.nn.functional library operators in float64 on the CPU.

Used only as an independent pin of the FP64 oracle (forward values, and gradients through
torch autograd); it shares no code with the oracle beyond the parameter names it reads.
"""
import torch
import torch.nn.functional as F


def _bn(x, P, R, name, train, new_running):
    rm = R[name][0].clone()
    rv = R[name][1].clone()
    out = F.batch_norm(x, rm, rv, P[name + '.gamma'], P[name + '.beta'], training=train,
                       momentum=0.1, eps=1e-5)
    new_running[name] = (rm, rv)
    return out


def _eca(y, w):
    g = y.mean(dim=(2, 3))                                  # [B, C]
    s = F.conv1d(g[:, None, :], w.view(1, 1, 3), padding=1)[:, 0]
    return torch.sigmoid(s)[:, :, None, None] * y


def forward(P, R, x, train=True, res_k=4, head='identity', pw='dense'):
    """P: dict name -> float64 tensor, R: dict bn name -> (mean, var) tensors.  res_k = 3 takes
    the decoder residual as ConvTranspose3x3-s2-p1 with output padding 1; head = 'sigmoid'
    applies a logistic sigmoid to the output; pw = 'depthwise' makes the stage-1 1x1 branch a
    grouped (groups = C) convolution."""
    newR = {}
    t = F.conv2d(x, P['stem.conv.w'], padding=1)
    s0 = F.relu(_bn(t, P, R, 'stem.bn', train, newR))
    h = s0
    outs = {}
    for name, dec in (('enc0', False), ('enc1', False), ('dec0', True), ('dec1', True)):
        c = h.shape[1]
        gp = c if pw == 'depthwise' else 1
        if dec:
            p = F.conv_transpose2d(h, P[name + '.s1.pw.w'], groups=gp)
            d = F.conv_transpose2d(h, P[name + '.s1.dw.w'], padding=1, groups=c)
        else:
            p = F.conv2d(h, P[name + '.s1.pw.w'], groups=gp)
            d = F.conv2d(h, P[name + '.s1.dw.w'], padding=1, groups=c)
        u = (_bn(p, P, R, name + '.s1.pw_bn', train, newR) + _bn(d, P, R, name + '.s1.dw_bn', train, newR)
             + _bn(h, P, R, name + '.s1.id_bn', train, newR))
        x1 = F.relu(u)
        if dec:
            t = F.conv_transpose2d(x1, P[name + '.s2.main.w'], stride=2, padding=1)
            r = F.conv_transpose2d(h, P[name + '.s2.res.w'], stride=2, padding=1, output_padding=4 - res_k)
        else:
            t = F.conv2d(x1, P[name + '.s2.main.w'], stride=2, padding=1)
            r = F.conv2d(h, P[name + '.s2.res.w'], stride=2, padding=1)
        y = F.relu(_bn(t, P, R, name + '.s2.main_bn', train, newR)) + r
        e = _eca(y, P[name + '.eca.w'])
        if name == 'dec0':
            e = e + outs['enc0']
        if name == 'dec1':
            e = e + s0
        outs[name] = e
        h = e
    z = F.conv2d(h, P['head.conv.w'], bias=P['head.conv.b'], padding=1)
    if head == 'sigmoid':
        z = torch.sigmoid(z)
    return z, newR
