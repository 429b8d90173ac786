"""Thin Python binding of libstda.so (include/stda.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; PyTorch supplies device memory and
the current stream.  Importing this module loads the library and raises if it is missing:
there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libstda.so')

STDA_OK = 0
FP32, BF16 = 0, 1
EVAL, TRAIN = 0, 1


class StdaError(RuntimeError):
    pass


class Segment(ctypes.Structure):
    _fields_ = [('n', ctypes.c_int32), ('H', ctypes.c_int32), ('W', ctypes.c_int32),
                ('x_off', ctypes.c_int64), ('z_off', ctypes.c_int64)]


class ParamDesc(ctypes.Structure):
    _fields_ = [('name', ctypes.c_char * 40), ('offset', ctypes.c_int64), ('ndim', ctypes.c_int32),
                ('shape', ctypes.c_int32 * 4), ('fan_in', ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise StdaError(f'{LIB_PATH} is missing: build it with `python -m paper_2307_09063_amd.build` '
                        '(there is no CPU fallback)')
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    F, U32 = ctypes.c_float, ctypes.c_uint32
    sig = {
        'stda_status_string': (ctypes.c_char_p, [I]),
        'stda_last_hip_error': (I, []),
        'stda_param_count': (SZ, []),
        'stda_param_table': (I, [P, I]),
        'stda_bn_layer_count': (I, []),
        'stda_running_count': (SZ, []),
        'stda_set_arch': (I, [I]),
        'stda_get_arch': (I, []),
        'stda_workspace_size': (I, [P, I, I, I, I, P, P]),
        'stda_forward': (I, [P, I, P, P, P, P, P, SZ, P, SZ, I, I, I, P]),
        'stda_forward_noalloc': (I, [P, I, P, P, P, P, I, P]),
        'stda_eval_fold_size': (I, [I, P]),
        'stda_eval_fold': (I, [P, P, P, SZ, I, P]),
        'stda_forward_folded': (I, [P, I, P, P, SZ, P, P, SZ, I, P]),
        'stda_forward_folded_graph_create': (I, [P, I, P, P, SZ, P, P, SZ, I, P, P]),
        'stda_backward': (I, [P, I, P, P, P, P, SZ, P, P, P, SZ, I, I, P]),
        'stda_mse_loss': (I, [P, I, P, P, P, P, P, SZ, P]),
        'stda_sgd_step': (I, [P, P, I64, F, F, P, P]),
        'stda_sinr': (I, [P, P, P, I, I, I, P, P]),
        'stda_train_step_graph_create': (I, [P, I, P, P, P, P, P, P, P, P, P, SZ, P, SZ, I, I, F, F, P, P,
                                             P]),
        'stda_graph_launch': (I, [P, P]),
        'stda_forward_graph_create': (I, [P, I, P, P, P, P, P, SZ, P, SZ, I, I, P, P]),
        'stda_graph_destroy': (I, [P]),
        'stda_profile_select': (I, [ctypes.c_char_p]),
        'stda_profile_read': (I, [P, P]),
        'stda_profile_report': (I, [P, SZ, P]),
        'stda_set_grid_cap': (I, [I]),
        'stda_get_grid_cap': (I, []),
        'stda_tune_count': (I, [I]),
        'stda_tune_set': (I, [I, I, I, I]),
        'stda_tune_get': (I, [I, I, I, P]),
        'stda_autotune': (I, [P, I, P, P, P, P, P, P, P, P, P, SZ, P, SZ, I, I, I, P, P, SZ, P]),
        'stda_cfar': (I, [P, I, I, I, I, I, I, I, ctypes.c_double, P, P, P, P]),
        'stda_evm': (I, [P, P, P, I, I, I, P, P]),
        'stda_adamw_step': (I, [P, P, P, P, I64, P, P, P]),
        'rd_synth_workspace_size': (SZ, [I, I, I]),
        'rd_synth': (I, [P, I, I, I, U32, F, I, P, P, P, SZ, P]),
        'rd_synth_host_workspace_size': (SZ, [I, I, I]),
        'rd_synth_host': (I, [P, I, I, I, U32, F, I, P, P, P, SZ, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTS = ('stda_status_string', 'stda_last_hip_error', 'stda_param_count', 'stda_param_table',
           'stda_bn_layer_count', 'stda_running_count', 'stda_set_arch', 'stda_get_arch', 'stda_workspace_size', 'stda_forward',
           'stda_forward_noalloc', 'stda_eval_fold_size', 'stda_eval_fold', 'stda_forward_folded',
           'stda_forward_folded_graph_create',
           'stda_backward', 'stda_mse_loss', 'stda_sgd_step', 'stda_sinr', 'stda_train_step_graph_create',
           'stda_graph_launch', 'stda_graph_destroy', 'stda_forward_graph_create', 'stda_profile_select',
           'stda_profile_read', 'stda_profile_report', 'stda_set_grid_cap', 'stda_get_grid_cap', 'stda_tune_count', 'stda_tune_set', 'stda_tune_get',
           'stda_autotune', 'stda_cfar', 'stda_evm', 'stda_adamw_step', 'rd_synth_workspace_size', 'rd_synth',
           'rd_synth_host_workspace_size', 'rd_synth_host')


def _check(status, what):
    if status != STDA_OK:
        msg = _lib.stda_status_string(status).decode()
        hip = _lib.stda_last_hip_error()
        raise StdaError(f'{what}: {msg} (status {status}, hip {hip})')


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise StdaError('tensor arguments must be device tensors')
    if not t.is_contiguous():
        raise StdaError('tensor arguments must be contiguous')
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _seg_array(segs):
    arr = (Segment * len(segs))()
    for i, s in enumerate(segs):
        arr[i] = s if isinstance(s, Segment) else Segment(*s)
    return arr


# ------------------------------------------------------------------------ tables
ARCH_RES3, ARCH_SIGMOID, ARCH_PW_DW = 1, 2, 4


def set_arch(res_k=4, head='identity', pw='dense'):
    """Process-wide architecture reading: res_k = 3 takes the decoder long residual as
    DeConv3x3-s2-p1 with output padding 1 (4: DeConv4x4-s2-p1), head = 'sigmoid' puts a logistic
    sigmoid on the output, pw = 'depthwise' makes the stage-1 1x1 branch depthwise.  Parameter
    vectors, saved buffers and graphs are tied to the setting they were made under."""
    if res_k not in (3, 4) or head not in ('identity', 'sigmoid') or pw not in ('dense', 'depthwise'):
        raise StdaError(f'unknown architecture res_k={res_k} head={head} pw={pw}')
    flags = ((ARCH_RES3 if res_k == 3 else 0) | (ARCH_SIGMOID if head == 'sigmoid' else 0)
             | (ARCH_PW_DW if pw == 'depthwise' else 0))
    _check(_lib.stda_set_arch(flags), 'stda_set_arch')


def get_arch():
    f = int(_lib.stda_get_arch())
    return {'res_k': 3 if f & ARCH_RES3 else 4, 'head': 'sigmoid' if f & ARCH_SIGMOID else 'identity',
            'pw': 'depthwise' if f & ARCH_PW_DW else 'dense'}


def param_count():
    return int(_lib.stda_param_count())


def running_count():
    return int(_lib.stda_running_count())


def param_table():
    n = _lib.stda_param_table(None, 0)
    arr = (ParamDesc * n)()
    _lib.stda_param_table(ctypes.cast(arr, ctypes.c_void_p), n)
    return [{'name': d.name.decode(), 'offset': d.offset, 'shape': tuple(d.shape[:d.ndim]),
             'fan_in': d.fan_in} for d in arr]


def param_specs():
    """(name, shape, fan_in) in buffer order, the form the input generators take."""
    return [(d['name'], d['shape'], d['fan_in']) for d in param_table()]


def bn_channels():
    """Channels of each BN layer in running-buffer order."""
    out = [16]
    for cin, cout in ((16, 32), (32, 64), (64, 32), (32, 16)):
        out += [cin, cin, cin, cout]
    return out


def uniform_segments(n, H, W):
    return [Segment(n, H, W, 0, 0)]


def packed_segments(sizes_counts):
    """[(n, H, W), ...] -> segments packed back to back."""
    segs, xo, zo = [], 0, 0
    for n, H, W in sizes_counts:
        segs.append(Segment(n, H, W, xo, zo))
        xo += 3 * n * H * W
        zo += n * H * W
    return segs


# ------------------------------------------------------------------------ network
def workspace_size(segs, dtype=FP32, mode=TRAIN, recompute=0):
    sv, ws = ctypes.c_size_t(0), ctypes.c_size_t(0)
    arr = _seg_array(segs)
    _check(_lib.stda_workspace_size(ctypes.cast(arr, ctypes.c_void_p), len(segs), dtype, mode, recompute,
                                    ctypes.byref(sv), ctypes.byref(ws)), 'stda_workspace_size')
    return sv.value, ws.value


def alloc_bytes(n, device='cuda'):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def forward(segs, x, w, running, z, saved, ws, dtype=FP32, mode=EVAL, recompute=0):
    arr = _seg_array(segs)
    _check(_lib.stda_forward(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(w), _ptr(running),
                             _ptr(z), _ptr(saved), saved.numel() if saved is not None else 0, _ptr(ws),
                             ws.numel(), dtype, mode, recompute, _stream()), 'stda_forward')


NOALLOC_WS_MAX = 32 << 20


def forward_noalloc(segs, x, w, running, z, dtype=FP32):
    """EVAL forward on the library's own static device scratch (no workspace argument)."""
    arr = _seg_array(segs)
    _check(_lib.stda_forward_noalloc(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(w), _ptr(running),
                                     _ptr(z), dtype, _stream()), 'stda_forward_noalloc')


def eval_fold_size(dtype=FP32):
    n = ctypes.c_size_t()
    _check(_lib.stda_eval_fold_size(dtype, ctypes.byref(n)), 'stda_eval_fold_size')
    return n.value


def eval_fold(w, running, folded, dtype=FP32):
    """Folded EVAL parameters of (w, running) into the device byte buffer `folded`."""
    _check(_lib.stda_eval_fold(_ptr(w), _ptr(running), _ptr(folded), folded.numel(), dtype, _stream()),
           'stda_eval_fold')


def forward_folded(segs, x, folded, z, ws, dtype=FP32):
    arr = _seg_array(segs)
    _check(_lib.stda_forward_folded(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(folded),
                                    folded.numel(), _ptr(z), _ptr(ws), ws.numel(), dtype, _stream()),
           'stda_forward_folded')


def backward(segs, x, dz, w, saved, dw, dx, ws, dtype=FP32, recompute=0):
    arr = _seg_array(segs)
    _check(_lib.stda_backward(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(dz), _ptr(w),
                              _ptr(saved), saved.numel(), _ptr(dw), _ptr(dx), _ptr(ws), ws.numel(), dtype,
                              recompute, _stream()), 'stda_backward')


def mse_loss(segs, z, y, loss, dz, ws):
    arr = _seg_array(segs)
    _check(_lib.stda_mse_loss(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(z), _ptr(y), _ptr(loss),
                              _ptr(dz), _ptr(ws), ws.numel(), _stream()), 'stda_mse_loss')


def sgd_step(w, dw, lr, weight_decay, w_bf16=None):
    _check(_lib.stda_sgd_step(_ptr(w), _ptr(dw), w.numel(), lr, weight_decay, _ptr(w_bf16), _stream()),
           'stda_sgd_step')


class AdamW:
    """Device state of stda_adamw_step: moments m, v and the hyper-parameter / step-counter record
    (lr, beta1, beta2, eps, weight_decay, gamma as FP64, then step_size and t as int32)."""
    STATE_BYTES, T_OFFSET = 56, 52

    def __init__(self, n, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=5e-4, gamma=0.1, step_size=0,
                 device='cuda'):
        import numpy as np
        self.n = n
        self.m = torch.zeros(n, device=device)
        self.v = torch.zeros(n, device=device)
        rec = np.zeros(7, dtype=np.float64)
        rec[:6] = [lr, betas[0], betas[1], eps, weight_decay, gamma]
        ints = rec.view(np.int32)
        ints[12], ints[13] = step_size, 0
        self.state = torch.from_numpy(rec.view(np.uint8).copy()).to(device)

    @property
    def t(self):
        import numpy as np
        return int(self.state.cpu().numpy().view(np.int32)[13])

    def step(self, w, dw, w_bf16=None):
        _check(_lib.stda_adamw_step(_ptr(w), _ptr(dw), _ptr(self.m), _ptr(self.v), self.n, _ptr(self.state),
                                    _ptr(w_bf16), _stream()), 'stda_adamw_step')


def sinr(maps, o_mask, n_mask, out):
    n, H, W = maps.shape[0], maps.shape[-2], maps.shape[-1]
    _check(_lib.stda_sinr(_ptr(maps), _ptr(o_mask), _ptr(n_mask), n, H, W, _ptr(out), _stream()), 'stda_sinr')


# ------------------------------------------------------------------------ detection step
CFAR_DEFAULT = dict(guard_r=2, guard_d=2, train_r=4, train_d=4, pfa=1e-3)


def cfar(maps, det, guard_r=2, guard_d=2, train_r=4, train_d=4, pfa=1e-3, o_mask=None, counts=None):
    """CA-CFAR of maps [n, (1,) H, W] (FP32, device) into det (uint8, same cells); counts
    (int32 [n, 2]) receives detections and detections on o_mask cells when given."""
    n, H, W = maps.shape[0], maps.shape[-2], maps.shape[-1]
    _check(_lib.stda_cfar(_ptr(maps), n, H, W, guard_r, guard_d, train_r, train_d, float(pfa), _ptr(det),
                          _ptr(o_mask), _ptr(counts), _stream()), 'stda_cfar')


def evm(est, clean, o_mask, out):
    """EVM per map (FP64 out [n]) over the o_mask cells."""
    n, H, W = est.shape[0], est.shape[-2], est.shape[-1]
    _check(_lib.stda_evm(_ptr(est), _ptr(clean), _ptr(o_mask), n, H, W, _ptr(out), _stream()), 'stda_evm')


# ------------------------------------------------------------------------ captured step
class TrainStepGraph:
    """One captured training step (forward, loss, backward, SGD) replayed with launch()."""

    def __init__(self, segs, x, y, w, running, z, loss, dz, dw, saved, ws, dtype=FP32, recompute=0, lr=1e-3,
                 weight_decay=5e-4, w_bf16=None, stream=None):
        self.stream = stream or torch.cuda.Stream()
        self._keep = (x, y, w, running, z, loss, dz, dw, saved, ws, w_bf16)
        arr = _seg_array(segs)
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(_lib.stda_train_step_graph_create(
                ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(y), _ptr(w), _ptr(running), _ptr(z),
                _ptr(loss), _ptr(dz), _ptr(dw), _ptr(saved), saved.numel(), _ptr(ws), ws.numel(), dtype, recompute,
                lr, weight_decay, _ptr(w_bf16), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                'stda_train_step_graph_create')
        self.handle = h

    def launch(self):
        _check(_lib.stda_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)), 'stda_graph_launch')

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(_lib.stda_graph_destroy(h), 'stda_graph_destroy')

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FoldedForwardGraph:
    """The folded EVAL forward captured into a graph and replayed with launch(); buffers bound at
    capture."""

    def __init__(self, segs, x, folded, z, ws, dtype=FP32, stream=None):
        self.stream = stream or torch.cuda.Stream()
        self._keep = (x, folded, z, ws)
        arr = _seg_array(segs)
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(_lib.stda_forward_folded_graph_create(
                ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(folded), folded.numel(), _ptr(z),
                _ptr(ws), ws.numel(), dtype, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                'stda_forward_folded_graph_create')
        self.handle = h

    def launch(self):
        _check(_lib.stda_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)), 'stda_graph_launch')

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(_lib.stda_graph_destroy(h), 'stda_graph_destroy')

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ForwardGraph:
    """One captured forward (EVAL by default) replayed with launch(); buffers bound at capture."""

    def __init__(self, segs, x, w, running, z, ws, dtype=FP32, mode=EVAL, saved=None, stream=None):
        self.stream = stream or torch.cuda.Stream()
        self._keep = (x, w, running, z, ws, saved)
        arr = _seg_array(segs)
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(_lib.stda_forward_graph_create(
                ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(w), _ptr(running), _ptr(z), _ptr(saved),
                saved.numel() if saved is not None else 0, _ptr(ws), ws.numel(), dtype, mode,
                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), 'stda_forward_graph_create')
        self.handle = h

    def launch(self):
        _check(_lib.stda_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)), 'stda_graph_launch')

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(_lib.stda_graph_destroy(h), 'stda_graph_destroy')

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------ timing hook
def profile_select(tag):
    _check(_lib.stda_profile_select(tag.encode() if tag else None), 'stda_profile_select')


def profile_read():
    tot, cnt = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(_lib.stda_profile_read(ctypes.byref(tot), ctypes.byref(cnt)), 'stda_profile_read')
    return tot.value, cnt.value


def profile_report():
    """{tag: (launches, total_ms)} of the launches recorded since the last select."""
    need = ctypes.c_size_t(0)
    _check(_lib.stda_profile_report(None, 0, ctypes.byref(need)), 'stda_profile_report')
    buf = ctypes.create_string_buffer(need.value + 1)
    _check(_lib.stda_profile_report(buf, need.value + 1, ctypes.byref(need)), 'stda_profile_report')
    out = {}
    for line in buf.value.decode().splitlines():
        tag, n, ms = line.split('\t')
        out[tag] = (int(n), float(ms))
    return out


# ------------------------------------------------------------------------ tile-shape autotuning
TUNE_FWD, TUNE_DGRAD, TUNE_WGRAD, TUNE_S1_BWD = 0, 1, 2, 3
TUNE_KINDS = (TUNE_FWD, TUNE_DGRAD, TUNE_WGRAD, TUNE_S1_BWD)


def set_grid_cap(cap):
    """Bound the workgroups of every tiled network kernel (0 = no bound), so that a small batch
    walks several tiles per workgroup as a large one does."""
    _check(_lib.stda_set_grid_cap(int(cap)), 'stda_set_grid_cap')


def get_grid_cap():
    return int(_lib.stda_get_grid_cap())


def tune_count(kind):
    n = _lib.stda_tune_count(kind)
    if n < 0:
        _check(n, 'stda_tune_count')
    return n


def tune_set(kind, dtype, block, variant):
    _check(_lib.stda_tune_set(kind, dtype, block, variant), 'stda_tune_set')


def tune_get(kind, dtype, block):
    v = ctypes.c_int(0)
    _check(_lib.stda_tune_get(kind, dtype, block, ctypes.byref(v)), 'stda_tune_get')
    return v.value


def tune_table(dtype):
    """{(kind, block): variant} currently in force for `dtype`."""
    return {(k, b): tune_get(k, dtype, b) for k in TUNE_KINDS for b in range(4)}


def autotune(segs, x, y, w, running, z, loss, dz, dw, saved, ws, dtype=FP32, recompute=0, reps=3):
    """Run the library's autotuner on these buffers (running is updated by the trial steps; w is
    not).  Returns {(kind, block): (chosen variant, [ms per variant])}; the choice is in force."""
    arr = _seg_array(segs)
    need = ctypes.c_size_t(0)
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.stda_autotune(ctypes.cast(arr, ctypes.c_void_p), len(segs), _ptr(x), _ptr(y), _ptr(w), _ptr(running),
                              _ptr(z), _ptr(loss), _ptr(dz), _ptr(dw), _ptr(saved), saved.numel(), _ptr(ws), ws.numel(),
                              dtype, recompute, reps, _stream(), buf, len(buf), ctypes.byref(need)), 'stda_autotune')
    out = {}
    for line in buf.value.decode().splitlines():
        f = line.split('\t')
        out[(int(f[0]), int(f[1]))] = (int(f[-1]), [float(v) for v in f[2:-1]])
    return out


# ------------------------------------------------------------------------ RD maps
def rd_synth_workspace_size(n_clips, N, M):
    return int(_lib.rd_synth_workspace_size(n_clips, N, M))


def rd_synth(scenes_dev, n_clips, N, M, seed, noise_sigma, x_out, clean_out=None, ws=None, clip_base=0):
    if ws is None:
        ws = alloc_bytes(rd_synth_workspace_size(n_clips, N, M), x_out.device)
    _check(_lib.rd_synth(_ptr(scenes_dev), n_clips, N, M, int(seed) & 0xFFFFFFFF, float(noise_sigma),
                         clip_base, _ptr(x_out), _ptr(clean_out), _ptr(ws), ws.numel(), _stream()), 'rd_synth')


def rd_synth_host_workspace_size(n_clips, N, M):
    return int(_lib.rd_synth_host_workspace_size(n_clips, N, M))


def rd_synth_host(tab, N, M, seed, noise_sigma, x_out, clean_out=None, ws=None, clip_base=0):
    """rd_synth from a host scene table (numpy array of the rd_scene layout), copied by the library."""
    raw = np.ascontiguousarray(tab)
    n = len(raw)
    if ws is None:
        ws = alloc_bytes(rd_synth_host_workspace_size(n, N, M), x_out.device)
    _check(_lib.rd_synth_host(ctypes.c_void_p(raw.ctypes.data), n, N, M, int(seed) & 0xFFFFFFFF,
                              float(noise_sigma), clip_base, _ptr(x_out), _ptr(clean_out), _ptr(ws), ws.numel(),
                              _stream()), 'rd_synth_host')


def upload_scenes(tab, device='cuda'):
    """Scene table (numpy array of the rd_scene layout) -> device bytes."""
    raw = np.ascontiguousarray(tab).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw.copy()).to(device)


def synthesize(tab, meta, device='cuda', with_clean=True):
    """RD maps of a scene table on the GPU: (x [B, 3, N, M], clean [B, 1, N, M] or None)."""
    B, N, M = len(tab), meta['N'], meta['M']
    x = torch.empty((B, 3, N, M), dtype=torch.float32, device=device)
    clean = torch.empty((B, 1, N, M), dtype=torch.float32, device=device) if with_clean else None
    rd_synth(upload_scenes(tab, device), B, N, M, meta['seed'], meta['noise_sigma'], x, clean)
    return x, clean


# ------------------------------------------------------------------------ autograd
class STDAFunction(torch.autograd.Function):
    """z = Radar-STDA(x; w) with the library's TRAIN forward and hand-written backward.

    forward(x [B, 3, H, W], w [137469], running [1184] (updated in place), dtype, recompute)
    backward returns (dx or None, dw, None, None, None).
    """

    @staticmethod
    def forward(ctx, x, w, running, dtype=FP32, recompute=0):
        B, _, H, W = x.shape
        segs = uniform_segments(B, H, W)
        sv_b, ws_b = workspace_size(segs, dtype, TRAIN, recompute)
        saved = alloc_bytes(sv_b, x.device)
        ws = alloc_bytes(ws_b, x.device)
        z = torch.empty((B, 1, H, W), dtype=torch.float32, device=x.device)
        xc = x.detach().contiguous()
        forward(segs, xc, w.detach(), running, z, saved, ws, dtype, TRAIN, recompute)
        ctx.save_for_backward(xc, w)
        ctx.saved_buf, ctx.ws, ctx.segs, ctx.dtype, ctx.recompute = saved, ws, segs, dtype, recompute
        return z

    @staticmethod
    def backward(ctx, dz):
        x, w = ctx.saved_tensors
        dw = torch.empty_like(w)
        dx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        backward(ctx.segs, x, dz.contiguous(), w.detach(), ctx.saved_buf, dw, dx, ctx.ws, ctx.dtype,
                 ctx.recompute)
        return dx, dw, None, None, None


def stda(x, w, running, dtype=FP32, recompute=0):
    return STDAFunction.apply(x, w, running, dtype, recompute)
