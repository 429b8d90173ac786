"""CPU checks of the C ABI: the library loads, exports every function include/stda.h declares,
its parameter table equals the oracle's layout, struct layouts agree between the header, ctypes
and the scene dtype, and invalid arguments are rejected before anything touches device memory."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import net
from paper_2307_09063_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'stda.h')


@pytest.fixture(scope='module')
def S():
    from paper_2307_09063_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2307_09063_amd import stda
    return stda


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    return sorted(set(re.findall(r'^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(', src, flags=re.M)))


def test_every_declared_symbol_is_exported(S):
    names = declared_functions()
    assert 'stda_forward' in names and 'rd_synth' in names and len(names) >= 14
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(S.EXPORTS)


def test_param_table_matches_oracle(S):
    got = [(d['name'], d['shape'], d['fan_in']) for d in S.param_table()]
    assert got == [(n, tuple(s), f) for n, s, f in net.param_specs()]
    assert S.param_count() == net.param_count() == 137469
    assert S.running_count() == net.running_count()
    assert S.bn_channels() == [c for _, c in net.bn_specs()]
    offs = [d['offset'] for d in S.param_table()]
    assert offs[0] == 0 and all(b > a for a, b in zip(offs, offs[1:]))


def test_struct_layouts_against_header(tmp_path):
    prog = tmp_path / 'layout.c'
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "stda.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rd_scene),'
                    ' offsetof(rd_scene, tone), offsetof(rd_scene, intf), sizeof(rd_intf),'
                    ' sizeof(stda_segment), offsetof(stda_segment, x_off), sizeof(stda_param_desc),'
                    ' sizeof(stda_adamw_state), offsetof(stda_adamw_state, t));return 0;}\n')
    exe = tmp_path / 'layout'
    subprocess.run(['gcc', '-D__HIP_PLATFORM_AMD__', '-I', os.path.join(ROOT, 'include'), '-I',
                    '/opt/rocm/include', str(prog), '-o', str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    d = inputs.SCENE_DTYPE
    from paper_2307_09063_amd import stda
    assert vals == [d.itemsize, d.fields['tone'][1], d.fields['intf'][1], inputs.INTF_DTYPE.itemsize,
                    ctypes.sizeof(stda.Segment), stda.Segment.x_off.offset, ctypes.sizeof(stda.ParamDesc),
                    stda.AdamW.STATE_BYTES, stda.AdamW.T_OFFSET]


def _segs(S, *t):
    arr = (S.Segment * len(t))(*[S.Segment(*x) for x in t])
    return ctypes.cast(arr, ctypes.c_void_p), len(t)


def test_validation_before_launch(S):
    lib = S._lib
    fake = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    sv, wb = ctypes.c_size_t(), ctypes.c_size_t()
    for shape, code in (((1, 10, 16, 0, 0), -2), ((1, 16, 6, 0, 0), -2), ((1, 4, 16, 0, 0), -2),
                        ((0, 16, 16, 0, 0), -1), ((1, 16, 8192, 0, 0), -2)):
        p, n = _segs(S, shape)
        assert lib.stda_workspace_size(p, n, 0, 1, 0, ctypes.byref(sv), ctypes.byref(wb)) == code
        assert lib.stda_forward(p, n, fake, fake, fake, fake, fake, 1 << 40, fake, 1 << 40, 0, 1, 0, None) == code
    p, n = _segs(S, (2, 16, 16, 0, 0))
    assert lib.stda_workspace_size(p, n, 7, 1, 0, ctypes.byref(sv), ctypes.byref(wb)) == -1   # dtype
    assert lib.stda_workspace_size(p, n, 0, 5, 0, ctypes.byref(sv), ctypes.byref(wb)) == -1   # mode
    assert lib.stda_workspace_size(p, n, 0, 1, 0, ctypes.byref(sv), ctypes.byref(wb)) == 0
    assert sv.value > 0 and wb.value > 0
    # too-small workspace / saved buffer
    assert lib.stda_forward(p, n, fake, fake, fake, fake, fake, sv.value, fake, wb.value - 1, 0, 1, 0, None) == -3
    assert lib.stda_forward(p, n, fake, fake, fake, fake, fake, sv.value - 1, fake, wb.value, 0, 1, 0, None) == -3
    assert lib.stda_backward(p, n, fake, fake, fake, fake, sv.value, fake, None, fake, wb.value - 1, 0, 0, None) == -3
    # null pointers
    assert lib.stda_forward(p, n, None, fake, fake, fake, fake, sv.value, fake, wb.value, 0, 1, 0, None) == -1
    assert lib.stda_sgd_step(None, fake, 10, ctypes.c_float(0.1), ctypes.c_float(0.0), None, None) == -1
    # no-allocation EVAL forward: shape, dtype and pointer checks, and batches whose EVAL workspace
    # exceeds the static scratch array, are refused before any device call
    for shape, code in (((1, 10, 16, 0, 0), -2), ((0, 16, 16, 0, 0), -1)):
        q, m = _segs(S, shape)
        assert lib.stda_forward_noalloc(q, m, fake, fake, fake, fake, 0, None) == code
    assert lib.stda_forward_noalloc(p, n, fake, fake, fake, fake, 3, None) == -1
    assert lib.stda_forward_noalloc(p, n, None, fake, fake, fake, 0, None) == -1
    for dt, clips in ((0, 2), (1, 3)):
        q, m = _segs(S, (clips, 256, 128, 0, 0))
        assert lib.stda_workspace_size(q, m, dt, 0, 0, ctypes.byref(sv), ctypes.byref(wb)) == 0
        assert wb.value > S.NOALLOC_WS_MAX
        assert lib.stda_forward_noalloc(q, m, fake, fake, fake, fake, dt, None) == -3
    # rd_synth: N and M powers of two in [8, 1024]
    big = 1 << 40
    assert lib.rd_synth(fake, 1, 48, 64, 1, ctypes.c_float(1.0), 0, fake, None, fake, big, None) == -2
    assert lib.rd_synth(fake, 1, 64, 2048, 1, ctypes.c_float(1.0), 0, fake, None, fake, big, None) == -2
    assert lib.rd_synth(fake, 1, 64, 64, 1, ctypes.c_float(1.0), 0, fake, None, fake, 16, None) == -3
    # rd_synth_host: the same checks, the host table's room counted in its workspace size
    lib.rd_synth_workspace_size.restype = ctypes.c_size_t
    lib.rd_synth_host_workspace_size.restype = ctypes.c_size_t
    from paper_2307_09063_amd import inputs
    assert (lib.rd_synth_host_workspace_size(4, 64, 64)
            >= lib.rd_synth_workspace_size(4, 64, 64) + 4 * inputs.SCENE_DTYPE.itemsize)
    assert lib.rd_synth_host(None, 1, 64, 64, 1, ctypes.c_float(1.0), 0, fake, None, fake, big, None) == -1
    assert lib.rd_synth_host(fake, 1, 48, 64, 1, ctypes.c_float(1.0), 0, fake, None, fake, big, None) == -2
    need = lib.rd_synth_host_workspace_size(1, 64, 64)
    assert lib.rd_synth_host(fake, 1, 64, 64, 1, ctypes.c_float(1.0), 0, fake, None, fake, need - 1, None) == -3
    assert lib.stda_status_string(-2).decode().startswith('unsupported shape')
    # CA-CFAR / EVM argument checks
    d = ctypes.c_double
    assert lib.stda_cfar(None, 1, 64, 64, 2, 2, 4, 4, d(1e-3), fake, None, None, None) == -1
    assert lib.stda_cfar(fake, 1, 64, 64, 2, 2, 0, 0, d(1e-3), fake, None, None, None) == -1  # no training
    assert lib.stda_cfar(fake, 1, 64, 64, 2, 2, 4, 4, d(1.0), fake, None, None, None) == -1   # pfa
    assert lib.stda_cfar(fake, 1, 64, 64, 2, 2, 7, 4, d(1e-3), fake, None, None, None) == -2  # halo > 8
    assert lib.stda_cfar(fake, 1, 12, 64, 2, 2, 4, 4, d(1e-3), fake, None, None, None) == -2  # window > map
    assert lib.stda_evm(fake, fake, None, 1, 8, 8, fake, None) == -1


def test_workspace_grows_with_batch(S):
    a = S.workspace_size(S.uniform_segments(2, 64, 64))
    b = S.workspace_size(S.uniform_segments(4, 64, 64))
    assert b[0] > a[0] and b[1] > a[1]
    ev = S.workspace_size(S.uniform_segments(2, 64, 64), S.FP32, S.EVAL)
    assert ev[0] == 0
    bf = S.workspace_size(S.uniform_segments(2, 64, 64), S.BF16, S.TRAIN)
    assert bf[0] < a[0]


@pytest.mark.parametrize('res_k,head,pw', [(3, 'identity', 'dense'), (4, 'sigmoid', 'dense'), (3, 'sigmoid', 'dense'),
                                          (4, 'identity', 'depthwise'), (3, 'sigmoid', 'depthwise')])
def test_architecture_readings_layout(S, res_k, head, pw):
    """The residual and 1x1-branch readings change the parameter table exactly as in the oracle;
    the sigmoid output adds one FP32 map per clip to the TRAIN saved buffer and nothing else."""
    segs = S.uniform_segments(3, 32, 24)
    sv0, ws0 = S.workspace_size(segs, S.FP32, S.TRAIN)
    ev0 = S.workspace_size(segs, S.FP32, S.EVAL)
    try:
        S.set_arch(res_k, head, pw)
        net.set_arch(res_k, head, pw)
        assert S.get_arch() == {'res_k': res_k, 'head': head, 'pw': pw}
        got = [(d['name'], d['shape'], d['fan_in']) for d in S.param_table()]
        assert got == [(n, tuple(s), f) for n, s, f in net.param_specs()]
        fewer = (res_k == 3) * 17920 + (pw == 'depthwise') * 6256
        assert S.param_count() == net.param_count() == 137469 - fewer
        sv, ws = S.workspace_size(segs, S.FP32, S.TRAIN)
        ev = S.workspace_size(segs, S.FP32, S.EVAL)
        extra = -(-(3 * 32 * 24 * 4) // 256) * 256 if head == 'sigmoid' else 0
        assert sv == sv0 + extra
        assert ev[0] == ev0[0] == 0
        # the working-weight copy in ws shrinks with the parameter count
        assert ws <= ws0 and ev[1] <= ev0[1]
    finally:
        S.set_arch()
        net.set_arch()
    assert S.get_arch() == {'res_k': 4, 'head': 'identity', 'pw': 'dense'}
    assert S.param_count() == 137469


def test_set_arch_rejects_unknown_bits(S):
    assert S._lib.stda_set_arch(8) == -1      # STDA_E_INVALID
    assert S._lib.stda_set_arch(-1) == -1
    assert S._lib.stda_get_arch() == 0
    with pytest.raises(S.StdaError):
        S.set_arch(5)


def test_folded_eval_validation(S):
    """The folded EVAL entry points: size query, refusal of the readings the fold does not cover
    and argument checks before anything touches the device."""
    assert S.eval_fold_size(0) > 4 * S.param_count() and S.eval_fold_size(1) > 4 * S.param_count()
    for kw in ({'res_k': 3}, {'pw': 'depthwise'}):
        S.set_arch(**kw)
        try:
            with pytest.raises(S.StdaError):
                S.eval_fold_size(0)
        finally:
            S.set_arch()
    lib, fake = S._lib, ctypes.c_void_p(16)
    need = S.eval_fold_size(0)
    assert lib.stda_eval_fold(fake, fake, fake, need - 1, 0, None) == -3
    assert lib.stda_eval_fold(None, fake, fake, need, 0, None) == -1
    assert lib.stda_eval_fold(fake, fake, fake, need, 5, None) == -1
    p, n = _segs(S, (1, 16, 16, 0, 0))
    sv, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.stda_workspace_size(p, n, 0, 0, 0, ctypes.byref(sv), ctypes.byref(wb)) == 0
    assert lib.stda_forward_folded(p, n, fake, fake, need, fake, fake, wb.value - 1, 0, None) == -3
    assert lib.stda_forward_folded(p, n, fake, fake, need - 1, fake, fake, wb.value, 0, None) == -3
    assert lib.stda_forward_folded(p, n, None, fake, need, fake, fake, wb.value, 0, None) == -1
    q, m = _segs(S, (1, 10, 16, 0, 0))
    assert lib.stda_forward_folded(q, m, fake, fake, need, fake, fake, wb.value, 0, None) == -2
