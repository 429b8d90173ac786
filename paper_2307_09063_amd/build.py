"""Build libstda.so (the HIP library behind include/stda.h) in-tree for gfx950.

    python -m paper_2307_09063_amd.build          # or build() from Python

Every HIP source is compiled with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libstda.so')
SOURCES = ['net.hip', 'rd.hip', 'detect.hip', 'optim.hip']
ARCH = os.environ.get('STDA_ARCH', 'gfx950')

HIPCC_FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}',
               '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
               '-I', os.path.join(ROOT, 'include')]


def build(verbose=False):
    """Compile every HIP source to an object and link libstda.so; returns the library path."""
    hipcc = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
    objdir = os.path.join(HERE, '_build')
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace('.hip', '.o'))
        cmd = [hipcc, *HIPCC_FLAGS, '-c', os.path.join(CSRC, src), '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors='replace')
        lines = [l for l in text.splitlines() if 'packed-fp32-ops' not in l and l.strip()]
        if p.returncode != 0:
            sys.stderr.write(text)
            raise RuntimeError(f'hipcc failed on {src}')
        if verbose and lines:
            print('\n'.join(lines))
    tmp = LIB + '.tmp'
    cmd = [hipcc, '-shared', '-fPIC', f'--offload-arch={ARCH}', *objs, '-o', tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose=True))
