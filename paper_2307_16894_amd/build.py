"""Build the HIP library libpodecm.so in-tree for gfx950.

    python -m paper_2307_16894_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, 'libpodecm.so')
SOURCES = ['rom_api.hip', 'rom_staged.hip', 'rom_fused.hip', 'rom_phased.hip', 'rom_sens.hip', 'mlp.hip', 'fe2.hip', 'offline.hip'] + [f'rom_fused_t{t}.hip' for t in range(2, 9)]
FLAGS = ['--offload-arch=gfx950', '-O3', '-std=c++17', '-fPIC',
         # packed FP32 instructions are left out of every kernel
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         # multiply-adds are fused within an expression only, the same way in
         # every kernel that inlines a shared helper (the fused and phased forms
         # agree bit for bit)
         '-ffp-contract=on',
         '-I' + os.path.join(ROOT, 'include')]


def _compile(src, verbose):
    obj = os.path.join(CSRC, src.replace('.hip', '.o'))
    cmd = ['hipcc', *FLAGS, '-c', os.path.join(CSRC, src), '-o', obj]
    if verbose:
        print(' '.join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False, jobs=None):
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + '.tmp'
    subprocess.run(['hipcc', '--offload-arch=gfx950', '-shared', '-fPIC', *objs, '-o', tmp, '-L/opt/rocm/lib',
                    '-lrocsolver', '-lrocblas', '-Wl,-rpath,/opt/rocm/lib'], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    build(verbose=True)
    sys.exit(0)
