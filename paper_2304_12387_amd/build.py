"""Build libhdivsp.so (HIP for gfx950) in-tree.

    python -m paper_2304_12387_amd.build [--jobs N]

Every source is compiled with hipcc for gfx950 with packed FP32 instructions
disabled, then linked into paper_2304_12387_amd/libhdivsp.so.
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(os.path.dirname(HERE), '_build')
LIB = os.path.join(HERE, 'libhdivsp.so')

SOURCES = ['tables.cpp', 'amg_host.cpp', 'unstructured.cpp', 'amg_gpu.hip', 'setup.hip', 'apply.hip', 'precond.hip', 'minres.hip', 'gmres.hip',
           'learned.hip', 'raddiff.hip',
           'capi.hip']
ARCH = 'gfx950'
FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}', '-munsafe-fp-atomics',
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-Wno-unused-command-line-argument']


def hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found')


def compile_one(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + '.o')
    cmd = [hipcc()] + FLAGS + ['-c', os.path.join(CSRC, src), '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [r for r in results if r[2] != 0]
    for src, _, rc, out in results:
        if rc != 0 or verbose:
            # hipcc's host pass warns about the device-only target feature; keep errors visible
            lines = [l for l in out.splitlines() if 'packed-fp32-ops' not in l or 'error' in l]
            if lines:
                print(f'--- {src} (rc={rc})', file=sys.stderr)
                print('\n'.join(lines), file=sys.stderr)
    if failed:
        raise RuntimeError('compilation failed: ' + ', '.join(r[0] for r in failed))
    tmp = LIB + '.tmp'
    cmd = [hipcc(), '-shared', '-fPIC', f'--offload-arch={ARCH}', '-o', tmp] + [r[1] for r in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    ap = argparse.ArgumentParser()
    ap.add_argument('--jobs', type=int, default=None)
    ap.add_argument('-v', '--verbose', action='store_true')
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))
