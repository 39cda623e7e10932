"""Build the HIP library libbipqn.so in-tree for gfx950 (hipcc), and the oracle's C parts (none).

Usage: python -m paper_2604_10089_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libbipqn.so')
SOURCES = ['host_math.cpp', 'kernels.hip', 'context.hip', 'precond.hip', 'lcp.hip', 'capi.hip']
ARCH = os.environ.get('BIPQN_ARCH', 'gfx950')


def hipcc():
    for c in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if c and os.path.exists(c):
            return c
    raise RuntimeError('hipcc not found')


def build(verbose=False, jobs=None):
    cc = hipcc()
    flags = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}',
             '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
             '-I', os.path.join(HERE, '..', 'include'), '-Wno-unused-command-line-argument']
    objdir = os.path.join(HERE, '_build')
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + '.o')
        objs.append(obj)
        cmd = [cc] + flags + ['-c', os.path.join(CSRC, src), '-o', obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors='replace')
        text = '\n'.join(l for l in text.splitlines() if 'packed-fp32-ops' not in l and 'not a recognized feature' not in l)
        if p.returncode != 0:
            raise RuntimeError(f'hipcc failed on {src}:\n{text}')
        if verbose and text.strip():
            print(text)
    tmp = LIB + '.tmp'
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(cc))), 'lib')
    cmd = [cc, '-shared', '-fPIC', f'--offload-arch={ARCH}', '-o', tmp] + objs + [
        f'-L{rocm_lib}', f'-Wl,-rpath,{rocm_lib}', '-lrocprofiler-sdk-roctx']
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stdout.decode(errors='replace'))
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose='-v' in sys.argv))
