"""Host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host-side FP64 set-up of the library (Gauss-Legendre rules, sphere grids,
harmonic tables, the singular self block) is compiled with the sanitizers on the
host pass only and run on four grids; it must finish without a report and
produce the self block the library's pqn_host_self_block returns."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2604_10089_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2604_10089_amd', 'csrc')

DRIVER = r'''
#include "common.hpp"
#include <cstdio>
int main() {
  const int grids[][2] = {{4, 8}, {6, 12}, {8, 16}, {12, 24}};
  for (auto& g : grids) {
    bipqn::SphereTables t;
    bipqn::build_sphere_tables(g[0], g[1], 1.0, 2, t);
    double s = 0.0, a = 0.0;
    for (double v : t.S) { s += v; a += v * v; }
    std::printf("%d %d %zu %.17g %.17g\n", g[0], g[1], t.S.size(), s, a);
  }
  return 0;
}
'''


def test_host_setup_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(hipcc):
        pytest.skip('no hipcc')
    drv = tmp_path / 'drv.cpp'
    drv.write_text(DRIVER)
    exe = tmp_path / 'drv'
    cmd = [hipcc, '-std=c++17', '-g', '-O1', '-I', os.path.join(ROOT, 'include'), '-I', CSRC,
           '-Xarch_host', '-fsanitize=address', '-Xarch_host', '-fsanitize=undefined',
           '-Xarch_host', '-fno-sanitize-recover=all', os.path.join(CSRC, 'host_math.cpp'), str(drv), '-o', str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS='detect_leaks=1:abort_on_error=0', UBSAN_OPTIONS='print_stacktrace=1')
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert 'runtime error' not in r.stderr and 'AddressSanitizer' not in r.stderr
    for line in r.stdout.splitlines():
        nt, nph, size, s, a = line.split()
        nt, nph = int(nt), int(nph)
        _, _, S = binding.pqn_host_self_block(nt, nph, 1.0)
        assert S.size == int(size)
        assert abs(S.sum() - float(s)) <= 1e-12 * np.abs(S).sum()
        assert abs((S * S).sum() - float(a)) <= 1e-12 * (S * S).sum()
