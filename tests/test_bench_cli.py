"""Host-side contract of bench.py: one GPU only, the traffic figure keyed to the far-kernel
source, and the roofline helpers (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert 'one GPU' in r.stderr or 'one MI355X' in r.stderr


def test_traffic_is_null_for_another_layout_or_source():
    t = bench.FAR_TRAFFIC
    assert bench.far_traffic_bytes(dict(tpt=2, chunks=8, split=0)) is None
    got = bench.far_traffic_bytes(t['layout'])
    if bench.far_source_sha1() == t['source_sha1']:
        assert got == int(1024 * (t['fetch_kib'] * t['fetch_scale'] + t['write_kib'] * t['write_scale']))
    else:
        assert got is None


def test_flop_convention():
    # 18 flop of geometry plus 12 per density (FMA = 2), one rsqrt counted once
    assert bench.flop_per_pair(1) == 30 and bench.flop_per_pair(6) == 90
