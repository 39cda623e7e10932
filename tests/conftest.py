import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def tiny_cases():
    """Dense oracle operators of the tiny 8-sphere workload for seeds 0 and 2 (cached)."""
    import numpy as np
    from oracle import bie
    from paper_2604_10089_amd import inputs
    out = []
    for seed in (0, 2):
        c = inputs.workload('tiny', seed)['centers']
        g = bie.Geometry(c, 1.0, 8, 16)
        out.append((seed, g, bie.dense_operator(g)))
    return out
