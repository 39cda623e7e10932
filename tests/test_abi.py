"""CPU checks of the C ABI library: it loads, exports every declared symbol,
rejects bad arguments without a device, and its host-side FP64 set-up (grid and
singular self block) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from paper_2604_10089_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), 'include', 'bipqn.h')


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r'\b(pqn_[a-z_]+)\s*\(', text)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = _declared()
    assert 'pqn_mobility_apply' in names and 'pqn_lcp_solve' in names and 'pqn_step' in names
    for name in names:
        assert hasattr(L, name), name


def test_invalid_create_rejected_without_device():
    L = binding.lib()
    d = binding.ConfigDesc()
    d.n_particles = 0
    h = binding.C.c_void_p()
    c = np.zeros(3)
    st = L.pqn_create(binding.C.byref(d), c.ctypes.data_as(binding._D), None, binding.C.byref(h))
    assert st == -1 and h.value is None
    assert b'n_particles' in L.pqn_last_error()
    d.n_particles = 1
    d.n_theta, d.n_phi = 8, 8
    st = L.pqn_create(binding.C.byref(d), c.ctypes.data_as(binding._D), None, binding.C.byref(h))
    assert st == -1
    assert L.pqn_destroy(None) == 0


@pytest.mark.parametrize("nt", [4, 6, 8])
def test_host_self_block_matches_oracle(nt):
    from oracle import bie, grid
    off, w, S = binding.pqn_host_self_block(nt, 2 * nt, 1.3)
    o2, _, w2 = grid.sphere_grid(nt, 2 * nt, 1.3)
    assert np.abs(off - o2).max() < 1e-14 and np.abs(w - w2).max() < 1e-14
    So = bie.self_block(nt, 2 * nt, 1.3).reshape(3 * nt * 2 * nt, -1)
    assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()


def test_host_self_block_rejects_bad_grid():
    with pytest.raises(binding.PqnError):
        binding.pqn_host_self_block(1, 2, 1.0)
    with pytest.raises(binding.PqnError):
        binding.pqn_host_self_block(6, 12, -1.0)
