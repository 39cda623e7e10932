"""The allocation-free contact search (pqn_find_contacts_noalloc) against pqn_find_contacts.

The variant stages the contact kernel's counter and list in a fixed device array of
the library instead of context buffers; its results must be those of the allocating
entry point, bit for bit, call after call (the array keeps the last call's contents),
and a configuration with more contacts than the array holds is rejected."""
import ctypes as C

import numpy as np
import pytest

from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu

MAX_CONTACTS = 32768


def _noalloc(ctx, delta, cap):
    L = binding.lib()
    n = C.c_int32(-1)
    pairs = np.full((max(cap, 1), 2), -7, dtype=np.int32)
    gaps = np.full(max(cap, 1), np.nan)
    st = L.pqn_find_contacts_noalloc(ctx.h, delta, cap, C.byref(n), pairs.ctypes.data_as(binding._I),
                                     gaps.ctypes.data_as(binding._D))
    return st, n.value, pairs[:max(0, min(n.value, cap))], gaps[:max(0, min(n.value, cap))]


def _check_same(ctx, delta):
    ref_pairs, ref_gaps = ctx.find_contacts(delta)
    st, n, pairs, gaps = _noalloc(ctx, delta, ref_pairs.shape[0] + 5)
    assert st == 0, binding.lib().pqn_last_error()
    assert n == ref_pairs.shape[0]
    assert np.array_equal(pairs, ref_pairs)
    assert np.array_equal(gaps, ref_gaps)
    return n


def test_noalloc_contacts_match_allocating_entry_point():
    big = inputs.workload('rsa216', 0)['centers']
    small = inputs.workload('tiny', 0)['centers']
    with binding.Context(big, None, 4, 8) as cb, binding.Context(small, None, 4, 8) as cs:
        n1 = _check_same(cb, 0.6)          # first call: 216 spheres
        n2 = _check_same(cs, 0.1)          # second call, smaller input: the array's old contents must not leak
        assert n1 > n2 > 0
        n3 = _check_same(cb, 0.05)         # fewer contacts than the previous call on the same context
        assert 0 < n3 < n1
        # cap too small: the count is reported, nothing beyond cap is written
        st, n, _, _ = _noalloc(cs, 0.1, n2 - 1)
        assert st == -1
        assert n == n2
        st, n, _, _ = _noalloc(cs, 0.1, 0)
        assert st == -1 and n == n2
        st, n, _, _ = _noalloc(cs, -10.0, 0)   # no pair within a negative gap
        assert st == 0 and n == 0


def test_noalloc_contacts_reject_more_than_the_staging_holds():
    """300 spheres with every pair a contact (44,850 > 32,768): rejected with a clear error,
    the count reported; the next call on a small input is correct again."""
    rng = np.random.default_rng(0)
    c = np.array([[3.0 * i, 0.0, 0.0] for i in range(300)]) + rng.uniform(0, 0.1, (300, 3))
    with binding.Context(c, None, 4, 8, near_gap=0.5) as ctx:
        st, n, _, _ = _noalloc(ctx, 1e4, 10)
        assert st == -1 and n == 300 * 299 // 2
        assert b'32768' in binding.lib().pqn_last_error()
    small = inputs.workload('tiny', 0)['centers']
    with binding.Context(small, None, 4, 8) as cs:
        _check_same(cs, 0.1)
