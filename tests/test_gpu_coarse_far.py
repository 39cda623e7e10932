"""The coarse-far low fidelity (far_coarse_lo): the same grid as the high fidelity, with
far sphere pairs summed from a coarse source grid carrying the density truncated to its
degree. Parity of the device operator with the oracle's (Geometry(far_coarse=...)), on
one and six densities, both precisions, side stream on and off; Bi-PQN with it as the
low-fidelity model against the oracle's Bi-PQN and brute force."""
import sys

import numpy as np
import pytest

from oracle import bie, dynamics, lcp
from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def tiny_cf():
    c = inputs.workload('tiny', 0)['centers']
    g = bie.Geometry(c, 1.0, 8, 16, far_coarse=(4, 8))
    return c, g, bie.dense_operator(g)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_coarse_far_operator_matches_oracle(tiny_cf, prec, tol):
    c, g, A = tiny_cf
    q = np.random.default_rng(3).standard_normal((6, g.N, 3))
    with binding.Context(c, None, 8, 16, lo=(8, 16), far_coarse_lo=4, precision=prec) as ctx:
        y1 = ctx.bie_apply(np.ascontiguousarray(q[0].T), fidelity=binding.PQN_LOFI)
        y6 = ctx.bie_apply_multi(np.ascontiguousarray(q.transpose(0, 2, 1)), fidelity=binding.PQN_LOFI)
        yh = ctx.bie_apply(np.ascontiguousarray(q[0].T))
    for r in range(6):
        ref = (A @ q[r].ravel()).reshape(-1, 3).T
        assert rel(y6[r], ref) < tol, r
    assert rel(y1, (A @ q[0].ravel()).reshape(-1, 3).T) < tol
    # the high fidelity keeps the node rule
    gh = bie.Geometry(c, 1.0, 8, 16)
    assert rel(yh, bie.operator_apply(gh, q[0]).T) < tol


def test_coarse_far_side_stream_bit_identical(tiny_cf):
    c, g, _ = tiny_cf
    FT = inputs.random_forces(5, g.M, k=3)
    out = {}
    for side in (False, True):
        with binding.Context(c, None, 8, 16, lo=(8, 16), far_coarse_lo=4, precision='mixed',
                             side_stream=side) as ctx:
            out[side] = ctx.mobility_apply_multi(FT, fidelity=binding.PQN_LOFI)[0]
    assert np.array_equal(out[False], out[True])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_coarse_far_rows_rsa216(prec, tol):
    """216 spheres, 12x24 grid, far sources on 6x12 (degree 5): sampled operator rows."""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, 12, 24, far_coarse=(6, 12))
    q = np.random.default_rng(9).standard_normal((g.N, 3))
    with binding.Context(c, None, 12, 24, lo=(12, 24), far_coarse_lo=6, precision=prec) as ctx:
        y = ctx.bie_apply(np.ascontiguousarray(q.T), fidelity=binding.PQN_LOFI)
    rng = np.random.default_rng(2)
    tg = sorted(set(rng.choice(g.N, size=6, replace=False).tolist()) | {0, g.N - 1})
    ref = bie.operator_rows(g, q, tg)
    err = np.abs(y[:, tg].T - ref).max() / np.abs(ref).max()
    say('coarse-far rows rsa216', prec, err)
    assert err < tol


def test_bi_pqn_with_coarse_far_model_matches_oracle(tiny_cf):
    c, gcf, Acf = tiny_cf
    g = bie.Geometry(c, 1.0, 8, 16)
    A = bie.dense_operator(g)
    pairs, _ = dynamics.find_contacts(c, 1.0, 0.1)
    n = pairs.shape[0]
    Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(g, F, dense=A), c, pairs)
    Alo = lcp.lcp_operator(lambda F: bie.mobility_apply(gcf, F, dense=Acf), c, pairs)
    Ad = np.column_stack([Aop(np.eye(n)[k]) for k in range(n)])
    xs, ws = inputs.planted_lcp(0, n)
    b = ws - Ad @ xs
    xo, _, so = lcp.bi_pqn(Aop, Alo, b)
    with binding.Context(c, None, 8, 16, lo=(8, 16), far_coarse_lo=4, gmres_tol=1e-13) as ctx:
        x, st = ctx.lcp_solve(pairs, b, 'bi')
        _, sm = ctx.lcp_solve(pairs, b, 'mono')
    say('bi coarse-far', st['mvp_hi'], st['mvp_lo'], 'oracle', so['mvp_hi'], so['mvp_lo'], 'mono', sm['mvp_hi'])
    assert st['converged'] == 1
    assert np.abs(x - xs).max() < 1e-7 * np.abs(xs).max()
    assert abs(st['mvp_hi'] - so['mvp_hi']) <= 1
    assert st['mvp_hi'] < sm['mvp_hi']
