"""Full-size parity against the oracle at the shapes the bench times.

The six-density pass on the 216-sphere suspension (k_far32<1,6> with the tuned
24-chunk layout, and k_far64<6>), and the 64-sphere packing at volume fraction
0.35 (gaps down to 0.01; with and without the close-pair class), compared
element by element with the oracle's operator rows at sampled targets: the
first and last nodes, random nodes, and the nodes of the closest near pairs
(where the near rule acts)."""
import sys

import numpy as np
import pytest

from oracle import bie
from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _targets(g, k, seed, n_near=4):
    """First/last nodes, k random nodes, and on the n_near closest sphere pairs the node
    of each sphere nearest to its partner."""
    rng = np.random.default_rng(seed)
    t = set(rng.choice(g.N, size=k, replace=False).tolist())
    t.update([0, g.n - 1, g.N - g.n, g.N - 1])
    d = np.linalg.norm(g.c[:, None, :] - g.c[None, :, :], axis=2) + np.eye(g.M) * 1e9
    flat = np.argsort(d, axis=None)
    seen = 0
    for f in flat:
        i, j = divmod(int(f), g.M)
        if i > j:
            continue
        for a, b in ((i, j), (j, i)):
            nodes = g.nodes(a)
            t.add(int(nodes.start + np.argmin(np.linalg.norm(g.x[nodes] - g.c[b], axis=1))))
        seen += 1
        if seen == n_near:
            break
    return sorted(t)


def _densities(N, K, seed):
    return np.random.default_rng(seed).standard_normal((K, 3, N))


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-6), ("fp64", 1e-12)])
def test_timed_six_density_pass_rsa216_matches_oracle(prec, tol):
    """The exact launch configuration of the timed step: six densities per pass, the
    tuned far layout for (precision, K = 6, 216 spheres, 12x24), side stream on."""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, w['n_theta'], w['n_phi'])
    q = _densities(g.N, 6, 21)
    with binding.Context(c, None, w['n_theta'], w['n_phi'], lo=w['lo'], precision=prec, tune_K=6,
                         side_stream=prec == 'mixed') as ctx:
        shape = ctx.far_shape
        say('rsa216 K=6', prec, 'far layout', shape)
        if prec == 'mixed':
            assert shape == dict(tpt=1, chunks=24, split=0)
        y = ctx.bie_apply_multi(q)
    tg = _targets(g, 4, 7, n_near=3)
    for r in range(6):
        ref = bie.operator_rows(g, q[r].T, tg)
        err = np.abs(y[r][:, tg].T - ref).max() / np.abs(ref).max()
        say('  density', r, 'rel err', err)
        assert err < tol


@pytest.mark.parametrize("close", [0.0, 0.05])
def test_packing64_rows_match_oracle(close):
    """The 64-sphere packing (16x32 grid, 32,768 nodes, gaps down to 0.01), six
    densities per pass and one, both precisions, with and without the close-pair
    class (pairs below gap 0.05 on the 3x grid)."""
    w = inputs.workload('packing64', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, 16, 32, near_close_gap=close, near_close_up=3)
    q = _densities(g.N, 6, 22)
    tg = _targets(g, 4, 8, n_near=3)
    ref = {r: bie.operator_rows(g, q[r].T, tg) for r in (0, 5)}
    for prec, tol in (("mixed", 1e-6), ("fp64", 1e-12)):
        with binding.Context(c, None, 16, 32, precision=prec, near_close_gap=close, near_close_up=3,
                             tune_K=6) as ctx:
            y6 = ctx.bie_apply_multi(q)
            y1 = ctx.bie_apply(q[0])
        for r, y in ((0, y6[0]), (5, y6[5]), (0, y1)):
            err = np.abs(y[:, tg].T - ref[r]).max() / np.abs(ref[r]).max()
            say('packing64', prec, 'close', close, 'density', r, 'rel err', err)
            assert err < tol


def test_lcp_mixed_vs_fp64_rsa216():
    """The 216-sphere LCP bar: a planted LCP on the suspension's contact set (gap < 0.1),
    b formed with an FP64 product at GMRES 1e-12, solved by Bi-PQN (6x12 model) and
    Mono-PQN to KKT 1e-10 on the mixed and the FP64 path with GMRES 1e-10 inside every
    product: both within 1e-6 of the planted x*, and of each other. (With GMRES 1e-8 the
    LCP matrix itself is only known to ~1e-8 relative, and its smallest eigenvalue
    ~8e-4 turns that into x errors of ~3e-6 on either path.)"""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    with binding.Context(c, None, w['n_theta'], w['n_phi'], precision='fp64', gmres_tol=1e-12) as ctx:
        pairs, _ = ctx.find_contacts(0.1)
        xs, ws = inputs.planted_lcp(0, pairs.shape[0])
        b = ws - ctx.lcp_apply(pairs, xs)
    out = {}
    for prec in ('fp64', 'mixed'):
        with binding.Context(c, None, w['n_theta'], w['n_phi'], lo=w['lo'], precision=prec, tune_K=1,
                             gmres_tol=1e-10) as ctx:
            for solver in ('bi', 'mono'):
                x, st = ctx.lcp_solve(pairs, b, solver, tol_abs=1e-10, k_max=300)
                err = np.abs(x - xs).max() / np.abs(xs).max()
                say('rsa216 LCP', prec, solver, 'contacts', pairs.shape[0], 'products', st['mvp_hi'], st['mvp_lo'],
                    'kkt', st['kkt_abs'], 'x err', err)
                assert st['converged'] == 1
                assert err < 1e-6
                out[(prec, solver)] = x
    for solver in ('bi', 'mono'):
        d = np.abs(out[('mixed', solver)] - out[('fp64', solver)]).max() / np.abs(out[('fp64', solver)]).max()
        say('rsa216 LCP mixed vs fp64', solver, d)
        assert d < 1e-6
