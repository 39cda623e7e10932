"""Graph-replayed GMRES iterations (use_graphs = 1) against the eager launches and the oracle.

Every solve replays each captured iteration once, so several solves in a row,
with eager work and synchronisations between them, replay every graph several
times; each replay is checked.
"""
import sys

import numpy as np
import pytest

from oracle import bie
from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    c = inputs.workload('tiny', 0)['centers']
    g = bie.Geometry(c, 1.0, 8, 16)
    return c, g, bie.dense_operator(g)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager_tiny(tiny, prec):
    c, g, A = tiny
    say('graph tiny', prec)
    kw = dict(gmres_tol=1e-12, precision=prec, refine=0)
    with binding.Context(c, None, 8, 16, graphs=True, **kw) as cg, \
            binding.Context(c, None, 8, 16, graphs=False, **kw) as ce:
        for rep in range(4):
            FT = inputs.random_forces(20 + rep, g.M)
            Ug, sg = cg.mobility_apply(FT)
            Ue, se = ce.mobility_apply(FT)      # eager work between replays
            say('  rep', rep, 'iters', sg['gmres_iters'], se['gmres_iters'], 'graph launches',
                sg['graph_launches'])
            assert sg['graph_launches'] == sg['gmres_iters'] > 0
            assert se['graph_launches'] == 0
            assert sg['gmres_iters'] == se['gmres_iters']
            assert rel(Ug, Ue) < 1e-12
            if prec == 'fp64':
                assert rel(Ug, bie.mobility_apply(g, FT, dense=A)) < 1e-10


def test_graph_rebuilt_after_state_change():
    w = inputs.workload('lattice27_contacts', 1)
    c = w['centers']
    say('graph state change', c.shape)
    kw = dict(gmres_tol=1e-10, precision='mixed', refine=0)
    FT = inputs.random_forces(5, c.shape[0])
    with binding.Context(c, None, 8, 16, graphs=True, **kw) as cg, \
            binding.Context(c, None, 8, 16, graphs=False, **kw) as ce:
        U0, _ = cg.mobility_apply(FT)
        c2 = c * 1.01                               # moves every sphere: new near list
        cg.set_state(c2)
        ce.set_state(c2)
        for rep in range(2):
            Ug, sg = cg.mobility_apply(FT)
            Ue, se = ce.mobility_apply(FT)
            assert sg['graph_launches'] == sg['gmres_iters'] > 0
            assert rel(Ug, Ue) < 1e-12
        assert rel(Ug, U0) > 1e-6                   # the new configuration was used


def test_graph_lcp_solve_matches_eager(tiny):
    c, g, A = tiny
    pairs = np.array([[i, j] for i in range(g.M) for j in range(i + 1, g.M)
                      if np.linalg.norm(c[i] - c[j]) < 2.3], dtype=np.int32)
    if pairs.shape[0] == 0:
        pytest.skip('no close pairs in this configuration')
    b = -0.1 * np.ones(pairs.shape[0])
    kw = dict(gmres_tol=1e-12, precision='fp64')
    with binding.Context(c, None, 8, 16, lo=(4, 8), graphs=True, **kw) as cg, \
            binding.Context(c, None, 8, 16, lo=(4, 8), graphs=False, **kw) as ce:
        for solver in ('mono', 'bi'):
            xg, sg = cg.lcp_solve(pairs, b, solver=solver, tol_abs=1e-10, tol_rel=1e-10)
            xe, se = ce.lcp_solve(pairs, b, solver=solver, tol_abs=1e-10, tol_rel=1e-10)
            say('  lcp', solver, sg['mvp_hi'], se['mvp_hi'])
            assert sg['mvp_hi'] == se['mvp_hi'] and sg['mvp_lo'] == se['mvp_lo']
            assert np.abs(xg - xe).max() <= 1e-10 * max(1.0, np.abs(xe).max())
