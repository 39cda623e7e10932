"""Far pair-sum launch layouts (targets per thread, split waves, chunk counts) against the oracle.

Every layout computes the same sums in a different order, so each one is held
to the mixed-precision bar against the oracle's rows, and the multi-density
and batched launches against their single-density counterparts.
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


def soa(q):
    return np.ascontiguousarray(q.T)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


LAYOUTS = [(1, 0, 0), (2, 0, 0), (1, 0, 1), (1, 5, 1), (1, 27, 1), (2, 7, 0)]   # (tpt, chunks, split)


@pytest.fixture(scope="module")
def lattice():
    w = inputs.workload('lattice27', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, w['n_theta'], w['n_phi'])
    q = np.random.default_rng(21).standard_normal((g.N, 3))
    rng = np.random.default_rng(22)
    tg = sorted(set(rng.choice(g.N, size=10, replace=False).tolist()) | {0, g.N - 1})
    return w, g, q, tg, bie.operator_rows(g, q, tg)


@pytest.mark.parametrize("tpt,chunks,split", LAYOUTS)
def test_layout_rows_match_oracle(lattice, tpt, chunks, split):
    w, g, q, tg, ref = lattice
    say('layout', tpt, chunks, split)
    with binding.Context(w['centers'], None, w['n_theta'], w['n_phi'], precision='mixed', tpt=tpt,
                         far_chunks=chunks, far_split=split) as ctx:
        y = ctx.bie_apply(soa(q))
    assert np.abs(y[:, tg].T - ref).max() < 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("K", [2, 6])
def test_split_multi_density_matches_single(K):
    w = inputs.workload('lattice27_contacts', 0)
    c = w['centers']
    FT = inputs.random_forces(31, c.shape[0], k=K)
    kw = dict(gmres_tol=1e-10, precision='mixed', far_split=1, tpt=1, far_chunks=9)
    say('split multi', K)
    with binding.Context(c, None, w['n_theta'], w['n_phi'], **kw) as ctx:
        U, _ = ctx.mobility_apply_multi(FT)
        for r in range(K):
            Ur, _ = ctx.mobility_apply(FT[r])
            assert rel(U[r], Ur) < 1e-6


def test_split_batch_matches_single_contexts():
    inst = inputs.batched_suspensions(3)[:6]
    FT = [inputs.random_forces(40 + b, ci.shape[0]) for b, (ci, _, _) in enumerate(inst)]
    kw = dict(gmres_tol=1e-10, precision='mixed', tpt=1, far_split=1)
    say('split batch', len(inst))
    with binding.BatchContext(inst, **kw) as bc:
        Ub, st = bc.mobility_apply(FT)
    for (ci, nt, nph), F, U in zip(inst, FT, Ub):
        with binding.Context(ci, None, nt, nph, gmres_tol=1e-10, precision='mixed', tpt=1, far_chunks=0,
                             far_split=0) as ctx:
            Us, _ = ctx.mobility_apply(F)
        assert rel(U, Us) < 1e-6
