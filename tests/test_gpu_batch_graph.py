"""Graph-captured GMRES of the batched suspensions (use_graphs on a batch context).

Every Arnoldi step of all suspensions is one captured graph (operator, CGS2, the
Givens step and the normalisation on the device; a suspension that has converged
turns its segments of the later launches into no-ops). The graph path runs the same
kernels in the same order as the eager lockstep loop, so results agree to rounding
of the Givens arithmetic (host vs device), replay after replay, with eager work in
between."""
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


def _small_batch(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        c = inputs.workload('tiny', 10 + b)['centers']
        nt = int(rng.choice([6, 8]))
        out.append((c, nt, 2 * nt))
    return out


@pytest.mark.parametrize("prec,side", [("fp64", False), ("mixed", False), ("mixed", True)])
def test_batch_graph_matches_eager_over_replays(prec, side):
    inst = _small_batch(3, 5)
    kw = dict(gmres_tol=1e-12, precision=prec, side_stream=side)
    with binding.BatchContext(inst, graphs=True, **kw) as bg, binding.BatchContext(inst, **kw) as be, \
            binding.Context(inst[0][0], None, 8, 16, gmres_tol=1e-10) as other:
        for rep in range(3):
            FTs = [inputs.random_forces(60 + 7 * rep + b, c.shape[0]) for b, (c, _, _) in enumerate(inst)]
            Ug, sg = bg.mobility_apply(FTs)
            Ue, se = be.mobility_apply(FTs)
            other.mobility_apply(FTs[0])        # eager work between the replays
            say('batch graph', prec, side, 'rep', rep, 'graph launches', sg['graph_launches'], 'iters',
                sg['gmres_iters'], se['gmres_iters'])
            assert sg['converged'] == 1 and sg['graph_launches'] > 0 and se['graph_launches'] == 0
            assert abs(sg['gmres_iters'] - se['gmres_iters']) <= len(inst)
            for b in range(len(inst)):
                assert rel(Ug[b], Ue[b]) < 1e-10, (rep, b)
    g = bie.Geometry(inst[1][0], 1.0, inst[1][1], inst[1][2])
    Uo = bie.mobility_apply(g, FTs[1], dense=bie.dense_operator(g))
    assert rel(Ug[1], Uo) < (1e-10 if prec == 'fp64' else 1e-6)


def test_batch_graph_restarts_and_zero_forces():
    """Short restart length (cycles fill and continue in the eager loop) and a suspension
    with zero forces (inactive from the start)."""
    inst = _small_batch(4, 4)
    FTs = [inputs.random_forces(80 + b, c.shape[0]) for b, (c, _, _) in enumerate(inst)]
    FTs[2] = np.zeros_like(FTs[2])
    kw = dict(gmres_tol=1e-11, precision='fp64', restart=8)
    with binding.BatchContext(inst, graphs=True, **kw) as bg, binding.BatchContext(inst, **kw) as be:
        Ug, sg = bg.mobility_apply(FTs)
        Ue, se = be.mobility_apply(FTs)
    say('batch graph restarts', sg['gmres_iters'], se['gmres_iters'], sg['graph_launches'])
    assert sg['converged'] == 1
    assert np.all(Ug[2] == 0.0)
    for b in (0, 1, 3):
        assert rel(Ug[b], Ue[b]) < 1e-9


def test_batch_graph_full_workload():
    """The 32-suspension workload (8-27 spheres, 8x16..16x32 grids), mixed precision with
    the side stream: graph path against the eager batch and per-instance contexts."""
    inst = inputs.batched_suspensions(0)
    FTs = [inputs.random_forces(40 + b, c.shape[0]) for b, (c, _, _) in enumerate(inst)]
    kw = dict(gmres_tol=1e-8, precision='mixed', side_stream=True)
    with binding.BatchContext(inst, graphs=True, **kw) as bg, binding.BatchContext(inst, **kw) as be:
        Ug, sg = bg.mobility_apply(FTs)
        Ug2, _ = bg.mobility_apply(FTs)
        Ue, se = be.mobility_apply(FTs)
    say('batch32 graph', sg, se['gmres_iters'])
    assert sg['converged'] == 1
    for b in range(len(inst)):
        assert np.array_equal(Ug[b], Ug2[b])
        assert rel(Ug[b], Ue[b]) < 1e-8
    for b in (0, 31):
        c, nt, nph = inst[b]
        with binding.Context(c, None, nt, nph, gmres_tol=1e-8, precision='mixed') as ctx:
            Us, _ = ctx.mobility_apply(FTs[b])
        assert rel(Ug[b], Us) < 1e-6
