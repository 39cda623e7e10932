"""GPU parity of the right-preconditioned GMRES (config precond): the oracle's solutions and
iteration counts, the unpreconditioned solves' velocities, fewer iterations, set-up after
every configuration change."""
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
    return np.ascontiguousarray(np.asarray(q).reshape(-1, 3).T)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_preconditioned_bie_solve_matches_oracle_and_its_iteration_count(tiny_cases):
    """FP64: the density of the oracle's dense solve, in the iterations of the oracle's
    right-preconditioned GMRES (the same preconditioner from the assembled matrix)."""
    for seed, g, A in tiny_cases:
        rhs = -bie.completion(g, inputs.random_forces(40 + seed, g.M))
        q = np.linalg.solve(A, rhs.ravel())
        P = bie.near_patch_preconditioner(g, A)
        _, its_o, _ = bie.gmres(lambda v: A @ v.ravel(), rhs, tol=1e-10, right=P)
        _, its_plain, _ = bie.gmres(lambda v: A @ v.ravel(), rhs, tol=1e-10)
        c = g.c
        with binding.Context(c, None, 8, 16, gmres_tol=1e-10, precond='eager') as ctx:
            qd, st = ctx.bie_solve(soa(rhs))
        say('precond tiny seed', seed, 'gpu its', st['gmres_iters'], 'oracle', its_o, 'plain', its_plain,
            'setup ms', round(st['t_precond_ms'], 2), 'fallback', st['precond_fallback'])
        assert st['converged'] == 1 and st['precond_fallback'] == 0
        assert abs(st['gmres_iters'] - its_o) <= 1
        assert st['gmres_iters'] < 0.6 * its_plain
        assert rel(qd, soa(q)) < 1e-8


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_preconditioned_mobility_matches_oracle(tiny_cases, prec, tol):
    _, g, A = tiny_cases[0]
    FT = inputs.random_forces(7, g.M)
    Uo = bie.mobility_apply(g, FT, dense=A)
    with binding.Context(g.c, None, 8, 16, gmres_tol=1e-11, precision=prec, precond='eager') as ctx:
        U, st = ctx.mobility_apply(FT)
    say('precond mobility tiny', prec, st['gmres_iters'], rel(U, Uo))
    assert st['converged'] == 1
    assert rel(U[:, :3], Uo[:, :3]) < tol and rel(U[:, 3:], Uo[:, 3:]) < tol


def test_lone_near_pair_is_solved_in_a_few_iterations():
    """Two spheres that are each other's only near partner: P is the inverse of the operator
    (Schur complement) up to the FP16 rounding of its blocks (~1e-3), so GMRES reaches 1e-10
    in about three iterations (plain GMRES: about 25)."""
    c = np.array([[0.0, 0.0, 0.0], [2.04, 0.2, -0.1]])
    rhs = np.random.default_rng(5).standard_normal((3, 2 * 128))
    with binding.Context(c, None, 8, 16, gmres_tol=1e-10) as plain:
        _, s0 = plain.bie_solve(rhs)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-10, precond='eager') as ctx:
        q, st = ctx.bie_solve(rhs)
        y = ctx.bie_apply(q)
    say('lone pair its', st['gmres_iters'], 'plain', s0['gmres_iters'])
    assert st['gmres_iters'] <= 4 < s0['gmres_iters']
    assert rel(y, rhs) < 1e-9


@pytest.mark.parametrize("coarse", [False, True])
def test_configuration_change_rebuilds_the_preconditioner(tiny_cases, coarse):
    """A new configuration rebuilds the preconditioner (one or two levels) at its first solve;
    a second product on the same configuration reuses it; both configurations' velocities are
    the oracle's."""
    (_, g0, A0), (_, g1, A1) = tiny_cases
    FT = inputs.random_forces(11, g0.M)
    with binding.Context(g0.c, None, 8, 16, gmres_tol=1e-11, precond='eager', precond_coarse=coarse) as ctx:
        U0, s0 = ctx.mobility_apply(FT)
        U0b, s0b = ctx.mobility_apply(FT)
        ctx.set_state(g1.c)
        U1, s1 = ctx.mobility_apply(FT)
    say('set-up ms', s0['t_precond_ms'], s0b['t_precond_ms'], s1['t_precond_ms'])
    assert s0['t_precond_ms'] > 0 and s0b['t_precond_ms'] == 0 and s1['t_precond_ms'] > 0
    assert np.array_equal(U0, U0b)
    assert rel(U0, bie.mobility_apply(g0, FT, dense=A0)) < 1e-9
    assert rel(U1, bie.mobility_apply(g1, FT, dense=A1)) < 1e-9


@pytest.mark.parametrize("close", [False, True])
def test_packing64_preconditioned_equals_plain(close):
    """64-sphere packing (gaps down to 0.01), FP64: the same velocities as the unpreconditioned
    solve, with and without the close-pair near class."""
    w = inputs.workload('packing64', 0)
    c = w['centers']
    kw = dict(near_close_gap=0.02) if close else {}
    FT = inputs.random_forces(17, c.shape[0])
    out = {}
    for pc in (False, True):
        with binding.Context(c, None, 12, 24, gmres_tol=1e-10, precond='eager' if pc else False, **kw) as ctx:
            out[pc] = ctx.mobility_apply(FT)
    (U0, s0), (U1, s1) = out[False], out[True]
    say('packing64 close', close, 'its', s0['gmres_iters'], s1['gmres_iters'], 'setup ms',
        round(s1['t_precond_ms'], 1), 'fallback', s1['precond_fallback'], 'diff', rel(U1, U0))
    assert s1['converged'] == 1 and s1['precond_fallback'] == 0
    assert rel(U1, U0) < 1e-8
    assert s1['gmres_iters'] < 0.6 * s0['gmres_iters']


def test_rsa216_six_force_sets_mixed():
    """The timed configuration with precond: 216 spheres, 12x24, six force sets per pass,
    mixed precision at GMRES 1e-8: the unpreconditioned velocities within the solve
    tolerance, in fewer iterations."""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    M = c.shape[0]
    FT = inputs.random_forces(100, M, k=6)
    out = {}
    for pc in (False, True):
        with binding.Context(c, None, 12, 24, gmres_tol=1e-8, precision='mixed', tune_K=6, side_stream=True,
                             precond='eager' if pc else False) as ctx:
            out[pc] = ctx.mobility_apply_multi(FT)
    (U0, s0), (U1, s1) = out[False], out[True]
    say('rsa216 K=6 its', s0['gmres_iters'], s1['gmres_iters'], 'setup ms', round(s1['t_precond_ms'], 1),
        'fallback', s1['precond_fallback'], 'diff', rel(U1, U0))
    assert s1['converged'] == 1 and s1['precond_fallback'] == 0
    assert rel(U1, U0) < 1e-6
    assert s1['gmres_iters'] < 0.6 * s0['gmres_iters']


def test_preconditioned_lcp_and_step_equal_plain(tiny_cases):
    """An LCP solve and a time step with precond give the unpreconditioned results."""
    _, g, _ = tiny_cases[0]
    ax = inputs.janus_axes(3, g.M)
    res = {}
    b = None
    for pc in (False, True):
        with binding.Context(g.c, ax, 8, 16, lo=(4, 8), gmres_tol=1e-11, precond=pc) as ctx:  # on reuse
            pairs, gaps = ctx.find_contacts(0.1)
            assert len(pairs) > 0
            if b is None:
                xs, ws = inputs.planted_lcp(4, len(pairs))
                b = ws - ctx.lcp_apply(pairs, xs)
            x, lst = ctx.lcp_solve(pairs, b, 'bi')
            ctx.step(0.1, 0.1, 'mono')
            res[pc] = (x, ctx.get_state()[0], lst)
    say('lcp products', res[False][2]['mvp_hi'], res[True][2]['mvp_hi'])
    assert rel(res[True][0], res[False][0]) < 1e-8
    assert np.abs(res[True][1] - res[False][1]).max() < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batch_preconditioned_equals_plain(prec, tol):
    """Uneven suspensions in one batch context, each with its own preconditioner (segmented
    launches): the plain batch's velocities, in fewer lockstep iterations; per-instance
    statistics and a second product without a new set-up."""
    inst = inputs.batched_suspensions(0, n_inst=8)
    FTs = [inputs.random_forces(600 + b, c.shape[0]) for b, (c, _, _) in enumerate(inst)]
    with binding.BatchContext(inst, gmres_tol=1e-10, precision=prec) as bc:
        U0, s0 = bc.mobility_apply(FTs, per_instance=True)
    with binding.BatchContext(inst, gmres_tol=1e-10, precision=prec, precond='eager') as bc:
        U1, s1 = bc.mobility_apply(FTs, per_instance=True)
        U2, s2 = bc.mobility_apply(FTs, per_instance=True)
    its0 = [p['gmres_iters'] for p in s0['per_instance']]
    its1 = [p['gmres_iters'] for p in s1['per_instance']]
    say('batch', prec, 'its plain', its0, 'precond', its1, 'set-up ms', round(s1['t_precond_ms'], 1),
        round(s2['t_precond_ms'], 1), 'lockstep', s0['n_far'], s1['n_far'])
    assert s1['converged'] == 1 and s1['precond_fallback'] == 0
    assert s1['t_precond_ms'] > 0 and s2['t_precond_ms'] == 0
    assert all(a < 0.7 * b for a, b in zip(its1, its0))
    for a, b, c in zip(U1, U0, U2):
        assert rel(a, b) < tol
        assert np.array_equal(a, c)


def test_precond_on_reuse_builds_at_the_second_solve_of_a_configuration(tiny_cases):
    """precond = 1: the first solve of a configuration is plain GMRES (no set-up), the second
    builds the preconditioner and uses it, later ones reuse it; a new configuration starts over."""
    (_, g0, A0), (_, g1, _) = tiny_cases
    FT = inputs.random_forces(13, g0.M)
    with binding.Context(g0.c, None, 8, 16, gmres_tol=1e-11) as plain:
        U_ref, s_ref = plain.mobility_apply(FT)
    with binding.Context(g0.c, None, 8, 16, gmres_tol=1e-11, precond=True) as ctx:
        U1, s1 = ctx.mobility_apply(FT)
        U2, s2 = ctx.mobility_apply(FT)
        U3, s3 = ctx.mobility_apply(FT)
        ctx.set_state(g1.c)
        _, s4 = ctx.mobility_apply(FT)
        _, s5 = ctx.mobility_apply(FT)
    say('on reuse: its', s1['gmres_iters'], s2['gmres_iters'], s3['gmres_iters'], s4['gmres_iters'],
        s5['gmres_iters'], 'set-up', s1['t_precond_ms'], s2['t_precond_ms'], s3['t_precond_ms'],
        s4['t_precond_ms'], s5['t_precond_ms'])
    assert s1['t_precond_ms'] == 0 and s1['precond_applies'] == 0 and s1['gmres_iters'] == s_ref['gmres_iters']
    assert np.array_equal(U1, U_ref)
    assert s2['t_precond_ms'] > 0 and s2['precond_applies'] > 0 and s2['gmres_iters'] < 0.6 * s1['gmres_iters']
    assert s3['t_precond_ms'] == 0 and s3['gmres_iters'] == s2['gmres_iters'] and np.array_equal(U3, U2)
    assert rel(U2, U1) < 1e-9
    assert s4['t_precond_ms'] == 0 and s4['precond_applies'] == 0
    assert s5['t_precond_ms'] > 0


def test_precond_on_reuse_counts_a_refined_solve_once(tiny_cases):
    """Mixed precision with an FP64 refinement sweep: the correction solves belong to the same
    solve, so precond = 1 still builds nothing in a configuration's first product."""
    _, g, _ = tiny_cases[0]
    FT = inputs.random_forces(19, g.M)
    with binding.Context(g.c, None, 8, 16, gmres_tol=1e-9, precision='mixed', refine=1, precond=True) as ctx:
        _, s1 = ctx.mobility_apply(FT)
        _, s2 = ctx.mobility_apply(FT)
    say('refined: sweeps', s1['refine_sweeps'], s2['refine_sweeps'], 'set-up', s1['t_precond_ms'],
        s2['t_precond_ms'])
    assert s1['t_precond_ms'] == 0 and s1['precond_applies'] == 0
    assert s2['t_precond_ms'] > 0 and s2['precond_applies'] > 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_side_stream_preconditioned_is_bit_identical(prec):
    """With the side stream on, the preconditioner's D^-1 v GEMM runs there beside the
    block product: K = 1 and 6 densities reproduce the one-stream context bit for bit
    (same kernels, same sums; the final sum waits for both streams)."""
    w = inputs.workload('lattice27', 1)
    c = w['centers']
    out = {}
    for side in (False, True):
        with binding.Context(c, None, 8, 16, precision=prec, gmres_tol=1e-10, side_stream=side,
                             precond='eager') as ctx:
            r = []
            for K in (1, 6):
                U, st = ctx.mobility_apply_multi(inputs.random_forces(30 + K, c.shape[0], k=K))
                assert st['converged'] == 1 and st['precond_applies'] > 0
                r.append(U)
            out[side] = r
    say('side stream precond', prec, 'equal', [np.array_equal(a, b) for a, b in zip(out[False], out[True])])
    for a, b in zip(out[False], out[True]):
        assert np.array_equal(a, b)


def test_two_level_matches_oracle_and_its_iteration_count(tiny_cases):
    """precond_coarse (a coarse correction on every sphere's degree <= 2 harmonics before
    the near patches; its far pairs on a 6x12 source grid when their centres are closer
    than 3.5 radii, else on a 3x6 grid, at 8x16 nodes): the oracle's density, in the
    oracle's two-level iteration count (+-1: inv(E) by Newton-Schulz to 1e-2 and stored in
    FP32 on the device), fewer than with one level."""
    for seed, g, A in tiny_cases:
        rhs = -bie.completion(g, inputs.random_forces(40 + seed, g.M))
        q = np.linalg.solve(A, rhs.ravel())
        P = bie.near_patch_preconditioner(g, A)
        d = np.linalg.norm(g.c[:, None] - g.c[None], axis=2)
        far = g.pair_class() == 0
        say('far pairs closer than 3.5:', int((far & (d < 3.5)).sum()), 'of', int(far.sum()))
        P2 = bie.two_level_preconditioner(g, A, P, coarse_theta=(6, 3), coarse_close=3.5)
        _, its1, _ = bie.gmres(lambda v: A @ v.ravel(), rhs, tol=1e-10, right=P)
        _, its2, _ = bie.gmres(lambda v: A @ v.ravel(), rhs, tol=1e-10, right=P2)
        with binding.Context(g.c, None, 8, 16, gmres_tol=1e-10, precond='eager', precond_coarse=True) as ctx:
            qd, st = ctx.bie_solve(soa(rhs))
        say('two-level tiny seed', seed, 'gpu its', st['gmres_iters'], 'oracle', its2, 'one level', its1,
            'setup ms', round(st['t_precond_ms'], 1))
        assert st['converged'] == 1
        assert rel(qd, soa(q)) < 1e-8
        assert abs(st['gmres_iters'] - its2) <= 1
        assert st['gmres_iters'] < its1


def test_two_level_rsa216_six_force_sets_mixed():
    """The timed configuration with the two-level preconditioner: the plain solves'
    velocities within the mixed tolerance, in fewer iterations than one level."""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    M = c.shape[0]
    FT = inputs.random_forces(100, M, k=6)
    out = {}
    for mode in ('plain', 'one', 'two'):
        with binding.Context(c, None, 12, 24, gmres_tol=1e-8, precision='mixed', tune_K=6, side_stream=True,
                             precond=False if mode == 'plain' else 'eager', precond_coarse=mode == 'two') as ctx:
            out[mode] = ctx.mobility_apply_multi(FT)
    say('rsa216 K=6 its plain', out['plain'][1]['gmres_iters'], 'one level', out['one'][1]['gmres_iters'],
        'two levels', out['two'][1]['gmres_iters'], 'setup ms', round(out['two'][1]['t_precond_ms'], 1),
        'diff', rel(out['two'][0], out['plain'][0]))
    assert out['two'][1]['converged'] == 1
    assert rel(out['two'][0], out['plain'][0]) < 1e-6
    assert out['two'][1]['gmres_iters'] < 0.8 * out['one'][1]['gmres_iters']


def test_two_level_warm_start_after_a_small_move():
    """A configuration moved a little, as by a time step (every sphere by 1e-3 radii), starts
    the coarse inverse's Newton-Schulz iteration from the previous configuration's inverse: in
    fewer steps than a cold set-up, with the plain solve's velocities."""
    w = inputs.workload('rsa216', 0)
    c0 = w['centers']
    M = c0.shape[0]
    d = np.random.default_rng(5).standard_normal(c0.shape)
    c1 = c0 + 1e-3 * d / np.linalg.norm(d, axis=1, keepdims=True)
    FT = inputs.random_forces(7, M)
    kw = dict(gmres_tol=1e-10, precision='fp64', precond='eager', precond_coarse=True)
    with binding.Context(c0, None, 12, 24, **kw) as ctx:
        _, s0 = ctx.mobility_apply(FT)
        ctx.set_state(c1)
        Uw, sw = ctx.mobility_apply(FT)
    with binding.Context(c1, None, 12, 24, **kw) as ctx:
        Uc, sc = ctx.mobility_apply(FT)
    with binding.Context(c1, None, 12, 24, gmres_tol=1e-10, precision='fp64') as ctx:
        Up, _ = ctx.mobility_apply(FT)
    say('warm start: Newton-Schulz steps cold', s0['precond_coarse_steps'], sc['precond_coarse_steps'], 'warm',
        sw['precond_coarse_steps'], 'its', sc['gmres_iters'], sw['gmres_iters'], 'set-up ms',
        round(sc['t_precond_ms'], 1), round(sw['t_precond_ms'], 1))
    assert s0['precond_coarse_warm'] == 0 and sc['precond_coarse_warm'] == 0 and sw['precond_coarse_warm'] == 1
    assert sw['precond_coarse_steps'] < sc['precond_coarse_steps']
    assert abs(sw['gmres_iters'] - sc['gmres_iters']) <= 1
    assert rel(Uw, Up) < 1e-8 and rel(Uc, Up) < 1e-8


def test_two_level_packing64_fp64_equals_plain():
    """64 spheres at gaps down to 0.01 (close class on), FP64: the plain velocities."""
    w = inputs.workload('packing64', 0)
    c = w['centers']
    FT = inputs.random_forces(7, c.shape[0])
    kw = dict(gmres_tol=1e-10, near_close_gap=0.05, near_close_up=3)
    out = {}
    for mode in ('plain', 'two'):
        with binding.Context(c, None, 12, 24, precond='eager' if mode == 'two' else False,
                             precond_coarse=mode == 'two', **kw) as ctx:
            out[mode] = ctx.mobility_apply(FT)
    say('packing64 two-level its', out['plain'][1]['gmres_iters'], out['two'][1]['gmres_iters'], 'diff',
        rel(out['two'][0], out['plain'][0]))
    assert out['two'][1]['converged'] == 1
    assert rel(out['two'][0], out['plain'][0]) < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_level_side_stream_is_bit_identical(prec):
    """With the side stream the coarse level's Z c accumulation follows the D^-1 v GEMM on
    that stream: bit for bit the one-stream result, K = 1 and 6."""
    w = inputs.workload('lattice27', 1)
    c = w['centers']
    out = {}
    for side in (False, True):
        with binding.Context(c, None, 8, 16, precision=prec, gmres_tol=1e-10, side_stream=side,
                             precond='eager', precond_coarse=True) as ctx:
            r = []
            for K in (1, 6):
                U, st = ctx.mobility_apply_multi(inputs.random_forces(30 + K, c.shape[0], k=K))
                assert st['converged'] == 1
                r.append(U)
            out[side] = r
    for a, b in zip(out[False], out[True]):
        assert np.array_equal(a, b)


def test_two_level_lcp_and_step_equal_plain(tiny_cases):
    """An LCP solve and a time step with the two-level preconditioner (built on reuse)."""
    _, g, _ = tiny_cases[0]
    ax = inputs.janus_axes(3, g.M)
    res = {}
    b = None
    for pc in (False, True):
        with binding.Context(g.c, ax, 8, 16, lo=(4, 8), gmres_tol=1e-11, precond=pc, precond_coarse=pc) as ctx:
            pairs, gaps = ctx.find_contacts(0.1)
            if b is None:
                xs, ws = inputs.planted_lcp(4, len(pairs))
                b = ws - ctx.lcp_apply(pairs, xs)
            x, lst = ctx.lcp_solve(pairs, b, 'bi')
            ctx.step(0.1, 0.1, 'mono')
            res[pc] = (x, ctx.get_state()[0])
    assert rel(res[True][0], res[False][0]) < 1e-8
    assert np.abs(res[True][1] - res[False][1]).max() < 1e-10


def test_two_level_is_refused_for_batch_contexts():
    inst = inputs.batched_suspensions(0, n_inst=2)
    with pytest.raises(Exception, match='precond_coarse'):
        binding.BatchContext(inst, gmres_tol=1e-10, precond=True, precond_coarse=True)


def test_two_level_fine_grid_lattice27():
    """27 spheres at 16x32 nodes (512 per sphere, the largest grid the two-level form takes;
    its far-block kernel then needs more than 64 KB of LDS): the plain FP64 velocities."""
    w = inputs.workload('lattice27', 1)
    c = w['centers']
    FT = inputs.random_forces(8, c.shape[0])
    out = {}
    for mode in ('plain', 'two'):
        with binding.Context(c, None, 16, 32, gmres_tol=1e-10, precond='eager' if mode == 'two' else False,
                             precond_coarse=mode == 'two') as ctx:
            out[mode] = ctx.mobility_apply(FT)
    say('lattice27 16x32 two-level its', out['plain'][1]['gmres_iters'], out['two'][1]['gmres_iters'],
        'diff', rel(out['two'][0], out['plain'][0]))
    assert out['two'][1]['converged'] == 1
    assert rel(out['two'][0], out['plain'][0]) < 1e-8
    assert out['two'][1]['gmres_iters'] < out['plain'][1]['gmres_iters']


@pytest.mark.parametrize("case", ["one sphere", "no near pairs"])
def test_two_level_without_near_pairs(case):
    """The two-level preconditioner where the near patches are empty: one sphere (P2 is
    then A^-1 up to the FP16 and Newton-Schulz roundings) and a dilute 2x2x2 lattice at
    centre distance 3 (gap 1 > the near gap, so no near blocks at all: D^-1 plus the coarse
    level). FP64 velocities as the oracle's dense solve."""
    if case == "one sphere":
        c = np.array([[0.3, -0.2, 0.1]])
    else:
        g = np.arange(2) * 3.0
        c = np.array([[x, y, z] for x in g for y in g for z in g]) + 0.05 * np.random.default_rng(3).standard_normal((8, 3))
    geo = bie.Geometry(c, 1.0, 8, 16)
    A = bie.dense_operator(geo)
    FT = inputs.random_forces(12, c.shape[0])
    Uo = bie.mobility_apply(geo, FT, dense=A)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-11, precond='eager', precond_coarse=True) as ctx:
        U, st = ctx.mobility_apply(FT)
    say('two-level', case, 'its', st['gmres_iters'], 'err', rel(U, Uo))
    assert st['converged'] == 1 and st['precond_applies'] > 0
    assert rel(U, Uo) < 1e-9
    if case == "one sphere":
        assert st['gmres_iters'] <= 3
