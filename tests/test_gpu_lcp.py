"""GPU parity of the LCP layer (products, BB-PGD, Mono-PQN, Bi-PQN, step) vs oracle."""
import sys

import numpy as np
import pytest

from oracle import bie, dynamics, lcp
from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cases():
    out = []
    for seed in (0, 2):
        c = inputs.workload('tiny', seed)['centers']
        g = bie.Geometry(c, 1.0, 8, 16)
        A = bie.dense_operator(g)
        glo = bie.Geometry(c, 1.0, 4, 8)
        Alo = bie.dense_operator(glo)
        pairs, gaps = dynamics.find_contacts(c, 1.0, 0.1)
        Aop = lcp.lcp_operator(lambda F, g=g, A=A: bie.mobility_apply(g, F, dense=A), c, pairs)
        n = pairs.shape[0]
        Ad = np.column_stack([Aop(np.eye(n)[k]) for k in range(n)])
        axes = -c / np.linalg.norm(c, axis=1)[:, None]
        b_real = lcp.lcp_b(gaps, 0.1, c, pairs, bie.nc_velocity(g, axes, 1.0, dense=A))
        xs, ws = inputs.planted_lcp(seed, n)
        out.append(dict(c=c, g=g, A=A, glo=glo, Alo=Alo, pairs=pairs, gaps=gaps, Ad=Ad, axes=axes,
                        b_real=b_real, x_pl=xs, b_pl=ws - Ad @ xs))
    return out


def test_lcp_apply_matches_oracle(cases):
    for cs in cases:
        x = np.random.default_rng(1).uniform(0, 1, cs['pairs'].shape[0])
        with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-13) as ctx:
            Ax = ctx.lcp_apply(cs['pairs'], x)
            Alox = ctx.lcp_apply(cs['pairs'], x, fidelity=binding.PQN_LOFI)
        assert np.abs(Ax - cs['Ad'] @ x).max() < 1e-10 * np.abs(cs['Ad'] @ x).max()
        Alo_ref = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'],
                                   cs['pairs'])(x)
        assert np.abs(Alox - Alo_ref).max() < 1e-10 * np.abs(Alo_ref).max()


@pytest.mark.parametrize("solver", ["mono", "bb", "bi"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lcp_solve_matches_brute_force(cases, solver, prec):
    # FP64: solve to 1e-12 and compare at 1e-10. Mixed: each fresh product carries the FP32
    # far-field rounding (~1e-8 relative), so the KKT floor is ~1e-9; compare x at 1e-6.
    tol = 1e-10 if prec == 'fp64' else 1e-6
    kkt = (1e-12, 1e-15) if prec == 'fp64' else (1e-9, 1e-9)
    for cs in cases:
        for name, b in (('real', cs['b_real']), ('planted', cs['b_pl'])):
            say('lcp_solve', solver, prec, name)
            xbf = lcp.brute_force_lcp(cs['Ad'], b)
            with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-12, precision=prec) as ctx:
                x, st = ctx.lcp_solve(cs['pairs'], b, solver, tol_abs=kkt[0], tol_rel=kkt[1], k_max=400)
            assert st['converged'] == 1, st
            assert np.abs(x - xbf).max() <= tol * max(np.abs(xbf).max(), 1e-300), (x, xbf, st)
            assert x.min() >= 0.0
            if solver == 'bi':
                assert st['mvp_lo'] >= 1 or np.all(xbf == 0)


def test_lcp_solver_counts_match_oracle(cases):
    """Same algorithm on the same operator: iteration counts agree (MVP counts may differ by rounding)."""
    cs = cases[0]
    b = cs['b_pl']
    Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
    Alo = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'], cs['pairs'])
    _, _, sm = lcp.mono_pqn(Aop, b)
    _, _, sb = lcp.bi_pqn(Aop, Alo, b)
    with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-13) as ctx:
        _, gm = ctx.lcp_solve(cs['pairs'], b, 'mono')
        _, gb = ctx.lcp_solve(cs['pairs'], b, 'bi')
    assert abs(gm['mvp_hi'] - sm['mvp']) <= 1
    assert abs(gb['mvp_hi'] - sb['mvp_hi']) <= 1
    say('mono', gm['mvp_hi'], sm['mvp'], 'bi', gb['mvp_hi'], gb['mvp_lo'], sb['mvp_hi'], sb['mvp_lo'])


@pytest.mark.parametrize("solver", ["mono", "bi", "bb"])
def test_step_matches_oracle(cases, solver):
    cs = cases[0]
    say('step', solver)
    c1, ax1, info = dynamics.step(cs['c'], cs['axes'], 1.0, (8, 16), (4, 8), 0.1, 0.1, 1.0, solver=solver,
                                  lcp_opts=dict(tol_abs=1e-12, tol_rel=1e-15), tol_gmres=1e-13)
    with binding.Context(cs['c'], cs['axes'], 8, 16, lo=(4, 8), gmres_tol=1e-13) as ctx:
        st = ctx.step(0.1, 0.1, solver, tol_abs=1e-12, tol_rel=1e-15)
        c2, ax2 = ctx.get_state()
    assert st['n_contacts'] == info['pairs'].shape[0]
    assert st['n_active'] == int((info['x'] > 0).sum())
    stages = [st[k] for k in ('t_contacts_ms', 't_nc_ms', 't_lcp_ms', 't_update_ms')]
    assert all(t > 0.0 for t in stages) and sum(stages) <= st['t_total_ms'] * 1.001
    assert np.abs(c2 - c1).max() < 1e-10
    assert np.abs(ax2 - ax1).max() < 1e-10


def test_lcp_edge_cases(cases):
    cs = cases[0]
    with binding.Context(cs['c'], None, 8, 16, lo=(4, 8)) as ctx:
        x, st = ctx.lcp_solve(np.zeros((0, 2), np.int32), np.zeros(0), 'bi')
        assert x.shape == (0,)
        # b >= 0: x = 0 with no product at all
        x, st = ctx.lcp_solve(cs['pairs'], np.abs(cs['b_real']) + 0.1, 'mono')
        assert np.all(x == 0.0) and st['mvp_hi'] == 0
        with pytest.raises(binding.PqnError):
            ctx.lcp_solve(np.array([[0, 99]], np.int32), np.array([-1.0]), 'mono')
        with pytest.raises(binding.PqnError):
            ctx.lcp_solve(cs['pairs'], np.full(cs['pairs'].shape[0], np.nan), 'mono')


def test_bi_pqn_exact_model_counts_match_oracle(cases):
    """Low fidelity = high fidelity grid: the device Bi-PQN needs as few high-fidelity
    products as the oracle's (2-4), fewer than Mono-PQN."""
    for cs in cases:
        b = cs['b_pl']
        Aop = lcp.lcp_operator(lambda F, cs=cs: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
        _, _, sb = lcp.bi_pqn(Aop, Aop, b)
        with binding.Context(cs['c'], None, 8, 16, lo=(8, 16), gmres_tol=1e-13) as ctx:
            x, gb = ctx.lcp_solve(cs['pairs'], b, 'bi')
            _, gm = ctx.lcp_solve(cs['pairs'], b, 'mono')
        say('bi exact model', gb['mvp_hi'], gb['mvp_lo'], 'oracle', sb['mvp_hi'], sb['mvp_lo'], 'mono', gm['mvp_hi'])
        assert abs(gb['mvp_hi'] - sb['mvp_hi']) <= 1
        assert gb['mvp_hi'] < gm['mvp_hi']
        assert np.abs(x - cs['x_pl']).max() < 1e-7 * np.abs(cs['x_pl']).max()


def test_bi_pqn_safe_when_low_fidelity_model_is_poor():
    """64-sphere packing with gaps down to 0.01 and the coarse 6x12 model: whatever the
    model's quality, Bi-PQN must return a solution of the LCP (complementarity within
    tolerance) that agrees with Mono-PQN's; a model that shows non-positive curvature is
    rejected (model_rejected) and the solve finishes as Mono-PQN on A."""
    w = inputs.workload('packing64', 1)
    c = w['centers']
    kw = dict(tol_abs=1e-10, tol_rel=1e-12, k_max=300)
    with binding.Context(c, None, 16, 32, lo=(6, 12), gmres_tol=1e-11, gmres_tol_lo=1e-11) as ctx:
        pairs, _ = ctx.find_contacts(0.1)
        xs, ws = inputs.planted_lcp(1, pairs.shape[0])
        b = ws - ctx.lcp_apply(pairs, xs)
        xb, sb = ctx.lcp_solve(pairs, b, 'bi', **kw)
        xm, sm = ctx.lcp_solve(pairs, b, 'mono', **kw)
        wb = ctx.lcp_apply(pairs, xb) + b
    say('bi on packing64', sb['mvp_hi'], sb['mvp_lo'], 'rejected', sb['model_rejected'], 'mono', sm['mvp_hi'])
    assert sb['converged'] == 1 and np.all(np.isfinite(xb))
    sw = max(1.0, np.abs(b).max())
    assert xb.min() >= 0.0 and wb.min() >= -1e-8 * sw
    assert np.abs(xb * wb).max() <= 1e-8 * max(1.0, np.abs(xb).max()) * sw
    assert np.abs(xb - xm).max() <= 1e-6 * np.abs(xm).max()


def test_warm_started_slip_solves_match_cold_steps():
    """Time steps whose slip-driven solve starts from the previous step's density reach
    the same trajectory (to the GMRES tolerance) in fewer Krylov iterations."""
    w = inputs.workload('lattice27', 0)
    c = w['centers']
    axes = inputs.janus_axes(3, c.shape[0])
    kw = dict(gmres_tol=1e-10, precision='fp64')
    its = {}
    pos = {}
    for warm in (False, True):
        with binding.Context(c, axes, 8, 16, lo=(4, 8), warm_start=warm, **kw) as ctx:
            its[warm] = [ctx.step(1e-3, 0.1, 'mono')['gmres_iters_nc'] for _ in range(3)]
            pos[warm] = ctx.get_state()[0]
    say('nc iterations cold', its[False], 'warm', its[True])
    disp = np.abs(pos[False] - c).max()
    assert np.abs(pos[True] - pos[False]).max() < 1e-7 * disp
    assert its[True][0] == its[False][0]
    assert sum(its[True][1:]) < sum(its[False][1:])


def test_warm_started_steps_match_oracle(cases):
    """Two consecutive time steps with the warm-started slip solve against two oracle steps."""
    cs = cases[0]
    c, ax = cs['c'], cs['axes']
    for _ in range(2):
        c, ax, _ = dynamics.step(c, ax, 1.0, (8, 16), (4, 8), 0.05, 0.1, 1.0, solver='mono',
                                 lcp_opts=dict(tol_abs=1e-12, tol_rel=1e-15), tol_gmres=1e-13)
    with binding.Context(cs['c'], cs['axes'], 8, 16, lo=(4, 8), gmres_tol=1e-13, warm_start=True) as ctx:
        its = [ctx.step(0.05, 0.1, 'mono', tol_abs=1e-12, tol_rel=1e-15)['gmres_iters_nc'] for _ in range(2)]
        c2, ax2 = ctx.get_state()
    say('warm steps vs oracle, nc iterations', its)
    assert np.abs(c2 - c).max() < 1e-10
    assert np.abs(ax2 - ax).max() < 1e-10


def _mid_operator(cs):
    gm = bie.Geometry(cs['c'], 1.0, 6, 12)
    Am = bie.dense_operator(gm)
    return gm, Am, lcp.lcp_operator(lambda F: bie.mobility_apply(gm, F, dense=Am), cs['c'], cs['pairs'])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bi_pqn_rec_matches_oracle(cases, prec):
    """Recursive Bi-PQN over the 8x16, 6x12 and 4x8 grids: the device solution equals the
    brute-force LCP solution, the product at the second low fidelity equals the oracle's
    operator, and in FP64 the products per fidelity match the oracle's recursion (+-1:
    inner tolerances are decided on rounding-level KKT values)."""
    tol = 1e-10 if prec == 'fp64' else 1e-6
    kkt = (1e-12, 1e-15) if prec == 'fp64' else (1e-9, 1e-9)
    for cs in cases:
        gm, Am, Amid = _mid_operator(cs)
        Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
        Alo = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'], cs['pairs'])
        with binding.Context(cs['c'], None, 8, 16, lo=(6, 12), lo2=(4, 8), gmres_tol=1e-13,
                             precision=prec) as ctx:
            v = np.random.default_rng(3).uniform(0, 1, cs['pairs'].shape[0])
            y2 = ctx.lcp_apply(cs['pairs'], v, fidelity=binding.PQN_LOFI2)
            y1 = ctx.lcp_apply(cs['pairs'], v, fidelity=binding.PQN_LOFI)
            ptol = 1e-10 if prec == 'fp64' else 1e-6
            assert np.abs(y2 - Alo(v)).max() < ptol * np.abs(Alo(v)).max()
            assert np.abs(y1 - Amid(v)).max() < ptol * np.abs(Amid(v)).max()
            for name, b in (('real', cs['b_real']), ('planted', cs['b_pl'])):
                say('birec', prec, name)
                xbf = lcp.brute_force_lcp(cs['Ad'], b)
                x, st = ctx.lcp_solve(cs['pairs'], b, 'birec', tol_abs=kkt[0], tol_rel=kkt[1], k_max=400)
                assert st['converged'] == 1, st
                assert x.min() >= 0.0
                assert np.abs(x - xbf).max() <= tol * max(np.abs(xbf).max(), 1e-300), (x, xbf, st)
                if prec == 'fp64':
                    _, _, so = lcp.bi_pqn_rec([Aop, Amid, Alo], b, tol_abs=kkt[0], tol_rel=kkt[1], k_max=400)
                    say('  device', st['mvp_hi'], st['mvp_lo'], st['mvp_lo2'], 'oracle', so['mvp'])
                    assert abs(st['mvp_hi'] - so['mvp'][0]) <= 1
                    assert abs(st['mvp_lo'] - so['mvp'][1]) <= 2
                    assert abs(st['mvp_lo2'] - so['mvp'][2]) <= 4
                    assert st['model_rejected'] == int(so['fallback'])
                if np.any(xbf > 0):
                    assert st['mvp_lo'] >= 1 and st['mvp_lo2'] >= 1


def test_bi_pqn_rec_counts_match_oracle_default_tolerance(cases):
    """Same recursion at the default KKT tolerance (1e-8): per-fidelity product counts
    agree with the oracle's."""
    for cs in cases:
        gm, Am, Amid = _mid_operator(cs)
        Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
        Alo = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'], cs['pairs'])
        b = cs['b_pl']
        _, _, so = lcp.bi_pqn_rec([Aop, Amid, Alo], b)
        with binding.Context(cs['c'], None, 8, 16, lo=(6, 12), lo2=(4, 8), gmres_tol=1e-13) as ctx:
            _, st = ctx.lcp_solve(cs['pairs'], b, 'birec')
        say('birec counts', st['mvp_hi'], st['mvp_lo'], st['mvp_lo2'], 'oracle', so['mvp'])
        assert st['mvp_hi'] == so['mvp'][0]
        assert abs(st['mvp_lo'] - so['mvp'][1]) <= 1
        assert abs(st['mvp_lo2'] - so['mvp'][2]) <= 2


def test_bi_pqn_rec_step_and_errors(cases):
    """A time step with recursive Bi-PQN reaches the oracle's configuration (the LCP
    solution is unique, whichever solver finds it); without a second low-fidelity grid
    the solver is refused."""
    cs = cases[0]
    c1, ax1, info = dynamics.step(cs['c'], cs['axes'], 1.0, (8, 16), (4, 8), 0.1, 0.1, 1.0, solver='mono',
                                  lcp_opts=dict(tol_abs=1e-12, tol_rel=1e-15), tol_gmres=1e-13)
    with binding.Context(cs['c'], cs['axes'], 8, 16, lo=(6, 12), lo2=(4, 8), gmres_tol=1e-13) as ctx:
        st = ctx.step(0.1, 0.1, 'birec', tol_abs=1e-12, tol_rel=1e-15)
        c2, ax2 = ctx.get_state()
    assert st['n_contacts'] == info['pairs'].shape[0]
    assert np.abs(c2 - c1).max() < 1e-10
    assert np.abs(ax2 - ax1).max() < 1e-10
    with binding.Context(cs['c'], None, 8, 16, lo=(4, 8)) as ctx:
        with pytest.raises(binding.PqnError):
            ctx.lcp_solve(cs['pairs'], cs['b_pl'], 'birec')
        with pytest.raises(binding.PqnError):
            ctx.lcp_apply(cs['pairs'], np.ones(cs['pairs'].shape[0]), fidelity=binding.PQN_LOFI2)


@pytest.mark.parametrize("solver", ["mono", "bb", "bi", "birec"])
def test_lcp_solve_from_an_initial_guess_matches_oracle(cases, solver):
    """x^(-1) given (a random guess with negative entries, projected on x >= 0): the device
    reaches the brute-force solution, with the products of the oracle's solver started
    from the same guess (within 1 high, 2 low)."""
    kw = dict(tol_abs=1e-12, tol_rel=1e-15)
    for cs in cases:
        b = cs['b_pl']
        g = np.random.default_rng(5).uniform(-0.5, 1.5, b.size)
        xbf = lcp.brute_force_lcp(cs['Ad'], b)
        Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
        Alo = lcp.lcp_operator(lambda F: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'], cs['pairs'])
        if solver == 'mono':
            _, _, so = lcp.mono_pqn(Aop, b, x0=np.maximum(g, 0.0), **kw)
            ref = (so['mvp'], 0)
        elif solver == 'bb':
            _, _, so = lcp.bb_pgd(Aop, b, x0=np.maximum(g, 0.0), tau0=3 * np.pi, k_max=500, **kw)
            ref = (so['mvp'], 0)
        elif solver == 'bi':
            _, _, so = lcp.bi_pqn(Aop, Alo, b, x0=g, **kw)
            ref = (so['mvp_hi'], so['mvp_lo'])
        else:
            Amid = _mid_operator(cs)[2]
            _, _, so = lcp.bi_pqn_rec([Aop, Amid, Alo], b, x0=g, **kw)
            ref = (so['mvp'][0], so['mvp'][1])
        lo = dict(lo=(6, 12), lo2=(4, 8)) if solver == 'birec' else dict(lo=(4, 8))
        with binding.Context(cs['c'], None, 8, 16, gmres_tol=1e-13, **lo) as ctx:
            x, st = ctx.lcp_solve(cs['pairs'], b, solver, x0=g, k_max=500, **kw)
        say('guess', solver, st['mvp_hi'], st['mvp_lo'], 'oracle', ref)
        assert st['converged'] == 1
        assert np.abs(x - xbf).max() <= 1e-10 * np.abs(xbf).max()
        assert abs(st['mvp_hi'] - ref[0]) <= 1 and abs(st['mvp_lo'] - ref[1]) <= 2
        assert 0.0 <= st['kkt_rel'] < 1.0


def test_lcp_solve_dev_matches_host_arrays(cases):
    """pqn_lcp_solve_dev on device pointers: the same solution and counts as the host-array
    entry point, guess included; an invalid pair is rejected and x is left as it was."""
    import torch
    cs = cases[0]
    b = cs['b_pl']
    n = b.size
    g = np.random.default_rng(6).uniform(-0.5, 1.5, n)
    with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-12) as ctx:
        xh, sh = ctx.lcp_solve(cs['pairs'], b, 'bi', x0=g)
        P = torch.as_tensor(np.ascontiguousarray(cs['pairs'], dtype=np.int32), device='cuda')
        B = torch.as_tensor(b, dtype=torch.float64, device='cuda')
        X = torch.as_tensor(g, dtype=torch.float64, device='cuda')
        torch.cuda.synchronize()
        sd = ctx.lcp_solve_dev(n, P.data_ptr(), B.data_ptr(), X.data_ptr(), 'bi')
        assert np.array_equal(X.cpu().numpy(), xh)
        assert (sd['mvp_hi'], sd['mvp_lo'], sd['iters']) == (sh['mvp_hi'], sh['mvp_lo'], sh['iters'])
        Pbad = P.clone()
        Pbad[0, 1] = 99
        X2 = X.clone()
        torch.cuda.synchronize()
        with pytest.raises(binding.PqnError):
            ctx.lcp_solve_dev(n, Pbad.data_ptr(), B.data_ptr(), X2.data_ptr(), 'mono')
        assert torch.equal(X2, X)


def test_step_with_close_pairs_matches_oracle():
    """A time step of the 8-sphere cluster swimming towards its centroid (dt 0.1) with the
    close-pair class (gap < 0.05 on the 3x grid): contacts, active set and the new
    configuration equal the oracle's step with the same near rule."""
    w = inputs.workload('tiny', 0)
    c = w['centers']
    ax = c.mean(axis=0) - c
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    near = dict(near_close_gap=0.05, near_close_up=3)
    c1, ax1, info = dynamics.step(c, ax, 1.0, (8, 16), (4, 8), 0.1, 0.1, 1.0, solver='mono',
                                  lcp_opts=dict(tol_abs=1e-12, tol_rel=1e-15), tol_gmres=1e-13, near=near)
    with binding.Context(c, ax, 8, 16, lo=(4, 8), gmres_tol=1e-13, **near) as ctx:
        st = ctx.step(0.1, 0.1, 'mono', tol_abs=1e-12, tol_rel=1e-15)
        c2, ax2 = ctx.get_state()
    say('close-pair step: contacts', st['n_contacts'], 'active', st['n_active'])
    assert st['n_contacts'] == info['pairs'].shape[0]
    assert st['n_active'] == int((info['x'] > 0).sum())
    stages = [st[k] for k in ('t_contacts_ms', 't_nc_ms', 't_lcp_ms', 't_update_ms')]
    assert all(t > 0.0 for t in stages) and sum(stages) <= st['t_total_ms'] * 1.001 and st['n_active'] > 0
    assert np.abs(c2 - c1).max() < 1e-10
    assert np.abs(ax2 - ax1).max() < 1e-10


@pytest.mark.parametrize("solver", ["mono", "bi"])
def test_printed_metric_matches_oracle(cases, solver):
    """Alg. 1 as printed (H^(0) = I throughout, printed_metric = 1): the device solvers
    reach the brute-force solution and need the oracle's product counts in that mode."""
    for cs in cases:
        b = cs['b_pl']
        Aop = lcp.lcp_operator(lambda F, cs=cs: bie.mobility_apply(cs['g'], F, dense=cs['A']), cs['c'], cs['pairs'])
        Alo = lcp.lcp_operator(lambda F, cs=cs: bie.mobility_apply(cs['glo'], F, dense=cs['Alo']), cs['c'],
                               cs['pairs'])
        kw = dict(tol_abs=1e-12, tol_rel=1e-15)
        if solver == 'mono':
            _, _, so = lcp.mono_pqn(Aop, b, k_max=300, printed_metric=True, **kw)
            hi_o, lo_o = so['mvp'], 0
        else:
            _, _, so = lcp.bi_pqn(Aop, Alo, b, k_max=100, printed_metric=True, **kw)
            hi_o, lo_o = so['mvp_hi'], so['mvp_lo']
        xbf = lcp.brute_force_lcp(cs['Ad'], b)
        with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-13) as ctx:
            x, st = ctx.lcp_solve(cs['pairs'], b, solver, k_max=300, printed_metric=True, **kw)
            _, st_s = ctx.lcp_solve(cs['pairs'], b, solver, k_max=300, **kw)
        say('printed metric', solver, 'device', st['mvp_hi'], st['mvp_lo'], 'oracle', hi_o, lo_o,
            'scaled metric', st_s['mvp_hi'], st_s['mvp_lo'])
        assert st['converged'] == 1
        assert np.abs(x - xbf).max() <= 1e-10 * np.abs(xbf).max()
        assert abs(st['mvp_hi'] - hi_o) <= 1
        assert abs(st['mvp_lo'] - lo_o) <= 2
    with binding.Context(cases[0]['c'], None, 8, 16) as ctx, pytest.raises(binding.PqnError):
        ctx.lcp_solve(cases[0]['pairs'], cases[0]['b_pl'], 'mono', printed_metric=2)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_recycled_products_match_oracle(cases, prec):
    """Krylov reuse across the products of one LCP solve (recycle = 1): the solutions equal
    brute force and the cold solves, and the GMRES iterations fall as the oracle's
    RecyclingMobility predicts (device CGS2 vs oracle MGS: counts within 2 per product)."""
    tol = 1e-10 if prec == 'fp64' else 1e-6
    kkt = (1e-12, 1e-15) if prec == 'fp64' else (1e-9, 1e-9)
    for cs in cases:
        b = cs['b_pl']
        xbf = lcp.brute_force_lcp(cs['Ad'], b)
        rec = bie.RecyclingMobility(cs['g'], tol=1e-13)
        Aop = lcp.lcp_operator(rec, cs['c'], cs['pairs'])
        xo, _, so = lcp.mono_pqn(Aop, b, tol_abs=1e-12, tol_rel=1e-15)
        with binding.Context(cs['c'], None, 8, 16, lo=(4, 8), gmres_tol=1e-13, precision=prec) as ctx:
            xc, sc = ctx.lcp_solve(cs['pairs'], b, 'mono', tol_abs=kkt[0], tol_rel=kkt[1])
            xr, sr = ctx.lcp_solve(cs['pairs'], b, 'mono', tol_abs=kkt[0], tol_rel=kkt[1], recycle=True)
            xb, sb = ctx.lcp_solve(cs['pairs'], b, 'bi', tol_abs=kkt[0], tol_rel=kkt[1], recycle=True)
            xcold, _ = ctx.lcp_solve(cs['pairs'], b, 'mono', tol_abs=kkt[0], tol_rel=kkt[1])
        say('recycle', prec, 'gmres cold', sc['gmres_iters'], 'recycled', sr['gmres_iters'], 'oracle',
            sum(rec.iters), 'products', sr['mvp_hi'], so['mvp'], 'bi', sb['mvp_hi'], sb['mvp_lo'], sb['gmres_iters'])
        for x, st in ((xc, sc), (xr, sr), (xb, sb)):
            assert st['converged'] == 1
            assert np.abs(x - xbf).max() <= tol * np.abs(xbf).max()
        assert np.abs(xo - xbf).max() <= 1e-10 * np.abs(xbf).max()
        assert np.array_equal(xc, xcold)          # the store does not outlive its call
        assert sr['gmres_iters'] < sc['gmres_iters']
        if prec == 'fp64':
            assert abs(sr['mvp_hi'] - so['mvp']) <= 1
            assert abs(sr['gmres_iters'] - sum(rec.iters)) <= 2 * sr['mvp_hi']
