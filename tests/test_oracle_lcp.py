"""Pins of the oracle's LCP layer: prox, step size, BFGS, solvers."""
import json
import os

import numpy as np
import pytest

from oracle import bie, dynamics, lcp
from paper_2604_10089_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'closed_forms.json')))


def _spd(n, seed, kappa=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(1.0, kappa, n)) @ Q.T


def _bfgs_memory(A, r, seed):
    rng = np.random.default_rng(seed)
    qn = lcp.QuasiNewton(A.shape[0])
    for _ in range(r):
        s = rng.standard_normal(A.shape[0])
        qn.update(s, A @ s)
    return qn


@pytest.mark.parametrize("n,r,seed", [(8, 3, 0), (8, 6, 1), (40, 5, 2), (40, 12, 3)])
def test_prox_kkt_and_primal(n, r, seed):
    A = _spd(n, seed)
    qn = _bfgs_memory(A, r, seed + 10)
    B = qn.dense()
    xt = np.random.default_rng(seed + 20).standard_normal(n) * 2.0
    xh, steps, conv = lcp.prox_ssn(xt, np.array(qn.U).T, np.array(qn.V).T)
    assert conv
    lam = B @ (xh - xt)
    scale = max(1.0, np.abs(xt).max())
    assert xh.min() >= 0.0
    assert lam.min() >= -1e-12 * scale
    assert np.abs(xh * lam).max() <= 1e-12 * scale * scale
    assert np.abs(xh - lcp.prox_primal(B, xt)).max() <= 1e-10 * scale


def test_prox_rank_zero_is_projection():
    xt = np.array([1.0, -2.0, 0.0, 3.5])
    xh, _, _ = lcp.prox_ssn(xt, None, None)
    assert np.array_equal(xh, np.maximum(xt, 0.0))


def test_bfgs_secant_and_inverse():
    n = 12
    A = _spd(n, 4)
    rng = np.random.default_rng(5)
    qn = lcp.QuasiNewton(n)
    H = np.eye(n)
    for _ in range(6):
        s = rng.standard_normal(n)
        y = A @ s
        assert qn.update(s, y)
        assert np.abs(qn.B_apply(s) - y).max() <= 1e-12 * np.abs(y).max()
        rho = 1.0 / (y @ s)
        E = np.eye(n) - rho * np.outer(s, y)
        H = E @ H @ E.T + rho * np.outer(s, s)        # textbook inverse BFGS update
    assert np.abs(H @ qn.dense() - np.eye(n)).max() < 1e-10
    g = rng.standard_normal(n)
    assert np.abs(qn.H_apply(g) - H @ g).max() < 1e-10 * np.abs(H @ g).max()


def test_step_size_is_constrained_minimiser():
    n = 10
    A = _spd(n, 6)
    rng = np.random.default_rng(7)
    for trial in range(20):
        x = np.maximum(rng.standard_normal(n), 0.0)
        b = rng.standard_normal(n)
        g = A @ x + b
        xh = np.maximum(x - 0.3 * g + 0.1 * rng.standard_normal(n), 0.0)
        p = xh - x
        if p @ g >= 0:
            continue
        eta, reset = lcp.step_size(g, x, p, A @ p)
        assert not reset
        neg = p < 0
        emax = np.min(-x[neg] / p[neg]) if neg.any() else 1e6
        grid = np.linspace(0.0, emax, 20001)
        fvals = [lcp.objective(A, b, x + e * p) for e in grid]
        assert lcp.objective(A, b, x + eta * p) <= min(fvals) + 1e-12
        assert (x + eta * p).min() >= -1e-14
        alpha = 0.49   # Lemma 1, sufficient decrease in the form of eq. (suffDecSimp)
        assert 0.5 * eta * (p @ A @ p) <= -(1 - alpha) * (g @ p) + 1e-14


def test_step_size_edge_cases():
    g = np.array([1.0, 1.0])
    x = np.array([1.0, 1.0])
    assert lcp.step_size(g, x, np.array([1.0, 0.0]), np.array([1.0, 0.0])) == (1.0, True)   # ascent
    assert lcp.step_size(g, x, np.array([-1.0, 0.0]), np.array([1.0, 0.0])) == (1.0, True)   # pAp < 0


def test_secant_transfer_invariant():
    n = 9
    rng = np.random.default_rng(8)
    Ahat = _spd(n, 9)
    corr = lcp.QuasiNewton(n, b0_apply=lambda v: Ahat @ v)
    Bk = Ahat.copy()
    S = [rng.standard_normal(n) for _ in range(4)]
    Y = [Bk @ s for s in S]
    s = rng.standard_normal(n)
    y = _spd(n, 10) @ s
    assert corr.update(s, y)
    S2, Y2 = lcp.secant_transfer(S, Y, corr.U[0], corr.V[0])
    Bk1 = Bk + np.outer(corr.U[0], corr.U[0]) - np.outer(corr.V[0], corr.V[0])
    for sh, yh in zip(S2, Y2):
        assert np.abs(Bk1 @ sh - yh).max() < 1e-12 * np.abs(yh).max()
    assert np.abs(Bk1 @ s - y).max() < 1e-12 * np.abs(y).max()


def _dense_lcp(g, A, pairs):
    mob = lambda FT: bie.mobility_apply(g, FT, dense=A)
    Aop = lcp.lcp_operator(mob, g.c, pairs)
    n = pairs.shape[0]
    return Aop, np.column_stack([Aop(np.eye(n)[k]) for k in range(n)])


def _check_complementarity(x, Ad, b):
    w = Ad @ x + b
    sx, sw = max(1.0, np.abs(x).max()), max(1.0, np.abs(b).max())
    assert x.min() >= 0.0
    assert w.min() >= -1e-10 * sw
    assert np.abs(x * w).max() <= 1e-10 * sx * sw


@pytest.fixture(scope="module")
def tiny_lcps(tiny_cases):
    out = []
    for seed, g, A in tiny_cases:
        pairs, gaps = dynamics.find_contacts(g.c, 1.0, 0.1)
        Aop, Ad = _dense_lcp(g, A, pairs)
        glo = bie.Geometry(g.c, 1.0, 4, 8)
        Alo_d = bie.dense_operator(glo)
        Alo = lcp.lcp_operator(lambda FT, glo=glo, Alo_d=Alo_d: bie.mobility_apply(glo, FT, dense=Alo_d), g.c, pairs)
        axes = -g.c / np.linalg.norm(g.c, axis=1)[:, None]
        b_real = lcp.lcp_b(gaps, 0.1, g.c, pairs, bie.nc_velocity(g, axes, 1.0, dense=A))
        xs, ws = inputs.planted_lcp(seed, pairs.shape[0])
        out.append(dict(seed=seed, Aop=Aop, Ad=Ad, Alo=Alo, b_real=b_real, x_pl=xs, b_pl=ws - Ad @ xs))
    return out


def test_lcp_matrix_positive_definite(tiny_lcps):
    for c in tiny_lcps:
        Ad = c['Ad']
        assert np.linalg.eigvalsh(0.5 * (Ad + Ad.T)).min() > 0.0
        assert np.linalg.norm(Ad - Ad.T) / np.linalg.norm(Ad) < 0.1


@pytest.mark.parametrize("solver", ["mono", "bb", "bi"])
def test_solvers_match_brute_force(tiny_lcps, solver):
    for c in tiny_lcps:
        for b, xref in ((c['b_real'], None), (c['b_pl'], c['x_pl'])):
            xbf = lcp.brute_force_lcp(c['Ad'], b)
            if xref is not None:
                assert np.abs(xbf - xref).max() < 1e-12
            kw = dict(tol_abs=1e-12, tol_rel=1e-15)
            if solver == 'mono':
                x, Ax, st = lcp.mono_pqn(c['Aop'], b, **kw)
            elif solver == 'bb':
                x, Ax, st = lcp.bb_pgd(c['Aop'], b, tau0=3 * np.pi, k_max=500, **kw)
            else:
                x, Ax, st = lcp.bi_pqn(c['Aop'], c['Alo'], b, **kw)
            assert st['converged']
            assert np.abs(x - xbf).max() <= 1e-10 * max(np.abs(xbf).max(), 1e-300)
            _check_complementarity(x, c['Ad'], b)
            # MVP reuse (Remark after Alg. 2): recurrence vs fresh product
            assert np.abs(Ax - c['Ad'] @ x).max() <= 1e-12 * max(1.0, np.abs(c['Ad'] @ x).max())


def test_mvp_counts_in_paper_range(tiny_lcps):
    """Soft check only (parity unpinned): Table 2's counts come from another discretisation."""
    soft = GOLD['paper_table2_mvps_soft']
    counts = []
    for c in tiny_lcps:
        _, _, sm = lcp.mono_pqn(c['Aop'], c['b_pl'])
        _, _, sb = lcp.bb_pgd(c['Aop'], c['b_pl'], tau0=3 * np.pi)
        counts.append((sm['mvp'], sb['mvp']))
    for m, bb in counts:
        assert m <= 3 * soft['mono_pqn_median'] and bb <= 5 * soft['bb_pgd_median']


def test_bi_pqn_with_exact_model_needs_few_high_fidelity_products(tiny_lcps):
    """Alg. 4 with the low-fidelity operator equal to A: each subproblem is the
    problem itself solved to 1e-2 of the current KKT error, so the high-fidelity
    products only confirm and polish (2-4 here), fewer than Mono-PQN needs."""
    for c in tiny_lcps:
        x, _, sb = lcp.bi_pqn(c['Aop'], c['Aop'], c['b_pl'])
        _, _, sm = lcp.mono_pqn(c['Aop'], c['b_pl'])
        assert np.abs(x - c['x_pl']).max() < 1e-7 * np.abs(c['x_pl']).max()
        assert sb['mvp_hi'] <= 4 and sb['mvp_hi'] < sm['mvp']


def test_bi_pqn_rejects_an_indefinite_model():
    """Model safeguard: with a low-fidelity matrix that has negative curvature, the
    subproblems of Alg. 4 are unbounded; the solve must notice (Alg. 2 edge case on
    the model), finish as Mono-PQN on A and still return the brute-force solution.
    With a positive definite model the safeguard stays silent."""
    rng = np.random.default_rng(7)
    n = 8
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(np.log(1e-2), np.log(1e-1), n))
    A = (Q * ev) @ Q.T
    Alo_bad = (Q * (ev * np.r_[1.0, -1.0, np.ones(n - 2)])) @ Q.T  # a direction the iterates explore
    Alo_good = (Q * (ev * np.exp(rng.uniform(-0.5, 0.5, n)))) @ Q.T
    xs, ws = inputs.planted_lcp(5, n)
    b = ws - A @ xs
    xbf = lcp.brute_force_lcp(A, b)
    assert np.abs(xbf - xs).max() < 1e-12
    kw = dict(tol_abs=1e-12, tol_rel=1e-15)
    x, _, st = lcp.bi_pqn(lambda v: A @ v, lambda v: Alo_bad @ v, b, **kw)
    assert st['fallback'] and st['converged']
    assert np.abs(x - xbf).max() < 1e-9 * np.abs(xbf).max()
    x2, _, st2 = lcp.bi_pqn(lambda v: A @ v, lambda v: Alo_good @ v, b, **kw)
    assert not st2['fallback'] and st2['converged']
    assert np.abs(x2 - xbf).max() < 1e-9 * np.abs(xbf).max()


def _counted(f, box, k):
    def g(v):
        box[k] += 1
        return f(v)
    return g


def test_bi_pqn_rec_with_two_fidelities_is_bi_pqn(tiny_lcps):
    """The recursion bottoms out in Alg. 4 itself: with two operators every iterate,
    KKT error and product count equals bi_pqn's."""
    for c in tiny_lcps:
        for b in (c['b_real'], c['b_pl']):
            x1, Ax1, s1 = lcp.bi_pqn(c['Aop'], c['Alo'], b, tol_abs=1e-12, tol_rel=1e-15)
            x2, Ax2, s2 = lcp.bi_pqn_rec([c['Aop'], c['Alo']], b, tol_abs=1e-12, tol_rel=1e-15)
            assert s1['hist'] == s2['hist']
            assert (s1['mvp_hi'], s1['mvp_lo']) == tuple(s2['mvp'])
            assert np.array_equal(x1, x2) and np.array_equal(Ax1, Ax2)


@pytest.fixture(scope="module")
def tiny_lcps3(tiny_lcps, tiny_cases):
    """tiny_lcps plus a middle fidelity (6x12 grid) between the 8x16 and 4x8 ones."""
    out = []
    for c, (seed, g, A) in zip(tiny_lcps, tiny_cases):
        pairs, _ = dynamics.find_contacts(g.c, 1.0, 0.1)
        gm = bie.Geometry(g.c, 1.0, 6, 12)
        Am = bie.dense_operator(gm)
        Amid = lcp.lcp_operator(lambda FT, gm=gm, Am=Am: bie.mobility_apply(gm, FT, dense=Am), g.c, pairs)
        out.append(dict(c, Amid=Amid))
    return out


def test_bi_pqn_rec_three_fidelities_match_brute_force(tiny_lcps3):
    """Three fidelities (8x16, 6x12, 4x8 grids): the solution is the LCP's (brute force over
    active sets), complementarity holds, A x carried by the recurrence equals a fresh
    product, and every fidelity is used; the counts are the operators' own call counts."""
    for c in tiny_lcps3:
        for b in (c['b_real'], c['b_pl']):
            box = [0, 0, 0]
            ops = [_counted(c['Aop'], box, 0), _counted(c['Amid'], box, 1), _counted(c['Alo'], box, 2)]
            x, Ax, st = lcp.bi_pqn_rec(ops, b, tol_abs=1e-12, tol_rel=1e-15)
            xbf = lcp.brute_force_lcp(c['Ad'], b)
            assert st['converged'] and not st['fallback']
            assert np.abs(x - xbf).max() <= 1e-10 * max(np.abs(xbf).max(), 1e-300)
            _check_complementarity(x, c['Ad'], b)
            assert np.abs(Ax - c['Ad'] @ x).max() <= 1e-12 * max(1.0, np.abs(c['Ad'] @ x).max())
            assert st['mvp'] == box
            if np.any(xbf > 0):
                assert min(box) >= 1


def test_bi_pqn_rec_with_exact_models_needs_few_high_fidelity_products(tiny_lcps):
    """All three fidelities equal A: the first subproblem is the LCP itself, so as with
    two exact fidelities the high-fidelity products only confirm and polish."""
    for c in tiny_lcps:
        x, _, st = lcp.bi_pqn_rec([c['Aop']] * 3, c['b_pl'], tol_abs=1e-10)
        assert np.abs(x - c['x_pl']).max() < 1e-8 * np.abs(c['x_pl']).max()
        assert st['mvp_hi'] <= 4


def test_bi_pqn_rec_safeguard_at_each_level():
    """An indefinite lowest model is caught inside the middle level (which finishes its
    subproblems as Mono-PQN on its own positive definite operator), so the top level keeps
    its model; an indefinite middle model makes the top level itself fall back. Both
    return the brute-force solution."""
    rng = np.random.default_rng(7)
    n = 8
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(np.log(1e-2), np.log(1e-1), n))
    A = (Q * ev) @ Q.T
    bad = (Q * (ev * np.r_[1.0, -1.0, np.ones(n - 2)])) @ Q.T
    good = (Q * (ev * np.exp(rng.uniform(-0.5, 0.5, n)))) @ Q.T
    good2 = (Q * (ev * np.exp(rng.uniform(-0.7, 0.7, n)))) @ Q.T
    xs, ws = inputs.planted_lcp(5, n)
    b = ws - A @ xs
    xbf = lcp.brute_force_lcp(A, b)
    kw = dict(tol_abs=1e-12, tol_rel=1e-15)
    mv = lambda M: (lambda v: M @ v)
    x, _, st = lcp.bi_pqn_rec([mv(A), mv(good), mv(bad)], b, **kw)
    assert st['converged'] and not st['fallback']
    assert np.abs(x - xbf).max() < 1e-9 * np.abs(xbf).max()
    x, _, st = lcp.bi_pqn_rec([mv(A), mv(bad), mv(good2)], b, **kw)
    assert st['converged'] and st['fallback']
    assert np.abs(x - xbf).max() < 1e-9 * np.abs(xbf).max()
    x, _, st = lcp.bi_pqn_rec([mv(A), mv(good), mv(good2)], b, **kw)
    assert st['converged'] and not st['fallback']
    assert np.abs(x - xbf).max() < 1e-9 * np.abs(xbf).max()


def test_solvers_from_an_initial_guess(tiny_lcps3):
    """x^(-1) given: every solver reaches the brute-force solution from a random guess
    (negative entries projected) and from the solution itself, where Mono-PQN and
    BB-PGD stop after the one product that evaluates A x^(-1) (Bi-PQN first moves to
    the low-fidelity solution, Alg. 4's x^(0)). Two-level recursion = bi_pqn also
    from a guess."""
    kw = dict(tol_abs=1e-12, tol_rel=1e-15)
    for c in tiny_lcps3:
        b = c['b_pl']
        xbf = lcp.brute_force_lcp(c['Ad'], b)
        g = np.random.default_rng(c['seed']).uniform(-0.5, 1.5, b.size)
        ops3 = [c['Aop'], c['Amid'], c['Alo']]
        runs = {
            'mono': lambda x0: lcp.mono_pqn(c['Aop'], b, x0=np.maximum(x0, 0.0), **kw),
            'bb': lambda x0: lcp.bb_pgd(c['Aop'], b, x0=np.maximum(x0, 0.0), tau0=3 * np.pi, k_max=500, **kw),
            'bi': lambda x0: lcp.bi_pqn(c['Aop'], c['Alo'], b, x0=x0, **kw),
            'birec': lambda x0: lcp.bi_pqn_rec(ops3, b, x0=x0, **kw),
        }
        for name, run in runs.items():
            x, _, st = run(g)
            assert st['converged'], name
            assert np.abs(x - xbf).max() <= 1e-10 * np.abs(xbf).max(), name
            x, _, st = run(xbf)
            if name in ('mono', 'bb'):
                assert st['mvp'] == 1, (name, st)
            assert st['converged'], name
            assert np.abs(x - xbf).max() <= 1e-10 * np.abs(xbf).max(), name
        x1, _, s1 = lcp.bi_pqn(c['Aop'], c['Alo'], b, x0=g, **kw)
        x2, _, s2 = lcp.bi_pqn_rec([c['Aop'], c['Alo']], b, x0=g, **kw)
        assert s1['hist'] == s2['hist'] and (s1['mvp_hi'], s1['mvp_lo']) == tuple(s2['mvp'])


@pytest.mark.parametrize("solver", ["mono", "bi", "birec"])
def test_printed_metric_matches_brute_force(tiny_lcps, solver):
    """Alg. 1 as printed (H^(0) = I at every start, no metric scale): the solvers still
    reach the brute-force solution, and the metric scale stays 1."""
    for c in tiny_lcps:
        b = c['b_pl']
        xbf = lcp.brute_force_lcp(c['Ad'], b)
        kw = dict(tol_abs=1e-12, tol_rel=1e-15, printed_metric=True)
        if solver == 'mono':
            x, _, st = lcp.mono_pqn(c['Aop'], b, k_max=300, **kw)
            assert st['sigma'] == 1.0
        elif solver == 'bi':
            x, _, st = lcp.bi_pqn(c['Aop'], c['Alo'], b, k_max=100, **kw)
        else:
            x, _, st = lcp.bi_pqn_rec([c['Aop'], c['Alo'], c['Alo']], b, k_max=100, **kw)
        assert st['converged']
        assert np.abs(x - xbf).max() <= 1e-10 * np.abs(xbf).max()
        _check_complementarity(x, c['Ad'], b)


def test_metric_scale_invariance():
    """The reading's metric (B0 = sigma I, sigma from the first step's curvature) makes
    Mono-PQN's iterates invariant to the units of A: under (A, b) -> (c A, c b) the
    solution is unchanged, H scales by 1/c and the gradient by c, so every search
    direction p (the vectors A is applied to) is the same for any c. Alg. 1 as printed
    (H^(0) = I) is not: from the second step on its BFGS matrix mixes I with c A. (The
    first direction is the projected gradient step in both forms, c times longer for c A;
    directions are compared after normalisation.)"""
    A = _spd(30, 7, kappa=20.0)
    xs, ws = inputs.planted_lcp(2, 30)
    b = ws - A @ xs
    dirs = {}
    for printed in (False, True):
        for c in (1.0, 1e-2, 1e2):
            seen = []

            def Aop(v, c=c, seen=seen):
                seen.append(np.array(v))
                return c * (A @ v)
            x, _, st = lcp.mono_pqn(Aop, c * b, tol_abs=1e-12 * c, tol_rel=1e-15, k_max=60,
                                    printed_metric=printed)
            if not printed:
                assert st['converged'] and np.abs(x - xs).max() < 1e-9
                assert np.isclose(st['sigma'], c * dirs.get((False, 1.0), (None, st['sigma'] / c))[1], rtol=1e-10)
            else:
                assert st['sigma'] == 1.0
            dirs[(printed, c)] = (seen, st['sigma'] / c)
    for printed in (False, True):
        ref = dirs[(printed, 1.0)][0]
        for c in (1e-2, 1e2):
            other = dirs[(printed, c)][0]
            k = min(len(ref), len(other), 8)
            unit = lambda v: v / np.linalg.norm(v)
            same = [np.abs(unit(ref[i]) - unit(other[i])).max() < 1e-9 for i in range(k)]
            assert same[0]                      # the first step uses H = I in both forms
            if printed:
                assert not all(same)
            else:
                assert all(same)
