"""GPU parity of the mobility product: HIP library (through the C ABI) vs oracle."""
import sys

import numpy as np
import pytest

from oracle import bie, dynamics, grid
from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def soa(q):
    return np.ascontiguousarray(q.T)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    w = inputs.workload('tiny', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, 8, 16)
    return c, g, bie.dense_operator(g)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_bie_apply_tiny(tiny, prec, tol):
    c, g, A = tiny
    say('bie_apply tiny', prec)
    q = np.random.default_rng(3).standard_normal((g.N, 3))
    with binding.Context(c, None, 8, 16, precision=prec) as ctx:
        y = ctx.bie_apply(soa(q))
    ref = (A @ q.ravel()).reshape(-1, 3).T
    assert rel(y, ref) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_mobility_tiny(tiny, prec, tol):
    c, g, A = tiny
    say('mobility tiny', prec)
    FT = inputs.random_forces(7, g.M)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-13, precision=prec, refine=0) as ctx:
        U, st = ctx.mobility_apply(FT)
    Uo = bie.mobility_apply(g, FT, dense=A)
    assert st['converged'] == 1
    assert rel(U[:, :3], Uo[:, :3]) < tol
    assert rel(U[:, 3:], Uo[:, 3:]) < tol


def test_mixed_refinement_reaches_fp64_operator(tiny):
    c, g, A = tiny
    FT = inputs.random_forces(8, g.M)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-12, precision='mixed', refine=3) as ctx:
        U, st = ctx.mobility_apply(FT)
    Uo = bie.mobility_apply(g, FT, dense=A)
    assert st['refine_sweeps'] >= 1
    assert rel(U, Uo) < 1e-9


@pytest.mark.parametrize("nt", [6, 12])
def test_single_sphere_drag(nt):
    say('drag', nt)
    FT = np.array([[1.0, -2.0, 0.5, 0.3, 0.7, -0.2]])
    with binding.Context([[0.5, 0.0, -1.0]], None, nt, 2 * nt, radius=1.5, mu=2.0, gmres_tol=1e-13) as ctx:
        U, _ = ctx.mobility_apply(FT)
    assert np.abs(U[0, :3] * 6 * np.pi * 2.0 * 1.5 - FT[0, :3]).max() < 1e-10
    assert np.abs(U[0, 3:] * 8 * np.pi * 2.0 * 1.5 ** 3 - FT[0, 3:]).max() < 1e-10


def test_nc_velocity_tiny(tiny):
    c, g, A = tiny
    axes = inputs.janus_axes(4, g.M)
    with binding.Context(c, axes, 8, 16, gmres_tol=1e-13) as ctx:
        U, _ = ctx.nc_velocity()
    Uo = bie.nc_velocity(g, axes, 1.0, dense=A)
    assert rel(U, Uo) < 1e-10


def test_zero_forces_give_zero_velocity(tiny):
    c, g, A = tiny
    with binding.Context(c, None, 8, 16) as ctx:
        U, st = ctx.mobility_apply(np.zeros((g.M, 6)))
    assert np.all(U == 0.0) and st['gmres_iters'] == 0


def test_contacts_match_oracle():
    for seed in range(3):
        c = inputs.workload('tiny', seed)['centers']
        with binding.Context(c, None, 4, 8) as ctx:
            pairs, gaps = ctx.find_contacts(0.1)
            none, _ = ctx.find_contacts(-1.0)
        po, go = dynamics.find_contacts(c, 1.0, 0.1)
        assert np.array_equal(pairs, po) and np.abs(gaps - go).max() < 1e-14
        assert none.shape[0] == 0


def _sample_targets(g, k, seed):
    rng = np.random.default_rng(seed)
    t = set(rng.choice(g.N, size=k, replace=False).tolist())
    t.update([0, g.n - 1, g.N - 1])        # first, last of the first sphere, last overall
    return sorted(t)


@pytest.mark.parametrize("name,prec,tol", [("lattice27", "fp64", 1e-12), ("lattice27", "mixed", 1e-6),
                                           ("rsa216", "fp64", 1e-12), ("rsa216", "mixed", 1e-6)])
def test_bie_apply_sampled_rows(name, prec, tol):
    w = inputs.workload(name, 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, w['n_theta'], w['n_phi'])
    say('bie_apply rows', name, prec, 'N', g.N)
    q = np.random.default_rng(11).standard_normal((g.N, 3))
    with binding.Context(c, None, w['n_theta'], w['n_phi'], precision=prec) as ctx:
        y = ctx.bie_apply(soa(q))
    tg = _sample_targets(g, 12, 5)
    ref = bie.operator_rows(g, q, tg)
    scale = np.abs(ref).max()
    assert np.abs(y[:, tg].T - ref).max() < tol * scale


def test_bie_solve_residual_rsa216():
    """Full-size property: the GPU density solves the oracle's equation at sampled rows."""
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, w['n_theta'], w['n_phi'])
    rhs = -bie.completion(g, inputs.random_forces(2, g.M))
    tg = _sample_targets(g, 8, 6)
    for prec, tol in (("fp64", 1e-9), ("mixed", 2e-6)):
        say('bie_solve rsa216', prec)
        with binding.Context(c, None, w['n_theta'], w['n_phi'], gmres_tol=1e-10, precision=prec) as ctx:
            q, st = ctx.bie_solve(soa(rhs))
        res = bie.operator_rows(g, q.T, tg) - rhs[tg]
        assert np.abs(res).max() < tol * np.abs(rhs).max(), (prec, st)


def test_mixed_vs_fp64_mobility_rsa216():
    w = inputs.workload('rsa216', 0)
    c = w['centers']
    FT = inputs.random_forces(3, c.shape[0])
    out = {}
    for prec in ('fp64', 'mixed'):
        say('mobility rsa216', prec)
        with binding.Context(c, None, w['n_theta'], w['n_phi'], gmres_tol=1e-10, precision=prec) as ctx:
            out[prec], st = ctx.mobility_apply(FT)
    for blk in (slice(0, 3), slice(3, 6)):
        assert rel(out['mixed'][:, blk], out['fp64'][:, blk]) < 1e-6


def test_set_state_without_axes_keeps_janus_axes(tiny):
    """Re-setting only the centres keeps the context's Janus axes (and hence U_nc)."""
    c, g, A = tiny
    axes = inputs.janus_axes(9, g.M)
    c2 = c + 0.01
    with binding.Context(c, axes, 8, 16, gmres_tol=1e-12) as ctx, \
            binding.Context(c2, axes, 8, 16, gmres_tol=1e-12) as ref:
        ctx.set_state(c2)
        _, ax = ctx.get_state()
        assert np.array_equal(ax, axes)
        U, _ = ctx.nc_velocity()
        Ur, _ = ref.nc_velocity()
    assert rel(U, Ur) < 1e-12


def test_precision_sweep_packing64():
    """64 spheres compressed to volume fraction 0.35 (16x32 grid): the mixed path against
    the FP64 path, per velocity block, for random forces and for contact forces D x, and
    for the solution of a planted LCP on the packing's contact set."""
    from oracle import lcp
    w = inputs.workload('packing64', 0)
    c = w['centers']
    M = c.shape[0]
    kw = dict(gmres_tol=1e-10)
    with binding.Context(c, None, 16, 32, precision='fp64', **kw) as c64, \
            binding.Context(c, None, 16, 32, precision='mixed', **kw) as cmx:
        pairs, _ = c64.find_contacts(0.1)
        say('packing64 contacts', pairs.shape[0])
        assert pairs.shape[0] >= 10
        x = np.abs(np.random.default_rng(30).standard_normal(pairs.shape[0]))
        for name, FT in (('random', inputs.random_forces(31, M)), ('contact', lcp.D_apply(c, pairs, x))):
            U64, _ = c64.mobility_apply(FT)
            Umx, _ = cmx.mobility_apply(FT)
            for blk in (slice(0, 3), slice(3, 6)):
                e = rel(Umx[:, blk], U64[:, blk])
                say('  ', name, blk, e)
                assert e < 1e-6
        xs, ws = inputs.planted_lcp(3, pairs.shape[0])
        b = ws - c64.lcp_apply(pairs, xs)
        x64, s64 = c64.lcp_solve(pairs, b, 'mono', tol_abs=1e-11, tol_rel=1e-14)
        xmx, smx = cmx.lcp_solve(pairs, b, 'mono', tol_abs=1e-9, tol_rel=1e-9)
        w64 = c64.lcp_apply(pairs, x64) + b
    say('  lcp', s64['mvp_hi'], smx['mvp_hi'], np.abs(xmx - x64).max() / np.abs(x64).max())
    # At gaps down to 0.01 the discrete A of this packing need not be a P-matrix, so the
    # planted x* need not be the only solution: check that x64 is one (complementarity),
    # and that the mixed path finds the same one.
    sw = max(1.0, np.abs(b).max())
    assert x64.min() >= 0.0 and w64.min() >= -1e-9 * sw
    assert np.abs(x64 * w64).max() <= 1e-9 * max(1.0, np.abs(x64).max()) * sw
    assert np.abs(xmx - x64).max() < 1e-6 * np.abs(x64).max()


@pytest.mark.parametrize("nt", [6, 12])
def test_grid_and_self_block_of_device_context(nt):
    """a1/a2: the context's grid and singular self block are the oracle's."""
    say('grid/self block', nt)
    with binding.Context([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]], None, nt, 2 * nt, radius=1.0) as ctx:
        off, w = ctx.get_grid()
        S = ctx.get_self_block()
    o2, _, w2 = grid.sphere_grid(nt, 2 * nt, 1.0)
    assert np.abs(off - o2).max() < 1e-14 and np.abs(w - w2).max() < 1e-14
    So = bie.self_block(nt, 2 * nt, 1.0).reshape(3 * nt * 2 * nt, -1)
    # both sides sum the rotated-pole rule's ~10^4 terms per entry in FP64, in different orders
    assert np.abs(S - So).max() <= 5e-12 * np.abs(So).max()


@pytest.mark.parametrize("nt", [5, 8, 12])
def test_single_sphere_operator_matches_oracle(nt):
    """The self block applied on the device through harmonic coefficients (T q, G coef),
    plus 1/2 q and the rigid projection, for one sphere (odd and even grids)."""
    say('single sphere operator', nt)
    c = [[0.3, -0.2, 0.1]]
    g = bie.Geometry(c, 1.0, nt, 2 * nt)
    A = bie.dense_operator(g)
    q = np.random.default_rng(nt).standard_normal((g.N, 3))
    with binding.Context(c, None, nt, 2 * nt) as ctx:
        y = ctx.bie_apply(soa(q))
    ref = (A @ q.ravel()).reshape(-1, 3).T
    assert rel(y, ref) < 1e-12


def test_mobility_apply_dev_matches_host(tiny):
    import torch
    c, g, A = tiny
    FT = inputs.random_forces(12, g.M)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-12) as ctx:
        U, _ = ctx.mobility_apply(FT)
        FTd = torch.as_tensor(FT, dtype=torch.float64, device='cuda:0').contiguous()
        UOd = torch.full((g.M, 6), float('nan'), dtype=torch.float64, device='cuda:0')
        st = ctx.mobility_apply_dev(FTd.data_ptr(), UOd.data_ptr())
        Ud = UOd.cpu().numpy()
    assert st['converged'] == 1
    assert np.array_equal(U, Ud)


def test_profile_stage_times(tiny):
    """profile = 1: every operator stage is timed with HIP events on one stream; the
    stage times are positive and add up to less than the call's wall time."""
    c, g, A = tiny
    F = inputs.random_forces(7, g.M, k=2)
    with binding.Context(c, None, 8, 16, gmres_tol=1e-10, profile=True, side_stream=True) as ctx:
        U, st = ctx.mobility_apply_multi(F)
        U1, _ = ctx.mobility_apply(F[0])
    stages = [st[k] for k in ('t_far_ms', 't_near_ms', 't_gemm_ms', 't_local_ms', 't_arnoldi_ms')]
    say('stage ms', stages, 'total', st['t_total_ms'])
    assert min(stages) > 0.0
    assert sum(stages) < st['t_total_ms']
    assert rel(U[0], U1) < 1e-9


def test_near_upsampling_factor_matches_oracle():
    """The near rule upsampled 3x per direction (used for time steps whose gaps close
    below the 2x rule's reach): the operator equals the oracle's matrix-free operator
    with the same upsampling, and the 1x1 LCP matrix of a pair at gap 3e-4 on the 8x16
    grid, negative with 2x upsampling, is positive and equals the oracle's."""
    up = 3
    w = inputs.workload('tiny', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, 8, 16, near_up=up)
    q = np.random.default_rng(5).standard_normal((g.N, 3))
    with binding.Context(c, None, 8, 16, near_up=up) as ctx:
        y = ctx.bie_apply(soa(q))
    assert rel(y, bie.operator_apply(g, q).reshape(-1, 3).T) < 1e-12
    d = np.ones(3) / np.sqrt(3.0)
    cp = np.array([np.zeros(3), (2.0 + 3e-4) * d])
    gp = bie.Geometry(cp, 1.0, 8, 16, near_up=up)
    Ap = bie.dense_operator(gp)
    F = np.zeros((2, 6))
    F[0, :3], F[1, :3] = -d, d  # unit push apart along the line of centres
    U = bie.mobility_apply(gp, F, dense=Ap)
    a_ref = float(d @ (U[1, :3] - U[0, :3]))
    with binding.Context(cp, None, 8, 16, gmres_tol=1e-13, near_up=up) as ctx:
        pairs, _ = ctx.find_contacts(0.1)
        a = ctx.lcp_apply(pairs, np.ones(1))[0]
    say('near_up', up, 'pair A', a, 'oracle', a_ref)
    assert a > 0.0 and abs(a - a_ref) < 1e-9 * abs(a_ref)


CLOSE = dict(near_close_gap=0.05, near_close_up=3)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_close_pair_class_matches_oracle(prec, tol):
    """Near pairs closer than near_close_gap on the finer grid: on the 8-sphere cluster
    (gaps 0.01-0.1) some pairs fall below 0.05; the operator equals the oracle's with the
    same two classes, and differs from the single-class operator."""
    w = inputs.workload('tiny', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, 8, 16, **CLOSE)
    nclose = sum(1 for i in range(g.M) for j in range(g.M)
                 if i != j and np.linalg.norm(c[i] - c[j]) - 2.0 < 0.05)
    assert nclose > 0
    q = np.random.default_rng(6).standard_normal((g.N, 3))
    with binding.Context(c, None, 8, 16, precision=prec, **CLOSE) as ctx:
        y = ctx.bie_apply(soa(q))
    ref = bie.operator_apply(g, q).reshape(-1, 3).T
    say('close class', prec, nclose, 'ordered close pairs, rel err', rel(y, ref))
    assert rel(y, ref) < tol
    assert rel(bie.operator_apply(bie.Geometry(c, 1.0, 8, 16), q).reshape(-1, 3).T, ref) > 1e-6


def test_close_pair_class_in_batch_and_graph_paths():
    """The batch context's segmented launches and the graph-replayed single-system
    iterations run the close pairs too: same velocities as the eager single context."""
    w = inputs.workload('tiny', 0)
    c = w['centers']
    F = inputs.random_forces(9, c.shape[0])
    kw = dict(gmres_tol=1e-12, **CLOSE)
    with binding.Context(c, None, 8, 16, **kw) as ctx:
        U, _ = ctx.mobility_apply(F)
    with binding.Context(c, None, 8, 16, graphs=True, **kw) as ctx:
        Ug, _ = ctx.mobility_apply(F)
    c2 = c + np.array([0.3, -0.2, 0.1])
    with binding.BatchContext([(c, 8, 16), (c2, 8, 16)], **kw) as bc:
        Ub, _ = bc.mobility_apply([F, F])
    assert rel(Ug, U) < 1e-12
    assert rel(Ub[0], U) < 1e-11 and rel(Ub[1], U) < 1e-11   # a translated copy moves the same way
