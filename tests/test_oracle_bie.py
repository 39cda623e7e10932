"""Pins of the oracle's discrete mobility operator (BIE, self block, MVP)."""
import json
import os

import numpy as np
import pytest

from oracle import bie, grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'closed_forms.json')))


def _band_limited_field(nt, seed, p=None):
    """Random vector field whose Cartesian components are harmonics of degree <= p."""
    p = nt - 1 if p is None else p
    rng = np.random.default_rng(seed)
    th, ph = grid.grid_angles(nt, 2 * nt)
    Y = grid.real_sh(p, th, ph)
    C = rng.standard_normal((Y.shape[1], 3))
    return Y @ C, C, p


def test_double_layer_of_constant_inside_and_outside():
    o, n, w = grid.sphere_grid(16, 32, 1.0)
    c = np.array([1.0, -2.0, 0.5])
    inside = bie.dl_apply(np.zeros((1, 3)), o, n, np.tile(c, (o.shape[0], 1)) * w[:, None])
    assert np.abs(inside[0] + c).max() < 1e-13
    outside = bie.dl_apply(np.array([[3.0, 0.4, -0.2]]), o, n, np.tile(c, (o.shape[0], 1)) * w[:, None])
    assert np.abs(outside).max() < 1e-10


@pytest.mark.parametrize("nt", [6, 8])
def test_self_block_maps_rigid_motions_to_minus_half(nt):
    g = bie.Geometry([[0, 0, 0]], 1.0, nt, 2 * nt)
    S = bie.self_block_nodemajor(bie.self_block(nt, 2 * nt, 1.0))
    rng = np.random.default_rng(nt)
    for q in (np.tile(rng.standard_normal(3), (g.n, 1)), np.cross(rng.standard_normal(3), g.o)):
        assert np.abs(S @ q.ravel() + 0.5 * q.ravel()).max() < 1e-12


def test_self_block_rotation_equivariant():
    nt = 6
    nph = 2 * nt
    S = bie.self_block_nodemajor(bie.self_block(nt, nph, 1.0))
    q, _, _ = _band_limited_field(nt, 1)
    ang = 2 * np.pi / nph
    R = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
    qr = np.roll(q.reshape(nt, nph, 3), 1, axis=1) @ R.T      # node (k, l+1) <- R q(k, l)
    lhs = S @ qr.ravel()
    rhs = np.roll((S @ q.ravel()).reshape(nt, nph, 3), 1, axis=1) @ R.T
    assert np.abs(lhs - rhs.ravel()).max() < 1e-12


def test_self_block_rule_is_converged():
    nt = 6
    q, _, _ = _band_limited_field(nt, 2)
    S2 = bie.self_block_nodemajor(bie.self_block(nt, 2 * nt, 1.0))
    S3 = bie.self_block_nodemajor(bie.self_block(nt, 2 * nt, 1.0, theta_factor=5, phi_factor=3))
    assert np.abs((S2 - S3) @ q.ravel()).max() < 1e-11 * np.abs(q).max()


def test_self_block_against_subtraction_on_fine_grid():
    """Independent singular rule: D_PV[q](x0) = sum_y w K (q_y - q(x0)) - q(x0)/2 on a fine grid.

    The subtracted integrand is bounded, so the plain fine-grid rule converges
    (slowly); the bound is loose but catches sign, index and scaling errors.
    """
    nt = 6
    q, C, p = _band_limited_field(nt, 3, p=3)
    S = bie.self_block_nodemajor(bie.self_block(nt, 2 * nt, 1.0))
    Sq = (S @ q.ravel()).reshape(-1, 3)
    o, _, _ = grid.sphere_grid(nt, 2 * nt, 1.0)
    nf = 96
    of, nrf, wf = grid.sphere_grid(nf, 2 * nf, 1.0)
    thf, phf = grid.grid_angles(nf, 2 * nf)
    qf = grid.real_sh(p, thf, phf) @ C
    for i in (0, 7, 20, 40):
        K = bie.dl_kernel(o[i:i + 1], of, nrf)[0] * wf[:, None, None]
        ref = np.einsum('fcd,fd->c', K, qf - q[i]) - 0.5 * q[i]
        assert np.abs(ref - Sq[i]).max() < 2e-2 * np.abs(q).max()


@pytest.mark.parametrize("nt", [6, 8])
def test_single_sphere_stokes_drag(nt):
    g = bie.Geometry([[0.3, -0.2, 1.0]], 1.3, nt, 2 * nt, mu=0.7)
    FT = np.array([[1.0, 2.0, -0.5, 0.3, 0.1, -0.4]])
    for dense in (bie.dense_operator(g), None):
        U = bie.mobility_apply(g, FT, dense=dense)
        ct = GOLD['stokes_drag_translation']['value'] * np.pi * g.mu * g.a
        cr = GOLD['stokes_drag_rotation']['value'] * np.pi * g.mu * g.a ** 3
        assert np.abs(U[0, :3] * ct - FT[0, :3]).max() < 1e-10
        assert np.abs(U[0, 3:] * cr - FT[0, 3:]).max() < 1e-10


def test_squirmer_speed():
    g = bie.Geometry([[0, 0, 0]], 1.0, 8, 16)
    e = np.array([0.3, -0.5, 0.8])
    e /= np.linalg.norm(e)
    n = g.normals
    B1 = 1.7
    us = -B1 * (e[None, :] - (n @ e)[:, None] * n)
    q = bie.solve_density(g, us, dense=bie.dense_operator(g))
    UO = bie.rigid_velocity(g, q)
    assert np.abs(UO[0, :3] - GOLD['squirmer_B1_speed']['value'] * B1 * e).max() < 1e-12
    assert np.abs(UO[0, 3:]).max() < 1e-12


def test_janus_half_cap_speed():
    g = bie.Geometry([[0, 0, 0]], 1.0, 12, 24)
    e = np.array([0.6, 0.0, -0.8])
    UO = bie.nc_velocity(g, [e], 1.0, dense=bie.dense_operator(g))
    assert abs(UO[0, :3] @ e - GOLD['janus_half_cap_speed']['value']) < 1e-10
    # the cap edge is not resolved by the grid: rotation vanishes only to O(grid)
    assert np.abs(UO[0, 3:]).max() < 2e-2


def test_two_sphere_far_field():
    ff = GOLD['two_sphere_far_field']
    for d in (6.0, 10.0):
        g = bie.Geometry([[0, 0, 0], [d, 0, 0]], 1.0, 8, 16)
        A = bie.dense_operator(g)
        U = bie.mobility_apply(g, np.array([[1.0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0]]), dense=A) * 6 * np.pi
        V = bie.mobility_apply(g, np.array([[0, 1.0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0]]), dense=A) * 6 * np.pi
        sa = ff['self_along']['c0'] + ff['self_along']['c4'] / d ** 4
        ca = ff['cross_along']['c1'] / d + ff['cross_along']['c3'] / d ** 3
        sx = ff['self_across']['c0'] + ff['self_across']['c6'] / d ** 6
        cx = ff['cross_across']['c1'] / d + ff['cross_across']['c3'] / d ** 3
        assert abs(U[0, 0] - sa) * d ** 6 < 10.0
        assert abs(U[1, 0] - ca) * d ** 7 < 30.0
        assert abs(V[0, 1] - sx) * d ** 8 < 50.0
        assert abs(V[1, 1] - cx) * d ** 7 < 30.0


def test_matrix_free_equals_dense(tiny_cases):
    seed, g, A = tiny_cases[0]
    q = np.random.default_rng(5).standard_normal((g.N, 3))
    assert np.abs(bie.operator_apply(g, q).ravel() - A @ q.ravel()).max() < 1e-12


def test_gmres_equals_dense_solve(tiny_cases):
    seed, g, A = tiny_cases[0]
    FT = np.random.default_rng(6).standard_normal((g.M, 6))
    U1 = bie.mobility_apply(g, FT, dense=A)
    U2 = bie.mobility_apply(g, FT, dense=None, tol=1e-13)
    assert np.abs(U1 - U2).max() < 1e-12 * np.abs(U1).max()


def test_mobility_nearly_symmetric_and_positive(tiny_cases):
    for seed, g, A in tiny_cases:
        Ainv = np.linalg.inv(A)
        M6 = np.zeros((6 * g.M, 6 * g.M))
        for k in range(6 * g.M):
            FT = np.zeros(6 * g.M)
            FT[k] = 1.0
            M6[:, k] = bie.rigid_velocity(g, (Ainv @ (-bie.completion(g, FT)).ravel()).reshape(-1, 3)).ravel()
        asym = np.linalg.norm(M6 - M6.T) / np.linalg.norm(M6)
        assert asym < 5e-2
        assert np.linalg.eigvalsh(0.5 * (M6 + M6.T)).min() > 0.0


def test_operator_rows_equal_full_apply(tiny_cases):
    seed, g, A = tiny_cases[1]
    q = np.random.default_rng(9).standard_normal((g.N, 3))
    full = (A @ q.ravel()).reshape(-1, 3)
    tg = [0, 5, 127, 128, 700, g.N - 1]
    assert np.abs(bie.operator_rows(g, q, tg) - full[tg]).max() < 1e-12 * np.abs(full).max()


def test_close_pairs_take_the_finer_near_rule():
    """Near pairs closer than near_close_gap use the near_close_up grid, the others
    near_up: each block equals the block of a geometry that uses that one factor for
    every near pair, and the close class moves only the close pair's block."""
    d = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    e = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    c = np.array([np.zeros(3), (2.0 + 3e-4) * d, (2.0 + 0.1) * e])   # one close, one near pair
    g = bie.Geometry(c, 1.0, 8, 16, near_close_gap=0.01, near_close_up=3)
    g2 = bie.Geometry(c, 1.0, 8, 16, near_up=2)
    g3 = bie.Geometry(c, 1.0, 8, 16, near_up=3)
    assert g.pair_up(0, 1) == g.pair_up(1, 0) == 3 and g.pair_up(0, 2) == 2
    assert np.array_equal(bie.near_block(g, 0, 1), bie.near_block(g3, 0, 1))
    assert np.array_equal(bie.near_block(g, 1, 0), bie.near_block(g3, 1, 0))
    assert np.array_equal(bie.near_block(g, 0, 2), bie.near_block(g2, 0, 2))
    assert np.abs(bie.near_block(g3, 0, 1) - bie.near_block(g2, 0, 1)).max() > 1e-3
    assert np.array_equal(bie.near_row(g, 0, 1, 5), bie.near_block(g3, 0, 1)[5])


def test_close_class_restores_a_positive_pair_mobility():
    """Two spheres at gap 3e-4 on the 8x16 grid, line of centres oblique to the pole:
    with the 2x near rule the relative mobility along the line of centres (the 1x1
    contact matrix) is negative; with the 3x rule for the close pair it is positive."""
    d = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    c = np.array([np.zeros(3), (2.0 + 3e-4) * d])
    F = np.zeros((2, 6))
    F[0, :3], F[1, :3] = -d, d
    vals = {}
    for name, kw in (('2x', {}), ('close 3x', dict(near_close_gap=0.01, near_close_up=3))):
        g = bie.Geometry(c, 1.0, 8, 16, **kw)
        U = bie.mobility_apply(g, F, dense=bie.dense_operator(g))
        vals[name] = float(d @ (U[1, :3] - U[0, :3]))
    assert vals['2x'] < 0.0 < vals['close 3x']
