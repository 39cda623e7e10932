"""Pins of the oracle's time step (contacts, forward Euler of the linearised DVI)."""
import numpy as np

from oracle import bie, dynamics, lcp
from paper_2604_10089_amd import inputs


def test_contact_forces_balance():
    c = inputs.workload('tiny', 1)['centers']
    pairs, _ = dynamics.find_contacts(c, 1.0, 0.1)
    x = np.random.default_rng(0).uniform(0, 2, pairs.shape[0])
    FT = lcp.D_apply(c, pairs, x)
    assert np.abs(FT[:, :3].sum(axis=0)).max() < 1e-13
    # torque about the origin also balances: forces act along the line of centres
    tq = np.cross(c, FT[:, :3]).sum(axis=0)
    assert np.abs(tq).max() < 1e-12


def test_contacts_match_brute_distance():
    c = inputs.workload('tiny', 2)['centers']
    pairs, gaps = dynamics.find_contacts(c, 1.0, 0.1)
    for (i, j), gp in zip(pairs, gaps):
        assert i < j and abs(np.linalg.norm(c[i] - c[j]) - 2.0 - gp) < 1e-14 and gp <= 0.1
    assert pairs.shape[0] == inputs.count_close(c, 0.1)


def test_single_sphere_step_moves_by_swim_velocity():
    e = np.array([[0.0, 0.6, 0.8]])
    c1, ax1, info = dynamics.step(np.zeros((1, 3)), e, 1.0, (8, 16), (4, 8), 0.01, 0.1, 1.0)
    assert np.abs(c1[0] - 0.01 * e[0] / 3.0).max() < 1e-12
    assert abs(np.linalg.norm(ax1[0]) - 1.0) < 1e-14


def test_step_linearised_gaps_feasible():
    for seed in (0, 2):
        c = inputs.workload('tiny', seed)['centers']
        axes = -c / np.linalg.norm(c, axis=1)[:, None]
        for solver in ('mono', 'bi', 'bb'):
            c1, ax1, info = dynamics.step(c, axes, 1.0, (8, 16), (4, 8), 0.1, 0.1, 1.0,
                                          solver=solver, lcp_opts=dict(tol_abs=1e-12, tol_rel=1e-15))
            pairs, gaps = info['pairs'], info['gaps']
            lin = gaps + 0.1 * lcp.DT_apply(c, pairs, info['U'])
            assert lin.min() >= -1e-10
            x = info['x']
            assert np.abs(x * lin).max() <= 1e-9
