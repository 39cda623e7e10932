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


# Orientation update (the Sec. 3 footnote: the orientation is advanced with the angular
# velocity; for an axisymmetric Janus sphere only its axis matters): closed-form rotations.

def test_rotate_axes_quarter_turns_follow_the_right_hand_rule():
    ex, ey, ez = np.eye(3)
    th = 0.37
    out = dynamics.rotate_axes([ex, ey, ez, ex], np.array([[0, 0, 2.0], [3.0, 0, 0], [0, 0.5, 0], [0, 0, -2.0]]),
                               th / 2.0)
    assert np.abs(out[0] - [np.cos(th), np.sin(th), 0.0]).max() < 1e-15       # x about +z by th
    assert np.abs(out[1] - [0.0, np.cos(1.5 * th), np.sin(1.5 * th)]).max() < 1e-15  # y about +x by 1.5 th
    assert np.abs(out[2] - [np.sin(th / 4), 0.0, np.cos(th / 4)]).max() < 1e-15  # z about +y by th/4
    assert np.abs(out[3] - [np.cos(th), -np.sin(th), 0.0]).max() < 1e-15      # x about -z by th
    q = dynamics.rotate_axes([ey], np.array([[np.pi / 2, 0, 0]]), 1.0)[0]      # y about x by pi/2 -> z
    assert np.abs(q - ez).max() < 1e-15


def test_rotate_axes_special_cases_and_composition():
    rng = np.random.default_rng(4)
    e = rng.standard_normal((5, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    w = rng.standard_normal((5, 3))
    assert np.array_equal(dynamics.rotate_axes(e, np.zeros((5, 3)), 0.3), e)     # Omega = 0
    par = dynamics.rotate_axes(e, 2.5 * e, 0.3)                                   # about the axis itself
    assert np.abs(par - e).max() < 1e-15
    two = dynamics.rotate_axes(dynamics.rotate_axes(e, w, 0.11), w, 0.29)         # same Omega: angles add
    assert np.abs(two - dynamics.rotate_axes(e, w, 0.4)).max() < 1e-14
    back = dynamics.rotate_axes(dynamics.rotate_axes(e, w, 0.4), -w, 0.4)         # and undo each other
    assert np.abs(back - e).max() < 1e-14
    # any Omega: the rotation by the vector Omega dt, as scipy's Rotation applies it
    from scipy.spatial.transform import Rotation
    ref = np.array([Rotation.from_rotvec(0.7 * w[i]).apply(e[i]) for i in range(5)])
    assert np.abs(dynamics.rotate_axes(e, w, 0.7) - ref).max() < 1e-14
    # the angle between the axis and Omega is kept; the axis turns by |Omega| dt about Omega
    new = dynamics.rotate_axes(e, w, 0.7)
    k = w / np.linalg.norm(w, axis=1)[:, None]
    assert np.abs(np.einsum('ij,ij->i', new, k) - np.einsum('ij,ij->i', e, k)).max() < 1e-14
    pe = e - np.einsum('ij,ij->i', e, k)[:, None] * k
    pn = new - np.einsum('ij,ij->i', new, k)[:, None] * k
    ang = np.arctan2(np.einsum('ij,ij->i', k, np.cross(pe, pn)), np.einsum('ij,ij->i', pe, pn))
    assert np.abs(ang - 0.7 * np.linalg.norm(w, axis=1)).max() < 1e-13
