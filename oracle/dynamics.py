"""Contact detection and one forward-Euler DVI step (oracle, FP64).

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import bie, lcp


def find_contacts(centers, radius, delta):
    """Candidate set A = {pairs with gap Phi_l <= delta} (eq. (collisional-set)).

    Pairs (i, j) with i < j in lexicographic order; gap = |c_i - c_j| - 2a.
    """
    c = np.asarray(centers, dtype=np.float64)
    pairs, gaps = [], []
    for i in range(c.shape[0]):
        for j in range(i + 1, c.shape[0]):
            g = np.linalg.norm(c[i] - c[j]) - 2.0 * radius
            if g <= delta:
                pairs.append((i, j))
                gaps.append(g)
    return np.array(pairs, dtype=np.int64).reshape(-1, 2), np.array(gaps)


def rotate_axes(axes, omega, dt):
    """Rotate each unit axis by angle |Omega| dt about Omega (Rodrigues' formula).

    The paper tracks orientation (with a quaternion, Sec. 3 footnote); for the
    axisymmetric Janus sphere only the axis matters.
    Pinned by: closed-form rotations about the coordinate axes (right-hand rule),
    Omega = 0 and Omega along the axis, composition and inversion, scipy's rotation
    by the vector Omega dt (tests/test_oracle_step.py).
    """
    out = np.array(axes, dtype=np.float64)
    for i in range(out.shape[0]):
        w = omega[i]
        th = np.linalg.norm(w) * dt
        if th == 0.0:
            continue
        k = w / np.linalg.norm(w)
        e = out[i]
        out[i] = e * np.cos(th) + np.cross(k, e) * np.sin(th) + k * (k @ e) * (1.0 - np.cos(th))
    return out


def step(centers, axes, radius, grid_hi, grid_lo, dt, delta, slip, solver='mono',
         tol_gmres=1e-13, lcp_opts=None, mu=1.0, near=None):
    """One step C <- C + dt (G U_nc + G M D x) with the LCP of eq. (LCP) (eq. (dvi)).

    Contacts at the current configuration, U_nc from the slip-driven solve,
    b = Phi/dt + D^T U_nc, x from the chosen solver, then the Euler update of
    centres and Janus axes. Dense operators are used (small suspensions).
    Returns (centers, axes, info). near: keyword arguments of the geometries'
    near rule (near_gap, near_up, near_close_gap, near_close_up).
    """
    lcp_opts = {} if lcp_opts is None else dict(lcp_opts)
    near = {} if near is None else dict(near)
    g_hi = bie.Geometry(centers, radius, grid_hi[0], grid_hi[1], mu, **near)
    A_hi = bie.dense_operator(g_hi)
    mob_hi = lambda FT: bie.mobility_apply(g_hi, FT, dense=A_hi)
    pairs, gaps = find_contacts(centers, radius, delta)
    U_nc = bie.nc_velocity(g_hi, axes, slip, dense=A_hi)
    info = {'pairs': pairs, 'gaps': gaps, 'U_nc': U_nc}
    if pairs.shape[0] > 0:
        b = lcp.lcp_b(gaps, dt, centers, pairs, U_nc)
        Aop = lcp.lcp_operator(mob_hi, centers, pairs)
        if solver == 'bi':
            g_lo = bie.Geometry(centers, radius, grid_lo[0], grid_lo[1], mu, **near)
            A_lo = bie.dense_operator(g_lo)
            Alo = lcp.lcp_operator(lambda FT: bie.mobility_apply(g_lo, FT, dense=A_lo), centers, pairs)
            x, _, st = lcp.bi_pqn(Aop, Alo, b, **lcp_opts)
        elif solver == 'bb':
            x, _, st = lcp.bb_pgd(Aop, b, tau0=3.0 * np.pi * mu * radius, **lcp_opts)
        else:
            x, _, st = lcp.mono_pqn(Aop, b, **lcp_opts)
        U = U_nc + mob_hi(lcp.D_apply(centers, pairs, x))
        info.update(b=b, x=x, stats=st)
    else:
        U = U_nc
    info['U'] = U
    c_new = np.asarray(centers, dtype=np.float64) + dt * U[:, :3]
    ax_new = rotate_axes(axes, U[:, 3:], dt)
    return c_new, ax_new, info
