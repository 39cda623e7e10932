"""Sphere surface grids and spherical-harmonic projection (oracle, FP64).

Test infrastructure only (see the package docstring).

The paper represents each particle's surface density with order-p spherical
harmonics (Sec. 5.1, "coarseness of discretization"). The grid used here is the
tensor rule that integrates degree-2p harmonics exactly: n_theta = p + 1
Gauss-Legendre nodes in cos(theta) times n_phi = 2 n_theta equispaced nodes in
phi (trapezoidal rule).

Node order on one sphere: theta index k (ascending cos(theta), i.e. the order
numpy's leggauss returns) outer, phi index l inner; node = k * n_phi + l.
"""
import numpy as np
from scipy.special import sph_harm_y


def sphere_grid(n_theta, n_phi, radius):
    """Offsets o = a*(sin t cos f, sin t sin f, cos t), unit normals and weights.

    Weight of node (k, l) is a^2 * W_k * 2*pi/n_phi with W_k the Gauss-Legendre
    weight of cos(theta_k); the weights sum to 4*pi*a^2.
    Pinned by: sum of weights, exact integration of spherical harmonics up to
    degree 2p, and nodes equal to numpy's leggauss (tests/test_oracle_grid.py).
    """
    t, wt = np.polynomial.legendre.leggauss(n_theta)
    st = np.sqrt(1.0 - t * t)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    T = np.repeat(t, n_phi)
    S = np.repeat(st, n_phi)
    F = np.tile(phi, n_theta)
    nrm = np.stack([S * np.cos(F), S * np.sin(F), T], axis=1)
    w = radius * radius * np.repeat(wt, n_phi) * (2.0 * np.pi / n_phi)
    return radius * nrm, nrm, w


def grid_angles(n_theta, n_phi):
    """(theta, phi) of every node, same order as sphere_grid."""
    t, _ = np.polynomial.legendre.leggauss(n_theta)
    th = np.arccos(t)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    return np.repeat(th, n_phi), np.tile(phi, n_theta)


def real_sh(p, theta, phi):
    """Orthonormal real spherical harmonics of degree <= p at (theta, phi).

    Returns an array of shape (len(theta), (p+1)^2). Built from scipy's complex
    harmonics: Y_l0, sqrt(2) Re Y_lm and sqrt(2) Im Y_lm for m > 0.
    """
    theta = np.asarray(theta, dtype=np.float64).ravel()
    phi = np.asarray(phi, dtype=np.float64).ravel()
    cols = []
    for l in range(p + 1):
        cols.append(sph_harm_y(l, 0, theta, phi).real)
        for m in range(1, l + 1):
            y = sph_harm_y(l, m, theta, phi)
            cols.append(np.sqrt(2.0) * y.real)
            cols.append(np.sqrt(2.0) * y.imag)
    return np.stack(cols, axis=1)


def projection_to_points(n_theta, n_phi, theta_t, phi_t):
    """Matrix mapping grid samples to values at arbitrary points.

    The grid function is projected onto harmonics of degree <= p = n_theta - 1
    with the grid quadrature (exact for band-limited data, since products of
    two degree-p harmonics are integrated exactly), then evaluated at the
    target points. Shape (n_points, n_theta * n_phi).
    """
    p = n_theta - 1
    th, ph = grid_angles(n_theta, n_phi)
    _, _, w_unit = sphere_grid(n_theta, n_phi, 1.0)
    Yg = real_sh(p, th, ph)                 # (n, L)
    Yt = real_sh(p, theta_t, phi_t)         # (m, L)
    return Yt @ (Yg * w_unit[:, None]).T
