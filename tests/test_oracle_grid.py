"""Pins of the sphere grid and the spherical-harmonic projection (oracle)."""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

from oracle import grid


@pytest.mark.parametrize("nt", [4, 6, 8, 12, 16])
def test_weights_sum_to_area(nt):
    _, _, w = grid.sphere_grid(nt, 2 * nt, 1.7)
    assert abs(w.sum() - 4 * np.pi * 1.7 ** 2) < 1e-12


@pytest.mark.parametrize("nt", [4, 8])
def test_nodes_are_golub_welsch(nt):
    # Gauss-Legendre nodes as eigenvalues of the Jacobi matrix (Golub-Welsch),
    # independent of numpy's leggauss
    k = np.arange(1, nt)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    ev, vec = eigh_tridiagonal(np.zeros(nt), beta)
    o, _, w = grid.sphere_grid(nt, 2 * nt, 1.0)
    cz = o[::2 * nt, 2]
    assert np.allclose(np.sort(cz), ev, atol=1e-14)
    wgl = 2.0 * vec[0, :] ** 2
    assert np.allclose(w[::2 * nt] / (2 * np.pi / (2 * nt)), wgl, atol=1e-14)


@pytest.mark.parametrize("nt", [4, 6])
def test_harmonics_integrated_exactly_to_degree_2p(nt):
    p = nt - 1
    th, ph = grid.grid_angles(nt, 2 * nt)
    _, _, w = grid.sphere_grid(nt, 2 * nt, 1.0)
    Y = grid.real_sh(2 * p, th, ph)
    integ = w @ Y
    expect = np.zeros_like(integ)
    expect[0] = np.sqrt(4 * np.pi)
    assert np.abs(integ - expect).max() < 1e-13


def test_projection_reproduces_band_limited_functions():
    nt = 6
    rng = np.random.default_rng(0)
    coef = rng.standard_normal(nt * nt)
    th, ph = grid.grid_angles(nt, 2 * nt)
    f = grid.real_sh(nt - 1, th, ph) @ coef
    tt = rng.uniform(0, np.pi, 50)
    pp = rng.uniform(0, 2 * np.pi, 50)
    exact = grid.real_sh(nt - 1, tt, pp) @ coef
    P = grid.projection_to_points(nt, 2 * nt, tt, pp)
    assert np.abs(P @ f - exact).max() < 1e-12
