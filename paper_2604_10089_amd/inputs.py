"""Seeded synthetic workloads: sphere packings, Janus axes, forces, planted LCPs.

This module generates inputs only; it holds none of the method's arithmetic.
Both the HIP path's tests and benchmarks and the CPU oracle's tests draw from
it. Every generator takes a seed and uses numpy's PCG64 (default_rng).

Sphere radius is 1 throughout (the paper's Janus spheres are identical). Gaps
are centre distance minus 2 radii.
"""
import numpy as np

RADIUS = 1.0


def _gaps(c):
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    iu = np.triu_indices(c.shape[0], 1)
    return d[iu] - 2.0 * RADIUS


def min_gap(c):
    c = np.asarray(c)
    return np.inf if c.shape[0] < 2 else float(_gaps(c).min())


def count_close(c, delta):
    return int((_gaps(np.asarray(c)) <= delta).sum())


def unit_vectors(rng, m):
    v = rng.standard_normal((m, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def growth_cluster(seed, m=8, gap_lo=0.01, gap_hi=0.1, contacts=(4, 8), delta=0.1):
    """Tiny cluster: each new sphere touches a random earlier one at gap U[lo, hi].

    Rejects attempts that bring any pair closer than gap_lo; accepts a cluster
    whose number of pairs with gap < delta lies in `contacts`.
    """
    rng = np.random.default_rng(seed)
    while True:
        c = np.zeros((1, 3))
        tries = 0
        while c.shape[0] < m and tries < 10000:
            tries += 1
            k = rng.integers(c.shape[0])
            g = rng.uniform(gap_lo, gap_hi)
            p = c[k] + (2.0 * RADIUS + g) * unit_vectors(rng, 1)[0]
            d = np.linalg.norm(c - p, axis=1) - 2.0 * RADIUS
            if d.min() >= gap_lo - 1e-12:
                c = np.vstack([c, p])
        if c.shape[0] == m:
            nc = int((_gaps(c) < delta).sum())
            if contacts[0] <= nc <= contacts[1]:
                return c - c.mean(axis=0)


def perturbed_lattice(seed, m=3, spacing=None, jitter=0.05, phi=0.3):
    """m^3 lattice at volume fraction phi (spacing (4 pi/3/phi)^(1/3)) plus U[-j, j] jitter."""
    rng = np.random.default_rng(seed)
    if spacing is None:
        spacing = (4.0 * np.pi / 3.0 / phi) ** (1.0 / 3.0)
    g = (np.arange(m) - 0.5 * (m - 1)) * spacing
    c = np.stack(np.meshgrid(g, g, g, indexing='ij'), axis=-1).reshape(-1, 3)
    return c + rng.uniform(-jitter, jitter, size=c.shape)


def lattice_with_contacts(seed, m=3, delta=0.1, jitter=0.05, n_desired=None, eps_desired=None,
                          min_gap_allowed=0.01, max_tries=50):
    """Alg. 5 of the paper (initial configuration): bisect a lattice scale gamma.

    A jittered m^3 lattice is scaled by gamma until the number of pairs with
    gap <= delta lies in [n_desired - eps, n_desired + eps] (defaults m^3/2 and
    m^3/10). Configurations with an overlap closer than min_gap_allowed are
    redrawn. Returns (centres, gamma).
    """
    n_desired = 0.5 * m ** 3 if n_desired is None else n_desired
    eps_desired = 0.1 * m ** 3 if eps_desired is None else eps_desired
    for t in range(max_tries):
        base = perturbed_lattice(seed * 1000 + t, m, spacing=2.0 * RADIUS + delta, jitter=jitter)
        lo, gam, hi = 0.0, 1.0, 1.0
        while count_close(base * hi, delta) > 0:
            hi *= 2.0
        for _ in range(200):
            k = count_close(base * gam, delta)
            if n_desired - eps_desired <= k <= n_desired + eps_desired:
                break
            if k < n_desired - eps_desired:
                hi = gam
                gam = gam + (lo - gam) * 0.5 if False else 0.5 * (lo + gam)
            else:
                lo = gam
                gam = 0.5 * (gam + hi)
        c = base * gam
        k = count_close(c, delta)
        if n_desired - eps_desired <= k <= n_desired + eps_desired and min_gap(c) >= min_gap_allowed:
            return c, gam
    raise RuntimeError('lattice_with_contacts: no configuration found')


def rsa_box(seed, m, side, min_gap=0.01, max_attempts=2_000_000):
    """Random sequential addition of m spheres with centres in [0, side]^3."""
    rng = np.random.default_rng(seed)
    c = np.empty((0, 3))
    att = 0
    while c.shape[0] < m:
        att += 1
        if att > max_attempts:
            raise RuntimeError('rsa_box: packing too dense')
        p = rng.uniform(0.0, side, 3)
        if c.shape[0] == 0 or (np.linalg.norm(c - p, axis=1) - 2.0 * RADIUS).min() >= min_gap:
            c = np.vstack([c, p])
    return c - 0.5 * side


def box_side(m, phi):
    return (m * 4.0 * np.pi / 3.0 / phi) ** (1.0 / 3.0)


def compressed_packing(seed, m=64, phi0=0.25, phi=0.35, min_gap_allowed=0.01, sweeps=10000):
    """RSA at phi0, affine compression to phi, then pairwise push-apart to min gap."""
    c = rsa_box(seed, m, box_side(m, phi0), min_gap=min_gap_allowed)
    c = c * (box_side(m, phi) / box_side(m, phi0))
    target = 2.0 * RADIUS + min_gap_allowed
    for _ in range(sweeps):
        moved = False
        for i in range(m):
            d = c - c[i]
            r = np.linalg.norm(d, axis=1)
            r[i] = np.inf
            bad = np.where(r < target)[0]
            for j in bad:
                s = 0.5 * (target - r[j]) + 1e-9
                u = d[j] / r[j]
                c[j] += s * u
                c[i] -= s * u
                moved = True
        if not moved:
            break
    return c


def batched_suspensions(seed, n_inst=32, m_range=(8, 27), n_thetas=(8, 10, 12, 14, 16),
                        phi_range=(0.2, 0.35)):
    """Independent suspensions of uneven size: list of (centres, n_theta, n_phi)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        nt = int(rng.choice(n_thetas))
        phi = float(rng.uniform(*phi_range))
        c = rsa_box(seed * 1000 + k, m, box_side(m, phi))
        out.append((c, nt, 2 * nt))
    return out


def largest_suspension(seed, m=216, phi=0.3):
    """216 spheres by RSA at volume fraction 0.3 in a cube (side ~14.45), min gap 0.01."""
    return rsa_box(seed, m, box_side(m, phi), min_gap=0.01)


def random_forces(seed, m, k=None):
    """N(0, 1) forces and torques, (m, 6) or (k, m, 6)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, 6) if k is None else (k, m, 6))


def janus_axes(seed, m):
    return unit_vectors(np.random.default_rng(seed), m)


def planted_lcp(seed, n, frac_active=0.5):
    """A complementary pair x* >= 0, w* >= 0, x*.w* = 0 (about frac_active with x* > 0).

    An LCP with solution x* is b = w* - A x*, which the caller forms with its own
    product A[x*].
    """
    rng = np.random.default_rng(seed)
    act = rng.uniform(size=n) < frac_active
    x = np.where(act, rng.uniform(0.5, 1.5, n), 0.0)
    w = np.where(act, 0.0, rng.uniform(0.5, 1.5, n))
    return x, w


def workload(name, seed=0):
    """Centres, grid and extra settings of the named workload (sizes in the docstring of each)."""
    if name == 'tiny':          # 8 spheres, 8x16 grid
        c = growth_cluster(seed)
        return dict(centers=c, n_theta=8, n_phi=16, lo=(4, 8), dt=0.1)
    if name == 'lattice27':     # 27 spheres, 16x32 grid, low fidelity 6x12
        return dict(centers=perturbed_lattice(seed), n_theta=16, n_phi=32, lo=(6, 12), dt=1e-3)
    if name == 'lattice27_contacts':
        c, _ = lattice_with_contacts(seed)
        return dict(centers=c, n_theta=16, n_phi=32, lo=(6, 12), dt=1e-3)
    if name == 'packing64':     # 64 spheres, 16x32 grid
        return dict(centers=compressed_packing(seed), n_theta=16, n_phi=32, lo=(6, 12), dt=1e-3)
    if name == 'rsa216':        # 216 spheres, 12x24 grid, low fidelity 6x12
        return dict(centers=largest_suspension(seed), n_theta=12, n_phi=24, lo=(6, 12), dt=1e-3)
    raise KeyError(name)
