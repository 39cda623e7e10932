"""Completed double-layer BIE and the rigid-body mobility MVP (oracle, FP64).

Test infrastructure only (see the package docstring).

The paper only fixes the structure of the mobility product, M ~ P M^stk P^T with
a second-kind boundary integral equation solved by GMRES inside every product
(Sec. 2, Fig. 1; Sec. 5.1, "tolerances"). The integral equation itself is not
written in the paper. The reading used throughout this repository is the
completed double-layer (Power-Miranda) second-kind formulation:

  exterior velocity   u(x) = D[q](x) + V[F,T](x)
  double layer        D[q](x) = 3/(4 pi) * int r (r.q(y)) (r.n(y)) / |r|^5 dS_y,
                      r = x - y, n the outward normal, so that D[const] is
                      -const inside a surface, -const/2 on it, 0 outside
  completion          V[F,T](x) = 1/(8 pi mu) sum_j F_j/|r_j| + r_j (r_j.F_j)/|r_j|^3
                                               + T_j x r_j/|r_j|^3,  r_j = x - c_j
  equation on Gamma   (1/2 I + D + P)[q] = u_s - V[F,T]
  rigid motion        U_i + Omega_i x (x - c_i) = -P_i[q]
                      U_i = -1/(4 pi a^2) int q,  Omega_i = -3/(8 pi a^4) int (y-c_i) x q

P_i is the orthogonal projector (in the quadrature inner product) onto the six
rigid motions of particle i, and u_s the prescribed slip (zero for the
collisional products). The double layer carries no force or torque, so the
particles feel exactly F, T.

Discretisation (one fixed rule so that every implementation computes the same
discrete operator):
  * nodes and weights of grid.sphere_grid on every sphere;
  * off-particle interactions by the plain node rule, sum_y w_y K(x,y) q_y;
  * near particle pairs (gap < near_gap): the source density is carried to an
    upsampled grid (near_up x n_theta by near_up x n_phi, by its degree-p
    spherical-harmonic projection) and summed with constant-density
    subtraction, sum_f w_f K(x,y_f) (q_f - q_j(x*)), where x* is the foot
    point of x on sphere j (the surface point nearest to x) and q_j(x*) the
    degree-p expansion of the density there. The subtraction uses
    D_j[const](x) = 0 outside sphere j. This stands in for the paper's
    near-singular evaluation, which the paper names by cost only (Sec. 5.1);
    optionally, pairs closer than near_close_gap use the finer factor
    near_close_up instead (a gap the near_up grid does not resolve);
  * optionally (Geometry(far_coarse=(nt_c, np_c)), a lower fidelity of the same
    discretisation) far pairs take their sources from a coarse grid carrying the
    density truncated to degree nt_c - 1 (far_coarse_rule);
  * the weakly singular self interaction by a rotated-pole rule: for each target
    node x0 the sphere is re-gridded with x0 at the pole (Gauss-Legendre in the
    polar angle theta' on [0, pi] with 3 n_theta points, trapezoid in phi' with
    2 n_phi points); the sin(theta') Jacobian cancels the 1/|r| singularity; the
    density is carried to the rotated nodes by its degree-p spherical-harmonic
    projection. This is the self-quadrature whose O(p^4) cost the paper quotes
    (Sec. 5.1).

Vector layout in this module: surface fields are (N, 3) arrays, node-major,
particle-major (all nodes of particle 0, then particle 1, ...).
"""
import numpy as np
import scipy.linalg

from . import grid as _grid

FOUR_PI = 4.0 * np.pi


class Geometry:
    """Centres plus the per-sphere grid of one suspension (plain container)."""

    def __init__(self, centers, radius=1.0, n_theta=8, n_phi=16, mu=1.0,
                 near_gap=None, near_up=2, near_close_gap=0.0, near_close_up=3, far_coarse=None):
        self.c = np.array(centers, dtype=np.float64).reshape(-1, 3)
        self.M = self.c.shape[0]
        self.a = float(radius)
        self.mu = float(mu)
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        self.o, self.nrm, self.w = _grid.sphere_grid(self.n_theta, self.n_phi, self.a)
        self.n = self.o.shape[0]
        self.N = self.M * self.n
        self.near_gap = 0.5 * self.a if near_gap is None else float(near_gap)
        self.near_up = int(near_up)
        self.near_close_gap = float(near_close_gap)
        self.near_close_up = int(near_close_up)
        # far pairs from a coarser source grid (n_theta_c, n_phi_c), or None (the node rule)
        self.far_coarse = None if far_coarse is None else (int(far_coarse[0]), int(far_coarse[1]))
        self.x = (self.c[:, None, :] + self.o[None, :, :]).reshape(-1, 3)
        self.normals = np.tile(self.nrm, (self.M, 1))
        self.weights = np.tile(self.w, self.M)

    def nodes(self, i):
        s = slice(i * self.n, (i + 1) * self.n)
        return s

    def pair_up(self, i, j):
        """Upsampling factor of the near pair (i, j): near_close_up below near_close_gap."""
        gap = np.linalg.norm(self.c[i] - self.c[j]) - 2.0 * self.a
        return self.near_close_up if gap < self.near_close_gap else self.near_up

    def pair_class(self):
        """(M, M) int array: 2 on the diagonal, 1 for near pairs, 0 otherwise."""
        d = np.linalg.norm(self.c[:, None, :] - self.c[None, :, :], axis=2)
        cls = np.where(d - 2.0 * self.a < self.near_gap, 1, 0)
        np.fill_diagonal(cls, 2)
        return cls


# ---------------------------------------------------------------- kernels

def dl_kernel(x, y, ny):
    """3x3 double-layer kernel matrices K(x, y), shape (m, k, 3, 3).

    K(x, y) q = 3/(4 pi) r (r.q)(r.n_y)/|r|^5 with r = x - y.
    Pinned by: D[const] = -const at a sphere centre and ~0 outside
    (tests/test_oracle_bie.py).
    """
    r = x[:, None, :] - y[None, :, :]
    r2 = np.einsum('mki,mki->mk', r, r)
    rn = np.einsum('mki,ki->mk', r, ny)
    coef = (3.0 / FOUR_PI) * rn / (r2 * r2 * np.sqrt(r2))
    return coef[:, :, None, None] * r[:, :, :, None] * r[:, :, None, :]


def dl_apply(x, y, ny, wq):
    """sum_y K(x, y) wq_y for targets x (m,3), sources y (k,3); returns (m,3)."""
    out = np.zeros((x.shape[0], 3))
    for s in range(0, x.shape[0], 256):
        r = x[s:s + 256, None, :] - y[None, :, :]
        r2 = np.einsum('mki,mki->mk', r, r)
        rn = np.einsum('mki,ki->mk', r, ny)
        rq = np.einsum('mki,ki->mk', r, wq)
        coef = (3.0 / FOUR_PI) * rn * rq / (r2 * r2 * np.sqrt(r2))
        out[s:s + 256] = np.einsum('mk,mki->mi', coef, r)
    return out


def completion(geom, FT, x=None):
    """Stokeslet + rotlet field V[F,T] at points x (default: all nodes), (m,3).

    FT is (M, 6): (Fx, Fy, Fz, Tx, Ty, Tz) per particle, the layout of the
    paper's force vector (Sec. 2).
    """
    x = geom.x if x is None else x
    FT = np.asarray(FT, dtype=np.float64).reshape(geom.M, 6)
    out = np.zeros((x.shape[0], 3))
    for j in range(geom.M):
        r = x - geom.c[j]
        d = np.linalg.norm(r, axis=1)
        F, T = FT[j, :3], FT[j, 3:]
        out += (F[None, :] / d[:, None]
                + r * (r @ F)[:, None] / d[:, None] ** 3
                + np.cross(T[None, :], r) / d[:, None] ** 3)
    return out / (8.0 * np.pi * geom.mu)


def janus_slip(geom, axes, speed):
    """Janus slip u_s(x) = -s (e - (e.n) n) on the cap n.e > 0, else 0.

    The paper's Janus interaction model is cited, not defined (Sec. 6); this
    tangential half-cap slip is the reading used here. An isolated sphere then
    swims along +e at s/3.
    """
    axes = np.asarray(axes, dtype=np.float64).reshape(geom.M, 3)
    e = np.repeat(axes, geom.n, axis=0)
    n = geom.normals
    en = np.einsum('ki,ki->k', e, n)
    u = -speed * (e - en[:, None] * n)
    u[en <= 0.0] = 0.0
    return u


# --------------------------------------------------------- rigid projection

def rigid_moments(geom, q):
    """Per particle: sum w q (M,3) and sum w (y-c) x q (M,3)."""
    q = q.reshape(geom.M, geom.n, 3)
    wq = q * geom.w[None, :, None]
    f = wq.sum(axis=1)
    t = np.cross(geom.o[None, :, :], wq).sum(axis=1)
    return f, t


def rigid_projection(geom, q):
    """P[q] (N,3): projection onto each particle's six rigid motions."""
    f, t = rigid_moments(geom, q)
    a = geom.a
    U = f / (FOUR_PI * a * a)
    W = t * (3.0 / (8.0 * np.pi * a ** 4))
    out = U[:, None, :] + np.cross(W[:, None, :], geom.o[None, :, :])
    return out.reshape(-1, 3)


def rigid_velocity(geom, q):
    """(U, Omega) per particle = -P[q] read as a rigid motion, (M, 6)."""
    f, t = rigid_moments(geom, q)
    a = geom.a
    U = -f / (FOUR_PI * a * a)
    W = -t * (3.0 / (8.0 * np.pi * a ** 4))
    return np.concatenate([U, W], axis=1)


# --------------------------------------------------------------- self block

def _rot(theta, phi):
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    Ry = np.array([[ct, 0.0, st], [0.0, 1.0, 0.0], [-st, 0.0, ct]])
    Rz = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
    return Rz @ Ry


_SELF_CACHE = {}
_SELF_ROW_CACHE = {}


def self_block_row(n_theta, n_phi, radius, i):
    """Row block S[:, i, :, :] (3, 3, n) of the self block for local target node i."""
    key = (n_theta, n_phi, float(radius), int(i))
    if key not in _SELF_ROW_CACHE:
        _SELF_ROW_CACHE[key] = self_block(n_theta, n_phi, radius, rows=[int(i)])[:, int(i), :, :]
    return _SELF_ROW_CACHE[key]


def self_block(n_theta, n_phi, radius, theta_factor=3, phi_factor=2, rows=None):
    """Self-interaction matrix S of one sphere, shape (3, n, 3, n).

    (S q)[c, i] = sum_{d,k} S[c, i, d, k] q[d, k] approximates the principal
    value int_Gamma K(x_i, y) q(y) dS_y by the rotated-pole rule described in
    the module docstring, computed target by target.
    Pinned by: rigid motions map to minus half of themselves; the single-sphere
    drag laws (tests/test_oracle_bie.py).
    """
    key = (n_theta, n_phi, float(radius), theta_factor, phi_factor)
    if rows is None and key in _SELF_CACHE:
        return _SELF_CACHE[key]
    a = float(radius)
    p = n_theta - 1
    o, nrm, w = _grid.sphere_grid(n_theta, n_phi, a)
    n = o.shape[0]
    th_n, ph_n = _grid.grid_angles(n_theta, n_phi)
    _, _, w_unit = _grid.sphere_grid(n_theta, n_phi, 1.0)
    Ygw = _grid.real_sh(p, th_n, ph_n) * w_unit[:, None]      # (n, L)

    xi, wx = np.polynomial.legendre.leggauss(theta_factor * n_theta)
    thp = 0.5 * np.pi * (xi + 1.0)
    wth = 0.5 * np.pi * wx
    nphp = phi_factor * n_phi
    php = 2.0 * np.pi * np.arange(nphp) / nphp
    TH = np.repeat(thp, nphp)
    PH = np.tile(php, theta_factor * n_theta)
    loc = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=1)
    Wz = a * a * np.sin(TH) * np.repeat(wth, nphp) * (2.0 * np.pi / nphp)

    S = np.zeros((3, n, 3, n))
    for i in (range(n) if rows is None else rows):
        R = _rot(th_n[i], ph_n[i])
        u = loc @ R.T
        thz = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
        phz = np.arctan2(u[:, 1], u[:, 0])
        Yz = _grid.real_sh(p, thz, phz)                        # (nz, L)
        K = dl_kernel(o[i:i + 1], a * u, u)[0]                 # (nz, 3, 3)
        G = np.einsum('z,zcd,zl->cdl', Wz, K, Yz)              # (3, 3, L)
        S[:, i, :, :] = G @ Ygw.T                              # (3, 3, n)
    if rows is None:
        _SELF_CACHE[key] = S
    return S


def self_block_nodemajor(S):
    """Reshape (3, n, 3, n) to a (3n, 3n) matrix acting on (n, 3) node-major vectors."""
    n = S.shape[1]
    return S.transpose(1, 0, 3, 2).reshape(3 * n, 3 * n)


# ------------------------------------------------------ operator (1/2 + D + P)

_UP_CACHE = {}


def upsample_matrix(n_theta, n_phi, up):
    """(n_fine, n) map from grid values to the up-times finer grid (degree-p projection)."""
    key = (n_theta, n_phi, up)
    if key not in _UP_CACHE:
        thf, phf = _grid.grid_angles(up * n_theta, up * n_phi)
        _UP_CACHE[key] = _grid.projection_to_points(n_theta, n_phi, thf, phf)
    return _UP_CACHE[key]


def near_sources(geom, j, up):
    """Nodes, normals and weights of sphere j on the up-times finer grid of near pairs."""
    of, nf, wf = _grid.sphere_grid(up * geom.n_theta, up * geom.n_phi, geom.a)
    return geom.c[j] + of, nf, wf


def near_block(geom, i, j):
    """Dense (n, 3, n, 3) near-pair block: upsampled plain rule with subtraction.

    Pinned by: the exterior double layer of sphere j's six rigid motions vanishes at
    every target (gaps 0.4 to 0.01); on band-limited densities the rule converges, as
    the upsampling grows, to a graded rotated-pole reference quadrature with the
    density in closed form; the subtracted value is the density at the foot point
    (tests/test_oracle_bie.py).
    """
    cache = geom.__dict__.setdefault('_near_cache', {})
    if (i, j) in cache:
        return cache[(i, j)]
    X = geom.x[geom.nodes(i)]
    up = geom.pair_up(i, j)
    yf, nf, wf = near_sources(geom, j, up)
    I = upsample_matrix(geom.n_theta, geom.n_phi, up)
    K = dl_kernel(X, yf, nf) * wf[None, :, None, None]          # (n, nf, 3, 3)
    u = X - geom.c[j]
    u /= np.linalg.norm(u, axis=1)[:, None]
    Ifoot = _grid.projection_to_points(geom.n_theta, geom.n_phi, np.arccos(np.clip(u[:, 2], -1.0, 1.0)),
                                       np.arctan2(u[:, 1], u[:, 0]))   # (n, n)
    blk = np.einsum('mfcd,fk->mckd', K, I)
    blk -= np.einsum('mcd,mk->mckd', K.sum(axis=1), Ifoot)
    cache[(i, j)] = blk
    return blk


def near_row(geom, i, j, k):
    """Row (3, n, 3) of the near block for the single target node k of sphere i.

    Pinned as near_block (the reference-quadrature and foot-point pins use rows).
    """
    X = geom.x[geom.nodes(i)][k:k + 1]
    up = geom.pair_up(i, j)
    yf, nf, wf = near_sources(geom, j, up)
    I = upsample_matrix(geom.n_theta, geom.n_phi, up)
    K = dl_kernel(X, yf, nf)[0] * wf[:, None, None]              # (nf, 3, 3)
    u = (X[0] - geom.c[j]) / np.linalg.norm(X[0] - geom.c[j])
    Ifoot = _grid.projection_to_points(geom.n_theta, geom.n_phi, np.array([np.arccos(np.clip(u[2], -1.0, 1.0))]),
                                       np.array([np.arctan2(u[1], u[0])]))[0]
    return np.einsum('fcd,fk->ckd', K, I) - np.einsum('cd,k->ckd', K.sum(axis=0), Ifoot)


def far_coarse_rule(geom):
    """Coarse source rule of far pairs: offsets, normals and weights of the coarse
    (n_theta_c, n_phi_c) grid, and the (n_c, n) map taking a sphere's node values to
    their projection on harmonics of degree <= p_c = n_theta_c - 1 evaluated at the
    coarse nodes. A lower fidelity of the same discretisation (Sec. 5.1 lowers the
    order p of the surface representation): far pairs see the source density only
    through its multipoles, whose fields decay like (a/d)^(l+1), so the degrees above
    p_c are dropped for them and the truncated density is summed on a grid that
    integrates it; the self and near terms keep the full grid and degree.
    Pinned by: on band-limited densities the coarse far sum converges to the node rule
    as p_c grows, geometrically, and equals it at p_c = p (tests/test_oracle_bie.py).
    """
    cache = geom.__dict__.setdefault('_far_coarse_cache', {})
    key = geom.far_coarse
    if key not in cache:
        ntc, npc = key
        pc = ntc - 1
        oc, nc, wc = _grid.sphere_grid(ntc, npc, geom.a)
        thc, phc = _grid.grid_angles(ntc, npc)
        th, ph = _grid.grid_angles(geom.n_theta, geom.n_phi)
        _, _, w_unit = _grid.sphere_grid(geom.n_theta, geom.n_phi, 1.0)
        analysis = (_grid.real_sh(pc, th, ph) * w_unit[:, None]).T      # (L_c, n): degrees <= p_c
        Pc = _grid.real_sh(pc, thc, phc) @ analysis
        cache[key] = (oc, nc, wc, Pc)
    return cache[key]


def far_sum(geom, x, j, qj):
    """Double layer of sphere j's density qj (n, 3) at far points x (m, 3): the node
    rule, or the coarse source rule when geom.far_coarse is set."""
    sj = geom.nodes(j)
    if geom.far_coarse is None:
        return dl_apply(x, geom.x[sj], geom.normals[sj], qj * geom.w[:, None])
    oc, nc, wc, Pc = far_coarse_rule(geom)
    return dl_apply(x, geom.c[j] + oc, nc, (Pc @ qj) * wc[:, None])


def offdiag_block(geom, i, j, near):
    """Dense (3n, 3n) block of D mapping q on sphere j to targets on sphere i."""
    if near:
        return near_block(geom, i, j).reshape(3 * geom.n, 3 * geom.n)
    si, sj = geom.nodes(i), geom.nodes(j)
    if geom.far_coarse is not None:
        oc, nc, wc, Pc = far_coarse_rule(geom)
        K = dl_kernel(geom.x[si], geom.c[j] + oc, nc) * wc[None, :, None, None]
        return np.einsum('mfcd,fk->mckd', K, Pc).reshape(3 * geom.n, 3 * geom.n)
    K = dl_kernel(geom.x[si], geom.x[sj], geom.normals[sj]) * geom.w[None, :, None, None]
    return K.transpose(0, 2, 1, 3).reshape(3 * geom.n, 3 * geom.n)


def dense_operator(geom):
    """Assembled (3N, 3N) matrix of (1/2 I + D + P) on node-major vectors."""
    n3 = 3 * geom.n
    A = np.zeros((3 * geom.N, 3 * geom.N))
    S = self_block_nodemajor(self_block(geom.n_theta, geom.n_phi, geom.a))
    cls = geom.pair_class()
    for i in range(geom.M):
        for j in range(geom.M):
            blk = S if i == j else offdiag_block(geom, i, j, cls[i, j] == 1)
            A[i * n3:(i + 1) * n3, j * n3:(j + 1) * n3] = blk
    A += 0.5 * np.eye(3 * geom.N)
    # rigid projection, column by column of each sphere
    a = geom.a
    for i in range(geom.M):
        o = geom.o
        cx = np.zeros((geom.n, 3, 3))
        cx[:, 0, 1], cx[:, 0, 2] = -o[:, 2], o[:, 1]
        cx[:, 1, 0], cx[:, 1, 2] = o[:, 2], -o[:, 0]
        cx[:, 2, 0], cx[:, 2, 1] = -o[:, 1], o[:, 0]
        Ptr = np.kron(np.ones((geom.n, 1)), np.kron(geom.w[None, :], np.eye(3))) / (FOUR_PI * a * a)
        Prot = -np.einsum('mab,kbc,k->makc', cx, cx, geom.w).reshape(n3, n3) * (3.0 / (8.0 * np.pi * a ** 4))
        A[i * n3:(i + 1) * n3, i * n3:(i + 1) * n3] += Ptr + Prot
    return A


def offdiag_apply(geom, q, i_targets=None):
    """Off-particle part of D applied to q (N,3); returns (N,3) (or rows of i_targets)."""
    q = q.reshape(geom.N, 3)
    cls = geom.pair_class()
    tgts = range(geom.M) if i_targets is None else i_targets
    out = np.zeros((geom.N, 3))
    for i in tgts:
        si = geom.nodes(i)
        xi = geom.x[si]
        acc = np.zeros((geom.n, 3))
        for j in range(geom.M):
            if j == i:
                continue
            sj = geom.nodes(j)
            if cls[i, j] == 1:
                acc += np.einsum('mckd,kd->mc', near_block(geom, i, j), q[sj])
            else:
                acc += far_sum(geom, xi, j, q[sj])
        out[si] = acc
    return out


def self_apply(geom, q):
    """Self-interaction part of D (block diagonal), (N,3) -> (N,3)."""
    S = self_block(geom.n_theta, geom.n_phi, geom.a)
    qq = q.reshape(geom.M, geom.n, 3)
    return np.einsum('cidk,mkd->mic', S, qq).reshape(-1, 3)


def operator_rows(geom, q, targets):
    """Rows of (1/2 I + D + P)[q] at the given global node indices, (len(targets), 3).

    The same definition as operator_apply, evaluated target by target, for
    suspensions too large to apply whole.
    """
    q = q.reshape(geom.N, 3)
    cls = geom.pair_class()
    P = rigid_projection(geom, q)
    out = np.zeros((len(targets), 3))
    for row, t in enumerate(targets):
        i, k = divmod(int(t), geom.n)
        xt = geom.x[t:t + 1]
        Sk = self_block_row(geom.n_theta, geom.n_phi, geom.a, k)
        acc = 0.5 * q[t] + np.einsum('cdm,md->c', Sk, q[geom.nodes(i)]) + P[t]
        for j in range(geom.M):
            if j == i:
                continue
            sj = geom.nodes(j)
            if cls[i, j] == 1:
                acc = acc + np.einsum('ckd,kd->c', near_row(geom, i, j, k), q[sj])
            else:
                acc = acc + far_sum(geom, xt, j, q[sj])[0]
        out[row] = acc
    return out


def operator_apply(geom, q):
    """Matrix-free (1/2 I + D + P)[q] for (N,3) densities."""
    q = q.reshape(geom.N, 3)
    return 0.5 * q + self_apply(geom, q) + offdiag_apply(geom, q) + rigid_projection(geom, q)


# ------------------------------------------------------------------- GMRES

def gmres(apply, rhs, tol=1e-13, restart=50, maxiter=1000, x0=None, right=None):
    """Restarted GMRES (modified Gram-Schmidt Arnoldi, Givens rotations).

    Textbook GMRES(m) from the initial guess x0 (default 0): stops when the
    residual norm falls below tol * ||rhs||. With a right preconditioner
    `right` (a linear map P), the Krylov space is built for the operator A P
    and every cycle ends with x += P (V y): the residual, and so the stopping
    rule, is that of x itself.
    Returns (x, iterations, final relative residual estimate).
    """
    if right is not None:
        a0 = apply
        apply = lambda v: a0(right(v.ravel()).reshape(v.shape))  # noqa: E731
    b = rhs.ravel().astype(np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).ravel()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    its = 0
    while True:
        r = b - (apply(x.reshape(rhs.shape)) if right is None else a0(x.reshape(rhs.shape))).ravel()
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm or its >= maxiter:
            return x, its, beta / bnorm
        V = np.zeros((restart + 1, b.size))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for k in range(restart):
            its += 1
            wv = apply(V[k].reshape(rhs.shape)).ravel()
            for i in range(k + 1):
                H[i, k] = V[i] @ wv
                wv -= H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(wv)
            if H[k + 1, k] > 0.0:
                V[k + 1] = wv / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            if abs(g[k + 1]) <= tol * bnorm or its >= maxiter:
                break
        m = k + 1
        y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
        x += V[:m].T @ y if right is None else right(V[:m].T @ y)


# --------------------------------------------------------- preconditioner

def near_patch_preconditioner(geom, A):
    """Right preconditioner of the BIE's GMRES from its assembled matrix A (node-major).

    Sec. 2 calls for preconditioned Krylov solves of the mobility problem
    without naming a preconditioner; this is the one the GPU path uses. With D
    the diagonal block of one sphere (the same for every sphere) and A_ij the
    block of a near pair (gap < near_gap), sphere i's part of P v is
        S_i^{-1} (v_i - sum_j A_ij D^{-1} v_j),   S_i = D - sum_j A_ij D^{-1} A_ji:
    the row of sphere i of the inverse of its near patch, partner-partner
    coupling dropped (a Schur complement). Returns P as a function of a flat
    node-major vector. Pinned by: one sphere gives P = D^{-1} = A^{-1}; two
    spheres that are each other's only near partner give P = A^{-1}
    (block inverse by Schur complements) (tests/test_oracle_bie.py).
    """
    n3, M = 3 * geom.n, geom.M
    blk = lambda i, j: A[i * n3:(i + 1) * n3, j * n3:(j + 1) * n3]  # noqa: E731
    D = blk(0, 0)
    Di = np.linalg.inv(D)
    cls = geom.pair_class()
    nbr = [[j for j in range(M) if j != i and cls[i, j] == 1] for i in range(M)]
    Sinv = []
    for i in range(M):
        S = D.copy()
        for j in nbr[i]:
            S -= blk(i, j) @ Di @ blk(j, i)
        Sinv.append(np.linalg.inv(S))

    def apply(v):
        v = np.asarray(v, dtype=np.float64).reshape(M, n3)
        y = v @ Di.T
        out = np.empty_like(v)
        for i in range(M):
            r = v[i].copy()
            for j in nbr[i]:
                r -= blk(i, j) @ y[j]
            out[i] = Sinv[i] @ r
        return out.ravel()
    return apply


def two_level_preconditioner(geom, A, P, lmax=2, coarse_theta=None, coarse_close=None):
    """Two-level right preconditioner: a coarse correction on every sphere's
    harmonics of degree <= lmax (3 (lmax + 1)^2 unknowns per sphere) applied
    before the near-patch preconditioner P (Sec. 2 leaves the preconditioner
    open; the far field's smooth low modes are what the near patches miss):
        c = E^{-1} R v,  z1 = Z c,  P2 v = z1 + P (v - A~ z1),  E = R A~ Z,
    with Z the synthesis of those harmonics at the nodes (per sphere and
    component), R the projection on them (quadrature-weighted analysis, R Z = I)
    and A~ the operator with its far pairs summed on a coarse source grid of
    coarse_theta x 2 coarse_theta nodes (far_coarse_rule; None: A~ = A). With
    coarse_close = d and coarse_theta = (t1, t2), a far pair whose centres are
    closer than d radii takes the t1 x 2 t1 grid and the others the t2 x 2 t2
    grid (the closest far pairs carry most of the coarse operator's error). The
    near and self blocks of A~ are A's. Returns P2 as a function of a flat
    node-major vector. Pinned by: for one sphere P2 = A^{-1} when P is; and
    P2 (A~ Z c) = Z c for every coarse vector c, whatever P
    (tests/test_oracle_bie.py).
    """
    n, M = geom.n, geom.M
    th, ph = _grid.grid_angles(geom.n_theta, geom.n_phi)
    _, _, w_unit = _grid.sphere_grid(geom.n_theta, geom.n_phi, 1.0)
    Y = _grid.real_sh(lmax, th, ph)                      # (n, nl)
    nl = Y.shape[1]
    nb = 3 * nl
    Zb = np.zeros((3 * n, nb))
    Rb = np.zeros((nb, 3 * n))
    for c in range(3):
        for k in range(nl):
            Zb[np.arange(n) * 3 + c, c * nl + k] = Y[:, k]
            Rb[c * nl + k, np.arange(n) * 3 + c] = Y[:, k] * w_unit
    Z = np.zeros((3 * geom.N, M * nb))
    R = np.zeros((M * nb, 3 * geom.N))
    for i in range(M):
        Z[i * 3 * n:(i + 1) * 3 * n, i * nb:(i + 1) * nb] = Zb
        R[i * nb:(i + 1) * nb, i * 3 * n:(i + 1) * 3 * n] = Rb
    def coarse_geometry(t):
        return Geometry(geom.c, geom.a, geom.n_theta, geom.n_phi, geom.mu, near_gap=geom.near_gap,
                        near_up=geom.near_up, near_close_gap=geom.near_close_gap,
                        near_close_up=geom.near_close_up, far_coarse=(t, 2 * t))

    if coarse_theta is None:
        At = A
    elif coarse_close is None:
        At = dense_operator(coarse_geometry(coarse_theta))
    else:
        At = A.copy()
        g1, g2 = coarse_geometry(coarse_theta[0]), coarse_geometry(coarse_theta[1])
        cls = geom.pair_class()
        d = np.linalg.norm(geom.c[:, None, :] - geom.c[None, :, :], axis=2)
        for i in range(M):
            for j in range(M):
                if cls[i, j] == 0:
                    g = g1 if d[i, j] < coarse_close * geom.a else g2
                    At[i * 3 * n:(i + 1) * 3 * n, j * 3 * n:(j + 1) * 3 * n] = offdiag_block(g, i, j, False)
    AZ = At @ Z
    Ei = np.linalg.inv(R @ AZ)

    def apply(v):
        v = np.asarray(v, dtype=np.float64).ravel()
        c = Ei @ (R @ v)
        return Z @ c + P(v - AZ @ c)
    apply.Z, apply.At = Z, At
    return apply


# --------------------------------------------------------------- mobility

def solve_density(geom, rhs, dense=None, tol=1e-13):
    """Density q solving (1/2 I + D + P) q = rhs; dense LU when a matrix is given."""
    if dense is not None:
        lu = geom.__dict__.get('_lu')
        if lu is None or lu[0] is not dense:
            lu = (dense, scipy.linalg.lu_factor(dense))
            geom._lu = lu
        return scipy.linalg.lu_solve(lu[1], rhs.ravel()).reshape(-1, 3)
    q, _, _ = gmres(lambda v: operator_apply(geom, v), rhs, tol=tol)
    return q.reshape(-1, 3)


def mobility_apply(geom, FT, dense=None, tol=1e-13):
    """U = M F: rigid velocities (M, 6) for forces/torques FT (M, 6).

    Sec. 2, eq. (mobility): the mobility product; Fig. 1: it is applied as
    lift (V[F,T]), second-kind surface solve, projection (-P[q]).
    Pinned by: Stokes drag U = F/(6 pi mu a), Omega = T/(8 pi mu a^3) for a
    single sphere; far-field two-sphere mobilities; symmetry and definiteness
    of the assembled matrix (tests/test_oracle_bie.py).
    """
    rhs = -completion(geom, FT)
    q = solve_density(geom, rhs, dense, tol)
    return rigid_velocity(geom, q)


def nc_velocity(geom, axes, speed, dense=None, tol=1e-13):
    """Slip-driven rigid velocities U_nc (M, 6) with F = T = 0 (Sec. 2, eq. (mobility))."""
    rhs = janus_slip(geom, axes, speed)
    q = solve_density(geom, rhs, dense, tol)
    return rigid_velocity(geom, q)


class RecyclingMobility:
    """U = M F with every GMRES solve started from the earlier solutions (Sec. 7
    names the reuse of Krylov information across the MVPs of one solve as future
    work; this is its simplest form).

    The densities q_k of the earlier solves and their operator images
    w_k = A q_k are kept (at most `keep`, oldest dropped). A new right-hand side
    r starts GMRES from x0 = sum_k c_k q_k with c = argmin |r - sum_k c_k w_k|_2,
    whose residual r - A x0 = r - W c is never larger than |r|. The stopping rule
    is the cold solve's (|residual| <= tol |r|), so the result equals the cold
    solution to the GMRES tolerance. A product whose force lies in the span of
    earlier forces has a right-hand side in the span of earlier right-hand sides,
    so its initial residual is zero up to the earlier solves' tolerance.
    Here w_k is evaluated by one more operator application (plain, not fast);
    `iters` records the GMRES iterations of each call.
    """

    def __init__(self, geom, tol=1e-13, keep=32, restart=50):
        self.geom, self.tol, self.keep, self.restart = geom, tol, keep, restart
        self.Q, self.W, self.iters, self.r0 = [], [], [], []

    def _apply(self, v):
        return operator_apply(self.geom, v.reshape(-1, 3)).ravel()

    def __call__(self, FT):
        rhs = -completion(self.geom, FT).ravel()
        x0 = None
        if self.Q:
            W = np.stack(self.W, axis=1)
            c = np.linalg.lstsq(W, rhs, rcond=None)[0]
            x0 = np.stack(self.Q, axis=1) @ c
            self.r0.append(np.linalg.norm(rhs - W @ c) / max(np.linalg.norm(rhs), 1e-300))
        else:
            self.r0.append(1.0)
        q, its, _ = gmres(lambda v: self._apply(v), rhs, tol=self.tol, restart=self.restart, x0=x0)
        self.iters.append(its)
        if np.linalg.norm(rhs) > 0.0:
            self.Q.append(q.copy())
            self.W.append(self._apply(q))
            if len(self.Q) > self.keep:
                self.Q.pop(0)
                self.W.pop(0)
        return rigid_velocity(self.geom, q.reshape(-1, 3))
