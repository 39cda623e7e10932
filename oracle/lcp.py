"""LCP operator and solvers: BB-PGD, Mono-PQN, Bi-PQN (oracle, FP64).

Test infrastructure only (see the package docstring).

All solvers only see the LCP matrix through products A[x] (Sec. 3), exactly as
in the paper: A = D^T M D is never formed except by brute-force tests.
Quasi-Newton matrices are kept explicitly here (dense n x n), so that H g is a
plain linear solve with B: this is the definition of H = B^{-1}, not the
recursions a fast implementation uses.

Readings of the paper taken here (each also listed in the design notes):
  * Alg. 1 search step: x~ = x - H (A x + b), tau = 1 (Table 1; Lemma 1).
  * Initial metric: Prop. 1 allows any positive diagonal D; Alg. 1 prints
    H^(0) = I, which is not invariant to the units of A. Here the first step
    uses H^(0) = I and, once its product A p is known, the quasi-Newton matrix
    starts from B0 = sigma I with sigma = p.Ap/p.p (no extra product). sigma is
    kept for the rest of one LCP solve (all Bi-PQN subproblems included).
    printed_metric=True keeps Alg. 1 as printed instead: H^(0) = I at every
    (re)start, sigma = 1 throughout.
  * Stopping rule: the KKT errors of eq. (kkt-error), 2-norm, absolute OR
    relative change below tolerance.
  * Prop. 1 root function: L~(a, a~) = [a; a~] + L(a, a~) with L as printed;
    its Jacobian is the printed J_L (which carries the "+ I").
  * quasiNewtonUpdate: BFGS in the form B+ = B + u u^T - v v^T with
    u = y/sqrt(y.s), v = B s/sqrt(s.B s); a pair with y.s <= 1e-12 |s||y| is
    skipped (safeguard, not in the paper).
  * Alg. 2 edge cases: p = 0 stops; p.Ap <= 0 or eta' <= 0 resets the memory
    and takes eta = 1. The new iterate is clamped at 0 against rounding.
  * Bi-PQN secant transfer: Y <- Y^ + (u u^T - v v^T) S^ (the sign that makes
    B^(k+1) S = Y hold; the printed minus contradicts that stated goal).
  * Bi-PQN inner tolerance: 1e-2 x the current high-fidelity KKT error (floor
    1e-12), at most k_max_inner low-fidelity products; the low-fidelity
    initialisation uses the same rule at x^(-1) = 0.
"""
import itertools

import numpy as np
from scipy.optimize import nnls


# ------------------------------------------------------------ contact maps

def contact_normals(centers, pairs):
    """Unit normals n_l = (c_j - c_i)/|c_j - c_i| for contact pairs (i, j)."""
    c = np.asarray(centers, dtype=np.float64)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    d = c[pairs[:, 1]] - c[pairs[:, 0]]
    return d / np.linalg.norm(d, axis=1)[:, None]


def D_apply(centers, pairs, x):
    """F_c = D x (M, 6): force -x_l n_l on i, +x_l n_l on j, no torque (spheres).

    Sec. 3: each column of D holds the force/torque of one contact (6 nonzeros
    for spheres).
    """
    M = np.asarray(centers).shape[0]
    n = contact_normals(centers, pairs)
    FT = np.zeros((M, 6))
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    for l, (i, j) in enumerate(pairs):
        FT[i, :3] -= x[l] * n[l]
        FT[j, :3] += x[l] * n[l]
    return FT


def DT_apply(centers, pairs, UO):
    """(D^T U)_l = n_l . (U_j - U_i): the rate of change of the gap of pair l."""
    n = contact_normals(centers, pairs)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    UO = np.asarray(UO).reshape(-1, 6)
    return np.einsum('li,li->l', n, UO[pairs[:, 1], :3] - UO[pairs[:, 0], :3])


def lcp_operator(mobility, centers, pairs):
    """A[x] = D^T M D x (eq. (defAandb)) from a mobility product FT -> UO."""
    return lambda x: DT_apply(centers, pairs, mobility(D_apply(centers, pairs, x)))


def lcp_b(gaps, dt, centers, pairs, U_nc):
    """b = Phi/dt + D^T U_nc (eq. (defAandb))."""
    return np.asarray(gaps) / dt + DT_apply(centers, pairs, U_nc)


# ------------------------------------------------------------- small tools

def kkt_error(x, g):
    """Absolute KKT error ||min(x, A x + b)||_2 (eq. (kkt-error))."""
    return float(np.linalg.norm(np.minimum(x, g)))


def objective(A, b, x):
    return 0.5 * x @ (A @ x) + b @ x


def step_size(g, x, p, Ap):
    """Optimal over-relaxation eta* (Alg. 2). Returns (eta, reset_memory).

    eta' = -p.g / p.Ap is the unconstrained minimiser of f(x + eta p); the
    constraint x + eta p >= 0 caps it at min over p_l < 0 of -x_l/p_l.
    Pinned by: exact 1-D minimisation over the feasible interval and Lemma 1's
    sufficient decrease (tests/test_oracle_lcp.py).
    """
    pAp = float(p @ Ap)
    gp = float(p @ g)
    if pAp <= 0.0:
        return 1.0, True
    eta = -gp / pAp
    if eta <= 0.0:
        return 1.0, True
    neg = p < 0.0
    if np.any(neg):
        eta = min(eta, float(np.min(-x[neg] / p[neg])))
    return eta, False


class QuasiNewton:
    """B = B0 + U U^T - V V^T with BFGS updates, kept densely (Sec. 4, App. E.1).

    B0 is the identity for Mono-PQN (Alg. 1: H^(0) = I) or, through b0_apply,
    the low-fidelity matrix for Bi-PQN (eq. (bifi-qnapprox)).
    Pinned by: B+ s = y and H B = I (tests/test_oracle_lcp.py).
    """

    def __init__(self, n, b0_apply=None, sigma=1.0):
        self.n = n
        self.b0 = b0_apply
        self.sigma = float(sigma)
        self.U, self.V, self.S, self.Y = [], [], [], []

    def lowrank(self, v):
        out = np.zeros(self.n)
        for u in self.U:
            out += u * (u @ v)
        for w in self.V:
            out -= w * (w @ v)
        return out

    def dense(self):
        B = self.sigma * np.eye(self.n)
        for u in self.U:
            B += np.outer(u, u)
        for v in self.V:
            B -= np.outer(v, v)
        return B

    def B_apply(self, s, b0s=None):
        base = self.sigma * s if self.b0 is None else (self.b0(s) if b0s is None else b0s)
        return base + self.lowrank(s)

    def H_apply(self, g):
        return np.linalg.solve(self.dense(), g)

    def update(self, s, y, Bs=None):
        ys = float(y @ s)
        if not ys > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            return False
        Bs = self.B_apply(s) if Bs is None else Bs
        sBs = float(s @ Bs)
        if not sBs > 0.0:
            return False
        self.U.append(y / np.sqrt(ys))
        self.V.append(Bs / np.sqrt(sBs))
        self.S.append(s.copy())
        self.Y.append(y.copy())
        return True


# ---------------------------------------------------------- weighted prox

def prox_ssn(xt, U, V, d=None, jmax=50, eps_rel=1e-14):
    """prox^B of the nonnegative orthant at xt for B = D + U U^T - V V^T.

    Prop. 1 and Alg. 3: x^ = (xt + C^{-1} V a~ - D^{-1} U a)_+ with C = D + U U^T
    and (a, a~) the root of L~ = [a; a~] + L(a, a~) found by semi-smooth Newton
    from 0 with the printed Jacobian J_L; stops when the Newton step is below
    eps_rel * max(1, |(a, a~)|) or after jmax steps.
    Returns (x^, newton_steps, converged).
    Pinned by: the KKT conditions of the weighted prox and the primal solve
    (tests/test_oracle_lcp.py).
    """
    n = xt.size
    U = np.zeros((n, 0)) if U is None else np.asarray(U).reshape(n, -1)
    V = np.zeros((n, 0)) if V is None else np.asarray(V).reshape(n, -1)
    d = np.ones(n) if d is None else d
    r = U.shape[1]
    if r == 0:
        return np.maximum(xt, 0.0), 0, True
    C = np.diag(d) + U @ U.T
    CiV = np.linalg.solve(C, V)
    DiU = U / d[:, None]
    z = np.zeros(2 * r)
    conv = False
    j = 0
    for j in range(1, jmax + 1):
        a, at = z[:r], z[r:]
        w = xt + CiV @ at - DiU @ a
        xh = np.maximum(w, 0.0)
        lam = (w > 0.0).astype(np.float64)
        L = np.concatenate([a + U.T @ (xt + CiV @ at - xh), at + V.T @ (xt - xh)])
        J = np.block([[np.eye(r) + U.T @ (lam[:, None] * DiU), U.T @ ((1.0 - lam)[:, None] * CiV)],
                      [V.T @ (lam[:, None] * DiU), np.eye(r) - V.T @ (lam[:, None] * CiV)]])
        znew = z - np.linalg.solve(J, L)
        step = np.linalg.norm(znew - z)
        z = znew
        if step <= eps_rel * max(1.0, np.linalg.norm(z)):
            conv = True
            break
    a, at = z[:r], z[r:]
    return np.maximum(xt + CiV @ at - DiU @ a, 0.0), j, conv


def prox_primal(B, xt):
    """argmin_{z >= 0} 1/2 (z - xt)^T B (z - xt), solved in the primal.

    With B = L L^T (Cholesky) this is the nonnegative least-squares problem
    min |L^T z - L^T xt|, solved by scipy's Lawson-Hanson NNLS. Independent of
    the dual route of Prop. 1.
    """
    L = np.linalg.cholesky(B)
    z, _ = nnls(L.T, L.T @ xt, maxiter=50 * xt.size)
    return z


def brute_force_lcp(A, b, tol=1e-12):
    """Solve 0 <= A x + b  perp  x >= 0 by enumerating all 2^n active sets.

    For every free set F: x_F = -A_FF^{-1} b_F, x = 0 elsewhere; accept when
    x >= 0 and (A x + b) >= 0 off F. Unique when A is a P-matrix.
    """
    n = b.size
    best = None
    for mask in itertools.product([False, True], repeat=n):
        F = np.array(mask)
        x = np.zeros(n)
        if F.any():
            try:
                x[F] = np.linalg.solve(A[np.ix_(F, F)], -b[F])
            except np.linalg.LinAlgError:
                continue
        w = A @ x + b
        scale = max(1.0, np.abs(b).max())
        if (x >= -tol * scale).all() and (w[~F] >= -tol * scale).all():
            viol = np.abs(np.minimum(np.maximum(x, 0.0), w)).max()
            if best is None or viol < best[1]:
                best = (np.maximum(x, 0.0), viol)
    return None if best is None else best[0]


# ----------------------------------------------------------------- solvers

class Stats(dict):
    pass


def _converged(e, e_prev, tol_abs, tol_rel):
    if e < tol_abs:
        return True
    if e_prev is not None and max(e, e_prev) > 0.0 and abs(e - e_prev) / max(e, e_prev) < tol_rel:
        return True
    return False


def bb_pgd(Aop, b, x0=None, tau0=1.0, k_max=200, tol_abs=1e-8, tol_rel=1e-8):
    """BB-PGD: x+ = (x - tau_bb (A x + b))_+ with eta = 1 (eq. (spectralStepSize), Table 1).

    tau_bb = |dx|^2 / dx.(A x - A x_prev); the first step uses tau0. One
    product per iteration.
    """
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    mvp = 0
    if np.any(x != 0.0):
        Ax = Aop(x)
        mvp += 1
    else:
        Ax = np.zeros(n)
    xp = Axp = None
    tau = tau0
    e_prev = None
    conv = False
    hist = []
    for k in range(k_max):
        g = Ax + b
        e = kkt_error(x, g)
        hist.append(e)
        if _converged(e, e_prev, tol_abs, tol_rel):
            conv = True
            break
        e_prev = e
        if xp is not None:
            dx, dg = x - xp, Ax - Axp
            den = float(dx @ dg)
            if den > 0.0:
                tau = float(dx @ dx) / den
        xn = np.maximum(x - tau * g, 0.0)
        Axn = Aop(xn)
        mvp += 1
        xp, Axp, x, Ax = x, Ax, xn, Axn
    else:
        e = kkt_error(x, Ax + b)
        hist.append(e)
        conv = _converged(e, e_prev, tol_abs, tol_rel)
    return x, Ax, Stats(iters=len(hist) - 1, mvp=mvp, kkt=hist[-1], converged=conv, hist=hist)


def mono_pqn(Aop, b, x0=None, Ax0=None, k_max=100, tol_abs=1e-8, tol_rel=1e-8,
             pairs=(), j_max=50, sigma=None, ssn_tol=1e-14, printed_metric=False):
    """Mono-PQN (Alg. 1) with the SSN prox (Alg. 3) and eta* (Alg. 2).

    sigma: scale of the initial metric B0 = sigma I; None = set from the first
    step's curvature p.Ap/p.p. printed_metric=True is Alg. 1 as printed,
    H^(0) = I (sigma = 1) at the start and after every memory reset.

    One product A[p] per iteration; A x is carried by the recurrence
    A x+ = A x + eta A p (Remark after Alg. 2). `pairs` are secant pairs
    (s, y) replayed into the memory before the first step (Bi-PQN warm start).
    Returns (x, A x, stats) with stats['S'], stats['Y'] the accepted pairs.
    """
    n = b.size
    if printed_metric:
        sigma = 1.0
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    mvp = 0
    if Ax0 is not None:
        Ax = np.array(Ax0, dtype=np.float64)
    elif np.any(x != 0.0):
        Ax = Aop(x)
        mvp += 1
    else:
        Ax = np.zeros(n)
    pairs = list(pairs)
    if pairs and sigma is None:
        raise ValueError('warm-start pairs need the metric scale sigma they were built with')
    qn = QuasiNewton(n, sigma=1.0 if sigma is None else sigma)
    for s, y in pairs:
        qn.update(s, y)
    e_prev = None
    conv = False
    hist = []
    ssn_total = 0
    resets = 0
    for k in range(k_max):
        g = Ax + b
        e = kkt_error(x, g)
        hist.append(e)
        if _converged(e, e_prev, tol_abs, tol_rel):
            conv = True
            break
        e_prev = e
        xt = x - qn.H_apply(g)
        Um = np.array(qn.U).T if qn.U else None
        Vm = np.array(qn.V).T if qn.V else None
        xh, nj, _ = prox_ssn(xt, Um, Vm, d=np.full(n, qn.sigma), jmax=j_max, eps_rel=ssn_tol)
        ssn_total += nj
        p = xh - x
        if not np.any(p != 0.0):
            conv = True
            break
        Ap = Aop(p)
        mvp += 1
        if sigma is None:
            pAp = float(p @ Ap)
            sigma = pAp / float(p @ p) if pAp > 0.0 else 1.0
            qn.sigma = sigma
        eta, reset = step_size(g, x, p, Ap)
        if reset:
            resets += 1
            qn = QuasiNewton(n, sigma=sigma)
        x = np.maximum(x + eta * p, 0.0)
        Ax = Ax + eta * Ap
        qn.update(eta * p, eta * Ap)
    else:
        e = kkt_error(x, Ax + b)
        hist.append(e)
        conv = _converged(e, e_prev, tol_abs, tol_rel)
    return x, Ax, Stats(iters=len(hist) - 1, mvp=mvp, kkt=hist[-1], converged=conv,
                        hist=hist, S=list(qn.S), Y=list(qn.Y), ssn=ssn_total, sigma=sigma, resets=resets)


def secant_transfer(S, Y, u, v):
    """Re-target secant pairs of B^(k) to B^(k+1) = B^(k) + u u^T - v v^T (Sec. 5.2).

    B^(k) S = Y implies B^(k+1) S = Y + (u u^T - v v^T) S, so S is kept and
    Y becomes Y + u (u.S) - v (v.S).
    Pinned by: B^(k+1) S = Y_new (tests/test_oracle_lcp.py).
    """
    return list(S), [yh + u * (u @ sh) - v * (v @ sh) for sh, yh in zip(S, Y)]


def bi_pqn(Ahi, Alo, b, k_max=50, k_max_inner=50, tol_abs=1e-8, tol_rel=1e-8, j_max=50, x0=None,
           ssn_tol=1e-14, printed_metric=False):
    """Bi-PQN (Alg. 4, App. E).

    x^(0) from Mono-PQN on the low-fidelity matrix; then per outer step the
    subproblem eq. (pqnSubproblem) with B^(k) = A^ + U U^T - V V^T is solved
    by Mono-PQN using only low-fidelity products, warm-started with the
    transferred secant pairs; one high-fidelity product A[p] per outer step;
    eta* by Alg. 2 on the high-fidelity A; BFGS correction of B^(k) with
    B^(k) s = A^ s + (U U^T - V V^T) s, where A^ s = eta (A^ x^ - A^ x)
    (App. E.2) costs no product.

    Model safeguard (not in the paper, which takes B^(k) positive definite):
    when a low-fidelity solve meets a step with non-positive curvature or no
    descent (the Alg. 2 edge cases, on the model), the model is rejected and
    the solve continues as Mono-PQN on A from the current iterate; the
    products of both phases are counted.
    """
    n = b.size
    # x^(-1): the caller's guess projected on x >= 0 (0 if none); the initial solve's
    # tolerance is 1e-2 x the low-fidelity KKT error there (|min(0, b)| at 0)
    xs = np.zeros(n) if x0 is None else np.maximum(np.asarray(x0, dtype=np.float64), 0.0)
    mvp_lo = 0
    Alox = np.zeros(n)
    if np.any(xs != 0.0):
        Alox = Alo(xs)
        mvp_lo += 1
    tol0 = max(1e-12, 1e-2 * kkt_error(xs, Alox + b))
    x, Alox, st0 = mono_pqn(Alo, b, xs, Alox, k_max=k_max_inner,
                            tol_abs=tol0, tol_rel=tol_rel, j_max=j_max, ssn_tol=ssn_tol,
                            printed_metric=printed_metric)
    mvp_lo += st0['mvp']

    def fallback(x0, Ax0, mvp_hi, mvp_lo, k_done, hist):
        xm, Axm, sm = mono_pqn(Ahi, b, x0, Ax0, k_max=max(1, k_max - k_done), tol_abs=tol_abs,
                               tol_rel=tol_rel, j_max=j_max, ssn_tol=ssn_tol,
                               printed_metric=printed_metric)
        return xm, Axm, Stats(iters=len(hist) + sm['iters'], mvp_hi=mvp_hi + sm['mvp'], mvp_lo=mvp_lo,
                              kkt=sm['kkt'], converged=sm['converged'], hist=hist + sm['hist'], fallback=True)

    if st0['resets'] > 0:
        return fallback(xs, None if np.any(xs != 0.0) else np.zeros(n), 0, mvp_lo, 0, [])
    S, Y = st0['S'], st0['Y']
    sigma = st0['sigma']
    if np.any(x != 0.0):
        Ax = Ahi(x)
        mvp_hi = 1
    else:
        Ax = np.zeros(n)
        mvp_hi = 0
    corr = QuasiNewton(n)            # holds the high-fidelity corrections U, V only
    e_prev = None
    conv = False
    hist = []
    for k in range(k_max):
        g = Ax + b
        e = kkt_error(x, g)
        hist.append(e)
        if _converged(e, e_prev, tol_abs, tol_rel):
            conv = True
            break
        e_prev = e
        Bx = Alox + corr.lowrank(x)
        c = g - Bx
        Bop = lambda v: Alo(v) + corr.lowrank(v)
        tol_in = max(1e-12, 1e-2 * e)
        xh, Bxh, st = mono_pqn(Bop, c, x, Bx, k_max=k_max_inner, tol_abs=tol_in,
                               tol_rel=tol_rel, pairs=list(zip(S, Y)), j_max=j_max, sigma=sigma,
                               ssn_tol=ssn_tol)
        mvp_lo += st['mvp']
        sigma = st['sigma']
        if st['resets'] > 0:
            return fallback(x, Ax, mvp_hi, mvp_lo, k, hist)
        p = xh - x
        if not np.any(p != 0.0):
            conv = True
            break
        Ap = Ahi(p)
        mvp_hi += 1
        eta, reset = step_size(g, x, p, Ap)
        Aloxh = Bxh - corr.lowrank(xh)
        Alos = eta * (Aloxh - Alox)
        s, y = eta * p, eta * Ap
        Bs = Alos + corr.lowrank(s)
        Shat, Yhat = st['S'], st['Y']
        if reset:
            # memory reset (Alg. 2 edge case): B^(k+1) restarts from A^, and the
            # stored subproblem pairs, secants of the discarded B^(k), are dropped
            corr = QuasiNewton(n)
            Shat, Yhat = [], []
            Bs = Alos.copy()
        nu = len(corr.U)
        if corr.update(s, y, Bs=Bs):
            S, Y = secant_transfer(Shat, Yhat, corr.U[nu], corr.V[nu])
        else:
            S, Y = list(Shat), list(Yhat)
        x = np.maximum(x + eta * p, 0.0)
        Ax = Ax + eta * Ap
        Alox = Alox + Alos
    else:
        e = kkt_error(x, Ax + b)
        hist.append(e)
        conv = _converged(e, e_prev, tol_abs, tol_rel)
    return x, Ax, Stats(iters=len(hist) - 1, mvp_hi=mvp_hi, mvp_lo=mvp_lo, kkt=hist[-1],
                        converged=conv, hist=hist, fallback=False)


def bi_pqn_rec(ops, b, k_max=50, k_max_inner=50, tol_abs=1e-8, tol_rel=1e-8, j_max=50, x0=None,
               ssn_tol=1e-14, printed_metric=False):
    """Recursive Bi-PQN over a hierarchy of fidelities (the extension of Sec. 7).

    ops[0] is the high-fidelity product A[.], ops[1], ops[2], ... ever cheaper
    models. Every subproblem of Bi-PQN is itself a non-negativity constrained
    quadratic program whose quadratic term is a (corrected) mobility product,
    so it is solved by Bi-PQN one fidelity down, and by Mono-PQN at the lowest
    fidelity. With two operators this is bi_pqn step for step.

    Level d minimises 1/2 z.H_d z + c.z over z >= 0, H_d = ops[d] + C_0 + ...
    + C_{d-1}, the C_e being the BFGS corrections (U U^T - V V^T) of the
    enclosing levels. A Bi-PQN level d models H_d by L_d + C_d with
    L_d = ops[d+1] + C_0 + ... + C_{d-1}; it learns C_d from its own steps
    exactly as bi_pqn (App. E.2: L_d s from L_d x^ - L_d x, no product).
    Readings (the paper only sketches the variant):
      * The top level keeps Alg. 4's initial solve from x = 0 (itself solved
        one level down). A nested level starts at the caller's iterate x with
        H_d x known and pays one product of ops[d+1] for L_d x (none if x = 0).
      * Secant pairs warm-start only a Mono-PQN subproblem (the lowest level).
        A nested Bi-PQN level keeps its correction C_d from one call to the
        next: H_d - L_d = ops[d] - ops[d+1] does not involve the enclosing
        corrections, so the secant information C_d holds stays valid when
        they change (a memory reset at level d clears it).
      * Tolerances: 1e-2 x the level's current KKT error (floor 1e-12), at most
        k_max_inner outer steps per nested level and products per Mono-PQN.
      * Model safeguard per level, as in bi_pqn: when the subproblem solve
        meets the Alg. 2 edge cases on its own operator (its steps, or the
        Mono-PQN it fell back to), the level finishes as Mono-PQN on H_d from
        its current iterate. A level reports those edge cases of its own
        steps and of its fallback to the caller.

    Returns (x, A x, stats) with stats['mvp'] = products per fidelity.
    """
    n = b.size
    nf = len(ops)
    if nf < 2:
        raise ValueError('recursive Bi-PQN needs at least two fidelities')
    cnt = [0] * nf
    kept = {}   # correction of each nested Bi-PQN level, kept across its calls

    def op(d, corrs):
        def H(v):
            cnt[d] += 1
            out = ops[d](v)
            for c in corrs:
                out = out + c.lowrank(v)
            return out
        return H

    def solve(d, corrs, c, x, Hx, tol, k_lim, pairs, sigma, top=False):
        H = op(d, corrs)
        if d == nf - 1:
            xs, Hxs, st = mono_pqn(H, c, x, Hx, k_max=k_lim, tol_abs=tol, tol_rel=tol_rel,
                                   pairs=pairs, j_max=j_max, sigma=sigma, ssn_tol=ssn_tol,
                                   printed_metric=printed_metric)
            return xs, Hxs, dict(resets=st['resets'], S=st['S'], Y=st['Y'], sigma=st['sigma'],
                                 iters=st['iters'], kkt=st['kkt'], converged=st['converged'],
                                 hist=st['hist'], fallback=False)
        last_in = d + 1 == nf - 1
        L = op(d + 1, corrs)
        resets = 0

        def fallback(x0, Hx0, k_done, hist):
            xm, Hxm, sm = mono_pqn(H, c, x0, Hx0, k_max=max(1, k_lim - k_done), tol_abs=tol,
                                   tol_rel=tol_rel, j_max=j_max, ssn_tol=ssn_tol,
                                   printed_metric=printed_metric)
            return xm, Hxm, dict(resets=resets + sm['resets'], S=[], Y=[], sigma=sigma,
                                 iters=len(hist) + sm['iters'], kkt=sm['kkt'],
                                 converged=sm['converged'], hist=hist + sm['hist'], fallback=True)

        if top:
            # from x^(-1) (the caller's guess, or 0): tolerance 1e-2 x the model's KKT error there
            xs = x
            Lx = L(x) if np.any(x != 0.0) else np.zeros(n)
            tol0 = max(1e-12, 1e-2 * kkt_error(x, Lx + c))
            x, Lx, si = solve(d + 1, corrs, c, x, Lx, tol0, k_max_inner, [], None)
            if si['resets'] > 0:
                return fallback(xs, None if np.any(xs != 0.0) else np.zeros(n), 0, [])
            S, Y = (si['S'], si['Y']) if last_in else ([], [])
            sigma = si['sigma']
            Hx = H(x) if np.any(x != 0.0) else np.zeros(n)
        else:
            Lx = L(x) if np.any(x != 0.0) else np.zeros(n)
            S, Y = [], []
        corr = QuasiNewton(n) if top else kept.setdefault(d, QuasiNewton(n))
        e_prev = None
        conv = False
        hist = []
        for k in range(k_lim):
            g = Hx + c
            e = kkt_error(x, g)
            hist.append(e)
            if _converged(e, e_prev, tol, tol_rel):
                conv = True
                break
            e_prev = e
            Bx = Lx + corr.lowrank(x)
            tol_in = max(1e-12, 1e-2 * e)
            xh, Bxh, si = solve(d + 1, corrs + [corr], g - Bx, x, Bx, tol_in, k_max_inner,
                                list(zip(S, Y)) if last_in else [], sigma)
            sigma = si['sigma']
            if si['resets'] > 0:
                return fallback(x, Hx, k, hist)
            p = xh - x
            if not np.any(p != 0.0):
                conv = True
                break
            Hp = H(p)
            eta, reset = step_size(g, x, p, Hp)
            Ls = eta * (Bxh - corr.lowrank(xh) - Lx)
            s, y = eta * p, eta * Hp
            Bs = Ls + corr.lowrank(s)
            Shat, Yhat = (si['S'], si['Y']) if last_in else ([], [])
            if reset:
                resets += 1
                corr = QuasiNewton(n)
                if not top:
                    kept[d] = corr
                Shat, Yhat = [], []
                Bs = Ls.copy()
            nu = len(corr.U)
            if corr.update(s, y, Bs=Bs):
                S, Y = secant_transfer(Shat, Yhat, corr.U[nu], corr.V[nu])
            else:
                S, Y = list(Shat), list(Yhat)
            x = np.maximum(x + eta * p, 0.0)
            Hx = Hx + eta * Hp
            Lx = Lx + Ls
        else:
            e = kkt_error(x, Hx + c)
            hist.append(e)
            conv = _converged(e, e_prev, tol, tol_rel)
        return x, Hx, dict(resets=resets, S=[], Y=[], sigma=sigma, iters=len(hist) - 1, kkt=hist[-1],
                           converged=conv, hist=hist, fallback=False)

    xs = np.zeros(n) if x0 is None else np.maximum(np.asarray(x0, dtype=np.float64), 0.0)
    x, Ax, st = solve(0, [], b, xs, None, tol_abs, k_max, [], None, top=True)
    return x, Ax, Stats(iters=st['iters'], mvp=list(cnt), mvp_hi=cnt[0], mvp_lo=sum(cnt[1:]),
                        kkt=st['kkt'], converged=st['converged'], hist=st['hist'],
                        fallback=st['fallback'])
