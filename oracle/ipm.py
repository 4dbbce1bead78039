"""Reference infeasible long-step IPM (Alg. 2) in plain FP64 NumPy/SciPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two inner solvers follow the paper:
  * "exact": the normal equations A D^2 A^T dy = p (eq. normal) solved by a
    dense Cholesky factorisation.  Then A D^2 A^T dy - p = 0, so the
    correction vector of eq. compv is zero and the direction is eq. system.
    This is the "IPM w/ Dir." column of the experiments (Sec. 6, Table 1).
  * "sketch": Alg. 1 - sketch B = A D W, SVD of B, Q^{-1/2} = U diag(1/sv) U^T,
    standard CG from z = 0 on eq. precond_alt, dy = Q^{-1/2} z (Alg. 2 step c);
    then v of eq. compv with (ADW)^+ = V diag(1/sv) U^T (proof of Lemma 4),
    ds of eq. delshat and dx of eq. delxhat (Alg. 2 step d).

Readings of points the paper leaves open (each also used by the GPU library):
  * residual dimensions: r_p = A x - b has m entries, r_d = A^T y + s - c has n
    (the introduction swaps them); ||r|| is the 2-norm of the concatenation.
  * neighbourhood N(gamma) (Sec. 4): x_i s_i >= (1-gamma) mu(alpha) uses the
    candidate point's own mu(alpha); the residual part ||r(alpha)||/||r0|| <=
    mu(alpha)/mu0 is evaluated with ||r(alpha)|| = (1-alpha)||r^k||, which is
    what the residual invariant (eq. addl) gives.
  * step (e): alpha_max is the first exit from N(gamma) along [0, 1]; each
    condition is a quadratic in alpha whose first sign change is found in closed
    form (`first_exit`).  A positivity guard keeps alpha_max below
    (1 - guard) times the distance to the boundary of x, s > 0.
  * step (f): the minimiser of the quadratic mu(alpha) on [0, alpha_max]
    (ties go to the larger alpha).
  * CG stopping: ||f^(j)|| <= tol_cg ||f^(0)|| (relative residual of the
    preconditioned system, Sec. 6 "relative stopping tolerance") or a cap.
  * outer stopping: relative duality gap |c^T x - b^T y| / max(1, |c^T x|) and
    x^T s / max(1, |c^T x|) at most eps_gap, ||r_p|| <= eps_feas ||b|| and
    ||r_d|| <= eps_feas ||c||.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .sketch import gaussian_sketch_matrix, sketch_matrix


# ----------------------------------------------------------------------------
# basic quantities (Sec. 4)
# ----------------------------------------------------------------------------

def _mv(A, u):
    return np.asarray(A @ u, dtype=np.float64).ravel()


def _rmv(A, u):
    return np.asarray(A.T @ u, dtype=np.float64).ravel()


def residuals(A, b, c, x, y, s):
    """Primal and dual residuals r_p = A x - b, r_d = A^T y + s - c
    (eqs. primalres, dualres)."""
    return _mv(A, x) - b, _rmv(A, y) + s - c


def duality_measure(x, s):
    """mu = x^T s / n (Sec. 4)."""
    return float(x @ s) / x.size


def normal_rhs(A, b, c, x, y, s, sigma, mu):
    """p = -r_p - sigma mu A S^{-1} 1 + A x - A D^2 r_d  (eq. pdef), D^2 = X S^{-1}."""
    rp, rd = residuals(A, b, c, x, y, s)
    d2 = x / s
    return -rp - sigma * mu * _mv(A, 1.0 / s) + _mv(A, x) - _mv(A, d2 * rd)


def normal_matrix(A, d2):
    """A D^2 A^T as a dense m x m array (eq. normal)."""
    if sp.issparse(A):
        return np.asarray((A @ sp.diags(d2) @ A.T).todense())
    return (A * d2) @ A.T


def scaled_matrix(A, d):
    """A D as a dense array (sparse A is densified: only for small tests)."""
    if sp.issparse(A):
        return np.asarray((A @ sp.diags(d)).todense())
    return A * d


# ----------------------------------------------------------------------------
# step length (Alg. 2 steps e, f)
# ----------------------------------------------------------------------------

def first_exit(qa, qb, qc):
    """Smallest alpha >= 0 at which q(alpha) = qa alpha^2 + qb alpha + qc becomes
    negative, for qc >= 0 (inf if q stays non-negative on [0, inf)).  Roots are
    taken in the cancellation-free form qq = -(qb + sgn(qb) sqrt(disc))/2,
    roots qq/qa and qc/qq."""
    qa, qb, qc = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in
                  np.broadcast_arrays(qa, qb, qc))
    out = np.full(qa.shape, np.inf)
    zero = qc == 0.0
    # q(0) = 0: the sign just after 0 is that of qb, or of qa when qb = 0
    out[zero & (qb < 0)] = 0.0
    out[zero & (qb == 0) & (qa < 0)] = 0.0
    sel = zero & (qb > 0) & (qa < 0)
    out[sel] = -qb[sel] / qa[sel]
    pos = qc > 0.0
    # linear
    sel = pos & (qa == 0) & (qb < 0)
    out[sel] = -qc[sel] / qb[sel]
    disc = qb * qb - 4.0 * qa * qc
    sq = np.sqrt(np.maximum(disc, 0.0))
    sgn = np.where(qb >= 0, 1.0, -1.0)
    qq = -0.5 * (qb + sgn * sq)
    # concave: exactly one positive root
    sel = pos & (qa < 0) & (qb >= 0)
    out[sel] = qq[sel] / qa[sel]
    sel = pos & (qa < 0) & (qb < 0)
    out[sel] = qc[sel] / qq[sel]
    # convex with two positive roots: the smaller one is qc/qq
    sel = pos & (qa > 0) & (qb < 0) & (disc > 0)
    out[sel] = qc[sel] / qq[sel]
    return out


@dataclasses.dataclass
class StepInfo:
    alpha_max: float
    alpha: float
    a0: float   # x^T s
    a1: float   # x^T ds + s^T dx
    a2: float   # dx^T ds


def step_length(x, s, dx, ds, gamma, mu0, eta, guard):
    """Alg. 2 steps (e) and (f).  mu(alpha) n = a0 + a1 alpha + a2 alpha^2.

    (e) alpha_max = first exit from N(gamma) on [0, 1]:
        x_i(alpha) s_i(alpha) >= (1-gamma) mu(alpha)   for every i, and
        (1-alpha) eta <= mu(alpha)/mu0                 (eta = ||r^k||/||r^0||),
        further capped by (1-guard) x the step to the boundary of x, s > 0.
    (f) alpha = argmin of mu(alpha) on [0, alpha_max]."""
    n = x.size
    a0 = float(x @ s)
    a1 = float(x @ ds + s @ dx)
    a2 = float(dx @ ds)
    g1 = 1.0 - gamma
    qa = dx * ds - g1 * a2 / n
    qb = x * ds + s * dx - g1 * a1 / n
    qc = np.maximum(x * s - g1 * a0 / n, 0.0)
    amax = min(1.0, float(first_exit(qa, qb, qc).min()))
    t = n * mu0 * eta
    amax = min(amax, float(first_exit(a2, a1 + t, max(a0 - t, 0.0))[0]))
    bound = np.inf
    if np.any(dx < 0):
        bound = min(bound, float(np.min(-x[dx < 0] / dx[dx < 0])))
    if np.any(ds < 0):
        bound = min(bound, float(np.min(-s[ds < 0] / ds[ds < 0])))
    amax = min(amax, (1.0 - guard) * bound)
    if a2 > 0:
        alpha = min(max(-a1 / (2.0 * a2), 0.0), amax)
    else:
        alpha = amax if a1 + a2 * amax <= 0 else 0.0
    return StepInfo(amax, alpha, a0, a1, a2)


def in_neighbourhood(x, s, gamma, mu, eta_ratio, mu_ratio):
    """Membership test for N(gamma): x_i s_i >= (1-gamma) mu and ||r||/||r0|| <= mu/mu0."""
    return bool(np.all(x * s >= (1.0 - gamma) * mu) and eta_ratio <= mu_ratio)


# ----------------------------------------------------------------------------
# Alg. 1: sketch-preconditioned CG
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PCGResult:
    z: np.ndarray          # CG iterate of eq. precond_alt
    dy: np.ndarray         # Q^{-1/2} z
    Qmh: np.ndarray        # Q^{-1/2}
    U: np.ndarray          # left singular vectors of A D W
    sv: np.ndarray         # singular values of A D W
    Vh: np.ndarray         # right singular vectors (rows) of A D W
    iters: int
    f_norms: list          # ||f^(j)||, j = 0..iters


def sketch_preconditioner(AD, W):
    """Alg. 1 steps 1-2: B = A D W, its thin SVD, and Q^{-1/2} = U diag(1/sv) U^T."""
    B = np.asarray((W.T @ AD.T).T) if sp.issparse(W) else AD @ W
    U, sv, Vh = np.linalg.svd(B, full_matrices=False)
    if sv.size < AD.shape[0] or sv[-1] <= 0 or not np.all(np.isfinite(sv)):
        raise np.linalg.LinAlgError("rank(A D W) < m")
    return (U / sv) @ U.T, U, sv, Vh


def sketch_richardson(AD, p, W, t=None, tol=None, max_it=1000):
    """Alg. 3 (App. A): z^j = z^{j-1} + Q^{-1/2}(p - A D^2 A^T Q^{-1/2} z^{j-1})
    from z^0 = 0, for exactly t iterations, or until ||f^(j)|| <= tol ||f^(0)||
    with f^(j) = Q^{-1/2}(A D^2 A^T Q^{-1/2} z^j - p)."""
    Qmh, U, sv, Vh = sketch_preconditioner(AD, W)

    def residual(z):
        return Qmh @ (AD @ (AD.T @ (Qmh @ z))) - Qmh @ p

    z = np.zeros_like(p)
    f = residual(z)
    f_norms = [float(np.linalg.norm(f))]
    limit = t if t is not None else max_it
    it = 0
    while it < limit:
        if t is None and f_norms[-1] <= tol * f_norms[0]:
            break
        z = z + Qmh @ (p - AD @ (AD.T @ (Qmh @ z)))
        f = residual(z)
        it += 1
        f_norms.append(float(np.linalg.norm(f)))
    return PCGResult(z, Qmh @ z, Qmh, U, sv, Vh, it, f_norms)


def sketch_sd(AD, p, W, t=None, tol=None, max_it=1000):
    """Alg. 4 (App. B): steepest descent on Q^{-1/2} A D^2 A^T Q^{-1/2} z =
    Q^{-1/2} p from z^0 = 0: alpha_j = f^T f / f^T M f, z^{j+1} = z^j - alpha_j f^(j),
    M = Q^{-1/2} A D^2 A^T Q^{-1/2}; stops as sketch_richardson."""
    Qmh, U, sv, Vh = sketch_preconditioner(AD, W)

    def op(u):
        return Qmh @ (AD @ (AD.T @ (Qmh @ u)))

    z = np.zeros_like(p)
    f = op(z) - Qmh @ p
    f_norms = [float(np.linalg.norm(f))]
    limit = t if t is not None else max_it
    it = 0
    while it < limit:
        if t is None and f_norms[-1] <= tol * f_norms[0]:
            break
        ff = float(f @ f)
        if ff == 0.0:
            break
        alpha = ff / float(f @ op(f))
        z = z - alpha * f
        f = op(z) - Qmh @ p
        it += 1
        f_norms.append(float(np.linalg.norm(f)))
    return PCGResult(z, Qmh @ z, Qmh, U, sv, Vh, it, f_norms)


def sketch_pcg(AD, p, W, t=None, tol=None, max_it=1000):
    """Alg. 1.  Step 1: B = A D W and its thin SVD.  Step 2: Q^{-1/2} =
    U diag(1/sv) U^T.  Step 3: standard CG from z = 0 on
    Q^{-1/2} A D^2 A^T Q^{-1/2} z = Q^{-1/2} p, for exactly t iterations, or until
    ||f^(j)|| <= tol ||f^(0)|| (at most max_it iterations)."""
    Qmh, U, sv, Vh = sketch_preconditioner(AD, W)

    def op(u):
        h = Qmh @ u
        return Qmh @ (AD @ (AD.T @ h))

    rhs = Qmh @ p
    z = np.zeros_like(p)
    r = rhs.copy()          # r = rhs - op(z) = -f
    d = r.copy()
    rr = float(r @ r)
    f_norms = [math.sqrt(rr)]
    limit = t if t is not None else max_it
    it = 0
    while it < limit:
        if t is None and f_norms[-1] <= tol * f_norms[0]:
            break
        if rr == 0.0:
            break
        od = op(d)
        alpha = rr / float(d @ od)
        z = z + alpha * d
        r = r - alpha * od
        rr_new = float(r @ r)
        d = r + (rr_new / rr) * d
        rr = rr_new
        it += 1
        f_norms.append(math.sqrt(rr))
    return PCGResult(z, Qmh @ z, Qmh, U, sv, Vh, it, f_norms)


def correction_vector(x, s, W, U, sv, Vh, g):
    """eq. compv: v = (XS)^{1/2} W (A D W)^+ g, with (A D W)^+ = V diag(1/sv) U^T
    and g = A D^2 A^T dy - p."""
    t = Vh.T @ ((U.T @ g) / sv)
    return np.sqrt(x * s) * _mv(W, t)


# ----------------------------------------------------------------------------
# one IPM direction, and the loop (Alg. 2)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Direction:
    dx: np.ndarray
    dy: np.ndarray
    ds: np.ndarray
    v: np.ndarray
    p: np.ndarray
    rp: np.ndarray
    rd: np.ndarray
    mu: float
    cg_iters: int = 0
    f_norm: float = 0.0
    pcg: PCGResult | None = None


def exact_direction(A, b, c, x, y, s, sigma):
    """eq. system with the normal equations solved by Cholesky; v = 0."""
    rp, rd = residuals(A, b, c, x, y, s)
    mu = duality_measure(x, s)
    d2 = x / s
    p = normal_rhs(A, b, c, x, y, s, sigma, mu)
    N = normal_matrix(A, d2)
    cf = sla.cho_factor(N, lower=True)
    dy = sla.cho_solve(cf, p)
    ds = -rd - _rmv(A, dy)
    dx = -x + sigma * mu / s - d2 * ds
    return Direction(dx, dy, ds, np.zeros_like(x), p, rp, rd, mu)


INNER_SOLVERS = {"cg": sketch_pcg, "sd": sketch_sd, "richardson": sketch_richardson}


def sketch_direction(A, b, c, x, y, s, sigma, W, tol_cg=1e-5, max_cg=1000, t=None,
                     inner="cg"):
    """Alg. 2 steps (b)-(d) with W from step (a); step (c)'s solver is CG
    (Alg. 1), steepest descent (Alg. 4) or Richardson (Alg. 3)."""
    rp, rd = residuals(A, b, c, x, y, s)
    mu = duality_measure(x, s)
    d2 = x / s
    p = normal_rhs(A, b, c, x, y, s, sigma, mu)
    AD = scaled_matrix(A, np.sqrt(d2))
    res = INNER_SOLVERS[inner](AD, p, W, t=t, tol=tol_cg, max_it=max_cg)
    dy = res.dy
    g = _mv(A, d2 * _rmv(A, dy)) - p
    v = correction_vector(x, s, W, res.U, res.sv, res.Vh, g)
    ds = -rd - _rmv(A, dy)
    dx = -x + sigma * mu / s - d2 * ds - v / s
    return Direction(dx, dy, ds, v, p, rp, rd, mu, res.iters, res.f_norms[-1], res)


@dataclasses.dataclass
class IPMParams:
    solver: str = "exact"       # "exact" | "sketch"
    sigma: float = 0.5
    gamma: float = 0.999
    eps_gap: float = 1e-6
    eps_feas: float = 1e-8
    guard: float = 1e-3
    max_outer: int = 300
    w: int = 0                  # sketch width (0: 4m)
    s_nnz: int = 1              # non-zeros per row of W
    seed: int = 0
    resketch: bool = True       # fresh W every iteration (salt = iteration index)
    tol_cg: float = 1e-5
    max_cg: int = 1000
    cg_t: int | None = None     # fixed CG iteration count instead of tol_cg
    inner: str = "cg"           # "cg" (Alg. 1) | "sd" (Alg. 4) | "richardson" (Alg. 3)
    sketch: str = "count"       # "count" (Sec. 2) | "gaussian" (W_G of Sec. 5)


@dataclasses.dataclass
class IPMResult:
    status: str
    iters: int
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    obj_p: float
    obj_d: float
    rel_gap: float
    rp_norm: float
    rd_norm: float
    history: list


def stop_test(A, b, c, x, y, s, eps_gap, eps_feas):
    rp, rd = residuals(A, b, c, x, y, s)
    ctx, bty = float(c @ x), float(b @ y)
    den = max(1.0, abs(ctx))
    rel_gap = abs(ctx - bty) / den
    ok = (rel_gap <= eps_gap and float(x @ s) <= eps_gap * den
          and np.linalg.norm(rp) <= eps_feas * np.linalg.norm(b)
          and np.linalg.norm(rd) <= eps_feas * np.linalg.norm(c))
    return ok, rp, rd, ctx, bty, rel_gap


def ipm(A, b, c, params: IPMParams | None = None, x0=None, y0=None, s0=None):
    """Alg. 2 from the start (x, y, s) = (1, 0, 1) unless given."""
    prm = params or IPMParams()
    m, n = A.shape
    x = np.ones(n) if x0 is None else np.array(x0, dtype=np.float64)
    y = np.zeros(m) if y0 is None else np.array(y0, dtype=np.float64)
    s = np.ones(n) if s0 is None else np.array(s0, dtype=np.float64)
    rp0, rd0 = residuals(A, b, c, x, y, s)
    r0 = math.hypot(np.linalg.norm(rp0), np.linalg.norm(rd0))
    mu0 = duality_measure(x, s)
    w = prm.w if prm.w else 4 * m
    history = []
    status = "max_outer"
    small = 0
    k = 0
    for k in range(prm.max_outer + 1):
        ok, rp, rd, ctx, bty, rel_gap = stop_test(A, b, c, x, y, s, prm.eps_gap,
                                                  prm.eps_feas)
        if ok:
            status = "optimal"
            break
        if k == prm.max_outer:
            break
        if not (np.all(np.isfinite(x)) and np.all(np.isfinite(s))):
            status = "nan"
            break
        eta = math.hypot(np.linalg.norm(rp), np.linalg.norm(rd)) / r0 if r0 > 0 else 0.0
        try:
            if prm.solver == "exact":
                dirn = exact_direction(A, b, c, x, y, s, prm.sigma)
            else:
                salt = k if prm.resketch else 0
                if prm.sketch == "gaussian":
                    W = gaussian_sketch_matrix(prm.seed, salt, n, w)
                else:
                    W = sketch_matrix(prm.seed, salt, prm.s_nnz, n, w)
                dirn = sketch_direction(A, b, c, x, y, s, prm.sigma, W, prm.tol_cg,
                                        prm.max_cg, prm.cg_t, prm.inner)
        except np.linalg.LinAlgError:
            status = "numerical"
            break
        st = step_length(x, s, dirn.dx, dirn.ds, prm.gamma, mu0, eta, prm.guard)
        history.append(dict(k=k, mu=dirn.mu, rp=float(np.linalg.norm(rp)),
                            rd=float(np.linalg.norm(rd)), eta=eta, rel_gap=rel_gap,
                            alpha_max=st.alpha_max, alpha=st.alpha,
                            cg_iters=dirn.cg_iters, v_norm=float(np.linalg.norm(dirn.v))))
        small = small + 1 if st.alpha < 1e-12 else 0
        if small >= 3:
            status = "stall"
            break
        x = x + st.alpha * dirn.dx
        y = y + st.alpha * dirn.dy
        s = s + st.alpha * dirn.ds
    rp, rd = residuals(A, b, c, x, y, s)
    ctx, bty = float(c @ x), float(b @ y)
    return IPMResult(status, k, x, y, s, ctx, bty, abs(ctx - bty) / max(1.0, abs(ctx)),
                     float(np.linalg.norm(rp)), float(np.linalg.norm(rd)), history)
