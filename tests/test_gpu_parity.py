"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Every case prints its name before touching the GPU.  Tolerances:
  * hash buckets and signs: bit-exact;
  * sketch B: |B - B_ref| <= k u sum|terms| (k = largest bucket, order of sums differs);
  * CG iterates at a fixed iteration count: relative 1e-9 (same Krylov method,
    different rounding order); at the IPM's stopping tolerance, a tenth of the
    iterate's own distance to the exact solve;
  * CG to a tight tolerance vs Cholesky: relative 1e-8 on iterates with
    kappa(A D^2 A^T) <= 1e7;
  * invariants eq. addl / iip_3 on the GPU's own FP64 directions: 1e-12 of the
    size of the terms that cancel in them;
  * step length from the GPU's directions vs the oracle's rule: relative 1e-10;
  * final objective vs the planted optimum and the exact oracle: the stopping
    tolerance eps_gap; KKT residuals <= 1e-8 ||b||, ||c||.
"""
import contextlib
import math
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from lpgen import config_lp, dense_planted
from oracle import ipm as O
from oracle.sketch import sketch_hash as ref_hash
from oracle.sketch import sketch_matrix

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def sk():
    import paper_2003_08072_amd as _sk
    _sk.load()
    return _sk


@contextlib.contextmanager
def cg_path(path):
    """LPs created inside take the one-workgroup CG ('small', the default for
    A up to 1 MiB) or the multi-workgroup fused CG ('multi')."""
    old = os.environ.get("SKIPM_CG_SMALL_BYTES")
    if path == "multi":
        os.environ["SKIPM_CG_SMALL_BYTES"] = "0"
    else:
        os.environ.pop("SKIPM_CG_SMALL_BYTES", None)
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("SKIPM_CG_SMALL_BYTES", None)
        else:
            os.environ["SKIPM_CG_SMALL_BYTES"] = old


def mid_iterate(lp, iters):
    x, y, s = np.ones(lp.n), np.zeros(lp.m), np.ones(lp.n)
    rp0, rd0 = O.residuals(lp.A, lp.b, lp.c, x, y, s)
    r0 = math.hypot(np.linalg.norm(rp0), np.linalg.norm(rd0))
    for _ in range(iters):
        d = O.exact_direction(lp.A, lp.b, lp.c, x, y, s, 0.5)
        eta = math.hypot(np.linalg.norm(d.rp), np.linalg.norm(d.rd)) / r0
        st = O.step_length(x, s, d.dx, d.ds, 0.999, 1.0, eta, 1e-3)
        x, y, s = x + st.alpha * d.dx, y + st.alpha * d.dy, s + st.alpha * d.ds
    return x, y, s


# ---------------------------------------------------------------------------
# a2: hash (bit-exact)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,k,s,n,w", [
    (0, 0, 1, 1000, 200),
    (0x5EED0001, 7, 1, 100_000, 2000),
    (123, 3, 2, 1_000_000, 4000),
    (9, 1, 4, 12345, 64),
    (1, 0, 1, 10, 7),
    (2**63 + 5, 2**40, 3, 3001, 33),
])
def test_hash_bit_exact(torch, sk, seed, k, s, n, w):
    say(f"hash seed={seed} k={k} s={s} n={n} w={w}")
    bucket = torch.empty(n * s, dtype=torch.int32, device="cuda")
    sign = torch.empty(n * s, dtype=torch.int8, device="cuda")
    sk.sketch_hash(seed, k, s, n, w, bucket, sign)
    rb, rs = ref_hash(seed, k, s, n, w)
    assert np.array_equal(bucket.cpu().numpy(), rb.ravel().astype(np.int32))
    assert np.array_equal(sign.cpu().numpy(), rs.ravel())


# ---------------------------------------------------------------------------
# a2: sketch B = A D W
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,w,s,dtype", [
    (37, 500, 150, 2, "f64"), (50, 1000, 200, 1, "f64"), (5, 64, 8, 1, "f64"),
    (130, 3000, 520, 4, "f64"), (61, 2000, 244, 1, "f32"), (257, 2000, 1028, 2, "f64"),
])
def test_sketch_apply(torch, sk, m, n, w, s, dtype):
    say(f"sketch m={m} n={n} w={w} s={s} {dtype}")
    rng = np.random.default_rng(m * 7 + n)
    lp = dense_planted(m, n, rng=rng, a_dtype=dtype)
    d = rng.uniform(0.01, 10.0, n) * rng.choice([-1.0, 1.0], n)
    with sk.LP(lp.A, lp.b, lp.c, a_dtype=dtype, w=w, s=s, seed=77) as h:
        B = h.sketch(d, 5).cpu().numpy()
    W = sketch_matrix(77, 5, s, n, w)
    AD = lp.A * d
    Bref = np.asarray((W.T @ AD.T).T)
    bound = np.asarray((abs(W).T @ abs(AD).T).T)
    kmax = int(np.diff(W.tocsc().indptr).max())
    assert np.all(np.abs(B - Bref) <= (kmax + 2) * EPS * bound + 1e-300)


def test_sketch_apply_f32_output(torch, sk):
    """out_dtype SKIPM_F32: the FP64 sketch rounded to nearest, element by element."""
    say("sketch to FP32, m=61 n=2000 w=244 s=2")
    rng = np.random.default_rng(404)
    lp = dense_planted(61, 2000, rng=rng)
    d = rng.uniform(0.01, 10.0, 2000)
    with sk.LP(lp.A, lp.b, lp.c, w=244, s=2, seed=9) as h:
        B64 = h.sketch(d, 3).cpu().numpy()
        B32 = h.sketch(d, 3, out_dtype="f32").cpu().numpy()
    assert B32.dtype == np.float32
    assert np.array_equal(B32, B64.astype(np.float32))


# ---------------------------------------------------------------------------
# a3/a4: preconditioned CG
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cg_case():
    lp = dense_planted(40, 800, rng=np.random.default_rng(8))
    x, y, s = mid_iterate(lp, 6)
    return lp, x, s


@pytest.mark.parametrize("path", ["small", "multi"])
@pytest.mark.parametrize("t", [1, 3, 8])
def test_pcg_fixed_iterations_match_alg1(torch, sk, cg_case, t, path):
    lp, x, s = cg_case
    say(f"pcg fixed t={t} {path}")
    d2 = x / s
    p = np.random.default_rng(t).standard_normal(lp.m)
    with cg_path(path), sk.LP(lp.A, lp.b, lp.c, seed=31, s=2) as h:
        dy, info = h.pcg(d2, p, 4, tol=0.0, max_it=t)
        dy = dy.cpu().numpy()
    assert info.iters == t
    W = sketch_matrix(31, 4, 2, lp.n, lp.w)
    ref = O.sketch_pcg(lp.A * np.sqrt(d2), p, W, t=t)
    assert np.linalg.norm(dy - ref.dy) <= 1e-9 * np.linalg.norm(ref.dy)
    assert info.f_norm == pytest.approx(ref.f_norms[-1], rel=1e-6)
    assert info.f0_norm == pytest.approx(ref.f_norms[0], rel=1e-10)


@pytest.mark.parametrize("inner,t,fmt", [("sd", 1, "dense"), ("sd", 6, "dense"),
                                         ("richardson", 1, "dense"), ("richardson", 6, "dense"),
                                         ("sd", 6, "dense-multi"), ("richardson", 6, "dense-multi"),
                                         ("sd", 6, "csr"), ("richardson", 6, "csr")])
def test_inner_solvers_fixed_iterations_match_oracle(torch, sk, cg_case, inner, t, fmt):
    """Steepest descent (App. B, Alg. 4) and Richardson (App. A, Alg. 3) in place
    of CG, on a sketch wide enough for Richardson to contract (w = n, s = 8)."""
    import scipy.sparse as ssp
    lp, x, s = cg_case
    say(f"inner solver {inner} t={t} {fmt}")
    code = {"sd": sk.SKIPM_INNER_SD, "richardson": sk.SKIPM_INNER_RICHARDSON}[inner]
    d2 = x / s
    p = np.random.default_rng(40 + t).standard_normal(lp.m)
    A = ssp.csr_matrix(lp.A) if fmt == "csr" else lp.A
    with cg_path("multi" if fmt == "dense-multi" else "small"), \
            sk.LP(A, lp.b, lp.c, seed=33, s=8, w=lp.n, inner=code) as h:
        dy, info = h.pcg(d2, p, 2, tol=0.0, max_it=t)
        dy = dy.cpu().numpy()
    assert info.iters == t
    W = sketch_matrix(33, 2, 8, lp.n, lp.n)
    solver = O.sketch_sd if inner == "sd" else O.sketch_richardson
    ref = solver(lp.A * np.sqrt(d2), p, W, t=t)
    assert np.linalg.norm(dy - ref.dy) <= 1e-9 * np.linalg.norm(ref.dy)
    assert info.f_norm == pytest.approx(ref.f_norms[-1], rel=1e-6)


@pytest.mark.parametrize("inner", ["sd", "richardson"])
def test_solve_with_inner_solver(torch, sk, inner):
    lp = dense_planted(30, 1200, rng=np.random.default_rng(12), eps_gap=1e-8)
    say(f"solve with inner solver {inner} (w = n, s = 8)")
    code = {"sd": sk.SKIPM_INNER_SD, "richardson": sk.SKIPM_INNER_RICHARDSON}[inner]
    with sk.LP(lp.A, lp.b, lp.c, w=lp.n, s=8, seed=5, eps_gap=1e-8, inner=code,
               max_cg=2000) as h:
        res = h.solve()
    check_solution(lp, res, 1e-8)


# ---------------------------------------------------------------------------
# Gaussian sketch W_G (Sec. 5)
# ---------------------------------------------------------------------------

# the last two take the K-split GEMM (19 and 12 slices, each with a ragged
# remainder of columns added into the first slice)
@pytest.mark.parametrize("m,n,w,k", [(37, 500, 148, 0), (64, 2000, 256, 5), (5, 64, 20, 2),
                                     (100, 20001, 200, 1), (300, 12345, 600, 4)])
def test_gaussian_sketch_apply(torch, sk, m, n, w, k):
    from oracle.sketch import gaussian_sketch_matrix
    say(f"gaussian sketch m={m} n={n} w={w} k={k}")
    rng = np.random.default_rng(m + n)
    lp = dense_planted(m, n, rng=rng)
    d = rng.uniform(0.01, 10.0, n)
    with sk.LP(lp.A, lp.b, lp.c, w=w, seed=19, sketch=sk.SKIPM_SKETCH_GAUSSIAN) as h:
        B = h.sketch(d, k).cpu().numpy()
    W = gaussian_sketch_matrix(19, k, n, w)
    AD = lp.A * d
    Bref = AD @ W
    bound = np.abs(AD) @ np.abs(W)
    assert np.all(np.abs(B - Bref) <= 4 * n * EPS * bound + 1e-300)


def test_gaussian_pcg_fixed_iterations_match_alg1(torch, sk, cg_case):
    from oracle.sketch import gaussian_sketch_matrix
    lp, x, s = cg_case
    say("pcg with the Gaussian sketch, fixed t = 4")
    d2 = x / s
    p = np.random.default_rng(6).standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, seed=23, sketch=sk.SKIPM_SKETCH_GAUSSIAN) as h:
        dy, info = h.pcg(d2, p, 3, tol=0.0, max_it=4)
        dy = dy.cpu().numpy()
    ref = O.sketch_pcg(lp.A * np.sqrt(d2), p, gaussian_sketch_matrix(23, 3, lp.n, lp.w), t=4)
    assert info.iters == 4
    assert np.linalg.norm(dy - ref.dy) <= 1e-9 * np.linalg.norm(ref.dy)


@pytest.mark.parametrize("m,n", [(50, 1000), (33, 700), (130, 4000)])
def test_solve_with_gaussian_sketch(torch, sk, m, n):
    lp = dense_planted(m, n, rng=np.random.default_rng(m), eps_gap=1e-8)
    say(f"solve with the Gaussian sketch m={m} n={n} w=4m")
    with sk.LP(lp.A, lp.b, lp.c, w=4 * m, seed=3, eps_gap=1e-8,
               sketch=sk.SKIPM_SKETCH_GAUSSIAN) as h:
        res = h.solve()
    check_solution(lp, res, 1e-8)
    assert res.cg_max <= 40


def test_gaussian_sketch_needs_dense_fp64(torch, sk):
    import scipy.sparse as ssp
    say("gaussian sketch argument checks")
    lp = dense_planted(10, 200, rng=np.random.default_rng(2))
    for A, dt in ((lp.A, "f32"), (ssp.csr_matrix(lp.A), "f64")):
        with pytest.raises(sk.SkipmError) as e:
            sk.LP(A, lp.b, lp.c, a_dtype=dt, sketch=sk.SKIPM_SKETCH_GAUSSIAN)
        assert e.value.code == sk.SKIPM_EINVAL


def test_solve_with_one_fixed_sketch(torch, sk):
    """resketch = 0: one W (salt 0) for every IPM iteration, its bucket order
    computed once."""
    lp = config_lp(0)
    say("solve config 0 with one fixed sketch (resketch = 0), s = 2")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, s=2, seed=lp.seed, eps_gap=lp.eps_gap,
               resketch=0) as h:
        res = h.solve()
    check_solution(lp, res, lp.eps_gap)


@pytest.mark.parametrize("iters", [2, 10])
def test_pcg_tight_tolerance_matches_cholesky(torch, sk, cg_case, iters):
    lp, _, _ = cg_case
    x, y, s = mid_iterate(lp, iters)
    say(f"pcg vs cholesky at exact-IPM iterate {iters}")
    d2 = x / s
    N = (lp.A * d2) @ lp.A.T
    assert np.linalg.cond(N) <= 1e7
    p = np.random.default_rng(1).standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, seed=3) as h:
        dy, info = h.pcg(d2, p, 0, tol=1e-13, max_it=300)
        dy = dy.cpu().numpy()
    ref = np.linalg.solve(N, p)
    assert np.linalg.norm(dy - ref) <= 1e-8 * np.linalg.norm(ref)


def test_pcg_signed_permutation_sketch_one_iteration(torch, sk):
    """w = n with s = n/w... a sketch whose buckets are all distinct makes
    Q = A D^2 A^T, so CG converges in one iteration (special case of Alg. 1)."""
    rng = np.random.default_rng(2)
    lp = dense_planted(12, 60, rng=rng)
    # find a seed whose hash is injective for n = w = 60 blocks of width 1 (s = 60 is
    # out of range), so use s = 1, w >> n and search a salt with no collision
    w = 4096
    for k in range(2000):
        b, _ = ref_hash(5, k, 1, lp.n, w)
        if len(np.unique(b)) == lp.n:
            break
    else:
        pytest.skip("no injective salt found")
    say(f"pcg injective sketch k={k}")
    d2 = rng.uniform(0.1, 10.0, lp.n)
    p = rng.standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, seed=5, w=w) as h:
        dy, info = h.pcg(d2, p, k, tol=1e-10, max_it=50)
        dy = dy.cpu().numpy()
    assert info.iters == 1
    ref = np.linalg.solve((lp.A * d2) @ lp.A.T, p)
    assert np.linalg.norm(dy - ref) <= 1e-9 * np.linalg.norm(ref)


# ---------------------------------------------------------------------------
# a1, a5-a9: one IPM step from an iterate shared with the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("iters,s_nnz", [(0, 1), (4, 1), (9, 2)])
def test_ipm_step_parity(torch, sk, iters, s_nnz):
    lp = dense_planted(45, 900, rng=np.random.default_rng(33))
    x, y, s = mid_iterate(lp, iters)
    say(f"ipm_step parity from exact-IPM iterate {iters}, s={s_nnz}")
    with sk.LP(lp.A, lp.b, lp.c, seed=17, s=s_nnz) as h:
        h.set_iterate(x, y, s, reset_origin=True)
        info = h.step()
        dx, dy, ds, v = (t.cpu().numpy() for t in h.get_direction())
        rp_gpu, rd_gpu, p_gpu, g_gpu = (t.cpu().numpy() for t in h.get_residuals())
        xn, yn, sn = (t.cpu().numpy() for t in h.get_iterate())
    assert info.converged == 0 and info.status == 0
    assert info.tier == sk.SKIPM_TIER_FP64 and info.refine_steps == 1
    assert info.resketches == 0 and info.shifts == 0
    A, b, c = lp.A, lp.b, lp.c
    rp, rd = O.residuals(A, b, c, x, y, s)
    mu = float(x @ s) / lp.n
    assert info.mu == pytest.approx(mu, rel=1e-12)
    # residual norms at the rounding scale of the products that form them
    tol_rp = 64 * EPS * (np.linalg.norm(abs(A) @ abs(x)) + np.linalg.norm(b))
    tol_rd = 64 * EPS * (np.linalg.norm(abs(A).T @ abs(y)) + np.linalg.norm(s) + np.linalg.norm(c))
    assert info.rp_norm == pytest.approx(np.linalg.norm(rp), rel=1e-10, abs=tol_rp)
    assert info.rd_norm == pytest.approx(np.linalg.norm(rd), rel=1e-10, abs=tol_rd)
    p = O.normal_rhs(A, b, c, x, y, s, 0.5, mu)
    d2 = x / s
    # a1 element by element: r_p, r_d and p of eq. pdef against the oracle's
    # definitions, each within the rounding of the sums that form it
    aA = abs(A)
    assert np.all(np.abs(rp_gpu - rp) <= 8 * lp.n * EPS * (aA @ abs(x) + abs(b)))
    bnd_rd = 8 * lp.m * EPS * (aA.T @ abs(y) + abs(s) + abs(c))
    assert np.all(np.abs(rd_gpu - rd) <= bnd_rd)
    bnd_p = 8 * lp.n * EPS * (abs(b) + aA @ (0.5 * mu / s + d2 * (abs(rd) + bnd_rd)))
    assert np.all(np.abs(p_gpu - p) <= bnd_p + 8 * lp.n * EPS * (aA @ abs(x)))
    g = A @ (d2 * (A.T @ dy)) - p
    # g cancels terms of size ~||p||: compare at the rounding scale of those terms
    scale_g = np.linalg.norm(abs(A) @ (d2 * abs(A.T @ dy))) + np.linalg.norm(p)
    assert np.linalg.norm(v) > 0
    # eq. addl (Lemma 3): A S^{-1} v = A D^2 A^T dy - p
    assert np.linalg.norm(A @ (v / s) - g) <= 1e-12 * scale_g
    # eq. iip_3
    scale_1 = np.linalg.norm(abs(A) @ abs(dx)) + np.linalg.norm(rp) + scale_g
    assert np.linalg.norm(A @ dx + rp) <= 1e-12 * scale_1
    scale_2 = np.linalg.norm(rd) + np.linalg.norm(abs(A).T @ abs(dy))
    assert np.linalg.norm(A.T @ dy + ds + rd) <= 1e-12 * scale_2
    r3 = x * ds + s * dx + x * s - 0.5 * mu + v
    scale_3 = (np.linalg.norm(x * ds) + np.linalg.norm(s * dx) + np.linalg.norm(x * s)
               + np.linalg.norm(v))
    assert np.linalg.norm(r3) <= 1e-12 * scale_3
    # the direction against the oracle's Alg. 1 + eq. compv with the same W
    W = sketch_matrix(17, 0, s_nnz, lp.n, lp.w)
    ref = O.sketch_direction(A, b, c, x, y, s, 0.5, W, tol_cg=1e-5, max_cg=500)
    assert info.cg_iters == ref.cg_iters
    # eq. compv element by element, at the g of this step (the GPU's own
    # epilogue output): the oracle's v = (XS)^{1/2} W (A D W)^+ g with
    # (A D W)^+ from the SVD.  The GPU refines t on B t = g from t = 0 with
    # corrections in range(B^T), so it must reach the minimum-norm solution
    # (A D W)^+ g itself, not just some t with B t = g (Lemma 4 bounds ||v||
    # for that choice).  Forward error of t: kappa(B) ||t|| times the rounding
    # of B (sums of at most kmax terms) plus the refinement's own residual
    # ||B t - g|| / ||g|| (info.v_resid); each entry of W t adds s of them.
    Bh = A * np.sqrt(d2) @ W.toarray()
    sv_b = np.linalg.svd(Bh, compute_uv=False)
    kappa_b = sv_b[0] / sv_b[-1]
    assert kappa_b <= 1e6, kappa_b
    kmax = int(np.diff(W.tocsc().indptr).max())
    vref = O.correction_vector(x, s, W, ref.pcg.U, ref.pcg.sv, ref.pcg.Vh, g_gpu)
    t_ref = ref.pcg.Vh.T @ ((ref.pcg.U.T @ g_gpu) / ref.pcg.sv)
    assert 0 <= info.v_resid <= 1e-13
    err_t = (16 * (kmax + 2) * EPS + 2 * info.v_resid) * kappa_b * np.linalg.norm(t_ref)
    rt_xs = np.sqrt(x * s)
    assert np.all(np.abs(v - vref) <= s_nnz * err_t * rt_xs), \
        float(np.max(np.abs(v - vref) / (rt_xs * s_nnz * err_t)))
    assert s_nnz * err_t * float(np.max(rt_xs)) <= 1e-6 * float(np.max(np.abs(vref)))
    # the GPU's g is A D^2 A^T dy - p of its own dy and p, up to the rounding
    # of the cancelling terms
    g_own = A @ (d2 * (A.T @ dy)) - p_gpu
    assert np.linalg.norm(g_gpu - g_own) <= 64 * EPS * scale_g
    # Both are CG iterates stopped by Alg. 1's relative rule (reading 6:
    # ||f^(j)|| <= tol_cg ||f^(0)|| on the split system); the GPU inverts the
    # Gram matrix and the oracle takes an SVD, so their rounding differs and
    # the iterates agree only up to the truncation they both allow.  The pin:
    # the GPU's dy itself meets the stopping rule, with f = Q^{-1/2}(A D^2 A^T
    # dy - p) formed on the host from the same W (the recursive residual the
    # GPU tests drifts from the true one at the rounding level), after the same
    # number of iterations as the oracle's CG.
    Qmh = ref.pcg.Qmh
    f_gpu = Qmh @ (A @ (d2 * (A.T @ dy)) - p)
    f0 = Qmh @ p
    assert np.linalg.norm(f_gpu) <= 1e-5 * np.linalg.norm(f0) * (1 + 1e-2) + 1e-12 * np.linalg.norm(f0)
    exact = O.exact_direction(A, b, c, x, y, s, 0.5)
    assert np.linalg.norm(dy - exact.dy) <= 2 * np.linalg.norm(ref.dy - exact.dy) + \
        1e-12 * np.linalg.norm(exact.dy)
    # Alg. 2 steps (e), (f) on the GPU's own direction (origin = this iterate)
    st = O.step_length(x, s, dx, ds, 0.999, mu, 1.0, 1e-3)
    assert info.alpha_max == pytest.approx(st.alpha_max, rel=1e-10)
    assert info.alpha == pytest.approx(st.alpha, rel=1e-10)
    # step (g)
    assert np.allclose(xn, x + info.alpha * dx, rtol=1e-15, atol=1e-300)
    assert np.allclose(yn, y + info.alpha * dy, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("iters", [2, 6])
def test_ipm_step_tight_cg_gives_the_exact_direction(torch, sk, iters):
    """With tol_cg = 1e-13 the step's dy is the exact solution of eq. normal
    (the oracle's Cholesky solve from the same iterate) to relative 1e-8, on
    iterates with kappa(A D^2 A^T) <= 1e7; ds of eq. delshat follows from it."""
    lp = dense_planted(45, 900, rng=np.random.default_rng(33))
    x, y, s = mid_iterate(lp, iters)
    N = O.normal_matrix(lp.A, x / s)
    assert np.linalg.cond(N) <= 1e7
    say(f"ipm_step with tol_cg 1e-13 from exact-IPM iterate {iters}")
    with sk.LP(lp.A, lp.b, lp.c, seed=17, s=2, tol_cg=1e-13, max_cg=400) as h:
        h.set_iterate(x, y, s, reset_origin=True)
        info = h.step()
        dx, dy, ds, v = (t.cpu().numpy() for t in h.get_direction())
    assert info.status == 0 and info.cg_iters < 400
    exact = O.exact_direction(lp.A, lp.b, lp.c, x, y, s, 0.5)
    assert np.linalg.norm(dy - exact.dy) <= 1e-8 * np.linalg.norm(exact.dy)
    assert np.linalg.norm(ds - exact.ds) <= 1e-8 * np.linalg.norm(exact.ds)


@contextlib.contextmanager
def step_tail(path):
    """LPs created inside run the step tail (Alg. 2 steps d-g) in one
    workgroup ('one', the default for n <= 1024) or as separate launches
    ('multi')."""
    old = os.environ.get("SKIPM_STEP_ONE")
    if path == "multi":
        os.environ["SKIPM_STEP_ONE"] = "0"
    else:
        os.environ.pop("SKIPM_STEP_ONE", None)
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("SKIPM_STEP_ONE", None)
        else:
            os.environ["SKIPM_STEP_ONE"] = old


def test_step_tail_one_workgroup_matches_the_launches(torch, sk):
    """The one-workgroup step tail takes the same per-entry arithmetic and the
    same sums in the same order as the separate direction, step-length and
    update launches: one step from a shared iterate, and a whole solve, are
    bitwise the same on both paths."""
    lp = dense_planted(45, 900, rng=np.random.default_rng(33))
    x, y, s = mid_iterate(lp, 4)
    say("step tail: one workgroup vs separate launches")
    out = {}
    for path in ("one", "multi"):
        with step_tail(path), sk.LP(lp.A, lp.b, lp.c, seed=17, s=2) as h:
            h.set_iterate(x, y, s, reset_origin=True)
            info = h.step()
            direc = [t.cpu().numpy() for t in h.get_direction()]
            it = [t.cpu().numpy() for t in h.get_iterate()]
            h.reset()
            res = h.solve()
            xf = h.get_iterate()[0].cpu().numpy()
        out[path] = (info, direc, it, res, xf)
    (i1, d1, it1, r1, x1), (i2, d2, it2, r2, x2) = out["one"], out["multi"]
    for f in ("alpha", "alpha_max", "v_norm", "mu", "cg_iters"):
        assert getattr(i1, f) == getattr(i2, f), f
    for a, b in zip(d1 + it1, d2 + it2):
        assert np.array_equal(a, b)
    for f in ("status", "iters", "cg_total", "obj_p", "obj_d", "rel_gap", "mu"):
        assert getattr(r1, f) == getattr(r2, f), f
    assert np.array_equal(x1, x2)
    check_solution(lp, r1, 1e-6)


def _zero_row_lp():
    """A planted LP whose A has a zero row: B = A D W then has a zero row for
    every W, so its Gram matrix has a zero pivot that neither a fresh sketch
    nor a relative diagonal shift lifts (Lemma 3's failure event, forced)."""
    lp = dense_planted(24, 600, rng=np.random.default_rng(77))
    A = lp.A.copy()
    A[5] = 0.0
    return A, A @ lp.x_star, A.T @ lp.y_star + lp.s_star


def test_rank_loss_resketches_then_shifts_then_erank(torch, sk):
    """rank(A D W) < m forced from the host: the step draws 3 fresh sketches
    (new salts), then factors the last one with 3 growing diagonal shifts, and
    ends with SKIPM_ERANK; lp_solve reports both counts."""
    A, b, c = _zero_row_lp()
    say("rank loss: zero row (24 x 600)")
    with sk.LP(A, b, c, s=2, seed=3) as h:
        with pytest.raises(sk.SkipmError) as e:
            h.step()
        assert e.value.code == sk.SKIPM_ERANK
        res = h.solve()
    assert res.status == sk.SKIPM_ERANK
    assert res.resketches >= 3 and res.shifts >= 3


# ---------------------------------------------------------------------------
# full solves
# ---------------------------------------------------------------------------

def check_solution(lp, res, gap):
    assert res.status == 0, res
    assert abs(res.obj_p - lp.opt) <= max(gap, 1e-12) * 2 * max(1.0, abs(lp.opt))
    assert res.rel_gap <= gap
    assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
    assert res.rd_norm <= 1e-8 * np.linalg.norm(lp.c)


def test_solve_config0_against_oracle(torch, sk):
    lp = config_lp(0)
    say("solve config 0 (50 x 1000, FP64, w=200, s=1, gap 1e-8)")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap) as h:
        res = h.solve()
    check_solution(lp, res, lp.eps_gap)
    ref = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="exact", eps_gap=lp.eps_gap))
    assert abs(res.obj_p - ref.obj_p) <= 2e-8 * abs(ref.obj_p)


@pytest.mark.parametrize("m,n", [(1, 10), (3, 50), (7, 300), (33, 700), (64, 1000),
                                 (65, 1500), (130, 4000), (257, 3000)])
def test_solve_ragged_shapes(torch, sk, m, n):
    lp = dense_planted(m, n, rng=np.random.default_rng(m + n), eps_gap=1e-8)
    say(f"solve ragged m={m} n={n}")
    with sk.LP(lp.A, lp.b, lp.c, eps_gap=1e-8, seed=m, s=2) as h:
        res = h.solve()
    check_solution(lp, res, 1e-8)


@pytest.mark.parametrize("s_nnz", [2, 4])
def test_solve_config0_block_sketch(torch, sk, s_nnz):
    lp = config_lp(0)
    say(f"solve config 0 with s={s_nnz}")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap, s=s_nnz) as h:
        res = h.solve()
    check_solution(lp, res, lp.eps_gap)


@pytest.mark.parametrize("fmt,prec", [("dense-f64", "fp64"), ("dense-f64", "mixed"),
                                      ("dense-f32", "fp64"), ("csr", "fp64")])
def test_solve_at_the_largest_m(torch, sk, fmt, prec):
    """m = 2048, the largest m the library takes: the column passes hold a whole
    2048-row column in one lane group (FP64: 16 registers' worth of 16-byte
    loads per lane), the sparse passes an m-vector in LDS, the factorisation
    64 panels."""
    m = 2048
    rng = np.random.default_rng(m)
    kw = {}
    if fmt == "csr":
        from lpgen import csr_planted
        lp = csr_planted(m, 12 * m, 0.004, rng=rng)
        kw = dict(a_dtype="f32", max_outer=1000)
    else:
        dt = "f32" if fmt == "dense-f32" else "f64"
        lp = dense_planted(m, 3 * m, rng=rng, a_dtype=dt)
        if dt == "f32":
            kw = dict(a_dtype="f32")
    precision = sk.SKIPM_PREC_MIXED if prec == "mixed" else sk.SKIPM_PREC_FP64
    say(f"solve at the largest m: {fmt} {lp.m} x {lp.n}, {prec}, s=2")
    with sk.LP(lp.A, lp.b, lp.c, s=2, seed=5, precision=precision, **kw) as h:
        res = h.solve()
    check_solution(lp, res, 1e-6)


def test_solve_f32_values(torch, sk):
    lp = dense_planted(60, 3000, rng=np.random.default_rng(4), a_dtype="f32")
    say("solve f32-valued 60 x 3000")
    with sk.LP(lp.A, lp.b, lp.c, a_dtype="f32", s=2) as h:
        res = h.solve()
    check_solution(lp, res, 1e-6)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_and_multi_workgroup_cg_solves(torch, sk, prec):
    """The one-workgroup CG and the fused multi-workgroup CG are the same
    iteration (their fixed-iteration iterates match Alg. 1 to 1e-9 in the test
    above).  Whole solves on either path meet the planted optimum and the exact
    oracle's objective; their iteration counts are not compared (a CG stopped
    at a tolerance can stop one iteration apart on rounding, and at s = 1 that
    moves later steps: counts are parity unpinned)."""
    lp = config_lp(0)
    say(f"small vs multi-workgroup CG, config 0, {prec}")
    pr = sk.SKIPM_PREC_MIXED if prec == "mixed" else sk.SKIPM_PREC_FP64
    ref = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="exact", eps_gap=lp.eps_gap))
    assert ref.status == "optimal"
    for path in ("small", "multi"):
        with cg_path(path), sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap,
                                  precision=pr) as h:
            res = h.solve()
        check_solution(lp, res, lp.eps_gap)
        assert abs(res.obj_p - ref.obj_p) <= 2e-8 * abs(ref.obj_p)
        assert abs(res.obj_d - ref.obj_d) <= 2e-8 * abs(ref.obj_d)


def test_solve_mixed_precision_small(torch, sk):
    lp = dense_planted(60, 2000, rng=np.random.default_rng(16))
    say("solve mixed precision 60 x 2000")
    with sk.LP(lp.A, lp.b, lp.c, s=2, precision=sk.SKIPM_PREC_MIXED) as h:
        res = h.solve()
    check_solution(lp, res, 1e-6)


def test_solve_mixed_precision(torch, sk):
    lp = dense_planted(80, 4000, rng=np.random.default_rng(6))
    say("solve mixed precision 80 x 4000")
    with sk.LP(lp.A, lp.b, lp.c, s=2, precision=sk.SKIPM_PREC_MIXED) as h:
        res = h.solve()
    check_solution(lp, res, 1e-6)


def test_solve_is_deterministic_and_resettable(torch, sk):
    lp = dense_planted(70, 2000, rng=np.random.default_rng(9))
    say("determinism 70 x 2000")
    with sk.LP(lp.A, lp.b, lp.c, s=2) as h:
        r1 = h.solve()
        h.reset()
        r2 = h.solve()
    assert r1.iters == r2.iters and r1.cg_total == r2.cg_total
    assert r1.obj_p == r2.obj_p and r1.obj_d == r2.obj_d


@pytest.mark.parametrize("fresh", [False, True])
def test_step_at_a_converged_iterate_changes_nothing(torch, sk, fresh):
    """After a solve, one more step finds the stopping test satisfied and
    leaves the iterate as it is.  With fresh = True the iterate is handed in
    again (lp_set_iterate), so the step does not know how close it is: it queues
    the sketch, factorisation and CG before it reads the test, and must still
    report convergence and leave the iterate untouched."""
    lp = dense_planted(40, 900, rng=np.random.default_rng(21))
    say(f"step at a converged iterate (fresh={fresh})")
    with sk.LP(lp.A, lp.b, lp.c, s=2, seed=4) as h:
        res = h.solve()
        assert res.status == 0
        x, y, s = (v.cpu().numpy() for v in h.get_iterate())
        if fresh:
            h.set_iterate(x, y, s, reset_origin=False)
        info = h.step()
        x2, y2, s2 = (v.cpu().numpy() for v in h.get_iterate())
    assert info.converged == 1 and info.status == 0
    assert np.array_equal(x, x2) and np.array_equal(y, y2) and np.array_equal(s, s2)


@pytest.fixture(scope="module")
def cfg1():
    """The 500 x 100000 FP64 LP the bench times, and a positive D^2 with a
    10^4 spread (what mid-solve iterates give the products)."""
    lp = config_lp(1)
    rng = np.random.default_rng(101)
    x = rng.uniform(0.1, 10.0, lp.n)
    s = rng.uniform(0.1, 10.0, lp.n)
    return lp, x, s


def test_sketch_at_full_size(torch, sk, cfg1):
    """k_sketch at the bench's shape (n = 100000 items in 2000 buckets, s = 1)
    against the oracle's hash turned into W."""
    lp, x, s = cfg1
    say("sketch at full size (500 x 100000, w=2000, s=1)")
    d = np.sqrt(x / s)
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed) as h:
        B = h.sketch(d, 3).cpu().numpy()
    W = sketch_matrix(lp.seed, 3, 1, lp.n, lp.w)
    AD = lp.A * d
    Bref = np.asarray((W.T @ AD.T).T)
    bound = np.asarray((abs(W).T @ abs(AD).T).T)
    kmax = int(np.diff(W.tocsc().indptr).max())
    assert np.all(np.abs(B - Bref) <= (kmax + 2) * EPS * bound + 1e-300)


def test_sketch_apply_f32_output(torch, sk):
    """out_dtype SKIPM_F32: the FP64 sketch rounded to nearest, element by element."""
    say("sketch to FP32, m=61 n=2000 w=244 s=2")
    rng = np.random.default_rng(404)
    lp = dense_planted(61, 2000, rng=rng)
    d = rng.uniform(0.01, 10.0, 2000)
    with sk.LP(lp.A, lp.b, lp.c, w=244, s=2, seed=9) as h:
        B64 = h.sketch(d, 3).cpu().numpy()
        B32 = h.sketch(d, 3, out_dtype="f32").cpu().numpy()
    assert B32.dtype == np.float32
    assert np.array_equal(B32, B64.astype(np.float32))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_normal_product_at_full_size(torch, sk, cfg1, prec):
    """The fused product A D^2 A^T u at the bench's shape and launch
    configuration (FP64 A, or its FP32 copy with FP64 accumulation in mixed
    precision) against the oracle's normal matrix of the same A; D^2 = x / s is
    what the prologue of one IPM step from (x, y, s) leaves behind."""
    lp, x, s = cfg1
    say(f"normal product at full size, {prec}")
    rng = np.random.default_rng(102)
    y = rng.standard_normal(lp.m)
    u = rng.standard_normal(lp.m)
    precision = sk.SKIPM_PREC_MIXED if prec == "mixed" else sk.SKIPM_PREC_FP64
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, s=2, precision=precision) as h:
        h.set_iterate(x, y, s)
        h.step()
        q = h.normal_matvec(u).cpu().numpy()
    A = lp.A if prec == "fp64" else lp.A.astype(np.float32).astype(np.float64)
    d2 = x / s
    ref = O.normal_matrix(A, d2) @ u
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 2 * (lp.m + lp.n) * EPS * bound)


@pytest.mark.parametrize("m,prec", [(256, "mixed"), (257, "mixed"), (300, "mixed"),
                                    (384, "mixed"), (385, "mixed"), (128, "fp64"),
                                    (129, "fp64"), (192, "fp64"), (193, "fp64"),
                                    (128, "mixed"), (129, "mixed"), (192, "mixed"),
                                    (193, "mixed"), (64, "fp64"), (65, "fp64"), (96, "fp64"),
                                    (97, "fp64")])
def test_normal_product_lane_group_shapes(torch, sk, m, prec):
    """The fused product on both sides of each edge of the lane groups with
    three 16-byte vectors per lane (16 lanes: 32V < lda <= 48V rows; 32 lanes:
    64V < lda <= 96V; V = 4 FP32 or 2 FP64 values per vector) and the groups
    around them, over a ragged number of columns, against the oracle's normal
    matrix."""
    n = 2501
    lp = dense_planted(m, n, rng=np.random.default_rng(m + 7))
    rng = np.random.default_rng(m + 8)
    x = rng.uniform(0.1, 10.0, n)
    s = rng.uniform(0.1, 10.0, n)
    y = rng.standard_normal(m)
    u = rng.standard_normal(m)
    say(f"normal product m={m} n={n} {prec}")
    precision = sk.SKIPM_PREC_MIXED if prec == "mixed" else sk.SKIPM_PREC_FP64
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, s=2, precision=precision) as h:
        h.set_iterate(x, y, s)
        h.step()
        q = h.normal_matvec(u).cpu().numpy()
    A = lp.A if prec == "fp64" else lp.A.astype(np.float32).astype(np.float64)
    d2 = x / s
    ref = O.normal_matrix(A, d2) @ u
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 2 * (m + n) * EPS * bound)


def test_streamed_fp32_product(torch, sk):
    """The mixed product over an FP32 copy larger than 240 MiB (500 x 130000:
    260 MB) takes the non-temporal instantiation of the pass; element by
    element against the oracle's normal matrix of the FP32-rounded A."""
    m, n = 500, 130_000
    lp = dense_planted(m, n, rng=np.random.default_rng(130))
    rng = np.random.default_rng(131)
    x, s_ = rng.uniform(0.1, 10.0, n), rng.uniform(0.1, 10.0, n)
    y, u = rng.standard_normal(m), rng.standard_normal(m)
    say("streamed FP32 product 500 x 130000 (mixed)")
    with sk.LP(lp.A, lp.b, lp.c, s=2, seed=3, precision=sk.SKIPM_PREC_MIXED) as h:
        h.set_iterate(x, y, s_)
        h.step()
        q = h.normal_matvec(u).cpu().numpy()
    A = lp.A.astype(np.float32).astype(np.float64)
    d2 = x / s_
    ref = O.normal_matrix(A, d2) @ u
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 2 * (m + n) * EPS * bound)


def test_pcg_at_full_size_matches_alg1(torch, sk, cfg1):
    """Three FP64 CG iterations at the bench's shape (the fused three-launch CG
    the solve runs) against Alg. 1 on the split system."""
    lp, x, s = cfg1
    say("pcg fixed t=3 at full size (FP64, s=1)")
    d2 = x / s
    p = np.random.default_rng(103).standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed) as h:
        dy, info = h.pcg(d2, p, 6, tol=0.0, max_it=3)
        dy = dy.cpu().numpy()
    assert info.iters == 3
    W = sketch_matrix(lp.seed, 6, 1, lp.n, lp.w)
    ref = O.sketch_pcg(lp.A * np.sqrt(d2), p, W, t=3)
    assert np.linalg.norm(dy - ref.dy) <= 1e-9 * np.linalg.norm(ref.dy)
    assert info.f0_norm == pytest.approx(ref.f_norms[0], rel=1e-10)


def test_mixed_pcg_at_full_size_matches_cholesky(torch, sk, cfg1):
    """The mixed-precision CG (FP32 copy of A in the products, FP64 residual
    refinement) at the bench's shape, run to 1e-12, against the oracle's
    Cholesky solve of the same normal equations (kappa 2 here).  Solving with
    the FP32-rounded A alone would leave a relative error of 6e-9; the bound
    asks for the FP64 solution."""
    lp, x, s = cfg1
    say("mixed pcg to 1e-12 at full size vs Cholesky")
    d2 = x / s
    p = np.random.default_rng(104).standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, precision=sk.SKIPM_PREC_MIXED) as h:
        dy, info = h.pcg(d2, p, 6, tol=1e-12, max_it=1000)
        dy = dy.cpu().numpy()
    ref = np.linalg.solve(O.normal_matrix(lp.A, d2), p)
    assert np.linalg.norm(dy - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_config1_full_size(torch, sk, prec):
    """The bench's headline workload at full size, in both precision modes the
    bench times (s = 1): planted optimum, KKT residuals, and the precision
    tier the run ended at."""
    lp = config_lp(1)
    say(f"solve config 1 (500 x 100000 FP64, w=2000, s=1), {prec}")
    pr = sk.SKIPM_PREC_MIXED if prec == "mixed" else sk.SKIPM_PREC_FP64
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap, precision=pr) as h:
        res = h.solve()
    check_solution(lp, res, lp.eps_gap)
    assert res.cg_max <= 1000   # the default cap per normal-equation solve
    if prec == "fp64":
        assert res.tier_final == sk.SKIPM_TIER_FP64 and res.demote_iter == -1
    else:
        assert res.tier_final in (sk.SKIPM_TIER_FP32, sk.SKIPM_TIER_FP64)
        assert (res.demote_iter == -1) == (res.tier_final == sk.SKIPM_TIER_FP32)
        assert res.demote_iter < res.iters


# ---------------------------------------------------------------------------
# sparse (CSR) problems
# ---------------------------------------------------------------------------

def test_csr_rejects_bad_structure(torch, sk):
    say("csr validation")
    lp = dense_planted(4, 30, rng=np.random.default_rng(1))
    A = sp.csr_matrix(lp.A)
    A.indices[3], A.indices[4] = A.indices[4], A.indices[3]   # unsorted columns in row 0
    A.has_sorted_indices = True                                  # keep the binding from sorting
    A.sort_indices = lambda: None
    with pytest.raises(sk.SkipmError) as e:
        sk.LP(A, lp.b, lp.c)
    assert e.value.code == sk.SKIPM_EINVAL


@pytest.mark.parametrize("m,n,dens,s_nnz", [(20, 3000, 0.02, 2), (37, 5000, 0.005, 1),
                                           (130, 20000, 0.002, 2)])
def test_csr_solve_matches_planted_objective(torch, sk, m, n, dens, s_nnz):
    from lpgen import csr_planted
    lp = csr_planted(m, n, dens, rng=np.random.default_rng(m), eps_gap=1e-8)
    say(f"csr solve m={m} n={n} density={dens} s={s_nnz}")
    with sk.LP(lp.A, lp.b, lp.c, a_dtype="f32", s=s_nnz, eps_gap=1e-8, seed=m) as h:
        res = h.solve()
    check_solution(lp, res, 1e-8)


def test_csr_and_dense_agree(torch, sk):
    from lpgen import csr_planted
    lp = csr_planted(25, 2000, 0.01, rng=np.random.default_rng(3))
    say("csr vs dense: pcg and sketch")
    rng = np.random.default_rng(4)
    d2 = rng.uniform(0.05, 20.0, lp.n)
    p = rng.standard_normal(lp.m)
    out = {}
    for kind, A in (("csr", lp.A), ("dense", lp.A.toarray())):
        with sk.LP(A, lp.b, lp.c, a_dtype="f32", seed=8, s=2) as h:
            dy, info = h.pcg(d2, p, 3, tol=0.0, max_it=6)
            B = h.sketch(np.sqrt(d2), 3).cpu().numpy()
            out[kind] = (dy.cpu().numpy(), info.iters, B)
    assert out["csr"][1] == out["dense"][1] == 6
    assert np.linalg.norm(out["csr"][0] - out["dense"][0]) <= 1e-9 * np.linalg.norm(out["dense"][0])
    W = sketch_matrix(8, 3, 2, lp.n, lp.w)
    Bref = np.asarray((W.T @ (lp.A.toarray() * np.sqrt(d2)).T).T)
    bound = np.asarray((abs(W).T @ abs(lp.A.toarray() * np.sqrt(d2)).T).T)
    for kind in ("csr", "dense"):
        assert np.all(np.abs(out[kind][2] - Bref) <= 64 * EPS * bound + 1e-300)


@pytest.fixture(scope="module")
def cfg2():
    lp = config_lp(2)
    rng = np.random.default_rng(201)
    return lp, rng.uniform(0.1, 10.0, lp.n), rng.uniform(0.1, 10.0, lp.n)


def test_csr_sketch_at_full_size(torch, sk, cfg2):
    """k_csc_sketch at config 2's shape (1000 x 1000000, ~2e6 non-zeros, 4000
    buckets) against the oracle's W."""
    lp, x, s = cfg2
    say("csr sketch at full size (1000 x 1000000, w=4000, s=1)")
    d = np.sqrt(x / s)
    with sk.LP(lp.A, lp.b, lp.c, a_dtype="f32", w=lp.w, seed=lp.seed) as h:
        B = h.sketch(d, 2).cpu().numpy()
    W = sketch_matrix(lp.seed, 2, 1, lp.n, lp.w)
    AD = lp.A @ sp.diags(d)
    Bref = np.asarray((AD @ W).todense())
    bound = np.asarray((abs(AD) @ abs(W)).todense())
    kmax = int(np.diff(W.tocsc().indptr).max())
    assert np.all(np.abs(B - Bref) <= (kmax + 2) * EPS * bound + 1e-300)


def test_sketch_apply_f32_output(torch, sk):
    """out_dtype SKIPM_F32: the FP64 sketch rounded to nearest, element by element."""
    say("sketch to FP32, m=61 n=2000 w=244 s=2")
    rng = np.random.default_rng(404)
    lp = dense_planted(61, 2000, rng=rng)
    d = rng.uniform(0.01, 10.0, 2000)
    with sk.LP(lp.A, lp.b, lp.c, w=244, s=2, seed=9) as h:
        B64 = h.sketch(d, 3).cpu().numpy()
        B32 = h.sketch(d, 3, out_dtype="f32").cpu().numpy()
    assert B32.dtype == np.float32
    assert np.array_equal(B32, B64.astype(np.float32))


def _csr_case(m, n, dens, ones, dense_col, empty_rows, seed):
    """Random CSR matrix with optional all-ones row 0, an empty column 7, a
    dense column 11 and empty rows 3 and 5."""
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="lil", random_state=rng,
                  data_rvs=rng.standard_normal)
    if ones:
        A[0, :] = 1.0
    A[:, 7] = 0.0
    if dense_col:
        A[:, 11] = rng.standard_normal((m, 1))
    if empty_rows:
        A[3, :] = 0.0
        A[5, :] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    return A


@pytest.mark.parametrize("m,n,dens,ones,dense_col,empty_rows,vdt", [
    (50, 30000, 0.001, True, True, False, "f32"),   # long all-ones row across many threads
    (300, 12000, 0.3, False, True, False, "f64"),   # blocks cut by the non-zero bound
    (37, 5000, 0.0, True, False, False, "f32"),     # the ones row alone
    (2048, 3000, 0.01, True, True, False, "f64"),   # largest m
    (5, 20000, 0.5, True, True, False, "f32"),      # few rows, long runs per row
    (64, 9000, 0.02, False, False, True, "f64"),    # empty rows
    # FP32 values keep the row order as 2-byte references into LDS
    (2048, 3000, 0.01, True, True, False, "f32"),   # largest m: the most LDS
    (300, 12000, 0.3, False, True, False, "f32"),   # blocks cut by the non-zero bound
    (64, 9000, 0.02, False, False, True, "f32"),    # empty rows
])
def test_csr_block_product(torch, sk, m, n, dens, ones, dense_col, empty_rows, vdt):
    """The one-pass sparse product (column blocks, coefficients in LDS, rows
    joined by the segmented scan) against the oracle's normal matrix, element
    by element, and bitwise equal on a second call.  D^2 = x / s comes from the
    prologue of one IPM step (rank-deficient cases end that step with an
    error after the prologue; the product does not need the rest)."""
    A = _csr_case(m, n, dens, ones, dense_col, empty_rows, seed=m + n)
    if vdt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    say(f"csr block product m={m} n={n} nnz={A.nnz} {vdt}")
    rng = np.random.default_rng(n)
    x, s = rng.uniform(0.1, 10.0, n), rng.uniform(0.1, 10.0, n)
    b = A @ x
    c = A.T @ rng.standard_normal(m) + s
    u = rng.standard_normal(m)
    with sk.LP(A, b, c, a_dtype=vdt, s=1, seed=3) as h:
        h.set_iterate(x, np.zeros(m), s)
        with contextlib.suppress(sk.SkipmError):
            h.step()
        q1 = h.normal_matvec(u).cpu().numpy()
        q2 = h.normal_matvec(u).cpu().numpy()
    d2 = x / s
    ref = O.normal_matrix(A, d2) @ u
    absA = abs(A)
    bound = absA @ (d2 * (absA.T @ np.abs(u)))
    kmax = max(int(np.diff(A.indptr).max()), int(np.diff(A.tocsc().indptr).max()))
    assert np.all(np.abs(q1 - ref) <= 2 * (kmax + 2) * EPS * bound + 1e-300)
    assert np.array_equal(q1, q2)


def test_csr_normal_product_at_full_size(torch, sk, cfg2):
    """The sparse product (one pass over column blocks of the CSC copy and
    their row-ordered copies, then the block partials' finish) at config 2's
    shape against the oracle's normal matrix."""
    lp, x, s = cfg2
    say("csr normal product at full size")
    rng = np.random.default_rng(202)
    y = rng.standard_normal(lp.m)
    u = rng.standard_normal(lp.m)
    with sk.LP(lp.A, lp.b, lp.c, a_dtype="f32", w=lp.w, seed=lp.seed, s=2) as h:
        h.set_iterate(x, y, s)
        h.step()
        q = h.normal_matvec(u).cpu().numpy()
    d2 = x / s
    ref = O.normal_matrix(lp.A, d2) @ u
    absA = abs(lp.A)
    bound = absA @ (d2 * (absA.T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 2 * (lp.m + lp.n) * EPS * bound)


def test_solve_config2_full_size(torch, sk):
    lp = config_lp(2)
    say("solve config 2 (CSR 1000 x 1000000, ~2e6 nnz, FP32 values, w=4000, s=1)")
    # the exact-Cholesky oracle needs 306 IPM iterations on this LP: long runs of
    # short steps, where a few columns sit on the neighbourhood's boundary
    with sk.LP(lp.A, lp.b, lp.c, a_dtype="f32", w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap,
               max_outer=1000) as h:
        res = h.solve()
    check_solution(lp, res, lp.eps_gap)


# ---------------------------------------------------------------------------
# degenerate and failing problems
# ---------------------------------------------------------------------------

def _no_optimum_lp(kind):
    rng = np.random.default_rng(5)
    m, n = 20, 200
    if kind == "infeasible":   # A > 0 elementwise, b < 0: no x >= 0 has A x = b
        A = np.abs(rng.standard_normal((m, n)))
        b = -np.ones(m)
        c = rng.uniform(0.5, 1.5, n)
    else:                      # A (e0 + e1) = 0 and c (e0 + e1) < 0: cost unbounded below
        A = rng.standard_normal((m, n))
        A[:, 1] = -A[:, 0]
        b = A @ rng.uniform(0.5, 1.0, n)
        c = np.ones(n)
        c[:2] = -1.0
    return A, b, c


@pytest.mark.parametrize("kind", ["infeasible", "unbounded"])
def test_solve_without_an_optimum_reports_failure(torch, sk, kind):
    """The method assumes an optimum exists (its theorem starts from a point
    that dominates one); without one the solve must end with an error status
    (not converged, stalled, non-finite or rank loss), like the oracle."""
    A, b, c = _no_optimum_lp(kind)
    say(f"solve a {kind} LP (20 x 200, max_outer 60)")
    with sk.LP(A, b, c, s=2, seed=4, max_outer=60) as h:
        res = h.solve()
    assert res.status in (sk.SKIPM_ENOTCONV, sk.SKIPM_ESTALL, sk.SKIPM_ENAN, sk.SKIPM_ERANK), res
    ref = O.ipm(A, b, c, O.IPMParams(solver="exact", max_outer=60))
    assert ref.status != "optimal"


def test_solve_square_lp(torch, sk):
    """n = m: the feasible set is the single point A^{-1} b."""
    lp = dense_planted(24, 24, rng=np.random.default_rng(24), eps_gap=1e-8)
    say("solve square 24 x 24")
    with sk.LP(lp.A, lp.b, lp.c, w=4 * 24, seed=2, s=2, eps_gap=1e-8) as h:
        res = h.solve()
    check_solution(lp, res, 1e-8)


def test_iteration_cap_reports_not_converged(torch, sk):
    lp = config_lp(0)
    say("config 0 with max_outer = 3")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap, max_outer=3) as h:
        res = h.solve()
    assert res.status == sk.SKIPM_ENOTCONV
    assert res.iters == 3
