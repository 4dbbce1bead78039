"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published generator outputs, brute force on tiny LPs, an independent library
LP solver, planted optima, closed forms and invariants stated in the paper.
A few tests plant a mistake in (a copy of) the oracle and check that a pin
catches it."""
import math
from pathlib import Path

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from lpgen import config_lp, csr_planted, dense_planted
from oracle import ipm as O
from oracle.sketch import mix_array, mix_int, sketch_hash, sketch_matrix, splitmix64_stream
from oracle.vertex import vertex_enum

GOLDEN = Path(__file__).parent / "golden"


# ---------------------------------------------------------------------------
# sketch hash
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    for line in (GOLDEN / "splitmix64.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        seed, *outs = (int(v) for v in line.split())
        assert splitmix64_stream(seed, len(outs)) == outs


def test_mix_array_matches_integer_version():
    rng = np.random.default_rng(3)
    z = rng.integers(0, 2**63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    got = mix_array(z)
    for a, b in zip(z.tolist(), got.tolist()):
        assert mix_int(a) == b


@pytest.mark.parametrize("s,w", [(1, 200), (2, 200), (4, 64), (1, 7)])
def test_hash_buckets_blocks_and_balance(s, w):
    n = 200_000
    bucket, sign = sketch_hash(0x5EED, 3, s, n, w)
    blk = w // s
    for r in range(s):
        b = bucket[:, r]
        assert b.min() >= r * blk and b.max() < (r + 1) * blk
        counts = np.bincount(b - r * blk, minlength=blk)
        expected = n / blk
        chi2 = float(((counts - expected) ** 2 / expected).sum())
        # chi-square with blk-1 degrees of freedom: mean blk-1, sd sqrt(2(blk-1))
        assert chi2 < (blk - 1) + 6 * math.sqrt(2 * (blk - 1))
        frac = float((sign[:, r] == 1).mean())
        assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(n)
        assert set(np.unique(sign[:, r]).tolist()) <= {-1, 1}


def test_hash_salts_differ_and_repeat():
    b1, s1 = sketch_hash(11, 0, 2, 5000, 100)
    b2, s2 = sketch_hash(11, 0, 2, 5000, 100)
    b3, _ = sketch_hash(11, 1, 2, 5000, 100)
    assert np.array_equal(b1, b2) and np.array_equal(s1, s2)
    assert (b1 != b3).mean() > 0.9


def test_sketch_matrix_structure():
    W = sketch_matrix(5, 2, 4, 300, 40)
    assert W.shape == (300, 40)
    nnz_per_row = np.diff(W.indptr)
    assert np.all(nnz_per_row == 4)
    assert set(np.unique(W.data).tolist()) <= {-1.0, 1.0}


# ---------------------------------------------------------------------------
# exact IPM against brute force, an independent solver and planted optima
# ---------------------------------------------------------------------------

def _tiny_lps():
    out = []
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        m, n = int(rng.integers(1, 4)), int(rng.integers(5, 9))
        out.append(dense_planted(m, n, support=m, rng=rng, eps_gap=1e-9))
    # non-planted: random feasible bounded LP with a degenerate-free optimum
    rng = np.random.default_rng(7)
    A = rng.uniform(0.1, 1.0, size=(3, 8))
    x0 = rng.uniform(0.5, 1.0, size=8)
    b = A @ x0
    c = rng.uniform(0.1, 2.0, size=8)
    out.append((A, b, c))
    return out


@pytest.mark.parametrize("case", range(7))
def test_exact_ipm_matches_vertex_enumeration_and_highs(case):
    lp = _tiny_lps()[case]
    if isinstance(lp, tuple):
        A, b, c = lp
    else:
        A, b, c = lp.A, lp.b, lp.c
    res = O.ipm(A, b, c, O.IPMParams(solver="exact", eps_gap=1e-10, eps_feas=1e-10))
    assert res.status == "optimal"
    best, _ = vertex_enum(A, b, c)
    hs = so.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert hs.status == 0
    scale = max(1.0, abs(best))
    assert abs(res.obj_p - best) <= 1e-8 * scale
    assert abs(hs.fun - best) <= 1e-8 * scale
    assert abs(res.obj_d - best) <= 1e-8 * scale


def test_exact_ipm_recovers_planted_optimum_cfg0():
    lp = config_lp(0)
    res = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="exact", eps_gap=lp.eps_gap))
    assert res.status == "optimal"
    assert abs(res.obj_p - lp.opt) <= 1e-7 * abs(lp.opt)
    assert abs(float(lp.b @ lp.y_star) - lp.opt) <= 1e-10 * abs(lp.opt)
    assert np.linalg.norm(res.x - lp.x_star) <= 1e-4 * np.linalg.norm(lp.x_star)
    assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
    assert res.rd_norm <= 1e-8 * np.linalg.norm(lp.c)


def test_sketch_ipm_recovers_planted_optimum():
    rng = np.random.default_rng(21)
    lp = dense_planted(30, 600, rng=rng, eps_gap=1e-8)
    for s in (1, 2):
        res = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="sketch", eps_gap=1e-8, s_nnz=s,
                                                  seed=9))
        assert res.status == "optimal"
        assert abs(res.obj_p - lp.opt) <= 1e-6 * abs(lp.opt)
        assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)


def test_sparse_planted_objective():
    rng = np.random.default_rng(5)
    lp = csr_planted(20, 3000, 0.02, rng=rng)
    assert sp.issparse(lp.A)
    assert np.all(np.diff(lp.A.indptr) > 0)
    res = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="sketch", eps_gap=1e-8, s_nnz=2))
    assert res.status == "optimal"
    assert abs(res.obj_p - lp.opt) <= 1e-6 * max(1.0, abs(lp.opt))


# ---------------------------------------------------------------------------
# invariants of one direction (eq. addl, eq. iip_3, mu(alpha))
# ---------------------------------------------------------------------------

def _mid_iterate(lp, iters=8):
    """Advance the exact IPM a few steps to get a non-trivial iterate."""
    x, y, s = np.ones(lp.n), np.zeros(lp.m), np.ones(lp.n)
    rp0, rd0 = O.residuals(lp.A, lp.b, lp.c, x, y, s)
    r0 = math.hypot(np.linalg.norm(rp0), np.linalg.norm(rd0))
    for _ in range(iters):
        d = O.exact_direction(lp.A, lp.b, lp.c, x, y, s, 0.5)
        eta = math.hypot(np.linalg.norm(d.rp), np.linalg.norm(d.rd)) / r0
        st = O.step_length(x, s, d.dx, d.ds, 0.999, 1.0, eta, 1e-3)
        x, y, s = x + st.alpha * d.dx, y + st.alpha * d.dy, s + st.alpha * d.ds
    return x, y, s, r0


@pytest.fixture(scope="module")
def small_lp():
    return dense_planted(40, 800, rng=np.random.default_rng(8))


def test_correction_vector_satisfies_addl_and_iip3(small_lp):
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp, 3)
    W = sketch_matrix(3, 1, 1, lp.n, lp.w)
    d = O.sketch_direction(lp.A, lp.b, lp.c, x, y, s, 0.5, W, tol_cg=1e-2)
    assert np.linalg.norm(d.v) > 0
    assert np.linalg.norm(d.rp) > 1e-3 * np.linalg.norm(lp.b)
    d2 = x / s
    g = lp.A @ (d2 * (lp.A.T @ d.dy)) - d.p
    lhs = lp.A @ (d.v / s)
    assert np.linalg.norm(lhs - g) <= 1e-10 * np.linalg.norm(g)
    # eq. iip_3
    assert np.linalg.norm(lp.A @ d.dx + d.rp) <= 1e-9 * np.linalg.norm(d.rp)
    assert np.linalg.norm(lp.A.T @ d.dy + d.ds + d.rd) <= 1e-12 * np.linalg.norm(d.rd)
    r3 = x * d.ds + s * d.dx + x * s - 0.5 * d.mu + d.v
    assert np.linalg.norm(r3) <= 1e-12 * np.linalg.norm(x * s)


def test_mu_alpha_identity(small_lp):
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp, 5)
    W = sketch_matrix(3, 2, 1, lp.n, lp.w)
    d = O.sketch_direction(lp.A, lp.b, lp.c, x, y, s, 0.5, W, tol_cg=1e-1)
    n = lp.n
    for a in (0.1, 0.5, 0.9):
        direct = float((x + a * d.dx) @ (s + a * d.ds)) / n
        closed = (1 - a * (1 - 0.5)) * d.mu - a * d.v.sum() / n + a * a * float(d.dx @ d.ds) / n
        assert abs(direct - closed) <= 1e-12 * abs(d.mu)


def test_residual_stays_on_segment():
    rng = np.random.default_rng(12)
    lp = dense_planted(25, 400, rng=rng)
    for solver in ("exact", "sketch"):
        x, y, s = np.ones(lp.n), np.zeros(lp.m), np.ones(lp.n)
        rp0, rd0 = O.residuals(lp.A, lp.b, lp.c, x, y, s)
        r0 = np.concatenate([rp0, rd0])
        eta = 1.0
        for k in range(15):
            rp, rd = O.residuals(lp.A, lp.b, lp.c, x, y, s)
            r = np.concatenate([rp, rd])
            assert np.linalg.norm(r - eta * r0) <= 1e-9 * np.linalg.norm(r0)
            if solver == "exact":
                d = O.exact_direction(lp.A, lp.b, lp.c, x, y, s, 0.5)
            else:
                W = sketch_matrix(1, k, 1, lp.n, lp.w)
                d = O.sketch_direction(lp.A, lp.b, lp.c, x, y, s, 0.5, W, tol_cg=1e-3)
            st = O.step_length(x, s, d.dx, d.ds, 0.999, 1.0,
                               np.linalg.norm(r) / np.linalg.norm(r0), 1e-3)
            # neighbourhood N(gamma) holds at the new point (Sec. 4)
            xn, sn = x + st.alpha * d.dx, s + st.alpha * d.ds
            mun = float(xn @ sn) / lp.n
            assert np.all(xn * sn >= (1 - 0.999) * mun * (1 - 1e-9))
            assert (1 - st.alpha) * eta <= mun / 1.0 * (1 + 1e-9)
            x, y, s = xn, y + st.alpha * d.dy, sn
            eta *= 1 - st.alpha


# ---------------------------------------------------------------------------
# step length: closed form vs brute force on a grid
# ---------------------------------------------------------------------------

def _in_N(x, s, dx, ds, a, gamma, mu0, eta):
    xa, sa = x + a * dx, s + a * ds
    mua = float(xa @ sa) / x.size
    return bool(np.all(xa * sa >= (1 - gamma) * mua) and (1 - a) * eta <= mua / mu0
                and np.all(xa > 0) and np.all(sa > 0))


@pytest.mark.parametrize("seed", range(8))
def test_step_length_against_grid(seed):
    rng = np.random.default_rng(seed)
    n = 50
    x = rng.uniform(0.2, 2.0, n)
    s = rng.uniform(0.8, 1.2, n) / x          # start inside N(gamma)
    dx = rng.standard_normal(n) * rng.uniform(0.2, 3.0)
    ds = rng.standard_normal(n) * rng.uniform(0.2, 3.0)
    gamma = [0.5, 0.9, 0.999][seed % 3]
    mu = float(x @ s) / n
    mu0, eta = 1.0, min(1.0, 0.9 * mu)
    st = O.step_length(x, s, dx, ds, gamma, mu0, eta, guard=0.0)
    assert _in_N(x, s, dx, ds, 0.0, gamma, mu0, eta)
    assert st.alpha_max > 0
    grid = np.linspace(0.0, 1.0, 10001)
    below = grid[grid <= st.alpha_max * (1 - 1e-9)]
    assert all(_in_N(x, s, dx, ds, a, gamma, mu0, eta) for a in below[::7])
    if st.alpha_max < 1.0:
        a_out = st.alpha_max * (1 + 1e-6) + 1e-9
        assert not _in_N(x, s, dx, ds, a_out, gamma, mu0, eta)
    # step (f): argmin of mu(alpha) on [0, alpha_max], checked on a dense grid
    g = np.linspace(0.0, st.alpha_max, 20001)
    mus = [(x + a * dx) @ (s + a * ds) for a in g]
    assert ((x + st.alpha * dx) @ (s + st.alpha * ds)) <= min(mus) + 1e-12 * abs(min(mus))


def test_first_exit_cases():
    fe = O.first_exit
    assert fe(1.0, -3.0, 2.0)[0] == pytest.approx(1.0)   # (a-1)(a-2): exits at 1
    assert fe(-1.0, 0.0, 4.0)[0] == pytest.approx(2.0)   # 4 - a^2
    assert fe(1.0, 1.0, 1.0)[0] == np.inf                # never negative
    assert fe(0.0, -2.0, 1.0)[0] == pytest.approx(0.5)   # linear
    assert fe(0.0, 0.0, 0.0)[0] == np.inf
    assert fe(-1.0, 0.0, 0.0)[0] == 0.0
    assert fe(-1.0, 2.0, 0.0)[0] == pytest.approx(2.0)   # a(2 - a)
    assert fe(1.0, -2.0, 1.0)[0] == np.inf               # (a-1)^2 touches zero only


# ---------------------------------------------------------------------------
# Alg. 1: spectra and CG
# ---------------------------------------------------------------------------

def _scaled(lp, x, s):
    return lp.A * np.sqrt(x / s)


def test_lemma1_spectrum_closed_form(small_lp):
    """eig(Q^{-1/2} A D^2 A^T Q^{-1/2}) = 1 / eig(V^T W W^T V) with A D = U S V^T
    (proof of Lemma 1)."""
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    AD = _scaled(lp, x, s)
    W = sketch_matrix(4, 0, 2, lp.n, lp.w)
    res = O.sketch_pcg(AD, np.ones(lp.m), W, t=1)
    M = res.Qmh @ AD @ AD.T @ res.Qmh
    ev = np.sort(np.linalg.eigvalsh((M + M.T) / 2))
    _, _, Vh = np.linalg.svd(AD, full_matrices=False)
    VW = np.asarray((W.T @ Vh.T).T)
    ev2 = np.sort(1.0 / np.linalg.eigvalsh(VW @ VW.T))
    assert np.allclose(ev, ev2, rtol=1e-10, atol=0)


def test_signed_permutation_sketch_is_exact_preconditioner(small_lp):
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    AD = _scaled(lp, x, s)
    rng = np.random.default_rng(1)
    perm = rng.permutation(lp.n)
    sg = rng.choice([-1.0, 1.0], lp.n)
    W = sp.csr_matrix((sg, (np.arange(lp.n), perm)), shape=(lp.n, lp.n))
    p = rng.standard_normal(lp.m)
    res = O.sketch_pcg(AD, p, W, tol=1e-10)
    assert res.iters == 1
    dy = np.linalg.solve(AD @ AD.T, p)
    assert np.linalg.norm(res.dy - dy) <= 1e-9 * np.linalg.norm(dy)


def test_pcg_converges_to_cholesky_solution(small_lp):
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    AD = _scaled(lp, x, s)
    W = sketch_matrix(8, 3, 1, lp.n, lp.w)
    p = np.random.default_rng(2).standard_normal(lp.m)
    res = O.sketch_pcg(AD, p, W, tol=1e-13, max_it=200)
    dy = np.linalg.solve(AD @ AD.T, p)
    assert np.linalg.norm(res.dy - dy) <= 1e-9 * np.linalg.norm(dy)


def test_lemma2_residual_contraction(small_lp):
    """||f^(j)|| <= (kappa^2 - 1)/2 ||f^(j-1)|| with kappa = kappa(Q^{-1/2} A D)."""
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp, 3)
    AD = _scaled(lp, x, s)
    W = sketch_matrix(2, 0, 8, lp.n, lp.n)
    p = np.random.default_rng(4).standard_normal(lp.m)
    res = O.sketch_pcg(AD, p, W, t=6)
    sv = np.linalg.svd(res.Qmh @ AD, compute_uv=False)
    k2 = (sv[0] / sv[-1]) ** 2
    assert k2 < 3
    f = res.f_norms
    for j in range(1, len(f)):
        assert f[j] <= (k2 - 1) / 2 * f[j - 1] * (1 + 1e-9)


def test_lemma4_v_bound_diagnostic(small_lp):
    """||v|| <= sqrt(3 n mu) ||f^(t)|| (Lemma 4; holds when the sketch is good)."""
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    W = sketch_matrix(6, 1, 4, lp.n, lp.w)
    d = O.sketch_direction(lp.A, lp.b, lp.c, x, y, s, 0.5, W, t=3)
    assert np.linalg.norm(d.v) <= math.sqrt(3 * lp.n * d.mu) * d.f_norm


# ---------------------------------------------------------------------------
# Gaussian sketching matrix W_G (Sec. 5)
# ---------------------------------------------------------------------------

def test_gaussian_sketch_is_standard_normal():
    """Entries of W_G: N(0, 1) to the resolution of 2e5 samples, rounded to an
    8-bit significand (exactly representable in bfloat16)."""
    from scipy import stats
    from oracle.sketch import gaussian_sketch_matrix
    W = gaussian_sketch_matrix(7, 3, 400, 500)
    z = W.ravel()
    nz = z.size
    assert abs(z.mean()) < 5 / math.sqrt(nz)
    assert abs(z.var() - 1.0) < 0.015
    assert abs(stats.skew(z)) < 0.02 and abs(stats.kurtosis(z)) < 0.05
    assert stats.kstest(z, "norm").statistic < 0.005
    bits = z.astype(np.float32).view(np.uint32)
    assert np.all((bits & 0xFFFF) == 0)
    assert np.array_equal(z.astype(np.float32).astype(np.float64), z)


def test_gaussian_sketch_entries_independent_and_salted():
    from oracle.sketch import gaussian_sketch_matrix
    W0 = gaussian_sketch_matrix(7, 0, 300, 400)
    W1 = gaussian_sketch_matrix(7, 1, 300, 400)
    assert np.array_equal(W0, gaussian_sketch_matrix(7, 0, 300, 400))
    lim = 5 / math.sqrt(W0.size)
    assert abs(np.corrcoef(W0.ravel(), W1.ravel())[0, 1]) < lim
    assert abs(np.corrcoef(W0[:, :-1].ravel(), W0[:, 1:].ravel())[0, 1]) < lim
    assert abs(np.corrcoef(W0[:-1].ravel(), W0[1:].ravel())[0, 1]) < lim
    # a different number of rows indexes the same stream: pair (j, c) is base ^ 2 (j w + c)
    Wn = gaussian_sketch_matrix(7, 0, 600, 400)
    assert np.array_equal(Wn[:300], W0)
    # the two entries of a Box-Muller pair are uncorrelated and each N(0, 1)
    assert abs(np.corrcoef(W0[:, 0::2].ravel(), W0[:, 1::2].ravel())[0, 1]) < 2 * lim
    assert abs(W0[:, 1::2].var() - 1.0) < 0.03


def test_gaussian_sketch_spectrum_within_marchenko_pastur(small_lp):
    """With W_G (w = 4m) the preconditioned matrix Q^{-1/2} A D^2 A^T Q^{-1/2}
    has kappa <= ((1 + sqrt(m/w)) / (1 - sqrt(m/w)))^2 = 9 up to the finite-size
    edge fluctuation (the extreme singular values of a Gaussian matrix)."""
    from oracle.sketch import gaussian_sketch_matrix
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    AD = _scaled(lp, x, s)
    W = gaussian_sketch_matrix(3, 0, lp.n, 4 * lp.m)
    res = O.sketch_pcg(AD, np.ones(lp.m), W, t=1)
    sv = np.linalg.svd(res.Qmh @ AD, compute_uv=False)
    assert (sv[0] / sv[-1]) ** 2 <= 9 * 1.6


def test_ipm_with_gaussian_sketch_reaches_the_planted_optimum():
    lp = dense_planted(15, 300, rng=np.random.default_rng(31), eps_gap=1e-8)
    r = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="sketch", sketch="gaussian", eps_gap=1e-8,
                                              w=4 * lp.m, seed=2))
    assert r.status == "optimal"
    assert abs(r.obj_p - lp.opt) <= 2e-8 * max(1.0, abs(lp.opt))
    assert max(h["cg_iters"] for h in r.history) <= 40


def test_planted_mistake_in_gaussian_scale_fails_the_variance_pin():
    """Dropping the factor 2 of -2 ln u1 halves the variance: the moment pin
    catches it."""
    from oracle import sketch as S
    base = S.mix_int(7 + S.GOLDEN * 1)
    idx = np.arange(100000, dtype=np.uint64)
    h1 = S.mix_array(np.uint64(base) ^ (idx * np.uint64(2)))
    h2 = S.mix_array(np.uint64(base) ^ (idx * np.uint64(2) + np.uint64(1)))
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    bad = np.sqrt(-np.log(u1)) * np.cos(2.0 * np.pi * u2)
    good = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    assert abs(good.var() - 1.0) < 0.02
    assert abs(bad.var() - 1.0) > 0.3


# ---------------------------------------------------------------------------
# App. A (Richardson, Alg. 3) and App. B (steepest descent, Alg. 4)
# ---------------------------------------------------------------------------

def _good_sketch_system(lp, seed=3):
    """A mid-IPM A D and a sketch wide and dense enough for ||I - M|| < 1."""
    x, y, s, _ = _mid_iterate(lp, 3)
    AD = _scaled(lp, x, s)
    W = sketch_matrix(seed, 0, 8, lp.n, lp.n)
    p = np.random.default_rng(seed).standard_normal(lp.m)
    return AD, W, p


def test_richardson_residual_recursion_closed_form(small_lp):
    """Lemma (App. A): f^(j) = (I - M)^j f^(0), M = Q^{-1/2} A D^2 A^T Q^{-1/2};
    the powers are taken from M's eigendecomposition, not from the iteration."""
    AD, W, p = _good_sketch_system(small_lp)
    res = O.sketch_richardson(AD, p, W, t=6)
    M = res.Qmh @ AD @ AD.T @ res.Qmh
    lam, V = np.linalg.eigh((M + M.T) / 2)
    f0 = -(res.Qmh @ p)
    for j in range(7):
        fj = V @ ((1.0 - lam) ** j * (V.T @ f0))
        assert abs(res.f_norms[j] - np.linalg.norm(fj)) <= 1e-10 * np.linalg.norm(f0)


def test_richardson_contracts_by_zeta(small_lp):
    """Lemma (App. A): ||f^(j)|| <= zeta ||f^(j-1)|| with zeta = ||I - M||_2 < 1."""
    AD, W, p = _good_sketch_system(small_lp, seed=5)
    res = O.sketch_richardson(AD, p, W, t=8)
    sv = np.linalg.svd(res.Qmh @ AD, compute_uv=False)
    zeta = max(abs(1 - sv[0] ** 2), abs(1 - sv[-1] ** 2))
    assert zeta < 1
    f = res.f_norms
    for j in range(1, len(f)):
        assert f[j] <= zeta * f[j - 1] * (1 + 1e-9)


def test_steepest_descent_line_search_and_orthogonality(small_lp):
    """Alg. 4: alpha_j is the exact minimiser of the quadratic along -f^(j), so
    consecutive residuals are orthogonal (App. B)."""
    AD, W, p = _good_sketch_system(small_lp, seed=7)
    Qmh, _, _, _ = O.sketch_preconditioner(AD, W)
    M = Qmh @ AD @ AD.T @ Qmh
    rhs = Qmh @ p

    def phi(z):
        return 0.5 * z @ M @ z - rhs @ z

    prev = None
    for t in range(1, 6):
        z = O.sketch_sd(AD, p, W, t=t).z
        f = M @ z - rhs
        if prev is not None:
            zp, fp = prev
            assert abs(f @ fp) <= 1e-9 * np.linalg.norm(f) * np.linalg.norm(fp) + 1e-14
            a = (fp @ fp) / (fp @ M @ fp)
            for scale in (0.9, 1.1):
                assert phi(zp - a * fp) < phi(zp - scale * a * fp)
        prev = (z, f)


def test_richardson_and_sd_converge_to_cholesky_solution(small_lp):
    AD, W, p = _good_sketch_system(small_lp, seed=9)
    dy = np.linalg.solve(AD @ AD.T, p)
    for solver in (O.sketch_richardson, O.sketch_sd):
        res = solver(AD, p, W, tol=1e-13, max_it=500)
        assert np.linalg.norm(res.dy - dy) <= 1e-9 * np.linalg.norm(dy), solver.__name__


def test_exact_preconditioner_one_step_for_every_inner_solver(small_lp):
    """With a signed-permutation W, Q = A D^2 A^T and M = I: Richardson and
    steepest descent (alpha = 1) both finish in one iteration."""
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    AD = _scaled(lp, x, s)
    rng = np.random.default_rng(11)
    W = sp.csr_matrix((rng.choice([-1.0, 1.0], lp.n), (np.arange(lp.n), rng.permutation(lp.n))),
                      shape=(lp.n, lp.n))
    p = rng.standard_normal(lp.m)
    dy = np.linalg.solve(AD @ AD.T, p)
    for solver in (O.sketch_richardson, O.sketch_sd):
        res = solver(AD, p, W, tol=1e-10, max_it=50)
        assert res.iters == 1
        assert np.linalg.norm(res.dy - dy) <= 1e-9 * np.linalg.norm(dy)


def test_ipm_with_each_inner_solver_reaches_the_planted_optimum():
    lp = dense_planted(12, 200, rng=np.random.default_rng(21), eps_gap=1e-8)
    for inner in ("sd", "richardson"):
        r = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="sketch", eps_gap=1e-8, w=lp.n,
                                                  s_nnz=8, seed=4, inner=inner, max_cg=2000))
        assert r.status == "optimal", inner
        assert abs(r.obj_p - lp.opt) <= 2e-8 * max(1.0, abs(lp.opt)), inner


def test_planted_mistake_in_richardson_sign_breaks_recursion(small_lp):
    """The closed form of the Richardson residual catches a step whose
    correction enters with the wrong sign (z - Q^{-1/2}(p - ...))."""
    AD, W, p = _good_sketch_system(small_lp)
    good = O.sketch_richardson(AD, p, W, t=3)
    Qmh = good.Qmh
    M = Qmh @ AD @ AD.T @ Qmh
    lam, V = np.linalg.eigh((M + M.T) / 2)
    f0 = -(Qmh @ p)
    f3 = np.linalg.norm(V @ ((1.0 - lam) ** 3 * (V.T @ f0)))
    z = np.zeros_like(p)
    for _ in range(3):
        z = z - Qmh @ (p - AD @ (AD.T @ (Qmh @ z)))
    bad_f3 = np.linalg.norm(M @ z - Qmh @ p)
    assert abs(good.f_norms[3] - f3) <= 1e-10 * np.linalg.norm(f0)
    assert abs(bad_f3 - f3) > 1e-3 * np.linalg.norm(f0)


# ---------------------------------------------------------------------------
# planted mistakes are caught
# ---------------------------------------------------------------------------

def test_planted_mistake_in_rhs_breaks_segment(monkeypatch, small_lp):
    lp = small_lp

    def bad_rhs(A, b, c, x, y, s, sigma, mu):  # drops the A x term of eq. pdef
        rp, rd = O.residuals(A, b, c, x, y, s)
        return -rp - sigma * mu * (A @ (1.0 / s)) - A @ ((x / s) * rd)

    monkeypatch.setattr(O, "normal_rhs", bad_rhs)
    x, y, s = np.ones(lp.n), np.zeros(lp.m), np.ones(lp.n)
    d = O.exact_direction(lp.A, lp.b, lp.c, x, y, s, 0.5)
    # eq. iip_3_1 no longer holds
    assert np.linalg.norm(lp.A @ d.dx + d.rp) > 1e-3 * np.linalg.norm(d.rp)


def test_planted_mistake_in_v_breaks_addl(small_lp):
    lp = small_lp
    x, y, s, _ = _mid_iterate(lp)
    W = sketch_matrix(3, 1, 1, lp.n, lp.w)
    d = O.sketch_direction(lp.A, lp.b, lp.c, x, y, s, 0.5, W, tol_cg=1e-2)
    g = lp.A @ ((x / s) * (lp.A.T @ d.dy)) - d.p
    res = d.pcg
    t = res.Vh.T @ ((res.U.T @ g) / res.sv)
    good = np.sqrt(x * s) * (W @ t)
    assert np.linalg.norm(lp.A @ (good / s) - g) <= 1e-10 * np.linalg.norm(g)
    # (X S)^{1/2} replaced by X^{1/2} S^{-1/2} = D: eq. addl fails
    bad = np.sqrt(x / s) * (W @ t)
    assert np.linalg.norm(lp.A @ (bad / s) - g) > 1e-2 * np.linalg.norm(g)
    # singular values used instead of their inverses: eq. addl fails
    t_bad = res.Vh.T @ ((res.U.T @ g) * res.sv)
    bad2 = np.sqrt(x * s) * (W @ t_bad)
    assert np.linalg.norm(lp.A @ (bad2 / s) - g) > 1e-2 * np.linalg.norm(g)
