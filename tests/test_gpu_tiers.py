"""Precision tiers of the CG products (SKIPM_PREC_MIXED / SKIPM_PREC_BF16)
through the C ABI.

The BF16 copy of A is A rounded to 8 significant bits (ties to even); the
product pass widens it exactly to FP64 and accumulates in FP64, so its result
is compared element by element with the oracle's normal matrix of that rounded
A, within the summation bound.  Solves at the BF16 start tier meet the same
bar as every other solve (planted optimum, KKT residuals), because the
normal-equation residual that decides each CG solve is the FP64 one; the tier
only moves up (BF16 -> FP32 -> FP64) and is reported per IPM iteration.
"""
import sys

import numpy as np
import pytest

from lpgen import config_lp, dense_planted
from oracle import ipm as O

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


def bf16_round(a):
    """a rounded to bfloat16: 8 significant bits, ties to even (exact in FP64:
    scaling by a power of two and numpy's half-to-even rounding)."""
    a = np.asarray(a, dtype=np.float64)
    _, e = np.frexp(a)                       # a = f 2^e, 0.5 <= |f| < 1
    return np.ldexp(np.round(np.ldexp(a, 8 - e)), e - 8)


def test_bf16_rounding_definition():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3 2^-8 rounds up
    assert bf16_round(1 + 2.0 ** -8) == 1.0
    assert bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert bf16_round(-255.5) == -256.0 and bf16_round(0.0) == 0.0
    x = np.random.default_rng(0).standard_normal(1000)
    r = bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))   # unit roundoff 2^-8
    assert np.array_equal(r.astype(np.float32).astype(np.float64), r)


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,dt", [(37, 3001, "f64"), (130, 5000, "f64"), (300, 20000, "f32"),
                                    (500, 100_000, "f64"), (2048, 6000, "f64")])
def test_bf16_product_matches_oracle(torch, sk, m, n, dt):
    """One fused pass over the BF16 copy (lane-group shapes 16x1, 16x2, 64x1
    and 64x4, the last the largest m) against the oracle's normal matrix of the
    BF16-rounded A with D^2 = x / s of the iterate the step starts from."""
    rng = np.random.default_rng(m + 7)
    lp = dense_planted(m, n, rng=rng, a_dtype=dt)
    x, s_ = rng.uniform(0.1, 10.0, n), rng.uniform(0.1, 10.0, n)
    y, u = rng.standard_normal(m), rng.standard_normal(m)
    say(f"bf16 product m={m} n={n} {dt}")
    with sk.LP(lp.A, lp.b, lp.c, a_dtype=dt, s=2, seed=3, precision=sk.SKIPM_PREC_BF16,
               max_cg=1) as h:
        h.set_iterate(x, y, s_)
        h.pcg(x / s_, np.ones(m), 0, tol=0.0, max_it=1)   # D^2 = X S^{-1}, tier stays BF16
        q = h.normal_matvec(u).cpu().numpy()
    Ab = bf16_round(lp.A)
    d2 = x / s_
    ref = O.normal_matrix(Ab, d2) @ u
    bound = np.abs(Ab) @ (d2 * (np.abs(Ab).T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 2 * (m + n) * EPS * bound)
    # and it is not the product of the unrounded A
    full = O.normal_matrix(lp.A, d2) @ u
    assert np.max(np.abs(q - full) / bound) > 100 * (m + n) * EPS


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,s_nnz", [(60, 2000, 2), (80, 4000, 1), (257, 3000, 2)])
def test_solve_bf16_start_tier(torch, sk, m, n, s_nnz):
    lp = dense_planted(m, n, rng=np.random.default_rng(m + n), eps_gap=1e-8)
    say(f"solve bf16 start tier {m} x {n} s={s_nnz}")
    with sk.LP(lp.A, lp.b, lp.c, s=s_nnz, seed=m, eps_gap=1e-8,
               precision=sk.SKIPM_PREC_BF16) as h:
        res = h.solve()
    assert res.status == 0, res
    assert abs(res.obj_p - lp.opt) <= 2e-8 * max(1.0, abs(lp.opt))
    assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
    assert res.rd_norm <= 1e-8 * np.linalg.norm(lp.c)
    assert res.cg_max <= 1000   # the default cap per normal-equation solve
    assert (res.demote_iter == -1) == (res.tier_final == sk.SKIPM_TIER_BF16)


@pytest.mark.gpu
def test_tier_trace_only_moves_up(torch, sk):
    """Step by step from the start: every iteration reports its tier and
    refinement steps; the tier never moves down, and the first iteration at a
    higher tier is the one lp_solve reports as demote_iter."""
    lp = dense_planted(80, 4000, rng=np.random.default_rng(6), eps_gap=1e-8)
    say("tier trace 80 x 4000 s=1 bf16")
    kw = dict(s=1, seed=2, eps_gap=1e-8, precision=sk.SKIPM_PREC_BF16)
    tiers = []
    with sk.LP(lp.A, lp.b, lp.c, **kw) as h:
        for _ in range(300):
            info = h.step()
            if info.converged:
                break
            tiers.append((info.tier, info.refine_steps, info.cg_iters))
        h.reset()
        res = h.solve()
    assert res.status == 0
    order = {sk.SKIPM_TIER_BF16: 0, sk.SKIPM_TIER_FP32: 1, sk.SKIPM_TIER_FP64: 2}
    ranks = [order[t] for t, _, _ in tiers]
    assert ranks == sorted(ranks)
    assert tiers[0][0] in (sk.SKIPM_TIER_BF16, sk.SKIPM_TIER_FP32)
    assert all(r >= 1 for _, r, _ in tiers)
    first_up = next((k for k, (t, _, _) in enumerate(tiers) if t != sk.SKIPM_TIER_BF16), -1)
    assert res.demote_iter == first_up
    assert res.iters == len(tiers)


@pytest.mark.gpu
def test_config1_bf16_solve(torch, sk):
    """The bench's 500 x 100000 LP from the BF16 start tier (s = 1): planted
    optimum and KKT residuals at rel. gap 1e-6."""
    lp = config_lp(1)
    say("solve config 1 from the bf16 tier (s=1)")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap,
               precision=sk.SKIPM_PREC_BF16) as h:
        res = h.solve()
    assert res.status == 0, res
    assert abs(res.obj_p - lp.opt) <= 2e-6 * max(1.0, abs(lp.opt))
    assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
    assert res.rd_norm <= 1e-8 * np.linalg.norm(lp.c)
