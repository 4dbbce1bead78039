"""The l1-SVM LPs of the paper's experiments (App. D.1), on synthetic stand-in
data, solved through the C ABI.

Expected values come from HiGHS (scipy's LP solver, independent of both the
oracle and the HIP path) and from the oracle run with the same sketch.
Tolerances: objective within 2 eps_gap of HiGHS's (relative); every point on
its margin to 1e-7; KKT residuals at most 1e-8 of ||b||, ||c||; outer iteration
count within 2 of the oracle's (same sketch matrices; rounding differs).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from lpgen import svm_lp, svm_shape_lp
from oracle import ipm as O

pytestmark = pytest.mark.gpu


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


def highs_opt(lp):
    import scipy.optimize as so
    r = so.linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert r.status == 0
    return r.fun


def check_svm(lp, res, x, opt, gap):
    assert res.status == 0, res
    assert abs(res.obj_p - opt) <= 2 * gap * opt
    assert res.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
    assert res.rd_norm <= 1e-8 * np.linalg.norm(lp.c)
    N = lp.X.shape[1]
    wv = x[:N] - x[N:2 * N]
    margins = lp.y * (np.asarray(lp.X @ wv).ravel() + x[2 * N])
    assert np.abs(margins - 1).max() <= 1e-7


CASES = [
    # (m, N, density, format, sketch, w / m, s)
    (40, 2000, 1.0, "dense", "gaussian", 2, 1),
    (40, 2000, 1.0, "dense", "count", 4, 2),
    (30, 3000, 0.01, "csr", "count", 4, 2),
    (30, 3000, 0.01, "dense", "gaussian", 2, 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-{c[3]}-{c[4]}")
def test_svm_solve_matches_highs_and_oracle(torch, sk, case):
    m, N, dens, fmt, sketch, wf, s = case
    lp = svm_lp(m, N, density=dens, seed=1)
    A = lp.A.toarray() if sp.issparse(lp.A) else lp.A
    Ain = sp.csr_matrix(A) if fmt == "csr" else A
    say(f"svm {m}x{N} density {dens} {fmt} {sketch} w={wf}m s={s}")
    with sk.LP(Ain, lp.b, lp.c, w=wf * m, s=s, seed=3, eps_gap=1e-9, max_outer=1000,
               sketch=sk.SKIPM_SKETCH_GAUSSIAN if sketch == "gaussian" else sk.SKIPM_SKETCH_COUNT) as h:
        h.kernel_timing(8)
        res = h.solve()
        x, _, _ = h.get_iterate()
        x = x.cpu().numpy()
        sk_ms, sk_n = h.sketch_time()
    check_svm(lp, res, x, highs_opt(lp), 1e-9)
    # one timed sketch product per IPM iteration that computed a direction
    assert sk_n == res.iters and sk_ms > 0
    ref = O.ipm(A, lp.b, lp.c, O.IPMParams(solver="sketch", sketch=sketch, w=wf * m, s_nnz=s,
                                            seed=3, eps_gap=1e-9, max_outer=1000))
    assert ref.status == "optimal"
    assert abs(res.iters - ref.iters) <= 2, (res.iters, ref.iters)


def test_svm_arcene_shape_gaussian(torch, sk):
    """The ARCENE shape of Table 1 (100 points, 10,000 features, LP 100 x 20,001,
    Gaussian sketch of width 200, the paper's setting) on stand-in data."""
    lp = svm_shape_lp("arcene")
    say("svm arcene shape 100 x 20001 gaussian w=200, gap 1e-9")
    with sk.LP(lp.A, lp.b, lp.c, w=lp.w, seed=lp.seed, eps_gap=1e-9, max_outer=1000,
               sketch=sk.SKIPM_SKETCH_GAUSSIAN) as h:
        res = h.solve()
        x, _, _ = h.get_iterate()
        x = x.cpu().numpy()
    check_svm(lp, res, x, highs_opt(lp), 1e-9)
    ref = O.ipm(lp.A, lp.b, lp.c, O.IPMParams(solver="sketch", sketch="gaussian", w=lp.w,
                                               seed=lp.seed, eps_gap=1e-9, max_outer=1000))
    assert ref.status == "optimal"
    assert abs(res.iters - ref.iters) <= 2, (res.iters, ref.iters)
    # the inner iteration count stays far below the unpreconditioned CG's
    assert res.cg_max <= 100
