"""The seeded synthetic LP generators: shapes, planted optimality, determinism."""
import numpy as np
import scipy.sparse as sp

from lpgen import batch_lp, config_lp, csr_planted, dense_planted, serving_lp, serving_trace


def _check_planted(lp, tol=1e-9):
    x, y, s = lp.x_star, lp.y_star, lp.s_star
    assert np.all(x >= 0) and np.all(s >= 0)
    assert float(np.abs(x * s).max()) == 0.0
    assert np.linalg.norm(lp.A @ x - lp.b) <= tol * max(1.0, np.linalg.norm(lp.b))
    assert np.linalg.norm(lp.A.T @ y + s - lp.c) <= tol * max(1.0, np.linalg.norm(lp.c))
    assert abs(lp.c @ x - lp.b @ y) <= 1e-9 * max(1.0, abs(lp.c @ x))


def test_config0_shape_and_planting():
    lp = config_lp(0)
    assert lp.A.shape == (50, 1000) and lp.w == 200 and lp.eps_gap == 1e-8
    assert int((lp.x_star > 0).sum()) == 50
    _check_planted(lp)
    lp2 = config_lp(0)
    assert np.array_equal(lp.A, lp2.A) and np.array_equal(lp.c, lp2.c)


def test_f32_values_are_representable():
    lp = dense_planted(10, 200, rng=np.random.default_rng(1), a_dtype="f32")
    assert np.array_equal(lp.A.astype(np.float32).astype(np.float64), lp.A)
    _check_planted(lp)


def test_csr_generator_structure():
    lp = csr_planted(30, 5000, 0.002, rng=np.random.default_rng(2))
    A = lp.A
    assert sp.isspmatrix_csr(A)
    counts = np.diff(A.indptr)
    assert np.all(counts[:-1] == 10) and counts[-1] == 5000
    assert np.all(A[-1].toarray() == 1.0)
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    vals = A.data[: A.indptr[-2]]
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    _check_planted(lp)


def test_batch_and_serving_shapes():
    for i in range(5):
        lp = batch_lp(i)
        assert 20 <= lp.m <= 400 and lp.n % lp.m == 0 and 20 <= lp.n // lp.m <= 200
        assert lp.w == 4 * lp.m
    tr = serving_trace(200)
    ts = [r["t"] for r in tr]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert 0.5 < ts[-1] / (200 / 200.0) < 1.5
    for r in tr:
        assert 50 <= r["m"] <= 2000 and 50 * r["m"] - 1 <= r["n"] <= 500 * r["m"] + 1
    small = min(tr, key=lambda r: r["m"] * r["n"])
    lp = serving_lp(small)
    _check_planted(lp)


def _check_device_planted(A, lp, support):
    x, y, s = lp.x_star.numpy(), lp.y_star.numpy(), lp.s_star.numpy()
    assert np.allclose(A @ x, lp.b.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(A.T @ y + s, lp.c.numpy(), rtol=1e-12, atol=1e-12)
    assert np.all(x >= 0) and np.all(s >= 0) and np.all(x * s == 0)
    assert np.count_nonzero(x) == support
    assert abs(lp.opt - float(lp.c.numpy() @ x)) <= 1e-12 * max(1.0, abs(lp.opt))
    assert abs(lp.opt - float(lp.b.numpy() @ y)) <= 1e-9 * max(1.0, abs(lp.opt))


def test_device_generators_plant_an_optimum_on_cpu():
    import scipy.sparse as ssp
    import torch
    from lpgen.device import csr_planted_device, dense_planted_device
    lp = dense_planted_device(30, 700, seed=5, dev="cpu")
    assert lp.A.dtype == torch.float32 and lp.A.t().is_contiguous()   # column-major storage
    _check_device_planted(lp.A.to(torch.float64).numpy(), lp, 30)
    sp = csr_planted_device(12, 3000, 0.01, seed=6, dev="cpu")
    rowptr, colidx, vals = (t.numpy() for t in sp.A)
    assert rowptr[0] == 0 and rowptr[-1] == colidx.size and np.all(np.diff(rowptr) >= 0)
    for i in range(sp.m - 1):
        cols = colidx[rowptr[i]:rowptr[i + 1]]
        assert cols.size == 30 and np.all(np.diff(cols) > 0)
        assert cols.min() >= 0 and cols.max() < sp.n
    last = slice(rowptr[-2], rowptr[-1])
    assert np.array_equal(colidx[last], np.arange(sp.n)) and np.all(vals[last] == 1.0)
    Asp = ssp.csr_matrix((vals.astype(np.float64), colidx, rowptr), shape=(sp.m, sp.n))
    _check_device_planted(Asp, sp, 12)


# ---------------------------------------------------------------------------
# l1-SVM stand-in LPs (App. D.1)
# ---------------------------------------------------------------------------

def test_svm_lp_structure():
    from lpgen import SVM_SHAPES, svm_lp
    for dens in (1.0, 0.02):
        lp = svm_lp(12, 80, density=dens, seed=4)
        A = lp.A.toarray() if sp.issparse(lp.A) else lp.A
        N = 80
        assert A.shape == (12, 2 * N + 1)          # m x (2N + 1)
        X = lp.X.toarray() if sp.issparse(lp.X) else lp.X
        assert np.all(X >= 0) and np.all(np.abs(lp.y) == 1)
        assert np.count_nonzero(lp.y > 0) == 6     # the upper half by score is class +1
        assert np.array_equal(A[:, :N], lp.y[:, None] * X)
        assert np.array_equal(A[:, N:2 * N], -A[:, :N])
        assert np.array_equal(A[:, 2 * N], lp.y)
        assert np.array_equal(lp.b, np.ones(12))
        assert np.array_equal(lp.c, np.r_[np.ones(2 * N), 0.0])
        assert np.all((X != 0).sum(axis=1) >= 1)
    again = svm_lp(12, 80, density=0.02, seed=4)
    assert (again.A != svm_lp(12, 80, density=0.02, seed=4).A).nnz == 0
    assert set(SVM_SHAPES) == {"arcene", "dexter", "drivface", "gene_rna"}


def test_svm_oracle_matches_an_independent_lp_solver():
    """Pin of the oracle on the SVM LPs: HiGHS (scipy's simplex / IPM code,
    shares nothing with the oracle) gives the same optimal value, and the
    oracle's solution is an SVM of that l1 norm with every point on its margin."""
    import scipy.optimize as so

    from lpgen import svm_lp
    from oracle import ipm as O
    for m, N, dens in ((20, 300, 1.0), (30, 3000, 0.01)):
        lp = svm_lp(m, N, density=dens, seed=1)
        ref = so.linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
        assert ref.status == 0
        A = lp.A.toarray() if sp.issparse(lp.A) else lp.A
        X = lp.X.toarray() if sp.issparse(lp.X) else lp.X
        for prm in (O.IPMParams(solver="sketch", sketch="gaussian", w=2 * m, seed=3, eps_gap=1e-9),
                    O.IPMParams(solver="sketch", w=4 * m, s_nnz=2, seed=3, eps_gap=1e-9)):
            r = O.ipm(A, lp.b, lp.c, prm)
            assert r.status == "optimal", (m, N, prm.sketch, r.status)
            assert abs(r.obj_p - ref.fun) <= 1e-8 * ref.fun
            wv = r.x[:N] - r.x[N:2 * N]
            bias = r.x[2 * N]
            assert np.abs(lp.y * (X @ wv + bias) - 1).max() <= 1e-7
            assert abs(np.abs(wv).sum() - ref.fun) <= 1e-7 * ref.fun
