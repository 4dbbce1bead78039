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
