"""Planted short-and-fat LPs  min c^T x  s.t.  A x = b, x >= 0  (m << n).

Every problem plants an optimum (x*, y*, s*): x* is Uniform(0,1) on a random
support of size `support`, s* is Uniform(0,1) off that support and zero on it,
y* ~ N(0,1); then b = A x* and c = A^T y* + s*.  Since x* o s* = 0 and both are
non-negative, (x*, y*, s*) is primal-dual optimal and the optimal objective is
exactly c^T x* = b^T y*.

Draw order (one numpy PCG64 stream per problem, seeded by SeedSequence([cfg, idx])):
A, then the support (choice without replacement), then x*[support], then s*
(s*[support] set to 0), then y*.  FP32-valued problems draw A in FP64 and round
it to FP32 (round to nearest even); that rounded matrix is the problem, and b, c
are formed in FP64 from it.

Workload shapes (sizes of the synthetic stand-ins for the paper's short-and-fat
LPs):
  cfg 0  dense 50 x 1000 FP64,             support 50,   w = 200,  gap 1e-8
  cfg 1  dense 500 x 100000 FP64,          support 500,  w = 2000, gap 1e-6
  cfg 2  CSR 1000 x 1000000, 0.1% density, FP32 values, plus an all-ones last
         row (no empty column), support 1000, w = 4000, gap 1e-6
  cfg 3  256 dense FP32 LPs, m ~ U{20..400}, n = m k, k ~ U{20..200}, w = 4m
  cfg 4  serving trace: Poisson arrivals (200/s), m log-uniform [50, 2000],
         n/m log-uniform [50, 500], 50/50 dense FP32 / 1%-density CSR (+ones row)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class PlantedLP:
    A: object            # numpy (m, n) float64 C-order array, or scipy.sparse.csr_matrix
    b: np.ndarray        # (m,) float64
    c: np.ndarray        # (n,) float64
    x_star: np.ndarray
    y_star: np.ndarray
    s_star: np.ndarray
    w: int               # sketch width
    eps_gap: float       # relative duality-gap stopping tolerance
    seed: int            # sketch seed
    a_dtype: str         # "f64" or "f32": the precision A's values are representable in
    fmt: str             # "dense" or "csr"
    name: str = ""

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def opt(self) -> float:
        """Planted optimal objective c^T x* (= b^T y*)."""
        return float(self.c @ self.x_star)


CONFIGS = {
    0: dict(m=50, n=1000, w=200, fmt="dense", a_dtype="f64", eps_gap=1e-8),
    1: dict(m=500, n=100_000, w=2000, fmt="dense", a_dtype="f64", eps_gap=1e-6),
    2: dict(m=1000, n=1_000_000, w=4000, fmt="csr", a_dtype="f32", eps_gap=1e-6,
            density=1e-3),
}


def sketch_seed(cfg: int, idx: int = 0) -> int:
    return 0x5EED0000 + cfg + (idx << 20)


def _plant(rng, A, n, support):
    supp = rng.choice(n, support, replace=False)
    x = np.zeros(n)
    x[supp] = rng.uniform(size=support)
    s = rng.uniform(size=n)
    s[supp] = 0.0
    y = rng.standard_normal(A.shape[0])
    b = np.asarray(A @ x, dtype=np.float64).ravel()
    c = np.asarray(A.T @ y, dtype=np.float64).ravel() + s
    return x, y, s, b, c


def dense_planted(m, n, support=None, rng=None, a_dtype="f64", w=None,
                  eps_gap=1e-6, seed=0, name="") -> PlantedLP:
    """Dense Gaussian A (m x n) with a planted optimum of the given support size."""
    rng = rng if rng is not None else np.random.default_rng(0)
    support = m if support is None else support
    A = rng.standard_normal((m, n))
    if a_dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    x, y, s, b, c = _plant(rng, A, n, support)
    return PlantedLP(A, b, c, x, y, s, w if w else 4 * m, eps_gap, seed, a_dtype,
                     "dense", name)


def csr_planted(m, n, density, support=None, rng=None, w=None, eps_gap=1e-6,
                seed=0, name="") -> PlantedLP:
    """Sparse A: rows 0..m-2 each get round(density*n) distinct uniform columns
    (sorted) with N(0,1) values rounded to FP32; the last row is all ones so no
    column is empty."""
    rng = rng if rng is not None else np.random.default_rng(0)
    support = m if support is None else support
    k = max(1, int(round(density * n)))
    cols = [np.sort(rng.choice(n, k, replace=False)) for _ in range(m - 1)]
    vals = rng.standard_normal((m - 1) * k).astype(np.float32).astype(np.float64)
    indptr = np.zeros(m + 1, dtype=np.int64)
    indptr[1:m] = k * np.arange(1, m)
    indptr[m] = k * (m - 1) + n
    indices = np.concatenate(cols + [np.arange(n)])
    data = np.concatenate([vals, np.ones(n)])
    A = sp.csr_matrix((data, indices, indptr), shape=(m, n))
    x, y, s, b, c = _plant(rng, A, n, support)
    return PlantedLP(A, b, c, x, y, s, w if w else 4 * m, eps_gap, seed, "f32",
                     "csr", name)


def config_lp(cfg: int, idx: int = 0) -> PlantedLP:
    """The single-LP workloads (configs 0, 1, 2)."""
    p = CONFIGS[cfg]
    rng = np.random.default_rng(np.random.SeedSequence([cfg, idx]))
    name = f"cfg{cfg}"
    if p["fmt"] == "dense":
        return dense_planted(p["m"], p["n"], p["m"], rng, p["a_dtype"], p["w"],
                             p["eps_gap"], sketch_seed(cfg, idx), name)
    return csr_planted(p["m"], p["n"], p["density"], p["m"], rng, p["w"],
                       p["eps_gap"], sketch_seed(cfg, idx), name)


def batch_shape(idx: int):
    """(m, k) of LP `idx` of the batched workload: m ~ U{20..400}, k ~ U{20..200}
    (the first two draws of that LP's stream)."""
    rng = np.random.default_rng(np.random.SeedSequence([3, idx]))
    return int(rng.integers(20, 401)), int(rng.integers(20, 201))


def batch_lp(idx: int) -> PlantedLP:
    """LP `idx` of the batched workload: m ~ U{20..400}, n = m*k, k ~ U{20..200},
    dense FP32 values, support m, w = 4m."""
    rng = np.random.default_rng(np.random.SeedSequence([3, idx]))
    m = int(rng.integers(20, 401))
    k = int(rng.integers(20, 201))
    return dense_planted(m, m * k, m, rng, "f32", 4 * m, 1e-6, sketch_seed(3, idx),
                         f"batch{idx}")


def serving_trace(n_req: int = 2000, rate: float = 200.0, seed: int = 4):
    """Arrival times and shapes of the serving workload: Poisson arrivals at
    `rate`/s; m = round(exp(U(ln 50, ln 2000))); n = round(m*exp(U(ln 50, ln 500)));
    kind alternates by a fair coin between dense and CSR."""
    rng = np.random.default_rng(np.random.SeedSequence([4, seed]))
    gaps = rng.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps)
    m = np.rint(np.exp(rng.uniform(math.log(50), math.log(2000), n_req))).astype(int)
    ratio = np.exp(rng.uniform(math.log(50), math.log(500), n_req))
    n = np.rint(m * ratio).astype(int)
    kind = np.where(rng.uniform(size=n_req) < 0.5, "dense", "csr")
    return [dict(idx=i, t=float(t[i]), m=int(m[i]), n=int(n[i]), kind=str(kind[i]))
            for i in range(n_req)]


def serving_lp(req: dict) -> PlantedLP:
    """Problem data of one serving request (see `serving_trace`)."""
    idx = req["idx"]
    rng = np.random.default_rng(np.random.SeedSequence([4, 1_000_000 + idx]))
    m, n = req["m"], req["n"]
    if req["kind"] == "dense":
        return dense_planted(m, n, m, rng, "f32", 4 * m, 1e-6, sketch_seed(4, idx),
                             f"req{idx}")
    return csr_planted(m, n, 0.01, m, rng, 4 * m, 1e-6, sketch_seed(4, idx),
                       f"req{idx}")
