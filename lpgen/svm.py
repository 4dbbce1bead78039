"""l1-regularised SVM LPs (the application of the paper's experiments, App. D.1).

The SVM problem  min ||w||_1  s.t.  y_i (w^T x_i + b') >= 1  is written as a
standard form LP (A x = b, x >= 0) of m rows and 2N + 1 columns, the size the
paper gives for it: w = w+ - w-, one column for the bias, and the m margin
constraints held with equality (every point on its margin; with m << N the
system is underdetermined, so this is a basis-pursuit LP that is feasible and
bounded).  A standard form LP of that size has no room for surplus columns, so
the bias is one non-negative variable:

    variables  (w+, w-, b')                   sizes N, N, 1
    A        = [ Y X,  -Y X,  y ]              (m x (2N + 1)),  Y = diag(y)
    b        = 1_m
    c        = (1_N, 1_N, 0)

The data are synthetic stand-ins for the paper's data sets (which are not
available here): m points with N non-negative features (U(0, 1), kept with
probability `density`, every point with at least one), split into two equal
classes by their score under a random sparse hyperplane.  The optimum is not
planted: its value comes from an independent LP solver.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class SvmLP:
    A: object       # dense (m, ncols) float64, or scipy.sparse CSR
    b: np.ndarray
    c: np.ndarray
    X: object       # the feature matrix (m, N)
    y: np.ndarray   # labels in {-1, +1}
    w: int          # sketch width
    eps_gap: float
    seed: int
    a_dtype: str
    fmt: str
    name: str = ""

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


# the shapes of the paper's Table 1 (m points x N features; the LP has
# 2N + 1 columns) with its sketch widths
SVM_SHAPES = {
    "arcene": dict(m=100, N=10_000, w=200, density=1.0),
    "dexter": dict(m=300, N=20_000, w=500, density=0.005),
    "drivface": dict(m=606, N=6_400, w=1000, density=1.0),
    "gene_rna": dict(m=801, N=20_531, w=2000, density=1.0),
}


def svm_lp(m, N, density=1.0, seed=0, w=None, eps_gap=1e-6, name="") -> SvmLP:
    rng = np.random.default_rng(np.random.SeedSequence([5, seed]))
    if density >= 1.0:
        X = rng.uniform(size=(m, N))
    else:
        X = sp.random(m, N, density=density, format="csr", random_state=rng,
                      data_rvs=lambda k: rng.uniform(size=k))
        # every point gets at least one feature
        X = (X + sp.csr_matrix((rng.uniform(size=m), (np.arange(m), rng.integers(0, N, m))),
                               shape=(m, N))).tocsr()
    # labels from a sparse hyperplane through the data's centre
    k = max(1, N // 20)
    wt = np.zeros(N)
    wt[rng.choice(N, k, replace=False)] = rng.standard_normal(k)
    score = np.asarray(X @ wt).ravel()
    # the upper half of the points by score (ties broken at random) is class +1
    order = np.lexsort((rng.uniform(size=m), score))
    y = -np.ones(m)
    y[order[m // 2:]] = 1.0
    if sp.issparse(X):
        YX = (sp.diags(y) @ X).tocsr()
        A = sp.hstack([YX, -YX, sp.csr_matrix(y[:, None])], format="csr")
        fmt = "csr"
    else:
        YX = y[:, None] * X
        A = np.hstack([YX, -YX, y[:, None]])
        fmt = "dense"
    b = np.ones(m)
    c = np.concatenate([np.ones(2 * N), np.zeros(1)])
    return SvmLP(A, b, c, X, y, w if w else 4 * m, eps_gap, 0x5EED0000 + 5 + (seed << 20),
                 "f64", fmt, name)


def svm_shape_lp(name: str, seed: int = 0) -> SvmLP:
    p = SVM_SHAPES[name]
    return svm_lp(p["m"], p["N"], p["density"], seed, p["w"], 1e-6, name)
