"""Brute-force LP solution by vertex enumeration (tiny problems only).

TEST INFRASTRUCTURE ONLY.  A bounded standard-form LP  min c^T x, A x = b,
x >= 0  attains its optimum at a basic feasible solution; enumerating every
choice of m columns (basis) and keeping the feasible ones finds it.
"""
from __future__ import annotations

import itertools

import numpy as np


def vertex_enum(A, b, c, det_tol=1e-12, feas_tol=1e-12):
    """Return (optimal value, x) over all basic feasible solutions, or
    (None, None) when no basis is feasible."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    best, best_x = None, None
    for basis in itertools.combinations(range(n), m):
        AB = A[:, basis]
        if abs(np.linalg.det(AB)) < det_tol:
            continue
        xB = np.linalg.solve(AB, b)
        if np.any(xB < -feas_tol):
            continue
        x = np.zeros(n)
        x[list(basis)] = np.maximum(xB, 0.0)
        val = float(c @ x)
        if best is None or val < best:
            best, best_x = val, x
    return best, best_x
