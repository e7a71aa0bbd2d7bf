"""Brute-force LP optimum by vertex enumeration (oracle; test infrastructure only).

For ``min c^T x, A x = b, x >= 0`` with A of full row rank m, an optimum, if
one exists, is attained at a basic feasible solution: choose m linearly
independent columns (a basis), solve A_B x_B = b, keep it if x_B >= 0. The
minimum of c^T x over all such points is the optimal value (fundamental
theorem of linear programming). Only for tiny m, n.
"""
from __future__ import annotations

import itertools

import numpy as np


def enumerate_vertices(A: np.ndarray, b: np.ndarray, tol: float = 1e-12):
    m, n = A.shape
    for basis in itertools.combinations(range(n), m):
        AB = A[:, basis]
        if abs(np.linalg.det(AB)) < 1e-12:
            continue
        xB = np.linalg.solve(AB, b)
        if np.all(xB >= -tol):
            x = np.zeros(n)
            x[list(basis)] = np.maximum(xB, 0.0)
            yield basis, x


def lp_optimum(A: np.ndarray, b: np.ndarray, c: np.ndarray):
    """Return (optimal value, list of optimal vertices) or (None, []) if infeasible."""
    best, xs = None, []
    for _, x in enumerate_vertices(A, b):
        val = float(c @ x)
        if best is None or val < best - 1e-10:
            best, xs = val, [x]
        elif abs(val - best) <= 1e-10:
            xs.append(x)
    return best, xs
