"""Brute-force LP solution by vertex enumeration (independent of the oracle).

For an LP  min c^T x  s.t.  lc <= A x <= uc,  lv <= x <= uv  with a finite
variable box, the optimum is attained at a vertex: a point where n linearly
independent constraints (rows at one of their finite bounds, variables at
one of their bounds) are tight.  Enumerate every such choice, solve the
n x n system, keep the feasible points and return the best objective.
Only for tiny problems (m, n <= 5).
"""
import itertools

import numpy as np


def solve(A_dense, c, lc, uc, lv, uv, tol=1e-9):
    A = np.asarray(A_dense, dtype=np.float64)
    m, n = A.shape
    hyper = []  # (row vector, rhs)
    for i in range(m):
        for b in (lc[i], uc[i]):
            if np.isfinite(b):
                hyper.append((A[i], b))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        for b in (lv[j], uv[j]):
            if np.isfinite(b):
                hyper.append((e, b))
    best, best_x = np.inf, None
    for comb in itertools.combinations(range(len(hyper)), n):
        M = np.array([hyper[k][0] for k in comb])
        rhs = np.array([hyper[k][1] for k in comb])
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, rhs)
        ax = A @ x
        scale = 1.0 + np.abs(x).max()
        if np.any(x < lv - tol * scale) or np.any(x > uv + tol * scale):
            continue
        if np.any(ax < lc - tol * scale) or np.any(ax > uc + tol * scale):
            continue
        val = float(c @ x)
        if val < best:
            best, best_x = val, x
    return best, best_x
