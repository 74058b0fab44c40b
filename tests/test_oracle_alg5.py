"""Pins for the oracle's Algorithm 5 mode (Appendix C): constant step and
primal weight, and every restart_period steps a restart to the plain average
of x with y = 0.

Held against: hand-derived iterates of a one-variable problem, the same
algorithm assembled from bare PDHG steps and a numpy mean, and both claims
of Theorem 1 on products of simplices, whose distance to the feasible set
is computed exactly (Euclidean projection onto a simplex) and whose Hoffman
constant is at least 1 (shown in `simplices_lp`).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle

INF = np.inf


def alg5_params(eta, ell, omega=1.0, **kw):
    return oracle.Params(fixed_step=True, fixed_eta=eta, restart_period=ell, fixed_omega=omega,
                         ruiz_iters=0, pc=False, detect_infeasibility=False, **kw)


def start_at(s, lp, x0):
    """Start point (x0, 0) of an unscaled solver."""
    s.x[:] = x0
    s.x0[:] = x0
    s.ax[:] = lp.csr() @ x0
    s.y[:] = 0.0
    s.aty[:] = 0.0


def simplices_lp(blocks, k, seed):
    """{x >= 0 : sum of each block of k variables = b_i}, c = 0.

    Hoffman constant >= 1 for x >= 0: with s = sum of a block, the point
    (b/s) x (or b/k * 1 when s = 0) is feasible and within |s - b| of x,
    because ||x||_2 <= ||x||_1 = s; blocks are independent, so
    dist(X_F, x) <= ||A x - b||_2.  ||A||_2 = sqrt(k).
    """
    rng = np.random.default_rng(seed)
    n = blocks * k
    rows = np.repeat(np.arange(blocks), k)
    A = sp.csr_matrix((np.ones(n), (rows, np.arange(n))), shape=(blocks, n))
    A.sort_indices()
    b = rng.uniform(0.5, 2.0, blocks)
    lp = lpgen.LP(blocks, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                  A.data.astype(np.float64), np.zeros(n), b.copy(), b.copy(), np.zeros(n),
                  np.full(n, INF))
    return lp, b


def simplex_projection(v, b):
    """Euclidean projection onto {z >= 0, sum z = b} (sort and threshold)."""
    u = np.sort(v)[::-1]
    css = np.cumsum(u) - b
    idx = np.arange(1, v.size + 1)
    rho = np.nonzero(u - css / idx > 0)[0][-1]
    return np.maximum(v - css[rho] / (rho + 1), 0.0)


def dist_to_simplices(x, b, k):
    X = x.reshape(-1, k)
    return math.sqrt(sum(float(np.sum((X[i] - simplex_projection(X[i], b[i])) ** 2))
                         for i in range(X.shape[0])))


def theorem1_constants(k, alpha):
    """eta = alpha / ||A||_2, q = 4 (1 + alpha) / (1 - alpha), and a period
    ell >= t* = ceil(2 (q + 2) / (eta H)) using H >= 1."""
    eta = alpha / math.sqrt(k)
    q = 4.0 * (1.0 + alpha) / (1.0 - alpha)
    return eta, q, math.ceil(2.0 * (q + 2.0) / eta)


def test_simplex_projection_is_exact():
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.standard_normal(7) * 3
        z = simplex_projection(v, 1.5)
        assert z.min() >= 0 and z.sum() == pytest.approx(1.5, rel=1e-14)
        # optimality: z = max(v - theta, 0) for one theta, and no random
        # feasible point is closer
        for _ in range(200):
            w = rng.random(7)
            w *= 1.5 / w.sum()
            assert np.linalg.norm(v - z) <= np.linalg.norm(v - w) + 1e-12


def test_one_variable_closed_forms():
    # min 0 s.t. x = b, x >= 0.  From (x0, 0): the first step leaves x (y = 0),
    # y1 = sigma (b - x0); the second gives x2 = x0 + tau sigma (b - x0).
    b, x0, eta = 2.0, 0.5, 0.25
    lp = lpgen.LP(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([1.0]),
                  np.zeros(1), np.array([b]), np.array([b]), np.zeros(1), np.array([INF]))
    # period 1: the average of one iterate equal to x0, y reset: no progress
    s = oracle.Solver(lp, alg5_params(eta, 1), scale=False)
    start_at(s, lp, np.array([x0]))
    s.iterate(5)
    assert s.x[0] == x0 and s.y[0] == 0.0 and s.st.restarts_iii == 5
    # period 2: x^{1,0} = (x1 + x2) / 2 = x0 + eta^2 (b - x0) / 2, any omega
    for omega in (1.0, 2.5):
        s = oracle.Solver(lp, alg5_params(eta, 2, omega), scale=False)
        start_at(s, lp, np.array([x0]))
        s.iterate(2)
        assert s.x[0] == pytest.approx(x0 + eta * eta * (b - x0) / 2, rel=1e-15)
        assert s.y[0] == 0.0 and s.st.n_outer == 1 and s.st.t == 0
        s.iterate(1)   # one more step from (x^{1,0}, 0): x unchanged, y = sigma (b - x)
        x10 = x0 + eta * eta * (b - x0) / 2
        assert s.x[0] == pytest.approx(x10, rel=1e-15)
        assert s.y[0] == pytest.approx(eta * omega * (b - x10), rel=1e-14)


@pytest.mark.parametrize("omega", [1.0, 2.5])
def test_restart_points_equal_bare_steps_and_means(omega):
    lp = lpgen.infeasible_lp("dual", 3, 120, 180, 3)   # feasible at x_feas
    lp.c = np.zeros(lp.n)
    ell, eta = 37, 0.3
    s = oracle.Solver(lp, alg5_params(eta, ell, omega), scale=False)
    bare = oracle.Solver(lp, alg5_params(eta, ell, omega), scale=False)
    bare.st.omega = omega
    A = lp.csr()
    for n in range(1, 4):
        xs = []
        for _ in range(ell):
            bare.step()
            xs.append(bare.x.copy())
        mean = np.mean(xs, axis=0)
        s.iterate(ell)
        assert np.allclose(s.x, mean, rtol=1e-13, atol=1e-15)
        assert not s.y.any() and not s.aty.any() and np.array_equal(s.x0, s.x)
        assert s.st.restarts_iii == n and s.st.n_outer == n and s.st.t == 0
        assert s.st.omega == omega
        bare.x[:] = s.x
        bare.ax[:] = A @ s.x
        bare.y[:] = 0.0
        bare.aty[:] = 0.0


@pytest.mark.parametrize("blocks,k,alpha,seed", [(40, 4, 0.5, 1), (25, 9, 0.5, 2),
                                                 (60, 3, 0.8, 3)])
def test_theorem1_contraction_on_simplices(blocks, k, alpha, seed):
    lp, b = simplices_lp(blocks, k, seed)
    eta, q, ell = theorem1_constants(k, alpha)
    s = oracle.Solver(lp, alg5_params(eta, ell), scale=False)
    x0 = np.random.default_rng(seed + 100).uniform(0.0, 3.0, lp.n)
    start_at(s, lp, x0)
    d0 = dist_to_simplices(x0, b, k)
    assert d0 > 0.5
    for n in range(1, 7):
        s.iterate(ell)
        d = dist_to_simplices(s.x, b, k)
        assert d <= 2.0 ** -n * d0 + 1e-13                       # eq. distance-contraction
        assert np.linalg.norm(s.x - x0) <= 2 * (q + 2) * d0       # eq. dist-bound-to-feas
        assert s.x.min() >= 0.0


def test_termination_in_the_mode():
    lp, b = simplices_lp(30, 4, 7)
    eta, q, ell = theorem1_constants(4, 0.5)
    s = oracle.Solver(lp, alg5_params(eta, ell, eps_feas=1e-10, max_iters=20_000), scale=False)
    r = s.solve()
    assert r["status_name"] == "OPTIMAL" and r["iterations"] % 64 == 0
    x, _ = s.solution()
    # dist <= ||A x - b||_2 (Hoffman constant >= 1) <= sqrt(m) * 1e-10 * max |b|
    assert dist_to_simplices(x, b, 4) <= np.sqrt(lp.m) * 1e-10 * np.abs(b).max()
