"""Pins for the FP64 CPU oracle: each test checks it against something other
than itself -- closed forms, the paper's worked case, invariants the paper
states, brute force on tiny inputs, or planted optima -- so that a dropped
term, a wrong sign or a transposed operand fails at least one of them."""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import lpgen
import oracle
from tests import bruteforce

INF = np.inf


def make_lp(A, c, lc, uc, lv, uv):
    A = sp.csr_matrix(np.asarray(A, dtype=np.float64))
    A.sort_indices()
    m, n = A.shape
    return lpgen.LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                    A.data.astype(np.float64), np.asarray(c, float), np.asarray(lc, float),
                    np.asarray(uc, float), np.asarray(lv, float), np.asarray(uv, float))


# ------------------------------------------------------------------ products

def test_spmv_exact_on_integers():
    rng = np.random.default_rng(1)
    dense = rng.integers(-4, 5, size=(37, 53)).astype(float)
    dense[rng.random(dense.shape) < 0.7] = 0.0
    dense[5] = 0.0  # empty row
    lp = make_lp(dense, np.zeros(53), np.zeros(37), np.zeros(37), np.zeros(53), np.zeros(53))
    v = oracle.LPView.of(lp)
    x = rng.integers(-9, 10, size=53).astype(float)
    y = rng.integers(-9, 10, size=37).astype(float)
    assert np.array_equal(oracle.spmv(v, x), dense @ x)
    assert np.array_equal(oracle.spmv_t(v, y), dense.T @ y)


# ---------------------------------------------------------------- dual step

def test_dual_case_worked_example():
    # Section 2: lc = -inf, uc finite: y+ = 0 if yhat >= -sigma*uc, else yhat + sigma*uc.
    sigma, uc = 0.7, 2.5
    for yhat in (-5.0, -1.76, -1.75, -1.0, 0.0, 3.0):
        want = 0.0 if yhat >= -sigma * uc else yhat + sigma * uc
        assert oracle.dual_case(yhat, sigma, -INF, uc) == want


def _prox_bruteforce(yhat, sigma, lc, uc):
    """argmin_v sigma*p(v; -uc, -lc) + 0.5 (v - yhat)^2 over v in Y (bounded 1-D search)."""
    def p(v):  # p(v; -uc, -lc) = (-lc) v+ - (-uc) v-
        s = 0.0
        if v > 0:
            s += -lc * v
        if v < 0:
            s += uc * (-v)
        return s
    lo = -1e3 if np.isfinite(uc) else 0.0
    hi = 1e3 if np.isfinite(lc) else 0.0
    f = lambda v: sigma * p(v) + 0.5 * (v - yhat) ** 2
    if lo == hi:
        return 0.0, f
    r = so.minimize_scalar(f, bounds=(lo, hi), method="bounded",
                           options={"xatol": 1e-12, "maxiter": 10000})
    # the kink at 0 is a common minimizer; compare objective values
    cands = [r.x, 0.0] if lo <= 0.0 <= hi else [r.x]
    return min(cands, key=f), f


@pytest.mark.parametrize("kind", ["eq", "ge", "le", "range", "free"])
def test_dual_case_equals_prox_and_literal(kind):
    rng = np.random.default_rng(["eq", "ge", "le", "range", "free"].index(kind))
    for _ in range(200):
        sigma = float(rng.uniform(0.1, 3.0))
        a, b = sorted(rng.uniform(-3, 3, size=2))
        lc, uc = {"eq": (a, a), "ge": (a, INF), "le": (-INF, b), "range": (a, b),
                  "free": (-INF, INF)}[kind]
        yhat = float(rng.uniform(-8, 8))
        got = oracle.dual_case(yhat, sigma, lc, uc)
        # literal form of the paper: yhat - sigma * proj_[-uc,-lc](yhat / sigma)
        lit = yhat - sigma * min(max(yhat / sigma, -uc), -lc)
        assert abs(got - lit) <= 1e-12 * (1 + abs(yhat))
        v, f = _prox_bruteforce(yhat, sigma, lc, uc)
        assert f(got) <= f(v) + 1e-9
        # y+ lies in Y
        if not np.isfinite(lc):
            assert got <= 0.0
        if not np.isfinite(uc):
            assert got >= 0.0


# ----------------------------------------------------------- preconditioning

def _row_col_norms(lp, val, kind):
    A = sp.csr_matrix((np.abs(val), lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    if kind == "inf":
        return A.max(axis=1).toarray().ravel(), A.max(axis=0).toarray().ravel()
    return np.asarray(A.sum(axis=1)).ravel(), np.asarray(A.sum(axis=0)).ravel()


def test_ruiz_norms_go_to_one_and_factors_reproduce_matrix():
    lp = lpgen.planted_skewed(3000, 4000, seed=11, n_dense=30)
    # skew the magnitudes so that scaling has work to do
    rows = np.repeat(np.arange(lp.m), np.diff(lp.row_ptr))
    val0 = lp.val * np.exp(3 * np.sin(rows))[:] * np.exp(2 * np.cos(lp.col))
    lp.val = val0
    val, d1, d2 = oracle.precondition(lp, ruiz_iters=40, pc=False)
    r, c = _row_col_norms(lp, val, "inf")
    assert np.all(np.abs(r[r > 0] - 1) < 1e-6) and np.all(np.abs(c[c > 0] - 1) < 1e-6)
    np.testing.assert_allclose(val, d1[rows] * val0 * d2[lp.col], rtol=1e-12)
    # 10 rounds move every norm closer to 1 than the raw matrix
    val10, _, _ = oracle.precondition(lp, ruiz_iters=10, pc=False)
    r0, _ = _row_col_norms(lp, val0, "inf")
    r10, _ = _row_col_norms(lp, val10, "inf")
    nz = r0 > 0
    assert np.abs(np.log(r10[nz])).max() < 0.05 * np.abs(np.log(r0[nz])).max()


def test_one_round_closed_forms():
    # Ruiz round on [[1, 4], [2, 0]]: row inf-norms (4, 2), column inf-norms (2, 4)
    # -> a_ij / (sqrt(rho_i) sqrt(kappa_j)) = [[1/(2*sqrt2), 1], [1, 0]]
    lp = make_lp([[1.0, 4.0], [2.0, 0.0]], [0, 0], [0, 0], [0, 0], [0, 0], [0, 0])
    val, d1, d2 = oracle.precondition(lp, ruiz_iters=1, pc=False)
    np.testing.assert_allclose(val, [1 / (2 * math.sqrt(2)), 1.0, 1.0], rtol=1e-15)
    np.testing.assert_allclose(d1, [0.5, 1 / math.sqrt(2)], rtol=1e-15)
    np.testing.assert_allclose(d2, [1 / math.sqrt(2), 0.5], rtol=1e-15)
    # Pock-Chambolle (alpha = 1) on [[1, 3], [0, 4]]: row 1-norms (4, 4), column 1-norms (1, 7)
    lp = make_lp([[1.0, 3.0], [0.0, 4.0]], [0, 0], [0, 0], [0, 0], [0, 0], [0, 0])
    val, d1, d2 = oracle.precondition(lp, ruiz_iters=0, pc=True)
    np.testing.assert_allclose(val, [0.5, 3 / math.sqrt(28), 4 / math.sqrt(28)], rtol=1e-15)
    np.testing.assert_allclose(d1, [0.5, 0.5], rtol=1e-15)
    np.testing.assert_allclose(d2, [1.0, 1 / math.sqrt(7)], rtol=1e-15)


@pytest.mark.parametrize("ruiz", [0, 10])
def test_pock_chambolle_spectral_norm_at_most_one(ruiz):
    lp = lpgen.planted_uniform(400, 700, 6, seed=5)
    val, d1, d2 = oracle.precondition(lp, ruiz_iters=ruiz, pc=True)
    A = sp.csr_matrix((val, lp.col, lp.row_ptr), shape=(lp.m, lp.n))
    smax = sla.svds(A, k=1, return_singular_vectors=False, tol=1e-12)[0]
    assert smax <= 1.0 + 1e-10


def test_scale_vectors_maps_bounds():
    lp = make_lp([[1.0, 2.0], [3.0, 0.0]], [1.0, -2.0], [-INF, 1.0], [4.0, INF], [0.0, -INF], [INF, 5.0])
    d1 = np.array([0.5, 2.0]); d2 = np.array([4.0, 0.25])
    c, lc, uc, lv, uv = oracle.scale_vectors(lp, d1, d2)
    assert list(c) == [4.0, -0.5]
    assert lc[0] == -INF and lc[1] == 2.0 and uc[0] == 2.0 and uc[1] == INF
    assert lv[0] == 0.0 and lv[1] == -INF and uv[0] == INF and uv[1] == 20.0


# ------------------------------------------------------------- primal weight

def test_initial_primal_weight_closed_form():
    lp = make_lp(np.ones((3, 2)), [3.0, 4.0], [-INF, 1.0, -2.0], [2.0, INF, 5.0], [0, 0], [1, 1])
    w = oracle.initial_primal_weight(oracle.LPView.of(lp))
    assert w == pytest.approx(5.0 / math.sqrt(4 + 1 + 25), rel=1e-15)
    lp0 = make_lp(np.ones((1, 2)), [0.0, 0.0], [1.0], [2.0], [0, 0], [1, 1])
    assert oracle.initial_primal_weight(oracle.LPView.of(lp0)) == 1.0
    lpf = make_lp(np.ones((1, 2)), [1.0, 0.0], [-INF], [INF], [0, 0], [1, 1])
    assert oracle.initial_primal_weight(oracle.LPView.of(lpf)) == 1.0


def test_primal_weight_update_closed_form():
    assert oracle.primal_weight_update(1.0, 4.0, 1.0) == pytest.approx(2.0, rel=1e-15)
    assert oracle.primal_weight_update(2.0, 2.0, 9.0) == pytest.approx(3.0, rel=1e-15)
    assert oracle.primal_weight_update(1e-11, 4.0, 7.0) == 7.0
    assert oracle.primal_weight_update(1.0, 1e11, 7.0) == 7.0
    assert oracle.primal_weight_update(2.0, 6.0, 7.0, theta=1.0) == pytest.approx(3.0, rel=1e-15)
    assert oracle.primal_weight_update(2.0, 6.0, 7.0, theta=0.0) == pytest.approx(7.0, rel=1e-15)


# --------------------------------------------------------- KKT / termination

def test_kkt_at_planted_optimum_and_weak_duality():
    lp = lpgen.planted_uniform(300, 600, 8, seed=21)
    s = oracle.Solver(lp, scale=False)
    for mode in (0, 1):
        k = s.kkt(lp.x_star, lp.y_star, mode)
        assert k["primal_res_rel"] <= 1e-12 and k["dual_res_rel"] <= 1e-12
        assert k["primal_obj"] == pytest.approx(lp.p_star, rel=1e-12)
        assert k["dual_obj"] == pytest.approx(lp.p_star, rel=1e-12)
        assert k["rel_gap"] <= 1e-13
    # any y in Y gives a lower bound when every variable is boxed (natural r)
    rng = np.random.default_rng(0)
    for _ in range(5):
        y = lp.y_star + rng.standard_normal(lp.m)
        y = np.where(np.isfinite(lp.lc), y, np.minimum(y, 0))
        y = np.where(np.isfinite(lp.uc), y, np.maximum(y, 0))
        k = s.kkt(lp.x_star, y, 0)
        assert k["dual_obj"] <= lp.p_star + 1e-9 * abs(lp.p_star)
        assert k["dual_res_abs"] == 0.0


@pytest.mark.parametrize("lc,uc,ax,want", [
    (2.0, INF, 1.0, 0.5),        # q = |lc|
    (-INF, -4.0, -2.0, 0.5),     # q = |uc|
    (-3.0, 6.0, 9.0, 0.5),       # q = max(|lc|, |uc|)
    (0.0, 0.0, 0.5, 0.5),        # q = 1
    (0.0, 8.0, 10.0, 0.25),      # lc = 0, uc finite nonzero: q = |uc|
    (-2.0, 0.0, -3.0, 0.5),      # uc = 0, lc finite nonzero: q = |lc|
])
def test_relative_primal_residual_q(lc, uc, ax, want):
    lp = make_lp([[1.0]], [0.0], [lc], [uc], [-INF], [INF])
    s = oracle.Solver(lp, scale=False)
    k = s.kkt(np.array([ax]), np.array([0.0]), 0)
    assert k["primal_res_rel"] == pytest.approx(want, rel=1e-15)


def test_dual_objective_and_reduced_costs_by_hand():
    # A = I (2x2); x = (0.9, 0.1); y = (2, -1); c = (1, -3)
    # row 0: lc = 1, uc = inf (Y = R+); row 1: lc = -inf, uc = 4 (Y = R-)
    # boxes: x0 in [0, 1]; x1 in [-inf, 5]
    lp = make_lp(np.eye(2), [1.0, -3.0], [1.0, -INF], [INF, 4.0], [0.0, -INF], [1.0, 5.0])
    s = oracle.Solver(lp, scale=False)
    x = np.array([0.9, 0.1]); y = np.array([2.0, -1.0])
    g = np.array([1.0 - 2.0, -3.0 + 1.0])  # c - A^T y = (-1, -2)
    # natural: R0 = R (boxed) -> r0 = -1; R1 = R- -> r1 = -2
    k = s.kkt(x, y, 0)
    want = 1.0 * 2.0 - 4.0 * 1.0 + (1.0 * -1.0) + (5.0 * -2.0)  # lc y+ - uc y- + lv r+ - uv r-
    assert k["dual_obj"] == pytest.approx(want, rel=1e-15)
    assert k["dual_res_abs"] == 0.0
    # Appendix A: r0 = g0 (g<0 and uv - x = 0.1 <= 0.9); r1 = g1 (uv - x = 4.9 > 0.1 -> 0)
    k1 = s.kkt(x, y, 1)
    assert k1["dual_res_abs"] == pytest.approx(2.0, rel=1e-15)
    assert k1["dual_res_rel"] == pytest.approx(2.0 / 3.0, rel=1e-15)
    assert k1["dual_obj"] == pytest.approx(2.0 - 4.0 - 1.0, rel=1e-15)
    assert k["primal_obj"] == pytest.approx(0.9 - 0.3, rel=1e-15)


# ------------------------------------------------- normalized duality gap

def _point(lp, rng, view):
    x = rng.uniform(lp.lv, lp.uv) if np.all(np.isfinite(lp.uv)) else rng.uniform(-1, 1, lp.n)
    y = rng.standard_normal(lp.m)
    y = np.where(np.isfinite(view.lc), y, np.minimum(y, 0))
    y = np.where(np.isfinite(view.uc), y, np.maximum(y, 0))
    return x, y


def test_gap_closed_form_one_variable():
    lp = make_lp(np.zeros((0, 1)), [1.0], [], [], [0.0], [1.0])
    v = oracle.LPView.of(lp)
    e = np.zeros(0)
    zero = np.zeros(1)
    # unclamped: omega=1, r=0.1 -> x^ = x - r, f = r, mu = 1
    assert oracle.norm_gap(v, [0.5], e, e, zero, [0.6], e, 1.0) == pytest.approx(1.0, rel=1e-14)
    # clamped at lv: x = 0.05, r = 0.2 -> x^ = 0, f = 0.05, mu = 0.25
    assert oracle.norm_gap(v, [0.05], e, e, zero, [0.25], e, 1.0) == pytest.approx(0.25, rel=1e-14)
    # omega = 4: ball sqrt(4)|dx| <= r -> |dx| <= r/2 -> mu = 0.5
    assert oracle.norm_gap(v, [0.5], e, e, zero, [0.6], e, 4.0) == pytest.approx(0.5, rel=1e-14)
    # r = 0 -> 0
    assert oracle.norm_gap(v, [0.5], e, e, zero, [0.5], e, 1.0) == 0.0


def test_gap_one_row_closed_form():
    # n = 1 fixed variable (lv = uv = 0), one range row lc=-1, uc=2, A = [1]; x = 0 so Ax = 0.
    # y = 0.3 > 0 with slope a = lc - Ax = -1 (moving down), then stuck at 0 until slope b = 2 > 0
    # never pulls below 0 -> y^ = max(0.3 - s*omega*1, 0); D = (y^-y)^2/omega.
    lp = make_lp([[1.0]], [0.0], [-1.0], [2.0], [0.0], [0.0])
    v = oracle.LPView.of(lp)
    x = np.zeros(1); ax = np.zeros(1); aty = np.array([0.3])
    # radius 0.1 (omega=1): y^ = 0.2; f = h(0.2) - h(0.3) = 0.2*(-1) - 0.3*(-1) = 0.1 -> mu = 1
    mu = oracle.norm_gap(v, x, [0.3], ax, aty, x, [0.4], 1.0)
    assert mu == pytest.approx(1.0, rel=1e-14)
    # radius 0.5: y^ stops at 0 -> f = 0.3 -> mu = 0.6
    mu = oracle.norm_gap(v, x, [0.3], ax, aty, x, [0.8], 1.0)
    assert mu == pytest.approx(0.6, rel=1e-14)


def test_gap_zero_at_planted_optimum():
    lp = lpgen.planted_uniform(200, 400, 6, seed=2)
    s = oracle.Solver(lp)
    xs = lp.x_star / s.d2
    ys = lp.y_star / s.d1
    ax = oracle.spmv(s.scaled, xs)
    aty = oracle.spmv_t(s.scaled, ys)
    rng = np.random.default_rng(3)
    scale = np.abs(s.scaled.c).max()
    for _ in range(5):
        xr = xs + 0.1 * rng.standard_normal(lp.n)
        yr = ys + 0.1 * rng.standard_normal(lp.m)
        mu = s.gap(xs, ys, ax, aty, xr, yr, s.omega)
        assert abs(mu) <= 1e-10 * scale


def test_gap_nonincreasing_in_radius_and_matches_bisection():
    lp = lpgen.planted_uniform(150, 300, 5, seed=4)
    s = oracle.Solver(lp)
    rng = np.random.default_rng(9)
    x, y = _point(lp, rng, s.scaled)
    x = np.clip(x / s.d2, s.scaled.lv, s.scaled.uv)
    ax = oracle.spmv(s.scaled, x); aty = oracle.spmv_t(s.scaled, y)
    d = np.concatenate([rng.standard_normal(lp.n), rng.standard_normal(lp.m)])
    prev = np.inf
    for t in np.geomspace(1e-4, 1e3, 30):
        xr = x + t * d[:lp.n]; yr = y + t * d[lp.n:]
        mu = s.gap(x, y, ax, aty, xr, yr, s.omega)
        mub = s.gap(x, y, ax, aty, xr, yr, s.omega, bisect=True)
        assert mu == pytest.approx(mub, rel=1e-9, abs=1e-14)
        assert mu <= prev * (1 + 1e-12)
        prev = mu


@pytest.mark.parametrize("seed", range(12))
def test_gap_beats_sampling_on_tiny_problems(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = int(rng.integers(1, 3)), int(rng.integers(1, 3))
    lp = lpgen.tiny_random_lp(seed, m, n, kinds=("eq", "ge", "le", "range", "free"))
    v = oracle.LPView.of(lp)
    x, y = _point(lp, rng, v)
    ax = lp.csr() @ x
    aty = lp.csr().T @ y
    omega = float(rng.uniform(0.3, 3.0))
    xr = x + rng.standard_normal(n) * 0.5
    yr = y + rng.standard_normal(m) * 0.5
    r = math.sqrt(omega * np.sum((x - xr) ** 2) + np.sum((y - yr) ** 2) / omega)
    mu = oracle.norm_gap(v, x, y, ax, aty, xr, yr, omega)
    fmax = mu * r

    def f(xh, yh):  # L(x, yh) - L(xh, y), straight from the Lagrangian
        def p(yy):  # p(y; -uc, -lc)
            out = 0.0
            for i in range(m):
                if yy[i] > 0:
                    out += -lp.lc[i] * yy[i]
                elif yy[i] < 0:
                    out += lp.uc[i] * (-yy[i])
            return out
        L1 = lp.c @ x - yh @ ax - p(yh)
        L2 = lp.c @ xh - y @ (lp.csr() @ xh) - p(y)
        return L1 - L2

    def proj(xh, yh):
        xh = np.clip(xh, lp.lv, lp.uv)
        yh = np.where(np.isfinite(lp.lc), yh, np.minimum(yh, 0))
        yh = np.where(np.isfinite(lp.uc), yh, np.maximum(yh, 0))
        return xh, yh

    best = -np.inf
    for _ in range(4000):
        d = rng.standard_normal(n + m)
        w = np.concatenate([np.full(n, math.sqrt(omega)), np.full(m, 1 / math.sqrt(omega))])
        d = d / np.linalg.norm(d * w) * r * rng.uniform(0.0, 1.0) ** (1 / (n + m))
        xh, yh = proj(x + d[:n], y + d[n:])
        best = max(best, f(xh, yh))
    assert best <= fmax + 1e-9 * (1 + abs(fmax))
    # the maximizer the oracle found is feasible, inside the ball and attains fmax:
    # locate s* by bisection on the exposed path distance
    lo, hi = 0.0, 1.0
    while oracle.path_value(v, x, y, ax, aty, omega, hi, 0)[0] < r * r and hi < 1e12:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if oracle.path_value(v, x, y, ax, aty, omega, mid, 0)[0] < r * r:
            lo = mid
        else:
            hi = mid
    _, xh, yh = oracle.path_value(v, x, y, ax, aty, omega, lo, 1)
    assert f(xh, yh) == pytest.approx(fmax, rel=1e-7, abs=1e-10)
    assert best >= fmax - 0.2 * abs(fmax) - 1e-9  # sampling gets close: fmax is not inflated


# ----------------------------------------------------------- iteration pins

def _spectral_norm(s):
    A = sp.csr_matrix((s.scaled.val, s.scaled.col, s.scaled.row_ptr), shape=(s.m, s.n))
    return sla.svds(A, k=1, return_singular_vectors=False, tol=1e-12)[0]


def test_step_size_bound_eta_bar():
    lp = lpgen.planted_uniform(200, 400, 6, seed=8)
    s = oracle.Solver(lp)
    nrm = _spectral_norm(s)
    for _ in range(300):
        s.step()
        c = s.counters()
        assert c["last_eta_bar"] >= (1 - 1e-12) / nrm
        assert c["last_eta"] <= c["last_eta_bar"]


def test_fejer_monotone_fixed_step():
    lp = lpgen.planted_uniform(200, 400, 6, seed=12)
    prm = oracle.Params(fixed_step=True)
    s = oracle.Solver(lp, prm)
    eta = 0.9 / _spectral_norm(s)
    s.params.fixed_eta = eta
    s.st.eta_hat = eta
    w = s.omega
    tau, sigma = eta / w, eta * w
    A = sp.csr_matrix((s.scaled.val, s.scaled.col, s.scaled.row_ptr), shape=(s.m, s.n))
    xs = lp.x_star / s.d2
    ys = lp.y_star / s.d1

    def mdist():
        dx = s.x - xs; dy = s.y - ys
        return dx @ dx / tau + dy @ dy / sigma + 2 * dy @ (A @ dx)
    prev = mdist()
    for _ in range(400):
        s.step()
        cur = mdist()
        assert cur <= prev * (1 + 1e-10) + 1e-14
        prev = cur


def test_restart_schedule_condition_iii_only():
    lp = lpgen.planted_uniform(100, 200, 5, seed=1)
    s = oracle.Solver(lp, oracle.Params(adaptive_restarts=False))
    s.iterate(200)
    c = s.counters()
    # t >= k/2 fires at k = 1, 2, 4, ..., 128
    assert c["n_outer"] == 8 and c["restarts_iii"] == 8 and c["t"] == 200 - 128


def test_iterate_is_resumable_bitwise():
    lp = lpgen.planted_uniform(300, 500, 6, seed=6)
    a = oracle.Solver(lp); a.iterate(150); a.iterate(170)
    b = oracle.Solver(lp); b.iterate(320)
    for k in ("x", "y", "sx", "sy", "x0", "y0"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.counters() == b.counters()


@pytest.mark.parametrize("seed", range(10))
def test_solve_matches_vertex_enumeration(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 4)), int(rng.integers(1, 4))
    lp = lpgen.tiny_random_lp(1000 + seed, m, n, kinds=("eq", "ge", "le", "range"))
    best, _ = bruteforce.solve(lp.csr().toarray(), lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    s = oracle.Solver(lp, oracle.Params(eps_feas=1e-9, eps_gap=1e-9, max_iters=400_000))
    r = s.solve()
    assert r["status_name"] == "OPTIMAL"
    x, _ = s.solution()
    assert lp.c @ x == pytest.approx(best, rel=1e-6, abs=1e-6)


def test_planted_small_lp_solves_to_tolerance():
    lp = lpgen.small_lp()
    s = oracle.Solver(lp, oracle.Params(eps_feas=1e-8, eps_gap=1e-8, max_iters=100_000))
    r = s.solve()
    assert r["status_name"] == "OPTIMAL"
    assert r["primal_res_rel"] <= 1e-8 and r["dual_res_rel"] <= 1e-8 and r["rel_gap"] <= 1e-8
    x, y = s.solution()
    assert lp.c @ x == pytest.approx(lp.p_star, rel=1e-6)
    assert np.all(x >= lp.lv - 1e-12) and np.all(x <= lp.uv + 1e-12)


def test_feasibility_polishing_on_planted_lp():
    lp = lpgen.planted_uniform(600, 1200, 8, seed=31)
    s = oracle.Solver(lp, oracle.Params(eps_feas=1e-8, eps_gap=1e-2, polish=True, max_iters=50_000))
    r = s.solve()
    assert r["status_name"] == "OPTIMAL"
    assert r["polish_attempts"] >= 1 and r["polished"] == 1
    assert r["primal_res_rel"] <= 1e-8 and r["dual_res_rel"] <= 1e-8 and r["rel_gap"] <= 1e-2
    x, _ = s.solution()
    assert abs(lp.c @ x - lp.p_star) <= 2e-2 * abs(lp.p_star)


# ------------------------------------------------------- unrolled map and adjoint
#
# The map of K accepted steps with the recorded decisions held fixed is
# affine in (c, lc, uc) and polynomial in the matrix values once the
# projection and dual-case selections are fixed; its adjoint is pinned by
# central differences of the replay (independent of the adjoint code), by the
# one-step closed form and by exact affinity in c.

def _unroll_case():
    lp = lpgen.planted_uniform(60, 100, 5, seed=3)
    return lp, oracle.Unroll(lp, 120)


def test_unroll_records_both_restart_kinds_and_replays_bitwise():
    lp, U = _unroll_case()
    kinds = set(np.unique(U.restart).tolist())
    assert kinds == {0, 1, 2}
    assert U.result["iterations"] == 120
    x, _ = U.replay()
    assert np.array_equal(x, U.x)
    # the recorded run is the oracle's Algorithm 1 on the same scaled data
    assert np.all(U.eta[:120] > 0) and np.all(U.omega[:120] > 0)


def _direction(rng, base, scale_rel=True):
    base = np.asarray(base, dtype=np.float64)
    fin = np.isfinite(base)
    mag = np.where(fin, np.abs(np.where(fin, base, 0.0)), 0.0).clip(1e-3) if scale_rel else 1.0
    return np.where(fin, rng.standard_normal(base.size) * mag, 0.0)


@pytest.mark.parametrize("name,h", [("c", 1e-5), ("lc", 1e-5), ("uc", 1e-5), ("val", 1e-5)])
def test_unroll_adjoint_matches_central_differences(name, h):
    lp, U = _unroll_case()
    rng = np.random.default_rng(1)
    gx = rng.standard_normal(lp.n)
    g = U.backward(gx)
    _, sig = U.replay()
    base = np.asarray(getattr(lp, name), dtype=np.float64)
    for trial in range(3):
        d = _direction(rng, base)
        xp, sp = U.replay(**{name: base + h * d})
        xm, sm = U.replay(**{name: base - h * d})
        assert sp == sig and sm == sig  # same projection / dual-case selections
        fd = (gx @ xp - gx @ xm) / (2 * h)
        an = g[name] @ d
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (name, trial, fd, an)


def test_unroll_is_affine_in_c():
    lp, U = _unroll_case()
    rng = np.random.default_rng(2)
    gx = rng.standard_normal(lp.n)
    g = U.backward(gx)
    d = _direction(rng, lp.c)
    _, sig = U.replay()
    vals = []
    for h in (2e-6, 1e-5):
        xp, sp = U.replay(c=lp.c + h * d)
        xm, sm = U.replay(c=lp.c - h * d)
        assert sp == sig and sm == sig
        vals.append((gx @ xp - gx @ xm) / (2 * h))
    assert vals[0] == pytest.approx(vals[1], rel=1e-7)
    assert g["c"] @ d == pytest.approx(vals[1], rel=1e-7)


def test_unroll_one_step_closed_form():
    """K = 1 from (proj_X(0), 0): x_1 = proj(x_0 - tau c~), so
    dL/dc_j = -tau p_j D2_j^2 g_j and every other gradient is 0."""
    lp = lpgen.planted_uniform(40, 70, 5, seed=9)
    U = oracle.Unroll(lp, 1)
    rng = np.random.default_rng(3)
    gx = rng.standard_normal(lp.n)
    g = U.backward(gx)
    tau = U.eta[0] / U.omega[0]
    x0 = np.clip(0.0, U.view.lv, U.view.uv)
    v = x0 - tau * U.view.c
    p = (v > U.view.lv) & (v < U.view.uv)
    expect = -tau * p * U.d2 ** 2 * gx
    np.testing.assert_allclose(g["c"], expect, rtol=1e-15, atol=0)
    assert not g["lc"].any() and not g["uc"].any() and not g["val"].any()


# ------------------------------------------------- tangent-linear (forward mode)
#
# The tangent is pinned by central differences of the replay, by the one-step
# closed form, by linearity in the direction, and by the dot-product test
# against the reverse sweep, <J v, w> = <v, J^T w>: the two modes share no
# derivative code, so a dropped or mis-signed term in either breaks the
# equality.  The test keeps its meaning where the map is ill-conditioned
# (large K), unlike finite differences.

def _full_direction(rng, lp):
    return dict(dc=_direction(rng, lp.c), dlc=_direction(rng, lp.lc), duc=_direction(rng, lp.uc),
                dval=_direction(rng, lp.val))


def test_unroll_tangent_one_step_closed_form():
    lp = lpgen.planted_uniform(40, 70, 5, seed=9)
    U = oracle.Unroll(lp, 1)
    rng = np.random.default_rng(4)
    d = _full_direction(rng, lp)
    dx = U.tangent(**d)
    tau = U.eta[0] / U.omega[0]
    x0 = np.clip(0.0, U.view.lv, U.view.uv)
    v = x0 - tau * U.view.c
    p = (v > U.view.lv) & (v < U.view.uv)
    np.testing.assert_allclose(dx, U.d2 * (-tau * p * (U.d2 * d["dc"])), rtol=1e-15, atol=0)


@pytest.mark.parametrize("which", ["dc", "dlc", "duc", "dval", "all"])
def test_unroll_tangent_matches_central_differences(which):
    lp, U = _unroll_case()
    rng = np.random.default_rng(5)
    _, sig = U.replay()
    names = {"dc": "c", "dlc": "lc", "duc": "uc", "dval": "val"}
    for trial in range(3):
        full = _full_direction(rng, lp)
        d = full if which == "all" else {which: full[which]}
        dx = U.tangent(**d)
        h = 1e-6
        plus = {names[k]: np.asarray(getattr(lp, names[k]), float) + h * v for k, v in d.items()}
        minus = {names[k]: np.asarray(getattr(lp, names[k]), float) - h * v for k, v in d.items()}
        xp, sp = U.replay(**plus)
        xm, sm = U.replay(**minus)
        assert sp == sig and sm == sig
        fd = (xp - xm) / (2 * h)
        assert np.linalg.norm(fd - dx) <= 1e-6 * np.linalg.norm(dx), (which, trial)


def test_unroll_tangent_is_linear_in_the_direction():
    lp, U = _unroll_case()
    rng = np.random.default_rng(6)
    a, b = _full_direction(rng, lp), _full_direction(rng, lp)
    ta, tb = U.tangent(**a), U.tangent(**b)
    tab = U.tangent(**{k: 2.5 * a[k] - b[k] for k in a})
    np.testing.assert_allclose(tab, 2.5 * ta - tb, rtol=1e-12, atol=1e-12 * np.abs(ta).max())


@pytest.mark.parametrize("m,n,k,K", [(60, 100, 5, 120), (200, 400, 6, 300), (2000, 4000, 10, 500)])
def test_unroll_dot_product_tangent_vs_adjoint(m, n, k, K):
    lp = lpgen.planted_uniform(m, n, k, seed=17)
    U = oracle.Unroll(lp, K)
    rng = np.random.default_rng(7)
    d = _full_direction(rng, lp)
    w = rng.standard_normal(lp.n)
    jv = U.tangent(**d)
    g = U.backward(w)
    lhs = jv @ w
    rhs = d["dc"] @ g["c"] + d["dlc"] @ g["lc"] + d["duc"] @ g["uc"] + d["dval"] @ g["val"]
    vnorm = np.sqrt(sum(np.linalg.norm(v) ** 2 for v in d.values()))
    gnorm = np.sqrt(sum(np.linalg.norm(v) ** 2 for v in g.values()))
    scale = np.linalg.norm(jv) * np.linalg.norm(w) + vnorm * gnorm
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    assert abs(lhs) > 1e-6 * scale   # not a trivially small pairing
