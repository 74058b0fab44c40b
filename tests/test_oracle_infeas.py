"""Pins for the oracle's infeasibility detection (Section 3, "Infeasibility
detection"; Appendix D).

The tests are held against things other than the oracle itself: certificates
worked out by hand on tiny LPs (each derivation is in the test), Farkas-type
inequalities that any feasible LP obeys, planted rays whose objective is
known by construction, HiGHS (scipy's linprog) for the infeasibility
classification, and the iterate history of a separate oracle run for the
three candidate sequences.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import lpgen
import oracle

INF = np.inf


def make_lp(A, c, lc, uc, lv, uv):
    A = sp.csr_matrix(np.asarray(A, dtype=np.float64))
    A.sort_indices()
    m, n = A.shape
    return lpgen.LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                    A.data.astype(np.float64), np.asarray(c, float), np.asarray(lc, float),
                    np.asarray(uc, float), np.asarray(lv, float), np.asarray(uv, float))


def q_weights(lp):
    """Row weights of eq. "rescaled-termination-criteria"."""
    q = np.ones(lp.m)
    for i in range(lp.m):
        lb = np.isfinite(lp.lc[i]) and lp.lc[i] != 0.0
        ub = np.isfinite(lp.uc[i]) and lp.uc[i] != 0.0
        if lb and ub:
            q[i] = max(abs(lp.lc[i]), abs(lp.uc[i]))
        elif lb:
            q[i] = abs(lp.lc[i])
        elif ub:
            q[i] = abs(lp.uc[i])
    return q


def linprog_status(lp):
    """HiGHS: 0 optimal, 2 infeasible, 3 unbounded."""
    A = lp.csr().toarray()
    a_ub, b_ub, a_eq, b_eq = [], [], [], []
    for i in range(lp.m):
        if lp.lc[i] == lp.uc[i]:
            a_eq.append(A[i]); b_eq.append(lp.lc[i])
            continue
        if np.isfinite(lp.uc[i]):
            a_ub.append(A[i]); b_ub.append(lp.uc[i])
        if np.isfinite(lp.lc[i]):
            a_ub.append(-A[i]); b_ub.append(-lp.lc[i])
    bounds = [(l if np.isfinite(l) else None, u if np.isfinite(u) else None)
              for l, u in zip(lp.lv, lp.uv)]
    r = so.linprog(lp.c, A_ub=np.array(a_ub) if a_ub else None, b_ub=b_ub or None,
                   A_eq=np.array(a_eq) if a_eq else None, b_eq=b_eq or None, bounds=bounds,
                   method="highs")
    return r.status


# ------------------------------------------------ hand-worked certificates

def test_primal_certificate_boxed_variable():
    # x in [0, 1] and the row x >= 2.  y = 1 (Y = R+): A^T y = 1, R = R (boxed)
    # so r = -1; objective lc*y + lv*r+ - uv*r- = 2 + 0 - 1*1 = 1, residual 0.
    lp = make_lp([[1.0]], [0.0], [2.0], [INF], [0.0], [1.0])
    t = oracle.primal_infeas_test(lp, [1.0])
    assert t["ok"] and t["obj"] == 1.0 and t["res"] == 0.0
    assert t["r"][0] == -1.0
    # the opposite sign is projected to 0 (Y = R+): objective 0, no certificate
    t = oracle.primal_infeas_test(lp, [-1.0])
    assert not t["ok"] and t["y"][0] == 0.0 and t["obj"] == 0.0


def test_primal_certificate_inconsistent_equalities():
    # x1 + x2 = 1 and x1 + x2 = 3, x free.  y = (-1, 1): A^T y = 0, r = 0
    # (R = {0} for free variables); objective lc2*1 - uc1*1 = 3 - 1 = 2.
    lp = make_lp([[1.0, 1.0], [1.0, 1.0]], [0.0, 0.0], [1.0, 3.0], [1.0, 3.0], [-INF, -INF],
                 [INF, INF])
    t = oracle.primal_infeas_test(lp, [-1.0, 1.0])
    assert t["ok"] and t["obj"] == 2.0 and t["res"] == 0.0
    # scaling the ray scales the objective; the ratio test is unchanged
    t = oracle.primal_infeas_test(lp, [-3.0, 3.0])
    assert t["ok"] and t["obj"] == 6.0
    # a free variable with c = 4 and a residual of 1e-3 in its column: the
    # residual is weighted by 1/|c_j| (eq. "rescaled-termination-criteria")
    lp = make_lp([[1.0, 1.0], [1.0, 1.001]], [0.0, 4.0], [1.0, 3.0], [1.0, 3.0],
                 [-INF, -INF], [INF, INF])
    t = oracle.primal_infeas_test(lp, [-1.0, 1.0], eps=1e-3)
    assert t["res"] == pytest.approx(1e-3 / 4, rel=1e-9)
    assert t["ok"]                      # 2.5e-4 <= 1e-3 * 2
    assert not oracle.primal_infeas_test(lp, [-1.0, 1.0], eps=1e-4)["ok"]


def test_primal_certificate_one_sided_sets():
    # x1 - x2 <= -1 with x1 >= 0 (R+) and x2 <= 0 (R-): x1 - x2 >= 0 always.
    # y = -1 (Y = R-): A^T y = (-1, 1), r = proj_R((1, -1)) = (1, -1);
    # objective -uc*y- + lv1*r1+ - uv2*r2- = (-1)(-1) + 0 - 0 = 1.
    lp = make_lp([[1.0, -1.0]], [1.0, 1.0], [-INF], [-1.0], [0.0, -INF], [INF, 0.0])
    t = oracle.primal_infeas_test(lp, [-1.0])
    assert t["ok"] and t["obj"] == 1.0 and t["res"] == 0.0
    assert list(t["r"]) == [1.0, -1.0]
    # with x1 <= 0 instead (R-), r1 = proj_{R-}(1) = 0 leaves a residual of 1
    # in column 1 (weight |c_1| = 1): ratio 1, no certificate
    lp = make_lp([[1.0, -1.0]], [1.0, 1.0], [-INF], [-1.0], [-INF, -INF], [0.0, 0.0])
    t = oracle.primal_infeas_test(lp, [-1.0])
    assert not t["ok"] and t["res"] == 1.0 and t["r"][0] == 0.0
    # a free row takes y = 0 (Y = {0}) whatever the candidate holds
    lp = make_lp([[1.0]], [0.0], [-INF], [INF], [0.0], [1.0])
    assert oracle.primal_infeas_test(lp, [5.0])["y"][0] == 0.0


def test_dual_certificate_cases():
    # min -x, x >= 0, no rows: the ray x = 1 has c^T x = -1 and no residual
    lp = make_lp(np.zeros((0, 1)), [-1.0], [], [], [0.0], [INF])
    t = oracle.dual_infeas_test(lp, [1.0])
    assert t["ok"] and t["obj"] == -1.0 and t["res"] == 0.0
    # a negative candidate is projected onto Xbar = R+ -> 0: no certificate
    t = oracle.dual_infeas_test(lp, [-1.0])
    assert not t["ok"] and t["x"][0] == 0.0
    # min -x1 s.t. x1 - x2 <= 5, x >= 0, x3 in [0, 1]: the ray (1, 1, 0.5)
    # projects to (1, 1, 0) (boxed -> {0}); A x = 0 so the residual is 0
    lp = make_lp([[1.0, -1.0, 1.0]], [-1.0, 0.0, 0.0], [-INF], [5.0], [0.0, 0.0, 0.0],
                 [INF, INF, 1.0])
    t = oracle.dual_infeas_test(lp, [1.0, 1.0, 0.5])
    assert t["ok"] and t["obj"] == -1.0 and t["res"] == 0.0
    assert list(t["x"]) == [1.0, 1.0, 0.0]
    # the ray (2, 1, 0): A x = 1 against a <= row (Sbar = R+, s = proj(-1) = 0),
    # residual 1 weighted by 1/q = 1/5; objective -2: ratio 0.1
    t = oracle.dual_infeas_test(lp, [2.0, 1.0, 0.0], eps=0.1)
    assert t["res"] == pytest.approx(0.2, rel=1e-15) and t["obj"] == -2.0 and t["ok"]
    assert not oracle.dual_infeas_test(lp, [2.0, 1.0, 0.0], eps=0.099)["ok"]
    # the same move against a >= row: s = proj_{R-}(-1) = -1 absorbs it
    lp = make_lp([[1.0, -1.0, 1.0]], [-1.0, 0.0, 0.0], [5.0], [INF], [0.0, 0.0, 0.0],
                 [INF, INF, 1.0])
    t = oracle.dual_infeas_test(lp, [2.0, 1.0, 0.0])
    assert t["ok"] and t["res"] == 0.0
    # an equality row (Sbar = {0}) keeps the whole of A x as residual, a free
    # row none of it
    lp = make_lp([[1.0, -1.0], [1.0, 1.0]], [-1.0, 0.0], [2.0, -INF], [2.0, INF],
                 [0.0, 0.0], [INF, INF])
    t = oracle.dual_infeas_test(lp, [1.0, 1.0])
    assert t["res"] == 0.0 and t["ok"]
    t = oracle.dual_infeas_test(lp, [1.0, 0.5], eps=1.0)
    assert t["res"] == pytest.approx(0.5 / 2.0, rel=1e-15)


def test_non_finite_candidates_never_certify():
    lp = make_lp([[1.0]], [-1.0], [2.0], [INF], [0.0], [INF])
    assert not oracle.primal_infeas_test(lp, [np.nan])["ok"]
    assert not oracle.dual_infeas_test(lp, [np.nan])["ok"]
    # an infinite ray would pass the ratio test as inf <= eps * inf
    assert not oracle.primal_infeas_test(lp, [INF])["ok"]
    assert not oracle.dual_infeas_test(lp, [INF])["ok"]


# ------------------------------------------------------- Farkas invariants

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_primal_test_obeys_farkas_bound_on_feasible_lps(seed):
    """For a feasible x^ and any (y, r) in Y x R:
    lc^T y+ - uc^T y- + lv^T r+ - uv^T r- <= (A^T y + r)^T x^
                                           <= sum_j res_j w_j |x^_j|.
    The dual-infeasible family is primal feasible (x_feas) with every bound kind."""
    lp = lpgen.infeasible_lp("dual", seed, 80, 120, 3)
    xf = lp.x_feas
    w = np.where(lp.c != 0.0, np.abs(lp.c), 1.0)
    rng = np.random.default_rng(seed)
    for _ in range(50):
        y = rng.standard_normal(lp.m) * rng.uniform(0.1, 10.0)
        t = oracle.primal_infeas_test(lp, y)
        per = np.abs(t["aty"] + t["r"]) / w
        assert np.max(per) == t["res"]
        bound = np.sum(per * w * np.abs(xf))
        assert t["obj"] <= bound + 1e-10 * (1.0 + np.abs(t["y"]).sum())
        assert not t["ok"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dual_test_obeys_farkas_bound_on_dual_feasible_lps(seed):
    """For a dual-feasible (y^, r^) and any x in Xbar, s in Sbar:
    c^T x = y^T (A x + s) - y^T s + r^T x >= -sum_i |y^_i| q_i res_i,
    since y^_i s_i <= 0 and r^_j x_j >= 0 on those cones.  The primal-infeasible
    family has c = A^T y_feas + r_feas."""
    lp = lpgen.infeasible_lp("primal", seed, 80, 120, 3)
    q = q_weights(lp)
    rng = np.random.default_rng(seed + 10)
    for _ in range(50):
        x = rng.standard_normal(lp.n) * rng.uniform(0.1, 10.0)
        t = oracle.dual_infeas_test(lp, x)
        lo = -np.sum(np.abs(lp.y_feas) * q * t["res"])
        assert t["obj"] >= lo - 1e-10 * (1.0 + np.abs(t["x"]).sum())
        assert not t["ok"]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_planted_rays_are_certificates(seed):
    for kind in ("primal", "primal_boxed"):
        lp = lpgen.infeasible_lp(kind, seed, 80, 120, 3)
        t = oracle.primal_infeas_test(lp, lp.ray_y)
        assert np.array_equal(t["y"], lp.ray_y)          # already in Y
        assert t["obj"] == pytest.approx(1.0, rel=1e-12)   # the planted margin
        assert t["res"] <= 1e-14 and t["ok"]
    lp = lpgen.infeasible_lp("dual", seed, 80, 120, 3)
    t = oracle.dual_infeas_test(lp, lp.ray_x)
    assert np.array_equal(t["x"], lp.ray_x)
    assert t["obj"] == pytest.approx(-1.0, rel=1e-12)
    assert t["res"] == 0.0 and t["ok"]
    assert not oracle.dual_infeas_test(lp, -lp.ray_x)["ok"]


# ------------------------------------------------------ detection in solves

@pytest.mark.parametrize("kind", ["primal", "dual"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solve_detects_planted_infeasibility(kind, seed):
    lp = lpgen.infeasible_lp(kind, seed, 60, 90, 3)
    assert linprog_status(lp) == (2 if kind == "primal" else 3)
    s = oracle.Solver(lp, oracle.Params(max_iters=200_000))
    r = s.solve()
    assert r["status_name"] == ("PRIMAL_INFEASIBLE" if kind == "primal" else "DUAL_INFEASIBLE")
    assert r["iterations"] % 64 == 0 and r["cert_source"] in (1, 2, 3)
    x, y = s.solution()
    if kind == "primal":
        t = oracle.primal_infeas_test(lp, y)
        assert t["ok"] and np.array_equal(t["y"], y)
        assert t["res"] <= 1e-9 * t["obj"]
    else:
        t = oracle.dual_infeas_test(lp, x)
        assert t["ok"] and np.array_equal(t["x"], x)
    assert t["obj"] == r["cert_obj"] and t["res"] == r["cert_res"]
    # without detection the same run goes to the iteration limit
    r2 = oracle.Solver(lp, oracle.Params(max_iters=r["iterations"] + 64,
                                          detect_infeasibility=False)).solve()
    assert r2["status_name"] == "ITERATION_LIMIT"


def _history(lp, k):
    """Iterates x^{k-1}, x^k, y^{k-1}, y^k and the average at step k from a
    run with restart checks and no termination test."""
    s = oracle.Solver(lp, oracle.Params())
    s.iterate(k - 1)
    xa, ya = s.x.copy(), s.y.copy()
    s.iterate(1)
    return s, xa, ya


@pytest.mark.parametrize("kind,seed,src", [("dual", 0, 2), ("dual", 1, 3), ("primal", 1, 3)])
def test_certificate_is_the_named_candidate(kind, seed, src):
    """The returned certificate is the candidate it names, rebuilt from an
    independent run: difference x^k - x^{k-1}, iterate x^k, or average."""
    lp = lpgen.infeasible_lp(kind, seed, 60, 90, 3)
    s = oracle.Solver(lp, oracle.Params(max_iters=200_000))
    r = s.solve()
    assert r["cert_source"] == src
    k = r["iterations"]
    h, xa, ya = _history(lp, k)
    if src == 1:
        cx, cy = h.x - xa, h.y - ya
    elif src == 2:
        cx, cy = h.x, h.y
    else:
        cx, cy = h.sx / h.st.seta, h.sy / h.st.seta
    x, y = s.solution()
    if kind == "primal":
        assert np.array_equal(y, oracle.primal_infeas_test(lp, s.d1 * cy)["y"])
    else:
        assert np.array_equal(x, oracle.dual_infeas_test(lp, s.d2 * cx)["x"])


def test_difference_candidate_detects():
    """An instance on which the difference of consecutive iterates certifies first."""
    for seed in range(12):
        lp = lpgen.infeasible_lp("dual", seed, 30, 45, 3)
        s = oracle.Solver(lp, oracle.Params(max_iters=300_000))
        r = s.solve()
        if r["cert_source"] == 1:
            break
    else:
        pytest.fail("no instance certified by the difference candidate")
    k = r["iterations"]
    h, xa, ya = _history(lp, k)
    x, _ = s.solution()
    assert np.array_equal(x, oracle.dual_infeas_test(lp, s.d2 * (h.x - xa))["x"])


def test_feasible_bounded_lps_are_not_declared_infeasible():
    for lp in (lpgen.planted_uniform(200, 300, 6, seed=5), lpgen.tiny_random_lp(9, 5, 8)):
        r = oracle.Solver(lp, oracle.Params(max_iters=100_000)).solve()
        assert r["status_name"] == "OPTIMAL" and r["cert_source"] == 0
