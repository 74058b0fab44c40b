"""GPU parity of infeasibility detection (Section 3, "Infeasibility
detection"; Appendix D) against the FP64 oracle, through the C ABI.

Trajectories of the two sides separate slowly (different summation orders,
amplified over tens of thousands of iterations on diverging iterates), so a
detection late in a run is compared in three ways:

* early checks: with a loose threshold the tests fire at the first checks,
  where both trajectories still agree to 1e-8; status, check, candidate and
  the certificate must then match the oracle's;
* transplanted state: the oracle's state one check before its own detection
  is loaded into the GPU solver, which must detect at the same check with
  the same candidate and the same certificate;
* whole runs: the status must be the planted one and the returned
  certificate must pass the oracle's own Appendix D test, with the objective
  and residual the GPU reported.
"""
import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import rel, say

pytestmark = pytest.mark.gpu

STATUS = {"primal": "PRIMAL_INFEASIBLE", "dual": "DUAL_INFEASIBLE"}


def _solve_both(lp, max_iters, **kw):
    r = pd.Problem(lp).solve(pd.pdlp_params_default(max_iters=max_iters, **kw))
    okw = dict(kw)
    if "eps_infeasible" in okw:
        okw["eps_infeas"] = okw.pop("eps_infeasible")
    if "detect_infeasibility" in okw:
        okw["detect_infeasibility"] = bool(okw["detect_infeasibility"])
    s = oracle.Solver(lp, oracle.Params(max_iters=max_iters, **okw))
    ro = s.solve()
    return r, ro, s


def _check_certificate(lp, r, eps=1e-9):
    """The returned certificate passes the oracle's Appendix D test with the
    values the GPU reported."""
    if r["status_name"] == "PRIMAL_INFEASIBLE":
        t = oracle.primal_infeas_test(lp, r["y"], eps)
        assert np.array_equal(t["y"], r["y"])            # already projected onto Y
        assert rel(r["r"], t["r"]) <= 1e-12
    else:
        t = oracle.dual_infeas_test(lp, r["x"], eps)
        assert np.array_equal(t["x"], r["x"])            # already projected onto Xbar
    assert t["ok"]
    assert r["certificate_objective"] == pytest.approx(t["obj"], rel=1e-10)
    assert abs(r["certificate_residual"] - t["res"]) <= 1e-10 * max(abs(t["obj"]), t["res"])
    return t


def _transplanted(lp, k, params):
    """GPU solve resumed from the oracle's state after k steps."""
    o = oracle.Solver(lp)
    o.iterate(k)
    blob = {key: getattr(o, key).copy() for key in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")}
    blob.update(o.counters())
    st = pd.Problem(lp).state(params)
    st.set(blob)
    return st.solve(params.max_iters, want_solution=True)


def _close_certificate(lp, r, xo, yo, params):
    """The certificate is the oracle's (xo, yo).  Candidates 2, 3: to the 1e-8
    the iterates agree at the first checks.  A difference of iterates
    (candidate 1) is far shorter than the iterates and carries both their
    errors (a restart at the same check also hides the iterate from a
    resumed run), so the GPU's difference is checked from the oracle's state
    one step before: one GPU step from the same state agrees to 1e-12.  The
    certificate of the run itself must then agree with that one to 1e-4:
    a wrong previous iterate would differ by O(1)."""
    if r["certificate"] != 1:
        assert rel(r["x"], xo) <= 1e-8 and rel(r["y"], yo) <= 1e-8
        return
    part = "y" if r["status_name"] == "PRIMAL_INFEASIBLE" else "x"
    ref = yo if part == "y" else xo
    r1 = _transplanted(lp, r["iterations"] - 1, params)
    assert r1["status_name"] == r["status_name"] and r1["certificate"] == 1
    assert r1["iterations"] == r["iterations"]
    assert rel(r1[part], ref) <= 1e-8
    assert rel(r[part], ref) <= 1e-4


EARLY = [("primal", 0, 900, 1350), ("dual", 0, 900, 1350), ("primal", 2, 433, 650),
         ("dual", 6, 433, 650)]


@pytest.mark.parametrize("eps", [1e30, 1e2, 1e-1])
@pytest.mark.parametrize("case", EARLY, ids=lambda c: f"{c[0]}{c[1]}_{c[2]}x{c[3]}")
def test_early_checks_match_oracle(case, eps):
    kind, i, m, n = case
    say(f"early infeasibility check {kind} {i} {m}x{n} eps={eps}")
    lp = lpgen.infeasible_lp(kind, i, m, n)
    r, ro, s = _solve_both(lp, 640, eps_infeasible=eps)
    prm = pd.pdlp_params_default(max_iters=640, eps_infeasible=eps)
    assert r["status_name"] == ro["status_name"]
    assert r["iterations"] == ro["iterations"]
    for key in ("attempts", "restarts_i", "restarts_ii", "restarts_iii", "kkt_passes"):
        assert r[key] == ro[key], key
    assert r["certificate"] == ro["cert_source"]
    if ro["cert_source"] == 0:
        return
    xo, yo = s.solution()
    _close_certificate(lp, r, xo, yo, prm)
    _check_certificate(lp, r, eps)


def test_early_checks_cover_every_candidate():
    """The loose thresholds above reach each of the three candidates."""
    seen = set()
    for kind, i, m, n in EARLY:
        lp = lpgen.infeasible_lp(kind, i, m, n)
        for eps in (1e30, 1e2, 1e-1):
            ro = oracle.Solver(lp, oracle.Params(max_iters=640, eps_infeas=eps)).solve()
            seen.add(ro["cert_source"])
    assert {1, 2, 3} <= seen


TRANSPLANT = [("primal", 1, 900, 1350), ("dual", 0, 900, 1350), ("primal", 2, 433, 650),
              ("dual", 6, 433, 650)]


@pytest.mark.parametrize("case", TRANSPLANT, ids=lambda c: f"{c[0]}{c[1]}_{c[2]}x{c[3]}")
def test_detection_from_transplanted_state(case):
    kind, i, m, n = case
    say(f"transplanted detection {kind} {i} {m}x{n}")
    lp = lpgen.infeasible_lp(kind, i, m, n)
    ref = oracle.Solver(lp, oracle.Params(max_iters=300_000))
    rr = ref.solve()
    assert rr["status_name"] == STATUS[kind]
    K = rr["iterations"]
    o = oracle.Solver(lp)
    o.iterate(K - 64)
    blob = {key: getattr(o, key).copy() for key in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")}
    blob.update(o.counters())
    prob = pd.Problem(lp)
    st = prob.state(pd.pdlp_params_default(max_iters=300_000))
    st.set(blob)
    r = st.solve(10_000, want_solution=True)
    assert r["status_name"] == STATUS[kind]
    assert r["iterations"] == K and r["certificate"] == rr["cert_source"]
    xo, yo = ref.solution()
    if kind == "primal":
        assert rel(r["y"], yo) <= 1e-9
    else:
        assert rel(r["x"], xo) <= 1e-9
    assert r["certificate_objective"] == pytest.approx(rr["cert_obj"], rel=1e-9)
    _check_certificate(lp, r)


@pytest.mark.parametrize("kind", ["primal", "dual"])
@pytest.mark.parametrize("i", [0, 1, 2])
def test_whole_runs_return_valid_certificates(kind, i):
    say(f"whole run {kind} {i}")
    lp = lpgen.infeasible_lp(kind, i, 900, 1350)
    r = pd.Problem(lp).solve(pd.pdlp_params_default(max_iters=300_000))
    assert r["status_name"] == STATUS[kind]
    assert r["iterations"] % 64 == 0 and r["certificate"] in (1, 2, 3)
    _check_certificate(lp, r)


def test_no_rows_unbounded_and_detection_off():
    say("infeasibility edge cases")
    # no rows: min c^T x with some c_j < 0 on a variable unbounded above
    rng = np.random.default_rng(3)
    n = 300
    import scipy.sparse as sp
    A = sp.csr_matrix((0, n))
    c = rng.standard_normal(n)
    lv = np.where(rng.random(n) < 0.5, 0.0, -1.0)
    uv = np.where(c < 0, np.inf, 1.0)
    lp = lpgen.LP(0, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                  A.data.astype(np.float64), c, np.zeros(0), np.zeros(0), lv, uv)
    r, ro, _ = _solve_both(lp, 10_000)
    assert r["status_name"] == ro["status_name"] == "DUAL_INFEASIBLE"
    assert r["iterations"] == ro["iterations"] and r["certificate"] == ro["cert_source"]
    _check_certificate(lp, r)
    # detection off: the planted infeasible LP runs to its limit
    lp = lpgen.infeasible_lp("primal", 1, 433, 650)
    r, ro, _ = _solve_both(lp, 6400, detect_infeasibility=0)
    assert r["status_name"] == ro["status_name"] == "ITERATION_LIMIT"
    assert r["certificate"] == 0 and r["kkt_passes"] == ro["kkt_passes"]
    with pytest.raises(pd.PdlpError):
        pd.Problem(lp).solve(pd.pdlp_params_default(eps_infeasible=-1.0))


def _batch_lps():
    return [lpgen.infeasible_lp("primal", 1, 433, 650), lpgen.planted_uniform(300, 450, 8, seed=7),
            lpgen.infeasible_lp("dual", 6, 433, 650), lpgen.infeasible_lp("primal", 2, 900, 1350),
            lpgen.infeasible_lp("dual", 0, 900, 1350)]


@pytest.mark.parametrize("eps", [1e30, 1e-1])
def test_batch_early_checks_match_oracle(eps):
    say(f"batch early infeasibility checks eps={eps}")
    lps = _batch_lps()
    prm = pd.pdlp_params_default(max_iters=640, eps_infeasible=eps)
    res = pd.Batch(lps).solve(prm)
    for i, (lp, r) in enumerate(zip(lps, res)):
        s = oracle.Solver(lp, oracle.Params(max_iters=640, eps_infeas=eps))
        ro = s.solve()
        assert r["status_name"] == ro["status_name"], i
        for key in ("iterations", "attempts", "restarts_i", "restarts_ii", "restarts_iii",
                    "kkt_passes"):
            assert r[key] == ro[key], (i, key)
        assert r["certificate"] == ro["cert_source"], i
        if r["iterations"] > 128:
            continue   # not declared early: decisions only (trajectories drift by k = 640)
        xo, yo = s.solution()
        if ro["cert_source"]:
            _close_certificate(lp, r, xo, yo, prm)
            _check_certificate(lp, r, eps)
        else:
            assert rel(r["x"], xo) <= 1e-8 and rel(r["y"], yo) <= 1e-8, i


def test_batch_whole_runs_detect_per_instance():
    say("batch whole runs with infeasible instances")
    lps = _batch_lps()
    res = pd.Batch(lps).solve(pd.pdlp_params_default(max_iters=300_000))
    expect = ["PRIMAL_INFEASIBLE", "OPTIMAL", "DUAL_INFEASIBLE", "PRIMAL_INFEASIBLE",
              "DUAL_INFEASIBLE"]
    for i, (lp, r) in enumerate(zip(lps, res)):
        assert r["status_name"] == expect[i], i
        if r["status_name"] != "OPTIMAL":
            _check_certificate(lp, r)
        else:
            assert r["certificate"] == 0
            assert r["primal_obj"] == pytest.approx(lp.p_star, rel=1e-6)


@pytest.mark.parametrize("i", [0, 1])
def test_all_boxed_primal_infeasible_matches_oracle(i):
    """Every variable boxed: Xbar = {0}, so the x part of the candidates is
    skipped (its test cannot pass); detection comes at the first check."""
    say(f"boxed primal infeasible {i}")
    lp = lpgen.infeasible_lp("primal_boxed", i, 900, 1350)
    r, ro, s = _solve_both(lp, 10_000)
    assert r["status_name"] == ro["status_name"] == "PRIMAL_INFEASIBLE"
    assert r["iterations"] == ro["iterations"] and r["certificate"] == ro["cert_source"]
    assert r["kkt_passes"] == ro["kkt_passes"]
    xo, yo = s.solution()
    _close_certificate(lp, r, xo, yo, pd.pdlp_params_default(max_iters=10_000))
    assert not r["x"].any()
    _check_certificate(lp, r)


def test_batch_all_boxed_matches_oracle():
    say("batch, all variables boxed")
    lps = [lpgen.infeasible_lp("primal_boxed", 0, 433, 650), lpgen.planted_uniform(300, 450, 8, seed=7),
           lpgen.infeasible_lp("primal_boxed", 1, 900, 1350)]
    prm = pd.pdlp_params_default(max_iters=20_000)
    res = pd.Batch(lps).solve(prm)
    for i, (lp, r) in enumerate(zip(lps, res)):
        s = oracle.Solver(lp, oracle.Params(max_iters=20_000))
        ro = s.solve()
        assert r["status_name"] == ro["status_name"], i
        assert r["certificate"] == ro["cert_source"], i
        if ro["cert_source"]:
            assert r["iterations"] == ro["iterations"], i
            xo, yo = s.solution()
            _close_certificate(lp, r, xo, yo, prm)
            _check_certificate(lp, r)
