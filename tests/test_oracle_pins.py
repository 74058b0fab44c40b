"""Pins of the oracle's Algorithm 2 step rule, its Algorithm 4 polishing
schedule and its numerical-error path (CPU only).

* Algorithm 2 (Section 3, "Step size choice"): every rejected attempt ends
  with eta' < eta_bar < eta; rejection happens exactly when eta > eta_bar;
  the counter in the factors advances by one per attempt; eta' follows the
  rule with the paper's exponents (0.3 on the reduction of eta_bar, 0.6 on
  the growth of eta, tests/golden/paper_constants.json).
* The reading of the step test (magnitude of the interaction) is pinned to
  Appendix B: PDHG there is the saddle form with K = -A, whose metric
  ||dz||_omega^2 / eta + 2 dy^T A dx must stay nonnegative on a step.  The
  magnitude rule keeps it nonnegative on every accepted step; the printed
  signed rule accepts steps where it is negative (and stalls), shown on a
  committed seed.  The traced movement and interaction are recomputed from
  the iterates with scipy.
* Algorithm 4: polishing is tested at k = 100, 200, 400, ... with sub-runs
  capped at k/8, each sub-run stopping at its start, at multiples of the
  check cadence or at the cap.
* Section 3, "Periodic checks" (termination also on a numerical error): an
  objective entry or a bound that overflows the step's squared norms ends
  the solve with NUMERICAL_ERROR and a finite returned point.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from tests.test_golden_constants import constant


def _traced(lp, eta_hat=None, **kw):
    s = oracle.Solver(lp, oracle.Params(**kw))
    if eta_hat is not None:
        s.st.eta_hat = eta_hat
    r = s.traced()
    return s, r, r["trace"]


CASES = [(100, 200, 5, seed, eta0) for seed in range(4) for eta0 in (None, 20.0)] + \
        [(50, 100, 4, 1, None), (300, 600, 6, 2, 50.0)]


@pytest.mark.parametrize("m,n,k,seed,eta0", CASES)
def test_rejections_land_below_eta_bar(m, n, k, seed, eta0):
    lp = lpgen.planted_uniform(m, n, k, seed=seed)
    s, r, t = _traced(lp, eta_hat=eta0, max_iters=3000)
    assert t["count"] == r["attempts"] == len(t["eta"])
    acc = t["accepted"] == 1
    # rejection happens exactly when the trial step exceeds eta_bar
    assert np.array_equal(~acc, t["eta"] > t["eta_bar"])
    rej = np.flatnonzero(~acc)
    for q in rej:
        assert t["eta_next"][q] < t["eta_bar"][q] < t["eta"][q], q
        assert t["eta"][q + 1] == t["eta_next"][q]          # the retry uses eta'
    # after an accepted step the next attempt starts from its eta' (eta_hat)
    for q in np.flatnonzero(acc[:-1]):
        assert t["eta"][q + 1] == t["eta_next"][q]
    # the counter of the factors advances by one per attempt, accepted or not
    assert np.array_equal(t["attempt"], np.arange(1, len(t["eta"]) + 1))
    # eta_bar >= 1/||A~||_2 on every attempt (Section 3, "Step size choice")
    A = sp.csr_matrix((s.scaled.val, s.scaled.col, s.scaled.row_ptr), shape=(s.m, s.n))
    nrm = np.linalg.norm(A.toarray(), 2)
    assert np.all(t["eta_bar"] >= (1 - 1e-12) / nrm)
    if eta0 is not None:
        assert len(rej) >= 1


def test_step_rule_factors_use_the_papers_exponents():
    """eta' = min((1 - (j+1)^-0.3) eta_bar, (1 + (j+1)^-0.6) eta) with j the
    attempt counter; the exponents come from the golden file (Algorithm 2),
    so swapping them or using the accepted count k fails here."""
    r_exp, g_exp = constant("red_exp"), constant("grow_exp")
    lp = lpgen.planted_uniform(100, 200, 5, seed=3)
    _, r, t = _traced(lp, eta_hat=20.0, max_iters=1500)
    j = t["attempt"].astype(float)
    want = np.minimum((1.0 - (j + 1.0) ** -r_exp) * t["eta_bar"],
                      (1.0 + (j + 1.0) ** -g_exp) * t["eta"])
    np.testing.assert_allclose(t["eta_next"], want, rtol=1e-15, atol=0)
    # the reduction branch is the one taken on every rejection (eta > eta_bar)
    rej = t["accepted"] == 0
    np.testing.assert_allclose(t["eta_next"][rej] / t["eta_bar"][rej],
                               1.0 - (j[rej] + 1.0) ** -r_exp, rtol=1e-14)
    # the attempt counter differs from the accepted count once a step was rejected
    assert np.any(t["attempt"] != t["k"] + 1)


def test_traced_movement_and_interaction_match_the_iterates():
    """num = omega ||dx||^2 + ||dy||^2 / omega and cross = dy^T A~ dx of an
    accepted step, recomputed from the iterates before and after it."""
    lp = lpgen.planted_uniform(80, 160, 5, seed=4)
    s = oracle.Solver(lp, oracle.Params(max_iters=5))
    A = sp.csr_matrix((s.scaled.val, s.scaled.col, s.scaled.row_ptr), shape=(s.m, s.n))
    x0, y0, w = s.x.copy(), s.y.copy(), s.omega
    r = s.traced(oracle.Params(max_iters=1, terminate=False))
    t = r["trace"]
    assert t["accepted"][-1] == 1
    dx, dy = s.x - x0, s.y - y0
    assert t["num"][-1] == pytest.approx(w * dx @ dx + dy @ dy / w, rel=1e-13)
    assert t["cross"][-1] == pytest.approx(dy @ (A @ dx), rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_accepted_steps_keep_the_appendix_b_metric_nonnegative(seed):
    lp = lpgen.planted_uniform(100, 200, 5, seed=seed)
    _, r, t = _traced(lp, eta_hat=20.0, max_iters=3000)
    acc = t["accepted"] == 1
    metric = t["num"][acc] / t["eta"][acc] + 2.0 * t["cross"][acc]
    assert np.all(metric >= -1e-12 * t["num"][acc] / t["eta"][acc])
    assert r["status_name"] == "OPTIMAL"


def test_printed_signed_rule_accepts_steps_with_negative_metric():
    """Committed seed: under the printed rule (eta_bar = inf unless the
    interaction is positive) the accepted steps have a negative Appendix B
    metric -- the interaction of these steps is negative -- and the solve
    stalls; the magnitude reading solves the same LP."""
    lp = lpgen.planted_uniform(100, 200, 5, seed=0)
    _, r_lit, t = _traced(lp, eta_hat=20.0, max_iters=2000, signed_step_rule=True)
    acc = t["accepted"] == 1
    metric = t["num"][acc] / t["eta"][acc] + 2.0 * t["cross"][acc]
    assert np.sum(metric < 0) > 0.9 * acc.sum()
    assert r_lit["status_name"] == "ITERATION_LIMIT" and r_lit["primal_res_rel"] > 1e-2
    _, r_abs, _ = _traced(lp, eta_hat=20.0, max_iters=2000)
    assert r_abs["status_name"] == "OPTIMAL"


# ------------------------------------------------------------- Algorithm 4

@pytest.mark.parametrize("m,n,k,seed", [(100, 200, 5, 0), (100, 200, 5, 1), (300, 600, 6, 0),
                                        (1000, 2000, 10, 0)])
def test_polishing_schedule(m, n, k, seed):
    """eps_gap = 2 makes the relative gap (always <= 1) pass at every point,
    so every polishing point runs its primal sub-run."""
    first, div, grow = (constant("polish_first"), constant("polish_cap_divisor"),
                        constant("polish_growth"))
    every = constant("check_every")
    lp = lpgen.planted_uniform(m, n, k, seed=seed)
    _, r, t = _traced(lp, max_iters=5000, polish=True, eps_gap=2.0)
    npol = len(t["pol_k"])
    assert npol == r["polish_attempts"] >= 3
    assert np.array_equal(t["pol_k"], first * grow ** np.arange(npol))
    assert np.array_equal(t["pol_cap"], t["pol_k"] // div)
    total = 0
    for q in range(npol):
        cap, p, d = t["pol_cap"][q], t["pol_primal"][q], t["pol_dual"][q]
        assert 0 <= p <= cap
        assert p == cap or p % every == 0        # checks at the start, every 64, at the cap
        if p < cap:
            assert d >= 0                        # primal sub-run passed: dual sub-run runs
        if d >= 0:
            assert d <= cap and (d == cap or d % every == 0)
        total += p + max(d, 0)
    assert total == r["polish_iters"]
    # sub-run attempts never exceed the cap of their polishing point
    ph = t["phase"]
    assert np.all(t["k"][ph > 0] < t["pol_cap"].max())
    if r["polished"]:
        # the polished pair is returned at the point that produced it
        assert r["iterations"] == t["pol_k"][-1]
    else:
        # no polishing point succeeded; the main run terminated by itself
        assert r["status_name"] == "OPTIMAL" and r["iterations"] % every == 0


def test_polishing_is_skipped_while_the_gap_is_above_eps():
    lp = lpgen.planted_uniform(100, 200, 5, seed=1)
    _, r, t = _traced(lp, max_iters=900, polish=True, eps_gap=1e-14, eps_feas=1e-14)
    assert np.array_equal(t["pol_k"], [100, 200, 400, 800])
    assert np.all(t["pol_gap"] >= 1e-14)
    assert np.all(t["pol_primal"] == -1) and np.all(t["pol_dual"] == -1)
    assert r["polish_iters"] == 0 and not np.any(t["phase"] > 0)


# ------------------------------------------------------- numerical error

def overflow_lp(kind: str):
    """LPs on which the first step overflows in FP64 (NUMERICAL_ERROR):
    'objective': equality rows with zero right-hand side (so omega = 1) and
    free variables, one objective entry 1e200, so ||x' - x||^2 overflows;
    'bound': one row's lower bound 1e300 (||b||^2 overflows, omega = 0, and
    the step norm becomes 0 * inf)."""
    lp = lpgen.planted_uniform(60, 120, 4, seed=11)
    if kind == "objective":
        lp.lc = np.zeros(lp.m)
        lp.uc = np.zeros(lp.m)
        lp.lv = np.full(lp.n, -np.inf)
        lp.uv = np.full(lp.n, np.inf)
        lp.c = lp.c.copy()
        lp.c[3] = 1e200
    else:
        lp.lc = lp.lc.copy()
        lp.uc = lp.uc.copy()
        lp.lc[5] = 1e300
        lp.uc[5] = np.inf
    return lp


@pytest.mark.parametrize("kind", ["objective", "bound"])
def test_overflow_ends_with_numerical_error(kind):
    lp = overflow_lp(kind)
    s = oracle.Solver(lp, oracle.Params(max_iters=500))
    r = s.solve()
    assert r["status_name"] == "NUMERICAL_ERROR"
    assert r["iterations"] == 0
    x, y = s.solution()
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
