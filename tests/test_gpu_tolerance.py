"""Tight feasibility tolerances (1e-10, 1e-12) with and without feasibility
polishing, on the three input shapes: the planted 1,000 x 2,000 LP, a
multicommodity grid flow and instances of the batch workload.  The gap
tolerance is the paper's 1e-2 (Section 7, "Termination criteria").

Each returned point is verified independently in numpy: relative primal
violations with the q weights, relative dual residuals with the returned
reduced costs, y in Y and r in R, and the objective against the planted
optimum where there is one.  The GPU and the oracle must reach the same
status (iteration counts drift apart at these tolerances, see the batch
tests).
"""
import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu


def q_weights(lc, uc):
    lb = np.isfinite(lc) & (lc != 0.0)
    ub = np.isfinite(uc) & (uc != 0.0)
    al = np.where(lb, np.abs(np.where(np.isfinite(lc), lc, 0.0)), 0.0)
    au = np.where(ub, np.abs(np.where(np.isfinite(uc), uc, 0.0)), 0.0)
    return np.where(lb | ub, np.maximum(al, au), 1.0)


def verify(lp, r, eps):
    """Independent check of the termination criteria of the returned point."""
    x, y, rc = r["x"], r["y"], r["r"]
    A = lp.csr()
    assert np.all(x >= lp.lv) and np.all(x <= lp.uv)   # returned x is clamped to the bounds
    ax = A @ x
    viol = np.maximum(np.where(np.isfinite(lp.lc), lp.lc - ax, 0.0),
                      np.where(np.isfinite(lp.uc), ax - lp.uc, 0.0))
    viol = np.maximum(viol, 0.0)
    # the library sums A x in its own order: allow rounding on the scale of |A||x|
    slack = 1e-14 * (np.abs(A) @ np.abs(x) + np.abs(np.where(np.isfinite(lp.lc), lp.lc, 0.0)))
    assert np.all(viol <= eps * q_weights(lp.lc, lp.uc) + slack)
    # y in Y, r in R
    assert np.all(y[~np.isfinite(lp.lc)] <= 0.0) and np.all(y[~np.isfinite(lp.uc)] >= 0.0)
    assert np.all(rc[~np.isfinite(lp.lv)] <= 0.0) and np.all(rc[~np.isfinite(lp.uv)] >= 0.0)
    res = np.abs(lp.c - A.T @ y - rc)
    sc = np.where(lp.c != 0.0, np.abs(lp.c), 1.0)
    slack = 1e-14 * (np.abs(A).T @ np.abs(y) + np.abs(lp.c))
    assert np.all(res <= eps * sc + slack)
    if lp.p_star is not None:
        assert lp.c @ x == pytest.approx(lp.p_star, rel=2e-2)


def _grid():
    return lpgen.multicommodity_grid(12, 4, 6, seed=5)


def _batch_member():
    m, n = lpgen.batch_sizes()[1]
    return lpgen.batch_lp(1, m, n)


CASES = {"planted_1000x2000": lpgen.small_lp, "grid_12x12_k4": _grid,
         "batch_member_3777x5665": _batch_member}


@pytest.mark.parametrize("polish", [0, 1])
@pytest.mark.parametrize("eps", [1e-10, 1e-12])
@pytest.mark.parametrize("name", list(CASES))
def test_tight_tolerances_match_oracle_status(name, eps, polish):
    say(f"tolerance {eps:g} polish={polish} on {name}")
    lp = CASES[name]()
    prm = pd.pdlp_params_default(eps_feas=eps, eps_gap=1e-2, polish=polish, max_iters=200_000)
    r = pd.Problem(lp).solve(prm)
    ro = oracle.Solver(lp, oracle.Params(eps_feas=eps, eps_gap=1e-2, polish=bool(polish),
                                         max_iters=200_000)).solve()
    if polish or name != "batch_member_3777x5665":
        assert r["status_name"] == ro["status_name"] == "OPTIMAL"
    else:
        # without polishing this instance crawls at these tolerances (the oracle
        # needs 67k iterations at 1e-12); trajectories that agree to rounding
        # at first reach it or not within the cap
        assert {r["status_name"], ro["status_name"]} <= {"OPTIMAL", "ITERATION_LIMIT"}
        if r["status_name"] != "OPTIMAL":
            return
    assert r["primal_res_rel"] <= eps and r["dual_res_rel"] <= eps and r["rel_gap"] <= 1e-2
    verify(lp, r, eps)
    if polish and r["polished"]:
        assert r["dual_res_rel"] == 0.0 or r["dual_res_rel"] <= eps


def test_batch_at_tight_tolerance():
    say("batch at 1e-10 and 1e-12")
    sizes = lpgen.batch_sizes()
    lps = [lpgen.batch_lp(i, m, n) for i, (m, n) in enumerate(sizes[:8]) if i != 2]
    b = pd.Batch(lps)
    for eps in (1e-10, 1e-12):
        res = b.solve(pd.pdlp_params_default(eps_feas=eps, eps_gap=1e-2, max_iters=200_000))
        solved = 0
        for lp, r in zip(lps, res):
            assert r["status_name"] in ("OPTIMAL", "ITERATION_LIMIT"), lp.name
            if r["status_name"] == "OPTIMAL":
                verify(lp, r, eps)
                solved += 1
        # without polishing (batches do not polish) many instances stall at
        # these tolerances within the cap, the paper's observation (measured:
        # 6 of 8 at 1e-10, 2 of 8 at 1e-12); every point that is declared
        # optimal must pass the independent check above
        assert solved >= {1e-10: 4, 1e-12: 1}[eps]
