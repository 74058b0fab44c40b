"""GPU parity of the Algorithm 5 mode (Appendix C) against the FP64 oracle.

Constant steps leave no step decision to diverge on, so the restart points
of the two sides agree to rounding (products of short rows are summed in
the oracle's order; only the reductions of the step norms differ, which
a constant step does not use).  The GPU's own restart points must also
satisfy both claims of Theorem 1 on products of simplices.
"""
import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import rel, say
from tests.test_oracle_alg5 import (alg5_params, dist_to_simplices, simplices_lp, start_at,
                                    theorem1_constants)

pytestmark = pytest.mark.gpu


def gpu_alg5(eta, ell, omega=1.0, **kw):
    return pd.pdlp_params_default(restart_period=ell, fixed_step_size=eta,
                                  fixed_primal_weight=omega, ruiz_iters=0, pock_chambolle=0,
                                  detect_infeasibility=0, **kw)


def _pair(lp, eta, ell, omega, x0):
    """Oracle solver and GPU state, both at (x0, 0) without scaling."""
    o = oracle.Solver(lp, alg5_params(eta, ell, omega), scale=False)
    start_at(o, lp, x0)
    prob = pd.Problem(lp, gpu_alg5(eta, ell, omega))
    st = prob.state(gpu_alg5(eta, ell, omega))
    blob = {key: getattr(o, key).copy() for key in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")}
    blob.update(o.counters())
    st.set(blob)
    return o, prob, st


@pytest.mark.parametrize("blocks,k,alpha", [(3000, 4, 0.5), (1111, 9, 0.8)])
def test_theorem1_on_gpu_and_parity(blocks, k, alpha):
    say(f"Algorithm 5 on simplices {blocks}x{k} alpha={alpha}")
    lp, b = simplices_lp(blocks, k, 11)
    eta, q, ell = theorem1_constants(k, alpha)
    x0 = np.random.default_rng(12).uniform(0.0, 3.0, lp.n)
    o, prob, st = _pair(lp, eta, ell, 1.0, x0)
    d0 = dist_to_simplices(x0, b, k)
    for n in range(1, 6):
        info = st.iterate(ell)
        o.iterate(ell)
        g = st.get()
        assert info["restarts_iii"] == n and info["n_outer"] == n and info["t"] == 0
        assert not g["y"].any()
        assert rel(g["x"], o.x) <= 1e-12
        d = dist_to_simplices(g["x"], b, k)
        assert d <= 2.0 ** -n * d0 + 1e-12
        assert np.linalg.norm(g["x"] - x0) <= 2 * (q + 2) * d0


@pytest.mark.parametrize("omega", [1.0, 2.5])
def test_restart_points_match_oracle_on_mixed_bounds(omega):
    say(f"Algorithm 5 on a mixed-bound feasibility LP, omega={omega}")
    lp = lpgen.infeasible_lp("dual", 3, 900, 1350)
    lp.c = np.zeros(lp.n)                     # feasible at x_feas
    eta, ell = 0.3, 97
    x0 = np.clip(np.zeros(lp.n), lp.lv, lp.uv)
    o, prob, st = _pair(lp, eta, ell, omega, x0)
    for n in range(1, 4):
        st.iterate(ell)
        o.iterate(ell)
        g = st.get()
        for key in ("x", "ax", "x0"):
            assert rel(g[key], getattr(o, key)) <= 1e-12, key
        assert not g["y"].any() and not g["aty"].any()
        assert g["omega"] == omega


def test_solve_terminates_like_the_oracle():
    say("Algorithm 5 solve to 1e-10 feasibility")
    lp, b = simplices_lp(2000, 4, 21)
    eta, q, ell = theorem1_constants(4, 0.5)
    prm = gpu_alg5(eta, ell, eps_feas=1e-10, max_iters=20_000)
    r = pd.Problem(lp, prm).solve(prm)
    o = oracle.Solver(lp, alg5_params(eta, ell, eps_feas=1e-10, max_iters=20_000), scale=False)
    ro = o.solve()
    assert r["status_name"] == ro["status_name"] == "OPTIMAL"
    assert r["iterations"] == ro["iterations"] and r["restarts"] == ro["restarts"]
    assert not r["y"].any()
    # dist <= ||A x - b||_2 (Hoffman constant >= 1) <= sqrt(m) * 1e-10 * max |b|
    assert dist_to_simplices(r["x"], b, 4) <= np.sqrt(lp.m) * 1e-10 * np.abs(b).max()
    xo, _ = o.solution()
    assert rel(r["x"], xo) <= 1e-12


def test_mode_rejections():
    say("Algorithm 5 rejections")
    lp, _ = simplices_lp(50, 4, 1)
    prob = pd.Problem(lp)
    for bad in (dict(restart_period=10), dict(restart_period=10, fixed_step_size=0.1,
                                              fixed_primal_weight=0.0),
                dict(restart_period=10, fixed_step_size=0.1, polish=1),
                dict(restart_period=-1)):
        with pytest.raises(pd.PdlpError) as ei:
            prob.solve(pd.pdlp_params_default(**bad))
        assert ei.value.code == pd.PDLP_ERR_INVALID_ARGUMENT
    b = pd.Batch([lp])
    with pytest.raises(pd.PdlpError):
        b.solve(pd.pdlp_params_default(restart_period=10, fixed_step_size=0.1))
