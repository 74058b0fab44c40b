"""Two-phase A~^T y' (segmented gathers) against the oracle and the one-pass product.

With segmented_gathers = 1 the library gathers y' in segments of its index
range (phase 1: pair sums per (row, segment)) and then stages the pair sums
per row block (phase 2).  A row of A^T with at most 64 nonzeros is summed in
the same order as by the one-pass product and the oracle (bitwise); a longer
row is summed per segment and then over the segments, bounded by 1e-14
relative to |A|^T |y|.  Iterations and solves follow the oracle as the
one-pass path does.
"""
import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import STAGE, gpu_params, make_lp, rel, say

pytestmark = pytest.mark.gpu


def _products(lp, seg, y, scale=False):
    prm = gpu_params(segmented_gathers=seg) if scale else \
        gpu_params(ruiz_iters=0, pock_chambolle=0, segmented_gathers=seg)
    prob = pd.Problem(lp, prm)
    aty, _ = prob.spmv(y, transpose=True)
    prob.close()
    return aty


@pytest.mark.parametrize("kind", ["skewed", "uniform", "ragged"])
def test_segmented_product_matches_oracle(kind):
    say(f"segmented A^T y parity {kind}")
    if kind == "skewed":
        lp = lpgen.planted_skewed(30000, 40000, seed=3, n_dense=40)
    elif kind == "uniform":
        lp = lpgen.planted_uniform(9001, 12007, 9, seed=5)
    else:
        # ragged: empty rows and columns, rows crossing every segment, a few
        # columns with more nonzeros than any segment boundary spacing
        rng = np.random.default_rng(11)
        m, n = 5003, 3001
        dense = np.zeros((m, n))
        for j in range(n):
            k = 2500 if j % 997 == 3 else int(rng.integers(0, 12))
            dense[rng.choice(m, size=k, replace=False), j] = rng.standard_normal(k)
        dense[17] = 0.0
        lp = make_lp(dense)
    v = oracle.LPView.of(lp)
    rng = np.random.default_rng(1)
    y = rng.standard_normal(lp.m)
    aty_o = oracle.spmv_t(v, y)
    aty_s = _products(lp, 1, y)
    aty_1 = _products(lp, 0, y)
    cl = np.bincount(lp.col, minlength=lp.n)
    short = cl <= STAGE
    assert np.array_equal(aty_s[short], aty_o[short])
    assert np.array_equal(aty_s[short], aty_1[short])
    scale = np.abs(lp.csr()).T @ np.abs(y)
    assert np.all(np.abs(aty_s - aty_o) <= 1e-14 * scale + 1e-300)
    if kind != "uniform":
        assert (cl > STAGE).any()


def test_segmented_product_exact_on_integers():
    say("segmented A^T y integer-valued")
    rng = np.random.default_rng(7)
    m, n = 6000, 40
    dense = np.zeros((m, n))
    for j in range(n):
        k = 5000 if j in (3, 17) else int(rng.integers(0, 400))
        rows = rng.choice(m, size=k, replace=False)
        dense[rows, j] = rng.integers(-5, 6, size=k)
    lp = make_lp(dense)
    y = rng.integers(-7, 8, size=m).astype(float)
    assert np.array_equal(_products(lp, 1, y), dense.T @ y)


def test_segmented_iterations_match_oracle():
    say("segmented: one and k iterations against the oracle")
    lp = lpgen.small_lp()
    prob = pd.Problem(lp, gpu_params(segmented_gathers=1))
    st = prob.state(gpu_params(segmented_gathers=1))
    o = oracle.Solver(lp)
    st.iterate(1)
    o.iterate(1)
    g = st.get()
    for k in ("x", "y", "ax", "aty", "sx", "sy"):
        assert rel(g[k], getattr(o, k)) <= 1e-12, k
    info = st.iterate(299)
    o.iterate(299)
    oc = o.counters()
    for key in ("k", "t", "n_outer", "attempts", "restarts_i", "restarts_ii", "restarts_iii"):
        assert info[key] == oc[key], key
    g = st.get()
    for key in ("x", "y", "x0", "y0"):
        assert rel(g[key], getattr(o, key)) <= 1e-8, key


def test_segmented_skewed_runs_follow_the_oracle():
    say("segmented on a skewed LP: 64 iterations against the oracle, then a solve")
    lp = lpgen.planted_skewed(20000, 25000, seed=9, n_dense=30)
    prob = pd.Problem(lp, gpu_params(segmented_gathers=1))
    st = prob.state(gpu_params(segmented_gathers=1))
    o = oracle.Solver(lp)
    info = st.iterate(64)
    o.iterate(64)
    oc = o.counters()
    for key in ("k", "t", "n_outer", "attempts", "restarts_i", "restarts_ii", "restarts_iii"):
        assert info[key] == oc[key], key
    g = st.get()
    # the tolerance of the one-pass path's 64-step parity test
    for key in ("x", "y", "x0", "y0"):
        assert rel(g[key], getattr(o, key)) <= 1e-8, key
    prob.close()


@pytest.mark.parametrize("polish", [0, 1])
def test_segmented_solves(polish):
    say(f"segmented solve, polish={polish}")
    lp = lpgen.planted_uniform(3000, 5000, 8, seed=41)
    eps_gap = 1e-2 if polish else 1e-8
    prm = gpu_params(segmented_gathers=1, eps_feas=1e-8, eps_gap=eps_gap, polish=polish,
                     max_iters=100000)
    prob = pd.Problem(lp, prm)
    r = prob.solve(prm)
    prob.close()
    ro = oracle.Solver(lp, oracle.Params(eps_feas=1e-8, eps_gap=eps_gap, polish=bool(polish),
                                         max_iters=100000)).solve()
    assert r["status_name"] == ro["status_name"] == "OPTIMAL"
    assert r["primal_res_rel"] <= 1e-8 and r["dual_res_rel"] <= 1e-8 and r["rel_gap"] <= eps_gap
    x = r["x"]
    ax = lp.csr() @ x
    q = np.maximum(1.0, np.maximum(np.abs(np.where(np.isfinite(lp.lc), lp.lc, 0)),
                                   np.abs(np.where(np.isfinite(lp.uc), lp.uc, 0))))
    assert np.all(ax >= lp.lc - 1e-8 * q) and np.all(ax <= lp.uc + 1e-8 * q)
    assert np.all(x >= lp.lv) and np.all(x <= lp.uv)
    if polish:
        assert r["polished"] == 1 and r["polish_attempts"] == ro["polish_attempts"]
        assert abs(lp.c @ x - lp.p_star) <= 2e-2 * abs(lp.p_star)
    else:
        assert r["primal_obj"] == pytest.approx(ro["primal_obj"], rel=1e-6)
        assert lp.c @ x == pytest.approx(lp.p_star, rel=1e-6)


def test_segmented_runs_are_deterministic():
    say("segmented determinism")
    lp = lpgen.planted_skewed(8000, 10000, seed=21, n_dense=20)
    out = []
    for _ in range(2):
        prob = pd.Problem(lp, gpu_params(segmented_gathers=1))
        st = prob.state(gpu_params(segmented_gathers=1))
        st.iterate(130)
        out.append(st.get())
        prob.close()
    for k in ("x", "y", "ax", "aty", "sx", "sy"):
        assert np.array_equal(out[0][k], out[1][k]), k


def test_segmented_layout_on_sparse_wide_index_ranges():
    """y' of 1.2M entries in 8 segments with only ~50k nonzeros: most rows
    empty and whole segments without a short-column nonzero, long columns
    crossing every segment, empty columns: the product against the oracle
    (short columns bitwise), then 64 iterations against the oracle."""
    say("segmented layout, sparse 1.2M-row LP")
    import scipy.sparse as sp
    rng = np.random.default_rng(17)
    m, n = 1_200_000, 1500
    rows, cols = [], []
    for j in range(n):
        if j % 500 == 7:
            k = 4000                       # long columns over the whole row range
            r = rng.choice(m, size=k, replace=False)
        elif j % 3 == 0:
            continue                       # empty columns
        else:
            k = int(rng.integers(1, 60))
            r = rng.choice(200_000, size=k, replace=False) + 600_000 * (j % 2)
        rows.append(r)
        cols.append(np.full(r.size, j))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    A = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(m, n))
    A.sort_indices()
    x0 = rng.uniform(0, 1, n)
    b = A @ x0
    lp = lpgen.LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data,
                  rng.standard_normal(n), b - 0.5, b + 0.5, np.zeros(n), np.ones(n))
    prob = pd.Problem(lp, gpu_params(ruiz_iters=0, pock_chambolle=0, segmented_gathers=1))
    y = rng.standard_normal(m)
    aty, _ = prob.spmv(y, transpose=True)
    aty_o = oracle.spmv_t(oracle.LPView.of(lp), y)
    cl = np.bincount(lp.col, minlength=n)
    assert np.array_equal(aty[cl <= STAGE], aty_o[cl <= STAGE])
    scale = np.abs(A).T @ np.abs(y)
    assert np.all(np.abs(aty - aty_o) <= 1e-14 * scale + 1e-300)
    prob.close()
    prob = pd.Problem(lp, gpu_params(segmented_gathers=1))
    st = prob.state(gpu_params(segmented_gathers=1))
    o = oracle.Solver(lp)
    info = st.iterate(64)
    o.iterate(64)
    oc = o.counters()
    for key in ("k", "t", "n_outer", "attempts", "restarts_i", "restarts_ii", "restarts_iii"):
        assert info[key] == oc[key], key
    g = st.get()
    for key in ("x", "y"):
        assert rel(g[key], getattr(o, key)) <= 1e-8, key
    prob.close()
