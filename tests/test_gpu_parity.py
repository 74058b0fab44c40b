"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Tolerances: integer-valued products are exact; a stream-mode row (at most
64 nonzeros) is summed in the same order as the oracle and must match
bitwise; longer rows use a wave or workgroup tree, bounded by 1e-14
relative.  The
scaled problem is computed in the same order on both sides (bitwise).  One
PDHG iteration from the same state matches to 1e-12 norm-wise relative with
identical decisions; whole solves match on relative feasibility <= 1e-8 and
objective within 1e-6 relative.
"""
import sys

import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd

pytestmark = pytest.mark.gpu

STAGE = 64  # longest row summed sequentially (stream path)


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    den = max(np.linalg.norm(b), 1e-300)
    return np.linalg.norm(a - b) / den


def gpu_params(**kw):
    return pd.pdlp_params_default(**kw)


def orc_params(**kw):
    return oracle.Params(**kw)


def make_lp(dense, c=None, lc=None, uc=None, lv=None, uv=None):
    import scipy.sparse as sp
    A = sp.csr_matrix(dense)
    A.sort_indices()
    m, n = A.shape
    z = lambda k: np.zeros(k)
    return lpgen.LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                    A.data.astype(np.float64), z(n) if c is None else c,
                    z(m) if lc is None else lc, z(m) if uc is None else uc,
                    z(n) if lv is None else lv, z(n) if uv is None else uv)


# ---------------------------------------------------------------- products

def test_spmv_exact_on_integer_matrix_with_long_rows():
    say("spmv integer-valued, long rows, no scaling")
    rng = np.random.default_rng(7)
    m, n = 40, 6000
    dense = np.zeros((m, n))
    for i in range(m):
        k = 5000 if i in (3, 17) else int(rng.integers(0, 40))  # two long rows, some empty
        cols = rng.choice(n, size=k, replace=False)
        dense[i, cols] = rng.integers(-5, 6, size=k)
    dense[dense == 0] = 0.0
    lp = make_lp(dense)
    prob = pd.Problem(lp, gpu_params(ruiz_iters=0, pock_chambolle=0))
    x = rng.integers(-7, 8, size=n).astype(float)
    y = rng.integers(-7, 8, size=m).astype(float)
    ax, _ = prob.spmv(x)
    aty, _ = prob.spmv(y, transpose=True)
    assert np.array_equal(ax, dense @ x)
    assert np.array_equal(aty, dense.T @ y)


@pytest.mark.parametrize("kind", ["small", "skewed"])
def test_spmv_matches_oracle(kind):
    say(f"spmv parity {kind}")
    lp = lpgen.small_lp() if kind == "small" else lpgen.planted_skewed(30000, 40000, seed=3, n_dense=40)
    prob = pd.Problem(lp, gpu_params(ruiz_iters=0, pock_chambolle=0))
    v = oracle.LPView.of(lp)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    ax, _ = prob.spmv(x)
    aty, _ = prob.spmv(y, transpose=True)
    ax_o = oracle.spmv(v, x)
    aty_o = oracle.spmv_t(v, y)
    rl = np.diff(lp.row_ptr)
    cl = np.bincount(lp.col, minlength=lp.n)
    short_r, short_c = rl <= STAGE, cl <= STAGE
    assert np.array_equal(ax[short_r], ax_o[short_r])
    assert np.array_equal(aty[short_c], aty_o[short_c])
    scale_r = np.abs(lp.csr()) @ np.abs(x)
    scale_c = np.abs(lp.csr()).T @ np.abs(y)
    assert np.all(np.abs(ax - ax_o) <= 1e-14 * scale_r + 1e-300)
    assert np.all(np.abs(aty - aty_o) <= 1e-14 * scale_c + 1e-300)
    if kind == "skewed":
        assert (cl > 1024).any() and ((cl > 64) & (cl <= 1024)).any()  # long and wave paths ran


# ------------------------------------------------------------ preconditioning

@pytest.mark.parametrize("kind", ["small", "skewed", "grid"])
def test_preconditioning_matches_oracle(kind):
    say(f"preconditioning parity {kind}")
    lp = {"small": lpgen.small_lp, "skewed": lambda: lpgen.planted_skewed(20000, 25000, seed=9, n_dense=30),
          "grid": lambda: lpgen.multicommodity_grid(20, 3, 4, seed=2)}[kind]()
    prob = pd.Problem(lp)
    g = prob.scaled()
    val, d1, d2 = oracle.precondition(lp, 10, True)
    c, lc, uc, lv, uv = oracle.scale_vectors(lp, d1, d2)
    for name, a, b in [("d1", g["d1"], d1), ("d2", g["d2"], d2), ("val", g["val"], val),
                       ("c", g["c"], c), ("lc", g["lc"], lc), ("uc", g["uc"], uc),
                       ("lv", g["lv"], lv), ("uv", g["uv"], uv)]:
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin), name
        assert np.array_equal(a[~fin], b[~fin]), name
        np.testing.assert_allclose(a[fin], b[fin], rtol=1e-15, atol=0, err_msg=name)


# ------------------------------------------------------- normalized duality gap

@pytest.mark.parametrize("kind", ["small", "grid", "tiny"])
def test_norm_gap_matches_oracle(kind):
    say(f"normalized gap parity {kind}")
    if kind == "tiny":
        lp = lpgen.tiny_random_lp(5, 3, 4)
    elif kind == "grid":
        lp = lpgen.multicommodity_grid(15, 2, 3, seed=4)
    else:
        lp = lpgen.small_lp()
    prob = pd.Problem(lp)
    s = oracle.Solver(lp)
    sv = s.scaled
    rng = np.random.default_rng(2)
    for trial in range(6):
        x = np.clip(rng.standard_normal(lp.n), sv.lv, sv.uv)
        y = rng.standard_normal(lp.m)
        y = np.where(np.isfinite(sv.lc), y, np.minimum(y, 0))
        y = np.where(np.isfinite(sv.uc), y, np.maximum(y, 0))
        ax = oracle.spmv(sv, x); aty = oracle.spmv_t(sv, y)
        scale = 10.0 ** rng.uniform(-3, 1)
        xr = x + scale * rng.standard_normal(lp.n)
        yr = y + scale * rng.standard_normal(lp.m)
        omega = 10.0 ** rng.uniform(-1, 1)
        mu_o = oracle.norm_gap(sv, x, y, ax, aty, xr, yr, omega)
        mu_g = pd.pdlp_norm_gap(prob.h, x, y, ax, aty, xr, yr, omega)
        assert mu_g == pytest.approx(mu_o, rel=1e-12, abs=1e-300), (trial, mu_g, mu_o)


# ------------------------------------------------------------ iteration parity

def _gpu_state(lp, **kw):
    prob = pd.Problem(lp)
    st = prob.state(gpu_params(**kw))
    return prob, st


def test_initial_state_matches_oracle():
    say("initial state parity")
    lp = lpgen.small_lp()
    prob, st = _gpu_state(lp)
    g = st.get()
    o = oracle.Solver(lp)
    assert g["omega"] == pytest.approx(o.omega, rel=1e-14)
    assert g["eta_hat"] == pytest.approx(o.eta_hat, rel=1e-15)
    for k in ("x", "y", "ax", "aty", "x0", "y0"):
        assert np.array_equal(g[k], getattr(o, k)), k


def test_one_iteration_matches_oracle():
    say("one-iteration parity")
    lp = lpgen.small_lp()
    prob, st = _gpu_state(lp)
    o = oracle.Solver(lp)
    info = st.iterate(1)
    o.iterate(1)
    g = st.get()
    oc = o.counters()
    for k in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy"):
        assert rel(g[k], getattr(o, k)) <= 1e-12, k
    assert info["k"] == oc["k"] and info["t"] == oc["t"] and info["n_outer"] == oc["n_outer"]
    assert info["attempts"] == oc["attempts"]
    assert info["omega"] == pytest.approx(oc["omega"], rel=1e-12)
    assert info["eta_hat"] == pytest.approx(oc["eta_hat"], rel=1e-12)


@pytest.mark.parametrize("k", [2, 64, 300])
def test_k_iterations_match_oracle(k):
    say(f"{k}-iteration parity")
    lp = lpgen.small_lp()
    prob, st = _gpu_state(lp)
    o = oracle.Solver(lp)
    info = st.iterate(k)
    o.iterate(k)
    oc = o.counters()
    for key in ("k", "t", "n_outer", "attempts", "restarts_i", "restarts_ii", "restarts_iii"):
        assert info[key] == oc[key], key
    g = st.get()
    tol = 1e-12 if k <= 2 else 1e-8
    for key in ("x", "y", "x0", "y0"):
        assert rel(g[key], getattr(o, key)) <= tol, key
    assert info["omega"] == pytest.approx(oc["omega"], rel=tol)


def test_iterations_are_deterministic_and_resumable():
    say("determinism / resume")
    lp = lpgen.planted_uniform(700, 1300, 7, seed=17)
    p1, a = _gpu_state(lp)
    a.iterate(150); a.iterate(190)
    p2, b = _gpu_state(lp)
    b.iterate(340)
    ga, gb = a.get(), b.get()
    for key in ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy"):
        assert np.array_equal(ga[key], gb[key]), key
    # export / import
    p3, c = _gpu_state(lp)
    c.set(ga)
    c.iterate(100); b.iterate(100)
    gc, gb = c.get(), b.get()
    for key in ("x", "y", "sx", "sy"):
        assert np.array_equal(gc[key], gb[key]), key


# ---------------------------------------------------------------- full solves

def test_full_solve_small_matches_oracle_and_planted_optimum():
    say("full solve small")
    lp = lpgen.small_lp()
    prob = pd.Problem(lp)
    r = prob.solve(gpu_params(eps_feas=1e-8, eps_gap=1e-8, max_iters=100000))
    o = oracle.Solver(lp, orc_params(eps_feas=1e-8, eps_gap=1e-8, max_iters=100000))
    ro = o.solve()
    assert r["status_name"] == "OPTIMAL" and ro["status_name"] == "OPTIMAL"
    assert r["primal_res_rel"] <= 1e-8 and r["dual_res_rel"] <= 1e-8 and r["rel_gap"] <= 1e-8
    assert r["primal_obj"] == pytest.approx(lp.p_star, rel=1e-6)
    assert r["primal_obj"] == pytest.approx(ro["primal_obj"], rel=1e-6)
    # independent check of the returned point in original units
    x, y = r["x"], r["y"]
    ax = lp.csr() @ x
    q = np.ones(lp.m)
    assert np.all(ax >= lp.lc - 1e-8 * np.maximum(np.abs(lp.lc), 1)) and \
        np.all(ax <= lp.uc + 1e-8 * np.maximum(np.abs(lp.uc), 1))
    assert lp.c @ x == pytest.approx(lp.p_star, rel=1e-6)
    assert abs(r["iterations"] - ro["iterations"]) <= 64


def test_full_solve_grid_flow():
    say("full solve grid flow")
    lp = lpgen.multicommodity_grid(30, 4, 5, seed=7)
    prob = pd.Problem(lp)
    r = prob.solve(gpu_params(eps_feas=1e-6, eps_gap=1e-6, max_iters=100000))
    ro = oracle.Solver(lp, orc_params(eps_feas=1e-6, eps_gap=1e-6, max_iters=100000)).solve()
    assert r["status_name"] == "OPTIMAL" and ro["status_name"] == "OPTIMAL"
    assert r["primal_res_rel"] <= 1e-6 and r["dual_res_rel"] <= 1e-6 and r["rel_gap"] <= 1e-6
    # both solves at relative KKT 1e-6: each objective within ~2e-6 of p*
    # (the gap test bounds |p - d| by 1e-6 (|p| + |d|)), so 4e-6 apart at most
    assert r["primal_obj"] == pytest.approx(ro["primal_obj"], rel=4e-6)


def test_polished_solve():
    say("feasibility polishing")
    lp = lpgen.planted_uniform(600, 1200, 8, seed=31)
    prob = pd.Problem(lp)
    r = prob.solve(gpu_params(eps_feas=1e-8, eps_gap=1e-2, polish=1, max_iters=50000))
    ro = oracle.Solver(lp, orc_params(eps_feas=1e-8, eps_gap=1e-2, polish=True, max_iters=50000)).solve()
    assert r["status_name"] == "OPTIMAL" and r["polished"] == 1
    assert r["primal_res_rel"] <= 1e-8 and r["dual_res_rel"] <= 1e-8 and r["rel_gap"] <= 1e-2
    assert r["polish_attempts"] == ro["polish_attempts"]
    assert abs(lp.c @ r["x"] - lp.p_star) <= 2e-2 * abs(lp.p_star)


def test_status_limits():
    say("iteration and time limits")
    lp = lpgen.small_lp()
    prob = pd.Problem(lp)
    r = prob.solve(gpu_params(max_iters=10))
    assert r["status_name"] == "ITERATION_LIMIT" and r["iterations"] == 10
    r = prob.solve(gpu_params(time_limit=0.0))
    assert r["status_name"] == "TIME_LIMIT" and r["iterations"] == 0


# ------------------------------------------------------------------ edge cases

def test_edge_cases_empty_rows_free_rows_and_no_rows():
    say("edge cases")
    rng = np.random.default_rng(4)
    # a few empty rows, an empty column, one free row, ragged sizes
    dense = np.round(rng.standard_normal((37, 301)) * (rng.random((37, 301)) < 0.05), 3)
    dense[5] = 0.0
    dense[:, 10] = 0.0
    lp = make_lp(dense)
    x0 = rng.uniform(0, 1, size=301)
    b = dense @ x0
    lp.lc = b - 0.1; lp.uc = b + 0.1
    lp.lc[7], lp.uc[7] = -np.inf, np.inf
    lp.lc[5], lp.uc[5] = 0.0, 0.0
    lp.c = rng.standard_normal(301); lp.lv = np.zeros(301); lp.uv = np.ones(301)
    prob = pd.Problem(lp)
    r = prob.solve(gpu_params(eps_feas=1e-7, eps_gap=1e-7, max_iters=200000))
    ro = oracle.Solver(lp, orc_params(eps_feas=1e-7, eps_gap=1e-7, max_iters=200000)).solve()
    assert r["status_name"] == ro["status_name"] == "OPTIMAL"
    assert r["primal_obj"] == pytest.approx(ro["primal_obj"], rel=1e-6, abs=1e-6)
    # m = 0: min c^T x over a box
    lp0 = lpgen.LP(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0),
                   np.array([1.0, -2.0, 0.0, 3.0, -1.0]), np.zeros(0), np.zeros(0),
                   -np.ones(5), 2 * np.ones(5))
    r0 = pd.Problem(lp0).solve(gpu_params())
    assert r0["status_name"] == "OPTIMAL"
    assert r0["primal_obj"] == pytest.approx(-1 - 4 + 0 - 3 - 2, rel=1e-9)


def test_internal_reordering_is_invisible():
    say("reorder on/off")
    lp = lpgen.planted_skewed(8000, 10000, seed=21, n_dense=20)
    outs = []
    for reorder in (0, 1):
        prob = pd.Problem(lp, gpu_params(reorder=reorder))
        g = prob.scaled()
        st = prob.state(gpu_params(reorder=reorder))
        st.iterate(130)
        outs.append((g, st.get(), prob.solve(gpu_params(reorder=reorder, eps_feas=1e-4,
                                                         eps_gap=1e-4, max_iters=3000))))
    (g0, s0, r0), (g1, s1, r1) = outs
    for k in ("d1", "d2", "val", "c", "lc", "uc", "lv", "uv"):
        assert np.array_equal(g0[k], g1[k]), k
    # the labels change only the order in which the step norms' partial sums
    # combine; such rounding differences grow along the trajectory (the
    # single path against the oracle: 2e-9 at k = 64, 2e-7 at 150)
    for k in ("x", "y", "x0", "y0"):
        assert rel(s0[k], s1[k]) <= 1e-8, k
    # long runs may end at different points of a non-unique optimal face:
    # compare what is unique
    assert r0["status"] == r1["status"]
    if r0["status_name"] == "OPTIMAL":
        assert r0["primal_obj"] == pytest.approx(r1["primal_obj"], rel=3e-4)
        for r in (r0, r1):
            assert r["primal_res_rel"] <= 1e-4 and r["dual_res_rel"] <= 1e-4 and r["rel_gap"] <= 1e-4


# --------------------------------------------------------- failure statuses

@pytest.mark.parametrize("kind", ["objective", "bound"])
def test_overflow_ends_with_numerical_error(kind):
    """Section 3, "Periodic checks": a step whose squared norms overflow ends
    the solve with NUMERICAL_ERROR, as in the oracle (same LPs as its pin),
    with a finite returned point."""
    from tests.test_oracle_pins import overflow_lp
    say(f"numerical error ({kind})")
    lp = overflow_lp(kind)
    r = pd.Problem(lp).solve(gpu_params(max_iters=500))
    ro = oracle.Solver(lp, orc_params(max_iters=500)).solve()
    assert r["status_name"] == ro["status_name"] == "NUMERICAL_ERROR"
    assert r["iterations"] == ro["iterations"] == 0
    assert np.all(np.isfinite(r["x"])) and np.all(np.isfinite(r["y"]))


def test_out_of_memory_is_reported():
    """A device allocation the GPU cannot hold (1 TiB of staging for the rate
    measurement) is refused with OUT_OF_MEMORY, and the library keeps working."""
    say("out of memory")
    with pytest.raises(pd.PdlpError) as ei:
        pd.pdlp_measure_device_rates(1 << 40, 1000)
    assert ei.value.code == pd.PDLP_ERR_OUT_OF_MEMORY
    r = pd.Problem(lpgen.small_lp()).solve(gpu_params(max_iters=64))
    assert r["status_name"] == "ITERATION_LIMIT" and r["iterations"] == 64
