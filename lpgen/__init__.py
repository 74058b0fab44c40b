"""Seeded synthetic LP generators.

These produce the inputs that both the FP64 CPU oracle and the GPU solver
consume.  They hold none of the solver's arithmetic: they only draw random
structure and values and assemble CSR arrays.  Planted instances also carry
an optimal primal/dual pair (x*, y*, r*) that satisfies the KKT conditions of
the LP form

    min c^T x   s.t.   lc <= A x <= uc,   lv <= x <= uv

(dual: max -p(-y; lc, uc) - p(-r; lv, uv) s.t. c - A^T y = r, y in Y, r in R),
so that an exact optimal objective is known.

Workload recipes (sizes, degree laws, value laws) are synthetic stand-ins for
the paper's large-scale instances, which are not available here:

* ``planted_uniform`` -- random sparse LP, k distinct uniform rows per column,
  N(0,1) values, planted optimum (1,000 x 2,000 with 10 per column is the
  small parity workload; 2,000 x 4,000 and the batch of uneven sizes reuse it).
* ``planted_skewed`` -- power-law column degrees capped at 10,000 with mean 5,
  5% of nonzeros falling into 5,000 "dense" rows (about 1,250 nonzeros each),
  planted optimum (20M x 25M, ~125M nonzeros at full size).
* ``multicommodity_grid`` -- multicommodity flow on an L x L grid with shared
  arc capacities (300 x 300 grid, 8 commodities at full size).

RNG: numpy's PCG64 ``Generator`` seeded with ``(config << 32) | instance``.
"""
from __future__ import annotations

import dataclasses
import math
import sys

import numpy as np
import scipy.sparse as sp

INF = np.inf

# config ids used to derive seeds
CFG_SMALL, CFG_GRID, CFG_SKEWED, CFG_BATCH, CFG_LAYER, CFG_INFEAS = 0, 1, 2, 3, 4, 5


def seed_of(config: int, instance: int = 0) -> int:
    return (int(config) << 32) | int(instance)


@dataclasses.dataclass
class LP:
    """CSR LP instance (int32 indices, float64 values)."""
    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col: np.ndarray      # int32 [nnz], strictly increasing within a row
    val: np.ndarray      # float64 [nnz]
    c: np.ndarray        # [n]
    lc: np.ndarray       # [m], -inf allowed
    uc: np.ndarray       # [m], +inf allowed
    lv: np.ndarray       # [n]
    uv: np.ndarray       # [n]
    obj_offset: float = 0.0
    # planted optimum (None when not planted)
    x_star: np.ndarray | None = None
    y_star: np.ndarray | None = None
    r_star: np.ndarray | None = None
    p_star: float | None = None
    name: str = ""
    # planted infeasibility rays (None when not planted)
    ray_y: np.ndarray | None = None   # Farkas ray of a primal-infeasible instance
    ray_r: np.ndarray | None = None
    ray_x: np.ndarray | None = None   # recession ray of a dual-infeasible instance
    x_feas: np.ndarray | None = None  # a primal feasible point
    y_feas: np.ndarray | None = None  # a dual feasible pair (c - A^T y = r, y in Y, r in R)
    r_feas: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.n))

    def stats(self) -> dict:
        rl = np.diff(self.row_ptr)
        cl = np.bincount(self.col, minlength=self.n) if self.nnz else np.zeros(self.n, np.int64)
        return {
            "m": self.m, "n": self.n, "nnz": self.nnz,
            "max_row": int(rl.max()) if self.m else 0,
            "max_col": int(cl.max()) if self.n else 0,
            "empty_rows": int((rl == 0).sum()),
            "empty_cols": int((cl == 0).sum()),
        }


def _csr_from_csc(m, n, colptr, rowidx, vals):
    """CSC (rows sorted within each column) -> CSR with sorted columns."""
    a = sp.csc_matrix((vals, rowidx, colptr), shape=(m, n))
    a = a.tocsr()
    a.sort_indices()
    return (a.indptr.astype(np.int32), a.indices.astype(np.int32),
            np.ascontiguousarray(a.data, dtype=np.float64))


def _distinct_rows_fixed_degree(rng, m, n, k):
    """n columns, each with k distinct rows drawn uniformly from range(m).

    Returns (colptr, rows) with rows sorted within each column.
    """
    if k > m:
        raise ValueError("degree larger than the number of rows")
    rows = rng.integers(0, m, size=(n, k), dtype=np.int64)
    rows.sort(axis=1)
    while True:
        dup = np.zeros_like(rows, dtype=bool)
        dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        rows[dup] = rng.integers(0, m, size=nd, dtype=np.int64)
        rows.sort(axis=1)
    colptr = np.arange(0, (n + 1) * k, k, dtype=np.int64)
    return colptr, rows.reshape(-1)


def _plant(rng, A: sp.csr_matrix, m, n, frac_fixed=0.30):
    """Plant an optimal (x*, y*, r*) and derive bounds and c (see module doc).

    Columns: x* ~ U[0,1], exactly ``frac_fixed`` of them (by permutation) set
    to 0 or 1 with probability 1/2; all variables boxed in [0, 1].
    Rows (by permutation): half equalities lc = uc = (A x*)_i; a quarter active
    one-sided rows (bound equal to (A x*)_i); a quarter inactive one-sided rows
    with slack U[0.1, 1]; each one-sided row is >= or <= with probability 1/2.
    y*: equalities N(0,1); active >= rows +|N|; active <= rows -|N|; else 0.
    r*: +|N| at x*=0, -|N| at x*=1, 0 for interior variables.
    c = A^T y* + r*.
    """
    x = rng.random(n)
    perm = rng.permutation(n)
    nfix = int(round(frac_fixed * n))
    fixed = perm[:nfix]
    at_one = rng.random(nfix) < 0.5
    x[fixed] = np.where(at_one, 1.0, 0.0)
    ax = A @ x

    rperm = rng.permutation(m)
    n_eq = m // 2
    n_act = (m - n_eq) // 2
    eq_rows = rperm[:n_eq]
    act_rows = rperm[n_eq:n_eq + n_act]
    ina_rows = rperm[n_eq + n_act:]
    ge_dir = rng.random(m) < 0.5  # one-sided direction: True means >=

    lc = np.full(m, -INF)
    uc = np.full(m, INF)
    y = np.zeros(m)
    lc[eq_rows] = ax[eq_rows]
    uc[eq_rows] = ax[eq_rows]
    y[eq_rows] = rng.standard_normal(n_eq)

    g = ge_dir[act_rows]
    mag = np.abs(rng.standard_normal(n_act))
    lc[act_rows[g]] = ax[act_rows[g]]
    uc[act_rows[~g]] = ax[act_rows[~g]]
    y[act_rows[g]] = mag[g]
    y[act_rows[~g]] = -mag[~g]

    g = ge_dir[ina_rows]
    slack = rng.uniform(0.1, 1.0, size=ina_rows.size)
    lc[ina_rows[g]] = ax[ina_rows[g]] - slack[g]
    uc[ina_rows[~g]] = ax[ina_rows[~g]] + slack[~g]

    r = np.zeros(n)
    rmag = np.abs(rng.standard_normal(n))
    r[x == 0.0] = rmag[x == 0.0]
    r[x == 1.0] = -rmag[x == 1.0]
    c = A.T @ y + r
    lv = np.zeros(n)
    uv = np.ones(n)
    p_star = math.fsum(c * x)  # exactly rounded sum
    return x, y, r, c, lc, uc, lv, uv, p_star


def planted_uniform(m: int, n: int, per_col: int, seed: int, name: str = "") -> LP:
    """Planted LP with ``per_col`` distinct uniform rows per column, N(0,1) values."""
    rng = np.random.default_rng(seed)
    colptr, rows = _distinct_rows_fixed_degree(rng, m, n, per_col)
    vals = rng.standard_normal(rows.size)
    row_ptr, col, val = _csr_from_csc(m, n, colptr, rows, vals)
    A = sp.csr_matrix((val, col, row_ptr), shape=(m, n))
    x, y, r, c, lc, uc, lv, uv, p = _plant(rng, A, m, n)
    return LP(m, n, row_ptr, col, val, c, lc, uc, lv, uv, 0.0, x, y, r, p,
              name or f"planted_uniform_{m}x{n}_k{per_col}")


def powerlaw_exponent(mean: float, cap: int) -> float:
    """Exponent a of pmf ~ k^-a on {1..cap} whose mean equals ``mean``."""
    k = np.arange(1, cap + 1, dtype=np.float64)
    lo, hi = 1.0001, 6.0
    for _ in range(200):
        a = 0.5 * (lo + hi)
        p = k ** (-a)
        mu = float((p * k).sum() / p.sum())
        if mu > mean:
            lo = a
        else:
            hi = a
    return 0.5 * (lo + hi)


def planted_skewed(m: int, n: int, seed: int, mean_degree: float = 5.0,
                   cap: int = 10_000, n_dense: int = 5_000, dense_frac: float = 0.05,
                   name: str = "", verbose: bool = False) -> LP:
    """Planted LP with power-law column degrees and a block of dense rows.

    Column degrees follow pmf ~ k^-a on {1..cap} with a chosen so the mean is
    ``mean_degree``; each nonzero's row is, with probability ``dense_frac``,
    uniform over a fixed set of ``n_dense`` rows, else uniform over all rows.
    Duplicate (row, column) draws are merged by dropping repeats, so the
    realized nnz is slightly below n*mean_degree.  Values are N(0,1).
    """
    import time
    t0 = time.time()
    rng = np.random.default_rng(seed)
    cap = min(cap, m)
    a = powerlaw_exponent(mean_degree, cap)
    k = np.arange(1, cap + 1, dtype=np.float64)
    pmf = k ** (-a)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    deg = np.searchsorted(cdf, rng.random(n), side="right").astype(np.int64) + 1
    np.minimum(deg, cap, out=deg)
    nnz0 = int(deg.sum())
    n_dense = min(n_dense, m)
    dense_set = rng.choice(m, size=n_dense, replace=False).astype(np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), deg)
    is_dense = rng.random(nnz0) < dense_frac
    rows = rng.integers(0, m, size=nnz0, dtype=np.int64)
    nd = int(is_dense.sum())
    rows[is_dense] = dense_set[rng.integers(0, n_dense, size=nd)]
    del is_dense
    if verbose:
        print(f"[lpgen] skewed: degrees drawn, nnz0={nnz0} ({time.time()-t0:.1f}s)", file=sys.stderr, flush=True)
    key = cols * np.int64(m) + rows
    del rows, cols
    key.sort()
    keep = np.empty(key.size, dtype=bool)
    keep[0] = True
    np.not_equal(key[1:], key[:-1], out=keep[1:])
    key = key[keep]
    del keep
    cols = (key // m).astype(np.int32)
    rows = (key - cols.astype(np.int64) * m).astype(np.int32)
    del key
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=n), out=colptr[1:])
    del cols
    if verbose:
        print(f"[lpgen] skewed: sorted/deduplicated, nnz={rows.size} ({time.time()-t0:.1f}s)", file=sys.stderr, flush=True)
    vals = rng.standard_normal(rows.size)
    row_ptr, col, val = _csr_from_csc(m, n, colptr, rows, vals)
    del rows, vals, colptr
    A = sp.csr_matrix((val, col, row_ptr), shape=(m, n))
    x, y, r, c, lc, uc, lv, uv, p = _plant(rng, A, m, n)
    if verbose:
        print(f"[lpgen] skewed: planted ({time.time()-t0:.1f}s)", file=sys.stderr, flush=True)
    return LP(m, n, row_ptr, col, val, c, lc, uc, lv, uv, 0.0, x, y, r, p,
              name or f"planted_skewed_{m}x{n}")


def multicommodity_grid(L: int, n_comm: int, pairs: int, seed: int,
                        name: str = "") -> LP:
    """Multicommodity flow on an L x L grid with bidirectional arcs.

    Variables f[k, a] >= 0 (no upper bound), cost U[1,10] per arc shared by
    all commodities.  Rows: one conservation equality per (commodity, node):
    out-flow minus in-flow equals supply; then one capacity row per arc:
    sum_k f[k, a] <= cap_a with cap_a ~ U[20, 60].  Each commodity has
    ``pairs`` (source, sink) pairs of distinct nodes with demand U[1, 10].
    Variable index k*num_arcs + a; row index k*num_nodes + v, then
    n_comm*num_nodes + a for capacities.  Not planted.
    """
    rng = np.random.default_rng(seed)
    V = L * L
    idx = np.arange(V).reshape(L, L)
    h_u = idx[:, :-1].ravel(); h_v = idx[:, 1:].ravel()
    v_u = idx[:-1, :].ravel(); v_v = idx[1:, :].ravel()
    eu = np.concatenate([h_u, v_u]); ev = np.concatenate([h_v, v_v])
    tail = np.concatenate([eu, ev]).astype(np.int64)
    head = np.concatenate([ev, eu]).astype(np.int64)
    E = tail.size
    cost = rng.uniform(1.0, 10.0, size=E)
    cap = rng.uniform(20.0, 60.0, size=E)
    supply = np.zeros((n_comm, V))
    for k in range(n_comm):
        for _ in range(pairs):
            s, t = rng.choice(V, size=2, replace=False)
            d = rng.uniform(1.0, 10.0)
            supply[k, s] += d
            supply[k, t] -= d
    m = n_comm * V + E
    n = n_comm * E
    # CSC assembly: column (k, a) has +1 at row k*V+tail, -1 at row k*V+head,
    # +1 at capacity row n_comm*V + a.
    kk = np.repeat(np.arange(n_comm, dtype=np.int64), E)
    aa = np.tile(np.arange(E, dtype=np.int64), n_comm)
    r_tail = kk * V + tail[aa]
    r_head = kk * V + head[aa]
    r_cap = n_comm * V + aa
    rows = np.stack([r_tail, r_head, r_cap], axis=1)
    vals = np.stack([np.ones(n), -np.ones(n), np.ones(n)], axis=1)
    order = np.argsort(rows, axis=1)
    rows = np.take_along_axis(rows, order, axis=1).reshape(-1)
    vals = np.take_along_axis(vals, order, axis=1).reshape(-1)
    colptr = np.arange(0, 3 * n + 1, 3, dtype=np.int64)
    row_ptr, col, val = _csr_from_csc(m, n, colptr, rows, vals)
    lc = np.concatenate([supply.reshape(-1), np.full(E, -INF)])
    uc = np.concatenate([supply.reshape(-1), cap])
    c = np.tile(cost, n_comm)
    lv = np.zeros(n)
    uv = np.full(n, INF)
    return LP(m, n, row_ptr, col, val, c, lc, uc, lv, uv, 0.0,
              name=name or f"multicommodity_grid_{L}x{L}_k{n_comm}")


# ---------------------------------------------------------------- configs

def small_lp(instance: int = 0) -> LP:
    """1,000 x 2,000, 10 uniform rows per column, planted (parity workload)."""
    return planted_uniform(1000, 2000, 10, seed_of(CFG_SMALL, instance), "small_1000x2000")


def grid_flow_lp(L: int = 300, n_comm: int = 8, pairs: int = 20, instance: int = 0) -> LP:
    return multicommodity_grid(L, n_comm, pairs, seed_of(CFG_GRID, instance))


def skewed_lp(m: int = 20_000_000, n: int = 25_000_000, instance: int = 0,
              verbose: bool = False, **kw) -> LP:
    return planted_skewed(m, n, seed_of(CFG_SKEWED, instance), verbose=verbose, **kw)


def batch_sizes(count: int = 1024, lo: int = 200, hi: int = 20_000, seed: int | None = None):
    rng = np.random.default_rng(seed_of(CFG_BATCH, 0xFFFFFFFF) if seed is None else seed)
    ms = rng.integers(lo, hi + 1, size=count)
    return [(int(m_), int(1.5 * m_)) for m_ in ms]


def batch_lp(i: int, m: int, n: int, per_col: int = 8) -> LP:
    return planted_uniform(m, n, per_col, seed_of(CFG_BATCH, i), f"batch_{i}_{m}x{n}")


def layer_lp(i: int, m: int = 2000, n: int = 4000, per_col: int = 10) -> LP:
    return planted_uniform(m, n, per_col, seed_of(CFG_LAYER, i), f"layer_{i}_{m}x{n}")


def tiny_random_lp(seed: int, m: int, n: int, density: float = 0.6,
                   box: float = 2.0, kinds=("eq", "ge", "le", "range", "free")) -> LP:
    """Tiny dense-ish LP with a finite variable box, for brute-force checks.

    Row kinds are drawn from ``kinds``: equality, >=, <=, two-sided range, or
    free (both bounds infinite).  Right-hand sides are placed around A x0 for
    a random x0 inside the box so the LP is feasible.
    """
    rng = np.random.default_rng(seed)
    dense = rng.standard_normal((m, n))
    mask = rng.random((m, n)) < density
    for i in range(m):
        if not mask[i].any():
            mask[i, rng.integers(n)] = True
    dense = np.where(mask, np.round(dense * 4) / 4, 0.0)
    dense[mask & (dense == 0.0)] = 0.5
    A = sp.csr_matrix(dense)
    A.sort_indices()
    x0 = rng.uniform(-box * 0.5, box * 0.5, size=n)
    ax = dense @ x0
    lc = np.full(m, -INF); uc = np.full(m, INF)
    for i in range(m):
        kind = kinds[rng.integers(len(kinds))]
        s = rng.uniform(0.1, 1.0)
        if kind == "eq":
            lc[i] = uc[i] = ax[i]
        elif kind == "ge":
            lc[i] = ax[i] - s
        elif kind == "le":
            uc[i] = ax[i] + s
        elif kind == "range":
            lc[i] = ax[i] - s; uc[i] = ax[i] + rng.uniform(0.1, 1.0)
    lv = np.full(n, -box); uv = np.full(n, box)
    c = np.round(rng.standard_normal(n) * 4) / 4
    return LP(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
              A.data.astype(np.float64), c, lc, uc, lv, uv, 0.0, name=f"tiny_{seed}")


# ------------------------------------------------------- infeasible instances
#
# Both generators start from a random point x0 and bounds placed around it,
# so that the constraints without the planted conflict are satisfiable, and
# mix every bound kind: variables boxed, lower-bounded, upper-bounded or free;
# rows equalities, >=, <=, two-sided ranges or free.


def _ray_matrix(rng, m, n, per_col):
    colptr, rows = _distinct_rows_fixed_degree(rng, m, n, per_col)
    vals = rng.standard_normal(rows.size)
    row_ptr, col, val = _csr_from_csc(m, n, colptr, rows, vals)
    return row_ptr, col, val, sp.csr_matrix((val, col, row_ptr), shape=(m, n))


def _var_bounds(rng, x0, kind):
    """kind: 0 boxed, 1 lower only, 2 upper only, 3 free."""
    n = x0.size
    a = rng.uniform(0.2, 1.0, n)
    b = rng.uniform(0.2, 1.0, n)
    lv = np.where((kind == 0) | (kind == 1), x0 - a, -INF)
    uv = np.where((kind == 0) | (kind == 2), x0 + b, INF)
    return lv, uv


def _row_bounds(rng, ax0, kind):
    """kind: 0 equality, 1 >=, 2 <=, 3 range, 4 free."""
    m = ax0.size
    s1 = rng.uniform(0.1, 1.0, m)
    s2 = rng.uniform(0.1, 1.0, m)
    lc = np.full(m, -INF)
    uc = np.full(m, INF)
    lc = np.where(kind == 0, ax0, lc)
    uc = np.where(kind == 0, ax0, uc)
    lc = np.where((kind == 1) | (kind == 3), ax0 - s1, lc)
    uc = np.where((kind == 2) | (kind == 3), ax0 + s2, uc)
    return lc, uc


def planted_primal_infeasible(m: int, n: int, per_col: int, seed: int, support: float = 0.1,
                              margin: float = 1.0, boxed: bool = False, name: str = "") -> LP:
    """Primal-infeasible LP with a planted Farkas ray (y*, r*).

    y* lives on about ``support * m`` rows with the sign each row kind allows
    (free rows excluded); r* = -A^T y*, and every column it touches gets a
    bound kind that admits that sign (boxed, or one-sided on the matching
    side).  The bounds of one ray row are then moved until
    lc^T y*+ - uc^T y*- + lv^T r*+ - uv^T r*- equals ``margin`` > 0, which
    makes the constraint system inconsistent (Farkas' lemma) while every
    other row keeps its slack around x0.  The objective is c = A^T y_f + r_f
    for a random (y_f in Y, r_f in R), so the dual is feasible (and, the
    primal being infeasible, unbounded); (y_f, r_f) is kept.  ``boxed``
    makes every variable boxed.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col, val, A = _ray_matrix(rng, m, n, per_col)
    x0 = rng.uniform(-1.0, 1.0, n)
    rkind = rng.choice(5, size=m, p=[0.3, 0.25, 0.25, 0.15, 0.05])
    cand = np.flatnonzero(rkind != 4)
    k = max(1, int(round(support * m)))
    S = rng.choice(cand, size=min(k, cand.size), replace=False)
    y = np.zeros(m)
    mag = np.abs(rng.standard_normal(S.size)) + 0.1
    sgn = np.where(rng.random(S.size) < 0.5, 1.0, -1.0)
    sgn = np.where(rkind[S] == 1, 1.0, np.where(rkind[S] == 2, -1.0, sgn))
    y[S] = sgn * mag
    g = A.T @ y
    r = -g
    vkind = rng.choice(4, size=n, p=[0.6, 0.15, 0.15, 0.1])
    touched = g != 0.0
    side = np.where(r > 0.0, 1, 2)            # lower-only admits r > 0, upper-only r < 0
    pick = rng.random(n) < 0.5
    vkind = np.where(touched, np.where(pick, 0, side), vkind)
    if boxed:
        vkind = np.zeros(n, dtype=vkind.dtype)
    lv, uv = _var_bounds(rng, x0, vkind)
    lc, uc = _row_bounds(rng, A @ x0, rkind)
    r = np.where(touched, r, 0.0)
    yp, yn, rp, rn = y > 0, y < 0, r > 0, r < 0
    obj = (math.fsum(lc[yp] * y[yp]) + math.fsum(uc[yn] * y[yn])
           + math.fsum(lv[rp] * r[rp]) + math.fsum(uv[rn] * r[rn]))
    i0 = S[int(np.argmax(np.abs(y[S])))]
    delta = (margin - obj) / abs(y[i0])        # > 0: obj <= 0 while x0 is feasible
    if y[i0] > 0:
        lc[i0] += delta
        if rkind[i0] == 0 or uc[i0] < lc[i0]:
            uc[i0] = lc[i0]
    else:
        uc[i0] -= delta
        if rkind[i0] == 0 or lc[i0] > uc[i0]:
            lc[i0] = uc[i0]
    yf = rng.standard_normal(m)
    yf = np.where(np.isfinite(lc), yf, np.minimum(yf, 0.0))
    yf = np.where(np.isfinite(uc), yf, np.maximum(yf, 0.0))
    rf = rng.standard_normal(n)
    rf = np.where(np.isfinite(lv), rf, np.minimum(rf, 0.0))
    rf = np.where(np.isfinite(uv), rf, np.maximum(rf, 0.0))
    c = A.T @ yf + rf
    lp = LP(m, n, row_ptr, col, val, c, lc, uc, lv, uv, 0.0,
            name=name or f"primal_infeasible_{m}x{n}_k{per_col}")
    lp.ray_y, lp.ray_r = y, r
    lp.y_feas, lp.r_feas = yf, rf
    return lp


def planted_dual_infeasible(m: int, n: int, per_col: int, seed: int, support: float = 0.1,
                            margin: float = 1.0, name: str = "") -> LP:
    """Feasible but unbounded LP (dual infeasible) with a planted ray x*.

    x* lives on about ``support * n`` columns, each one-sided on the side x*
    moves away from (or free); every row it touches becomes >= or <= in the
    direction A x* moves (or free), so x0 + t x* stays feasible for all
    t >= 0, and c is corrected so that c^T x* = -``margin``.  x0 is kept as
    a feasible point.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col, val, A = _ray_matrix(rng, m, n, per_col)
    x0 = rng.uniform(-1.0, 1.0, n)
    k = max(1, int(round(support * n)))
    J = rng.choice(n, size=k, replace=False)
    x = np.zeros(n)
    x[J] = np.where(rng.random(k) < 0.5, 1.0, -1.0) * rng.uniform(0.5, 1.5, k)
    vkind = rng.choice(4, size=n, p=[0.6, 0.15, 0.15, 0.1])
    free = rng.random(n) < 0.2
    vkind = np.where(x > 0, np.where(free, 3, 1), np.where(x < 0, np.where(free, 3, 2), vkind))
    ax = A @ x
    rkind = rng.choice(5, size=m, p=[0.3, 0.25, 0.25, 0.15, 0.05])
    freer = rng.random(m) < 0.1
    rkind = np.where(ax > 0, np.where(freer, 4, 1), np.where(ax < 0, np.where(freer, 4, 2), rkind))
    lv, uv = _var_bounds(rng, x0, vkind)
    lc, uc = _row_bounds(rng, A @ x0, rkind)
    c = rng.standard_normal(n)
    c -= ((c @ x + margin) / (x @ x)) * x
    lp = LP(m, n, row_ptr, col, val, c, lc, uc, lv, uv, 0.0,
            name=name or f"dual_infeasible_{m}x{n}_k{per_col}")
    lp.ray_x = x
    lp.x_feas = x0
    return lp


def infeasible_lp(kind: str, i: int, m: int, n: int, per_col: int = 4) -> LP:
    """Seeded member ``i`` of the primal- ('primal'), boxed primal- ('primal_boxed') or
    dual- ('dual') infeasible family."""
    seed = seed_of(CFG_INFEAS, 2 * i + (kind == "dual"))
    if kind in ("primal", "primal_boxed"):
        return planted_primal_infeasible(m, n, per_col, seed, boxed=kind == "primal_boxed")
    return planted_dual_infeasible(m, n, per_col, seed)
