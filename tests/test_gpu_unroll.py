"""GPU parity of the differentiable unrolled map (pdlp_unroll_*).

The forward pass must make the oracle's decisions (step sizes, primal
weights, restarts) and reach its x_K; the replay must reproduce the forward
pass bitwise; gradients must match the oracle's reverse sweep (norm-wise per
block, 1e-7) and central differences of the GPU replay taken with unchanged
projection / dual-case selections.  Checkpointing must not change anything.

Where the checks can hold.  The map with frozen decisions is piecewise
smooth, and its linearization grows with K: on a 2000 x 4000 planted
instance the oracle's own gradient norm is 87 at K = 25, 777 at 100, 3e3 at
200, 6e5 at 300 and 3e10 at 500, and its central differences stop matching
from K ~ 200 (a perturbation of 1e-7 already changes some selection).  The
comparison with the oracle runs at K = 100 and the central differences
(h = 1e-6) at K = 40, on instances whose selections are not decided by
rounding.  Degenerate instances (short rows whose columns all
sit at their bounds, where yhat meets its threshold up to rounding) make the
oracle and the GPU select different branches once the trajectories differ in
the last bits; instances with wave- and workgroup-length rows are compared
at K = 12, before that happens (activity signatures equal).
"""
import numpy as np
import pytest

import lpgen
import oracle
import paper_2501_07018_amd as pd
from tests.test_gpu_parity import rel, say

pytestmark = pytest.mark.gpu

K = 100


def _lps():
    return [
        lpgen.planted_uniform(60, 100, 5, seed=3),
        lpgen.planted_uniform(150, 225, 8, seed=101),
        lpgen.layer_lp(0),
        lpgen.layer_lp(1),
    ]


def _short_k_lps():
    """Wave- and workgroup-length rows, and a tiny LP with free and ranged rows."""
    return [
        lpgen.planted_skewed(1000, 2000, seed=106, mean_degree=4.0, cap=500, n_dense=10,
                             dense_frac=0.3),
        lpgen.planted_skewed(3000, 5000, seed=103, mean_degree=4.0, cap=2500, n_dense=3,
                             dense_frac=0.4),
        lpgen.tiny_random_lp(104, 7, 12),
    ]


def _split(arr, sizes):
    out, o = [], 0
    for s in sizes:
        out.append(arr[o:o + s])
        o += s
    return out


def _compare_with_oracle(lps, u, K_, gx, g, tol):
    sizes = {"c": [lp.n for lp in lps], "lc": [lp.m for lp in lps], "uc": [lp.m for lp in lps],
             "val": [lp.nnz for lp in lps]}
    parts = {k: _split(g[k], sizes[k]) for k in sizes}
    gxs = _split(gx, sizes["c"])
    _, sig = u.replay()
    for i, lp in enumerate(lps):
        o = oracle.Unroll(lp, K_)
        _, so = o.replay()
        assert sig[i] == so, (i, sig[i], so)
        go = o.backward(gxs[i])
        for k in sizes:
            if np.linalg.norm(go[k]) == 0.0:
                assert np.linalg.norm(parts[k][i]) == 0.0, (i, k)
            else:
                assert rel(parts[k][i], go[k]) <= tol, (i, k, rel(parts[k][i], go[k]))


@pytest.fixture(scope="module")
def case():
    lps = _lps()
    u = pd.Unroll(lps)
    x = u.forward(K, 25)
    orc = [oracle.Unroll(lp, K) for lp in lps]
    return lps, u, x, orc


def test_forward_makes_the_oracles_decisions(case):
    say("unroll forward vs oracle")
    lps, u, x, orc = case
    eta, omega, rst = u.tape()
    xs = _split(x, [lp.n for lp in lps])
    for i, (lp, o) in enumerate(zip(lps, orc)):
        assert np.array_equal(rst[i] != 0, o.restart[:K] != 0), i
        # right after a restart the average of one step is the iterate itself
        # (in exact arithmetic), so the candidate choice is a tie there
        t = 0
        for k in range(K):
            t += 1
            if rst[i, k]:
                if t > 1:
                    assert rst[i, k] == o.restart[k], (i, k)
                t = 0
        np.testing.assert_allclose(eta[i], o.eta[:K], rtol=1e-7, err_msg=str(i))
        np.testing.assert_allclose(omega[i], o.omega[:K], rtol=1e-7, err_msg=str(i))
        assert rel(xs[i], o.x) <= 1e-7, i
    assert (rst == 2).any() and (rst == 1).any()


def test_replay_reproduces_the_forward_pass_bitwise(case):
    say("unroll replay")
    lps, u, x, _ = case
    xr, sig = u.replay()
    assert np.array_equal(xr, x)
    assert (sig > 0).all()


K_FD = 40


@pytest.fixture(scope="module")
def fd_case():
    lps = _lps()
    u = pd.Unroll(lps)
    x = u.forward(K_FD, 25)
    gx = np.random.default_rng(17).standard_normal(u.N)
    return lps, u, x, gx, u.backward(gx)


@pytest.fixture(scope="module")
def grads(case):
    lps, u, x, orc = case
    rng = np.random.default_rng(7)
    gx = rng.standard_normal(u.N)
    return gx, u.backward(gx)


def test_gradients_match_the_oracle(case, grads):
    say("unroll gradients vs oracle")
    lps, u, x, orc = case
    gx, g = grads
    _compare_with_oracle(lps, u, K, gx, g, 1e-7)


def _direction(lps, seed):
    """A random data direction (original units) over every part, zero on infinite bounds."""
    rng = np.random.default_rng(seed)
    cat = lambda k: np.concatenate([np.asarray(getattr(lp, k), dtype=np.float64) for lp in lps])
    lc, uc = cat("lc"), cat("uc")
    return {"dc": rng.standard_normal(cat("c").size),
            "dlc": np.where(np.isfinite(lc), rng.standard_normal(lc.size), 0.0),
            "duc": np.where(np.isfinite(uc), rng.standard_normal(uc.size), 0.0),
            "dval": rng.standard_normal(cat("val").size)}


def test_tangent_matches_the_oracle(case):
    """The GPU tangent-linear replay against the oracle's (each along its own
    recorded decisions) at K = 100, 1e-7 norm-wise per instance, as the
    gradients."""
    say("unroll tangent vs oracle")
    lps, u, x, orc = case
    d = _direction(lps, 23)
    dx = u.tangent(**d)
    dxs = _split(dx, [lp.n for lp in lps])
    parts = {k: _split(d[k], [lp.n if k == "dc" else (lp.nnz if k == "dval" else lp.m)
                              for lp in lps]) for k in d}
    for i, o in enumerate(orc):
        dxo = o.tangent(**{k: parts[k][i] for k in parts})
        assert rel(dxs[i], dxo) <= 1e-7, (i, rel(dxs[i], dxo))


def test_tangent_and_adjoint_pass_the_dot_product_test(case, grads):
    """<J v, w> = <v, J^T w> between the GPU's two modes at K = 100."""
    say("unroll dot-product test (K = 100)")
    lps, u, x, orc = case
    gx, g = grads
    d = _direction(lps, 29)
    lhs = gx @ u.tangent(**d)
    rhs = g["c"] @ d["dc"] + g["lc"] @ d["dlc"] + g["uc"] @ d["duc"] + g["val"] @ d["dval"]
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs), (lhs, rhs)


def test_tangent_matches_central_differences(fd_case):
    """GPU tangent against central differences of the GPU replay along a
    direction on the small instances (h = 1e-6 relative, selections
    unchanged), K = 40, 1e-6 norm-wise."""
    say("unroll tangent vs central differences")
    lps, u, x, gx, g = fd_case
    small = [0, 1]
    names = {"dc": "c", "dlc": "lc", "duc": "uc", "dval": "val"}
    base = {k: np.concatenate([np.asarray(getattr(lp, v), dtype=np.float64) for lp in lps])
            for k, v in names.items()}
    rng = np.random.default_rng(31)
    d = {}
    for k, v in names.items():
        off = _offsets(lps, v)
        keep = np.zeros(base[k].size, dtype=bool)
        for i in small:
            keep[off[i]:off[i + 1]] = True
        keep &= np.isfinite(base[k]) & _free_to_move(lps, v)
        mag = np.abs(np.where(keep, base[k], 0.0)).clip(1e-3)
        d[k] = np.where(keep, rng.standard_normal(base[k].size) * mag, 0.0)
    _, sig0 = u.replay()
    h = 1e-6
    try:
        u.set_data(**{names[k]: base[k] + h * d[k] for k in d})
        xp, sp = u.replay()
        u.set_data(**{names[k]: base[k] - h * d[k] for k in d})
        xm, sm = u.replay()
    finally:
        u.set_data(**{names[k]: base[k] for k in d})
    assert np.array_equal(sp, sig0) and np.array_equal(sm, sig0)
    fd = (xp - xm) / (2 * h)
    dx = u.tangent(**d)
    n_small = sum(lps[i].n for i in small)
    assert rel(dx[:n_small], fd[:n_small]) <= 1e-6, rel(dx[:n_small], fd[:n_small])
    assert not dx[n_small:].any()  # the direction is zero on the other instances


def test_long_rows_and_ranged_rows_match_the_oracle():
    say("unroll wave / workgroup rows, free and ranged rows vs oracle")
    lps = _short_k_lps()
    u = pd.Unroll(lps)
    u.forward(4, 3)
    gx = np.random.default_rng(5).standard_normal(u.N)
    _compare_with_oracle(lps, u, 4, gx, u.backward(gx), 1e-9)


def _free_to_move(lps, name):
    """Entries that may be perturbed: row bounds of equality rows stay tied."""
    if name not in ("lc", "uc"):
        return np.ones(sum(getattr(lp, "nnz" if name == "val" else "n") for lp in lps), bool)
    lc = np.concatenate([lp.lc for lp in lps])
    uc = np.concatenate([lp.uc for lp in lps])
    return lc < uc


def _offsets(lps, name):
    size = {"c": "n", "lc": "m", "uc": "m", "val": "nnz"}[name]
    return np.concatenate([[0], np.cumsum([getattr(lp, size) for lp in lps])])


@pytest.mark.parametrize("name", ["c", "lc", "uc", "val"])
def test_directional_central_differences(fd_case, name):
    """Small instances: a random direction over all of their data (step 1e-6
    relative), selections unchanged, 1e-7 relative, at K = 40.  (At K = 100
    the rounding of <gx, x_K> divided by h already reaches ~1e-6 at this
    step: the map's conditioning, see the module notes.)"""
    say(f"unroll directional differences {name}")
    lps, u, x, gx, g = fd_case
    small = [0, 1]
    base = np.concatenate([np.asarray(getattr(lp, name), dtype=np.float64) for lp in lps])
    off = _offsets(lps, name)
    keep = np.zeros(base.size, dtype=bool)
    for i in small:
        keep[off[i]:off[i + 1]] = True
    keep &= _free_to_move(lps, name)
    fin = np.isfinite(base) & keep
    rng = np.random.default_rng(11)
    mag = np.where(fin, np.abs(np.where(fin, base, 0.0)), 0.0).clip(1e-3)
    _, sig0 = u.replay()
    h = 1e-6
    try:
        for trial in range(2):
            d = np.where(fin, rng.standard_normal(base.size) * mag, 0.0)
            u.set_data(**{name: base + h * d})
            xp, sp = u.replay()
            u.set_data(**{name: base - h * d})
            xm, sm = u.replay()
            assert np.array_equal(sp, sig0) and np.array_equal(sm, sig0)
            fd = (gx @ xp - gx @ xm) / (2 * h)
            an = g[name] @ d
            assert abs(fd - an) <= 1e-7 * abs(an), (name, trial, fd, an)
    finally:
        u.set_data(**{name: base})
    xr, _ = u.replay()
    assert np.array_equal(xr, x)


@pytest.mark.parametrize("name", ["c", "lc", "uc", "val"])
def test_sampled_coordinate_central_differences(fd_case, name):
    """2000 x 4000 instances at K = 40: single coordinates, h = 1e-6 relative
    (to the entry, or to the block's median magnitude for entries near 0),
    selections of the instance unchanged.  The floor of a central difference
    is the rounding of <gx, x_K> divided by h, so the error is bounded
    relative to the block's largest derivative (1e-7)."""
    say(f"unroll sampled-coordinate differences {name}")
    lps, u, x, gx, g = fd_case
    base = np.concatenate([np.asarray(getattr(lp, name), dtype=np.float64) for lp in lps])
    off = _offsets(lps, name)
    rng = np.random.default_rng(13)
    _, sig0 = u.replay()
    try:
        movable = _free_to_move(lps, name)
        for i in (2, 3):
            blk = np.arange(off[i], off[i + 1])
            blk = blk[np.isfinite(base[blk]) & movable[blk]]
            scale = np.max(np.abs(g[name][off[i]:off[i + 1]]))
            typ = np.median(np.abs(base[blk]))  # step floor for entries near 0
            for j in rng.choice(blk, 3, replace=False):
                h = 1e-6 * max(abs(base[j]), typ)
                bp = base.copy()
                bp[j] += h
                u.set_data(**{name: bp})
                xp, sp = u.replay()
                bp[j] -= 2 * h
                u.set_data(**{name: bp})
                xm, sm = u.replay()
                assert sp[i] == sig0[i] and sm[i] == sig0[i], (i, j)
                fd = (gx @ xp - gx @ xm) / (2 * h)
                assert abs(fd - g[name][j]) <= 1e-7 * scale, (i, j, fd, g[name][j], scale)
    finally:
        u.set_data(**{name: base})


def test_checkpoint_cadence_does_not_change_anything(case, grads):
    say("unroll checkpoint cadence")
    lps, u, x, _ = case
    gx, g = grads
    v = pd.Unroll(lps)
    for ck in (7, 100):
        x2 = v.forward(K, ck)
        assert np.array_equal(x2, x)
        g2 = v.backward(gx)
        for k in g:
            assert np.array_equal(g2[k], g[k]), (ck, k)


def test_zero_steps_and_linearity_in_the_upstream_gradient(case, grads):
    say("unroll K=0 / linearity")
    lps, u, x, _ = case
    gx, g = grads
    g2 = u.backward(2.0 * gx)
    for k in g:
        assert np.array_equal(g2[k], 2.0 * g[k]), k
    v = pd.Unroll(lps[:2])
    x0 = v.forward(0, 25)
    lv = np.concatenate([lp.lv for lp in lps[:2]])
    uv = np.concatenate([lp.uv for lp in lps[:2]])
    np.testing.assert_array_equal(x0, np.clip(0.0, lv, uv))
    g0 = v.backward(np.ones(v.N))
    assert all(not g0[k].any() for k in g0)


def test_autograd_function_wraps_the_same_map(case):
    say("unroll autograd.Function")
    torch = pytest.importorskip("torch")
    from paper_2501_07018_amd.layer import LPLayer
    lps = _lps()[:2]
    layer = LPLayer(lps, K=60, ckpt=25)
    cat = lambda k: torch.tensor(np.concatenate([np.asarray(getattr(lp, k), dtype=np.float64)
                                                 for lp in lps]), requires_grad=True)
    c, lc, uc, val = cat("c"), cat("lc"), cat("uc"), cat("val")
    x = layer(c, lc, uc, val)
    gx = torch.randn(x.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    (x * gx).sum().backward()
    ref = pd.Unroll(lps)
    xr = ref.forward(60, 25)
    gr = ref.backward(gx.numpy())
    assert np.array_equal(x.detach().numpy(), xr)
    for t, k in ((c, "c"), (lc, "lc"), (uc, "uc"), (val, "val")):
        assert np.array_equal(t.grad.numpy(), gr[k]), k
