"""HIP-graph replay of step attempts against eager launches.

The graphs hold exactly the launches an eager loop makes, so every result
must be bitwise identical with graphs on and off.  The comparisons are made
after every iteration block (each one many graph replays, with the
program's eager checks, restarts and synchronizations in between), on whole
solves with feasibility polishing (whose sub-runs swap the vectors the
graphs were captured for), and on batches whose set of running instances
changes as instances finish.
"""
import numpy as np
import pytest

import lpgen
import paper_2501_07018_amd as pd
from tests.test_gpu_batch import _mixed_batch
from tests.test_gpu_parity import say

pytestmark = pytest.mark.gpu

STATE_KEYS = ("x", "y", "ax", "aty", "x0", "y0", "sx", "sy")


def test_iteration_blocks_bitwise_equal_with_and_without_graphs():
    say("graphs vs eager, iteration blocks")
    lp = lpgen.planted_uniform(700, 1300, 7, seed=17)
    prob = pd.Problem(lp)
    on = prob.state(pd.pdlp_params_default(graphs=1))
    off = prob.state(pd.pdlp_params_default(graphs=0))
    for block in (1, 63, 64, 200, 7, 64, 129):
        a, b = on.iterate(block), off.iterate(block)
        assert a == b
        ga, gb = on.get(), off.get()
        for key in STATE_KEYS:
            assert np.array_equal(ga[key], gb[key]), (block, key)


def test_solve_with_polishing_bitwise_equal():
    say("graphs vs eager, solve with polishing")
    lp = lpgen.small_lp()
    out = []
    for g in (1, 0):
        r = pd.Problem(lp).solve(pd.pdlp_params_default(eps_feas=1e-10, eps_gap=1e-2, polish=1,
                                                        graphs=g))
        out.append(r)
    a, b = out
    assert a["status_name"] == b["status_name"] == "OPTIMAL" and a["polished"] == 1
    for key in ("iterations", "attempts", "polish_iters", "polish_attempts", "kkt_passes"):
        assert a[key] == b[key], key
    for key in ("x", "y", "r"):
        assert np.array_equal(a[key], b[key]), key


def test_batch_bitwise_equal_with_and_without_graphs():
    say("graphs vs eager, batch")
    lps = _mixed_batch()[:6]
    b = pd.Batch(lps)
    prm = dict(eps_feas=1e-7, eps_gap=1e-7, max_iters=5000)
    runs = [b.solve(pd.pdlp_params_default(graphs=g, **prm)) for g in (1, 0, 1)]
    for other in runs[1:]:
        for r0, r1 in zip(runs[0], other):
            assert r0["status_name"] == r1["status_name"]
            for key in ("iterations", "attempts", "kkt_passes", "restarts"):
                assert r0[key] == r1[key], key
            for key in ("x", "y", "r"):
                assert np.array_equal(r0[key], r1[key]), key


def test_stream_block_sizes_leave_products_unchanged():
    """The block partition of the CSR stream products (fixed sizes and the
    autotuner) never splits a stream row, so every product is bitwise the
    same; only the order of the step norms' partial sums may differ."""
    say("stream block sizes")
    lp = lpgen.planted_skewed(3000, 5000, seed=103, mean_degree=4.0, cap=2500, n_dense=3,
                              dense_frac=0.4)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    ref = None
    for sb in (0, 2048, 512, 64):
        prob = pd.Problem(lp, pd.pdlp_params_default(stream_block=sb))
        out = (prob.spmv(x)[0], prob.spmv(y, transpose=True)[0])
        if ref is None:
            ref = out
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), sb
        assert prob.schedule() == {"stream_block": 2048 if sb == 0 else sb, "med_row": 64}
        small = pd.Problem(lpgen.planted_uniform(900, 1350, 8, seed=102),
                           pd.pdlp_params_default(stream_block=sb))
        r = small.solve(pd.pdlp_params_default(eps_feas=1e-6, eps_gap=1e-6, max_iters=100_000))
        assert r["status_name"] == "OPTIMAL", sb
    for bad in (10, 4096, -2):
        with pytest.raises(pd.PdlpError):
            pd.Problem(lp, pd.pdlp_params_default(stream_block=bad))


def test_autotuned_schedules_are_scored_on_steps():
    """stream_block = -1 on a single problem: the schedule (block size, longest
    row of the stream class) is picked by timing the solver's own steps.  It
    is one of the candidates; rows within the stream class of both the
    default and the pick are summed in stored order (bitwise the default
    products), the others by a tree (1e-14 of |A||x|); solves reach their
    tolerance."""
    say("autotuned schedules")
    cands = {(2048, 64), (2048, 32), (2048, 128), (1024, 64), (1024, 32), (512, 64)}
    lp = lpgen.planted_skewed(3000, 5000, seed=103, mean_degree=4.0, cap=2500, n_dense=3,
                              dense_frac=0.4)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    ref = pd.Problem(lp)
    tuned = pd.Problem(lp, pd.pdlp_params_default(stream_block=-1))
    sch = tuned.schedule()
    assert (sch["stream_block"], sch["med_row"]) in cands, sch
    short = min(sch["med_row"], 64)
    rl = np.diff(lp.row_ptr)
    cl = np.bincount(lp.col, minlength=lp.n)
    for (a, b), lens, scale in (
            ((tuned.spmv(x)[0], ref.spmv(x)[0]), rl, np.abs(lp.csr()) @ np.abs(x)),
            ((tuned.spmv(y, transpose=True)[0], ref.spmv(y, transpose=True)[0]), cl,
             np.abs(lp.csr()).T @ np.abs(y))):
        assert np.array_equal(a[lens <= short], b[lens <= short])
        assert np.all(np.abs(a - b) <= 1e-14 * scale + 1e-300)
    lp2 = lpgen.planted_uniform(900, 1350, 8, seed=102)
    prm = pd.pdlp_params_default(stream_block=-1, eps_feas=1e-6, eps_gap=1e-6, max_iters=100_000)
    r = pd.Problem(lp2, prm).solve(prm)
    assert r["status_name"] == "OPTIMAL"
    assert r["primal_res_rel"] <= 1e-6 and r["dual_res_rel"] <= 1e-6 and r["rel_gap"] <= 1e-6
    assert lp2.c @ r["x"] == pytest.approx(lp2.p_star, rel=3e-6)
