#!/usr/bin/env python3
"""PDLP throughput on one MI355X.

Workload: the planted skewed LP with 20,000,000 rows, 25,000,000 columns and
~125M nonzeros (power-law column degrees capped at 10,000, 5,000 dense rows,
N(0,1) values, planted optimum), solved with the paper's settings for this
instance class: relative feasibility 1e-8, relative gap 1e-2, feasibility
polishing on.  Inputs are generated on the host, uploaded, transposed and
preconditioned before the timed region (reported as setup).

A step is one iteration block of the solver: 64 accepted PDHG iterations
(Algorithm 2 attempts, rejections included) followed by the periodic check
(average, two normalized duality gaps, termination test on the restart
candidate, restart decision with the primal-weight update), plus any
feasibility polishing that falls due.  value = accepted PDHG iterations
(main + polishing) per second.

The roofline object reports the dominant kernel, timed live with HIP events
on the library's stream over the timed region, against its algorithmic
bytes.  The CPU baseline times the FP64 oracle on a bounded sample of the
same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GRAPHS = 1   # step attempts replayed from HIP graphs (--no-graphs: eager launches)

METRIC = "PDHG iters/s + SpMV HBM GB/s at 125M nnz; batched LPs/s; bwd/fwd time at KKT tol"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the fused products on this workload, from two
# rocprofv3 counter runs of this script (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000;
# factors from a copy kernel of known size; see profiles/k_spmv_pair_skewed_20Mx25M.md).
# Valid only for the kernel source they were taken on (hash of the hot-path
# region of the kernels and constants); reported as null otherwise.
TRAFFIC_RECORD = {
    "hot_source": "672f4d36f6d08e1c",
    "workload": ("skewed", 124695196),                 # the default 20M x 25M LP only
    "k_spmv_dual": 9175810240,
    "k_seg_gather_primal+k_seg_primal": 8243926464,   # 5636830336 + 2607096128
    "k_spmv_primal": None,                             # not run on this workload any more
}


def hot_source_hash():
    import hashlib
    base = os.path.join(ROOT, "paper_2501_07018_amd", "csrc")
    def region(fname, tag):
        text = open(os.path.join(base, fname)).read()
        return text.split(f"// [hot-path {tag} begin]")[1].split(f"// [hot-path {tag} end]")[0]
    parts = (region("pdlp_kernels.hip", "kernels"), region("pdlp_device.h", "device"),
             region("pdlp_internal.h", "constants"), region("pdlp_host.hip", "layout"))
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(m, n, nnz):
    """Bytes each fused kernel must move at least once per launch (FP64 values, int32 indices).

    A x' + dual step, per row: row_ptr 4, y/Ax/lc/uc reads 32, A x'/y' writes 16,
    dual-average read-modify-write 16 -> 68; per nonzero val+col 12; x' read once 8 n.
    A^T y' + average + next primal step, per column: row_ptr 4, A^T y' write 8, x read 8,
    primal-average read-modify-write 16, c/lv/uv reads 24, x' write 8 -> 68; per
    nonzero 12; y' read once 8 m.
    """
    dual = 12 * nnz + 68 * m + 8 * n
    primal = 12 * nnz + 68 * n + 8 * m
    return dual, primal


def verify_point(lp, x, y, r):
    """Relative residuals of eq. "rescaled-termination-criteria" and the objective of a
    returned point, recomputed in numpy from the LP as generated (independent of the
    library and the oracle)."""
    import numpy as np
    A = lp.csr()
    ax = A @ x
    aty = A.T @ y
    lc, uc, c = lp.lc, lp.uc, lp.c
    fin_l, fin_u = np.isfinite(lc), np.isfinite(uc)
    al = np.where(fin_l & (lc != 0), np.abs(lc), 0.0)
    au = np.where(fin_u & (uc != 0), np.abs(uc), 0.0)
    q = np.where((al > 0) | (au > 0), np.maximum(al, au), 1.0)
    viol = np.maximum(np.maximum(np.where(fin_l, lc - ax, 0.0), np.where(fin_u, ax - uc, 0.0)), 0.0)
    w = np.where(c != 0, np.abs(c), 1.0)
    out = {"primal_res_rel_numpy": float(np.max(viol / q)) if lp.m else 0.0,
           "dual_res_rel_numpy": float(np.max(np.abs(c - aty - r) / w)) if lp.n else 0.0,
           "bounds_violation": float(max(np.max(lp.lv - x), np.max(x - lp.uv), 0.0)),
           "objective": float(c @ x + lp.obj_offset)}
    if lp.p_star is not None:
        out["p_star"] = float(lp.p_star)
        out["objective_rel_err"] = abs(out["objective"] - lp.p_star) / max(abs(lp.p_star), 1e-300)
    return out


def solve_section(lp, state, r, solve_wall, polish_iters, budget):
    """Continue the bench's solve (Algorithm 1 with the checks, polishing at
    k = 100, 200, 400, ... once the average's gap is below 1%) until the
    termination criteria hold or `budget` seconds pass; the returned point is
    then checked in numpy."""
    t0 = time.perf_counter()
    chunk = 1280
    while r["status_name"] == "ITERATION_LIMIT" and time.perf_counter() - t0 < budget:
        tc = time.perf_counter()
        # the point of a polished termination exists only in the call that found it
        r = state.solve(chunk, want_solution=True)
        solve_wall += time.perf_counter() - tc
        polish_iters += r["polish_iters"]
        log(f"solve: k={r['iterations']} gap={r['rel_gap']:.3e} pres={r['primal_res_rel']:.2e} "
            f"dres={r['dual_res_rel']:.2e} polish_attempts={r['polish_attempts']} "
            f"status={r['status_name']} ({solve_wall:.1f}s)")
    out = {"status": r["status_name"], "iterations": r["iterations"],
           "polish_attempts": r["polish_attempts"], "polish_iterations": polish_iters,
           "polished": r["polished"], "restarts": r["restarts"], "kkt_passes": r["kkt_passes"],
           "seconds_to_solution": solve_wall, "rel_gap": r["rel_gap"],
           "primal_res_rel": r["primal_res_rel"], "dual_res_rel": r["dual_res_rel"],
           "note": ("seconds_to_solution = wall time of all iteration blocks from the initial "
                    "point (setup excluded); residuals recomputed in numpy from the generated LP")}
    if r["status_name"] == "OPTIMAL" and "x" in r:
        out.update(verify_point(lp, r["x"], r["y"], r["r"]))
    return out


def host_identity():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(lp, steps):
    """The FP64 oracle as it stands, single-threaded, on the preconditioned LP
    (10 Ruiz rounds + Pock-Chambolle, as the GPU path runs it): `steps`
    accepted adaptive steps (Algorithm 2, rejected attempts included), with
    the oracle's KKT passes counted over the sample."""
    import oracle
    t0 = time.perf_counter()
    s = oracle.Solver(lp, oracle.Params(), scale=True)
    t_setup = time.perf_counter() - t0
    log(f"oracle preconditioned and initialized in {t_setup:.1f}s; timing {steps} steps")
    p0 = s.counters()["kkt_passes"]
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    dt = time.perf_counter() - t0
    passes = s.counters()["kkt_passes"] - p0
    out = {"value": steps / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
           "kkt_passes_per_s": passes / dt,
           "sample": (f"{steps} adaptive PDHG steps (Algorithm 2, accepted steps incl. any "
                      f"rejected attempts) of the single-threaded FP64 oracle on the same "
                      f"{lp.m}x{lp.n} LP after its preconditioning (restart/termination checks "
                      f"excluded); {dt:.1f} s timed, {t_setup:.1f} s of preconditioning before")}
    out.update(host_identity())
    # all host cores: the OpenMP build of the same oracle source (row shards,
    # Section 5 "Multithreading"), same LP and sample
    try:
        oracle.set_threaded(True)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or out["usable_cores"]
        s2 = oracle.Solver(lp, oracle.Params(), precond=(s.scaled.val, s.d1, s.d2))
        p0 = s2.counters()["kkt_passes"]
        t0 = time.perf_counter()
        for _ in range(steps):
            s2.step()
        dt2 = time.perf_counter() - t0
        out["all_cores"] = {"value": steps / dt2, "unit": "iters/s", "cores": threads,
                            "kkt_passes_per_s": (s2.counters()["kkt_passes"] - p0) / dt2,
                            "sample": f"the same {steps} steps with the OpenMP build; {dt2:.1f} s"}
        log(f"oracle all cores ({threads} threads): {steps / dt2:.3f} iters/s")
    finally:
        oracle.set_threaded(False)
    return out


def batch_section(pd, count, loop_n, cap):
    """Batched solver on the planted batch workload: `count` LPs with m ~ U{200..20000},
    n = 1.5 m, 8 distinct rows per column, relative KKT tolerance 1e-6, against
    pdlp_solve looped over a seeded sample of the same instances."""
    import numpy as np
    import lpgen
    t0 = time.perf_counter()
    sizes = lpgen.batch_sizes()[:count]
    lps = [lpgen.batch_lp(i, m, n) for i, (m, n) in enumerate(sizes)]
    nnz = sum(lp.nnz for lp in lps)
    log(f"batch: generated {count} LPs ({nnz} nonzeros) in {time.perf_counter() - t0:.1f}s")
    prm = pd.pdlp_params_default(eps_feas=1e-6, eps_gap=1e-6, max_iters=cap, graphs=GRAPHS)
    b = pd.Batch(lps)
    t0 = time.perf_counter()
    res = b.solve(prm, want_solution=False)
    tb = time.perf_counter() - t0
    st = b.stats()
    status = {}
    for r in res:
        status[r["status_name"]] = status.get(r["status_name"], 0) + 1
    log(f"batch: solved in {tb:.2f}s {status} {st}")
    b.close()
    # the loop leg on equal terms: problems created (uploaded, scaled) before the
    # timed region, as the batch's are
    rng = np.random.default_rng(2025)
    idx = rng.choice(count, size=min(loop_n, count), replace=False)
    probs = [pd.Problem(lps[i], prm) for i in idx]
    t0 = time.perf_counter()
    loop_it, loop_ok = 0, 0
    for p in probs:
        r = p.solve(prm)
        loop_it += r["iterations"]
        loop_ok += r["status_name"] == "OPTIMAL"
    tl = time.perf_counter() - t0
    for p in probs:
        p.close()
    log(f"batch: loop of {len(idx)} pdlp_solve in {tl:.2f}s ({loop_ok} optimal)")
    n_opt = status.get("OPTIMAL", 0)
    stragglers = [{"instance": i, "m": sizes[i][0], "n": sizes[i][1],
                   "status": r["status_name"], "iterations": r["iterations"]}
                  for i, r in enumerate(res) if r["status_name"] != "OPTIMAL"]
    return {
        "workload": (f"{count} planted LPs, m ~ U{{200..20000}}, n = 1.5 m, 8 rows per column, "
                     f"{nnz} nonzeros in total; relative KKT 1e-6, iteration cap {cap}"),
        "lps_per_s": count / tb, "optimal_lps_per_s": n_opt / tb, "seconds": tb,
        "status": status, "not_optimal": stragglers,
        "iters_per_s_aggregate": st["total_iterations"] / tb,
        "max_iterations": st["max_iterations"], "total_iterations": st["total_iterations"],
        "rounds": st["rounds"], "step_seconds": st["step_seconds"],
        "check_seconds": st["check_seconds"],
        "loop_sample": int(len(idx)), "loop_optimal": int(loop_ok),
        "loop_lps_per_s": len(idx) / tl, "loop_iters_per_s": loop_it / tl,
        "speedup_lps": (count / tb) / (len(idx) / tl),
        "note": ("lps_per_s = instances / wall time of one pdlp_batch_solve; loop figures time "
                 "pdlp_solve over a seeded random sample of the same instances; both legs "
                 "start from problems already created on the GPU (creation excluded from both)"),
    }


def tolerance_sweep_section(pd, grid_L, sample, time_limit):
    """Feasibility tolerance 1e-8, 1e-10, 1e-12 (primal and dual), relative gap
    1e-2, with and without feasibility polishing, on the planted 1,000 x 2,000
    LP, an L x L multicommodity grid (8 commodities, 20 pairs each) and a
    seeded sample of the batch workload's instances (single solves, and the
    sample as one batch without polishing)."""
    import lpgen
    sizes = lpgen.batch_sizes()
    work = [("planted_1000x2000", lpgen.small_lp()),
            (f"grid_{grid_L}x{grid_L}_k8", lpgen.grid_flow_lp(L=grid_L))]
    members = [lpgen.batch_lp(i, m, n) for i, (m, n) in enumerate(sizes[:sample])]
    rows = []
    for eps in (1e-8, 1e-10, 1e-12):
        for polish in (0, 1):
            prm = pd.pdlp_params_default(eps_feas=eps, eps_gap=1e-2, polish=polish, graphs=GRAPHS,
                                         max_iters=200_000, time_limit=time_limit)
            for name, lp in work:
                p = pd.Problem(lp)
                t0 = time.perf_counter()
                r = p.solve(prm)
                dt = time.perf_counter() - t0
                p.close()
                rows.append({"workload": name, "eps_feas": eps, "polish": polish,
                             "status": r["status_name"], "iterations": r["iterations"],
                             "polish_iters": r["polish_iters"], "seconds": dt,
                             "primal_res_rel": r["primal_res_rel"],
                             "dual_res_rel": r["dual_res_rel"], "rel_gap": r["rel_gap"]})
                log(f"sweep: {rows[-1]}")
            solved, its, t_all = 0, 0, 0.0
            for lp in members:
                p = pd.Problem(lp)
                t0 = time.perf_counter()
                r = p.solve(prm)
                t_all += time.perf_counter() - t0
                p.close()
                solved += r["status_name"] == "OPTIMAL"
                its += r["iterations"] + r["polish_iters"]
            rows.append({"workload": f"batch_members_x{len(members)}", "eps_feas": eps,
                         "polish": polish, "solved": solved, "iterations": its,
                         "seconds": t_all})
            log(f"sweep: {rows[-1]}")
        b = pd.Batch(members)
        prm = pd.pdlp_params_default(eps_feas=eps, eps_gap=1e-2, max_iters=200_000, graphs=GRAPHS,
                                     time_limit=time_limit)
        t0 = time.perf_counter()
        res = b.solve(prm, want_solution=False)
        dt = time.perf_counter() - t0
        b.close()
        rows.append({"workload": f"batch_of_{len(members)}", "eps_feas": eps, "polish": 0,
                     "solved": sum(r["status_name"] == "OPTIMAL" for r in res),
                     "iterations": sum(r["iterations"] for r in res), "seconds": dt})
        log(f"sweep: {rows[-1]}")
    return {"rows": rows, "iteration_cap": 200_000, "time_limit_s": time_limit}


def unroll_section(pd, count, K):
    """Differentiable layer: `count` planted 2,000 x 4,000 LPs (10 rows per column),
    K unrolled steps with decisions recorded and checkpoints every 25 steps, an
    N(0,1) upstream gradient on x; backward = gradients for c, lc, uc and the
    nonzeros of A."""
    import numpy as np
    import lpgen
    t0 = time.perf_counter()
    lps = [lpgen.layer_lp(i) for i in range(count)]
    log(f"unroll: generated {count} LPs in {time.perf_counter() - t0:.1f}s")
    u = pd.Unroll(lps)
    gx = np.random.default_rng(2501).standard_normal(u.N)
    # warm-up pair (first-touch allocation of the work buffers)
    u.forward(K, 25, pd.pdlp_params_default(graphs=GRAPHS))
    u.backward(gx)
    fw, bw, rp = [], [], []
    for _ in range(3):
        u.forward(K, 25, pd.pdlp_params_default(graphs=GRAPHS))
        u.backward(gx)
        u.replay()
        st = u.stats()
        fw.append(st["forward_seconds"])
        bw.append(st["backward_seconds"])
        rp.append(st["replay_seconds"])
    log(f"unroll: forward {fw} backward {bw} replay {rp} stats {st}")
    nnz = sum(lp.nnz for lp in lps)
    tf, tb = float(np.median(fw)), float(np.median(bw))
    return {
        "workload": (f"{count} planted LPs of 2000 x 4000, 10 rows per column ({nnz} nonzeros), "
                     f"K = {K} unrolled steps, checkpoints every 25, N(0,1) upstream gradient"),
        "forward_s": tf, "backward_s": tb, "bwd_over_fwd": tb / tf,
        "replay_s": float(np.median(rp)),
        "backward_replay_s": st["backward_replay_seconds"],
        "backward_reverse_s": st["backward_reverse_seconds"],
        "restarts": st["restarts"],
        "note": ("forward = Algorithm 1 with decisions recorded (adaptive steps, restart checks); "
                 "backward = segment replays from checkpoints + reverse steps; median of 3, "
                 "host transfers excluded"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("skewed", "grid"), default="skewed",
                    help="single-LP workload: the planted skewed LP (--m x --n, the default) or "
                         "the L x L multicommodity grid (--grid-side; kernel profiles only)")
    ap.add_argument("--grid-side", type=int, default=300)
    ap.add_argument("--m", type=int, default=20_000_000)
    ap.add_argument("--n", type=int, default=25_000_000)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-count", type=int, default=1024,
                    help="instances of the batched-solver measurement (0 skips it)")
    ap.add_argument("--batch-loop", type=int, default=48,
                    help="instances solved one by one for the loop comparison")
    ap.add_argument("--batch-cap", type=int, default=200_000,
                    help="iteration cap per instance of the batched-solver measurement")
    ap.add_argument("--unroll-count", type=int, default=256,
                    help="instances of the differentiable-layer measurement (0 skips it)")
    ap.add_argument("--unroll-k", type=int, default=500)
    ap.add_argument("--solve-budget", type=float, default=0.0,
                    help="after the timed steps, continue the same solve to its tolerances "
                         "(1%% gap, polishing to 1e-8) for at most this many seconds")
    ap.add_argument("--stream-block", type=int, default=0,
                    help="stream-block schedule of the 20M x 25M problem: 0 default, -1 autotune "
                         "on the solver's steps, else nonzeros per block")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch step attempts one by one (same results; for tracing tools)")
    ap.add_argument("--tol-sweep", action="store_true",
                    help="add the feasibility-tolerance sweep (1e-8/1e-10/1e-12, polishing on/off)")
    ap.add_argument("--sweep-grid", type=int, default=100, help="grid side L of the sweep")
    ap.add_argument("--sweep-sample", type=int, default=8, help="batch instances in the sweep")
    ap.add_argument("--sweep-time-limit", type=float, default=30.0)
    args = ap.parse_args()
    global GRAPHS
    GRAPHS = 0 if args.no_graphs else 1
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import lpgen
    import paper_2501_07018_amd as pd

    t0 = time.perf_counter()
    if args.workload == "grid":
        lp = lpgen.grid_flow_lp(L=args.grid_side)
        log(f"generated the {args.grid_side} x {args.grid_side} grid ({lp.m} x {lp.n}, "
            f"{lp.nnz} nonzeros) in {time.perf_counter() - t0:.1f}s")
        prm = pd.pdlp_params_default(eps_feas=1e-6, eps_gap=1e-6, profile=1,
                                     stream_block=args.stream_block)
    else:
        lp = lpgen.skewed_lp(args.m, args.n, verbose=True)
        st = lp.stats()
        log(f"generated {st} in {time.perf_counter() - t0:.1f}s")
        prm = pd.pdlp_params_default(eps_feas=1e-8, eps_gap=1e-2, polish=1, profile=1,
                                     stream_block=args.stream_block)
    t0 = time.perf_counter()
    prob = pd.Problem(lp, prm)
    state = prob.state(prm)
    setup_s = time.perf_counter() - t0
    log(f"problem on the GPU (upload, transpose, scaling, init) in {setup_s:.2f}s")

    step_k = 64
    solve_wall = 0.0
    for w in range(args.warmup):
        tw = time.perf_counter()
        r = state.solve(step_k)
        solve_wall += time.perf_counter() - tw
        log(f"warmup {w}: k={r['iterations']} gap={r['rel_gap']:.3e} pres={r['primal_res_rel']:.2e}")
    state.kernel_stats(reset=True)
    k0 = r["iterations"] if args.warmup else 0
    passes0 = r["kkt_passes"] if args.warmup else 0
    polish_iters = 0
    status = "ITERATION_LIMIT"
    steps_done = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = state.solve(step_k)
        polish_iters += r["polish_iters"]
        steps_done += 1
        if r["status_name"] != "ITERATION_LIMIT":
            status = r["status_name"]
            break
    elapsed = time.perf_counter() - t0
    solve_wall += elapsed
    ks = state.kernel_stats()
    iters = r["iterations"] - k0 + polish_iters
    log(f"timed {steps_done} steps: {iters} iterations in {elapsed:.3f}s; last: k={r['iterations']} "
        f"gap={r['rel_gap']:.3e} pres={r['primal_res_rel']:.2e} dres={r['dual_res_rel']:.2e} "
        f"restarts={r['restarts']} polish_attempts={r['polish_attempts']}")
    log(f"kernel stats: {ks}")

    m, n, nnz = lp.m, lp.n, lp.nnz
    b_dual, b_primal = algorithmic_bytes(m, n, nnz)
    avg_dual = ks["dual_ms"] / max(ks["dual_launches"], 1)
    avg_primal = ks["primal_ms"] / max(ks["primal_launches"], 1)
    gbs_dual = b_dual / (avg_dual * 1e-3) / 1e9 if avg_dual > 0 else 0.0
    gbs_primal = b_primal / (avg_primal * 1e-3) / 1e9 if avg_primal > 0 else 0.0
    seg = ks.get("primal_gather_ms", 0.0) > 0.0
    primal_name = "k_seg_gather_primal+k_seg_primal" if seg else "k_spmv_primal"
    if ks["dual_ms"] >= ks["primal_ms"]:
        dom = ("k_spmv_dual", gbs_dual, avg_dual, b_dual, ks["dual_launches"])
    else:
        dom = (primal_name, gbs_primal, avg_primal, b_primal, ks["primal_launches"])
    pair_gbs = (b_dual + b_primal) / ((avg_dual + avg_primal) * 1e-3) / 1e9
    # achievable device rates: streaming copy, and random FP64 gathers from
    # an array the size of each product's gathered vector
    rates_n = pd.pdlp_measure_device_rates(2 << 30, n)
    rates_m = pd.pdlp_measure_device_rates(2 << 30, m)
    log(f"device rates: {rates_n} (gather domain n), {rates_m} (gather domain m)")

    out = {
        "metric": METRIC,
        "value": iters / elapsed,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(steps_done, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"planted skewed LP {m}x{n}, {nnz} nonzeros (power-law column degrees "
                         f"capped at 10,000, 5,000 dense rows); eps_feas 1e-8, eps_gap 1e-2, "
                         f"polishing on; step = 64 accepted PDHG iterations + periodic check"
                         if args.workload == "skewed" else
                         f"multicommodity grid {args.grid_side}x{args.grid_side} (8 commodities, "
                         f"20 pairs each), {m}x{n}, {nnz} nonzeros; relative KKT 1e-6; step = 64 "
                         f"accepted PDHG iterations + periodic check"),
            "m": m, "n": n, "nnz": nnz, "iterations_per_step": step_k,
            "schedule": prob.schedule(),
            "status_at_end": status, "rel_gap_at_end": r["rel_gap"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom[0],
            "achieved": dom[1],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom[1] / HBM_PEAK_GBS,
            "traffic": (TRAFFIC_RECORD.get(dom[0])
                        if (hot_source_hash() == TRAFFIC_RECORD["hot_source"]
                            and (args.workload, nnz) == TRAFFIC_RECORD["workload"]) else None),
            "avg_launch_ms": dom[2],
            "algorithmic_bytes_per_launch": dom[3],
            "launches": dom[4],
        },
        "spmv_pair": {"achieved_gbs": pair_gbs, "frac": pair_gbs / HBM_PEAK_GBS,
                      "dual_ms": avg_dual, "primal_ms": avg_primal,
                      "primal_gather_ms": (ks.get("primal_gather_ms", 0.0)
                                           / max(ks["primal_launches"], 1)),
                      "primal_product": ("two-phase (segmented gathers of y')" if seg
                                         else "one pass"),
                      "dual_gbs": gbs_dual, "primal_gbs": gbs_primal},
        "device_rates": {
            "copy_gbs": rates_n["copy_gbs"],
            "random_gather_gps_domain_n": rates_n["gather_gps"],
            "random_gather_gps_domain_m": rates_m["gather_gps"],
            "random_gather_gps_l2_resident": rates_n["gather_l2_gps"],
            "note": ("each nonzero of A x' and A^T y' gathers one FP64 word at a random index; "
                     "nnz / random_gather_gps bounds a product from below when the gathers miss L2"),
            "dual_gather_floor_ms": nnz / rates_n["gather_gps"] / 1e6,
            "primal_gather_floor_ms": nnz / rates_m["gather_gps"] / 1e6,
        },
        "kkt_passes_per_s": (r["kkt_passes"] - passes0) / elapsed,
        "setup_s": setup_s,
        "check_ms_per_step": ks["check_ms"] / max(steps_done, 1),
    }
    if args.solve_budget > 0:
        out["solve_to_tolerance"] = solve_section(lp, state, r, solve_wall, polish_iters,
                                                  args.solve_budget)
    if args.batch_count > 0:
        out["batched"] = batch_section(pd, args.batch_count, args.batch_loop, args.batch_cap)
    if args.unroll_count > 0:
        out["unroll"] = unroll_section(pd, args.unroll_count, args.unroll_k)
    if args.tol_sweep:
        out["tolerance_sweep"] = tolerance_sweep_section(pd, args.sweep_grid, args.sweep_sample,
                                                         args.sweep_time_limit)
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(lp, args.cpu_steps)
        except Exception as e:  # the baseline never blocks the GPU number
            log(f"cpu baseline failed: {e!r}")
            out["cpu_baseline"] = None
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
