/*
 * pdlp.h -- C ABI of the MI355X (gfx950) PDLP library.
 *
 * PDLP is the restarted, diagonally preconditioned primal-dual hybrid
 * gradient method of Applegate et al., "PDLP: A Practical First-Order Method
 * for Large-Scale Linear Programming" (arXiv 2501.07018), for the LP
 *
 *     min c^T x  s.t.  lc <= A x <= uc,  lv <= x <= uv          (Section 2, eq. "lp")
 *
 * with dual  max -p(-y; lc, uc) - p(-r; lv, uv)  s.t. c - A^T y = r, y in Y, r in R,
 * where p(y; l, u) = u^T y+ - l^T y-.
 *
 * Every floating-point quantity is IEEE binary64, on the host and on the GPU.
 *
 * Conventions shared by all entry points
 *   - Absent bounds are +-HUGE_VAL (+-infinity).  lc = uc encodes an equality.
 *   - A is CSR: row_ptr[m+1] (int32, row_ptr[0] = 0, nondecreasing),
 *     col[nnz] (int32, strictly increasing inside each row, in [0, n)),
 *     val[nnz] (finite doubles).  Empty rows and columns, and m = 0, are allowed.
 *   - Pointers named *_host are host memory; the library copies what it
 *     needs before returning and never keeps a caller pointer.
 *   - Output arrays are caller-owned and may be NULL when not wanted.
 *   - Return codes: PDLP_OK (0) or a negative PDLP_ERR_*; the message of the
 *     last error on the calling thread is returned by pdlp_last_error().
 *   - One problem (and its states) is used from one host thread at a time;
 *     all GPU work is ordered on the stream given at creation (NULL = the
 *     default stream), and every entry point returns after that work ends.
 */
#ifndef PDLP_H
#define PDLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDLP_OK 0
#define PDLP_ERR_INVALID_ARGUMENT (-1)
#define PDLP_ERR_HIP (-2)
#define PDLP_ERR_OUT_OF_MEMORY (-3)
#define PDLP_ERR_STATE (-4)

/* Solve status (Section 7 outcomes: solved, time limit, numerical error). */
#define PDLP_STATUS_OPTIMAL 0
#define PDLP_STATUS_ITERATION_LIMIT 1
#define PDLP_STATUS_TIME_LIMIT 2
#define PDLP_STATUS_NUMERICAL_ERROR 3
#define PDLP_STATUS_PRIMAL_INFEASIBLE 4  /* Appendix D certificate (y, r) found */
#define PDLP_STATUS_DUAL_INFEASIBLE 5    /* Appendix D certificate (x, s) found */

typedef struct pdlp_problem pdlp_problem; /* opaque: device copy of A, A^T, scaling */
typedef struct pdlp_state pdlp_state;     /* opaque: iterate state on the device */

/*
 * Parameters.  Defaults (pdlp_params_default) are the paper's constants:
 * restart/termination checks every 64 accepted steps (Section 3, "Periodic
 * checks"), beta_sufficient 0.1, beta_necessary 0.9, beta_artificial 0.5
 * (Section 3, "Adaptive restarts"), theta 0.5 and eps_zero 1e-10
 * (Algorithm 3), step exponents 0.3 and 0.6 (Algorithm 2), 10 Ruiz rounds
 * then Pock-Chambolle with alpha = 1 (Section 3, "Diagonal Preconditioning"),
 * feasibility polishing at k = 100, 200, 400, ... with k/8 caps (Algorithm 4).
 */
typedef struct pdlp_params {
    double eps_feas;          /* relative primal/dual residual tolerance (1e-8) */
    double eps_gap;           /* relative duality gap tolerance (1e-8) */
    int64_t max_iters;        /* limit on accepted PDHG steps */
    double time_limit;        /* seconds; <= 0 means the limit is already reached */
    int32_t check_every;      /* 64 */
    int32_t ruiz_iters;       /* 10 */
    int32_t pock_chambolle;   /* 1: one Pock-Chambolle round (alpha = 1) after Ruiz */
    int32_t polish;           /* feasibility polishing (Algorithm 4) on/off */
    int64_t polish_first;     /* 100 */
    int32_t reduced_cost_mode;/* -1: App. A choice without polishing, projection with it;
                                 0: projection onto R; 1: Appendix A choice */
    int32_t adaptive_restarts;/* 1: criteria (i)-(iii); 0: only (iii) */
    double beta_suff, beta_nec, beta_art;
    double theta, eps_zero;
    double red_exp, grow_exp;
    int32_t verbose;          /* 1: one line per check on stderr */
    int32_t profile;          /* 1: time the step kernels with HIP events (pdlp_state_kernel_stats) */
    int32_t reorder;          /* 1 (default): relabel rows/columns by decreasing length inside the
                                 library (cache locality of the gathers); results are unaffected */
    int32_t detect_infeasibility; /* 1 (default): Appendix D tests at every termination check */
    double eps_infeasible;    /* threshold of those tests (1e-9) */
    /* Algorithm 5 mode (Appendix C), single problems only: with restart_period > 0 every step
       uses the constant step fixed_step_size (> 0) and primal weight fixed_primal_weight (> 0),
       and after every restart_period accepted steps the iterate restarts to the plain average
       of x with y = 0; no adaptive steps or restarts, no primal weight update, no polishing.
       Termination checks (at check_every) test the average.  Default 0 (off). */
    int64_t restart_period;
    double fixed_step_size;
    double fixed_primal_weight;
    int32_t graphs;           /* 1 (default): step attempts are replayed from HIP graphs captured
                                 once (per vector set, or per set of running batch instances);
                                 0: launched one by one.  Results are identical either way. */
    int32_t stream_block;     /* nonzeros per block of the CSR stream products (problem and batch
                                 creation): 0 (default) 2048; else a value in [64, 2048]; -1
                                 autotune.  A single problem autotunes on the solver's own
                                 steps: for (block size, longest row of the stream class) in
                                 (2048, 64), (2048, 32), (2048, 128), (1024, 64), (1024, 32),
                                 (512, 64) it runs 4 + 16 accepted steps from the initial point
                                 and keeps the fastest (pdlp_problem_schedule reports it); rows
                                 longer than the chosen length are summed by a wave or a
                                 workgroup tree instead of in stored order.  A batch times 256,
                                 512, 1024 and 2048 with plain products, for A and A^T
                                 separately.  With a fixed row class, row sums are the same
                                 whatever the blocks; only the order in which the step norms'
                                 partial sums combine changes. */
    int32_t sorted_gathers;   /* batch and unroll creation: 1 (default) keeps a copy of the
                                 short-row blocks of A and A^T sorted by column (22 bytes per
                                 nonzero) where that cuts the cache lines a wave gathers from;
                                 0 leaves it out.  Results are identical either way. */
    int32_t segmented_gathers;/* single problems: the product A~^T y' of every step in two
                                 phases (y' cut into 2 MB segments, each gathered by one XCD
                                 while it sits in that XCD's L2; then the pair sums staged per
                                 row block and the primal step run on them).  -1 (default):
                                 when y' exceeds 32 MB; 1 always; 0 never.  Rows of at most 64
                                 nonzeros are summed exactly as by the one-pass product; longer
                                 rows per segment, then over the segments. */
} pdlp_params;

/* Result of a solve.  x, y, r are caller buffers of length n, m, n (or NULL);
 * they receive the unscaled solution x = D2 x~ (clamped to [lv, uv]: the
 * scaled bounds carry the rounding of the preconditioning, a few ulps),
 * y = D1 y~ and the reduced costs used in the termination test.  Residuals follow Section 7, eq.
 * "rescaled-termination-criteria" (relative) and its l_inf absolute form.
 *
 * Infeasibility (Section 3, "Infeasibility detection"; Appendix D): at every
 * termination check that does not terminate, three candidates are tested in
 * this order -- the difference of the two latest iterates, the current
 * iterate, and the average since the last restart (the tests are invariant
 * under positive scaling, so the paper's normalization is implied) -- first
 * for primal, then for dual infeasibility.  A candidate's y is projected onto
 * Y and its x onto the recession cone Xbar of the variable bounds; the primal
 * test takes r = proj_R(-A^T y) and needs lc^T y+ - uc^T y- + lv^T r+ - uv^T r-
 * > 0 with max_j |A^T y + r|_j / w_j <= eps_infeasible times it (w_j = |c_j|,
 * or 1 where c_j = 0); the dual test takes s = proj_Sbar(-A x) and needs
 * c^T x < 0 with max_i |A x + s|_i / q_i <= eps_infeasible |c^T x| (q as in
 * the relative primal residual).  The weights are those of the termination
 * criteria: the paper states the tests on instances rescaled to unit
 * objective and right-hand-side entries.  On an infeasible status x, y hold
 * the certifying candidate projected onto Xbar x Y (unscaled) and r holds
 * proj_R(-A^T y); the KKT fields keep the last termination evaluation. */
typedef struct pdlp_result {
    double *x, *y, *r;        /* in: caller buffers or NULL */
    int32_t status;
    int32_t polished;         /* 1 when the returned point came from polishing */
    int64_t iterations;       /* accepted PDHG steps of the main run */
    int64_t attempts;         /* step attempts including rejected ones */
    int64_t kkt_passes;       /* products A x + A^T y computed (all phases) */
    int64_t restarts, restarts_i, restarts_ii, restarts_iii;
    int64_t polish_attempts, polish_iters;
    double primal_obj, dual_obj, rel_gap;
    double primal_res_abs, primal_res_rel, dual_res_abs, dual_res_rel;
    double omega, eta;        /* final primal weight and step size */
    double seconds;           /* wall time inside pdlp_solve */
    double seconds_setup;     /* preconditioning + initialization part of it */
    int32_t certificate;      /* infeasible status: 1 difference of iterates, 2 iterate,
                                 3 average; else 0 */
    int32_t reserved;
    double certificate_objective; /* the test's objective (> 0 primal, < 0 dual) */
    double certificate_residual;  /* its weighted residual */
} pdlp_result;

/* Counters after pdlp_iterate_k. */
typedef struct pdlp_iter_info {
    int64_t k, t, n_outer, attempts, kkt_passes;
    int64_t restarts_i, restarts_ii, restarts_iii;
    double omega, eta_hat, last_eta, last_eta_bar, seta, mu_ref, mu_c_prev;
} pdlp_iter_info;

/* Full iterate state in the scaled space, for export and bitwise resume.
 * Arrays are caller buffers: x, x0, sx, aty of length n; y, y0, sy, ax of
 * length m (any may be NULL on get; none may be NULL on set). */
typedef struct pdlp_state_blob {
    double *x, *y, *ax, *aty, *x0, *y0, *sx, *sy;
    double seta, omega, eta_hat, mu_ref, mu_c_prev, last_eta;
    int64_t k, t, n_outer, attempts, kkt_passes;
    int64_t restarts_i, restarts_ii, restarts_iii;
} pdlp_state_blob;

/*
 * Create a problem from host CSR arrays (see conventions).  Validates the
 * input, uploads it, builds A^T on the GPU and applies the diagonal
 * preconditioning of params (NULL = defaults): ruiz_iters Ruiz rounds then
 * an optional Pock-Chambolle round (Section 3, "Diagonal Preconditioning").
 * hip_stream: a hipStream_t or NULL.  Errors: INVALID_ARGUMENT for bad sizes,
 * unsorted/duplicate/out-of-range columns, non-finite values or c, NaN
 * bounds, lc > uc, lv > uv, a lower bound of +inf or an upper bound of -inf;
 * OUT_OF_MEMORY; HIP_ERROR.
 */
int pdlp_problem_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr_host,
                        const int32_t *col_host, const double *val_host, const double *c_host,
                        const double *lc_host, const double *uc_host, const double *lv_host,
                        const double *uv_host, double obj_offset, const pdlp_params *params,
                        void *hip_stream, pdlp_problem **out);

/*
 * Same as pdlp_problem_create, with every array in GPU memory (for instance
 * the storage of torch tensors on the device; host memory is accepted too).
 * Validation and the internal row/column labelling run on the host, so the
 * arrays are first copied to the host on hip_stream, after the work already
 * queued there; the caller keeps ownership and may free them when the call
 * returns.  The lengths are trusted: row_ptr_dev must hold m + 1 entries,
 * col_dev and val_dev nnz, c_dev, lv_dev and uv_dev n, lc_dev and uc_dev m
 * (the library copies exactly those byte counts; shorter arrays are read
 * past their end).  Errors as for pdlp_problem_create; HIP_ERROR for a
 * pointer the runtime cannot copy from.
 */
int pdlp_problem_create_device(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr_dev,
                               const int32_t *col_dev, const double *val_dev, const double *c_dev,
                               const double *lc_dev, const double *uc_dev, const double *lv_dev,
                               const double *uv_dev, double obj_offset, const pdlp_params *params,
                               void *hip_stream, pdlp_problem **out);

void pdlp_problem_destroy(pdlp_problem *p);

/* Sizes of a created problem. */
int pdlp_problem_dims(const pdlp_problem *p, int32_t *m, int32_t *n, int64_t *nnz);

/* The block schedule of a created problem's products: nonzeros per stream
 * block and the longest row of the stream class (rows summed in stored
 * order by one lane); either pointer may be NULL. */
int pdlp_problem_schedule(const pdlp_problem *p, int32_t *stream_block, int32_t *med_row);

/* Copy out the preconditioned problem: D1 (m), D2 (n), the scaled values of
 * A in the caller's CSR order (nnz), and the scaled c~, lc~, uc~, lv~, uv~
 * (Section 3: c~ = D2 c, (lc~, uc~) = D1 (lc, uc), (lv~, uv~) = D2^-1 (lv, uv)). */
int pdlp_problem_get_scaled(const pdlp_problem *p, double *d1, double *d2, double *val,
                            double *c, double *lc, double *uc, double *lv, double *uv);

/* One GPU sparse product on host vectors: transpose = 0 gives out = A x
 * (x: n, out: m), transpose = 1 gives out = A^T x (x: m, out: n); scaled = 1
 * uses the preconditioned matrix A~, 0 the original one (original = D1^-1 A~ D2^-1,
 * applied through the diagonals).  `repeat` >= 1 runs the product that many
 * times (for timing); *ms receives the average kernel time if not NULL. */
int pdlp_spmv(const pdlp_problem *p, int32_t transpose, int32_t scaled, const double *x_host,
              double *out_host, int32_t repeat, double *ms);

/*
 * pdlp_spmv without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  x_dev (length n, or m when transpose = 1) and out_dev (m, or n)
 * are caller buffers in GPU memory, in the caller's order; scaled as for
 * pdlp_spmv.  The work is enqueued on hip_stream (NULL: the problem's stream)
 * and the call returns without waiting; out_dev is valid once the stream has
 * reached it.  Staging of the permuted vectors lives in a fixed device array
 * of 2^23 doubles (64 MiB) per GPU, kept until the process ends: m + n above
 * 2^23 is rejected with INVALID_ARGUMENT, and so is a call while another GPU
 * than the problem's is current.  Every call on a GPU shares that
 * array (and the problem's own product buffers), so calls that overlap on one
 * GPU race; nothing in the array needs clearing between calls.  Allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.
 */
int pdlp_spmv_noalloc(const pdlp_problem *p, int32_t transpose, int32_t scaled,
                      const double *x_dev, double *out_dev, void *hip_stream);

void pdlp_params_default(pdlp_params *params);

/*
 * Solve (Algorithm 1 with Algorithm 2 steps, adaptive restarts, Algorithm 3
 * primal weights, Algorithm 4 polishing when params->polish; termination by
 * eq. "rescaled-termination-criteria" and eq. "relative-gap").  params NULL
 * = defaults.  x0_host/y0_host (unscaled, length n and m, both or neither)
 * give a warm start; NULL starts from (proj_X(0), 0).  result must not be
 * NULL.  Returns PDLP_OK when a status was reached (the status is in result).
 */
int pdlp_solve(pdlp_problem *p, const pdlp_params *params, const double *x0_host,
               const double *y0_host, pdlp_result *result);

/* Create a state: preconditioned problem + initial point of Algorithm 1
 * (eta_hat = 1/max|A~_ij|, omega from InitializePrimalWeight, z = (proj_X(0), 0)). */
int pdlp_state_create(pdlp_problem *p, const pdlp_params *params, pdlp_state **out);
void pdlp_state_destroy(pdlp_state *s);

/* Run exactly k more accepted steps with the restart checks of Algorithm 1
 * but no termination test or polishing; info may be NULL.  k >= 0. */
int pdlp_iterate_k(pdlp_state *s, int64_t k, pdlp_iter_info *info);

/* Continue the solve of pdlp_solve from the state for at most k more
 * accepted steps: termination test at every check (and at the start when no
 * step has been taken yet), feasibility polishing when params->polish.
 * result as in pdlp_solve (status ITERATION_LIMIT when k steps passed
 * without termination); its x, y, r buffers may be NULL. */
int pdlp_state_solve(pdlp_state *s, int64_t k, pdlp_result *result);

/* Per-kernel GPU time of the step loop, accumulated while params->profile
 * is set: HIP events around every launch on the library's stream.  The
 * "dual" kernel is A x' fused with the dual step, the "primal" kernel A^T y'
 * fused with the primal average and the next primal step; launches count
 * the ones that did work.  reset != 0 zeroes the counters after reading. */
typedef struct pdlp_kernel_stats {
    int64_t dual_launches, primal_launches, attempts;
    double dual_ms, primal_ms, decide_ms, standalone_primal_ms;
    double check_ms;          /* host wall time spent at block boundaries */
    double primal_gather_ms;  /* part of primal_ms spent in the gather phase of the two-phase
                                 product (0 when the one-pass product runs) */
} pdlp_kernel_stats;
int pdlp_state_kernel_stats(pdlp_state *s, pdlp_kernel_stats *stats, int32_t reset);

/* Copy the state out (get) or in (set); see pdlp_state_blob. */
int pdlp_state_get(const pdlp_state *s, pdlp_state_blob *blob);
int pdlp_state_set(pdlp_state *s, const pdlp_state_blob *blob);

/* Normalized duality gap mu(z, z_ref) = rho_r(z), r = ||z - z_ref||_omega
 * (Section 3, "Adaptive restarts") of scaled host points; ax/aty are A~x and
 * A~^T y.  Vectors: x, aty, xr of length n; y, ax, yr of length m. */
int pdlp_norm_gap(const pdlp_problem *p, const double *x, const double *y, const double *ax,
                  const double *aty, const double *xr, const double *yr, double omega,
                  double *mu);

/* Achievable device rates for the roofline of the sparse products, measured
 * on the library's default stream: a streaming copy of `copy_bytes` bytes
 * (read + write GB/s) and random FP64 gathers from an array of `gather_len`
 * doubles (indices from a fixed hash, 125M gathers; G gathers/s).  Allocates
 * and frees its own buffers. */
typedef struct pdlp_device_rates {
    double copy_gbs;          /* bytes read + written per second / 1e9 */
    double gather_gps;        /* random 8-byte gathers per second / 1e9 */
    double gather_l2_gps;     /* the same from a 1 MiB array (cache-resident) */
} pdlp_device_rates;
int pdlp_measure_device_rates(int64_t copy_bytes, int64_t gather_len, pdlp_device_rates *out);

/*
 * Batches: many independent LPs solved together in the same kernel launches.
 *
 * The instances are packed block-diagonally on the device; each keeps its
 * own step size, primal weight, restart state and termination (Algorithm 1
 * per instance, with the same readings as pdlp_solve), so a batch result
 * equals that of solving each instance alone up to the rounding order of
 * the reductions.  Scaling (Ruiz + Pock-Chambolle) is per row and column and
 * hence per instance.  Feasibility polishing and warm starts are not
 * offered for batches.
 */
typedef struct pdlp_batch pdlp_batch;     /* opaque: packed instances on the device */

/*
 * Create a batch of `count` >= 1 instances from host arrays.  Instance i has
 * m[i] >= 0 rows, n[i] >= 1 columns and nnz[i] nonzeros.  Arrays are the
 * instances' own arrays concatenated in instance order:
 *   row_ptr: sum(m[i] + 1) entries, each instance's CSR row pointers starting at 0;
 *   col, val: sum(nnz[i]) entries, column indices local to the instance;
 *   c, lv, uv: sum(n[i]);  lc, uc: sum(m[i]);
 *   obj_offset: count entries, or NULL for zeros.
 * Each instance obeys the conventions above; the batch totals of rows,
 * columns and nonzeros must stay below 2^31.  params: scaling parameters
 * (ruiz_iters, pock_chambolle), NULL = defaults.  Errors as
 * pdlp_problem_create, with the instance named in the message.
 */
int pdlp_batch_create(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                      const int32_t *row_ptr_host, const int32_t *col_host,
                      const double *val_host, const double *c_host, const double *lc_host,
                      const double *uc_host, const double *lv_host, const double *uv_host,
                      const double *obj_offset_host, const pdlp_params *params,
                      void *hip_stream, pdlp_batch **out);

/*
 * Same as pdlp_batch_create, with the eight data arrays (row_ptr, col, val,
 * c, lc, uc, lv, uv) in GPU memory, for instance torch tensors on the device
 * (host memory is accepted too).  The sizes m, n, nnz and obj_offset stay
 * host arrays: they fix how many bytes are read.  Validation and the packing
 * run on the host, so the arrays are first copied there on hip_stream,
 * after the work already queued on it; the caller keeps ownership and may
 * free them when the call returns.  The lengths are trusted: row_ptr_dev
 * must hold sum(m[i] + 1) entries, col_dev and val_dev sum(nnz[i]), c_dev,
 * lv_dev and uv_dev sum(n[i]), lc_dev and uc_dev sum(m[i]).  Errors as
 * pdlp_batch_create (the sizes are checked before anything is copied);
 * HIP_ERROR for a pointer the runtime cannot copy from.
 */
int pdlp_batch_create_device(int32_t count, const int32_t *m, const int32_t *n,
                             const int64_t *nnz, const int32_t *row_ptr_dev,
                             const int32_t *col_dev, const double *val_dev, const double *c_dev,
                             const double *lc_dev, const double *uc_dev, const double *lv_dev,
                             const double *uv_dev, const double *obj_offset_host,
                             const pdlp_params *params, void *hip_stream, pdlp_batch **out);

void pdlp_batch_destroy(pdlp_batch *b);

/* Instance count and batch totals. */
int pdlp_batch_dims(const pdlp_batch *b, int32_t *count, int64_t *m_total, int64_t *n_total,
                    int64_t *nnz_total);

/*
 * Solve every instance from (proj_X(0), 0) with the same params (NULL =
 * defaults; params->polish and params->restart_period must be 0, else
 * INVALID_ARGUMENT; max_iters and
 * time_limit apply to each instance, the time limit measured from the start
 * of the call).  results: `count` entries, filled as by pdlp_solve (their
 * x, y, r pointers are ignored and set to NULL; seconds is the wall time of
 * the whole batch).  x, r (sum(n[i])) and y (sum(m[i])) receive the unscaled
 * outputs concatenated in instance order, or may be NULL.  Repeated calls
 * solve again from the start and reuse the device work buffers.
 */
int pdlp_batch_solve(pdlp_batch *b, const pdlp_params *params, pdlp_result *results, double *x,
                     double *y, double *r);

/* Where the time of the last pdlp_batch_solve went.  A round advances every
 * unfinished instance to its next iteration-block boundary (step seconds),
 * then runs the checks of the instances at a boundary (check seconds). */
typedef struct pdlp_batch_stats {
    int64_t rounds;            /* iteration blocks run */
    int64_t attempt_launches;  /* step attempts enqueued (each serves every instance) */
    int64_t max_iterations;    /* accepted steps of the slowest instance */
    int64_t total_iterations;  /* accepted steps summed over instances */
    int64_t gap_evals;         /* normalized-duality-gap evaluations */
    int64_t gap_steps;         /* active-set steps they took */
    int64_t gap_capped;        /* evaluations that ended without an exact root (step cap) */
    double seconds, setup_seconds, step_seconds, check_seconds;
} pdlp_batch_stats;
int pdlp_batch_get_stats(const pdlp_batch *b, pdlp_batch_stats *stats);

/*
 * Differentiable unrolled PDHG over a batch of LPs.
 *
 * The map: K accepted steps of the PDHG update (Section 2, eq.
 * "specialized-pdhg" with tau = eta/omega, sigma = eta*omega, the case form
 * of the dual step) with the averages and restarts of Algorithm 1, from
 * (proj_X(0), 0), with every decision of a recorded Algorithm 1 run held
 * fixed: the step size eta and primal weight omega of each accepted step
 * (Algorithm 2, Algorithm 3) and each restart with its candidate (Section 3,
 * "Adaptive restarts").  Per instance it sends the data (c, lc, uc and the
 * nonzeros of A) to x_K (original units).  Its derivative treats the
 * projection onto the variable box and the case of the dual step as fixed
 * selections (derivative 1 strictly inside the box, 0 on it).  The diagonal
 * scalings D1, D2 are computed at creation (Ruiz + Pock-Chambolle) and are
 * constants: every scaled quantity is formed from the data as
 * A~_ij = (D1_i A_ij) D2_j, c~ = D2 c, (lc~, uc~) = D1 (lc, uc),
 * (lv~, uv~) = (lv, uv) / D2.
 */
typedef struct pdlp_unroll pdlp_unroll;   /* opaque: batch, data, tape, checkpoints */

/* Create from host arrays laid out as for pdlp_batch_create (no objective
 * offsets).  params: scaling parameters (NULL = defaults).  Errors as
 * pdlp_batch_create. */
int pdlp_unroll_create(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                       const int32_t *row_ptr_host, const int32_t *col_host,
                       const double *val_host, const double *c_host, const double *lc_host,
                       const double *uc_host, const double *lv_host, const double *uv_host,
                       const pdlp_params *params, void *hip_stream, pdlp_unroll **out);
/* The same from data arrays in GPU memory, staged on the host on hip_stream
 * as for pdlp_batch_create_device (sizes m, n, nnz on the host, lengths
 * trusted).  Errors as pdlp_batch_create_device. */
int pdlp_unroll_create_device(int32_t count, const int32_t *m, const int32_t *n,
                              const int64_t *nnz, const int32_t *row_ptr_dev,
                              const int32_t *col_dev, const double *val_dev,
                              const double *c_dev, const double *lc_dev, const double *uc_dev,
                              const double *lv_dev, const double *uv_dev,
                              const pdlp_params *params, void *hip_stream, pdlp_unroll **out);
void pdlp_unroll_destroy(pdlp_unroll *u);

/* Replace the data (original units, concatenated as at creation; any
 * pointer may be NULL to keep that part).  The sparsity pattern, lv, uv and
 * D1, D2 are unchanged.  Errors: INVALID_ARGUMENT for non-finite c or
 * values, NaN or inverted constraint bounds, a lower bound of +inf or an
 * upper bound of -inf. */
int pdlp_unroll_set_data(pdlp_unroll *u, const double *c, const double *lc, const double *uc,
                         const double *val);

/* Forward pass: Algorithm 1 with restart checks and no termination test
 * runs exactly K accepted steps on every instance (params: the algorithm's
 * constants, NULL = defaults; tolerances and polishing are not used),
 * recording its decisions and checkpointing the state every ckpt_every
 * steps.  x (sum n) receives x_K in original units, or may be NULL.
 * K >= 0, ckpt_every >= 1.  Errors: STATE on a numerical error;
 * INVALID_ARGUMENT for params->restart_period > 0. */
int pdlp_unroll_forward(pdlp_unroll *u, const pdlp_params *params, int64_t K, int32_t ckpt_every,
                        double *x);

/* The map at the current data with the recorded decisions: x (sum n) as in
 * pdlp_unroll_forward; signature (count entries, nullable) receives per
 * instance the number of (step, coordinate) pairs with x strictly inside its
 * box plus those where the dual step moves y, which identifies the fixed
 * selections (equal signatures for two data sets: same selections, in
 * practice).  Needs a forward pass. */
int pdlp_unroll_replay(pdlp_unroll *u, double *x, int64_t *signature);

/* Backward pass: given gx = dL/dx_K (sum n, original units), the gradients
 * of L with respect to c (sum n), lc and uc (sum m; 0 where the bound is
 * infinite) and the nonzeros of A (sum nnz, in the caller's CSR order), at
 * the current data along the recorded decisions.  Segments between
 * checkpoints are replayed, then reversed.  Outputs may be NULL. */
int pdlp_unroll_backward(pdlp_unroll *u, const double *gx, double *gc, double *glc,
                         double *guc, double *gval);

/* Tangent-linear map (forward mode) of the same linearization as
 * pdlp_unroll_backward: dx (sum n, original units) receives the directional
 * derivative of x_K along the data direction (dc (sum n), dlc, duc (sum m),
 * dval (sum nnz, CSR order), original units; NULL parts are zero), with the
 * recorded decisions and the replay's selections held fixed.  For any gx,
 * <dx, gx> equals the pairing of the direction with pdlp_unroll_backward's
 * gradients of <gx, x_K> up to rounding (the dot-product test).  Needs a
 * forward pass. */
int pdlp_unroll_tangent(pdlp_unroll *u, const double *dc, const double *dlc, const double *duc,
                        const double *dval, double *dx);

/* Device-memory variants of set_data, forward, backward and tangent, for
 * callers whose tensors live on the GPU (e.g. torch): the same arguments as
 * GPU pointers (same lengths and layouts; the data checks of set_data run
 * on the device).  The work runs on the library's stream after the work
 * queued on hip_stream so far (an event join; NULL or the library's own
 * stream: no join) and the call returns when its outputs are written, so
 * they may be used on hip_stream at once.  Errors as the host variants. */
int pdlp_unroll_set_data_device(pdlp_unroll *u, const double *c_dev, const double *lc_dev,
                                const double *uc_dev, const double *val_dev, void *hip_stream);
int pdlp_unroll_forward_device(pdlp_unroll *u, const pdlp_params *params, int64_t K,
                               int32_t ckpt_every, double *x_dev, void *hip_stream);
int pdlp_unroll_backward_device(pdlp_unroll *u, const double *gx_dev, double *gc_dev,
                                double *glc_dev, double *guc_dev, double *gval_dev,
                                void *hip_stream);
int pdlp_unroll_tangent_device(pdlp_unroll *u, const double *dc_dev, const double *dlc_dev,
                               const double *duc_dev, const double *dval_dev, double *dx_dev,
                               void *hip_stream);

/* Recorded decisions, count x K each (instance-major): eta and omega of
 * every accepted step; restart[i K + k] = 0, 1 (to the current iterate) or
 * 2 (to the average) for a restart right after step k. */
int pdlp_unroll_get_tape(const pdlp_unroll *u, double *eta, double *omega, int32_t *restart);

typedef struct pdlp_unroll_stats {
    int64_t K, ckpt, restarts;
    double forward_seconds;          /* pdlp_unroll_forward, before copying x out */
    double replay_seconds;           /* pdlp_unroll_replay, likewise */
    double backward_seconds;         /* pdlp_unroll_backward, after copying gx in, before copying out */
    double backward_replay_seconds;  /* its segment replays */
    double backward_reverse_seconds; /* its reverse steps */
    double tangent_seconds;          /* pdlp_unroll_tangent, after copying the direction in */
} pdlp_unroll_stats;
int pdlp_unroll_get_stats(const pdlp_unroll *u, pdlp_unroll_stats *stats);

/* Message for the last error on this thread ("" if none). */
const char *pdlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
