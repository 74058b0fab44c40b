/*
 * FP64 CPU oracle for PDLP (restarted, diagonally preconditioned PDHG).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code with the GPU library.
 *
 * Precision: IEEE binary64 throughout, compiled with -ffp-contract=off, all
 * sums accumulated sequentially in index order.
 *
 * Problem form (paper, Section 2, eq. "lp"):
 *     min c^T x  s.t.  lc <= A x <= uc,  lv <= x <= uv
 * Absent bounds are +-HUGE_VAL.  A is CSR (int32 row_ptr/col, double val)
 * with strictly increasing columns inside each row.
 *
 * Parity status of each function is stated in the function comment in
 * pdlp_oracle.c.
 */
#ifndef PDLP_ORACLE_H
#define PDLP_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t m, n;
    const int32_t *row_ptr, *col;
    const double *val;
    const double *c, *lc, *uc, *lv, *uv;
} orc_lp;

typedef struct {
    double eps_feas, eps_gap;      /* termination tolerances */
    int64_t max_iters;             /* limit on accepted steps */
    int32_t check_every;           /* cadence of restart/termination checks (64) */
    int32_t terminate;             /* 0: run exactly max_iters steps, no termination test */
    double beta_suff, beta_nec, beta_art;   /* 0.1, 0.9, 0.5 */
    double theta, eps_zero;        /* 0.5, 1e-10 */
    double red_exp, grow_exp;      /* 0.3, 0.6 */
    int32_t reduced_cost_mode;     /* 0: projection onto R, 1: Appendix A choice */
    int32_t polish;                /* feasibility polishing on/off */
    int64_t polish_first;          /* 100 */
    int32_t fixed_step;            /* test mode: constant eta, no adaptive rule */
    double fixed_eta;
    int32_t adaptive_restarts;     /* 0: only condition (iii) */
    int32_t detect_infeas;         /* Appendix D tests at every termination check */
    double eps_infeas;             /* their threshold (1e-9) */
    int64_t restart_period;        /* > 0: Algorithm 5 (Appendix C) restarts every that
                                      many steps; needs fixed_step */
    double fixed_omega;            /* primal weight held in that mode */
    int32_t signed_step_rule;      /* 0 (default): eta_bar from |2 (y'-y)^T A (x'-x)|;
                                      1: the printed signed rule (eta_bar = inf when that
                                      product is <= 0), kept only so that the tests can show
                                      which steps it accepts (see orc_adaptive_step) */
} orc_params;

/* Iterate state; every array is owned by the caller. */
typedef struct {
    double *x, *y, *ax, *aty;      /* current z^{n,t} and cached A x, A^T y (scaled) */
    double *x0, *y0;               /* restart point z^{n,0} */
    double *sx, *sy;               /* sums of eta_i x^i and eta_i y^i since restart */
    double seta;                   /* sum of eta_i */
    double omega, eta_hat;
    int64_t k, t, n_outer, attempts, kkt_passes;
    double mu_ref, mu_c_prev;
    int64_t restarts_i, restarts_ii, restarts_iii;
    double last_eta;               /* eta of the last accepted step */
    double last_eta_bar;           /* eta_bar of the last attempt */
} orc_state;

/* Scratch arrays (caller owned): 6 of length n, 6 of length m. */
typedef struct {
    double *n0, *n1, *n2, *n3, *n4, *n5;
    double *m0, *m1, *m2, *m3, *m4, *m5;
} orc_scratch;

/* Original-unit data for termination criteria. */
typedef struct {
    orc_lp orig;                   /* unscaled problem */
    const double *d1, *d2;         /* diagonal scalings, A~ = D1 A D2 */
    double obj_offset;
} orc_unscale;

typedef struct {
    int32_t status;                /* 0 optimal, 1 iteration limit, 3 numerical error,
                                      4 primal infeasible, 5 dual infeasible */
    int64_t iterations, attempts, kkt_passes;
    int64_t restarts, restarts_i, restarts_ii, restarts_iii;
    double primal_obj, dual_obj, rel_gap;
    double primal_res_abs, primal_res_rel, dual_res_abs, dual_res_rel;
    double omega, eta;
    int64_t polish_attempts, polish_iters;
    int32_t polished;
    int32_t cert_source;           /* infeasible status: 1 difference of consecutive
                                      iterates, 2 current iterate, 3 average */
    double cert_obj, cert_res;     /* objective and weighted residual of that certificate */
} orc_result;

typedef struct {
    double primal_obj, dual_obj, rel_gap;
    double primal_res_abs, primal_res_rel, dual_res_abs, dual_res_rel;
} orc_kkt;

/*
 * Decisions of an Algorithm 1 run, recorded per accepted step k = 0 .. cap-1
 * (caller-owned arrays): the step size eta and primal weight omega the step
 * used, and restart[k] = 0 (none), 1 (restart to the current iterate) or 2
 * (restart to the average) for a restart taken right after that step.
 */
typedef struct {
    int64_t cap;
    double *eta, *omega;
    int32_t *restart;
} orc_tape;

/*
 * Optional trace of a run (caller-owned arrays, NULL pointers allowed).
 *
 * Every step attempt of Algorithm 2, main run and polishing sub-runs alike,
 * appends one entry while count < cap: the attempt counter j that entered
 * the factors (1 - (j+1)^-red_exp), (1 + (j+1)^-grow_exp), the trial step
 * eta, the test value eta_bar, the next step eta', the movement
 * num = ||z'-z||_omega^2, the signed interaction cross = (y'-y)^T A (x'-x),
 * whether the attempt was accepted, the phase (0 main run, 1 primal
 * feasibility sub-run, 2 dual feasibility sub-run) and the phase's accepted
 * count k before the attempt.  `count` keeps counting past cap.
 *
 * Every feasibility-polishing point of Algorithm 4 (main-run k = polish_first
 * * 2^i) appends one polishing entry while pcount < pcap: that k, the
 * relative gap of the average tested against eps_gap, the sub-run cap, and
 * the accepted steps of the primal and dual sub-runs (-1 when not run).
 */
typedef struct {
    int64_t cap, count;
    int64_t *attempt, *k;
    double *eta, *eta_bar, *eta_next, *num, *cross;
    int32_t *accepted, *phase;
    int64_t pcap, pcount;
    int64_t *pol_k, *pol_cap, *pol_primal, *pol_dual;
    double *pol_gap;
} orc_trace;

/*
 * Outcome of one Appendix D test: `obj` is the certificate's objective
 * (primal test: lc^T y+ - uc^T y- + lv^T r+ - uv^T r-; dual test: c^T x),
 * `res` the largest weighted residual component, `ok` 1 when the candidate
 * certifies infeasibility at the threshold.
 */
typedef struct {
    double obj, res;
    int32_t ok;
} orc_cert;

void orc_primal_infeas_test(const orc_unscale *u, const double *ys, double eps, double *yo,
                            double *atyo, double *ro, orc_cert *out);
void orc_dual_infeas_test(const orc_unscale *u, const double *xs, double eps, double *xo,
                          double *axo, orc_cert *out);

/* Sparse products and the dual case step (pdlp_oracle.c). */
void orc_spmv(const orc_lp *lp, const double *x, double *out);
void orc_spmv_t(const orc_lp *lp, const double *y, double *out);
double orc_dual_case(double yhat, double sigma, double lc, double uc);

#endif
