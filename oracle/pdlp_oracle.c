/*
 * FP64 CPU oracle for PDLP -- restarted, diagonally preconditioned PDHG for
 *     min c^T x  s.t.  lc <= A x <= uc,  lv <= x <= uv.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark; never by the product path.  It
 * shares no code with the GPU library.
 *
 * Written from the paper (Applegate et al., "PDLP: A Practical First-Order
 * Method for Large-Scale Linear Programming", arXiv 2501.07018):
 *   - problem form and dual sets Y, R ........ Section 2, eq. "lp"
 *   - PDHG step ................................ Section 2, eq. "specialized-pdhg"
 *                                                and the case form of the dual step
 *   - step reparameterization, omega-norm ..... Section 2
 *   - main loop ................................ Algorithm 1 (Section 3)
 *   - adaptive step ............................ Algorithm 2
 *   - normalized duality gap, restart
 *     candidate, restart criteria (i)-(iii) .... Section 3, "Adaptive restarts"
 *   - primal weight update / initialization ... Algorithm 3, "Initialization of
 *                                                the primal weights"
 *   - Ruiz + Pock-Chambolle preconditioning ... Section 3, "Diagonal Preconditioning"
 *   - feasibility polishing .................... Algorithm 4 (Section 4)
 *   - termination criteria ..................... Section 7, eq.
 *                                                "rescaled-termination-criteria"
 *   - relative gap ............................. Section 4, eq. "relative-gap"
 *   - reduced-cost choice ...................... Section 2 and Appendix A
 *   - infeasibility detection .................. Section 3, "Infeasibility
 *                                                detection", and Appendix D
 *   - fixed-frequency restarts ................. Algorithm 5 and Theorem 1
 *                                                (Appendix C)
 *
 * Readings of points the paper leaves open are listed in the design notes and
 * repeated at the place they apply ("reading: ...").
 *
 * Plain and sequential on purpose: every sum runs in index order, there is
 * no blocking or fusion, and the code is compiled with -ffp-contract=off.
 * The few OpenMP pragmas and the _OPENMP branch of orc_spmv_t matter only in
 * a separate threaded build of this file, used for the all-cores CPU
 * baseline (row shards as in the paper's Section 5); the build the tests use
 * ignores them.
 */
#include "pdlp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_LIMIT 1
#define ORC_NUMERR 3
#define ORC_PINF 4
#define ORC_DINF 5
#define ORC_POLISHED 10

static int is_fin(double v) { return isfinite(v); }

/* ------------------------------------------------------------ products */

/* out = A x, each row summed in column order starting from 0. */
void orc_spmv(const orc_lp *lp, const double *x, double *out) {
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t i = 0; i < lp->m; ++i) {
        double s = 0.0;
        for (int32_t p = lp->row_ptr[i]; p < lp->row_ptr[i + 1]; ++p)
            s += lp->val[p] * x[lp->col[p]];
        out[i] = s;
    }
}

/* out = A^T y; each column accumulates its terms in increasing row order.
 * The threaded build (OpenMP, for the all-cores CPU baseline only) follows
 * the paper's multithreading scheme (Section 5): T shards of consecutive
 * rows balanced by nonzeros, each accumulated in increasing row order into
 * its own vector, the shard vectors then added in shard order -- the same
 * products in a fixed order for a fixed T.  The plain build is the oracle. */
static void spmv_t_seq(const orc_lp *lp, const double *y, double *out, int32_t r0, int32_t r1) {
    for (int32_t i = r0; i < r1; ++i)
        for (int32_t p = lp->row_ptr[i]; p < lp->row_ptr[i + 1]; ++p)
            out[lp->col[p]] += lp->val[p] * y[i];
}

void orc_spmv_t(const orc_lp *lp, const double *y, double *out) {
    for (int32_t j = 0; j < lp->n; ++j) out[j] = 0.0;
#ifdef _OPENMP
    const int T = omp_get_max_threads();
    double *part = T > 1 ? malloc(sizeof(double) * (size_t)(T - 1) * (size_t)(lp->n + 1)) : NULL;
    if (part) {
        const int64_t nnz = lp->row_ptr[lp->m];
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            /* shard t: rows whose first entry lies in [t nnz / T, (t+1) nnz / T) */
            int32_t lo = 0, hi = lp->m;
            {
                const int64_t a = nnz * t / T, z = nnz * (t + 1) / T;
                int32_t l = 0, h = lp->m;
                while (l < h) { int32_t mid = l + (h - l) / 2; if (lp->row_ptr[mid] < a) l = mid + 1; else h = mid; }
                lo = l;
                l = 0; h = lp->m;
                while (l < h) { int32_t mid = l + (h - l) / 2; if (lp->row_ptr[mid] < z) l = mid + 1; else h = mid; }
                hi = t == T - 1 ? lp->m : l;
            }
            double *dst = t == 0 ? out : part + (size_t)(t - 1) * (size_t)(lp->n + 1);
            if (t > 0) memset(dst, 0, sizeof(double) * (size_t)lp->n);
            spmv_t_seq(lp, y, dst, lo, hi);
#pragma omp barrier
#pragma omp for schedule(static)
            for (int32_t j = 0; j < lp->n; ++j)
                for (int q = 1; q < T; ++q) out[j] += part[(size_t)(q - 1) * (size_t)(lp->n + 1) + j];
        }
        free(part);
        return;
    }
#endif
    spmv_t_seq(lp, y, out, 0, lp->m);
}

static double dot(const double *a, const double *b, int64_t len) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i] * b[i];
    return s;
}

static double dist2(const double *a, const double *b, int64_t len) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double d = a[i] - b[i];
        s += d * d;
    }
    return s;
}

static double clampd(double v, double lo, double hi) {
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

/* --------------------------------------------------- preconditioning */

/*
 * Diagonal preconditioning (Section 3, "Diagonal Preconditioning"):
 * A~ = D1 A D2.  `ruiz_iters` rounds of Ruiz scaling (row/column infinity
 * norms), then, if `pc` is set, one Pock-Chambolle round with alpha = 1
 * (row and column 1-norms).
 * Reading: in each round both factors come from the same current A~; a zero
 * norm gives factor 1; each entry is updated as a / (sqrt(rho_i)*sqrt(kappa_j)).
 * val is scaled in place; d1[m], d2[n] receive the accumulated diagonals.
 * Pins: after Ruiz every nonzero row/column has infinity norm -> 1; after
 * PC the spectral norm of A~ is at most 1.
 */
void orc_precondition(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col,
                      double *val, int32_t ruiz_iters, int32_t pc, double *d1, double *d2) {
    double *rn = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    double *cn = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int32_t i = 0; i < m; ++i) d1[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) d2[j] = 1.0;
    for (int32_t round = 0; round < ruiz_iters + (pc ? 1 : 0); ++round) {
        int use_inf = round < ruiz_iters;
        for (int32_t i = 0; i < m; ++i) rn[i] = 0.0;
        for (int32_t j = 0; j < n; ++j) cn[j] = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double a = fabs(val[p]);
                int32_t j = col[p];
                if (use_inf) {
                    if (a > rn[i]) rn[i] = a;
                    if (a > cn[j]) cn[j] = a;
                } else {
                    rn[i] += a;
                    cn[j] += a;
                }
            }
        }
        for (int32_t i = 0; i < m; ++i) rn[i] = rn[i] > 0.0 ? sqrt(rn[i]) : 1.0;
        for (int32_t j = 0; j < n; ++j) cn[j] = cn[j] > 0.0 ? sqrt(cn[j]) : 1.0;
        for (int32_t i = 0; i < m; ++i)
            for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                val[p] = val[p] / (rn[i] * cn[col[p]]);
        for (int32_t i = 0; i < m; ++i) d1[i] = d1[i] / rn[i];
        for (int32_t j = 0; j < n; ++j) d2[j] = d2[j] / cn[j];
    }
    free(rn);
    free(cn);
}

/*
 * Scaled problem vectors (Section 3): c~ = D2 c, (lc~, uc~) = D1 (lc, uc),
 * (lv~, uv~) = D2^{-1} (lv, uv).  Infinite bounds stay infinite.
 */
void orc_scale_vectors(int32_t m, int32_t n, const double *d1, const double *d2,
                       const double *c, const double *lc, const double *uc,
                       const double *lv, const double *uv, double *c_s, double *lc_s,
                       double *uc_s, double *lv_s, double *uv_s) {
    for (int32_t j = 0; j < n; ++j) {
        c_s[j] = d2[j] * c[j];
        lv_s[j] = is_fin(lv[j]) ? lv[j] / d2[j] : lv[j];
        uv_s[j] = is_fin(uv[j]) ? uv[j] / d2[j] : uv[j];
    }
    for (int32_t i = 0; i < m; ++i) {
        lc_s[i] = is_fin(lc[i]) ? d1[i] * lc[i] : lc[i];
        uc_s[i] = is_fin(uc[i]) ? d1[i] * uc[i] : uc[i];
    }
}

/* ------------------------------------------------------ initialization */

/*
 * InitializePrimalWeight (Section 3): ||c||_2 / ||Combine(lc, uc)||_2 when
 * both norms are positive, else 1; Combine_i = max{0, |lc_i|*, |uc_i|*}
 * where v* is |v| for finite v and 0 otherwise.
 */
double orc_initial_primal_weight(const orc_lp *lp) {
    double cc = 0.0, bb = 0.0;
    for (int32_t j = 0; j < lp->n; ++j) cc += lp->c[j] * lp->c[j];
    for (int32_t i = 0; i < lp->m; ++i) {
        double v = 0.0;
        double a = is_fin(lp->lc[i]) ? fabs(lp->lc[i]) : 0.0;
        double b = is_fin(lp->uc[i]) ? fabs(lp->uc[i]) : 0.0;
        if (a > v) v = a;
        if (b > v) v = b;
        bb += v * v;
    }
    double nc = sqrt(cc), nb = sqrt(bb);
    if (nc > 0.0 && nb > 0.0) return nc / nb;
    return 1.0;
}

/*
 * Initial state (Algorithm 1): eta_hat = 1/||A~||_inf, omega from
 * InitializePrimalWeight, z^{0,0} = (proj_X(0), 0).
 * Reading: ||A~||_inf is the largest absolute entry of the scaled matrix
 * (1 for an all-zero matrix); the initial point projects 0 onto the box.
 */
void orc_init_state(const orc_lp *lp, orc_state *st) {
    double amax = 0.0;
    for (int64_t p = 0; p < lp->row_ptr[lp->m]; ++p)
        if (fabs(lp->val[p]) > amax) amax = fabs(lp->val[p]);
    st->eta_hat = amax > 0.0 ? 1.0 / amax : 1.0;
    st->omega = orc_initial_primal_weight(lp);
    for (int32_t j = 0; j < lp->n; ++j) {
        st->x[j] = clampd(0.0, lp->lv[j], lp->uv[j]);
        st->x0[j] = st->x[j];
        st->sx[j] = 0.0;
    }
    for (int32_t i = 0; i < lp->m; ++i) {
        st->y[i] = 0.0;
        st->y0[i] = 0.0;
        st->sy[i] = 0.0;
    }
    orc_spmv(lp, st->x, st->ax);
    orc_spmv_t(lp, st->y, st->aty);
    st->seta = 0.0;
    st->k = st->t = st->n_outer = st->attempts = 0;
    st->kkt_passes = 1;
    st->mu_ref = INFINITY;
    st->mu_c_prev = INFINITY;
    st->restarts_i = st->restarts_ii = st->restarts_iii = 0;
    st->last_eta = 0.0;
    st->last_eta_bar = INFINITY;
}

/* ------------------------------------------------------------ PDHG step */

/*
 * Dual update in case form (Section 2, the case analysis after eq.
 * "specialized-pdhg"): with yhat = y - sigma A(2x'-x),
 *   y' = yhat + sigma*uc  if yhat < -sigma*uc,
 *        yhat + sigma*lc  if yhat > -sigma*lc,
 *        0                otherwise.
 * This equals yhat - sigma proj_[-uc,-lc](yhat/sigma) (the prox identity of
 * Appendix B) and always lands in Y.
 */
double orc_dual_case(double yhat, double sigma, double lc, double uc) {
    if (is_fin(uc)) {
        double su = sigma * uc;
        if (yhat < -su) return yhat + su;
    }
    if (is_fin(lc)) {
        double sl = sigma * lc;
        if (yhat > -sl) return yhat + sl;
    }
    return 0.0;
}

/*
 * One primal-dual candidate for step size eta (eq. "specialized-pdhg" with
 * tau = eta/omega, sigma = eta*omega).  Writes x', A x', y'; returns
 * num = ||z'-z||_omega^2 and the signed interaction cross = (y'-y)^T A (x'-x).
 */
static void pdhg_candidate(const orc_lp *lp, const orc_state *st, double eta,
                           double *xn, double *axn, double *yn, double *num, double *cross) {
    double tau = eta / st->omega, sigma = eta * st->omega;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < lp->n; ++j) {
        double g = lp->c[j] - st->aty[j];
        xn[j] = clampd(st->x[j] - tau * g, lp->lv[j], lp->uv[j]);
    }
    orc_spmv(lp, xn, axn);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < lp->m; ++i) {
        double yhat = st->y[i] - sigma * (2.0 * axn[i] - st->ax[i]);
        yn[i] = orc_dual_case(yhat, sigma, lp->lc[i], lp->uc[i]);
    }
    double dx2 = dist2(xn, st->x, lp->n);
    double dy2 = dist2(yn, st->y, lp->m);
    double cr = 0.0;
    for (int32_t i = 0; i < lp->m; ++i) cr += (yn[i] - st->y[i]) * (axn[i] - st->ax[i]);
    *num = st->omega * dx2 + dy2 / st->omega;
    *cross = cr;
}

static void trace_attempt(orc_trace *tr, int phase, const orc_state *st, double eta,
                          double eta_bar, double eta_next, double num, double cross, int acc) {
    if (!tr) return;
    int64_t q = tr->count++;
    if (q >= tr->cap) return;
    if (tr->attempt) tr->attempt[q] = st->attempts;
    if (tr->k) tr->k[q] = st->k;
    if (tr->eta) tr->eta[q] = eta;
    if (tr->eta_bar) tr->eta_bar[q] = eta_bar;
    if (tr->eta_next) tr->eta_next[q] = eta_next;
    if (tr->num) tr->num[q] = num;
    if (tr->cross) tr->cross[q] = cross;
    if (tr->accepted) tr->accepted[q] = acc;
    if (tr->phase) tr->phase[q] = phase;
}

/*
 * AdaptiveStepOfPDHG (Algorithm 2).
 *
 * Reading of the step test: the algorithm splits on the sign of
 * 2 (y'-y)^T A (x'-x).  With the paper's own conventions (Appendix B: the
 * saddle form with K = -A) PDHG is a proximal-point method in the metric
 * M = [[I/tau, A^T], [A, I/sigma]], and a step is safe when
 * ||z'-z||_M^2 = ||z'-z||_omega^2 / eta + 2 (y'-y)^T A (x'-x) >= 0; that
 * quantity is threatened when the interaction is negative, exactly the case
 * the printed rule accepts unconditionally.  The magnitude
 * |2 (y'-y)^T A (x'-x)| is used instead, so every accepted step keeps the
 * metric nonnegative and the stated bound eta_bar >= 1/||A||_2 holds.
 * (signed_step_rule = 1 follows the printed rule; the tests use it to show a
 * step it accepts with a negative metric.)
 *
 * Reading of the counter: the k in (1 - (k+1)^-0.3), (1 + (k+1)^-0.6) is the
 * number of step attempts made so far, incremented before use (the literal
 * first-iteration factor 1 - 1^-0.3 is 0 and would stall the method).
 *
 * Returns 0, or ORC_NUMERR when the step produced a non-finite value.  On
 * return the accepted candidate is the new iterate, and st->last_eta holds
 * the eta that was used.
 */
static int adaptive_step(const orc_lp *lp, const orc_params *prm, orc_state *st,
                         orc_scratch *scr, orc_trace *tr, int phase) {
    double eta = prm->fixed_step ? prm->fixed_eta : st->eta_hat;
    double *xn = scr->n0, *atyn = scr->n1, *yn = scr->m0, *axn = scr->m1;
    for (;;) {
        st->attempts += 1;
        double num, cross;
        pdhg_candidate(lp, st, eta, xn, axn, yn, &num, &cross);
        double den = prm->signed_step_rule ? 2.0 * cross : 2.0 * fabs(cross);
        if (!is_fin(num) || !is_fin(den)) {
            trace_attempt(tr, phase, st, eta, NAN, NAN, num, cross, 0);
            return ORC_NUMERR;
        }
        double eta_bar = den > 0.0 ? num / den : INFINITY;
        st->last_eta_bar = eta_bar;
        double jj = (double)(st->attempts + 1);
        double e1 = (1.0 - pow(jj, -prm->red_exp)) * eta_bar;
        double e2 = (1.0 + pow(jj, -prm->grow_exp)) * eta;
        double eta_next = e1 < e2 ? e1 : e2;
        int acc = prm->fixed_step || eta <= eta_bar;
        trace_attempt(tr, phase, st, eta, eta_bar, eta_next, num, cross, acc);
        if (acc) {
            orc_spmv_t(lp, yn, atyn);
            st->kkt_passes += 1;
            memcpy(st->x, xn, sizeof(double) * lp->n);
            memcpy(st->aty, atyn, sizeof(double) * lp->n);
            memcpy(st->y, yn, sizeof(double) * lp->m);
            memcpy(st->ax, axn, sizeof(double) * lp->m);
            st->last_eta = eta;
            st->eta_hat = prm->fixed_step ? prm->fixed_eta : eta_next;
            return ORC_OK;
        }
        eta = eta_next;
    }
}

int orc_adaptive_step(const orc_lp *lp, const orc_params *prm, orc_state *st,
                      orc_scratch *scr) {
    return adaptive_step(lp, prm, st, scr, NULL, 0);
}

/* ------------------------------------------------ normalized duality gap */

static int cmp_dbl(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

typedef struct {
    const orc_lp *lp;
    const double *x, *y, *g, *ax;
    double omega;
} gap_ctx;

/* Point on the path at parameter s (s > 0):
 *   x^_j(s) = clamp(x_j - s g_j / omega, lv_j, uv_j)
 *   y^_i(s) = y_i + s*omega*a_i if that is > 0, y_i + s*omega*b_i if that is < 0, else 0
 * with a_i = lc_i - (A x)_i (slope of the Lagrangian difference for positive
 * y^), b_i = uc_i - (A x)_i (slope for negative y^). */
static double path_x(const gap_ctx *q, int32_t j, double s) {
    double v = q->x[j] - s * q->g[j] / q->omega;
    return clampd(v, q->lp->lv[j], q->lp->uv[j]);
}

static double path_y(const gap_ctx *q, int32_t i, double s) {
    const orc_lp *lp = q->lp;
    if (is_fin(lp->lc[i])) {
        double a = lp->lc[i] - q->ax[i];
        double v = q->y[i] + s * q->omega * a;
        if (v > 0.0) return v;
    }
    if (is_fin(lp->uc[i])) {
        double b = lp->uc[i] - q->ax[i];
        double v = q->y[i] + s * q->omega * b;
        if (v < 0.0) return v;
    }
    return 0.0;
}

/* h_i(v) = v*(lc_i - (Ax)_i) for v > 0, v*(uc_i - (Ax)_i) for v < 0, 0 at 0. */
static double h_row(const gap_ctx *q, int32_t i, double v) {
    if (v > 0.0) return v * (q->lp->lc[i] - q->ax[i]);
    if (v < 0.0) return v * (q->lp->uc[i] - q->ax[i]);
    return 0.0;
}

/* D(s) = ||z^(s) - z||_omega^2 evaluated directly. */
static double path_D(const gap_ctx *q, double s) {
    double sx = 0.0, sy = 0.0;
    for (int32_t j = 0; j < q->lp->n; ++j) {
        double d = path_x(q, j, s) - q->x[j];
        sx += d * d;
    }
    for (int32_t i = 0; i < q->lp->m; ++i) {
        double d = path_y(q, i, s) - q->y[i];
        sy += d * d;
    }
    return q->omega * sx + sy / q->omega;
}

/* f(z^) = L(x, y^) - L(x^, y) = -g^T (x^ - x) + sum_i [h_i(y^_i) - h_i(y_i)]. */
static double path_f(const gap_ctx *q, double s) {
    double fx = 0.0, fy = 0.0;
    for (int32_t j = 0; j < q->lp->n; ++j) fx += -q->g[j] * (path_x(q, j, s) - q->x[j]);
    for (int32_t i = 0; i < q->lp->m; ++i) fy += h_row(q, i, path_y(q, i, s)) - h_row(q, i, q->y[i]);
    return fx + fy;
}

/*
 * Normalized duality gap mu(z, z_ref) = rho_r(z) with r = ||z - z_ref||_omega
 * (Section 3, "Adaptive restarts"):
 *     rho_r(z) = (1/r) max { L(x, y^) - L(x^, y) : z^ in X x Y, ||z^ - z||_omega <= r }.
 * The paper computes this with a cited linear-time routine that is not
 * reproduced in the paper; here the maximum is taken from its definition.
 * The objective is concave and separable, so the maximizer is the point on
 * the proximal path z^(s) (s >= 0, see path_x/path_y) whose distance
 * D(s) = ||z^(s)-z||_omega^2 equals r^2 (or the end of the path when
 * D(inf) <= r^2).  Between consecutive breakpoints D(s) = A s^2 + B; the
 * breakpoints are sorted, the segment containing r^2 is found by binary
 * search on directly evaluated D, A and B are read off by classifying each
 * coordinate at the segment midpoint, and s* = sqrt((r^2 - B)/A).
 * Reading: mu = 0 when r = 0.
 * Pins: brute-force maximization on tiny problems, mu(z*) = 0 at a planted
 * optimum, D(s*) = r^2, agreement with bisection on s.
 */
double orc_norm_gap(const orc_lp *lp, const double *x, const double *y, const double *ax,
                    const double *aty, const double *xr, const double *yr, double omega,
                    double *g_scratch, double *bp_scratch /* 2*(m+n) */) {
    double r2 = omega * dist2(x, xr, lp->n) + dist2(y, yr, lp->m) / omega;
    if (!(r2 > 0.0)) return 0.0;
    double r = sqrt(r2);
    for (int32_t j = 0; j < lp->n; ++j) g_scratch[j] = lp->c[j] - aty[j];
    gap_ctx q = {lp, x, y, g_scratch, ax, omega};
    /* breakpoints: where a coordinate stops, starts, or changes slope */
    int64_t nb = 0;
    for (int32_t j = 0; j < lp->n; ++j) {
        double g = g_scratch[j];
        double s = -1.0;
        if (g > 0.0 && is_fin(lp->lv[j])) s = omega * (x[j] - lp->lv[j]) / g;
        if (g < 0.0 && is_fin(lp->uv[j])) s = omega * (lp->uv[j] - x[j]) / (-g);
        if (s > 0.0 && is_fin(s)) bp_scratch[nb++] = s;
    }
    for (int32_t i = 0; i < lp->m; ++i) {
        if (is_fin(lp->lc[i])) {
            double a = lp->lc[i] - ax[i];
            if (a != 0.0) {
                double s = -y[i] / (omega * a);
                if (s > 0.0 && is_fin(s)) bp_scratch[nb++] = s;
            }
        }
        if (is_fin(lp->uc[i])) {
            double b = lp->uc[i] - ax[i];
            if (b != 0.0) {
                double s = -y[i] / (omega * b);
                if (s > 0.0 && is_fin(s)) bp_scratch[nb++] = s;
            }
        }
    }
    qsort(bp_scratch, (size_t)nb, sizeof(double), cmp_dbl);
    /* find the first breakpoint index with D(bp) >= r^2 */
    double s_lo = 0.0, s_hi = INFINITY;
    {
        int64_t lo = 0, hi = nb; /* answer in [lo, hi]; hi = nb means none */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (path_D(&q, bp_scratch[mid]) >= r2) hi = mid;
            else lo = mid + 1;
        }
        if (lo > 0) s_lo = bp_scratch[lo - 1];
        if (lo < nb) s_hi = bp_scratch[lo];
    }
    /* classify coordinates inside (s_lo, s_hi) */
    double s_mid = is_fin(s_hi) ? 0.5 * (s_lo + s_hi) : (s_lo > 0.0 ? 2.0 * s_lo : 1.0);
    double Acoef = 0.0, Bcoef = 0.0;
    for (int32_t j = 0; j < lp->n; ++j) {
        double g = g_scratch[j];
        double v = x[j] - s_mid * g / omega;
        if (g != 0.0 && v > lp->lv[j] && v < lp->uv[j]) {
            Acoef += g * g / omega;
        } else {
            double d = path_x(&q, j, s_mid) - x[j];
            Bcoef += omega * d * d;
        }
    }
    for (int32_t i = 0; i < lp->m; ++i) {
        double yh = path_y(&q, i, s_mid);
        if (yh != 0.0) {
            double slope = yh > 0.0 ? lp->lc[i] - ax[i] : lp->uc[i] - ax[i];
            Acoef += omega * slope * slope;
        } else {
            Bcoef += y[i] * y[i] / omega;
        }
    }
    double s_star;
    if (Acoef > 0.0) {
        s_star = sqrt((r2 - Bcoef) / Acoef);
        if (!(s_star >= s_lo)) s_star = s_lo;
        if (s_star > s_hi) s_star = s_hi;
    } else {
        /* nothing moves beyond s_lo: the path has ended inside the ball */
        s_star = s_lo > 0.0 ? s_lo : s_mid;
    }
    return path_f(&q, s_star) / r;
}

/* Bisection cross-check of the same quantity (60 halvings on s). */
double orc_norm_gap_bisect(const orc_lp *lp, const double *x, const double *y, const double *ax,
                           const double *aty, const double *xr, const double *yr,
                           double omega, double *g_scratch) {
    double r2 = omega * dist2(x, xr, lp->n) + dist2(y, yr, lp->m) / omega;
    if (!(r2 > 0.0)) return 0.0;
    for (int32_t j = 0; j < lp->n; ++j) g_scratch[j] = lp->c[j] - aty[j];
    gap_ctx q = {lp, x, y, g_scratch, ax, omega};
    double hi = 1.0;
    int grow = 0;
    while (path_D(&q, hi) < r2 && grow < 2000) { hi *= 2.0; ++grow; }
    if (grow == 2000) return path_f(&q, hi) / sqrt(r2);
    double lo = 0.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (path_D(&q, mid) < r2) lo = mid; else hi = mid;
    }
    return path_f(&q, lo) / sqrt(r2);
}

/* Expose D and f on the path for tests. */
double orc_path_value(const orc_lp *lp, const double *x, const double *y, const double *ax,
                      const double *aty, double omega, double s, int32_t which,
                      double *g_scratch, double *xhat, double *yhat) {
    for (int32_t j = 0; j < lp->n; ++j) g_scratch[j] = lp->c[j] - aty[j];
    gap_ctx q = {lp, x, y, g_scratch, ax, omega};
    if (xhat) for (int32_t j = 0; j < lp->n; ++j) xhat[j] = path_x(&q, j, s);
    if (yhat) for (int32_t i = 0; i < lp->m; ++i) yhat[i] = path_y(&q, i, s);
    return which == 0 ? path_D(&q, s) : path_f(&q, s);
}

/* ------------------------------------------------- termination criteria */

/*
 * KKT quantities in original units for a scaled point (x~, y~):
 * x = D2 x~, y = D1 y~ (reading: the dual unscaling follows from
 * y~^T A~ x~ = y^T A x), A x and A^T y recomputed with the original A.
 * Reduced costs (Section 2, Appendix A): mode 0 projects c - A^T y onto R;
 * mode 1 keeps (c - A^T y)_j only when x_j is within |x_j| of the matching
 * finite bound.
 * Relative primal residual: max_i violation_i / q_i with q from eq.
 * "rescaled-termination-criteria"; relative dual residual:
 * max_j |c - A^T y - r|_j / (|c_j| or 1).
 * Objectives: c^T x and -p(-y; lc, uc) - p(-r; lv, uv) = lc^T y+ - uc^T y-
 * + lv^T r+ - uv^T r- (terms with a zero multiplier contribute 0), both plus
 * the objective offset.  Relative gap per eq. "relative-gap" (reading: 0/0 = 0).
 * Scratch: n-length xo, atyo, ro; m-length yo, axo.
 */
void orc_kkt_eval(const orc_unscale *u, const double *xs, const double *ys, int32_t mode,
                  double *xo, double *ro, double *atyo, double *yo, double *axo, orc_kkt *out) {
    const orc_lp *lp = &u->orig;
    for (int32_t j = 0; j < lp->n; ++j) xo[j] = u->d2[j] * xs[j];
    for (int32_t i = 0; i < lp->m; ++i) yo[i] = u->d1[i] * ys[i];
    orc_spmv(lp, xo, axo);
    orc_spmv_t(lp, yo, atyo);
    double pres_abs = 0.0, pres_rel = 0.0;
    for (int32_t i = 0; i < lp->m; ++i) {
        double lc = lp->lc[i], uc = lp->uc[i];
        double viol = 0.0;
        if (is_fin(lc) && lc - axo[i] > viol) viol = lc - axo[i];
        if (is_fin(uc) && axo[i] - uc > viol) viol = axo[i] - uc;
        int l_big = is_fin(lc) && lc != 0.0;   /* lc not in {-inf, 0} */
        int u_big = is_fin(uc) && uc != 0.0;   /* uc not in {0, +inf} */
        double q;
        if (l_big && !u_big) q = fabs(lc);
        else if (!l_big && u_big) q = fabs(uc);
        else if (l_big && u_big) q = fabs(lc) > fabs(uc) ? fabs(lc) : fabs(uc);
        else q = 1.0;
        if (viol > pres_abs) pres_abs = viol;
        if (viol / q > pres_rel) pres_rel = viol / q;
    }
    double dres_abs = 0.0, dres_rel = 0.0;
    for (int32_t j = 0; j < lp->n; ++j) {
        double g = lp->c[j] - atyo[j];
        double lv = lp->lv[j], uv = lp->uv[j];
        double r;
        if (mode == 0) {
            /* projection onto R_j: {0}, R-, R+ or R by bound finiteness */
            if (!is_fin(lv) && !is_fin(uv)) r = 0.0;
            else if (!is_fin(lv)) r = g < 0.0 ? g : 0.0;
            else if (!is_fin(uv)) r = g > 0.0 ? g : 0.0;
            else r = g;
        } else {
            r = 0.0;
            if (g > 0.0 && xo[j] - lv <= fabs(xo[j])) r = g;
            if (g < 0.0 && uv - xo[j] <= fabs(xo[j])) r = g;
        }
        ro[j] = r;
        double res = fabs(g - r);
        double sc = lp->c[j] != 0.0 ? fabs(lp->c[j]) : 1.0;
        if (res > dres_abs) dres_abs = res;
        if (res / sc > dres_rel) dres_rel = res / sc;
    }
    double pobj = dot(lp->c, xo, lp->n) + u->obj_offset;
    double dobj = 0.0;
    for (int32_t i = 0; i < lp->m; ++i) {
        if (ys[i] > 0.0) dobj += lp->lc[i] * yo[i];
        else if (ys[i] < 0.0) dobj += lp->uc[i] * yo[i];
    }
    for (int32_t j = 0; j < lp->n; ++j) {
        if (ro[j] > 0.0) dobj += lp->lv[j] * ro[j];
        else if (ro[j] < 0.0) dobj += lp->uv[j] * ro[j];
    }
    dobj += u->obj_offset;
    double den = fabs(pobj) + fabs(dobj);
    out->primal_obj = pobj;
    out->dual_obj = dobj;
    out->rel_gap = den > 0.0 ? fabs(pobj - dobj) / den : 0.0;
    out->primal_res_abs = pres_abs;
    out->primal_res_rel = pres_rel;
    out->dual_res_abs = dres_abs;
    out->dual_res_rel = dres_rel;
}

/* ------------------------------------------ infeasibility certificates */

/*
 * Appendix D, primal infeasibility.  A point (y, r) in Y x R certifies it
 * when lc^T y+ - uc^T y- + lv^T r+ - uv^T r- > 0 and ||A^T y + r||_inf is at
 * most eps times that objective.
 *
 * Readings: the candidate arrives in the scaled space and is taken to
 * original units (y = D1 y~) on the instance as given; it is projected onto
 * Y (eq. "lp": {0}, R-, R+ or R by the finiteness of lc_i, uc_i), which
 * changes only components of the wrong sign; r is the projection of
 * -A^T y onto R, the reduced-cost rule of the dual objective with c = 0.
 * The paper states the test on instances rescaled so that objective entries
 * are -1, 0 or 1 (Section 6); on the instance as given that weights residual
 * component j by 1/|c_j| (1 where c_j = 0), the weights of the dual residual
 * in eq. "rescaled-termination-criteria", and leaves the objective unchanged.
 * Outputs: yo (m), atyo and ro (n), all original units.
 */
void orc_primal_infeas_test(const orc_unscale *u, const double *ys, double eps, double *yo,
                            double *atyo, double *ro, orc_cert *out) {
    const orc_lp *lp = &u->orig;
    for (int32_t i = 0; i < lp->m; ++i) {
        double y = u->d1[i] * ys[i];
        int lf = is_fin(lp->lc[i]), uf = is_fin(lp->uc[i]);
        if (!lf && !uf) y = 0.0;
        else if (!lf && y > 0.0) y = 0.0;      /* Y_i = R- */
        else if (!uf && y < 0.0) y = 0.0;      /* Y_i = R+ */
        yo[i] = y;
    }
    orc_spmv_t(lp, yo, atyo);
    double obj = 0.0, res = 0.0;
    for (int32_t i = 0; i < lp->m; ++i) {
        if (yo[i] > 0.0) obj += lp->lc[i] * yo[i];
        else if (yo[i] < 0.0) obj += lp->uc[i] * yo[i];
    }
    for (int32_t j = 0; j < lp->n; ++j) {
        double g = -atyo[j];
        int lf = is_fin(lp->lv[j]), uf = is_fin(lp->uv[j]);
        double r;
        if (!lf && !uf) r = 0.0;
        else if (!lf) r = g < 0.0 ? g : 0.0;   /* R_j = R- */
        else if (!uf) r = g > 0.0 ? g : 0.0;   /* R_j = R+ */
        else r = g;
        ro[j] = r;
        if (r > 0.0) obj += lp->lv[j] * r;
        else if (r < 0.0) obj += lp->uv[j] * r;
        double w = lp->c[j] != 0.0 ? fabs(lp->c[j]) : 1.0;
        double e = fabs(atyo[j] + r) / w;
        if (e > res || e != e) res = e;        /* NaN propagates */
    }
    out->obj = obj;
    out->res = res;
    out->ok = is_fin(obj) && is_fin(res) && obj > 0.0 && res <= eps * obj;
}

/*
 * Appendix D, dual infeasibility.  A point (x, s) in Xbar x Sbar certifies
 * it when c^T x < 0 and ||A x + s||_inf is at most eps |c^T x|; Xbar and Sbar
 * are the recession cones of the variable and constraint bounds.
 *
 * Readings: x = D2 x~ projected onto Xbar ({0} for boxed variables, R+ or R-
 * for one-sided ones, R for free ones); s is the projection of -A x onto
 * Sbar, so each residual component is the distance of -(A x)_i to Sbar_i.
 * As for the primal test, residual component i is weighted by 1/q_i with
 * the q of eq. "rescaled-termination-criteria" (the row scaling that takes
 * right-hand sides to -1, 0 or 1).  Outputs: xo (n), axo (m), original units.
 */
void orc_dual_infeas_test(const orc_unscale *u, const double *xs, double eps, double *xo,
                          double *axo, orc_cert *out) {
    const orc_lp *lp = &u->orig;
    for (int32_t j = 0; j < lp->n; ++j) {
        double x = u->d2[j] * xs[j];
        int lf = is_fin(lp->lv[j]), uf = is_fin(lp->uv[j]);
        if (lf && uf) x = 0.0;
        else if (lf && x < 0.0) x = 0.0;       /* Xbar_j = R+ */
        else if (uf && x > 0.0) x = 0.0;       /* Xbar_j = R- */
        xo[j] = x;
    }
    orc_spmv(lp, xo, axo);
    double res = 0.0;
    for (int32_t i = 0; i < lp->m; ++i) {
        double lc = lp->lc[i], uc = lp->uc[i];
        int lf = is_fin(lc), uf = is_fin(uc);
        double g = -axo[i], sv;
        if (lf && uf) sv = 0.0;
        else if (uf) sv = g > 0.0 ? g : 0.0;   /* Sbar_i = R+ */
        else if (lf) sv = g < 0.0 ? g : 0.0;   /* Sbar_i = R- */
        else sv = g;
        int l_big = lf && lc != 0.0, u_big = uf && uc != 0.0;
        double q;
        if (l_big && !u_big) q = fabs(lc);
        else if (!l_big && u_big) q = fabs(uc);
        else if (l_big && u_big) q = fabs(lc) > fabs(uc) ? fabs(lc) : fabs(uc);
        else q = 1.0;
        double e = fabs(axo[i] + sv) / q;
        if (e > res || e != e) res = e;
    }
    double obj = dot(lp->c, xo, lp->n);
    out->obj = obj;
    out->res = res;
    out->ok = is_fin(obj) && is_fin(res) && obj < 0.0 && res <= eps * fabs(obj);
}

/* ------------------------------------------------------------ main loop */

/*
 * PrimalWeightUpdate (Algorithm 3): with Delta_x = ||x^{n,0} - x^{n-1,0}||_2
 * and Delta_y likewise, return exp(theta log(Delta_y/Delta_x) + (1-theta)
 * log(omega)) when both lie in (eps_zero, 1/eps_zero), else omega.
 */
double orc_primal_weight_update(double dx, double dy, double omega, double theta, double ez) {
    if (dx > ez && dx < 1.0 / ez && dy > ez && dy < 1.0 / ez)
        return exp(theta * log(dy / dx) + (1.0 - theta) * log(omega));
    return omega;
}

enum { TERM_NONE = 0, TERM_FULL = 1, TERM_PRIMAL = 2, TERM_DUAL = 3 };

typedef struct {
    const orc_lp *lp;
    const orc_unscale *u;
    const orc_params *prm;
    orc_state *st;
    orc_scratch *scr;
    orc_tape *tape;                    /* optional record of the decisions */
    orc_trace *trace;                  /* optional trace of attempts and polishing */
    int phase;                         /* 0 main run, 1 primal / 2 dual feasibility sub-run */
    /* extra buffers */
    double *xb, *yb, *axb, *atyb;      /* average and its products */
    double *xp, *yp;                   /* previous restart point */
    double *gs, *bps;                  /* gap scratch */
    double *kx, *kr, *katy, *ky, *kax; /* kkt scratch */
    double *xprev, *yprev;             /* iterate before the latest accepted step */
    double *xc, *yc;                   /* infeasibility candidate */
} loop_ctx;

static int term_met(const loop_ctx *L, int mode, const orc_kkt *k) {
    double e = L->prm->eps_feas;
    if (mode == TERM_PRIMAL) return k->primal_res_rel <= e;
    if (mode == TERM_DUAL) return k->dual_res_rel <= e;
    return k->primal_res_rel <= e && k->dual_res_rel <= e && k->rel_gap <= L->prm->eps_gap;
}

static int all_finite(const double *a, int64_t len) {
    for (int64_t i = 0; i < len; ++i) if (!is_fin(a[i])) return 0;
    return 1;
}

static void compute_average(loop_ctx *L) {
    const orc_lp *lp = L->lp;
    orc_state *st = L->st;
    for (int32_t j = 0; j < lp->n; ++j) L->xb[j] = st->sx[j] / st->seta;
    for (int32_t i = 0; i < lp->m; ++i) L->yb[i] = st->sy[i] / st->seta;
    orc_spmv(lp, L->xb, L->axb);
    orc_spmv_t(lp, L->yb, L->atyb);
    st->kkt_passes += 1;
}

/* Projection of a scaled point onto Xbar x Y (sign-only, as in the tests). */
static void project_cones(const orc_lp *lp, const double *xs, const double *ys, double *px,
                          double *py) {
    for (int32_t j = 0; j < lp->n; ++j) {
        double x = xs[j];
        int lf = is_fin(lp->lv[j]), uf = is_fin(lp->uv[j]);
        if ((lf && uf) || (lf && x < 0.0) || (uf && x > 0.0)) x = 0.0;
        px[j] = x;
    }
    for (int32_t i = 0; i < lp->m; ++i) {
        double y = ys[i];
        int lf = is_fin(lp->lc[i]), uf = is_fin(lp->uc[i]);
        if ((!lf && !uf) || (!lf && y > 0.0) || (!uf && y < 0.0)) y = 0.0;
        py[i] = y;
    }
}

/*
 * Infeasibility detection (Section 3, "Infeasibility detection", with the
 * tests of Appendix D).  Three candidates, in this order: the difference of
 * the two latest iterates, the current iterate, and the average since the
 * last restart.  The paper normalizes the last two by the iteration count;
 * both tests are invariant under positive scaling of the candidate, so they
 * are tested as they are.  Reading: primal infeasibility is tested on all
 * three candidates before dual infeasibility.  Each candidate costs one
 * A x and one A^T y, counted as three KKT passes per check.  Returns 0,
 * ORC_PINF or ORC_DINF; on detection out_x/out_y (scaled) receive the
 * certifying candidate projected onto Xbar x Y.
 */
static int infeas_check(loop_ctx *L, double *out_x, double *out_y, orc_result *res) {
    const orc_lp *lp = L->lp;
    orc_state *st = L->st;
    st->kkt_passes += 3;
    const double eps = L->prm->eps_infeas;
    int32_t m = lp->m, n = lp->n;
    for (int32_t j = 0; j < n; ++j) L->xc[j] = st->x[j] - L->xprev[j];
    for (int32_t i = 0; i < m; ++i) L->yc[i] = st->y[i] - L->yprev[i];
    const double *cx[3] = {L->xc, st->x, L->xb};
    const double *cy[3] = {L->yc, st->y, L->yb};
    orc_cert ct;
    for (int pass = 0; pass < 2; ++pass) {
        for (int c = 0; c < 3; ++c) {
            if (pass == 0)
                orc_primal_infeas_test(L->u, cy[c], eps, L->ky, L->katy, L->kr, &ct);
            else
                orc_dual_infeas_test(L->u, cx[c], eps, L->kx, L->kax, &ct);
            if (!ct.ok) continue;
            project_cones(lp, cx[c], cy[c], out_x, out_y);
            res->cert_source = c + 1;
            res->cert_obj = ct.obj;
            res->cert_res = ct.res;
            return pass == 0 ? ORC_PINF : ORC_DINF;
        }
    }
    return 0;
}

static int pdlp_loop(loop_ctx *L, int64_t max_k, int term_mode, int allow_polish,
                     double *out_x, double *out_y, orc_kkt *out_kkt, orc_result *res);
static int alloc_ctx(loop_ctx *L, int32_t m, int32_t n);
static void free_ctx(loop_ctx *L);

/* Appends a polishing entry; returns its index or -1. */
static int64_t trace_polish(orc_trace *tr, int64_t k, double gap, int64_t cap) {
    if (!tr) return -1;
    int64_t q = tr->pcount++;
    if (q >= tr->pcap) return -1;
    if (tr->pol_k) tr->pol_k[q] = k;
    if (tr->pol_gap) tr->pol_gap[q] = gap;
    if (tr->pol_cap) tr->pol_cap[q] = cap;
    if (tr->pol_primal) tr->pol_primal[q] = -1;
    if (tr->pol_dual) tr->pol_dual[q] = -1;
    return q;
}

/*
 * Feasibility polishing (Algorithm 4), called after the k-th accepted step
 * for k = polish_first * 2^i once the relative gap of the average is below
 * eps_gap.  Primal feasibility LP (objective 0) from (x_bar, 0), then dual
 * feasibility LP (every finite bound set to 0, which leaves Y and R alone)
 * from (0, y_bar); each runs PDLP with the current omega and eta_hat for at
 * most floor(k/8) accepted steps or until its own residual passes (checked at
 * its start, every check_every steps and at the cap; reading).  The polished
 * pair is accepted when it meets the full termination criteria.
 */
static int feasibility_polish(loop_ctx *L, double *out_x, double *out_y, orc_kkt *out_kkt,
                              orc_result *res, int64_t pe) {
    const orc_lp *lp = L->lp;
    orc_state *st = L->st;
    int32_t m = lp->m, n = lp->n;
    int64_t cap = st->k / 8;
    res->polish_attempts += 1;
    /* sub-problem vectors */
    double *zc = calloc((size_t)n + 1, sizeof(double));
    double *lc0 = malloc(sizeof(double) * (m + 1)), *uc0 = malloc(sizeof(double) * (m + 1));
    double *lv0 = malloc(sizeof(double) * (n + 1)), *uv0 = malloc(sizeof(double) * (n + 1));
    for (int32_t i = 0; i < m; ++i) {
        lc0[i] = is_fin(lp->lc[i]) ? 0.0 : lp->lc[i];
        uc0[i] = is_fin(lp->uc[i]) ? 0.0 : lp->uc[i];
    }
    for (int32_t j = 0; j < n; ++j) {
        lv0[j] = is_fin(lp->lv[j]) ? 0.0 : lp->lv[j];
        uv0[j] = is_fin(lp->uv[j]) ? 0.0 : lp->uv[j];
    }
    /* sub-run state (own arrays) */
    size_t bn = sizeof(double) * (n + 1), bm = sizeof(double) * (m + 1);
    orc_state s2;
    memset(&s2, 0, sizeof s2);
    s2.x = malloc(bn); s2.aty = malloc(bn); s2.x0 = malloc(bn); s2.sx = malloc(bn);
    s2.y = malloc(bm); s2.ax = malloc(bm); s2.y0 = malloc(bm); s2.sy = malloc(bm);
    double *px = malloc(bn), *py = malloc(bm), *dx = malloc(bn), *dy = malloc(bm);
    int ok = 0;
    orc_params p2 = *L->prm;
    p2.polish = 0;
    p2.reduced_cost_mode = 0;
    /* the sub-runs get buffers of their own so the main average survives */
    loop_ctx Ls = *L;
    if (!alloc_ctx(&Ls, m, n)) { free_ctx(&Ls); return 0; }
    orc_kkt kk;
    orc_result r2;
    memset(&r2, 0, sizeof r2);

    /* primal feasibility problem: c = 0, start (x_bar, 0) */
    orc_lp lpP = *lp;
    lpP.c = zc;
    memcpy(s2.x, L->xb, bn - sizeof(double));
    for (int32_t i = 0; i < m; ++i) s2.y[i] = 0.0;
    int64_t base_passes = st->kkt_passes;
    {
        loop_ctx L2 = Ls;
        L2.lp = &lpP;
        L2.prm = &p2;
        L2.st = &s2;
        L2.phase = 1;
        orc_spmv(&lpP, s2.x, s2.ax);
        orc_spmv_t(&lpP, s2.y, s2.aty);
        memcpy(s2.x0, s2.x, bn - sizeof(double));
        memcpy(s2.y0, s2.y, bm - sizeof(double));
        memset(s2.sx, 0, bn); memset(s2.sy, 0, bm);
        s2.seta = 0.0; s2.omega = st->omega; s2.eta_hat = st->eta_hat;
        s2.k = s2.t = s2.n_outer = s2.attempts = 0; s2.kkt_passes = 1;
        s2.mu_ref = s2.mu_c_prev = INFINITY; s2.last_eta = 0.0;
        int rc = pdlp_loop(&L2, cap, TERM_PRIMAL, 0, px, py, &kk, &r2);
        res->polish_iters += s2.k;
        if (pe >= 0 && L->trace->pol_primal) L->trace->pol_primal[pe] = s2.k;
        base_passes += s2.kkt_passes;
        ok = (rc == ORC_OK);
    }
    if (ok) {
        orc_lp lpD = *lp;
        lpD.lc = lc0; lpD.uc = uc0; lpD.lv = lv0; lpD.uv = uv0;
        for (int32_t j = 0; j < n; ++j) s2.x[j] = 0.0;
        memcpy(s2.y, L->yb, bm - sizeof(double));
        loop_ctx L2 = Ls;
        L2.lp = &lpD;
        L2.prm = &p2;
        L2.st = &s2;
        L2.phase = 2;
        orc_spmv(&lpD, s2.x, s2.ax);
        orc_spmv_t(&lpD, s2.y, s2.aty);
        memcpy(s2.x0, s2.x, bn - sizeof(double));
        memcpy(s2.y0, s2.y, bm - sizeof(double));
        memset(s2.sx, 0, bn); memset(s2.sy, 0, bm);
        s2.seta = 0.0; s2.omega = st->omega; s2.eta_hat = st->eta_hat;
        s2.k = s2.t = s2.n_outer = s2.attempts = 0; s2.kkt_passes = 1;
        s2.mu_ref = s2.mu_c_prev = INFINITY; s2.last_eta = 0.0;
        int rc = pdlp_loop(&L2, cap, TERM_DUAL, 0, dx, dy, &kk, &r2);
        res->polish_iters += s2.k;
        if (pe >= 0 && L->trace->pol_dual) L->trace->pol_dual[pe] = s2.k;
        base_passes += s2.kkt_passes;
        ok = (rc == ORC_OK);
    }
    st->kkt_passes = base_passes;
    if (ok) {
        orc_kkt_eval(L->u, px, dy, 0, L->kx, L->kr, L->katy, L->ky, L->kax, &kk);
        if (term_met(L, TERM_FULL, &kk)) {
            memcpy(out_x, px, sizeof(double) * n);
            memcpy(out_y, dy, sizeof(double) * m);
            *out_kkt = kk;
        } else {
            ok = 0;
        }
    }
    free_ctx(&Ls);
    free(zc); free(lc0); free(uc0); free(lv0); free(uv0);
    free(s2.x); free(s2.aty); free(s2.x0); free(s2.sx);
    free(s2.y); free(s2.ax); free(s2.y0); free(s2.sy);
    free(px); free(py); free(dx); free(dy);
    return ok;
}

/*
 * Algorithm 1 with the periodic checks of Section 3: condition (iii) after
 * every accepted step; conditions (i), (ii) and termination every
 * check_every accepted steps; termination also at the start, at the
 * iteration cap (term modes only) and on numerical error.
 * Readings: at n = 0 only (iii) applies; mu_c_prev in (ii) is the candidate
 * gap of the previous evaluation in the same outer loop (+inf at the first);
 * a restart takes the candidate, then updates omega (Algorithm 3), then sets
 * mu_ref = mu(z^{n,0}, z^{n-1,0}) under the new omega; a tie in
 * GetRestartCandidate goes to the average; rejected attempts advance no
 * counter of Algorithm 1.
 */
/*
 * Check of Algorithm 5 (Appendix C): a constant step (fixed_step) and a
 * constant primal weight, and after every restart_period steps a restart to
 * the plain average of x with y reset to 0 (the constant step makes the
 * step-weighted average of Algorithm 1 the plain average).  No adaptive
 * restart criteria and no primal weight update.  Readings: the termination
 * test (at the usual cadence) takes the point a restart would produce,
 * (x average, 0), as its candidate (for c = 0 this is optimal exactly when x
 * is feasible: y = 0, r = 0 is dual feasible with the primal objective 0);
 * the restart follows it at the same k; restarts are counted as (iii).
 * Returns a status, or -1 to continue.
 */
static int fixed_period_check(loop_ctx *L, int full, int per, int capchk, int term_mode,
                              int detect, double *out_x, double *out_y, orc_kkt *out_kkt,
                              orc_result *res) {
    const orc_lp *lp = L->lp;
    orc_state *st = L->st;
    int32_t m = lp->m, n = lp->n;
    if ((full || capchk) && term_mode != TERM_NONE) {
        orc_kkt kk;
        memset(L->yc, 0, sizeof(double) * m);
        orc_kkt_eval(L->u, L->xb, L->yc, L->prm->reduced_cost_mode, L->kx, L->kr, L->katy,
                     L->ky, L->kax, &kk);
        memcpy(out_x, L->xb, sizeof(double) * n);
        memset(out_y, 0, sizeof(double) * m);
        *out_kkt = kk;
        if (term_met(L, term_mode, &kk)) return ORC_OK;
        if (detect) {
            int inf = infeas_check(L, out_x, out_y, res);
            if (inf) return inf;
        }
        if (capchk) return ORC_LIMIT;
    }
    if (!per) return -1;
    st->restarts_iii += 1;
    if (L->tape && st->k - 1 < L->tape->cap) L->tape->restart[st->k - 1] = 2;
    memcpy(st->x, L->xb, sizeof(double) * n);
    memcpy(st->ax, L->axb, sizeof(double) * m);
    memset(st->y, 0, sizeof(double) * m);
    memset(st->aty, 0, sizeof(double) * n);
    memcpy(st->x0, st->x, sizeof(double) * n);
    memset(st->y0, 0, sizeof(double) * m);
    st->n_outer += 1;
    st->t = 0;
    st->seta = 0.0;
    memset(st->sx, 0, sizeof(double) * n);
    memset(st->sy, 0, sizeof(double) * m);
    return -1;
}

static int pdlp_loop(loop_ctx *L, int64_t max_k, int term_mode, int allow_polish,
                     double *out_x, double *out_y, orc_kkt *out_kkt, orc_result *res) {
    const orc_lp *lp = L->lp;
    const orc_params *prm = L->prm;
    orc_state *st = L->st;
    int32_t m = lp->m, n = lp->n;
    int mode_rc = prm->reduced_cost_mode;
    orc_kkt kk;
    int64_t next_polish = prm->polish_first;
    while (allow_polish && next_polish <= st->k) next_polish *= 2;

    if (term_mode != TERM_NONE) {
        orc_kkt_eval(L->u, st->x, st->y, mode_rc, L->kx, L->kr, L->katy, L->ky, L->kax, &kk);
        memcpy(out_x, st->x, sizeof(double) * n);
        memcpy(out_y, st->y, sizeof(double) * m);
        *out_kkt = kk;
        if (term_met(L, term_mode, &kk)) return ORC_OK;
        if (st->k >= max_k) return ORC_LIMIT;
    }
    const int detect = term_mode == TERM_FULL && prm->detect_infeas;
    const int fixed_period = prm->restart_period > 0;
    if (fixed_period) st->omega = prm->fixed_omega;
    while (st->k < max_k) {
        if (detect) {
            memcpy(L->xprev, st->x, sizeof(double) * n);
            memcpy(L->yprev, st->y, sizeof(double) * m);
        }
        int rc = adaptive_step(lp, prm, st, L->scr, L->trace, L->phase);
        if (rc != ORC_OK) return ORC_NUMERR;
        double eta = st->last_eta;
        if (L->tape && st->k < L->tape->cap) {
            L->tape->eta[st->k] = eta;
            L->tape->omega[st->k] = st->omega;
            L->tape->restart[st->k] = 0;
        }
        st->seta += eta;
        for (int32_t j = 0; j < n; ++j) st->sx[j] += eta * st->x[j];
        for (int32_t i = 0; i < m; ++i) st->sy[i] += eta * st->y[i];
        st->t += 1;
        st->k += 1;

        int full = (st->k % prm->check_every) == 0;
        int art = !fixed_period && (double)st->t >= prm->beta_art * (double)st->k;
        int per = fixed_period && st->t >= prm->restart_period;
        int capchk = (term_mode != TERM_NONE) && st->k == max_k;
        int pol = !fixed_period && allow_polish && prm->polish && st->k == next_polish;
        if (!(full || art || per || capchk || pol)) continue;

        compute_average(L);
        if (!all_finite(L->xb, n) || !all_finite(L->yb, m)) return ORC_NUMERR;
        if (fixed_period) {
            int rc = fixed_period_check(L, full, per, capchk, term_mode, detect, out_x, out_y,
                                        out_kkt, res);
            if (rc >= 0) return rc;
            continue;
        }

        if (pol) {
            next_polish *= 2;
            orc_kkt_eval(L->u, L->xb, L->yb, 0, L->kx, L->kr, L->katy, L->ky, L->kax, &kk);
            int64_t pe = trace_polish(L->trace, st->k, kk.rel_gap, st->k / 8);
            if (kk.rel_gap < prm->eps_gap) {
                if (feasibility_polish(L, out_x, out_y, out_kkt, res, pe)) {
                    res->polished = 1;
                    return ORC_POLISHED;
                }
            }
            if (!(full || art || capchk)) continue;
        }

        double mu_cur = orc_norm_gap(lp, st->x, st->y, st->ax, st->aty, st->x0, st->y0,
                                     st->omega, L->gs, L->bps);
        double mu_avg = orc_norm_gap(lp, L->xb, L->yb, L->axb, L->atyb, st->x0, st->y0,
                                     st->omega, L->gs, L->bps);
        if (!is_fin(mu_cur) || !is_fin(mu_avg)) return ORC_NUMERR;
        int use_cur = mu_cur < mu_avg;
        double mu_c = use_cur ? mu_cur : mu_avg;
        const double *cx = use_cur ? st->x : L->xb;
        const double *cy = use_cur ? st->y : L->yb;

        if ((full || capchk) && term_mode != TERM_NONE) {
            orc_kkt_eval(L->u, cx, cy, mode_rc, L->kx, L->kr, L->katy, L->ky, L->kax, &kk);
            memcpy(out_x, cx, sizeof(double) * n);
            memcpy(out_y, cy, sizeof(double) * m);
            *out_kkt = kk;
            if (term_met(L, term_mode, &kk)) return ORC_OK;
            if (detect) {
                int inf = infeas_check(L, out_x, out_y, res);
                if (inf) return inf;
            }
            if (capchk) return ORC_LIMIT;
        }

        int restart = 0, why = 0;
        if (!prm->adaptive_restarts || st->n_outer == 0) {
            if (art) { restart = 1; why = 3; }
        } else {
            if (full && mu_c <= prm->beta_suff * st->mu_ref) { restart = 1; why = 1; }
            else if (full && mu_c <= prm->beta_nec * st->mu_ref && mu_c > st->mu_c_prev) {
                restart = 1; why = 2;
            } else if (art) { restart = 1; why = 3; }
        }
        if (!restart) {
            if (full) st->mu_c_prev = mu_c;
            continue;
        }
        if (why == 1) st->restarts_i += 1;
        if (why == 2) st->restarts_ii += 1;
        if (why == 3) st->restarts_iii += 1;
        if (L->tape && st->k - 1 < L->tape->cap) L->tape->restart[st->k - 1] = use_cur ? 1 : 2;
        /* previous restart point */
        memcpy(L->xp, st->x0, sizeof(double) * n);
        memcpy(L->yp, st->y0, sizeof(double) * m);
        if (!use_cur) {
            memcpy(st->x, L->xb, sizeof(double) * n);
            memcpy(st->y, L->yb, sizeof(double) * m);
            memcpy(st->ax, L->axb, sizeof(double) * m);
            memcpy(st->aty, L->atyb, sizeof(double) * n);
        }
        memcpy(st->x0, st->x, sizeof(double) * n);
        memcpy(st->y0, st->y, sizeof(double) * m);
        double dxn = sqrt(dist2(st->x0, L->xp, n));
        double dyn = sqrt(dist2(st->y0, L->yp, m));
        st->omega = orc_primal_weight_update(dxn, dyn, st->omega, prm->theta, prm->eps_zero);
        st->n_outer += 1;
        st->t = 0;
        st->seta = 0.0;
        memset(st->sx, 0, sizeof(double) * n);
        memset(st->sy, 0, sizeof(double) * m);
        st->mu_ref = orc_norm_gap(lp, st->x0, st->y0, st->ax, st->aty, L->xp, L->yp,
                                  st->omega, L->gs, L->bps);
        st->mu_c_prev = INFINITY;
    }
    return ORC_LIMIT;
}

static int alloc_ctx(loop_ctx *L, int32_t m, int32_t n) {
    size_t bn = sizeof(double) * ((size_t)n + 1), bm = sizeof(double) * ((size_t)m + 1);
    L->xb = malloc(bn); L->atyb = malloc(bn); L->xp = malloc(bn); L->gs = malloc(bn);
    L->kx = malloc(bn); L->kr = malloc(bn); L->katy = malloc(bn);
    L->yb = malloc(bm); L->axb = malloc(bm); L->yp = malloc(bm);
    L->ky = malloc(bm); L->kax = malloc(bm);
    L->xprev = malloc(bn); L->xc = malloc(bn);
    L->yprev = malloc(bm); L->yc = malloc(bm);
    L->bps = malloc(sizeof(double) * (2 * ((size_t)m + n) + 1));
    return L->xb && L->atyb && L->xp && L->gs && L->kx && L->kr && L->katy && L->yb &&
           L->axb && L->yp && L->ky && L->kax && L->bps && L->xprev && L->xc && L->yprev &&
           L->yc;
}

static void free_ctx(loop_ctx *L) {
    free(L->xb); free(L->atyb); free(L->xp); free(L->gs); free(L->kx); free(L->kr);
    free(L->katy); free(L->yb); free(L->axb); free(L->yp); free(L->ky); free(L->kax);
    free(L->bps); free(L->xprev); free(L->xc); free(L->yprev); free(L->yc);
}

/*
 * Run PDLP on a scaled problem from state `st` (prepared by orc_init_state or
 * by earlier calls).  With prm->terminate == 0 runs exactly
 * max_iters - st->k further accepted steps with restart checks and no
 * termination test.  out_x/out_y (scaled, caller owned) receive the returned
 * point (the candidate of the last termination evaluation; the current
 * iterate in the no-termination mode; the certificate on an infeasible
 * status).  Returns the status code.  When
 * `tape` is not NULL the decisions of every accepted step are recorded in it
 * (see orc_tape); when `trace` is not NULL every step attempt and every
 * polishing point are appended to it (see orc_trace).
 */
int32_t orc_pdlp_trace(const orc_lp *lp, const orc_unscale *u, const orc_params *prm,
                       orc_state *st, orc_scratch *scr, double *out_x, double *out_y,
                       orc_result *res, orc_tape *tape, orc_trace *trace) {
    loop_ctx L;
    memset(&L, 0, sizeof L);
    L.lp = lp; L.u = u; L.prm = prm; L.st = st; L.scr = scr; L.tape = tape; L.trace = trace;
    if (!alloc_ctx(&L, lp->m, lp->n)) { free_ctx(&L); return -3; }
    orc_kkt kk;
    memset(&kk, 0, sizeof kk);
    res->cert_source = 0;
    res->cert_obj = res->cert_res = 0.0;
    int term_mode = prm->terminate ? TERM_FULL : TERM_NONE;
    int rc = pdlp_loop(&L, prm->max_iters, term_mode, prm->polish && prm->terminate,
                       out_x, out_y, &kk, res);
    if (term_mode == TERM_NONE) {
        memcpy(out_x, st->x, sizeof(double) * lp->n);
        memcpy(out_y, st->y, sizeof(double) * lp->m);
        orc_kkt_eval(u, st->x, st->y, prm->reduced_cost_mode, L.kx, L.kr, L.katy, L.ky, L.kax, &kk);
    }
    res->status = rc == ORC_POLISHED ? 0 : rc;
    res->iterations = st->k;
    res->attempts = st->attempts;
    res->kkt_passes = st->kkt_passes;
    res->restarts = st->restarts_i + st->restarts_ii + st->restarts_iii;
    res->restarts_i = st->restarts_i;
    res->restarts_ii = st->restarts_ii;
    res->restarts_iii = st->restarts_iii;
    res->primal_obj = kk.primal_obj;
    res->dual_obj = kk.dual_obj;
    res->rel_gap = kk.rel_gap;
    res->primal_res_abs = kk.primal_res_abs;
    res->primal_res_rel = kk.primal_res_rel;
    res->dual_res_abs = kk.dual_res_abs;
    res->dual_res_rel = kk.dual_res_rel;
    res->omega = st->omega;
    res->eta = st->eta_hat;
    free_ctx(&L);
    return res->status;
}

/* orc_pdlp_trace without a trace. */
int32_t orc_pdlp_record(const orc_lp *lp, const orc_unscale *u, const orc_params *prm,
                        orc_state *st, orc_scratch *scr, double *out_x, double *out_y,
                        orc_result *res, orc_tape *tape) {
    return orc_pdlp_trace(lp, u, prm, st, scr, out_x, out_y, res, tape, NULL);
}

/* orc_pdlp_record without a record. */
int32_t orc_pdlp(const orc_lp *lp, const orc_unscale *u, const orc_params *prm, orc_state *st,
                 orc_scratch *scr, double *out_x, double *out_y, orc_result *res) {
    return orc_pdlp_record(lp, u, prm, st, scr, out_x, out_y, res, NULL);
}
