/*
 * FP64 CPU oracle for the unrolled, differentiable PDHG map.
 *
 * TEST INFRASTRUCTURE ONLY (see pdlp_oracle.c).  Shares no code with the GPU
 * library.
 *
 * The map.  With the decisions of an Algorithm 1 run held fixed (the step
 * size eta_k and primal weight omega_k of every accepted step, and the
 * restarts with their choice of candidate), K accepted steps send the
 * scaled data (c~, lc~, uc~, A~) to the iterate x_K:
 *
 *   tau = eta_k / omega_k, sigma = eta_k * omega_k                (Section 2)
 *   v    = x - tau (c~ - A~^T y),            x+ = proj_[lv~, uv~](v)
 *   yhat = y - sigma A~ (2 x+ - x),          y+ = dual case step of yhat
 *   Sx += eta_k x+, Sy += eta_k y+, S += eta_k                    (Algorithm 1)
 *   restart to the average: (x, y) <- (Sx, Sy) / S;  any restart: sums <- 0
 *
 * starting from x_0 = proj_X(0), y_0 = 0.  The products A~x and A~^T y used
 * by the next step are those of the current point, so they are functions of
 * it (recomputed after a restart to the average, as in Algorithm 1).
 *
 * The adjoint of the map (reverse sweep) with the projection and the dual
 * case taken as fixed selections: derivative 1 strictly inside the box and
 * 0 on it for x+, and for y+ derivative 1 in yhat in the two moving cases
 * (plus sigma in the bound that moves it), 0 in the case that sets y+ = 0.
 *
 * The tangent-linear map (orc_unroll_tangent) is the same derivative in
 * forward mode.
 *
 * Parity: pinned by central finite differences of orc_unroll_replay (the
 * replay itself is pinned by reproducing the recorded run bitwise), by a
 * one-step closed form, by exact linearity when no bound is ever met and by
 * the dot-product test between the two modes (tests/test_oracle.py).
 */
#include "pdlp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double clampv(double v, double lo, double hi) {
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

/* Which branch of the dual case step (orc_dual_case) yhat takes:
 * 1: y+ = yhat + sigma uc,  2: y+ = yhat + sigma lc,  0: y+ = 0. */
static int dual_branch(double yhat, double sigma, double lc, double uc) {
    if (isfinite(uc) && yhat < -(sigma * uc)) return 1;
    if (isfinite(lc) && yhat > -(sigma * lc)) return 2;
    return 0;
}

/*
 * Replay K steps of the map on `lp` (scaled data) with the decisions of
 * `tp`.  x_out (n) receives x_K.  xs ((K+1) n) and ys ((K+1) m), when not
 * NULL, receive the state before every step and the final state; seta
 * (K) receives the sum of step sizes since the last restart after each step.
 * sig (when not NULL) receives the activity signature: the number of
 * (step, coordinate) pairs where x+ is strictly inside its box plus the
 * number where y+ takes a moving case.
 */
void orc_unroll_replay(const orc_lp *lp, const orc_tape *tp, int64_t K, double *x_out,
                       double *xs, double *ys, double *seta_out, int64_t *sig) {
    const int32_t m = lp->m, n = lp->n;
    double *x = malloc(sizeof(double) * (n + 1)), *aty = malloc(sizeof(double) * (n + 1));
    double *xn = malloc(sizeof(double) * (n + 1)), *sx = calloc(n + 1, sizeof(double));
    double *y = calloc(m + 1, sizeof(double)), *ax = malloc(sizeof(double) * (m + 1));
    double *axn = malloc(sizeof(double) * (m + 1)), *sy = calloc(m + 1, sizeof(double));
    double seta = 0.0;
    int64_t act = 0;
    for (int32_t j = 0; j < n; ++j) x[j] = clampv(0.0, lp->lv[j], lp->uv[j]);
    orc_spmv(lp, x, ax);
    orc_spmv_t(lp, y, aty);
    for (int64_t k = 0; k < K; ++k) {
        if (xs) memcpy(xs + k * n, x, sizeof(double) * n);
        if (ys) memcpy(ys + k * m, y, sizeof(double) * m);
        const double eta = tp->eta[k], tau = eta / tp->omega[k], sigma = eta * tp->omega[k];
        for (int32_t j = 0; j < n; ++j) {
            const double g = lp->c[j] - aty[j];
            const double v = x[j] - tau * g;
            xn[j] = clampv(v, lp->lv[j], lp->uv[j]);
            act += (v > lp->lv[j] && v < lp->uv[j]);
        }
        orc_spmv(lp, xn, axn);
        for (int32_t i = 0; i < m; ++i) {
            const double yhat = y[i] - sigma * (2.0 * axn[i] - ax[i]);
            act += dual_branch(yhat, sigma, lp->lc[i], lp->uc[i]) != 0;
            y[i] = orc_dual_case(yhat, sigma, lp->lc[i], lp->uc[i]);
        }
        memcpy(x, xn, sizeof(double) * n);
        memcpy(ax, axn, sizeof(double) * m);
        orc_spmv_t(lp, y, aty);
        seta += eta;
        for (int32_t j = 0; j < n; ++j) sx[j] += eta * x[j];
        for (int32_t i = 0; i < m; ++i) sy[i] += eta * y[i];
        if (seta_out) seta_out[k] = seta;
        const int32_t r = tp->restart[k];
        if (r == 2) {
            for (int32_t j = 0; j < n; ++j) x[j] = sx[j] / seta;
            for (int32_t i = 0; i < m; ++i) y[i] = sy[i] / seta;
            orc_spmv(lp, x, ax);
            orc_spmv_t(lp, y, aty);
        }
        if (r != 0) {
            seta = 0.0;
            memset(sx, 0, sizeof(double) * n);
            memset(sy, 0, sizeof(double) * m);
        }
    }
    if (xs) memcpy(xs + K * n, x, sizeof(double) * n);
    if (ys) memcpy(ys + K * m, y, sizeof(double) * m);
    memcpy(x_out, x, sizeof(double) * n);
    if (sig) *sig = act;
    free(x); free(aty); free(xn); free(sx); free(y); free(ax); free(axn); free(sy);
}

/*
 * Adjoint of the replayed map: given gx = dL/dx_K (scaled space, n), returns
 * dL/dc~ (n), dL/dlc~ and dL/duc~ (m), and dL/dA~ per stored nonzero of A~
 * (nnz, CSR order).  Outputs are overwritten.  Returns 0, or -3 when memory
 * runs out.
 */
int32_t orc_unroll_adjoint(const orc_lp *lp, const orc_tape *tp, int64_t K, const double *gx,
                           double *gc, double *glc, double *guc, double *gval) {
    const int32_t m = lp->m, n = lp->n;
    const int64_t nnz = lp->row_ptr[m];
    double *xs = malloc(sizeof(double) * ((size_t)(K + 1) * n + 1));
    double *ys = malloc(sizeof(double) * ((size_t)(K + 1) * m + 1));
    double *seta = malloc(sizeof(double) * (K + 1));
    double *xb = malloc(sizeof(double) * (n + 1)), *yb = calloc(m + 1, sizeof(double));
    double *sxb = calloc(n + 1, sizeof(double)), *syb = calloc(m + 1, sizeof(double));
    double *aty = malloc(sizeof(double) * (n + 1)), *xp = malloc(sizeof(double) * (n + 1));
    double *w = malloc(sizeof(double) * (n + 1)), *vb = malloc(sizeof(double) * (n + 1));
    double *wb = malloc(sizeof(double) * (n + 1)), *xpb = malloc(sizeof(double) * (n + 1));
    double *ax = malloc(sizeof(double) * (m + 1)), *axp = malloc(sizeof(double) * (m + 1));
    double *yhb = malloc(sizeof(double) * (m + 1)), *ypb = malloc(sizeof(double) * (m + 1));
    double *av = malloc(sizeof(double) * (m + 1)), *xfin = malloc(sizeof(double) * (n + 1));
    int *p = malloc(sizeof(int) * (n + 1)), *q = malloc(sizeof(int) * (m + 1));
    if (!xs || !ys || !seta || !xb || !yb || !sxb || !syb || !aty || !xp || !w || !vb || !wb ||
        !xpb || !ax || !axp || !yhb || !ypb || !av || !xfin || !p || !q) {
        free(xs); free(ys); free(seta); free(xb); free(yb); free(sxb); free(syb); free(aty);
        free(xp); free(w); free(vb); free(wb); free(xpb); free(ax); free(axp); free(yhb);
        free(ypb); free(av); free(xfin); free(p); free(q);
        return -3;
    }
    orc_unroll_replay(lp, tp, K, xfin, xs, ys, seta, NULL);
    memset(gc, 0, sizeof(double) * n);
    memset(glc, 0, sizeof(double) * m);
    memset(guc, 0, sizeof(double) * m);
    memset(gval, 0, sizeof(double) * nnz);
    memcpy(xb, gx, sizeof(double) * n);    /* adjoint of the state after the last step */
    for (int64_t k = K - 1; k >= 0; --k) {
        const double eta = tp->eta[k], tau = eta / tp->omega[k], sigma = eta * tp->omega[k];
        const double *xk = xs + k * n, *yk = ys + k * m;
        /* restart right after step k: (x, y) <- sums / S, sums <- 0 */
        const int32_t r = tp->restart[k];
        if (r == 2) {
            for (int32_t j = 0; j < n; ++j) { sxb[j] = xb[j] / seta[k]; xb[j] = 0.0; }
            for (int32_t i = 0; i < m; ++i) { syb[i] = yb[i] / seta[k]; yb[i] = 0.0; }
        } else if (r == 1) {
            memset(sxb, 0, sizeof(double) * n);
            memset(syb, 0, sizeof(double) * m);
        }
        /* sums: Sx += eta x+, Sy += eta y+ */
        for (int32_t j = 0; j < n; ++j) xpb[j] = xb[j] + eta * sxb[j];
        for (int32_t i = 0; i < m; ++i) ypb[i] = yb[i] + eta * syb[i];
        /* recompute step k */
        orc_spmv_t(lp, yk, aty);
        orc_spmv(lp, xk, ax);
        for (int32_t j = 0; j < n; ++j) {
            const double v = xk[j] - tau * (lp->c[j] - aty[j]);
            p[j] = v > lp->lv[j] && v < lp->uv[j];
            xp[j] = clampv(v, lp->lv[j], lp->uv[j]);
            w[j] = 2.0 * xp[j] - xk[j];
        }
        orc_spmv(lp, xp, axp);
        /* dual case step */
        for (int32_t i = 0; i < m; ++i) {
            const double yhat = yk[i] - sigma * (2.0 * axp[i] - ax[i]);
            q[i] = dual_branch(yhat, sigma, lp->lc[i], lp->uc[i]);
            yhb[i] = q[i] ? ypb[i] : 0.0;
            if (q[i] == 1) guc[i] += sigma * ypb[i];
            if (q[i] == 2) glc[i] += sigma * ypb[i];
        }
        /* yhat = y - sigma A~ w */
        orc_spmv_t(lp, yhb, wb);
        for (int32_t j = 0; j < n; ++j) wb[j] = -sigma * wb[j];
        for (int32_t i = 0; i < m; ++i)
            for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
                gval[e] += -sigma * yhb[i] * w[lp->col[e]];
        /* w = 2 x+ - x;  x+ = proj(v);  v = x - tau c~ + tau A~^T y */
        for (int32_t j = 0; j < n; ++j) {
            const double xplus_b = xpb[j] + 2.0 * wb[j];
            vb[j] = p[j] ? xplus_b : 0.0;
            xb[j] = -wb[j] + vb[j];
            gc[j] += -tau * vb[j];
        }
        orc_spmv(lp, vb, av);
        for (int32_t i = 0; i < m; ++i) {
            yb[i] = yhb[i] + tau * av[i];
            for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
                gval[e] += tau * yk[i] * vb[lp->col[e]];
        }
    }
    free(xs); free(ys); free(seta); free(xb); free(yb); free(sxb); free(syb); free(aty);
    free(xp); free(w); free(vb); free(wb); free(xpb); free(ax); free(axp); free(yhb);
    free(ypb); free(av); free(xfin); free(p); free(q);
    return 0;
}

/*
 * Tangent-linear (forward-mode) derivative of the replayed map: given a
 * direction (dc~ (n), dlc~, duc~ (m), dA~ per stored nonzero (nnz, CSR
 * order)) in the scaled data, returns dx_K (n), the directional derivative
 * of x_K, with the same fixed selections as orc_unroll_adjoint.  Per step,
 * with d(.) the tangent of each quantity:
 *   d(A~^T y) = dA~^T y + A~^T dy,  d(A~ x) = dA~ x + A~ dx
 *   dv   = dx - tau (dc~ - d(A~^T y)),          dx+ = dv inside the box, else 0
 *   dyhat = dy - sigma (2 d(A~ x+) - d(A~ x)),  dy+ = dyhat + sigma duc~ (case 1),
 *                                               dyhat + sigma dlc~ (case 2), 0 (case 0)
 *   dSx += eta dx+, dSy += eta dy+;  a restart to the average sets (dx, dy) =
 *   (dSx, dSy) / S and recomputes the product tangents; any restart clears dS.
 * The pairing <dx_K, gx> equals <(dc~, dlc~, duc~, dA~), adjoint of gx> up to
 * rounding (the dot-product test).  Returns 0, or -3 when memory runs out.
 */
int32_t orc_unroll_tangent(const orc_lp *lp, const orc_tape *tp, int64_t K, const double *dc,
                           const double *dlc, const double *duc, const double *dval,
                           double *dx_out) {
    const int32_t m = lp->m, n = lp->n;
    orc_lp dl = *lp;          /* the direction as a matrix with A's pattern */
    dl.val = dval;
    double *x = calloc(n + 1, sizeof(double)), *aty = malloc(sizeof(double) * (n + 1));
    double *xn = malloc(sizeof(double) * (n + 1)), *sx = calloc(n + 1, sizeof(double));
    double *y = calloc(m + 1, sizeof(double)), *ax = malloc(sizeof(double) * (m + 1));
    double *axn = malloc(sizeof(double) * (m + 1)), *sy = calloc(m + 1, sizeof(double));
    double *dx = calloc(n + 1, sizeof(double)), *daty = malloc(sizeof(double) * (n + 1));
    double *dxn = malloc(sizeof(double) * (n + 1)), *dsx = calloc(n + 1, sizeof(double));
    double *dy = calloc(m + 1, sizeof(double)), *dax = malloc(sizeof(double) * (m + 1));
    double *daxn = malloc(sizeof(double) * (m + 1)), *dsy = calloc(m + 1, sizeof(double));
    double *tn = malloc(sizeof(double) * (n + 1)), *tm = malloc(sizeof(double) * (m + 1));
    if (!x || !aty || !xn || !sx || !y || !ax || !axn || !sy || !dx || !daty || !dxn || !dsx ||
        !dy || !dax || !daxn || !dsy || !tn || !tm) {
        free(x); free(aty); free(xn); free(sx); free(y); free(ax); free(axn); free(sy);
        free(dx); free(daty); free(dxn); free(dsx); free(dy); free(dax); free(daxn); free(dsy);
        free(tn); free(tm);
        return -3;
    }
    double seta = 0.0;
    for (int32_t j = 0; j < n; ++j) x[j] = clampv(0.0, lp->lv[j], lp->uv[j]);
    /* x_0 = proj_X(0) does not depend on the data; y_0 = 0 */
    orc_spmv(lp, x, ax);
    orc_spmv_t(lp, y, aty);
    orc_spmv(&dl, x, dax);             /* d(A~ x_0) = dA~ x_0 */
    for (int32_t j = 0; j < n; ++j) daty[j] = 0.0;
    for (int64_t k = 0; k < K; ++k) {
        const double eta = tp->eta[k], tau = eta / tp->omega[k], sigma = eta * tp->omega[k];
        for (int32_t j = 0; j < n; ++j) {
            const double g = lp->c[j] - aty[j];
            const double v = x[j] - tau * g;
            const int inside = v > lp->lv[j] && v < lp->uv[j];
            xn[j] = clampv(v, lp->lv[j], lp->uv[j]);
            dxn[j] = inside ? dx[j] - tau * (dc[j] - daty[j]) : 0.0;
        }
        orc_spmv(lp, xn, axn);
        orc_spmv(&dl, xn, daxn);
        orc_spmv(lp, dxn, tm);
        for (int32_t i = 0; i < m; ++i) daxn[i] += tm[i];
        for (int32_t i = 0; i < m; ++i) {
            const double yhat = y[i] - sigma * (2.0 * axn[i] - ax[i]);
            const double dyhat = dy[i] - sigma * (2.0 * daxn[i] - dax[i]);
            const int br = dual_branch(yhat, sigma, lp->lc[i], lp->uc[i]);
            dy[i] = br == 1 ? dyhat + sigma * duc[i] : br == 2 ? dyhat + sigma * dlc[i] : 0.0;
            y[i] = orc_dual_case(yhat, sigma, lp->lc[i], lp->uc[i]);
        }
        memcpy(x, xn, sizeof(double) * n);
        memcpy(dx, dxn, sizeof(double) * n);
        memcpy(ax, axn, sizeof(double) * m);
        memcpy(dax, daxn, sizeof(double) * m);
        orc_spmv_t(lp, y, aty);
        orc_spmv_t(&dl, y, daty);
        orc_spmv_t(lp, dy, tn);
        for (int32_t j = 0; j < n; ++j) daty[j] += tn[j];
        seta += eta;
        for (int32_t j = 0; j < n; ++j) { sx[j] += eta * x[j]; dsx[j] += eta * dx[j]; }
        for (int32_t i = 0; i < m; ++i) { sy[i] += eta * y[i]; dsy[i] += eta * dy[i]; }
        const int32_t r = tp->restart[k];
        if (r == 2) {
            for (int32_t j = 0; j < n; ++j) { x[j] = sx[j] / seta; dx[j] = dsx[j] / seta; }
            for (int32_t i = 0; i < m; ++i) { y[i] = sy[i] / seta; dy[i] = dsy[i] / seta; }
            orc_spmv(lp, x, ax);
            orc_spmv_t(lp, y, aty);
            orc_spmv(&dl, x, dax);
            orc_spmv(lp, dx, tm);
            for (int32_t i = 0; i < m; ++i) dax[i] += tm[i];
            orc_spmv_t(&dl, y, daty);
            orc_spmv_t(lp, dy, tn);
            for (int32_t j = 0; j < n; ++j) daty[j] += tn[j];
        }
        if (r != 0) {
            seta = 0.0;
            memset(sx, 0, sizeof(double) * n);
            memset(sy, 0, sizeof(double) * m);
            memset(dsx, 0, sizeof(double) * n);
            memset(dsy, 0, sizeof(double) * m);
        }
    }
    memcpy(dx_out, dx, sizeof(double) * n);
    free(x); free(aty); free(xn); free(sx); free(y); free(ax); free(axn); free(sy);
    free(dx); free(daty); free(dxn); free(dsx); free(dy); free(dax); free(daxn); free(dsy);
    free(tn); free(tm);
    return 0;
}
