/*
 * Driver for the ASan/UBSan build of the oracle (test infrastructure only):
 * reads an LP from a binary file, preconditions it (Section 3, "Diagonal
 * Preconditioning"), solves it with Algorithm 1 twice (polishing off, then
 * on, with infeasibility detection), then runs the unrolled map's replay,
 * adjoint and tangent for a few recorded steps.  Exits 0 when every call
 * returned; the sanitizers abort on the first memory or undefined-behaviour
 * error.
 *
 * File layout (little-endian): int32 m, n; int64 nnz; int32 row_ptr[m+1],
 * col[nnz]; double val[nnz], c[n], lc[m], uc[m], lv[n], uv[n].
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pdlp_oracle.h"

void orc_precondition(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col,
                      double *val, int32_t ruiz_iters, int32_t pc, double *d1, double *d2);
void orc_scale_vectors(int32_t m, int32_t n, const double *d1, const double *d2,
                       const double *c, const double *lc, const double *uc,
                       const double *lv, const double *uv, double *c_s, double *lc_s,
                       double *uc_s, double *lv_s, double *uv_s);
void orc_init_state(const orc_lp *lp, orc_state *st);
int32_t orc_pdlp_record(const orc_lp *lp, const orc_unscale *u, const orc_params *prm,
                        orc_state *st, orc_scratch *scr, double *out_x, double *out_y,
                        orc_result *res, orc_tape *tape);
void orc_unroll_replay(const orc_lp *lp, const orc_tape *tp, int64_t K, double *x_out,
                       double *xs, double *ys, double *seta_out, int64_t *sig);
int32_t orc_unroll_adjoint(const orc_lp *lp, const orc_tape *tp, int64_t K, const double *gx,
                           double *gc, double *glc, double *guc, double *gval);
int32_t orc_unroll_tangent(const orc_lp *lp, const orc_tape *tp, int64_t K, const double *dc,
                           const double *dlc, const double *duc, const double *dval,
                           double *dx_out);

static void *read_n(FILE *f, size_t size, size_t count) {
    void *p = malloc(size * (count ? count : 1));
    if (!p || (count && fread(p, size, count, f) != count)) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

static double *alloc_d(size_t count) { return calloc(count ? count : 1, sizeof(double)); }

static orc_params defaults(void) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.eps_feas = 1e-6;
    p.eps_gap = 1e-6;
    p.max_iters = 20000;
    p.check_every = 64;
    p.terminate = 1;
    p.beta_suff = 0.1;
    p.beta_nec = 0.9;
    p.beta_art = 0.5;
    p.theta = 0.5;
    p.eps_zero = 1e-10;
    p.red_exp = 0.3;
    p.grow_exp = 0.6;
    p.reduced_cost_mode = 1;
    p.polish_first = 100;
    p.adaptive_restarts = 1;
    p.detect_infeas = 1;
    p.eps_infeas = 1e-9;
    p.fixed_omega = 1.0;
    return p;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t mn[2];
    int64_t nnz;
    if (fread(mn, sizeof(int32_t), 2, f) != 2 || fread(&nnz, sizeof(int64_t), 1, f) != 1) return 2;
    const int32_t m = mn[0], n = mn[1];
    int32_t *rp = read_n(f, sizeof(int32_t), (size_t)m + 1);
    int32_t *col = read_n(f, sizeof(int32_t), (size_t)nnz);
    double *val = read_n(f, sizeof(double), (size_t)nnz);
    double *c = read_n(f, sizeof(double), (size_t)n);
    double *lc = read_n(f, sizeof(double), (size_t)m);
    double *uc = read_n(f, sizeof(double), (size_t)m);
    double *lv = read_n(f, sizeof(double), (size_t)n);
    double *uv = read_n(f, sizeof(double), (size_t)n);
    fclose(f);

    double *sval = alloc_d((size_t)nnz), *d1 = alloc_d(m), *d2 = alloc_d(n);
    memcpy(sval, val, sizeof(double) * (size_t)nnz);
    orc_precondition(m, n, rp, col, sval, 10, 1, d1, d2);
    double *cs = alloc_d(n), *lcs = alloc_d(m), *ucs = alloc_d(m), *lvs = alloc_d(n),
           *uvs = alloc_d(n);
    orc_scale_vectors(m, n, d1, d2, c, lc, uc, lv, uv, cs, lcs, ucs, lvs, uvs);
    orc_lp lp = {m, n, rp, col, sval, cs, lcs, ucs, lvs, uvs};
    orc_lp orig = {m, n, rp, col, val, c, lc, uc, lv, uv};
    orc_unscale u = {orig, d1, d2, 0.0};

    double *st_n[4], *st_m[4];
    for (int k = 0; k < 4; ++k) {
        st_n[k] = alloc_d(n);
        st_m[k] = alloc_d(m);
    }
    double *scr_arr[12];
    for (int k = 0; k < 6; ++k) scr_arr[k] = alloc_d(n);
    for (int k = 6; k < 12; ++k) scr_arr[k] = alloc_d(m);
    orc_scratch scr = {scr_arr[0], scr_arr[1], scr_arr[2], scr_arr[3], scr_arr[4], scr_arr[5],
                       scr_arr[6], scr_arr[7], scr_arr[8], scr_arr[9], scr_arr[10], scr_arr[11]};
    double *ox = alloc_d(n), *oy = alloc_d(m);
    for (int polish = 0; polish < 2; ++polish) {
        orc_state st;
        memset(&st, 0, sizeof st);
        st.x = st_n[0]; st.aty = st_n[1]; st.x0 = st_n[2]; st.sx = st_n[3];
        st.y = st_m[0]; st.ax = st_m[1]; st.y0 = st_m[2]; st.sy = st_m[3];
        orc_init_state(&lp, &st);
        orc_params p = defaults();
        p.polish = polish;
        if (polish) {
            p.eps_feas = 1e-8;
            p.eps_gap = 1e-2;
            p.reduced_cost_mode = 0;
        }
        orc_result res;
        memset(&res, 0, sizeof res);
        const int32_t rc = orc_pdlp_record(&lp, &u, &p, &st, &scr, ox, oy, &res, NULL);
        printf("solve polish=%d status=%d iterations=%lld rc=%d\n", polish, res.status,
               (long long)res.iterations, rc);
    }
    /* recorded run of K steps, then the map's derivatives */
    const int64_t K = 40;
    orc_state st;
    memset(&st, 0, sizeof st);
    st.x = st_n[0]; st.aty = st_n[1]; st.x0 = st_n[2]; st.sx = st_n[3];
    st.y = st_m[0]; st.ax = st_m[1]; st.y0 = st_m[2]; st.sy = st_m[3];
    orc_init_state(&lp, &st);
    orc_params p = defaults();
    p.terminate = 0;
    p.max_iters = K;
    double *eta = alloc_d(K), *omega = alloc_d(K);
    int32_t *rst = calloc(K, sizeof(int32_t));
    orc_tape tape = {K, eta, omega, rst};
    orc_result res;
    memset(&res, 0, sizeof res);
    orc_pdlp_record(&lp, &u, &p, &st, &scr, ox, oy, &res, &tape);
    double *xk = alloc_d(n);
    int64_t sig = 0;
    orc_unroll_replay(&lp, &tape, K, xk, NULL, NULL, NULL, &sig);
    double *gx = alloc_d(n), *gc = alloc_d(n), *glc = alloc_d(m), *guc = alloc_d(m),
           *gval = alloc_d((size_t)nnz), *dx = alloc_d(n);
    for (int32_t j = 0; j < n; ++j) gx[j] = 1.0 / (1.0 + j);
    const int32_t ra = orc_unroll_adjoint(&lp, &tape, K, gx, gc, glc, guc, gval);
    const int32_t rt = orc_unroll_tangent(&lp, &tape, K, gc, glc, guc, gval, dx);
    printf("unroll K=%lld signature=%lld adjoint=%d tangent=%d\n", (long long)K, (long long)sig,
           ra, rt);
    free(rp); free(col); free(val); free(c); free(lc); free(uc); free(lv); free(uv);
    free(sval); free(d1); free(d2); free(cs); free(lcs); free(ucs); free(lvs); free(uvs);
    for (int k = 0; k < 4; ++k) { free(st_n[k]); free(st_m[k]); }
    for (int k = 0; k < 12; ++k) free(scr_arr[k]);
    free(ox); free(oy); free(eta); free(omega); free(rst); free(xk);
    free(gx); free(gc); free(glc); free(guc); free(gval); free(dx);
    return (ra == 0 && rt == 0) ? 0 : 1;
}
