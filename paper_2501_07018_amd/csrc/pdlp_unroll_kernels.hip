// Kernels of the unrolled, differentiable PDHG map (batched, FP64).
//
// The map: K accepted steps of the PDHG update of Section 2 with the step
// sizes, primal weights and restarts of a recorded Algorithm 1 run held
// fixed, from (proj_X(0), 0), per instance of a batch:
//   v = x - tau (c~ - A~^T y),  x+ = proj(v),  yhat = y - sigma A~ (2 x+ - x),
//   y+ = dual case step(yhat),  Sx += eta x+,  Sy += eta y+,
//   restart to the average: (x, y) <- (Sx, Sy) / S;  any restart: sums <- 0.
// Replay kernels (ku_primal, ku_dual, ku_aty) run one step for every
// instance at once with the arithmetic of the solver's step kernels, so a
// replay reproduces the recorded run bitwise.  Reverse kernels (ku_rrow,
// ku_rcol, ku_rA, ku_restart_adj) run the adjoint of one step; the
// projection and the dual case are fixed selections (derivative 1 strictly
// inside the box, 0 on it; y+ moves with yhat in its two moving cases).
//
// Per-step storage of a replayed segment (for the reverse): w = 2 x+ - x
// (n), y before the step (m), interior flag of v (n bytes), dual case (m bytes).
#include "pdlp_device.h"

#include <algorithm>

namespace pdlp {

// Decisions of step s of every instance.
struct UStep {
    const double *eta, *omega;  // [B * K]
    int64_t K, s;
    const int32_t *ablk_inst, *tblk_inst;
    __device__ __forceinline__ double eta_of(int i) const { return eta[(size_t)i * K + s]; }
    __device__ __forceinline__ double omega_of(int i) const { return omega[(size_t)i * K + s]; }
};

// Branch of dual_case: 1 -> yhat + sigma uc, 2 -> yhat + sigma lc, 0 -> 0.
__device__ __forceinline__ int dual_branch(double yhat, double sigma, double lc, double uc) {
    if (isfinite(uc) && yhat < -(sigma * uc)) return 1;
    if (isfinite(lc) && yhat > -(sigma * lc)) return 2;
    return 0;
}

__device__ __forceinline__ void add_count(double c, double *red, unsigned long long *sig, int inst) {
    double t[1] = {c};
    block_reduce<1>(t, red);
    if (threadIdx.x == 0 && t[0] > 0.0) atomicAdd(sig + inst, (unsigned long long)t[0]);
}

// ------------------------------------------------------------------ replay

__global__ __launch_bounds__(kThreads) void ku_primal(DCsr AT, Vecs v, UStep us,
                                                      const double *x, const double *aty,
                                                      double *xn, uint8_t *pm,
                                                      unsigned long long *sig) {
    __shared__ double red[kThreads / 64];
    for (int b = blockIdx.x; b < AT.nblk; b += gridDim.x) {
        const int i = us.tblk_inst[b];
        const double tau = us.eta_of(i) / us.omega_of(i);
        double cnt = 0.0;
        for (int j = AT.blk[b] + threadIdx.x; j < AT.blk[b + 1]; j += kThreads) {
            const double xj = x[j];
            const double vj = xj - tau * (v.c[j] - aty[j]);
            xn[j] = clampd(vj, v.lv[j], v.uv[j]);
            const bool in = vj > v.lv[j] && vj < v.uv[j];
            if (pm) pm[j] = in;
            cnt += in;
        }
        if (sig) add_count(cnt, red, sig, i);
    }
}

struct UDualEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    UStep us;
    Vecs v;
    const double *gsrc, *y, *ax;
    double *axn, *yn, *sy, *seg_y;
    uint8_t *qm;
    unsigned long long *sig;
    int inst;
    double eta, sigma;
    __device__ __forceinline__ int count(const DCsr &A) const { return A.nblk; }
    __device__ __forceinline__ int block(int bi) const { return bi; }
    __device__ __forceinline__ bool begin(int b) {
        inst = us.ablk_inst[b];
        eta = us.eta_of(inst);
        sigma = eta * us.omega_of(inst);
        return true;
    }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    __device__ __forceinline__ void apply(int r, double s, double (&acc)[1], const Pre &) const {
        axn[r] = s;
        const double yr = y[r];
        const double yhat = yr - sigma * (2.0 * s - ax[r]);
        const int br = dual_branch(yhat, sigma, v.lc[r], v.uc[r]);
        const double ynew = dual_case(yhat, sigma, v.lc[r], v.uc[r]);
        yn[r] = ynew;
        sy[r] += eta * ynew;
        if (seg_y) seg_y[r] = yr;
        if (qm) qm[r] = (uint8_t)br;
        acc[0] += br != 0;
    }
    __device__ __forceinline__ void end(int, double (&acc)[1], double *red) {
        if (sig) add_count(acc[0], red, sig, inst);
        acc[0] = 0.0;
    }
};

PDLP_STREAM_KERNEL void ku_dual(DCsr A, UDualEpi epi) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    stream_spmv<1>(A, epi, acc, prod, red);
}

struct UPrimalEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    UStep us;
    const double *gsrc, *x, *xn;
    double *atyn, *sx, *seg_w;
    double eta;
    __device__ __forceinline__ int count(const DCsr &A) const { return A.nblk; }
    __device__ __forceinline__ int block(int bi) const { return bi; }
    __device__ __forceinline__ bool begin(int b) {
        eta = us.eta_of(us.tblk_inst[b]);
        return true;
    }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    __device__ __forceinline__ void apply(int j, double s, double (&)[1], const Pre &) const {
        atyn[j] = s;
        const double xj = xn[j];
        sx[j] += eta * xj;
        if (seg_w) seg_w[j] = 2.0 * xj - x[j];
    }
    __device__ __forceinline__ void end(int, double (&)[1], double *) {}
};

PDLP_STREAM_KERNEL void ku_aty(DCsr AT, UPrimalEpi epi) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    stream_spmv<1>(AT, epi, acc, prod, red);
}

// ----------------------------------------------------------------- reverse

// Adjoint of a restart right after the step: rt[i] = 2 (to the average):
// adjoint of the sums = adjoint of the point / S, point adjoint 0; rt[i] = 1:
// adjoint of the sums 0.
__global__ __launch_bounds__(kThreads) void ku_restart_adj(DCsr A, DCsr AT, BatchMaps bm,
                                                           const int32_t *rt, const double *seta,
                                                           double *xb, double *yb, double *sxb,
                                                           double *syb) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        const int inst = cb < bm.nT ? bm.tblk_inst[cb] : bm.ablk_inst[cb - bm.nT];
        const int r = rt[inst];
        if (r == 0) continue;
        const double S = seta[inst];
        const bool col = cb < bm.nT;
        const int lo = col ? AT.blk[cb] : A.blk[cb - bm.nT];
        const int hi = col ? AT.blk[cb + 1] : A.blk[cb - bm.nT + 1];
        double *pb = col ? xb : yb, *sb = col ? sxb : syb;
        for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
            if (r == 2) {
                sb[k] = pb[k] / S;
                pb[k] = 0.0;
            } else {
                sb[k] = 0.0;
            }
        }
    }
}

// Rows: adjoint through the sums and the dual case step.
__global__ __launch_bounds__(kThreads) void ku_rrow(DCsr A, UStep us, const double *yb,
                                                    const double *syb, const uint8_t *qm,
                                                    double *yhb, double *glc, double *guc) {
    for (int b = blockIdx.x; b < A.nblk; b += gridDim.x) {
        const int i = us.ablk_inst[b];
        const double eta = us.eta_of(i), sigma = eta * us.omega_of(i);
        for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads) {
            const double ypb = yb[r] + eta * syb[r];
            const int q = qm[r];
            yhb[r] = q ? ypb : 0.0;
            if (q == 1) guc[r] += sigma * ypb;
            if (q == 2) glc[r] += sigma * ypb;
        }
    }
}

// Columns: wb = -sigma A~^T yhb, through w = 2 x+ - x, the projection and v.
struct URColEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    UStep us;
    const double *gsrc, *sxb;
    const uint8_t *pm;
    double *xb, *gc, *vb;
    double eta, tau, sigma;
    __device__ __forceinline__ int count(const DCsr &A) const { return A.nblk; }
    __device__ __forceinline__ int block(int bi) const { return bi; }
    __device__ __forceinline__ bool begin(int b) {
        const int i = us.tblk_inst[b];
        eta = us.eta_of(i);
        const double om = us.omega_of(i);
        tau = eta / om;
        sigma = eta * om;
        return true;
    }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    __device__ __forceinline__ void apply(int j, double s, double (&)[1], const Pre &) const {
        const double wb = -sigma * s;
        const double xplus_b = (xb[j] + eta * sxb[j]) + 2.0 * wb;
        const double v = pm[j] ? xplus_b : 0.0;
        xb[j] = -wb + v;
        gc[j] += -tau * v;
        vb[j] = v;
    }
    __device__ __forceinline__ void end(int, double (&)[1], double *) {}
};

PDLP_STREAM_KERNEL void ku_rcol(DCsr AT, URColEpi epi) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    stream_spmv<1>(AT, epi, acc, prod, red);
}

// Rows of A~: yb = yhb + tau A~ vb, and per nonzero
// gval += -sigma yhb_i w_j, then gval += tau y_i vb_j.
__global__ __launch_bounds__(kThreads) void ku_rA(DCsr A, UStep us, const double *vb,
                                                  const double *w, const double *y,
                                                  const double *yhb, double *yb, double *gval) {
    constexpr int kPer = kStage / kThreads;
    __shared__ double prod[kStage];
    __shared__ int rowof[kStage];
    __shared__ double red[kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int b = blockIdx.x; b < A.nblk; b += gridDim.x) {
        const int inst = us.ablk_inst[b];
        const double eta = us.eta_of(inst), om = us.omega_of(inst);
        const double tau = eta / om, sigma = eta * om;
        const int r0 = A.blk[b], r1 = A.blk[b + 1];
        const int e0 = A.row_ptr[r0], e1 = A.row_ptr[r1];
        const int len = e1 - e0;
        const int len0 = A.row_ptr[r0 + 1] - e0;
        if (len0 > A.med_row && len0 <= kWaveMax) {
            const int r = r0 + wid;
            if (r < r1) {
                const double yh = yhb[r], yr = y[r];
                double s = 0.0;
                for (int e = A.row_ptr[r] + lane; e < A.row_ptr[r + 1]; e += 64) {
                    const int cj = A.col[e];
                    const double vj = vb[cj];
                    s += A.val[e] * vj;
                    double g = gval[e];
                    g += -sigma * yh * w[cj];
                    g += tau * yr * vj;
                    gval[e] = g;
                }
                s = wave_sum(s);
                if (lane == 0) yb[r] = yh + tau * s;
            }
        } else if (len <= kStage && len0 <= A.med_row) {
            double gv[kPer], gw[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int q = k * kThreads + threadIdx.x;
                gv[k] = gw[k] = 0.0;
                if (q < len) {
                    const int cj = A.col[e0 + q];
                    gv[k] = vb[cj];
                    gw[k] = w[cj];
                    prod[q] = A.val[e0 + q] * gv[k];
                }
            }
            __syncthreads();
            for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
                const int a = A.row_ptr[r] - e0, z = A.row_ptr[r + 1] - e0;
                double s = 0.0;
                for (int q = a; q < z; ++q) {
                    s += prod[q];
                    rowof[q] = r;
                }
                yb[r] = yhb[r] + tau * s;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int q = k * kThreads + threadIdx.x;
                if (q < len) {
                    const int r = rowof[q];
                    double g = gval[e0 + q];
                    g += -sigma * yhb[r] * gw[k];
                    g += tau * y[r] * gv[k];
                    gval[e0 + q] = g;
                }
            }
            __syncthreads();
        } else {
            const double yh = yhb[r0], yr = y[r0];
            double s = 0.0;
            for (int e = e0 + threadIdx.x; e < e1; e += kThreads) {
                const int cj = A.col[e];
                const double vj = vb[cj];
                s += A.val[e] * vj;
                double g = gval[e];
                g += -sigma * yh * w[cj];
                g += tau * yr * vj;
                gval[e] = g;
            }
            double t[1] = {s};
            block_reduce<1>(t, red);
            if (threadIdx.x == 0) yb[r0] = yh + tau * t[0];
        }
    }
}

// ----------------------------------------------------------------- tangent
//
// Forward-mode derivative of one replayed step with the selections of the
// replay (which runs beside it with the value kernels above): with d(.) the
// tangent of each quantity,
//   dx+ = dx - tau (dc~ - d(A~^T y)) where v lies strictly inside the box, else 0
//   d(A~ x+) = dA~ x+ + A~ dx+,   dyhat = dy - sigma (2 d(A~ x+) - d(A~ x))
//   dy+ = dyhat + sigma duc~ (case 1), dyhat + sigma dlc~ (case 2), 0 (case 0)
//   d(A~^T y+) = dA~^T y+ + A~^T dy+,   dSx += eta dx+,  dSy += eta dy+.
// v and yhat are recomputed with the value kernels' arithmetic, so the
// selections are bitwise those of the replay.

__global__ __launch_bounds__(kThreads) void kt_primal(DCsr AT, Vecs v, UStep us, const double *dc,
                                                      const double *x, const double *aty,
                                                      const double *dx, const double *daty,
                                                      double *dxn) {
    for (int b = blockIdx.x; b < AT.nblk; b += gridDim.x) {
        const int i = us.tblk_inst[b];
        const double tau = us.eta_of(i) / us.omega_of(i);
        for (int j = AT.blk[b] + threadIdx.x; j < AT.blk[b + 1]; j += kThreads) {
            const double vj = x[j] - tau * (v.c[j] - aty[j]);
            const bool in = vj > v.lv[j] && vj < v.uv[j];
            dxn[j] = in ? dx[j] - tau * (dc[j] - daty[j]) : 0.0;
        }
    }
}

// rows: d(A~ x+) = t1 + t2 (dA~ x+ and A~ dx+), the dual tangent and dSy
__global__ __launch_bounds__(kThreads) void kt_dual(DCsr A, Vecs v, UStep us, const double *y,
                                                    const double *ax, const double *axn,
                                                    const double *dy, const double *dax,
                                                    const double *t1, const double *t2,
                                                    const double *dlc, const double *duc,
                                                    double *daxn, double *dyn, double *dsy) {
    for (int b = blockIdx.x; b < A.nblk; b += gridDim.x) {
        const int i = us.ablk_inst[b];
        const double eta = us.eta_of(i), sigma = eta * us.omega_of(i);
        for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads) {
            const double da = t1[r] + t2[r];
            daxn[r] = da;
            const double yhat = y[r] - sigma * (2.0 * axn[r] - ax[r]);
            const int br = dual_branch(yhat, sigma, v.lc[r], v.uc[r]);
            const double dyhat = dy[r] - sigma * (2.0 * da - dax[r]);
            const double d = br == 1 ? dyhat + sigma * duc[r] : (br == 2 ? dyhat + sigma * dlc[r] : 0.0);
            dyn[r] = d;
            dsy[r] += eta * d;
        }
    }
}

// columns: d(A~^T y+) = t1 + t2 (dA~^T y+ and A~^T dy+) and dSx
__global__ __launch_bounds__(kThreads) void kt_col(DCsr AT, UStep us, const double *t1,
                                                   const double *t2, const double *dxn,
                                                   double *datyn, double *dsx) {
    for (int b = blockIdx.x; b < AT.nblk; b += gridDim.x) {
        const double eta = us.eta_of(us.tblk_inst[b]);
        for (int j = AT.blk[b] + threadIdx.x; j < AT.blk[b + 1]; j += kThreads) {
            datyn[j] = t1[j] + t2[j];
            dsx[j] += eta * dxn[j];
        }
    }
}

__global__ __launch_bounds__(kThreads) void kt_add(int64_t len, const double *a, const double *b,
                                                   double *out) {
    for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < len;
         k += (int64_t)gridDim.x * kThreads)
        out[k] = a[k] + b[k];
}

// Checks of new data in device memory: counts non-finite objective entries
// and matrix values, and rows whose bounds are invalid (NaN, lc = +inf,
// uc = -inf or lc > uc), taking the current bound where one is not given.
__global__ __launch_bounds__(kThreads) void ku_check_data(int64_t N, int64_t M, int64_t NZ,
                                                          const double *c, const double *lc,
                                                          const double *uc, const double *val,
                                                          const double *cur_lc,
                                                          const double *cur_uc,
                                                          unsigned long long *bad) {
    unsigned long long nb = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t t0 = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (c)
        for (int64_t j = t0; j < N; j += stride) nb += !isfinite(c[j]);
    if (val)
        for (int64_t e = t0; e < NZ; e += stride) nb += !isfinite(val[e]);
    if (lc || uc)
        for (int64_t i = t0; i < M; i += stride) {
            const double a = lc ? lc[i] : cur_lc[i], z = uc ? uc[i] : cur_uc[i];
            nb += isnan(a) || isnan(z) || a == INFINITY || z == -INFINITY || a > z;
        }
    if (nb) atomicAdd(bad, nb);
}

// ------------------------------------------------------- data and results

// A~ = D1 A D2 entry by entry as (d1_i a_ij) d2_j, into A~ and (through a2t) A~^T.
__global__ __launch_bounds__(kThreads) void ku_scale_values(DCsr A, const double *val,
                                                            const double *d1, const double *d2,
                                                            const int32_t *a2t, double *va,
                                                            double *vt) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < A.rows; r += gridDim.x * kThreads) {
        const double di = d1[r];
        for (int e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e) {
            const double s = (di * val[e]) * d2[A.col[e]];
            va[e] = s;
            vt[a2t[e]] = s;
        }
    }
}

// Gradients in original units: dc = D2 dc~, dlc = D1 dlc~ (0 where lc is
// infinite), likewise uc, dA_ij = (D1_i D2_j) dA~_ij.
__global__ __launch_bounds__(kThreads) void ku_finish(DCsr A, int64_t N, const double *d1,
                                                      const double *d2, const double *lc,
                                                      const double *uc, const double *gc,
                                                      const double *glc, const double *guc,
                                                      const double *gval, double *oc, double *olc,
                                                      double *ouc, double *oval) {
    const int stride = gridDim.x * kThreads;
    for (int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x; j < N; j += stride)
        oc[j] = d2[j] * gc[j];
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < A.rows; r += stride) {
        olc[r] = isfinite(lc[r]) ? d1[r] * glc[r] : 0.0;
        ouc[r] = isfinite(uc[r]) ? d1[r] * guc[r] : 0.0;
        const double di = d1[r];
        for (int e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e)
            oval[e] = (di * d2[A.col[e]]) * gval[e];
    }
}

// --------------------------------------------------------------- launchers

static inline int grid_of(int64_t n, int cap) {
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
static inline int blk_grid(int nblk, int cap) { return nblk < 1 ? 1 : (nblk > cap ? cap : nblk); }

hipError_t launch_u_step(hipStream_t s, const DCsr &A, const DCsr &AT, Vecs v, UStepArgs u,
                         const double *x, const double *y, const double *ax, const double *aty,
                         double *xn, double *yn, double *axn, double *atyn, double *sx, double *sy,
                         double *seg_w, double *seg_y, uint8_t *seg_p, uint8_t *seg_q,
                         unsigned long long *sig) {
    const UStep us{u.eta, u.omega, u.K, u.s, u.ablk_inst, u.tblk_inst};
    hipLaunchKernelGGL(ku_primal, dim3(blk_grid(AT.nblk, 4096)), dim3(kThreads), 0, s, AT, v, us,
                       x, aty, xn, seg_p, sig);
    if (A.nblk > 0) {
        UDualEpi de{{}, us, v, xn, y, ax, axn, yn, sy, seg_y, seg_q, sig, 0, 0.0, 0.0};
        hipLaunchKernelGGL(ku_dual, dim3(blk_grid(A.nblk, 2048)), dim3(kThreads), 0, s, A, de);
    }
    UPrimalEpi pe{{}, us, yn, x, xn, atyn, sx, seg_w, 0.0};
    hipLaunchKernelGGL(ku_aty, dim3(blk_grid(AT.nblk, 2048)), dim3(kThreads), 0, s, AT, pe);
    return hipGetLastError();
}

hipError_t launch_u_restart_adj(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                                const int32_t *rt, const double *seta, double *xb, double *yb,
                                double *sxb, double *syb) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(ku_restart_adj, dim3(blk_grid(bm.nc, 4096)), dim3(kThreads), 0, s, A,
                           AT, bm, rt, seta, xb, yb, sxb, syb);
    return hipGetLastError();
}

hipError_t launch_u_reverse(hipStream_t s, const DCsr &A, const DCsr &AT, UStepArgs u,
                            const double *seg_w, const double *seg_y, const uint8_t *seg_p,
                            const uint8_t *seg_q, double *xb, double *yb, const double *sxb,
                            const double *syb, double *yhb, double *vb, double *gc, double *glc,
                            double *guc, double *gval) {
    const UStep us{u.eta, u.omega, u.K, u.s, u.ablk_inst, u.tblk_inst};
    if (A.nblk > 0)
        hipLaunchKernelGGL(ku_rrow, dim3(blk_grid(A.nblk, 4096)), dim3(kThreads), 0, s, A, us, yb,
                           syb, seg_q, yhb, glc, guc);
    URColEpi ce{{}, us, yhb, sxb, seg_p, xb, gc, vb, 0.0, 0.0, 0.0};
    hipLaunchKernelGGL(ku_rcol, dim3(blk_grid(AT.nblk, 2048)), dim3(kThreads), 0, s, AT, ce);
    if (A.nblk > 0)
        hipLaunchKernelGGL(ku_rA, dim3(blk_grid(A.nblk, 2048)), dim3(kThreads), 0, s, A, us, vb,
                           seg_w, seg_y, yhb, yb, gval);
    return hipGetLastError();
}

hipError_t launch_u_tangent_step(hipStream_t s, const DCsr &A, const DCsr &AT, const DCsr &dA,
                                 const DCsr &dAT, Vecs v, UStepArgs u, const double *dc,
                                 const double *dlc, const double *duc, const double *x,
                                 const double *y, const double *ax, const double *aty,
                                 double *xn, double *yn, double *axn, double *atyn, double *sx,
                                 double *sy, const double *dx, const double *dy, const double *dax,
                                 const double *daty, double *dxn, double *dyn, double *daxn,
                                 double *datyn, double *dsx, double *dsy, double *tm1,
                                 double *tm2, double *tn1, double *tn2) {
    const UStep us{u.eta, u.omega, u.K, u.s, u.ablk_inst, u.tblk_inst};
    hipLaunchKernelGGL(kt_primal, dim3(blk_grid(AT.nblk, 4096)), dim3(kThreads), 0, s, AT, v, us,
                       dc, x, aty, dx, daty, dxn);
    hipError_t e = launch_u_step(s, A, AT, v, u, x, y, ax, aty, xn, yn, axn, atyn, sx, sy, nullptr,
                                 nullptr, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return e;
    if (A.nblk > 0) {
        e = launch_spmv_plain(s, dA, xn, tm1);
        if (e != hipSuccess) return e;
        e = launch_spmv_plain(s, A, dxn, tm2);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kt_dual, dim3(blk_grid(A.nblk, 4096)), dim3(kThreads), 0, s, A, v, us,
                           y, ax, axn, dy, dax, tm1, tm2, dlc, duc, daxn, dyn, dsy);
    }
    e = launch_spmv_plain(s, dAT, yn, tn1);
    if (e != hipSuccess) return e;
    e = launch_spmv_plain(s, AT, dyn, tn2);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kt_col, dim3(blk_grid(AT.nblk, 4096)), dim3(kThreads), 0, s, AT, us, tn1,
                       tn2, dxn, datyn, dsx);
    return hipGetLastError();
}

hipError_t launch_u_add(hipStream_t s, int64_t len, const double *a, const double *b, double *out) {
    if (len > 0)
        hipLaunchKernelGGL(kt_add, dim3(grid_of(len, 4096)), dim3(kThreads), 0, s, len, a, b, out);
    return hipGetLastError();
}

hipError_t launch_u_check_data(hipStream_t s, int64_t N, int64_t M, int64_t NZ, const double *c,
                               const double *lc, const double *uc, const double *val,
                               const double *cur_lc, const double *cur_uc,
                               unsigned long long *bad) {
    const int64_t len = std::max(N, std::max(M, NZ));
    hipLaunchKernelGGL(ku_check_data, dim3(grid_of(len, 4096)), dim3(kThreads), 0, s, N, M, NZ, c,
                       lc, uc, val, cur_lc, cur_uc, bad);
    return hipGetLastError();
}

hipError_t launch_u_scale_values(hipStream_t s, const DCsr &A, const double *val, const double *d1,
                                 const double *d2, const int32_t *a2t, double *va, double *vt) {
    if (A.rows > 0)
        hipLaunchKernelGGL(ku_scale_values, dim3(grid_of(A.rows, 4096)), dim3(kThreads), 0, s, A,
                           val, d1, d2, a2t, va, vt);
    return hipGetLastError();
}

hipError_t launch_u_finish(hipStream_t s, const DCsr &A, int64_t N, const double *d1,
                           const double *d2, const double *lc, const double *uc, const double *gc,
                           const double *glc, const double *guc, const double *gval, double *oc,
                           double *olc, double *ouc, double *oval) {
    hipLaunchKernelGGL(ku_finish, dim3(grid_of(N > A.rows ? N : A.rows, 4096)), dim3(kThreads), 0,
                       s, A, N, d1, d2, lc, uc, gc, glc, guc, gval, oc, olc, ouc, oval);
    return hipGetLastError();
}

}  // namespace pdlp
