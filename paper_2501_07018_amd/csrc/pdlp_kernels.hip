// gfx950 kernels of the PDLP hot path (FP64 values, int32 indices).
//
// Step attempt (Algorithm 2 with the PDHG update of Section 2):
//   k_primal        x' = proj_X(x - tau (c - A^T y))       (after a rejection or at block start)
//   k_spmv_dual     A x' by CSR stream + dual step (case form), ||dy||^2, dy^T A dx partials
//   k_step_decide   eta_bar, eta', accept/reject, counters    (one workgroup)
//   k_spmv_primal   A^T y' by CSR stream + primal average + next x' (after an acceptance)
// Every kernel reads the device control block and switches itself off for
// work that a rejection or the end of an iteration block makes void, so a
// whole block of attempts is enqueued without host synchronization.
//
// Reductions are deterministic: fixed grids, per-thread accumulation in a
// fixed order, wave butterfly + LDS in a fixed order, and a one-workgroup
// final pass in a fixed order.  No floating-point atomics anywhere.
#include "pdlp_device.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace pdlp {

// [hot-path kernels begin]
struct PlainEpi : SingleEpi {
    double *out;
    template <int N>
    __device__ __forceinline__ void apply(int r, double s, double (&)[N], const Pre &) const {
        out[r] = s;
    }
};

PDLP_STREAM_KERNEL void k_spmv_plain(DCsr A, const double *__restrict__ x,
                                                         double *__restrict__ out) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    PlainEpi epi;
    epi.gsrc = x;
    epi.out = out;
    stream_spmv<1>(A, epi, acc, prod, red);
}

struct DualEpi : SingleEpi {
    DualRow row;
    using Pre = DualRow::Pre;
    __device__ __forceinline__ Pre prefetch(int r) const { return row.pre(r); }
    __device__ __forceinline__ void apply(int r, double s, double (&acc)[2], const Pre &p) const {
        row.apply(r, s, acc, p);
    }
};

PDLP_STREAM_KERNEL void k_spmv_dual(DCsr A, Vecs v, Iter it, const Ctrl *ctrl,
                                                        double *part) {
    if (ctrl->stop) return;
    __shared__ double prod[kStage];
    __shared__ double red[2 * (kThreads / 64)];
    const int cur = ctrl->cur;
    DualEpi epi;
    epi.gsrc = it.X[cur ^ 1];
    epi.row = DualRow{it.Y[cur], it.AX[cur], v.lc, v.uc, it.AX[cur ^ 1], it.Y[cur ^ 1], it.sy,
                      ctrl->eta * ctrl->omega, ctrl->eta_avg_y, ctrl->pending_sy};
    double acc[2] = {0.0, 0.0};
    stream_spmv<2>(A, epi, acc, prod, red);
    write_partials<2>(acc, red, part);
}

struct PrimalEpi : SingleEpi {
    PrimalRow row;
    using Pre = PrimalRow::Pre;
    __device__ __forceinline__ Pre prefetch(int j) const { return row.pre(j); }
    __device__ __forceinline__ void apply(int j, double s, double (&acc)[1], const Pre &p) const {
        row.apply(j, s, acc, p);
    }
};

PDLP_STREAM_KERNEL void k_spmv_primal(DCsr AT, Vecs v, Iter it,
                                                          const Ctrl *ctrl, double *part) {
    if (!ctrl->run_at) return;
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    const int cur = ctrl->cur;
    const int next = !ctrl->stop;
    PrimalEpi epi;
    epi.gsrc = it.Y[cur];
    epi.row = PrimalRow{it.X[cur], v.c, v.lv, v.uv, it.ATY[cur], it.X[cur ^ 1], it.sx,
                        ctrl->eta_used, ctrl->eta / ctrl->omega, next};
    double acc[1] = {0.0};
    stream_spmv<1>(AT, epi, acc, prod, red);
    if (next) write_partials<1>(acc, red, part);
}

// Two-phase A^T y' (SegCsr): phase 1 sums the (row, segment) pairs of G,
// whose blocks are dealt to XCDs by segment through sg.glist (workgroup w
// of the persistent grid, a multiple of 8, runs on XCD w mod 8 and visits
// list positions = w mod 8); phase 2 stages the pair sums per row block and
// runs the primal row work.
#ifndef PDLP_SEG_NT_Q
#define PDLP_SEG_NT_Q 0
#endif
struct SegGatherEpi : NoPrefetch {
    const int32_t *list;
    int32_t len;
    const double *gsrc;
    double *out;
    __device__ __forceinline__ int count(const DCsr &) const { return len; }
    __device__ __forceinline__ int block(int bi) const { return list[bi]; }
    __device__ __forceinline__ bool begin(int b) const { return b >= 0; }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    template <int N>
    __device__ __forceinline__ void apply(int r, double s, double (&)[N], const Pre &) const {
#if PDLP_SEG_NT_Q
        __builtin_nontemporal_store(s, out + r);
#else
        out[r] = s;
#endif
    }
    template <int N>
    __device__ __forceinline__ void end(int, double (&)[N], double *) {}
};

__device__ __forceinline__ void seg_gather(const SegCsr &sg, const double *__restrict__ v) {
    constexpr int kPer = kStage / kThreads;
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    SegGatherEpi epi;
    epi.list = sg.glist;
    epi.len = sg.glen;
    epi.gsrc = v;
    epi.out = sg.Q + sg.n1;
    double acc[1] = {0.0};
    for (int bi = blockIdx.x; bi < sg.glen; bi += gridDim.x) {
        const int item = sg.glist[bi];
        if (item >= 0) {
            stream_block<1>(sg.G, epi, item, acc, prod, red);
        } else if (item <= -2) {
            // single-entry pairs: plain products, kPer gathers in flight per lane
            const int k = -2 - item;
            const int lo = sg.chunk[2 * k], hi = sg.chunk[2 * k + 1];
            int ci[kPer];
            double vv[kPer];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int q = lo + i * kThreads + (int)threadIdx.x;
                ci[i] = q < hi ? stream_load(sg.c1 + q) : 0;
                vv[i] = q < hi ? stream_load(sg.v1 + q) : 0.0;
            }
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int q = lo + i * kThreads + (int)threadIdx.x;
#if PDLP_SEG_NT_Q
                if (q < hi) __builtin_nontemporal_store(vv[i] * v[ci[i]], sg.Q + q);
#else
                if (q < hi) sg.Q[q] = vv[i] * v[ci[i]];
#endif
            }
        }
    }
}

PDLP_STREAM_KERNEL void k_seg_gather_primal(SegCsr sg, Iter it, const Ctrl *ctrl) {
    if (!ctrl->run_at) return;
    seg_gather(sg, it.Y[ctrl->cur]);
}

PDLP_STREAM_KERNEL void k_seg_primal(SegCsr sg, Vecs v, Iter it, const Ctrl *ctrl, double *part) {
    if (!ctrl->run_at) return;
    __shared__ double prod[kStage];
    __shared__ int32_t lds_i[2 * kThreads + kWaveRows];
    __shared__ double red[kThreads / 64];
    const int cur = ctrl->cur;
    const int next = !ctrl->stop;
    PrimalEpi epi;
    epi.gsrc = nullptr;
    epi.row = PrimalRow{it.X[cur], v.c, v.lv, v.uv, it.ATY[cur], it.X[cur ^ 1], it.sx,
                        ctrl->eta_used, ctrl->eta / ctrl->omega, next};
    double acc[1] = {0.0};
    staged_spmv<1>(sg, epi, acc, prod, lds_i);
    if (next) write_partials<1>(acc, red, part);
}

// [hot-path kernels end]

// Plain two-phase product out = M v (SegCsr; row sums as in k_seg_primal).
PDLP_STREAM_KERNEL void k_seg_gather_plain(SegCsr sg, const double *v) { seg_gather(sg, v); }

PDLP_STREAM_KERNEL void k_seg_plain(SegCsr sg, double *out) {
    __shared__ double prod[kStage];
    __shared__ int32_t lds_i[2 * kThreads + kWaveRows];
    PlainEpi epi;
    epi.gsrc = nullptr;
    epi.out = out;
    double acc[1] = {0.0};
    staged_spmv<1>(sg, epi, acc, prod, lds_i);
}

// Standalone primal step: x' = proj_X(x - tau (c - A^T y)).
__global__ __launch_bounds__(kThreads) void k_primal(int n, Vecs v, Iter it, const Ctrl *ctrl,
                                                     double *part) {
    if (ctrl->stop || !ctrl->need_primal) return;
    __shared__ double red[kThreads / 64];
    const int cur = ctrl->cur;
    const double tau = ctrl->eta / ctrl->omega;
    const double *x = it.X[cur], *aty = it.ATY[cur];
    double *xn = it.X[cur ^ 1];
    double acc[1] = {0.0};
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += gridDim.x * kThreads) {
        const double xj = x[j];
        const double g = v.c[j] - aty[j];
        const double xv = clampd(xj - tau * g, v.lv[j], v.uv[j]);
        xn[j] = xv;
        const double d = xv - xj;
        acc[0] += d * d;
    }
    write_partials<1>(acc, red, part);
}

// Algorithm 2 decision for one attempt (one workgroup).
__global__ __launch_bounds__(kThreads) void k_step_decide(Ctrl *ctrl, const double *pd, int gd,
                                                          const double *pps, int gps,
                                                          const double *ppf, int gpf) {
    __shared__ double red[3 * (kThreads / 64)];
    if (ctrl->stop) {
        if (threadIdx.x == 0) ctrl->run_at = 0;
        return;
    }
    const int np = ctrl->need_primal;
    const double *pp = np ? pps : ppf;
    const int gp = np ? gps : gpf;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < gp; i += kThreads) a[0] += pp[i];
    for (int i = threadIdx.x; i < gd; i += kThreads) {
        a[1] += pd[2 * i];
        a[2] += pd[2 * i + 1];
    }
    block_reduce<3>(a, red);
    if (threadIdx.x != 0) return;
    Ctrl c = *ctrl;
    const double eta = c.eta, omega = c.omega;
    const double num = omega * a[0] + a[1] / omega;
    const double den = 2.0 * fabs(a[2]);
    c.attempts += 1;
    if (!isfinite(num) || !isfinite(den)) {
        c.numerr = 1;
        c.stop = 1;
        c.run_at = 0;
        *ctrl = c;
        return;
    }
    const double eta_bar = den > 0.0 ? num / den : INFINITY;
    const double jj = (double)(c.attempts + 1);
    const double e1 = (1.0 - pow(jj, -c.red_exp)) * eta_bar;
    const double e2 = (1.0 + pow(jj, -c.grow_exp)) * eta;
    const double eta_next = e1 < e2 ? e1 : e2;
    c.last_eta_bar = eta_bar;
    if (c.fixed_step || eta <= eta_bar) {
        c.cur ^= 1;
        c.k += 1;
        c.t += 1;
        c.block_acc += 1;
        c.seta += eta;
        c.eta_used = eta;
        c.eta_avg_y = eta;
        c.pending_sy = 1;
        c.eta_hat = c.fixed_step ? c.fixed_eta : eta_next;
        c.eta = c.eta_hat;
        c.stop = c.block_acc >= c.block_target;
        c.need_primal = c.stop;
        c.run_at = 1;
    } else {
        c.eta = eta_next;
        c.need_primal = 1;
        c.run_at = 0;
        c.pending_sy = 0;
    }
    *ctrl = c;
}

// Dual average owed by the last accepted step of a block.
__global__ __launch_bounds__(kThreads) void k_flush_sy(int m, Iter it, Ctrl *ctrl) {
    if (!ctrl->pending_sy) return;
    const int cur = ctrl->cur;
    const double e = ctrl->eta_avg_y;
    const double *y = it.Y[cur];
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += gridDim.x * kThreads)
        it.sy[i] += e * y[i];
}

__global__ void k_clear_pending(Ctrl *ctrl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->pending_sy = 0;
}

// ------------------------------------------------------------ vector ops

__global__ __launch_bounds__(kThreads) void k_div(int64_t len, const double *a, const double *d,
                                                  double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[i] = a[i] / d[i];
}

__global__ __launch_bounds__(kThreads) void k_mul(int64_t len, const double *a, const double *d,
                                                  double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[i] = a[i] * d[i];
}

__global__ __launch_bounds__(kThreads) void k_average(int64_t len, const double *sum, double seta,
                                                      double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[i] = sum[i] / seta;
}

__global__ __launch_bounds__(kThreads) void k_fill(int64_t len, double *a, double v) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        a[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_take(int64_t len, const int64_t *perm,
                                                    const double *src, double *dst) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(kThreads) void k_copy(int64_t len, const double *a, double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[i] = a[i];
}

__global__ __launch_bounds__(kThreads) void k_gather(int64_t len, const int32_t *perm,
                                                     const double *in, double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[i] = in[perm[i]];
}

__global__ __launch_bounds__(kThreads) void k_scatter(int64_t len, const int32_t *perm,
                                                      const double *in, double *out) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        out[perm[i]] = in[i];
}

__global__ __launch_bounds__(kThreads) void k_clamp0(int n, const double *lv, const double *uv,
                                                     double *x) {
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += gridDim.x * kThreads)
        x[j] = clampd(0.0, lv[j], uv[j]);
}

__global__ __launch_bounds__(kThreads) void k_dist2(int64_t len, const double *a, const double *b,
                                                    double *part) {
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads) {
        const double d = a[i] - b[i];
        acc[0] += d * d;
    }
    write_partials<1>(acc, red, part);
}

__global__ __launch_bounds__(kThreads) void k_absmax(int64_t len, const double *a, double *part) {
    __shared__ double red[kThreads / 64];
    double acc[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        acc[0] = nan_max(acc[0], fabs(a[i]));
    write_partials<1, 1u>(acc, red, part);
}

// Final pass of a reduction: out[i] = sum or max over the grid of part[g*nv + i].
__global__ __launch_bounds__(kThreads) void k_sum_max(const double *part, int grid, int nv,
                                                      unsigned maxmask, double *out) {
    __shared__ double red[8 * (kThreads / 64)];
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.0;
    for (int g = threadIdx.x; g < grid; g += kThreads) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < nv) {
                const double p = part[g * nv + i];
                v[i] = ((maxmask >> i) & 1u) ? nan_max(v[i], p) : v[i] + p;
            }
        }
    }
    // generic mask: reduce as sums and maxes separately
    double s[8], mx[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        s[i] = ((maxmask >> i) & 1u) ? 0.0 : v[i];
        mx[i] = ((maxmask >> i) & 1u) ? v[i] : 0.0;
    }
    block_reduce<8, 0u>(s, red);
    block_reduce<8, 0xFFu>(mx, red);
    if (threadIdx.x == 0)
        for (int i = 0; i < nv; ++i) out[i] = ((maxmask >> i) & 1u) ? mx[i] : s[i];
}

// -------------------------------------------------------- preconditioning

// Row norms of a CSR matrix, one lane per row, in column order (infinity
// norm for Ruiz, 1-norm for Pock-Chambolle with alpha = 1).
__global__ __launch_bounds__(kThreads) void k_row_norms(DCsr A, int use_inf, double *out) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < A.rows; r += gridDim.x * kThreads) {
        double s = 0.0;
        for (int e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e) {
            const double a = fabs(A.val[e]);
            if (use_inf) {
                if (a > s) s = a;
            } else {
                s += a;
            }
        }
        out[r] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_norm_to_factor(int len, double *nrm) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < len; i += gridDim.x * kThreads)
        nrm[i] = nrm[i] > 0.0 ? sqrt(nrm[i]) : 1.0;
}

// a_ij <- a_ij / (rf_i * cf_j)
__global__ __launch_bounds__(kThreads) void k_scale_matrix(DCsr A, const double *rf,
                                                           const double *cf) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < A.rows; r += gridDim.x * kThreads) {
        const double f = rf[r];
        for (int e = A.row_ptr[r]; e < A.row_ptr[r + 1]; ++e) A.val[e] = A.val[e] / (f * cf[A.col[e]]);
    }
}

__global__ __launch_bounds__(kThreads) void k_div_inplace(int len, double *d, const double *f) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < len; i += gridDim.x * kThreads)
        d[i] = d[i] / f[i];
}

// c~ = D2 c, (lc~, uc~) = D1 (lc, uc), (lv~, uv~) = D2^-1 (lv, uv); infinities kept.
__global__ __launch_bounds__(kThreads) void k_scale_vectors(int m, int n, const double *d1,
                                                            const double *d2, const double *c,
                                                            const double *lc, const double *uc,
                                                            const double *lv, const double *uv,
                                                            double *cs, double *lcs, double *ucs,
                                                            double *lvs, double *uvs) {
    const int stride = gridDim.x * kThreads;
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride) {
        cs[j] = d2[j] * c[j];
        lvs[j] = isfinite(lv[j]) ? lv[j] / d2[j] : lv[j];
        uvs[j] = isfinite(uv[j]) ? uv[j] / d2[j] : uv[j];
    }
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride) {
        lcs[i] = isfinite(lc[i]) ? d1[i] * lc[i] : lc[i];
        ucs[i] = isfinite(uc[i]) ? d1[i] * uc[i] : uc[i];
    }
}

// ||c||^2 and ||Combine(lc, uc)||^2 (InitializePrimalWeight).
__global__ __launch_bounds__(kThreads) void k_pw_init(int m, int n, const double *c,
                                                      const double *lc, const double *uc,
                                                      double *part) {
    __shared__ double red[2 * (kThreads / 64)];
    double acc[2] = {0.0, 0.0};
    const int stride = gridDim.x * kThreads;
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride) acc[0] += c[j] * c[j];
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride) {
        double v = 0.0;
        const double a = isfinite(lc[i]) ? fabs(lc[i]) : 0.0;
        const double b = isfinite(uc[i]) ? fabs(uc[i]) : 0.0;
        if (a > v) v = a;
        if (b > v) v = b;
        acc[1] += v * v;
    }
    write_partials<2>(acc, red, part);
}

// -------------------------------------------------------------- transpose

__global__ __launch_bounds__(kThreads) void k_row_ids(int m, const int32_t *row_ptr,
                                                      int32_t *rowid) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < m; r += gridDim.x * kThreads)
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) rowid[e] = r;
}

__global__ __launch_bounds__(kThreads) void k_row_ids_mapped(int m, const int32_t *row_ptr,
                                                             const int32_t *new_row,
                                                             int32_t *rowid) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < m; r += gridDim.x * kThreads) {
        const int32_t nr = new_row[r];
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) rowid[e] = nr;
    }
}

__global__ __launch_bounds__(kThreads) void k_relabel(int64_t nnz, const int32_t *col,
                                                      const int32_t *new_col, uint32_t *key) {
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kThreads)
        key[e] = (uint32_t)new_col[col[e]];
}

__global__ __launch_bounds__(kThreads) void k_permute_rows(int m, const int32_t *row_order,
                                                           const int32_t *old_rp,
                                                           const int32_t *old_col,
                                                           const double *old_val,
                                                           const int32_t *new_col,
                                                           const int32_t *new_rp, int32_t *ncol,
                                                           double *nval, int32_t *orig_pos) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < m; r += gridDim.x * kThreads) {
        const int32_t o = row_order[r];
        const int32_t a = old_rp[o], len = old_rp[o + 1] - a, d = new_rp[r];
        for (int k = 0; k < len; ++k) {
            ncol[d + k] = new_col[old_col[a + k]];
            nval[d + k] = old_val[a + k];
            orig_pos[d + k] = a + k;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_iota(int64_t len, int32_t *a) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * kThreads)
        a[i] = (int32_t)i;
}

// Stable LSD radix sort of (key, value) pairs, 8 key bits per pass (used to
// build A^T: sorting the caller-order entries by column label keeps each
// column's entries in caller row order).  One pass is three steps:
//   k_radix_count   per wave tile of kRadixTile consecutive items, the count
//                   of every digit, stored digit-major (counts[d * ntiles + t]);
//   k_scan_*        exclusive prefix sum of the counts in that order, i.e. the
//                   first output slot of digit d from tile t;
//   k_radix_scatter each wave re-reads its tile in order, 64 items per round;
//                   lanes holding the same digit find each other with eight
//                   ballots (one per digit bit), take their rank among the
//                   lower lanes, and the lowest of them advances the tile's
//                   running slot of that digit.  Items keep their input order
//                   within a digit, so the pass is stable.
// Integer counts only; results do not depend on scheduling.
constexpr int kRadixBins = 256;
constexpr int kRadixRounds = 64;
constexpr int64_t kRadixTile = 64 * kRadixRounds;  // items per wave tile
constexpr int kScanItems = 16;                     // per thread in the count scan
constexpr int64_t kScanChunk = (int64_t)kThreads * kScanItems;

__global__ __launch_bounds__(kThreads) void k_radix_count(int64_t n, const uint32_t *__restrict__ key,
                                                          int shift, int64_t ntiles,
                                                          int32_t *__restrict__ counts) {
    __shared__ int32_t hist[kWaveRows][kRadixBins];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * kWaveRows + w;
    for (int d = lane; d < kRadixBins; d += 64) hist[w][d] = 0;
    __syncthreads();
    if (tile < ntiles) {
        const int64_t base = tile * kRadixTile;
        for (int r = 0; r < kRadixRounds; ++r) {
            const int64_t i = base + (int64_t)r * 64 + lane;
            if (i < n) atomicAdd(&hist[w][(key[i] >> shift) & (kRadixBins - 1)], 1);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int d = lane; d < kRadixBins; d += 64) counts[(int64_t)d * ntiles + tile] = hist[w][d];
}

// sums[b] = sum of chunk b (kScanChunk consecutive counts)
__global__ __launch_bounds__(kThreads) void k_scan_chunks(int64_t len, const int32_t *__restrict__ in,
                                                          int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kWaveRows];
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    int32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = b0 + (int64_t)q * kThreads + threadIdx.x;
        if (i < len) s += in[i];
    }
    int32_t total = 0;
    (void)block_excl_scan_i32(s, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the chunk sums in place (one workgroup)
__global__ __launch_bounds__(kThreads) void k_scan_sums(int64_t len, int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kWaveRows];
    int32_t carry = 0;
    for (int64_t b = 0; b < len; b += kThreads) {
        const int64_t i = b + threadIdx.x;
        const int32_t v = i < len ? sums[i] : 0;
        int32_t total = 0;
        const int32_t ex = block_excl_scan_i32(v, lds, &total);
        if (i < len) sums[i] = carry + ex;
        carry += total;
    }
}

// exclusive scan of each chunk from its base; thread t owns kScanItems
// consecutive counts of the chunk
__global__ __launch_bounds__(kThreads) void k_scan_apply(int64_t len, int32_t *__restrict__ a,
                                                         const int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kWaveRows];
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (b0 + q < len) ? a[b0 + q] : 0;
        s += v[q];
    }
    int32_t total = 0;
    int32_t run = sums[blockIdx.x] + block_excl_scan_i32(s, lds, &total);
    for (int q = 0; q < kScanItems; ++q) {
        if (b0 + q < len) a[b0 + q] = run;
        run += v[q];
    }
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(int64_t n, const uint32_t *__restrict__ kin,
                                                            const int32_t *__restrict__ vin,
                                                            uint32_t *__restrict__ kout,
                                                            int32_t *__restrict__ vout, int shift,
                                                            int64_t ntiles,
                                                            const int32_t *__restrict__ offs) {
    __shared__ int32_t slot[kWaveRows][kRadixBins];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * kWaveRows + w;
    if (tile < ntiles)
        for (int d = lane; d < kRadixBins; d += 64) slot[w][d] = offs[(int64_t)d * ntiles + tile];
    __syncthreads();
    if (tile >= ntiles) return;
    const uint64_t lower = (1ull << lane) - 1ull;
    const int64_t base = tile * kRadixTile;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t first = base + (int64_t)r * 64;
        if (first >= n) break;  // uniform over the wave
        const int64_t i = first + lane;
        const bool ok = i < n;
        const uint32_t k = ok ? kin[i] : 0u;
        const int32_t v = ok ? vin[i] : 0;
        const uint32_t d = (k >> shift) & (kRadixBins - 1);
        uint64_t same = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t set = __ballot(bit);
            same &= bit ? set : ~set;
        }
        if (!ok) same = 0;
        const uint64_t below = same & lower;
        const int32_t at = slot[w][d];  // all lanes read before the leader advances it
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (ok) {
            const int32_t pos = at + __popcll(below);
            kout[pos] = k;
            vout[pos] = v;
            if (below == 0) slot[w][d] = at + __popcll(same);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// A^T from a stable sort of A's entries by column: row_ptr by lower_bound,
// col = original row, val gathered.
__global__ __launch_bounds__(kThreads) void k_transpose_finish(int64_t nnz, int n,
                                                               const int32_t *sorted_cols,
                                                               const int32_t *perm,
                                                               const int32_t *rowid,
                                                               const double *val,
                                                               int32_t *t_row_ptr, int32_t *t_col,
                                                               double *t_val) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x; j <= n; j += stride) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted_cols[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        t_row_ptr[j] = (int32_t)lo;
    }
    for (int64_t p = blockIdx.x * (int64_t)kThreads + threadIdx.x; p < nnz; p += stride) {
        const int32_t q = perm[p];
        t_col[p] = rowid[q];
        t_val[p] = val[q];
    }
}

// ------------------------------------------------- termination evaluation
//
// Section 7, eq. "rescaled-termination-criteria", in original units from a
// scaled point: x = D2 x~, y = D1 y~, A x = (A~ x~)/D1, A^T y = (A~^T y~)/D2.
// Values: 0 primal abs (max), 1 primal rel (max), 2 dual abs (max),
// 3 dual rel (max), 4 c^T x (sum), 5 dual objective terms (sum),
// 6 non-finite count (sum).

__global__ __launch_bounds__(kThreads) void k_kkt(int m, int n, const double *xs, const double *ys,
                                                  const double *axs, const double *atys,
                                                  const double *d1, const double *d2,
                                                  const double *c, const double *lc,
                                                  const double *uc, const double *lv,
                                                  const double *uv, int mode, double *part,
                                                  double *r_out, double *x_out, double *y_out) {
    __shared__ double red[7 * (kThreads / 64)];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    const int stride = gridDim.x * kThreads;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride) {
        const double y = d1[i] * ys[i];
        const double ax = axs[i] / d1[i];
        if (y_out) y_out[i] = y;
        const double l = lc[i], u = uc[i];
        double viol = 0.0;
        if (isfinite(l) && l - ax > viol) viol = l - ax;
        if (isfinite(u) && ax - u > viol) viol = ax - u;
        const bool lb = isfinite(l) && l != 0.0, ub = isfinite(u) && u != 0.0;
        double q;
        if (lb && !ub) q = fabs(l);
        else if (!lb && ub) q = fabs(u);
        else if (lb && ub) q = fmax(fabs(l), fabs(u));
        else q = 1.0;
        acc[0] = nan_max(acc[0], viol);
        acc[1] = nan_max(acc[1], viol / q);
        if (ys[i] > 0.0) acc[5] += l * y;
        else if (ys[i] < 0.0) acc[5] += u * y;
        if (!isfinite(y) || !isfinite(ax)) acc[6] += 1.0;
    }
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride) {
        const double x = d2[j] * xs[j];
        const double aty = atys[j] / d2[j];
        const double g = c[j] - aty;
        const double l = lv[j], u = uv[j];
        // the scaled bounds carry the rounding of the preconditioning rounds:
        // the output is clamped to the caller's bounds (a move of a few ulps)
        if (x_out) x_out[j] = clampd(x, l, u);
        double r;
        if (mode == 0) {
            if (!isfinite(l) && !isfinite(u)) r = 0.0;
            else if (!isfinite(l)) r = g < 0.0 ? g : 0.0;
            else if (!isfinite(u)) r = g > 0.0 ? g : 0.0;
            else r = g;
        } else {
            r = 0.0;
            if (g > 0.0 && x - l <= fabs(x)) r = g;
            if (g < 0.0 && u - x <= fabs(x)) r = g;
        }
        if (r_out) r_out[j] = r;
        const double res = fabs(g - r);
        const double sc = c[j] != 0.0 ? fabs(c[j]) : 1.0;
        acc[2] = nan_max(acc[2], res);
        acc[3] = nan_max(acc[3], res / sc);
        acc[4] += c[j] * x;
        if (r > 0.0) acc[5] += l * r;
        else if (r < 0.0) acc[5] += u * r;
        if (!isfinite(x) || !isfinite(aty)) acc[6] += 1.0;
    }
    write_partials<7, 0x0Fu>(acc, red, part);
}

__global__ void k_kkt_final(const double *part, int grid, double obj_offset, KktOut *out) {
    __shared__ double red[7 * (kThreads / 64)];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int g = threadIdx.x; g < grid; g += kThreads) {
        for (int i = 0; i < 4; ++i) v[i] = nan_max(v[i], part[g * 7 + i]);
        for (int i = 4; i < 7; ++i) v[i] += part[g * 7 + i];
    }
    block_reduce<7, 0x0Fu>(v, red);
    if (threadIdx.x == 0) {
        KktOut o;
        o.primal_res_abs = v[0];
        o.primal_res_rel = v[1];
        o.dual_res_abs = v[2];
        o.dual_res_rel = v[3];
        o.primal_obj = v[4] + obj_offset;
        o.dual_obj = v[5] + obj_offset;
        const double den = fabs(o.primal_obj) + fabs(o.dual_obj);
        o.rel_gap = den > 0.0 ? fabs(o.primal_obj - o.dual_obj) / den : 0.0;
        if (v[6] > 0.0) o.rel_gap = NAN;
        o.pad = v[6];
        *out = o;
    }
}

// ------------------------------------------- infeasibility certificates
//
// Section 3, "Infeasibility detection", Appendix D: a candidate (difference
// of the two latest iterates, the iterate, or the average) projected onto
// Xbar x Y in the scaled space, then its products, then the test values of
// cert_row / cert_col.

__global__ __launch_bounds__(kThreads) void k_cert_point(int m, int n, const double *xa,
                                                         const double *xb, const double *ya,
                                                         const double *yb, const double *lc,
                                                         const double *uc, const double *lv,
                                                         const double *uv, double *px,
                                                         double *py) {
    const int stride = gridDim.x * kThreads;
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride) {
        const double x = xb ? xa[j] - xb[j] : xa[j];
        px[j] = proj_xbar(x, lv[j], uv[j]);
    }
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride) {
        const double y = yb ? ya[i] - yb[i] : ya[i];
        py[i] = proj_ycone(y, lc[i], uc[i]);
    }
}

__global__ __launch_bounds__(kThreads) void k_cert(int m, int n, const double *px,
                                                   const double *py, const double *pax,
                                                   const double *paty, const double *d1,
                                                   const double *d2, const double *c,
                                                   const double *lc, const double *uc,
                                                   const double *lv, const double *uv,
                                                   double *part) {
    __shared__ double red[kCertVals * (kThreads / 64)];
    double acc[kCertVals] = {0, 0, 0, 0, 0};
    const int stride = gridDim.x * kThreads;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride)
        cert_row(py[i], pax ? pax[i] : 0.0, d1[i], lc[i], uc[i], acc);
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride)
        cert_col(px ? px[j] : 0.0, paty[j], d2[j], c[j], lv[j], uv[j], acc);
    write_partials<kCertVals, kCertMax>(acc, red, part);
}

__global__ void k_cert_final(const double *part, int grid, CertOut *out) {
    __shared__ double red[kCertVals * (kThreads / 64)];
    double v[kCertVals] = {0, 0, 0, 0, 0};
    for (int g = threadIdx.x; g < grid; g += kThreads) {
        for (int i = 0; i < kCertVals; ++i) {
            const double p = part[g * kCertVals + i];
            v[i] = ((kCertMax >> i) & 1u) ? nan_max(v[i], p) : v[i] + p;
        }
    }
    block_reduce<kCertVals, kCertMax>(v, red);
    if (threadIdx.x == 0) *out = CertOut{v[0], v[1], v[2], v[3], v[4]};
}

__global__ __launch_bounds__(kThreads) void k_cert_out(int m, int n, const double *px,
                                                       const double *py, const double *paty,
                                                       const double *d1, const double *d2,
                                                       const double *lv, const double *uv,
                                                       double *x_out, double *y_out,
                                                       double *r_out) {
    const int stride = gridDim.x * kThreads;
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < n; j += stride) {
        x_out[j] = px ? d2[j] * px[j] : 0.0;
        r_out[j] = proj_rcone(-(paty[j] / d2[j]), lv[j], uv[j]);
    }
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += stride) y_out[i] = d1[i] * py[i];
}

// -------------------------------------------------- normalized duality gap
//
// mu(z, z_ref) = (1/r) max { L(x, y^) - L(x^, y) : z^ in X x Y, ||z^ - z||_omega <= r },
// r = ||z - z_ref||_omega (Section 3, "Adaptive restarts").  The maximizer is
// the point of the proximal path
//   x^_j(s) = clamp(x_j - s g_j / omega, lv_j, uv_j),  g = c - A^T y,
//   y^_i(s) = y_i + s omega a_i if > 0; y_i + s omega b_i if < 0; else 0,
//   a_i = lc_i - (A x)_i,  b_i = uc_i - (A x)_i,
// at which D(s) = ||z^(s) - z||_omega^2 reaches r^2.
//
// Each coordinate's share of D is piecewise with at most two breakpoints,
//   D_i(s) = a1 s^2 (s < b1),  c (b1 <= s < b2),  a3 s^2 (s >= b2),
// and its share of the objective is linear on the same pieces,
//   f_i(s) = f1 s,  f0,  f3 s + f3b.
// The search evaluates D at 32 abscissae per pass (geometric first, then
// uniform inside the bracket) together with S(s) = sum of segment indices,
// whose difference between neighbouring abscissae counts the breakpoints in
// between.  Once the bracket holding r^2 has none, D = A s^2 + B and
// f = F1 s + F0 there, so s* = sqrt((r^2 - B)/A) and mu = (F1 s* + F0)/r.

__device__ __forceinline__ Seg coord_seg(int idx, int n, Vecs v, const double *x, const double *y,
                                         const double *ax, const double *aty, double omega) {
    if (idx < n) return seg_x(x[idx], v.c[idx] - aty[idx], v.lv[idx], v.uv[idx], omega);
    const int i = idx - n;
    const bool af = isfinite(v.lc[i]), bf = isfinite(v.uc[i]);
    return seg_y(y[i], af, af ? v.lc[i] - ax[i] : 0.0, bf, bf ? v.uc[i] - ax[i] : 0.0, omega);
}

// setup: 0 r^2, 1 A0 (weight of coordinates moving at s -> 0+), 2 D(inf), 3 non-finite count
__global__ __launch_bounds__(kThreads) void k_gap_setup(int m, int n, Vecs v, const double *x,
                                                        const double *y, const double *ax,
                                                        const double *aty, const double *xr,
                                                        const double *yr, double omega,
                                                        double *part) {
    __shared__ double red[4 * (kThreads / 64)];
    double acc[4] = {0, 0, 0, 0};
    const int total = n + m;
    for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
        double d, zi;
        if (idx < n) {
            zi = x[idx];
            d = zi - xr[idx];
            acc[0] += omega * d * d;
        } else {
            zi = y[idx - n];
            d = zi - yr[idx - n];
            acc[0] += d * d / omega;
        }
        const Seg q = coord_seg(idx, n, v, x, y, ax, aty, omega);
        if (q.b1 > 0.0) acc[1] += q.a1;
        acc[2] += isfinite(q.b2) ? INFINITY : (isfinite(q.b1) ? q.c : (q.a1 > 0.0 ? INFINITY : 0.0));
        if (!isfinite(zi) || !isfinite(q.a1)) acc[3] += 1.0;
    }
    write_partials<4>(acc, red, part);
}

__global__ void k_gap_init(const double *part, int grid, double omega, GapState *gs) {
    __shared__ double red[4 * (kThreads / 64)];
    double v[4] = {0, 0, 0, 0};
    for (int g = threadIdx.x; g < grid; g += kThreads)
        for (int i = 0; i < 4; ++i) v[i] += part[g * 4 + i];
    block_reduce<4>(v, red);
    if (threadIdx.x != 0) return;
    GapState s;
    s.r2 = v[0];
    s.r = sqrt(v[0]);
    s.omega = omega;
    s.A0 = v[1];
    s.Dinf = v[2];
    s.lo = 0.0;
    s.hi = INFINITY;
    s.npass = 0;
    s.done = 0;
    s.pathend = 0;
    s.linear = 0;
    s.s_star = 0.0;
    s.Acoef = s.Bcoef = s.f = s.mu = 0.0;
    s.bad = (v[3] > 0.0 || !isfinite(v[0]) || !isfinite(v[1])) ? 1 : 0;

    if (s.bad) {
        s.done = 2;
        s.mu = NAN;
    } else if (!(s.r2 > 0.0) || !(s.A0 > 0.0)) {
        s.done = 2;  // mu = 0: zero radius, or nothing on the path moves
        s.mu = 0.0;
    } else if (s.Dinf <= s.r2) {
        s.done = 1;  // the whole path lies inside the ball: evaluate at its end
        s.pathend = 1;
    } else {
        const double sg = s.r / sqrt(s.A0);
        for (int i = 0; i < kGapPts; ++i) s.pts[i] = sg * exp2(0.5 * i);
    }
    // active-set iteration: the first abscissa is the step from s -> 0+
    s.newton = s.done ? 0 : 1;
    s.s_prev = 2.2250738585072014e-308;
    s.D_prev = 0.0;
    s.s_cur = s.done ? 0.0 : s.r / sqrt(s.A0);
    s.nsteps = 0;
    s.exact = 0;
    *gs = s;
}

// Active-set step: at s = s_cur, D(s), the coefficients A, B of the segment
// containing s, the objective pieces F1, F0, and the number of coordinates
// whose segment differs between s_prev and s_cur.
__global__ __launch_bounds__(kThreads) void k_gap_step(int m, int n, Vecs v, const double *x,
                                                       const double *y, const double *ax,
                                                       const double *aty, const GapState *gs,
                                                       double *part) {
    if (gs->done || !gs->newton) return;
    __shared__ double red[6 * (kThreads / 64)];
    const double omega = gs->omega, sc = gs->s_cur, sp = gs->s_prev;
    const double sc2 = sc * sc;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int total = n + m;
    for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
        const Seg q = coord_seg(idx, n, v, x, y, ax, aty, omega);
        const int gc = (int)(sc >= q.b1) + (int)(sc >= q.b2);
        const int gp = (int)(sp >= q.b1) + (int)(sp >= q.b2);
        if (gc == 2) {
            acc[0] += q.a3 * sc2;
            acc[1] += q.a3;
            acc[3] += q.f3;
            acc[4] += q.f3b;
        } else if (gc == 1) {
            acc[0] += q.c;
            acc[2] += q.c;
            acc[4] += q.f0;
        } else {
            acc[0] += q.a1 * sc2;
            acc[1] += q.a1;
            acc[3] += q.f1;
        }
        if (gc != gp) acc[5] += 1.0;
    }
    write_partials<6>(acc, red, part);
}

__global__ void k_gap_update(const double *part, int grid, GapState *gs) {
    if (gs->done || !gs->newton) return;
    __shared__ double red[6 * (kThreads / 64)];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int g = threadIdx.x; g < grid; g += kThreads)
        for (int i = 0; i < 6; ++i) v[i] += part[g * 6 + i];
    block_reduce<6>(v, red);
    if (threadIdx.x != 0) return;
    GapState s = *gs;
    const double Dk = v[0], A = v[1], B = v[2], F1 = v[3], F0 = v[4], cnt = v[5];
    const double sc = s.s_cur;
    if (Dk < s.r2) s.lo = fmax(s.lo, sc);
    else s.hi = fmin(s.hi, sc);
    s.nsteps += 1;
    // root of D = A s^2 + B on the segment holding s_cur
    double st = A > 0.0 ? sqrt((s.r2 - B) / A) : NAN;
    const double a = fmin(s.s_prev, sc), b = fmax(s.s_prev, sc);
    const bool at_root = fabs(st - sc) <= 1e-13 * sc;  // D(s_cur) = r^2 on its own segment
    if (at_root || (cnt == 0.0 && st >= a * (1.0 - 1e-12) && st <= b * (1.0 + 1e-12))) {
        // the root of the segment holding s_cur is s_cur itself, or there is no
        // breakpoint between s_prev and s_cur and the root lies there: exact
        // up to rounding
        st = at_root ? sc : fmin(fmax(st, a), b);
        s.s_star = st;
        s.Acoef = A;
        s.Bcoef = B;
        s.f = F1 * st + F0;
        s.mu = s.f / s.r;
        s.done = 3;
        s.newton = 0;
        s.exact = 1;
        *gs = s;
        return;
    }
    double nxt = A > 0.0 ? st : INFINITY;
    if (!(nxt > s.lo && nxt < s.hi) || nxt == sc)
        nxt = isfinite(s.hi) ? 0.5 * (s.lo + s.hi) : 2.0 * fmax(s.lo, sc);
    s.s_prev = sc;
    s.D_prev = Dk;
    s.s_cur = nxt;
    if (s.nsteps >= kGapNewton || !(s.hi > s.lo)) {
        // hand the bracket to the multisection search
        s.newton = 0;
        if (isfinite(s.hi)) {
            const double w = (s.hi - s.lo) / (double)(kGapPts - 1);
            for (int i = 0; i < kGapPts; ++i) s.pts[i] = s.lo + w * (double)i;
            s.pts[kGapPts - 1] = s.hi;
            s.linear = 1;
            if (!(w > 0.0)) s.done = 1;
        } else {
            const double b0 = s.lo > 0.0 ? s.lo : sc;
            for (int i = 0; i < kGapPts; ++i) s.pts[i] = b0 * exp2(0.5 * (i + 1));
        }
    }
    *gs = s;
}

// One multisection pass: D at pts[p] (values 0..31) and S = sum of segment
// indices at pts[p] (values 32..63).
constexpr int kGapNV = 2 * kGapPts;

__global__ __launch_bounds__(kThreads) void k_gap_pass(int m, int n, Vecs v, const double *x,
                                                       const double *y, const double *ax,
                                                       const double *aty, const GapState *gs,
                                                       double *part) {
    if (gs->done || gs->newton) return;
    __shared__ double red[kGapNV * (kThreads / 64)];
    __shared__ double pts[kGapPts], pts2[kGapPts];
    if (threadIdx.x < kGapPts) {
        const double s = gs->pts[threadIdx.x];
        pts[threadIdx.x] = s;
        pts2[threadIdx.x] = s * s;
    }
    const double omega = gs->omega;
    __syncthreads();
    double acc[kGapPts];
    int cnt[kGapPts];
#pragma unroll
    for (int i = 0; i < kGapPts; ++i) {
        acc[i] = 0.0;
        cnt[i] = 0;
    }
    const int total = n + m;
    for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
        const Seg q = coord_seg(idx, n, v, x, y, ax, aty, omega);
#pragma unroll
        for (int p = 0; p < kGapPts; ++p) {
            const double s = pts[p];
            const bool s1 = s >= q.b1, s2 = s >= q.b2;
            acc[p] += s2 ? q.a3 * pts2[p] : (s1 ? q.c : q.a1 * pts2[p]);
            cnt[p] += (int)s1 + (int)s2;
        }
    }
    double all[kGapNV];
#pragma unroll
    for (int i = 0; i < kGapPts; ++i) {
        all[i] = acc[i];
        all[kGapPts + i] = (double)cnt[i];
    }
    write_partials<kGapNV>(all, red, part);
}

__global__ __launch_bounds__(kThreads) void k_gap_select(const double *part, int grid,
                                                         GapState *gs) {
    if (gs->done || gs->newton) return;
    // value i is summed by the four lanes i, i+64, i+128, i+192 (grid slices
    // g = t/64 mod 4), then combined in a fixed order
    __shared__ double quarter[4][kGapNV];
    __shared__ double tot[kGapNV];
    {
        const int i = threadIdx.x % kGapNV, q = threadIdx.x / kGapNV;
        double a = 0.0;
        for (int g = q; g < grid; g += 4) a += part[g * kGapNV + i];
        quarter[q][i] = a;
    }
    __syncthreads();
    if (threadIdx.x < kGapNV)
        tot[threadIdx.x] = ((quarter[0][threadIdx.x] + quarter[1][threadIdx.x]) +
                            quarter[2][threadIdx.x]) + quarter[3][threadIdx.x];
    __syncthreads();
    if (threadIdx.x != 0) return;
    GapState s = *gs;
    int q = -1;
    for (int p = 0; p < kGapPts; ++p)
        if (tot[p] >= s.r2) {
            q = p;
            break;
        }
    s.npass += 1;
    bool refine = true;
    double count = 1.0;
    if (q < 0) {
        // all abscissae inside the ball: continue geometrically (never in linear mode)
        s.lo = s.pts[kGapPts - 1];
        for (int i = 0; i < kGapPts; ++i) s.pts[i] = s.lo * exp2(0.5 * (i + 1));
        refine = false;
    } else if (q == 0) {
        // bracket (lo, pts[0]] -- its inside has not been counted yet
        s.hi = s.pts[0];
        count = 1.0;
    } else {
        s.lo = s.pts[q - 1];
        s.hi = s.pts[q];
        count = tot[kGapPts + q] - tot[kGapPts + q - 1];
    }
    if (refine) {
        if (count == 0.0) {
            s.done = 1;
        } else {
            const double w = (s.hi - s.lo) / (double)(kGapPts - 1);
            s.linear = 1;
            for (int i = 0; i < kGapPts; ++i) s.pts[i] = s.lo + w * (double)i;
            s.pts[kGapPts - 1] = s.hi;
            if (!(w > 0.0) || s.pts[1] == s.lo) s.done = 1;  // cannot split further
        }
    }
    if (s.npass >= kGapMaxPass) s.done = 1;
    *gs = s;
}

// Coefficients of D = A s^2 + B and f = F1 s + F0 on the final bracket
// (evaluated at its midpoint, or at the end of the path).
__global__ __launch_bounds__(kThreads) void k_gap_classify(int m, int n, Vecs v, const double *x,
                                                           const double *y, const double *ax,
                                                           const double *aty, const GapState *gs,
                                                           double *part) {
    if (gs->done != 1) return;
    __shared__ double red[4 * (kThreads / 64)];
    const double omega = gs->omega;
    const double sm = gs->pathend ? 1e300 : 0.5 * (gs->lo + gs->hi);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int total = n + m;
    for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
        const Seg q = coord_seg(idx, n, v, x, y, ax, aty, omega);
        if (sm >= q.b2) {
            acc[0] += q.a3;
            acc[2] += q.f3;
            acc[3] += q.f3b;
        } else if (sm >= q.b1) {
            acc[1] += q.c;
            acc[3] += q.f0;
        } else {
            acc[0] += q.a1;
            acc[2] += q.f1;
        }
    }
    write_partials<4>(acc, red, part);
}

__global__ void k_gap_solve(const double *part, int grid, GapState *gs) {
    if (gs->done != 1) return;
    __shared__ double red[4 * (kThreads / 64)];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = threadIdx.x; g < grid; g += kThreads)
        for (int i = 0; i < 4; ++i) v[i] += part[g * 4 + i];
    block_reduce<4>(v, red);
    if (threadIdx.x != 0) return;
    GapState s = *gs;
    s.Acoef = v[0];
    s.Bcoef = v[1];
    double st;
    if (s.pathend) {
        st = 0.0;  // nothing moves at the end of the path: f = F0
    } else if (s.Acoef > 0.0) {
        st = sqrt((s.r2 - s.Bcoef) / s.Acoef);
        if (!(st >= s.lo)) st = s.lo;
        if (st > s.hi) st = s.hi;
    } else {
        st = s.lo;
    }
    s.s_star = st;
    s.f = v[2] * st + v[3];
    s.mu = s.f / s.r;
    s.done = 3;
    *gs = s;
}

// ------------------------------------------------------------ rate probes

// Streaming copy with four 16-byte loads in flight per lane (the fastest of
// 1, 2, 4 and 8 measured on MI355X: 4.5, 4.8, 5.3 and 3.8 TB/s).
__global__ __launch_bounds__(kThreads) void k_rate_copy(int64_t len2, const double2 *a,
                                                        double2 *b) {
    constexpr int kU = 4;
    const int64_t stride = (int64_t)gridDim.x * kThreads * kU;
    for (int64_t base = blockIdx.x * (int64_t)kThreads * kU + threadIdx.x; base < len2;
         base += stride) {
        double2 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + (int64_t)u * kThreads;
            if (i < len2) v[u] = a[i];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + (int64_t)u * kThreads;
            if (i < len2) b[i] = v[u];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_rate_idx(int64_t n, uint32_t domain, uint32_t *idx) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
        h ^= h >> 29;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 32;
        idx[i] = (uint32_t)(h % domain);
    }
}

__global__ __launch_bounds__(kThreads) void k_rate_gather(int64_t n, const uint32_t *idx,
                                                          const double *x, double *out) {
    constexpr int kPer = 8;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads * kPer;
    for (int64_t base = (int64_t)blockIdx.x * kThreads * kPer + threadIdx.x; base < n;
         base += stride) {
        uint32_t k[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int64_t i = base + (int64_t)j * kThreads;
            k[j] = i < n ? __builtin_nontemporal_load(idx + i) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (base + (int64_t)j * kThreads < n) s += x[k[j]];
    }
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// --------------------------------------------------------------- launchers

static inline int grid_for(int64_t len, int cap = 2048) {
    int64_t g = (len + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// With events, the launch records its own start/stop timestamps in the
// dispatch (no extra packets on the stream), for kernel timing.
#define PDLP_LAUNCH(kern, grid, ev, s, ...)                                                  \
    do {                                                                                     \
        if (ev)                                                                              \
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, (ev)[0], (ev)[1], 0, \
                                  __VA_ARGS__);                                              \
        else                                                                                 \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__);         \
    } while (0)

hipError_t launch_primal(hipStream_t s, int n, Vecs v, Iter it, const Ctrl *ctrl, double *part,
                         int grid, hipEvent_t *ev) {
    PDLP_LAUNCH(k_primal, grid, ev, s, n, v, it, ctrl, part);
    return hipGetLastError();
}

hipError_t launch_spmv_dual(hipStream_t s, const DCsr &A, Vecs v, Iter it, const Ctrl *ctrl,
                            double *part, hipEvent_t *ev) {
    if (A.grid > 0) PDLP_LAUNCH(k_spmv_dual, A.grid, ev, s, A, v, it, ctrl, part);
    return hipGetLastError();
}

hipError_t launch_step_decide(hipStream_t s, Ctrl *ctrl, const double *part_dual, int gd,
                              const double *part_ps, int gps, const double *part_pf, int gpf,
                              hipEvent_t *ev) {
    PDLP_LAUNCH(k_step_decide, 1, ev, s, ctrl, part_dual, gd, part_ps, gps, part_pf, gpf);
    return hipGetLastError();
}

hipError_t launch_spmv_primal(hipStream_t s, const DCsr &AT, Vecs v, Iter it, const Ctrl *ctrl,
                              double *part, hipEvent_t *ev) {
    if (AT.grid > 0) PDLP_LAUNCH(k_spmv_primal, AT.grid, ev, s, AT, v, it, ctrl, part);
    return hipGetLastError();
}

hipError_t launch_flush_sy(hipStream_t s, int m, Iter it, Ctrl *ctrl) {
    if (m > 0) hipLaunchKernelGGL(k_flush_sy, dim3(grid_for(m)), dim3(kThreads), 0, s, m, it, ctrl);
    hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

hipError_t launch_seg_primal(hipStream_t s, const SegCsr &sg, Vecs v, Iter it, const Ctrl *ctrl,
                             double *part, hipEvent_t *ev) {
    if (sg.grid1 > 0) PDLP_LAUNCH(k_seg_gather_primal, sg.grid1, ev, s, sg, it, ctrl);
    if (sg.P.grid > 0) PDLP_LAUNCH(k_seg_primal, sg.P.grid, ev ? ev + 2 : nullptr, s, sg, v, it, ctrl, part);
    return hipGetLastError();
}

hipError_t launch_seg_plain(hipStream_t s, const SegCsr &sg, const double *v, double *out) {
    if (sg.grid1 > 0)
        hipLaunchKernelGGL(k_seg_gather_plain, dim3(sg.grid1), dim3(kThreads), 0, s, sg, v);
    if (sg.P.grid > 0)
        hipLaunchKernelGGL(k_seg_plain, dim3(sg.P.grid), dim3(kThreads), 0, s, sg, out);
    return hipGetLastError();
}

hipError_t launch_spmv_plain(hipStream_t s, const DCsr &A, const double *x, double *out) {
    if (A.grid > 0)
        hipLaunchKernelGGL(k_spmv_plain, dim3(A.grid), dim3(kThreads), 0, s, A, x, out);
    return hipGetLastError();
}

hipError_t launch_scale_div(hipStream_t s, int64_t len, const double *a, const double *d,
                            double *out) {
    if (len > 0) hipLaunchKernelGGL(k_div, dim3(grid_for(len)), dim3(kThreads), 0, s, len, a, d, out);
    return hipGetLastError();
}

hipError_t launch_scale_mul(hipStream_t s, int64_t len, const double *a, const double *d,
                            double *out) {
    if (len > 0) hipLaunchKernelGGL(k_mul, dim3(grid_for(len)), dim3(kThreads), 0, s, len, a, d, out);
    return hipGetLastError();
}

hipError_t launch_average(hipStream_t s, int64_t len, const double *sum, double seta,
                          double *out) {
    if (len > 0)
        hipLaunchKernelGGL(k_average, dim3(grid_for(len)), dim3(kThreads), 0, s, len, sum, seta, out);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, int64_t len, double *a, double v) {
    if (len > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(len)), dim3(kThreads), 0, s, len, a, v);
    return hipGetLastError();
}

hipError_t launch_take(hipStream_t s, int64_t len, const int64_t *perm, const double *src,
                       double *dst) {
    if (len > 0)
        hipLaunchKernelGGL(k_take, dim3(grid_for(len)), dim3(kThreads), 0, s, len, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, int64_t len, const double *a, double *out) {
    if (len > 0) hipLaunchKernelGGL(k_copy, dim3(grid_for(len)), dim3(kThreads), 0, s, len, a, out);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, int64_t len, const int32_t *perm, const double *in,
                         double *out) {
    if (len > 0)
        hipLaunchKernelGGL(k_gather, dim3(grid_for(len)), dim3(kThreads), 0, s, len, perm, in, out);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t len, const int32_t *perm, const double *in,
                          double *out) {
    if (len > 0)
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(len)), dim3(kThreads), 0, s, len, perm, in, out);
    return hipGetLastError();
}

hipError_t launch_clamp0(hipStream_t s, int n, const double *lv, const double *uv, double *x) {
    if (n > 0) hipLaunchKernelGGL(k_clamp0, dim3(grid_for(n)), dim3(kThreads), 0, s, n, lv, uv, x);
    return hipGetLastError();
}

hipError_t launch_dist2(hipStream_t s, int64_t len, const double *a, const double *b, double *part,
                        int grid, double *out) {
    hipLaunchKernelGGL(k_dist2, dim3(grid), dim3(kThreads), 0, s, len, a, b, part);
    hipLaunchKernelGGL(k_sum_max, dim3(1), dim3(kThreads), 0, s, part, grid, 1, 0u, out);
    return hipGetLastError();
}

hipError_t launch_sum_max(hipStream_t s, const double *part, int grid, int nv, const int *is_max,
                          double *out) {
    unsigned mask = 0;
    for (int i = 0; i < nv; ++i)
        if (is_max[i]) mask |= 1u << i;
    hipLaunchKernelGGL(k_sum_max, dim3(1), dim3(kThreads), 0, s, part, grid, nv, mask, out);
    return hipGetLastError();
}

hipError_t launch_absmax(hipStream_t s, int64_t len, const double *a, double *part, int grid,
                         double *out) {
    hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(kThreads), 0, s, len, a, part);
    hipLaunchKernelGGL(k_sum_max, dim3(1), dim3(kThreads), 0, s, part, grid, 1, 1u, out);
    return hipGetLastError();
}

hipError_t launch_primal_weight_init(hipStream_t s, int m, int n, const double *c,
                                     const double *lc, const double *uc, double *part, int grid,
                                     double *out) {
    hipLaunchKernelGGL(k_pw_init, dim3(grid), dim3(kThreads), 0, s, m, n, c, lc, uc, part);
    hipLaunchKernelGGL(k_sum_max, dim3(1), dim3(kThreads), 0, s, part, grid, 2, 0u, out);
    return hipGetLastError();
}

hipError_t launch_row_norms(hipStream_t s, const DCsr &A, int use_inf, double *out) {
    if (A.rows > 0)
        hipLaunchKernelGGL(k_row_norms, dim3(grid_for(A.rows, 65535)), dim3(kThreads), 0, s, A,
                           use_inf, out);
    return hipGetLastError();
}

hipError_t launch_norm_to_factor(hipStream_t s, int len, double *nrm) {
    if (len > 0)
        hipLaunchKernelGGL(k_norm_to_factor, dim3(grid_for(len)), dim3(kThreads), 0, s, len, nrm);
    return hipGetLastError();
}

hipError_t launch_scale_matrix(hipStream_t s, const DCsr &A, const double *rf, const double *cf) {
    if (A.rows > 0)
        hipLaunchKernelGGL(k_scale_matrix, dim3(grid_for(A.rows, 65535)), dim3(kThreads), 0, s, A,
                           rf, cf);
    return hipGetLastError();
}

hipError_t launch_div_inplace(hipStream_t s, int len, double *d, const double *f) {
    if (len > 0)
        hipLaunchKernelGGL(k_div_inplace, dim3(grid_for(len)), dim3(kThreads), 0, s, len, d, f);
    return hipGetLastError();
}

hipError_t launch_scale_vectors(hipStream_t s, int m, int n, const double *d1, const double *d2,
                                const double *c, const double *lc, const double *uc,
                                const double *lv, const double *uv, double *cs, double *lcs,
                                double *ucs, double *lvs, double *uvs) {
    hipLaunchKernelGGL(k_scale_vectors, dim3(grid_for(m > n ? m : n)), dim3(kThreads), 0, s, m, n,
                       d1, d2, c, lc, uc, lv, uv, cs, lcs, ucs, lvs, uvs);
    return hipGetLastError();
}

hipError_t launch_row_ids(hipStream_t s, int m, const int32_t *row_ptr, int32_t *rowid) {
    if (m > 0)
        hipLaunchKernelGGL(k_row_ids, dim3(grid_for(m, 65535)), dim3(kThreads), 0, s, m, row_ptr,
                           rowid);
    return hipGetLastError();
}

hipError_t launch_row_ids_mapped(hipStream_t s, int m, const int32_t *row_ptr,
                                 const int32_t *new_row, int32_t *rowid) {
    if (m > 0)
        hipLaunchKernelGGL(k_row_ids_mapped, dim3(grid_for(m, 65535)), dim3(kThreads), 0, s, m,
                           row_ptr, new_row, rowid);
    return hipGetLastError();
}

hipError_t launch_relabel(hipStream_t s, int64_t nnz, const int32_t *col, const int32_t *new_col,
                          uint32_t *key) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(nnz, 65535)), dim3(kThreads), 0, s, nnz, col,
                           new_col, key);
    return hipGetLastError();
}

hipError_t launch_permute_rows(hipStream_t s, int m, const int32_t *row_order,
                               const int32_t *old_rp, const int32_t *old_col,
                               const double *old_val, const int32_t *new_col,
                               const int32_t *new_rp, int32_t *ncol, double *nval,
                               int32_t *orig_pos) {
    if (m > 0)
        hipLaunchKernelGGL(k_permute_rows, dim3(grid_for(m, 65535)), dim3(kThreads), 0, s, m,
                           row_order, old_rp, old_col, old_val, new_col, new_rp, ncol, nval,
                           orig_pos);
    return hipGetLastError();
}

hipError_t launch_iota(hipStream_t s, int64_t len, int32_t *a) {
    if (len > 0) hipLaunchKernelGGL(k_iota, dim3(grid_for(len)), dim3(kThreads), 0, s, len, a);
    return hipGetLastError();
}

int64_t radix_sort_temp_ints(int64_t n) {
    const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    const int64_t len = ntiles * kRadixBins;
    const int64_t nchunks = (len + kScanChunk - 1) / kScanChunk;
    return len + nchunks + 64;
}

hipError_t radix_sort_pairs(hipStream_t s, int64_t n, int key_bits, uint32_t *keys[2],
                            int32_t *vals[2], int32_t *temp, int *which) {
    int cur = 0;
    if (n > 0) {
        const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
        const int64_t len = ntiles * kRadixBins;
        const int64_t nchunks = (len + kScanChunk - 1) / kScanChunk;
        int32_t *counts = temp, *sums = temp + len;
        const int64_t wgs = (ntiles + kWaveRows - 1) / kWaveRows;
        if (wgs > 0x7fffffffLL || nchunks > 0x7fffffffLL) return hipErrorInvalidValue;
        for (int shift = 0; shift < key_bits; shift += 8) {
            hipLaunchKernelGGL(k_radix_count, dim3((unsigned)wgs), dim3(kThreads), 0, s, n,
                               keys[cur], shift, ntiles, counts);
            hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(kThreads), 0, s, len,
                               counts, sums);
            hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, s, nchunks, sums);
            hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(kThreads), 0, s, len,
                               counts, sums);
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)wgs), dim3(kThreads), 0, s, n,
                               keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], shift, ntiles,
                               counts);
            cur ^= 1;
        }
    }
    *which = cur;
    return hipGetLastError();
}

hipError_t launch_transpose_finish(hipStream_t s, int64_t nnz, int n, const int32_t *sorted_cols,
                                   const int32_t *perm, const int32_t *rowid, const double *val,
                                   int32_t *t_row_ptr, int32_t *t_col, double *t_val) {
    const int64_t len = nnz > (int64_t)n + 1 ? nnz : (int64_t)n + 1;
    hipLaunchKernelGGL(k_transpose_finish, dim3(grid_for(len, 65535)), dim3(kThreads), 0, s, nnz,
                       n, sorted_cols, perm, rowid, val, t_row_ptr, t_col, t_val);
    return hipGetLastError();
}

hipError_t launch_cert_point(hipStream_t s, int m, int n, const double *xa, const double *xb,
                             const double *ya, const double *yb, const double *lc,
                             const double *uc, const double *lv, const double *uv, double *px,
                             double *py) {
    const int64_t len = std::max(m, n);
    if (len > 0)
        hipLaunchKernelGGL(k_cert_point, dim3(grid_for(len)), dim3(kThreads), 0, s, m, n, xa, xb,
                           ya, yb, lc, uc, lv, uv, px, py);
    return hipGetLastError();
}

hipError_t launch_cert(hipStream_t s, int m, int n, const double *px, const double *py,
                       const double *pax, const double *paty, const double *d1, const double *d2,
                       const double *c, const double *lc, const double *uc, const double *lv,
                       const double *uv, double *part, int grid, CertOut *out) {
    hipLaunchKernelGGL(k_cert, dim3(grid), dim3(kThreads), 0, s, m, n, px, py, pax, paty, d1, d2,
                       c, lc, uc, lv, uv, part);
    hipLaunchKernelGGL(k_cert_final, dim3(1), dim3(kThreads), 0, s, part, grid, out);
    return hipGetLastError();
}

hipError_t launch_cert_out(hipStream_t s, int m, int n, const double *px, const double *py,
                           const double *paty, const double *d1, const double *d2,
                           const double *lv, const double *uv, double *x_out, double *y_out,
                           double *r_out) {
    const int64_t len = std::max(m, n);
    if (len > 0)
        hipLaunchKernelGGL(k_cert_out, dim3(grid_for(len)), dim3(kThreads), 0, s, m, n, px, py,
                           paty, d1, d2, lv, uv, x_out, y_out, r_out);
    return hipGetLastError();
}

hipError_t launch_kkt(hipStream_t s, int m, int n, const double *xs, const double *ys,
                      const double *axs, const double *atys, const double *d1, const double *d2,
                      const double *c, const double *lc, const double *uc, const double *lv,
                      const double *uv, int mode, double obj_offset, double *part, int grid,
                      double *r_out, double *x_out, double *y_out, KktOut *out) {
    hipLaunchKernelGGL(k_kkt, dim3(grid), dim3(kThreads), 0, s, m, n, xs, ys, axs, atys, d1, d2, c,
                       lc, uc, lv, uv, mode, part, r_out, x_out, y_out);
    hipLaunchKernelGGL(k_kkt_final, dim3(1), dim3(kThreads), 0, s, part, grid, obj_offset, out);
    return hipGetLastError();
}

hipError_t launch_rate_copy(hipStream_t s, int64_t len, const double *a, double *b) {
    hipLaunchKernelGGL(k_rate_copy, dim3(4096), dim3(kThreads), 0, s, len / 2,
                       reinterpret_cast<const double2 *>(a), reinterpret_cast<double2 *>(b));
    return hipGetLastError();
}

hipError_t launch_rate_idx(hipStream_t s, int64_t n, uint32_t domain, uint32_t *idx) {
    hipLaunchKernelGGL(k_rate_idx, dim3(4096), dim3(kThreads), 0, s, n, domain, idx);
    return hipGetLastError();
}

hipError_t launch_rate_gather(hipStream_t s, int64_t n, const uint32_t *idx, const double *x,
                              double *out, int grid) {
    hipLaunchKernelGGL(k_rate_gather, dim3(grid), dim3(kThreads), 0, s, n, idx, x, out);
    return hipGetLastError();
}

hipError_t launch_gap_head(hipStream_t s, int m, int n, Vecs v, const double *x,
                           const double *y, const double *ax, const double *aty,
                           const double *xr, const double *yr, double omega, double *part,
                           int grid, GapState *gs) {
    hipLaunchKernelGGL(k_gap_setup, dim3(grid), dim3(kThreads), 0, s, m, n, v, x, y, ax, aty, xr,
                       yr, omega, part);
    hipLaunchKernelGGL(k_gap_init, dim3(1), dim3(kThreads), 0, s, part, grid, omega, gs);
    for (int p = 0; p < kGapHead; ++p) {
        hipLaunchKernelGGL(k_gap_step, dim3(grid), dim3(kThreads), 0, s, m, n, v, x, y, ax, aty,
                           gs, part);
        hipLaunchKernelGGL(k_gap_update, dim3(1), dim3(kThreads), 0, s, part, grid, gs);
    }
    return hipGetLastError();
}

hipError_t launch_gap(hipStream_t s, int m, int n, Vecs v, const double *x, const double *y,
                      const double *ax, const double *aty, const double *xr, const double *yr,
                      double omega, double *part, int grid, GapState *gs) {
    const hipError_t e = launch_gap_head(s, m, n, v, x, y, ax, aty, xr, yr, omega, part, grid, gs);
    if (e != hipSuccess) return e;
    return launch_gap_tail(s, m, n, v, x, y, ax, aty, part, grid, gs);
}

hipError_t launch_gap_tail(hipStream_t s, int m, int n, Vecs v, const double *x,
                           const double *y, const double *ax, const double *aty, double *part,
                           int grid, GapState *gs) {
    for (int p = kGapHead; p < kGapNewton; ++p) {
        hipLaunchKernelGGL(k_gap_step, dim3(grid), dim3(kThreads), 0, s, m, n, v, x, y, ax, aty,
                           gs, part);
        hipLaunchKernelGGL(k_gap_update, dim3(1), dim3(kThreads), 0, s, part, grid, gs);
    }
    for (int p = 0; p < kGapMaxPass; ++p) {
        hipLaunchKernelGGL(k_gap_pass, dim3(grid), dim3(kThreads), 0, s, m, n, v, x, y, ax, aty,
                           gs, part);
        hipLaunchKernelGGL(k_gap_select, dim3(1), dim3(kThreads), 0, s, part, grid, gs);
    }
    hipLaunchKernelGGL(k_gap_classify, dim3(grid), dim3(kThreads), 0, s, m, n, v, x, y, ax, aty,
                       gs, part);
    hipLaunchKernelGGL(k_gap_solve, dim3(1), dim3(kThreads), 0, s, part, grid, gs);
    return hipGetLastError();
}

}  // namespace pdlp
