// Batched kernels: many independent LPs packed block-diagonally, each with
// its own control block (step size, primal weight, counters, flags), run in
// the same launches.  Row blocks never straddle two instances, so a block
// reads its instance's control block once; partial sums are kept per block
// and reduced per instance (one wave per instance, fixed order).
//
// "Check blocks" index both partitions: cb < nT are blocks of A^T (columns of
// an instance), cb >= nT are blocks of A (rows), so segmented reductions over
// the primal and dual coordinates of an instance share one partial array.
// Every launch walks the host-set lists of running instances and their
// blocks (BatchMaps), so finished instances cost nothing.  The lists are
// interleaved by XCD: list position p goes to workgroup p mod grid, which the
// dispatcher places on XCD p mod 8 (grids are multiples of 8 or cover the
// list), and each instance's blocks sit at positions of one residue, so an
// instance's vectors stay in one XCD's L2.  Padding entries are -1.
#include "pdlp_device.h"

#include <cmath>

namespace pdlp {

__device__ __forceinline__ int cb_inst(const BatchMaps &bm, int cb) {
    return cb < bm.nT ? bm.tblk_inst[cb] : bm.ablk_inst[cb - bm.nT];
}

// ---------------------------------------------------------- step attempt
//
// An attempt is three launches: the dual product, the Algorithm 2 decision
// (kb_decide), and the primal product, which for an instance whose attempt
// was rejected recomputes the primal candidate with the reduced step
// instead.  The primal candidate of the first attempt of a round comes from
// kb_primal.

// Primal candidate x' = proj_X(x - tau (c - A^T y)) on the columns of A^T
// block b, with the block's partial sum of |x' - x|^2.
__device__ __forceinline__ void primal_block(const DCsr &AT, const Vecs &v, const Iter &it,
                                             const Ctrl &c, int b, double *red, double *part) {
    // buffers chosen by select, not by indexing (keeps Iter out of scratch)
    const bool one = c.cur != 0;
    const double tau = c.eta / c.omega;
    const double *x = one ? it.X[1] : it.X[0], *aty = one ? it.ATY[1] : it.ATY[0];
    double *xn = one ? it.X[0] : it.X[1];
    double acc[1] = {0.0};
    for (int j = AT.blk[b] + threadIdx.x; j < AT.blk[b + 1]; j += kThreads) {
        const double xj = x[j];
        const double xv = clampd(xj - tau * (v.c[j] - aty[j]), v.lv[j], v.uv[j]);
        xn[j] = xv;
        const double d = xv - xj;
        acc[0] += d * d;
    }
    block_reduce<1>(acc, red);
    if (threadIdx.x == 0) part[b] = acc[0];
}

__global__ __launch_bounds__(kThreads) void kb_primal(DCsr AT, Vecs v, Iter it, const Ctrl *ctrl,
                                                      BatchMaps bm, double *part) {
    __shared__ double red[kThreads / 64];
    for (int bi = blockIdx.x; bi < bm.nt; bi += gridDim.x) {
        const int b = bm.tlist[bi];
        if (b < 0) continue;  // padding of the per-XCD interleave
        const Ctrl &c = ctrl[bm.tblk_inst[b]];
        if (c.stop || !c.need_primal) continue;
        primal_block(AT, v, it, c, b, red, part);
    }
}

// Algorithm 2 decision of running instance i by one wave: the step norms
// and the interaction term are summed from the per-block partials in a
// fixed order (lane-strided, then the wave butterfly); lane 0 updates the
// control block.
__device__ __forceinline__ void decide_instance(Ctrl *ctrl, const BatchMaps &bm, int i,
                                                const double *pd, const double *pps,
                                                const double *ppf) {
    const int lane = threadIdx.x & 63;
    const Ctrl c0 = ctrl[i];
    const double *pp = c0.need_primal ? pps : ppf;
    double dx2 = 0.0, dy2 = 0.0, cr = 0.0;
    for (int b = bm.tblk_off[i] + lane; b < bm.tblk_off[i + 1]; b += 64) dx2 += pp[b];
    for (int b = bm.ablk_off[i] + lane; b < bm.ablk_off[i + 1]; b += 64) {
        dy2 += pd[2 * b];
        cr += pd[2 * b + 1];
    }
    dx2 = wave_sum(dx2);
    dy2 = wave_sum(dy2);
    cr = wave_sum(cr);
    if (lane != 0) return;
    Ctrl c = c0;
    const double eta = c.eta, omega = c.omega;
    const double num = omega * dx2 + dy2 / omega;
    const double den = 2.0 * fabs(cr);
    c.attempts += 1;
    if (!isfinite(num) || !isfinite(den)) {
        c.numerr = 1;
        c.stop = 1;
        c.run_at = 0;
        ctrl[i] = c;
        return;
    }
    const double eta_bar = den > 0.0 ? num / den : INFINITY;
    const double jj = (double)(c.attempts + 1);
    const double e1 = (1.0 - pow(jj, -c.red_exp)) * eta_bar;
    const double e2 = (1.0 + pow(jj, -c.grow_exp)) * eta;
    const double eta_next = e1 < e2 ? e1 : e2;
    c.last_eta_bar = eta_bar;
    if (c.fixed_step || eta <= eta_bar) {
        if (bm.tape_eta && c.k < bm.tape_K) {
            bm.tape_eta[(size_t)i * bm.tape_K + c.k] = eta;
            bm.tape_omega[(size_t)i * bm.tape_K + c.k] = omega;
        }
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
    ctrl[i] = c;
}

struct BatchDualEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    const Ctrl *ctrl;
    BatchMaps bm;
    Iter it;
    Vecs v;
    double *part;
    const double *gsrc;
    DualRow row;
    __device__ __forceinline__ int count(const DCsr &) const { return bm.na; }
    __device__ __forceinline__ int block(int bi) const { return bm.alist[bi]; }
    __device__ __forceinline__ bool begin(int b) {
        if (b < 0) return false;
        const Ctrl &c = ctrl[bm.ablk_inst[b]];
        if (c.stop) return false;
        // buffers chosen by select, not by indexing (keeps Iter out of scratch)
        const bool one = c.cur != 0;
        gsrc = one ? it.X[0] : it.X[1];
        row = DualRow{one ? it.Y[1] : it.Y[0], one ? it.AX[1] : it.AX[0], v.lc, v.uc,
                      one ? it.AX[0] : it.AX[1], one ? it.Y[0] : it.Y[1], it.sy,
                      c.eta * c.omega, c.eta_avg_y, c.pending_sy};
        return true;
    }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    // no early operand loads: they would cost this kernel an occupancy step
    __device__ __forceinline__ void apply(int r, double s, double (&acc)[2], const Pre &) const {
        row.apply(r, s, acc, row.pre(r));
    }
    __device__ __forceinline__ void end(int b, double (&acc)[2], double *red) {
        block_reduce<2>(acc, red);
        if (threadIdx.x == 0) {
            part[2 * b] = acc[0];
            part[2 * b + 1] = acc[1];
        }
        acc[0] = acc[1] = 0.0;
    }
};

PDLP_STREAM_KERNEL void kb_spmv_dual(DCsr A, Vecs v, Iter it, const Ctrl *ctrl,
                                                         BatchMaps bm, double *part) {
    __shared__ double prod[kStage];
    __shared__ double red[2 * (kThreads / 64)];
    BatchDualEpi epi;
    epi.ctrl = ctrl;
    epi.bm = bm;
    epi.it = it;
    epi.v = v;
    epi.part = part;
    double acc[2] = {0.0, 0.0};
    stream_spmv<2>(A, epi, acc, prod, red);
}

struct BatchPrimalEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    const Ctrl *ctrl;
    BatchMaps bm;
    DCsr AT;
    Iter it;
    Vecs v;
    double *part, *pps;
    double *red;
    const double *gsrc;
    PrimalRow row;
    __device__ __forceinline__ int count(const DCsr &) const { return bm.nt; }
    __device__ __forceinline__ int block(int bi) const { return bm.tlist[bi]; }
    __device__ __forceinline__ bool begin(int b) {
        if (b < 0) return false;
        const Ctrl &c = ctrl[bm.tblk_inst[b]];
        if (!c.run_at) {
            // rejected attempt: the next candidate with the reduced step
            if (!c.stop && c.need_primal) primal_block(AT, v, it, c, b, red, pps);
            return false;
        }
        const bool one = c.cur != 0;
        gsrc = one ? it.Y[1] : it.Y[0];
        row = PrimalRow{one ? it.X[1] : it.X[0], v.c, v.lv, v.uv, one ? it.ATY[1] : it.ATY[0],
                        one ? it.X[0] : it.X[1], it.sx, c.eta_used, c.eta / c.omega, !c.stop};
        return true;
    }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    __device__ __forceinline__ void apply(int j, double s, double (&acc)[1], const Pre &) const {
        row.apply(j, s, acc, row.pre(j));
    }
    __device__ __forceinline__ void end(int b, double (&acc)[1], double *rbuf) {
        if (row.next) {
            block_reduce<1>(acc, rbuf);
            if (threadIdx.x == 0) part[b] = acc[0];
        }
        acc[0] = 0.0;
    }
};

PDLP_STREAM_KERNEL void kb_spmv_primal(DCsr AT, Vecs v, Iter it, const Ctrl *ctrl,
                                       BatchMaps bm, double *part, double *pps) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    BatchPrimalEpi epi;
    epi.ctrl = ctrl;
    epi.bm = bm;
    epi.AT = AT;
    epi.it = it;
    epi.v = v;
    epi.part = part;
    epi.pps = pps;
    epi.red = red;
    double acc[1] = {0.0};
    stream_spmv<1>(AT, epi, acc, prod, red);
}

// Algorithm 2 decision, one wave per listed instance.
__global__ __launch_bounds__(kThreads) void kb_decide(Ctrl *ctrl, BatchMaps bm, const double *pd,
                                                      const double *pps, const double *ppf) {
    const int lane = threadIdx.x & 63;
    const int ii = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (ii >= bm.ni) return;
    const int i = bm.ilist[ii];
    if (ctrl[i].stop) {
        if (lane == 0) ctrl[i].run_at = 0;
        return;
    }
    decide_instance(ctrl, bm, i, pd, pps, ppf);
}

// Dual average owed by the last accepted step, then the current iterate is
// moved to buffer 0 so the checks see every instance in the same buffers.
// The move is a swap: buffer 1 keeps the previous iterate, the other point
// of the difference candidate of infeasibility detection.
__global__ __launch_bounds__(kThreads) void kb_settle(DCsr A, DCsr AT, Iter it, const Ctrl *ctrl,
                                                      BatchMaps bm) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const Ctrl &c = ctrl[cb_inst(bm, cb)];
        if (cb < bm.nT) {
            if (c.cur != 1) continue;
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                const double x0 = it.X[0][j], a0 = it.ATY[0][j];
                it.X[0][j] = it.X[1][j];
                it.ATY[0][j] = it.ATY[1][j];
                it.X[1][j] = x0;
                it.ATY[1][j] = a0;
            }
        } else {
            const int b = cb - bm.nT;
            const int cur = c.cur;
            const bool pend = c.pending_sy && !c.numerr;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads) {
                const double yr = it.Y[cur][r];
                if (pend) it.sy[r] += c.eta_avg_y * yr;
                if (cur == 1) {
                    const double y0 = it.Y[0][r], a0 = it.AX[0][r];
                    it.Y[0][r] = yr;
                    it.AX[0][r] = it.AX[1][r];
                    it.Y[1][r] = y0;
                    it.AX[1][r] = a0;
                }
            }
        }
    }
}

// ------------------------------------------------------------ check kernels

// Elementwise over the coordinates of masked instances.
//   op 0: out = a / s_inst      (average; s = per-instance scalar)
//   op 1: out = a               (copy)
//   op 2: out = s_inst          (fill)
// for the column part (xa -> xo) and the row part (ya -> yo); null pointers skip a part.
__global__ __launch_bounds__(kThreads) void kb_elementwise(DCsr A, DCsr AT, BatchMaps bm,
                                                           const int32_t *mask, int op,
                                                           const double *sv, const double *xa,
                                                           double *xo, const double *ya,
                                                           double *yo) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int inst = cb_inst(bm, cb);
        if (!mask[inst]) continue;
        const double s = sv ? sv[inst] : 0.0;
        const bool col = cb < bm.nT;
        const double *a = col ? xa : ya;
        double *o = col ? xo : yo;
        if (!o) continue;
        const int lo = col ? AT.blk[cb] : A.blk[cb - bm.nT];
        const int hi = col ? AT.blk[cb + 1] : A.blk[cb - bm.nT + 1];
        for (int k = lo + threadIdx.x; k < hi; k += kThreads)
            o[k] = op == 0 ? a[k] / s : (op == 1 ? a[k] : s);
    }
}

struct BatchPlainEpi : NoPrefetch {
    static constexpr bool kSortable = true;
    const int32_t *inst, *mask, *list;
    int nlist;
    const double *gsrc;
    double *out;
    __device__ __forceinline__ int count(const DCsr &) const { return nlist; }
    __device__ __forceinline__ int block(int bi) const { return list[bi]; }
    __device__ __forceinline__ bool begin(int b) const { return b >= 0 && mask[inst[b]] != 0; }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    template <int N>
    __device__ __forceinline__ void apply(int r, double s, double (&)[N], const Pre &) const {
        out[r] = s;
    }
    template <int N>
    __device__ __forceinline__ void end(int, double (&)[N], double *) {}
};

PDLP_STREAM_KERNEL void kb_spmv_plain(DCsr M, const int32_t *blk_inst,
                                                          const int32_t *list, int nlist,
                                                          const int32_t *mask, const double *x,
                                                          double *out) {
    __shared__ double prod[kStage];
    __shared__ double red[kThreads / 64];
    BatchPlainEpi epi{{}, blk_inst, mask, list, nlist, x, out};
    double acc[1] = {0.0};
    stream_spmv<1>(M, epi, acc, prod, red);
}

// Per-instance reduction of per-check-block partials: out[i*nv + k] = sum
// (or max, bit k of maxmask) over the instance's A^T blocks then A blocks.
__global__ __launch_bounds__(kThreads) void kb_inst_reduce(const double *part, int nv,
                                                           unsigned maxmask, BatchMaps bm,
                                                           const int32_t *mask, double *out) {
    const int lane = threadIdx.x & 63;
    const int ii = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (ii >= bm.ni) return;
    const int i = bm.ilist[ii];
    if (mask && !mask[i]) return;
    for (int k = 0; k < nv; ++k) {
        const bool mx = (maxmask >> k) & 1u;
        double a = 0.0;
        for (int b = bm.tblk_off[i] + lane; b < bm.tblk_off[i + 1]; b += 64) {
            const double p = part[(size_t)b * nv + k];
            a = mx ? nan_max(a, p) : a + p;
        }
        for (int b = bm.ablk_off[i] + lane; b < bm.ablk_off[i + 1]; b += 64) {
            const double p = part[(size_t)(bm.nT + b) * nv + k];
            a = mx ? nan_max(a, p) : a + p;
        }
        a = mx ? wave_max(a) : wave_sum(a);
        if (lane == 0) out[(size_t)i * nv + k] = a;
    }
}

// Partials per check block of: 0 ||x - xr||^2 (or |a| max for A^T values
// when xr is null and op = 1), 1 ||y - yr||^2; op 2: ||c||^2 and
// ||Combine(lc, uc)||^2; op 3: max |A^T value| per block (columns).
__global__ __launch_bounds__(kThreads) void kb_norms(DCsr A, DCsr AT, BatchMaps bm,
                                                     const int32_t *mask, int op, const double *xa,
                                                     const double *xb, const double *ya,
                                                     const double *yb, Vecs v, double *part) {
    __shared__ double red[2 * (kThreads / 64)];
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int inst = cb_inst(bm, cb);
        if (mask && !mask[inst]) continue;
        double acc[2] = {0.0, 0.0};
        if (cb < bm.nT) {
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                if (op == 0) {
                    const double d = xa[j] - xb[j];
                    acc[0] += d * d;
                } else if (op == 2) {
                    acc[0] += v.c[j] * v.c[j];
                } else {
                    for (int e = AT.row_ptr[j]; e < AT.row_ptr[j + 1]; ++e)
                        acc[0] = nan_max(acc[0], fabs(AT.val[e]));
                }
            }
        } else {
            const int b = cb - bm.nT;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads) {
                if (op == 0) {
                    const double d = ya[r] - yb[r];
                    acc[1] += d * d;
                } else if (op == 2) {
                    double w = 0.0;
                    const double a = isfinite(v.lc[r]) ? fabs(v.lc[r]) : 0.0;
                    const double u = isfinite(v.uc[r]) ? fabs(v.uc[r]) : 0.0;
                    if (a > w) w = a;
                    if (u > w) w = u;
                    acc[1] += w * w;
                }
            }
        }
        if (op == 3) {
            double t[1] = {acc[0]};
            block_reduce<1, 1u>(t, red);
            if (threadIdx.x == 0) part[2 * cb] = t[0], part[2 * cb + 1] = 0.0;
        } else {
            block_reduce<2>(acc, red);
            if (threadIdx.x == 0) part[2 * cb] = acc[0], part[2 * cb + 1] = acc[1];
        }
    }
}

// Termination evaluation per check block (Section 7, original units), for
// the point chosen per instance by sel (0: buffers *0, 1: buffers *1).
__global__ __launch_bounds__(kThreads) void kb_kkt(DCsr A, DCsr AT, BatchMaps bm,
                                                   const int32_t *mask, const int32_t *sel,
                                                   const double *x0, const double *y0,
                                                   const double *ax0, const double *aty0,
                                                   const double *x1, const double *y1,
                                                   const double *ax1, const double *aty1,
                                                   const double *d1, const double *d2,
                                                   Vecs orig, int mode, double *part,
                                                   double *r_out, double *x_out, double *y_out) {
    __shared__ double red[7 * (kThreads / 64)];
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int inst = cb_inst(bm, cb);
        if (mask && !mask[inst]) continue;
        const int s = sel ? sel[inst] : 0;
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        if (cb >= bm.nT) {
            const double *ys = s ? y1 : y0, *axs = s ? ax1 : ax0;
            const int b = cb - bm.nT;
            for (int i = A.blk[b] + threadIdx.x; i < A.blk[b + 1]; i += kThreads) {
                const double y = d1[i] * ys[i];
                const double ax = axs[i] / d1[i];
                if (y_out) y_out[i] = y;
                const double l = orig.lc[i], u = orig.uc[i];
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
        } else {
            const double *xs = s ? x1 : x0, *atys = s ? aty1 : aty0;
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                const double x = d2[j] * xs[j];
                const double aty = atys[j] / d2[j];
                const double g = orig.c[j] - aty;
                const double l = orig.lv[j], u = orig.uv[j];
                if (x_out) x_out[j] = clampd(x, l, u);   // see k_kkt
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
                const double sc = orig.c[j] != 0.0 ? fabs(orig.c[j]) : 1.0;
                acc[2] = nan_max(acc[2], res);
                acc[3] = nan_max(acc[3], res / sc);
                acc[4] += orig.c[j] * x;
                if (r > 0.0) acc[5] += l * r;
                else if (r < 0.0) acc[5] += u * r;
                if (!isfinite(x) || !isfinite(aty)) acc[6] += 1.0;
            }
        }
        block_reduce<7, 0x0Fu>(acc, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < 7; ++k) part[(size_t)cb * 7 + k] = acc[k];
    }
}

// ------------------------------------------------------------- gap search
//
// The normalized duality gap of Section 3 per instance, by the active-set
// iteration of the single-LP kernels (segment model in pdlp_device.h), with a
// bisection bracket; one GapState per instance.

__device__ __forceinline__ bool coord_range(const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                                            int cb, int &lo, int &hi) {
    if (cb < bm.nT) {
        lo = AT.blk[cb];
        hi = AT.blk[cb + 1];
        return true;
    }
    lo = A.blk[cb - bm.nT];
    hi = A.blk[cb - bm.nT + 1];
    return false;
}

// Infeasibility candidate per check block of masked instances (Section 3,
// "Infeasibility detection"): cand 0 the difference of buffers 0 and 1
// (current and previous iterate), 1 the current iterate, 2 the average
// (xb, yb); x projected onto Xbar into px; for cand 0 y projected onto Y
// into py (the iterate's and the average's y already lie in Y).
__global__ __launch_bounds__(kThreads) void kb_cert_point(DCsr A, DCsr AT, BatchMaps bm,
                                                          const int32_t *mask, int cand, Iter it,
                                                          const double *xb, Vecs orig,
                                                          double *px, double *py) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        if (!mask[cb_inst(bm, cb)]) continue;
        if (cb < bm.nT) {
            if (!px) continue;
            const double *xa = cand == 2 ? xb : it.X[0];
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                const double x = cand == 0 ? xa[j] - it.X[1][j] : xa[j];
                px[j] = proj_xbar(x, orig.lv[j], orig.uv[j]);
            }
        } else if (cand == 0) {
            const int b = cb - bm.nT;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads)
                py[r] = proj_ycone(it.Y[0][r] - it.Y[1][r], orig.lc[r], orig.uc[r]);
        }
    }
}

// Appendix D test values per check block (cert_row / cert_col).
__global__ __launch_bounds__(kThreads) void kb_cert(DCsr A, DCsr AT, BatchMaps bm,
                                                    const int32_t *mask, const double *px,
                                                    const double *py, const double *pax,
                                                    const double *paty, const double *d1,
                                                    const double *d2, Vecs orig, double *part) {
    __shared__ double red[kCertVals * (kThreads / 64)];
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        if (!mask[cb_inst(bm, cb)]) continue;
        double acc[kCertVals] = {0, 0, 0, 0, 0};
        if (cb < bm.nT) {
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads)
                cert_col(px ? px[j] : 0.0, paty[j], d2[j], orig.c[j], orig.lv[j], orig.uv[j],
                         acc);
        } else {
            const int b = cb - bm.nT;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads)
                cert_row(py[r], pax ? pax[r] : 0.0, d1[r], orig.lc[r], orig.uc[r], acc);
        }
        block_reduce<kCertVals, kCertMax>(acc, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < kCertVals; ++k) part[(size_t)cb * kCertVals + k] = acc[k];
    }
}

// Unscaled certificate outputs of masked instances: x = D2 px, y = D1 py,
// r = proj_R(-(A^T y)).
__global__ __launch_bounds__(kThreads) void kb_cert_out(DCsr A, DCsr AT, BatchMaps bm,
                                                        const int32_t *mask, const double *px,
                                                        const double *py, const double *paty,
                                                        const double *d1, const double *d2,
                                                        Vecs orig, double *x_out, double *y_out,
                                                        double *r_out) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        if (!mask[cb_inst(bm, cb)]) continue;
        if (cb < bm.nT) {
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                x_out[j] = px ? d2[j] * px[j] : 0.0;
                r_out[j] = proj_rcone(-(paty[j] / d2[j]), orig.lv[j], orig.uv[j]);
            }
        } else {
            const int b = cb - bm.nT;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads)
                y_out[r] = d1[r] * py[r];
        }
    }
}

__global__ __launch_bounds__(kThreads) void kb_gap_setup(DCsr A, DCsr AT, BatchMaps bm,
                                                         const int32_t *mask, Vecs v,
                                                         const double *x, const double *y,
                                                         const double *ax, const double *aty,
                                                         const double *xr, const double *yr,
                                                         const double *omega, double *part) {
    __shared__ double red[4 * (kThreads / 64)];
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int inst = cb_inst(bm, cb);
        if (!mask[inst]) continue;
        const double w = omega[inst];
        int lo, hi;
        const bool col = coord_range(A, AT, bm, cb, lo, hi);
        double acc[4] = {0, 0, 0, 0};
        for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
            Seg q;
            double zi;
            if (col) {
                zi = x[k];
                const double d = zi - xr[k];
                acc[0] += w * d * d;
                q = seg_x(zi, v.c[k] - aty[k], v.lv[k], v.uv[k], w);
            } else {
                zi = y[k];
                const double d = zi - yr[k];
                acc[0] += d * d / w;
                const bool af = isfinite(v.lc[k]), bf = isfinite(v.uc[k]);
                q = seg_y(zi, af, af ? v.lc[k] - ax[k] : 0.0, bf, bf ? v.uc[k] - ax[k] : 0.0, w);
            }
            if (q.b1 > 0.0) acc[1] += q.a1;
            acc[2] += isfinite(q.b2) ? INFINITY : (isfinite(q.b1) ? q.c : (q.a1 > 0.0 ? INFINITY : 0.0));
            if (!isfinite(zi) || !isfinite(q.a1)) acc[3] += 1.0;
        }
        block_reduce<4>(acc, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; ++k) part[(size_t)cb * 4 + k] = acc[k];
    }
}

__global__ __launch_bounds__(kThreads) void kb_gap_init(const double *part, BatchMaps bm,
                                                        const int32_t *mask, const double *omega,
                                                        GapState *gs) {
    const int lane = threadIdx.x & 63;
    const int ii = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (ii >= bm.ni) return;
    const int i = bm.ilist[ii];
    if (!mask[i]) return;
    double v[4];
    for (int k = 0; k < 4; ++k) {
        double a = 0.0;
        for (int b = bm.tblk_off[i] + lane; b < bm.tblk_off[i + 1]; b += 64) a += part[(size_t)b * 4 + k];
        for (int b = bm.ablk_off[i] + lane; b < bm.ablk_off[i + 1]; b += 64)
            a += part[(size_t)(bm.nT + b) * 4 + k];
        v[k] = wave_sum(a);
    }
    if (lane != 0) return;
    GapState s;
    s.r2 = v[0];
    s.r = sqrt(v[0]);
    s.omega = omega[i];
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
        s.done = 3;
        s.mu = NAN;
    } else if (!(s.r2 > 0.0) || !(s.A0 > 0.0)) {
        s.done = 3;
        s.mu = 0.0;
    } else if (s.Dinf <= s.r2) {
        s.pathend = 1;  // evaluated by one step at the end of the path
    }
    s.newton = s.done ? 0 : 1;
    s.s_prev = 2.2250738585072014e-308;
    s.D_prev = 0.0;
    s.s_cur = s.done ? 0.0 : (s.pathend ? 1e300 : s.r / sqrt(s.A0));
    s.nsteps = 0;
    s.exact = 0;
    gs[i] = s;
}

__global__ __launch_bounds__(kThreads) void kb_gap_step(DCsr A, DCsr AT, BatchMaps bm,
                                                        const int32_t *mask, Vecs v,
                                                        const double *x, const double *y,
                                                        const double *ax, const double *aty,
                                                        const GapState *gs, double *part) {
    __shared__ double red[6 * (kThreads / 64)];
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int inst = cb_inst(bm, cb);
        if (!mask[inst]) continue;
        const GapState &g = gs[inst];
        if (g.done || !g.newton) continue;
        const double w = g.omega, sc = g.s_cur, sp = g.s_prev, sc2 = sc * sc;
        int lo, hi;
        const bool col = coord_range(A, AT, bm, cb, lo, hi);
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
            Seg q;
            if (col) {
                q = seg_x(x[k], v.c[k] - aty[k], v.lv[k], v.uv[k], w);
            } else {
                const bool af = isfinite(v.lc[k]), bf = isfinite(v.uc[k]);
                q = seg_y(y[k], af, af ? v.lc[k] - ax[k] : 0.0, bf, bf ? v.uc[k] - ax[k] : 0.0, w);
            }
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
        block_reduce<6>(acc, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < 6; ++k) part[(size_t)cb * 6 + k] = acc[k];
    }
}

__global__ __launch_bounds__(kThreads) void kb_gap_update(const double *part, BatchMaps bm,
                                                          const int32_t *mask, GapState *gs,
                                                          int last) {
    const int lane = threadIdx.x & 63;
    const int ii = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (ii >= bm.ni) return;
    const int i = bm.ilist[ii];
    if (!mask[i]) return;
    if (gs[i].done || !gs[i].newton) return;
    double v[6];
    for (int k = 0; k < 6; ++k) {
        double a = 0.0;
        for (int b = bm.tblk_off[i] + lane; b < bm.tblk_off[i + 1]; b += 64) a += part[(size_t)b * 6 + k];
        for (int b = bm.ablk_off[i] + lane; b < bm.ablk_off[i + 1]; b += 64)
            a += part[(size_t)(bm.nT + b) * 6 + k];
        v[k] = wave_sum(a);
    }
    if (lane != 0) return;
    GapState s = gs[i];
    const double Dk = v[0], A_ = v[1], B_ = v[2], F1 = v[3], F0 = v[4], cnt = v[5];
    const double sc = s.s_cur;
    s.nsteps += 1;
    if (s.pathend) {
        // every coordinate ends on a constant piece: f = F0
        s.f = F0;
        s.mu = F0 / s.r;
        s.done = 3;
        s.newton = 0;
        s.exact = 1;
        gs[i] = s;
        return;
    }
    if (Dk < s.r2) s.lo = fmax(s.lo, sc);
    else s.hi = fmin(s.hi, sc);
    double st = A_ > 0.0 ? sqrt((s.r2 - B_) / A_) : NAN;
    const double a = fmin(s.s_prev, sc), b = fmax(s.s_prev, sc);
    const bool at_root = fabs(st - sc) <= 1e-13 * sc;
    const bool exact = at_root || (cnt == 0.0 && st >= a * (1.0 - 1e-12) && st <= b * (1.0 + 1e-12));
    if (exact || last || !(s.hi > s.lo)) {
        // exact, or the step budget is spent: the root of the segment at
        // s_cur, kept inside the bracket
        if (exact) st = at_root ? sc : fmin(fmax(st, a), b);
        else if (!(st >= s.lo && st <= s.hi)) st = isfinite(s.hi) ? 0.5 * (s.lo + s.hi) : s.lo;
        s.exact = exact ? 1 : 0;
        s.s_star = st;
        s.Acoef = A_;
        s.Bcoef = B_;
        s.f = F1 * st + F0;
        s.mu = s.f / s.r;
        s.done = 3;
        s.newton = 0;
        gs[i] = s;
        return;
    }
    double nxt = A_ > 0.0 ? st : INFINITY;
    if (!(nxt > s.lo && nxt < s.hi) || nxt == sc)
        nxt = isfinite(s.hi) ? 0.5 * (s.lo + s.hi) : 2.0 * fmax(s.lo, sc);
    s.s_prev = sc;
    s.D_prev = Dk;
    s.s_cur = nxt;
    gs[i] = s;
}

// Checkpoint copy of a recorded run (see launch_b_checkpoint).
__global__ __launch_bounds__(kThreads) void kb_checkpoint(DCsr A, DCsr AT, BatchMaps bm,
                                                          const int32_t *slot, const double *x,
                                                          const double *y, const double *sx,
                                                          const double *sy, double *ck,
                                                          int64_t N, int64_t M) {
    for (int ci = blockIdx.x; ci < bm.nc; ci += gridDim.x) {
        const int cb = bm.clist[ci];
        if (cb < 0) continue;
        const int sl = slot[cb_inst(bm, cb)];
        if (sl < 0) continue;
        double *base = ck + (size_t)sl * 2 * (size_t)(N + M);
        if (cb < bm.nT) {
            for (int j = AT.blk[cb] + threadIdx.x; j < AT.blk[cb + 1]; j += kThreads) {
                base[j] = x[j];
                base[N + M + j] = sx[j];
            }
        } else {
            const int b = cb - bm.nT;
            for (int r = A.blk[b] + threadIdx.x; r < A.blk[b + 1]; r += kThreads) {
                base[N + r] = y[r];
                base[2 * N + M + r] = sy[r];
            }
        }
    }
}

// --------------------------------------------------------------- launchers

static inline int wave_grid(int ni) {
    const int g = (ni + kThreads / 64 - 1) / (kThreads / 64);
    return g > 0 ? g : 1;
}
static inline int list_grid(int n, int cap) { return n < cap ? (n > 0 ? n : 1) : cap; }
constexpr int kBatchGridCap = 4096;   // elementwise / check kernels
constexpr int kBatchSpmvCap = 2048;   // persistent CSR stream kernels (8 per CU)

hipError_t launch_b_primal(hipStream_t s, const DCsr &AT, Vecs v, Iter it, const Ctrl *ctrl,
                           const BatchMaps &bm, double *pps) {
    if (bm.nt > 0)
        hipLaunchKernelGGL(kb_primal, dim3(list_grid(bm.nt, kBatchGridCap)), dim3(kThreads), 0, s,
                           AT, v, it, ctrl, bm, pps);
    return hipGetLastError();
}

hipError_t launch_b_attempt(hipStream_t s, const DCsr &A, const DCsr &AT, Vecs v, Iter it,
                            Ctrl *ctrl, const BatchMaps &bm, double *pd, double *pps,
                            double *ppf) {
    if (bm.ni == 0) return hipSuccess;
    if (bm.na > 0)
        hipLaunchKernelGGL(kb_spmv_dual, dim3(list_grid(bm.na, kBatchSpmvCap)), dim3(kThreads), 0,
                           s, A, v, it, ctrl, bm, pd);
    hipLaunchKernelGGL(kb_decide, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, ctrl, bm, pd, pps,
                       ppf);
    if (bm.nt > 0)
        hipLaunchKernelGGL(kb_spmv_primal, dim3(list_grid(bm.nt, kBatchSpmvCap)), dim3(kThreads), 0,
                           s, AT, v, it, ctrl, bm, ppf, pps);
    return hipGetLastError();
}

hipError_t launch_b_settle(hipStream_t s, const DCsr &A, const DCsr &AT, Iter it, Ctrl *ctrl,
                           const BatchMaps &bm) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(kb_settle, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0, s,
                           A, AT, it, ctrl, bm);
    return hipGetLastError();
}

hipError_t launch_b_elementwise(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                                const int32_t *mask, int op, const double *sv, const double *xa,
                                double *xo, const double *ya, double *yo) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(kb_elementwise, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0,
                           s, A, AT, bm, mask, op, sv, xa, xo, ya, yo);
    return hipGetLastError();
}

hipError_t launch_b_spmv_plain(hipStream_t s, const DCsr &M, const int32_t *blk_inst,
                               const int32_t *list, int nlist, const int32_t *mask,
                               const double *x, double *out) {
    if (nlist > 0)
        hipLaunchKernelGGL(kb_spmv_plain, dim3(list_grid(nlist, kBatchSpmvCap)), dim3(kThreads), 0,
                           s, M, blk_inst, list, nlist, mask, x, out);
    return hipGetLastError();
}

hipError_t launch_b_norms(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                          const int32_t *mask, int op, const double *xa, const double *xb,
                          const double *ya, const double *yb, Vecs v, double *part,
                          unsigned maxmask, double *out) {
    if (bm.ni == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_norms, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0, s, A,
                       AT, bm, mask, op, xa, xb, ya, yb, v, part);
    hipLaunchKernelGGL(kb_inst_reduce, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, part, 2,
                       maxmask, bm, mask, out);
    return hipGetLastError();
}

hipError_t launch_b_kkt(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                        const int32_t *mask, const int32_t *sel, const double *const *p0,
                        const double *const *p1, const double *d1, const double *d2, Vecs orig,
                        int mode, double *part, double *out, double *r_out, double *x_out,
                        double *y_out) {
    if (bm.ni == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_kkt, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0, s, A, AT,
                       bm, mask, sel, p0[0], p0[1], p0[2], p0[3], p1[0], p1[1], p1[2], p1[3], d1,
                       d2, orig, mode, part, r_out, x_out, y_out);
    hipLaunchKernelGGL(kb_inst_reduce, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, part, 7, 0x0Fu,
                       bm, mask, out);
    return hipGetLastError();
}

hipError_t launch_b_cert_point(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, int cand, Iter it, const double *xb,
                              Vecs orig, double *px, double *py) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(kb_cert_point, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0,
                           s, A, AT, bm, mask, cand, it, xb, orig, px, py);
    return hipGetLastError();
}

hipError_t launch_b_cert(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                         const int32_t *mask, const double *px, const double *py,
                         const double *pax, const double *paty, const double *d1,
                         const double *d2, Vecs orig, double *part, double *out) {
    if (bm.ni == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_cert, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0, s, A,
                       AT, bm, mask, px, py, pax, paty, d1, d2, orig, part);
    hipLaunchKernelGGL(kb_inst_reduce, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, part,
                       kCertVals, kCertMax, bm, mask, out);
    return hipGetLastError();
}

hipError_t launch_b_cert_out(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                             const int32_t *mask, const double *px, const double *py,
                             const double *paty, const double *d1, const double *d2, Vecs orig,
                             double *x_out, double *y_out, double *r_out) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(kb_cert_out, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0,
                           s, A, AT, bm, mask, px, py, paty, d1, d2, orig, x_out, y_out, r_out);
    return hipGetLastError();
}

hipError_t launch_b_gap_begin(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, Vecs v, const double *x, const double *y,
                              const double *ax, const double *aty, const double *xr,
                              const double *yr, const double *omega, double *part, GapState *gs) {
    if (bm.ni == 0) return hipSuccess;
    hipLaunchKernelGGL(kb_gap_setup, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0, s,
                       A, AT, bm, mask, v, x, y, ax, aty, xr, yr, omega, part);
    hipLaunchKernelGGL(kb_gap_init, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, part, bm, mask,
                       omega, gs);
    return hipGetLastError();
}

hipError_t launch_b_gap_steps(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, Vecs v, const double *x, const double *y,
                              const double *ax, const double *aty, double *part, GapState *gs,
                              int first, int count, int total) {
    if (bm.ni == 0) return hipSuccess;
    for (int k = first; k < first + count && k < total; ++k) {
        hipLaunchKernelGGL(kb_gap_step, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0,
                           s, A, AT, bm, mask, v, x, y, ax, aty, gs, part);
        hipLaunchKernelGGL(kb_gap_update, dim3(wave_grid(bm.ni)), dim3(kThreads), 0, s, part, bm,
                           mask, gs, k == total - 1 ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t launch_b_checkpoint(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                               const int32_t *slot, const double *x, const double *y,
                               const double *sx, const double *sy, double *ck, int64_t N,
                               int64_t M) {
    if (bm.nc > 0)
        hipLaunchKernelGGL(kb_checkpoint, dim3(list_grid(bm.nc, kBatchGridCap)), dim3(kThreads), 0,
                           s, A, AT, bm, slot, x, y, sx, sy, ck, N, M);
    return hipGetLastError();
}

}  // namespace pdlp
