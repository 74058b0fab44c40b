// Device helpers shared by the single-LP and the batched kernels.
#pragma once

#include "pdlp_internal.h"

namespace pdlp {

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double nan_max(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return b > a ? b : a;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce NV per-thread values over the workgroup; bit i of MAXMASK selects a
// max instead of a sum for value i.  The result is valid in thread 0.
// lds must hold (kThreads/64)*NV doubles.
template <int NV, unsigned MAXMASK = 0u>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = ((MAXMASK >> i) & 1u) ? wave_max(v[i]) : wave_sum(v[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[wid * NV + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double a = lds[i];
            for (int w = 1; w < kThreads / 64; ++w)
                a = ((MAXMASK >> i) & 1u) ? nan_max(a, lds[w * NV + i]) : a + lds[w * NV + i];
            v[i] = a;
        }
    }
    __syncthreads();
}

template <int NV, unsigned MAXMASK = 0u>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *lds, double *part) {
    block_reduce<NV, MAXMASK>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) part[blockIdx.x * NV + i] = v[i];
    }
}

__device__ __forceinline__ int32_t wave_incl_scan_i32(int32_t v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum over the kThreads threads of a workgroup (in thread
// order); returns the block total through *total.
__device__ __forceinline__ int32_t block_excl_scan_i32(int32_t v, int32_t *lds, int32_t *total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t inc = wave_incl_scan_i32(v);
    __syncthreads();
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int q = 0; q < kWaveRows; ++q) {
        if (q < w) before += lds[q];
        all += lds[q];
    }
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// ------------------------------------------ infeasibility certificates
//
// Appendix D tests, evaluated in original units from scaled candidates
// (x = D2 x~, y = D1 y~, A x = (A~ x~)/D1, A^T y = (A~^T y~)/D2).  Projections
// depend only on signs and on which bounds are finite, so they commute with
// the positive diagonal scalings.  Values accumulated per coordinate:
//   0 primal-test objective lc^T y+ - uc^T y- + lv^T r+ - uv^T r-   (sum)
//   1 primal-test residual max_j |A^T y + r|_j / w_j                (max)
//   2 dual-test objective c^T x                                     (sum)
//   3 dual-test residual max_i |A x + s|_i / q_i                    (max)
//   4 count of non-finite inputs                                     (sum)
// with r = proj_R(-A^T y), s = proj_Sbar(-A x), w_j = |c_j| (1 if c_j = 0)
// and q_i the weight of the relative primal residual.
// x onto Xbar: {0} boxed, R+ lower bound only, R- upper bound only, R free.
__device__ __forceinline__ double proj_xbar(double x, double l, double u) {
    const bool lf = isfinite(l), uf = isfinite(u);
    return ((lf && uf) || (lf && x < 0.0) || (uf && x > 0.0)) ? 0.0 : x;
}

// y onto Y (Section 2): {0} free row, R- upper bound only, R+ lower bound only.
__device__ __forceinline__ double proj_ycone(double y, double l, double u) {
    const bool lf = isfinite(l), uf = isfinite(u);
    return ((!lf && !uf) || (!lf && y > 0.0) || (!uf && y < 0.0)) ? 0.0 : y;
}

// g onto R_j: {0} free variable, R- upper bound only, R+ lower bound only.
__device__ __forceinline__ double proj_rcone(double g, double l, double u) {
    const bool lf = isfinite(l), uf = isfinite(u);
    if (!lf && !uf) return 0.0;
    if (!lf) return g < 0.0 ? g : 0.0;
    if (!uf) return g > 0.0 ? g : 0.0;
    return g;
}

__device__ __forceinline__ double row_weight(double l, double u) {
    const bool lb = isfinite(l) && l != 0.0, ub = isfinite(u) && u != 0.0;
    if (lb && !ub) return fabs(l);
    if (!lb && ub) return fabs(u);
    if (lb && ub) return fmax(fabs(l), fabs(u));
    return 1.0;
}

// Row i of a projected scaled candidate: y~ (py) and A~ x~ (pax).
__device__ __forceinline__ void cert_row(double py, double pax, double d1, double l, double u,
                                         double (&acc)[kCertVals]) {
    const double y = d1 * py;
    if (y > 0.0) acc[0] += l * y;
    else if (y < 0.0) acc[0] += u * y;
    const double ax = pax / d1;
    const bool lf = isfinite(l), uf = isfinite(u);
    const double g = -ax;
    double sv;
    if (lf && uf) sv = 0.0;
    else if (uf) sv = g > 0.0 ? g : 0.0;     // Sbar_i = R+
    else if (lf) sv = g < 0.0 ? g : 0.0;     // Sbar_i = R-
    else sv = g;
    acc[3] = nan_max(acc[3], fabs(ax + sv) / row_weight(l, u));
    if (!isfinite(y) || !isfinite(ax)) acc[4] += 1.0;
}

// Column j: x~ (px) and A~^T y~ (paty).
__device__ __forceinline__ void cert_col(double px, double paty, double d2, double c, double l,
                                         double u, double (&acc)[kCertVals]) {
    const double aty = paty / d2;
    const double r = proj_rcone(-aty, l, u);
    if (r > 0.0) acc[0] += l * r;
    else if (r < 0.0) acc[0] += u * r;
    const double w = c != 0.0 ? fabs(c) : 1.0;
    acc[1] = nan_max(acc[1], fabs(aty + r) / w);
    const double x = d2 * px;
    acc[2] += c * x;
    if (!isfinite(x) || !isfinite(aty)) acc[4] += 1.0;
}

// Dual update in case form (Section 2): with yhat = y - sigma A(2x' - x),
// y' = yhat + sigma uc if yhat < -sigma uc; yhat + sigma lc if yhat > -sigma lc; else 0.
__device__ __forceinline__ double dual_case(double yhat, double sigma, double lc, double uc) {
    if (isfinite(uc)) {
        const double su = sigma * uc;
        if (yhat < -su) return yhat + su;
    }
    if (isfinite(lc)) {
        const double sl = sigma * lc;
        if (yhat > -sl) return yhat + sl;
    }
    return 0.0;
}

// [hot-path device begin]
// Matrix streams (values, column indices) are read once per product: load
// them with the non-temporal hint so they do not displace the gathered
// vector from the caches.
#ifndef PDLP_NT_STREAM
#define PDLP_NT_STREAM 1
#endif
template <class T>
__device__ __forceinline__ T stream_load(const T *p) {
#if PDLP_NT_STREAM
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// ------------------------------------------------------- CSR stream SpMV
//
// Workgroup-per-row-block CSR product.  A short-row block stages its
// products in LDS with fully coalesced loads of val/col (one gather of x per
// nonzero), then one lane per row sums its slice in stored order -- the
// same order as a sequential row loop.  Medium rows get one wave each
// (lane-strided partial sums, butterfly reduction); a long row is reduced
// across the workgroup.  The grid is persistent: workgroup g handles blocks
// g, g + grid, ...

// Hooks of the epilogue: count(A) blocks are visited, the bi-th being
// block(bi) (all blocks in order for one LP, a list of the blocks of running
// instances in a batch); begin(b) says whether block b runs (and may load
// per-block parameters), src() is the gathered vector, prefetch(r) loads the
// row work's operands (type Pre) and apply(r, s, acc, pre) does the row work
// with the row's product s; end(b, acc, red) is called after the block
// (per-block partial sums in the batched solver).
template <int NACC, class Epi>
__device__ __forceinline__ void stream_block(const DCsr &A, Epi &epi, int b, double (&acc)[NACC],
                                             double *prod, double *red) {
    constexpr int kPer = kStage / kThreads;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    {
        const double *__restrict__ x = epi.src();
        const int r0 = A.blk[b], r1 = A.blk[b + 1];
        const int e0 = A.row_ptr[r0], e1 = A.row_ptr[r1];
        const int len = e1 - e0;
        const int len0 = A.row_ptr[r0 + 1] - e0;
        if (len0 > A.med_row && len0 <= kWaveMax) {
            // wave block: row r0 + wid
            const int r = r0 + wid;
            if (r < r1) {
                const int a = A.row_ptr[r], z = A.row_ptr[r + 1];
                double s = 0.0;
                for (int e = a + lane; e < z; e += 64)
                    s += stream_load(A.val + e) * x[stream_load(A.col + e)];
                s = wave_sum(s);
                if (lane == 0) epi.apply(r, s, acc, epi.prefetch(r));
            }
        } else if (len <= kStage && len0 <= A.med_row) {
            // the first row of each lane: its slice bounds and epilogue operands
            // are loaded before the matrix stream so they arrive with it
            const int rr = r0 + threadIdx.x;
            int ra = 0, rz = 0;
            typename Epi::Pre pre{};
            if (rr < r1) {
                ra = A.row_ptr[rr] - e0;
                rz = A.row_ptr[rr + 1] - e0;
                pre = epi.prefetch(rr);
            }
            int ci[kPer];
            double vv[kPer];
            bool sorted = false;
            if constexpr (Epi::kSortable) sorted = A.sblk != nullptr && A.sblk[b] != 0;
            if (sorted) {
                // column-sorted copy: neighbouring lanes gather neighbouring
                // words; each product goes to its entry's slot in the block
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int q = i * kThreads + threadIdx.x;
                    if (q < len) {
                        ci[i] = stream_load(A.scol + e0 + q);
                        vv[i] = stream_load(A.sval + e0 + q);
                    } else {
                        ci[i] = 0;
                        vv[i] = 0.0;
                    }
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int q = i * kThreads + threadIdx.x;
                    if (q < len) prod[stream_load(A.slot + e0 + q)] = vv[i] * x[ci[i]];
                }
            } else {
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int q = i * kThreads + threadIdx.x;
                    if (q < len) {
                        ci[i] = stream_load(A.col + e0 + q);
                        vv[i] = stream_load(A.val + e0 + q);
                    } else {
                        ci[i] = 0;
                        vv[i] = 0.0;
                    }
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int q = i * kThreads + threadIdx.x;
                    if (q < len) prod[q] = vv[i] * x[ci[i]];
                }
            }
            __syncthreads();
            if (rr < r1) {
                double s = 0.0;
                for (int q = ra; q < rz; ++q) s += prod[q];
                epi.apply(rr, s, acc, pre);
            }
            for (int r = rr + kThreads; r < r1; r += kThreads) {
                const int a = A.row_ptr[r] - e0, z = A.row_ptr[r + 1] - e0;
                double s = 0.0;
                for (int q = a; q < z; ++q) s += prod[q];
                epi.apply(r, s, acc, epi.prefetch(r));
            }
            __syncthreads();
        } else {
            double s = 0.0;
            for (int e = e0 + threadIdx.x; e < e1; e += kThreads)
                s += stream_load(A.val + e) * x[stream_load(A.col + e)];
            double t[1] = {s};
            block_reduce<1>(t, red);
            if (threadIdx.x == 0) epi.apply(r0, t[0], acc, epi.prefetch(r0));
        }
    }
}

template <int NACC, class Epi>
__device__ __forceinline__ void stream_spmv(const DCsr &A, Epi &epi, double (&acc)[NACC],
                                            double *prod, double *red) {
    const int nb = epi.count(A);
    for (int bi = blockIdx.x; bi < nb; bi += gridDim.x) {
        const int b = epi.block(bi);
        if (!epi.begin(b)) continue;
        stream_block<NACC>(A, epi, b, acc, prod, red);
        epi.end(b, acc, red);
    }
}

// Phase 2 of the two-phase product (SegCsr): the pair sums of each row block
// of sg.P are read from their 2S runs of Q and staged in LDS at their slots;
// then one lane per row sums the row's pairs in slot order and runs the row
// work, as in the short-row path of stream_spmv.  Every block of sg.P fits
// the stage (at most kStage pairs).  lds_i holds 2 * kThreads + kWaveRows ints.
template <int NACC, class Epi>
__device__ __forceinline__ void staged_spmv(const SegCsr &sg, Epi &epi, double (&acc)[NACC],
                                            double *prod, int32_t *lds_i) {
    const DCsr &M = sg.P;
    const int S = 2 * sg.S;  // runs per block
    int32_t *run_lo = lds_i, *run_at = lds_i + kThreads;
    const int nb = epi.count(M);
    for (int bi = blockIdx.x; bi < nb; bi += gridDim.x) {
        const int b = epi.block(bi);
        if (!epi.begin(b)) continue;
        const int r0 = M.blk[b], r1 = M.blk[b + 1];
        const int p0 = M.row_ptr[r0];
        const int len = M.row_ptr[r1] - p0;
        const int rr = r0 + threadIdx.x;
        int ra = 0, rz = 0;
        typename Epi::Pre pre{};
        if (rr < r1) {
            ra = M.row_ptr[rr] - p0;
            rz = M.row_ptr[rr + 1] - p0;
            pre = epi.prefetch(rr);
        }
        // runs of the block: start in Q and position in the block's pair list
        int32_t cnt = 0, lo = 0;
        if ((int)threadIdx.x < S) {
            lo = sg.qoff[(int64_t)b * S + threadIdx.x];
            cnt = sg.qoff[(int64_t)(b + 1) * S + threadIdx.x] - lo;
        }
        int32_t total = 0;
        const int32_t at = block_excl_scan_i32(cnt, lds_i + 2 * kThreads, &total);
        if ((int)threadIdx.x < S) {
            run_lo[threadIdx.x] = lo;
            run_at[threadIdx.x] = at;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < len; q += kThreads) {
            // the last run that starts at or before q holds it
            int a = 0, z = S - 1;
            while (a < z) {
                const int mid = (a + z + 1) >> 1;
                if (run_at[mid] <= q) a = mid;
                else z = mid - 1;
            }
            const int64_t qi = (int64_t)run_lo[a] + (q - run_at[a]);
            // plain loads: the runs are short and unaligned, so neighbouring
            // runs (other lanes, the next block on this CU) share cache lines
            // that the non-temporal hint would keep out of L1
            prod[sg.slot[qi]] = sg.Q[qi];
        }
        __syncthreads();
        if (rr < r1) {
            double s = 0.0;
            for (int q = ra; q < rz; ++q) s += prod[q];
            epi.apply(rr, s, acc, pre);
        }
        for (int r = rr + kThreads; r < r1; r += kThreads) {
            const int a = M.row_ptr[r] - p0, z = M.row_ptr[r + 1] - p0;
            double s = 0.0;
            for (int q = a; q < z; ++q) s += prod[q];
            epi.apply(r, s, acc, epi.prefetch(r));
        }
        __syncthreads();
        epi.end(b, acc, nullptr);
    }
}


// Row work fused after A x': the dual step (case form), the lazy dual
// average, and the partials acc[0] = ||y'-y||^2, acc[1] = (y'-y)^T (A x' - A x).
struct DualRow {
    const double *y, *ax, *lc, *uc;
    double *ax_new, *y_new, *sy;
    double sigma, eta_avg;
    int pend;
    struct Pre {
        double y, ax, lc, uc, sy;
    };
    __device__ __forceinline__ Pre pre(int r) const {
        Pre p;
        p.y = y[r];
        p.ax = ax[r];
        p.lc = lc[r];
        p.uc = uc[r];
        p.sy = pend ? sy[r] : 0.0;
        return p;
    }
    __device__ __forceinline__ void apply(int r, double s, double (&acc)[2], const Pre &p) const {
        ax_new[r] = s;
        const double yr = p.y;
        if (pend) sy[r] = p.sy + eta_avg * yr;
        const double axr = p.ax;
        const double yhat = yr - sigma * (2.0 * s - axr);
        const double yn = dual_case(yhat, sigma, p.lc, p.uc);
        y_new[r] = yn;
        const double dy = yn - yr;
        acc[0] += dy * dy;
        acc[1] += dy * (s - axr);
    }
};

// Column work fused after A^T y': the primal average and (next != 0) the
// next candidate x' = proj_X(x - tau (c - A^T y')), acc[0] = ||x'-x||^2.
struct PrimalRow {
    const double *x, *c, *lv, *uv;
    double *aty, *x_new, *sx;
    double eta_used, tau;
    int next;
    struct Pre {
        double x, c, lv, uv, sx;
    };
    __device__ __forceinline__ Pre pre(int j) const {
        Pre p;
        p.x = x[j];
        p.sx = sx[j];
        if (next) {
            p.c = c[j];
            p.lv = lv[j];
            p.uv = uv[j];
        } else {
            p.c = p.lv = p.uv = 0.0;
        }
        return p;
    }
    __device__ __forceinline__ void apply(int j, double s, double (&acc)[1], const Pre &p) const {
        aty[j] = s;
        const double xj = p.x;
        sx[j] = p.sx + eta_used * xj;
        if (next) {
            const double g = p.c - s;
            const double xn = clampd(xj - tau * g, p.lv, p.uv);
            x_new[j] = xn;
            const double d = xn - xj;
            acc[0] += d * d;
        }
    }
};

// Epilogues without operands to prefetch.
struct NoPrefetch {
    struct Pre {};
    __device__ __forceinline__ Pre prefetch(int) const { return {}; }
    static constexpr bool kSortable = false;  // reads DCsr's column-sorted copy when present
};

// Epilogue base for a single LP: one gathered vector, partial sums
// accumulate per thread across blocks.  Blocks are dealt to the XCDs in
// chunks of kXcdChunk consecutive blocks: workgroup w of a launch runs on
// XCD w mod 8 and, with the persistent grid a multiple of 8, visits loop
// indices bi = w (mod 8), so each XCD works through whole chunks of
// neighbouring rows (which, after the library's relabelling, share cache
// lines of the gathered vector) while the chunks still spread the heavy
// first rows over all XCDs.  Every block is visited exactly once for any
// grid (indices past the blocks skip).
#ifndef PDLP_XCD_CHUNK
#define PDLP_XCD_CHUNK 64
#endif
constexpr int kXcdChunk = PDLP_XCD_CHUNK;
struct SingleEpi : NoPrefetch {
    const double *gsrc;
    int nblk = 0;
    __device__ __forceinline__ int count(const DCsr &A) {
        nblk = A.nblk;
        constexpr int span = 8 * kXcdChunk;
        return (A.nblk + span - 1) / span * span;
    }
    __device__ __forceinline__ int block(int bi) const {
        const int x = bi & 7, p = bi >> 3;
        return ((p / kXcdChunk) * 8 + x) * kXcdChunk + p % kXcdChunk;
    }
    __device__ __forceinline__ bool begin(int b) const { return b < nblk; }
    __device__ __forceinline__ const double *src() const { return gsrc; }
    template <int N>
    __device__ __forceinline__ void end(int, double (&)[N], double *) {}
};
// [hot-path device end]

// Proximal-path segments of one coordinate for the normalized duality gap
// (Section 3): D_i(s) = a1 s^2 (s < b1), c (b1 <= s < b2), a3 s^2 (s >= b2);
// objective share f1 s, f0, f3 s + f3b on the same pieces.
struct Seg {
    double b1, b2, a1, c, a3, f1, f0, f3, f3b;
};

__device__ __forceinline__ Seg seg_x(double x, double g, double lv, double uv, double omega) {
    Seg q;
    q.b2 = INFINITY;
    q.a3 = 0.0;
    q.f3 = 0.0;
    q.f3b = 0.0;
    if (g == 0.0) {
        q.b1 = INFINITY;
        q.a1 = q.c = q.f1 = q.f0 = 0.0;
        return q;
    }
    const double dist = g > 0.0 ? x - lv : uv - x;  // may be +inf
    q.a1 = g * g / omega;
    q.f1 = q.a1;
    q.b1 = omega * dist / fabs(g);
    q.c = isfinite(dist) ? omega * dist * dist : INFINITY;
    q.f0 = isfinite(dist) ? fabs(g) * dist : INFINITY;
    return q;
}

// y in Y; af/bf: lc/uc finite; a/b: slopes for positive/negative y^.
__device__ __forceinline__ Seg seg_y(double y, bool af, double a, bool bf, double b, double omega) {
    Seg q;
    q.b1 = q.b2 = INFINITY;
    q.a1 = q.c = q.a3 = q.f1 = q.f0 = q.f3 = q.f3b = 0.0;
    if (y > 0.0) {
        if (af && a > 0.0) {          // moves up without end
            q.a1 = q.f1 = omega * a * a;
        } else if (af && a == 0.0) {  // static
        } else {
            q.a1 = q.f1 = af ? omega * a * a : 0.0;
            q.b1 = af ? y / (omega * (-a)) : 0.0;  // reaches 0
            q.c = y * y / omega;
            q.f0 = af ? -a * y : 0.0;
            if (bf && b < 0.0) {                   // leaves 0 downwards
                q.b2 = y / (omega * (-b));
                q.a3 = q.f3 = omega * b * b;
                q.f3b = (b - (af ? a : 0.0)) * y;
            }
        }
    } else if (y < 0.0) {
        if (bf && b < 0.0) {
            q.a1 = q.f1 = omega * b * b;
        } else if (bf && b == 0.0) {
        } else {
            q.a1 = q.f1 = bf ? omega * b * b : 0.0;
            q.b1 = bf ? -y / (omega * b) : 0.0;
            q.c = y * y / omega;
            q.f0 = bf ? -b * y : 0.0;
            if (af && a > 0.0) {
                q.b2 = -y / (omega * a);
                q.a3 = q.f3 = omega * a * a;
                q.f3b = (a - (bf ? b : 0.0)) * y;
            }
        }
    } else {
        if (af && a > 0.0) q.a1 = q.f1 = omega * a * a;
        else if (bf && b < 0.0) q.a1 = q.f1 = omega * b * b;
    }
    return q;
}


}  // namespace pdlp
