// Internal declarations shared by the kernel and host translation units of
// the gfx950 PDLP library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdlp {

// [hot-path constants begin]
constexpr int kThreads = 256;        // threads per workgroup (4 wave64)
#ifndef PDLP_STAGE
#define PDLP_STAGE 2048
#endif
constexpr int kStage = PDLP_STAGE;   // LDS product stage of the CSR stream kernels (doubles)
constexpr int kMaxBlockRows = 1024;  // rows per stream block
constexpr int kMedRow = 64;          // rows longer than this leave the stream path ...
constexpr int kWaveMax = 1024;       // ... for one wave per row up to this length, then a workgroup
constexpr int kWaveRows = kThreads / 64;
// Persistent CSR stream kernels keep 8 waves per SIMD (8 workgroups per CU,
// the persistent grid of 2048 on 256 CUs): at most 64 VGPRs.
#ifndef PDLP_STREAM_WAVES
#define PDLP_STREAM_WAVES 8
#endif
#define PDLP_STREAM_KERNEL \
    __global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(PDLP_STREAM_WAVES)))
// [hot-path constants end]
constexpr int kGapPts = 32;          // abscissae per multisection pass of the gap search
constexpr int kGapMaxPass = 24;
constexpr int kGapNewton = 12;       // active-set steps before the multisection fallback
constexpr int kGapHead = 8;          // active-set steps launched before the first look at the state

// CSR matrix on the device with a row-block partition: block b covers rows
// [blk[b], blk[b+1]) and is one of
//   stream: rows of at most med_row (default kMedRow) nonzeros whose nonzeros fit
//           the LDS stage;
//   wave:   up to kWaveRows rows of (med_row, kWaveMax] nonzeros, one wave each;
//   long:   a single row of more than kWaveMax nonzeros (whole workgroup).
// Entries inside a row may appear in any column order.
struct DCsr {
    int32_t rows = 0, cols = 0;
    int64_t nnz = 0;
    int32_t *row_ptr = nullptr, *col = nullptr;
    double *val = nullptr;
    int32_t nblk = 0;
    int32_t *blk = nullptr;
    int32_t grid = 0;  // workgroups of the persistent stream kernels
    int32_t med_row = kMedRow;  // longest row of the stream class (the block partition's)
    int32_t stage = kStage;     // nonzeros per stream block of the partition
    // Optional copy of the entries of short-row blocks sorted by column
    // (scol, sval) with each entry's position in the block (slot), so that
    // the lanes of a wave gather neighbouring words; the products are staged
    // at their slots, so row sums keep the stored order.  sblk[b] = 1 marks
    // the blocks that use the copy.  Null when absent.
    const int32_t *scol = nullptr;
    const double *sval = nullptr;
    const uint16_t *slot = nullptr;
    const uint8_t *sblk = nullptr;
};

// Two-phase product out = M v for a gathered vector v too large for the
// caches: v's index range is cut into S segments of a few MB (balanced by
// nonzeros, S a multiple of 8, at most 128), and segment s is worked by XCD
// s mod 8 only, so that its slice of v stays in that XCD's L2 while it is
// gathered.  Pairs: a row of at most kMedRow nonzeros makes one pair per
// nonzero, a longer row one pair per segment it touches (its entries there
// in stored order).
//   phase 1 (gather): Q receives the sum of every pair -- single-entry pairs
//     (Q[0, n1)) as plain products in chunks of consecutive entries, pairs of
//     two or more entries (Q[n1, ...)) as rows of the CSR matrix G; the work
//     items of segment s are listed for XCD s mod 8 (glist);
//   phase 2 (stage): per row block of P, the block's pairs are read from
//     their 2S runs of Q (run (b, c, s) = Q[qoff[b*2S+c*S+s] ..
//     qoff[(b+1)*2S+c*S+s]) for the single (c = 0) and multi-entry (c = 1)
//     pairs of segment s), staged in LDS at their slot (the pair's position
//     in the block: rows in order and, inside a row, its entries' stored
//     order or its pairs' segment order), and each row is summed in that
//     order before the row work.
// A row of at most kMedRow nonzeros is thus summed exactly as by the single
// pass (same products, same order).
struct SegCsr {
    int32_t S = 0;                    // segments (0: not built)
    int64_t n1 = 0;                   // single-entry pairs
    const int32_t *c1 = nullptr;      // their gathered index
    const double *v1 = nullptr;       // and value
    const int32_t *chunk = nullptr;   // singles chunk k: Q[chunk[2k], chunk[2k+1])
    DCsr G;                           // multi-entry pairs: row t -> Q[n1 + t]
    const int32_t *glist = nullptr;   // work items by XCD, glist[t*8 + x]: G block (>= 0),
                                      // singles chunk -2-k, or nothing (-1)
    int32_t glen = 0;
    int32_t grid1 = 0;                // workgroups of phase 1 (a multiple of 8)
    double *Q = nullptr;              // pair sums
    const uint16_t *slot = nullptr;   // slot of pair q in its phase-2 block
    const int32_t *qoff = nullptr;    // (P.nblk + 1) * 2S run starts
    DCsr P;                           // phase 2: rows of M, row_ptr over pairs, blocks
};

// Scaled problem vectors seen by the iteration.
struct Vecs {
    const double *c, *lc, *uc, *lv, *uv;
};

// Double-buffered iterate: index `cur` (in Ctrl) is the accepted point,
// cur^1 receives the candidate.
struct Iter {
    double *X[2], *Y[2], *AX[2], *ATY[2];
    double *sx, *sy;
};

// Device control block of the step loop.  Written by the step-decision
// kernel (one thread) and by the host between iteration blocks; every other
// kernel only reads it, which is what lets a block of step attempts run
// without host synchronization.
struct Ctrl {
    double eta;           // step size of the next attempt
    double eta_hat;       // starting step size of the next accepted step
    double omega;         // primal weight
    double eta_used;      // step of the last accepted attempt (primal average)
    double eta_avg_y;     // step pending for the dual average
    double seta;          // sum of accepted steps since the restart
    double last_eta_bar;
    double red_exp, grow_exp;
    double fixed_eta;
    long long k, t, attempts, block_acc, block_target;
    int cur;              // which buffer holds the accepted iterate
    int stop;             // block target reached or numerical error
    int need_primal;      // the next attempt starts with the standalone primal step
    int run_at;           // last attempt accepted: run the A^T product
    int pending_sy;       // dual average owes eta_avg_y * y_cur
    int numerr;
    int fixed_step;
    int pad;
};

// Device-side state of one normalized-duality-gap evaluation.
struct GapState {
    double r2, r, omega, A0, Dinf;
    double lo, hi;
    double pts[kGapPts];
    int npass, done, pathend, linear;
    double s_star, Acoef, Bcoef, f, mu;
    int bad;
    int newton;           // 1 while the active-set iteration runs
    double s_cur, s_prev, D_prev;
    int nsteps;
    int exact;            // 1 when the root was found on its segment (no cap, no bracket fallback)
};

// Results of the termination evaluation (Section 7).
struct KktOut {
    double primal_obj, dual_obj, rel_gap;
    double primal_res_abs, primal_res_rel, dual_res_abs, dual_res_rel;
    double pad;
};

// Appendix D test values of one infeasibility candidate: primal-test
// objective and weighted residual, c^T x and the dual-test weighted
// residual, and the count of non-finite inputs.
struct CertOut {
    double pobj, pres, dobj, dres, nonfinite;
};
constexpr int kCertVals = 5;           // the fields of CertOut, in order
constexpr unsigned kCertMax = 0x0Au;   // pres and dres reduce by max, the rest by sum

// Block maps of a batch of LPs packed block-diagonally: rows (columns) of
// instance i are [roff[i], roff[i+1]) ([coff[i], coff[i+1])); row blocks of
// A and of A^T never straddle two instances.
struct BatchMaps {
    int32_t B = 0;                       // instances
    int32_t nA = 0, nT = 0;              // blocks of A and of A^T
    const int32_t *ablk_inst = nullptr;  // instance of each A block [nA]
    const int32_t *tblk_inst = nullptr;  // instance of each A^T block [nT]
    const int32_t *ablk_off = nullptr;   // first A block of each instance [B+1]
    const int32_t *tblk_off = nullptr;   // first A^T block of each instance [B+1]
    // The instances a launch serves and their blocks, set by the host: ilist
    // (ni instances), alist (na A blocks), tlist (nt A^T blocks) and clist
    // (nc check blocks: c < nT is A^T block c, c >= nT is A block c - nT).
    int32_t ni = 0, na = 0, nt = 0, nc = 0;
    const int32_t *ilist = nullptr, *alist = nullptr, *tlist = nullptr, *clist = nullptr;
    // Decision record of an unrolled run (null otherwise): the step-decision
    // kernel stores eta and omega of accepted step k of instance i at i * tape_K + k.
    double *tape_eta = nullptr, *tape_omega = nullptr;
    int64_t tape_K = 0;
};

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return hipGetLastError().

// step attempt pieces; ev (optional) = {start, stop} events recorded by the launch itself
hipError_t launch_primal(hipStream_t s, int n, Vecs v, Iter it, const Ctrl *ctrl, double *part,
                         int grid, hipEvent_t *ev = nullptr);
hipError_t launch_spmv_dual(hipStream_t s, const DCsr &A, Vecs v, Iter it, const Ctrl *ctrl,
                            double *part, hipEvent_t *ev = nullptr);
hipError_t launch_step_decide(hipStream_t s, Ctrl *ctrl, const double *part_dual, int gd,
                              const double *part_ps, int gps, const double *part_pf, int gpf,
                              hipEvent_t *ev = nullptr);
hipError_t launch_spmv_primal(hipStream_t s, const DCsr &AT, Vecs v, Iter it, const Ctrl *ctrl,
                              double *part, hipEvent_t *ev = nullptr);
hipError_t launch_flush_sy(hipStream_t s, int m, Iter it, Ctrl *ctrl);
// A^T y' + primal row work in two phases (SegCsr); ev = {start, stop} of
// phase 1 then phase 2 (four events)
hipError_t launch_seg_primal(hipStream_t s, const SegCsr &sg, Vecs v, Iter it, const Ctrl *ctrl,
                             double *part, hipEvent_t *ev = nullptr);
// plain two-phase product out = M v (both phases)
hipError_t launch_seg_plain(hipStream_t s, const SegCsr &sg, const double *v, double *out);

// plain products and vector helpers
hipError_t launch_spmv_plain(hipStream_t s, const DCsr &A, const double *x, double *out);
hipError_t launch_scale_div(hipStream_t s, int64_t len, const double *a, const double *d,
                            double *out);  // out = a / d
hipError_t launch_scale_mul(hipStream_t s, int64_t len, const double *a, const double *d,
                            double *out);  // out = a * d
hipError_t launch_average(hipStream_t s, int64_t len, const double *sum, double seta,
                          double *out);
hipError_t launch_fill(hipStream_t s, int64_t len, double *a, double v);
hipError_t launch_clamp0(hipStream_t s, int n, const double *lv, const double *uv, double *x);
hipError_t launch_copy(hipStream_t s, int64_t len, const double *a, double *out);
// out[i] = in[perm[i]] (gather) / out[perm[i]] = in[i] (scatter)
hipError_t launch_gather(hipStream_t s, int64_t len, const int32_t *perm, const double *in,
                         double *out);
hipError_t launch_scatter(hipStream_t s, int64_t len, const int32_t *perm, const double *in,
                          double *out);

// reductions (deterministic): result written to out[0..]
hipError_t launch_dist2(hipStream_t s, int64_t len, const double *a, const double *b, double *part,
                        int grid, double *out);
hipError_t launch_sum_max(hipStream_t s, const double *part, int grid, int nv, const int *is_max,
                          double *out);

// preconditioning
hipError_t launch_row_norms(hipStream_t s, const DCsr &A, int use_inf, double *out);
hipError_t launch_norm_to_factor(hipStream_t s, int len, double *nrm);  // sqrt, 0 -> 1
hipError_t launch_scale_matrix(hipStream_t s, const DCsr &A, const double *rf, const double *cf);
hipError_t launch_div_inplace(hipStream_t s, int len, double *d, const double *f);
hipError_t launch_scale_vectors(hipStream_t s, int m, int n, const double *d1, const double *d2,
                                const double *c, const double *lc, const double *uc,
                                const double *lv, const double *uv, double *cs, double *lcs,
                                double *ucs, double *lvs, double *uvs);
hipError_t launch_absmax(hipStream_t s, int64_t len, const double *a, double *part, int grid,
                         double *out);
hipError_t launch_primal_weight_init(hipStream_t s, int m, int n, const double *c,
                                     const double *lc, const double *uc, double *part, int grid,
                                     double *out);  // out[0] = ||c||^2, out[1] = ||Combine||^2

// transpose and relabelling
hipError_t launch_row_ids(hipStream_t s, int m, const int32_t *row_ptr, int32_t *rowid);
// rowid[e] = new_row[r] for the entries e of old row r
hipError_t launch_row_ids_mapped(hipStream_t s, int m, const int32_t *row_ptr,
                                 const int32_t *new_row, int32_t *rowid);
// key[e] = new_col[col[e]]
hipError_t launch_relabel(hipStream_t s, int64_t nnz, const int32_t *col, const int32_t *new_col,
                          uint32_t *key);
// rows of the relabelled matrix: new row r' is old row row_order[r'] with its entries in stored
// order and columns relabelled; orig_pos[e'] = old entry index
hipError_t launch_permute_rows(hipStream_t s, int m, const int32_t *row_order,
                               const int32_t *old_rp, const int32_t *old_col,
                               const double *old_val, const int32_t *new_col,
                               const int32_t *new_rp, int32_t *ncol, double *nval,
                               int32_t *orig_pos);
hipError_t launch_iota(hipStream_t s, int64_t len, int32_t *a);
// Stable LSD radix sort of n (key, value) pairs by the low key_bits bits of
// the keys (8 bits per pass).  keys[0]/vals[0] hold the input, keys[1]/vals[1]
// are buffers of the same length; the sorted pairs end in keys[*which] /
// vals[*which].  temp holds radix_sort_temp_ints(n) int32.
int64_t radix_sort_temp_ints(int64_t n);
hipError_t radix_sort_pairs(hipStream_t s, int64_t n, int key_bits, uint32_t *keys[2],
                            int32_t *vals[2], int32_t *temp, int *which);
hipError_t launch_transpose_finish(hipStream_t s, int64_t nnz, int n, const int32_t *sorted_cols,
                                   const int32_t *perm, const int32_t *rowid, const double *val,
                                   int32_t *t_row_ptr, int32_t *t_col, double *t_val);

// termination evaluation (original units)
hipError_t launch_kkt(hipStream_t s, int m, int n, const double *xs, const double *ys,
                      const double *axs, const double *atys, const double *d1, const double *d2,
                      const double *c, const double *lc, const double *uc, const double *lv,
                      const double *uv, int mode, double obj_offset, double *part, int grid,
                      double *r_out, double *x_out, double *y_out, KktOut *out);

// infeasibility certificates (Appendix D): candidate (xa - xb, ya - yb), or
// (xa, ya) when xb/yb are null, projected onto Xbar x Y; its test values from
// the products of the projected point; its unscaled output (x, y, r).  A null
// px / pax (no variable with an infinite bound) reads as zeros.
hipError_t launch_cert_point(hipStream_t s, int m, int n, const double *xa, const double *xb,
                             const double *ya, const double *yb, const double *lc,
                             const double *uc, const double *lv, const double *uv, double *px,
                             double *py);
hipError_t launch_cert(hipStream_t s, int m, int n, const double *px, const double *py,
                       const double *pax, const double *paty, const double *d1, const double *d2,
                       const double *c, const double *lc, const double *uc, const double *lv,
                       const double *uv, double *part, int grid, CertOut *out);
hipError_t launch_cert_out(hipStream_t s, int m, int n, const double *px, const double *py,
                           const double *paty, const double *d1, const double *d2,
                           const double *lv, const double *uv, double *x_out, double *y_out,
                           double *r_out);

// normalized duality gap: launch_gap = launch_gap_head then launch_gap_tail.
// The head sets up the evaluation and runs kGapHead active-set steps; the
// tail (the remaining steps, the multisection fallback and the final
// segment) does nothing once gs->done is 2 or 3, so a caller that reads the
// state after the head may leave it out then.
hipError_t launch_gap(hipStream_t s, int m, int n, Vecs v, const double *x, const double *y,
                      const double *ax, const double *aty, const double *xr, const double *yr,
                      double omega, double *part, int grid, GapState *gs);
hipError_t launch_gap_head(hipStream_t s, int m, int n, Vecs v, const double *x,
                           const double *y, const double *ax, const double *aty,
                           const double *xr, const double *yr, double omega, double *part,
                           int grid, GapState *gs);
hipError_t launch_gap_tail(hipStream_t s, int m, int n, Vecs v, const double *x,
                           const double *y, const double *ax, const double *aty, double *part,
                           int grid, GapState *gs);

// device-rate probes (timed by the caller)
hipError_t launch_rate_copy(hipStream_t s, int64_t len, const double *a, double *b);
hipError_t launch_rate_idx(hipStream_t s, int64_t n, uint32_t domain, uint32_t *idx);
hipError_t launch_rate_gather(hipStream_t s, int64_t n, const uint32_t *idx, const double *x,
                              double *out, int grid);

// batched solver (one control block per instance; per-block partial sums)
// dst[k] = src[perm[k]], k < len
hipError_t launch_take(hipStream_t s, int64_t len, const int64_t *perm, const double *src,
                       double *dst);
// primal candidates of the first attempt of a round (instances with need_primal)
hipError_t launch_b_primal(hipStream_t s, const DCsr &AT, Vecs v, Iter it, const Ctrl *ctrl,
                           const BatchMaps &bm, double *pps);
// one step attempt of every listed running instance: dual product, step
// decision, then the primal product (or the primal candidate again after a
// rejection)
hipError_t launch_b_attempt(hipStream_t s, const DCsr &A, const DCsr &AT, Vecs v, Iter it,
                            Ctrl *ctrl, const BatchMaps &bm, double *pd, double *pps,
                            double *ppf);
hipError_t launch_b_settle(hipStream_t s, const DCsr &A, const DCsr &AT, Iter it, Ctrl *ctrl,
                           const BatchMaps &bm);
// masked per-instance elementwise ops: op 0 out = a / sv[i], 1 out = a, 2 out = sv[i]
hipError_t launch_b_elementwise(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                                const int32_t *mask, int op, const double *sv, const double *xa,
                                double *xo, const double *ya, double *yo);
// product over the listed blocks of M whose instance is masked in
hipError_t launch_b_spmv_plain(hipStream_t s, const DCsr &M, const int32_t *blk_inst,
                               const int32_t *list, int nlist, const int32_t *mask,
                               const double *x, double *out);
// per-instance pairs out[2i], out[2i+1]: op 0 ||xa-xb||^2, ||ya-yb||^2;
// op 2 ||c||^2, ||Combine(lc, uc)||^2; op 3 max |A^T value| (maxmask 1)
hipError_t launch_b_norms(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                          const int32_t *mask, int op, const double *xa, const double *xb,
                          const double *ya, const double *yb, Vecs v, double *part,
                          unsigned maxmask, double *out);
// termination sums per instance, out[7i + k]: 0 primal res abs, 1 rel, 2 dual res abs, 3 rel
// (max), 4 c^T x, 5 dual objective terms, 6 non-finite count; p0/p1 = {x, y, ax, aty}
// chosen per instance by sel
hipError_t launch_b_kkt(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                        const int32_t *mask, const int32_t *sel, const double *const *p0,
                        const double *const *p1, const double *d1, const double *d2, Vecs orig,
                        int mode, double *part, double *out, double *r_out, double *x_out,
                        double *y_out);
// checkpoint of a recorded run: instances with slot[i] >= 0 copy x | y | Sx | Sy into
// ck + slot[i] * 2 (N + M)
hipError_t launch_b_checkpoint(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                               const int32_t *slot, const double *x, const double *y,
                               const double *sx, const double *sy, double *ck, int64_t N,
                               int64_t M);
// normalized duality gap per instance: begin = radius, slopes and the first
// abscissa; then active-set steps first .. first+count-1 of at most `total`
// infeasibility candidates of masked instances (see launch_cert_point)
hipError_t launch_b_cert_point(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, int cand, Iter it, const double *xb,
                              Vecs orig, double *px, double *py);
hipError_t launch_b_cert(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                         const int32_t *mask, const double *px, const double *py,
                         const double *pax, const double *paty, const double *d1,
                         const double *d2, Vecs orig, double *part, double *out);
hipError_t launch_b_cert_out(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                             const int32_t *mask, const double *px, const double *py,
                             const double *paty, const double *d1, const double *d2, Vecs orig,
                             double *x_out, double *y_out, double *r_out);
hipError_t launch_b_gap_begin(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, Vecs v, const double *x, const double *y,
                              const double *ax, const double *aty, const double *xr,
                              const double *yr, const double *omega, double *part, GapState *gs);
hipError_t launch_b_gap_steps(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                              const int32_t *mask, Vecs v, const double *x, const double *y,
                              const double *ax, const double *aty, double *part, GapState *gs,
                              int first, int count, int total);

// unrolled (differentiable) map: decisions of step s of every instance
struct UStepArgs {
    const double *eta, *omega;  // recorded [B * K]
    int64_t K, s;
    const int32_t *ablk_inst, *tblk_inst;
};
// one replayed step for every instance: x -> xn, y -> yn with products, sums;
// seg_* (nullable) receive w = 2 xn - x, y, the interior flags and the dual
// cases; sig (nullable) counts interior and moving coordinates per instance
hipError_t launch_u_step(hipStream_t s, const DCsr &A, const DCsr &AT, Vecs v, UStepArgs u,
                         const double *x, const double *y, const double *ax, const double *aty,
                         double *xn, double *yn, double *axn, double *atyn, double *sx, double *sy,
                         double *seg_w, double *seg_y, uint8_t *seg_p, uint8_t *seg_q,
                         unsigned long long *sig);
hipError_t launch_u_restart_adj(hipStream_t s, const DCsr &A, const DCsr &AT, const BatchMaps &bm,
                                const int32_t *rt, const double *seta, double *xb, double *yb,
                                double *sxb, double *syb);
// adjoint of one step for every instance (xb, yb: adjoint of the state, in place)
hipError_t launch_u_reverse(hipStream_t s, const DCsr &A, const DCsr &AT, UStepArgs u,
                            const double *seg_w, const double *seg_y, const uint8_t *seg_p,
                            const uint8_t *seg_q, double *xb, double *yb, const double *sxb,
                            const double *syb, double *yhb, double *vb, double *gc, double *glc,
                            double *guc, double *gval);
// one replayed step (as launch_u_step, without segment storage) and its
// tangent: dA / dAT carry the direction's scaled values in A's pattern,
// (dc, dlc, duc) the rest of the direction; (dx, dy, dax, daty) -> (dxn, dyn,
// daxn, datyn), tangent sums dsx, dsy; tm*, tn* are work vectors (m, n)
hipError_t launch_u_tangent_step(hipStream_t s, const DCsr &A, const DCsr &AT, const DCsr &dA,
                                 const DCsr &dAT, Vecs v, UStepArgs u, const double *dc,
                                 const double *dlc, const double *duc, const double *x,
                                 const double *y, const double *ax, const double *aty,
                                 double *xn, double *yn, double *axn, double *atyn, double *sx,
                                 double *sy, const double *dx, const double *dy, const double *dax,
                                 const double *daty, double *dxn, double *dyn, double *daxn,
                                 double *datyn, double *dsx, double *dsy, double *tm1,
                                 double *tm2, double *tn1, double *tn2);
hipError_t launch_u_add(hipStream_t s, int64_t len, const double *a, const double *b, double *out);
// bad[0] += invalid entries of new data in device memory (see ku_check_data)
hipError_t launch_u_check_data(hipStream_t s, int64_t N, int64_t M, int64_t NZ, const double *c,
                               const double *lc, const double *uc, const double *val,
                               const double *cur_lc, const double *cur_uc,
                               unsigned long long *bad);
hipError_t launch_u_scale_values(hipStream_t s, const DCsr &A, const double *val, const double *d1,
                                 const double *d2, const int32_t *a2t, double *va, double *vt);
hipError_t launch_u_finish(hipStream_t s, const DCsr &A, int64_t N, const double *d1,
                           const double *d2, const double *lc, const double *uc, const double *gc,
                           const double *glc, const double *guc, const double *gval, double *oc,
                           double *olc, double *ouc, double *oval);

}  // namespace pdlp
