// Host driver and C ABI of the unrolled, differentiable PDHG map over a
// batch of LPs.
//
// Forward: Algorithm 1 runs exactly K accepted steps per instance on the
// batched solver (restart checks, no termination), recording every accepted
// step's step size and primal weight (written by the step-decision kernel)
// and every restart with its candidate, and checkpointing the state every
// `ckpt` steps.  Those decisions are then constants: the map from the data
// (c, lc, uc, values of A) to x_K is the replay of K steps with them
// (pdlp_unroll_kernels.hip), and the backward pass is its adjoint, run
// segment by segment backwards: restore the segment's checkpoint, replay it
// storing what the reverse needs, then the reverse steps.
//
// Scaling: D1, D2 come from the preconditioning at creation and stay fixed;
// every scaled quantity is formed from the original data as
// A~_ij = (D1_i A_ij) D2_j, c~ = D2 c, (lc~, uc~) = D1 (lc, uc),
// (lv~, uv~) = (lv, uv) / D2, for the recorded run and for new data alike.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "pdlp_batch.h"

using namespace pdlp::host;
using pdlp::BatchMaps;
using pdlp::DCsr;
using pdlp::UStepArgs;
using pdlp::Vecs;

struct pdlp_unroll {
    pdlp_batch *b = nullptr;
    Arena *arena = nullptr;       // data, identity lists, work buffers
    Arena *tape_arena = nullptr;  // tape and checkpoints of the last forward
    int64_t N = 0, M = 0, NZ = 0;
    double *val_orig = nullptr;
    int32_t *a2t = nullptr;
    BatchMaps all;                // every instance and block, in order
    BatchRecord rec;
    bool recorded = false;
    std::vector<double> eta_h, omega_h, seta_h;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> rst;  // per step: (instance, kind)
    // work
    int32_t work_ckpt = 0;
    double *rx, *ry, *rax, *raty, *rxn, *ryn, *raxn, *ratyn, *rsx, *rsy;
    double *seg_w, *seg_y;
    uint8_t *seg_p, *seg_q;
    double *xb, *yb, *sxb, *syb, *yhb, *vb, *gc, *glc, *guc, *gval, *gx_d;
    double *oc, *olc, *ouc, *oval, *tmp_n;
    int32_t *rt_d, *mavg_d, *many_d, *rt_h, *mavg_h, *many_h;
    double *sv_d, *sv_h, *zero_d;
    unsigned long long *sig_d, *sig_h;
    pdlp_unroll_stats stats{};
    // tangent (forward-mode) buffers, allocated at the first tangent
    Arena *tan_arena = nullptr;
    double *dav, *datv, *dcs, *dlcs, *ducs, *dir_c, *dir_l, *dir_u, *dir_v;
    double *tdx, *tdxn, *tdaty, *tdatyn, *tdsx, *tn1, *tn2;
    double *tdy, *tdyn, *tdax, *tdaxn, *tdsy, *tm1, *tm2;
    // checks of data in device memory
    unsigned long long *bad_d = nullptr, *bad_h = nullptr;
    hipEvent_t join = nullptr;  // orders the library's stream after a caller's stream
    ~pdlp_unroll() {
        if (join) (void)hipEventDestroy(join);
        delete tan_arena;
        delete tape_arena;
        delete arena;
        delete b;
    }
};

namespace {

hipStream_t stream_of(const pdlp_unroll *u) { return u->b->P->stream; }

void sync(pdlp_unroll *u) { HIPCHECK(hipStreamSynchronize(stream_of(u))); }

// Where the caller's arrays live.  Device arrays are read and written on the
// library's stream after the work already queued on the caller's stream
// (join_caller); every call returns after its work has finished.
enum class Mem { host, device };

void join_caller(pdlp_unroll *u, hipStream_t caller) {
    hipStream_t own = stream_of(u);
    if (!caller || caller == own) return;
    if (!u->join) HIPCHECK(hipEventCreateWithFlags(&u->join, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(u->join, caller));
    HIPCHECK(hipStreamWaitEvent(own, u->join, 0));
}

void copy_in(pdlp_unroll *u, double *dst, const double *src, int64_t len, Mem mem) {
    if (len > 0 && src)
        HIPCHECK(hipMemcpyAsync(dst, src, sizeof(double) * len,
                                mem == Mem::host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                stream_of(u)));
}

void copy_out(pdlp_unroll *u, double *dst, const double *src, int64_t len, Mem mem) {
    if (len > 0 && dst)
        HIPCHECK(hipMemcpyAsync(dst, src, sizeof(double) * len,
                                mem == Mem::host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                stream_of(u)));
}

// Replay and reverse buffers for segments of `ckpt` steps (allocated once per cadence).
void ensure_work(pdlp_unroll *u, int32_t ckpt) {
    if (u->work_ckpt == ckpt) return;
    Arena &a = *u->arena;
    const int64_t N = u->N, M = u->M;
    const int B = u->b->B;
    double **vn[] = {&u->rx, &u->raty, &u->rxn, &u->ratyn, &u->rsx, &u->xb, &u->sxb, &u->vb,
                     &u->gc, &u->gx_d, &u->oc, &u->tmp_n};
    double **vm[] = {&u->ry, &u->rax, &u->ryn, &u->raxn, &u->rsy, &u->yb, &u->syb, &u->yhb,
                     &u->glc, &u->guc, &u->olc, &u->ouc};
    if (u->work_ckpt == 0) {
        for (auto p : vn) *p = a.dev<double>(N);
        for (auto p : vm) *p = a.dev<double>(M);
        u->gval = a.dev<double>(u->NZ);
        u->oval = a.dev<double>(u->NZ);
        u->rt_d = a.dev<int32_t>(B);
        u->mavg_d = a.dev<int32_t>(B);
        u->many_d = a.dev<int32_t>(B);
        u->rt_h = a.host<int32_t>(B);
        u->mavg_h = a.host<int32_t>(B);
        u->many_h = a.host<int32_t>(B);
        u->sv_d = a.dev<double>(B);
        u->sv_h = a.host<double>(B);
        u->zero_d = a.dev<double>(B);
        u->sig_d = a.dev<unsigned long long>(B);
        u->sig_h = a.host<unsigned long long>(B);
        HIPCHECK(pdlp::launch_fill(stream_of(u), B, u->zero_d, 0.0));
    } else {
        a.release(u->seg_w);
        a.release(u->seg_y);
        a.release(u->seg_p);
        a.release(u->seg_q);
    }
    u->seg_w = a.dev<double>((size_t)ckpt * N);
    u->seg_y = a.dev<double>((size_t)ckpt * M);
    u->seg_p = a.dev<uint8_t>((size_t)ckpt * N);
    u->seg_q = a.dev<uint8_t>((size_t)ckpt * M);
    sync(u);
    u->work_ckpt = ckpt;
}

UStepArgs step_args(const pdlp_unroll *u, int64_t s) {
    return UStepArgs{u->rec.eta, u->rec.omega, u->rec.K, s, u->b->bm.ablk_inst,
                     u->b->bm.tblk_inst};
}

void upload_i32(pdlp_unroll *u, int32_t *d, const int32_t *h) {
    HIPCHECK(hipMemcpyAsync(d, h, sizeof(int32_t) * u->b->B, hipMemcpyHostToDevice, stream_of(u)));
}

// Restarts right after replayed step s: (x, y) <- sums / S for the average
// kind, then the sums of every restarting instance are cleared.
void apply_restarts(pdlp_unroll *u, int64_t s) {
    const int B = u->b->B;
    const int64_t K = u->rec.K;
    for (int i = 0; i < B; ++i) u->mavg_h[i] = u->many_h[i] = 0;
    for (auto &e : u->rst[s]) {
        u->many_h[e.first] = 1;
        u->mavg_h[e.first] = e.second == 2;
        u->sv_h[e.first] = u->seta_h[(size_t)e.first * K + s];
    }
    hipStream_t st = stream_of(u);
    upload_i32(u, u->mavg_d, u->mavg_h);
    upload_i32(u, u->many_d, u->many_h);
    HIPCHECK(hipMemcpyAsync(u->sv_d, u->sv_h, sizeof(double) * B, hipMemcpyHostToDevice, st));
    const pdlp_problem *P = u->b->P;
    HIPCHECK(pdlp::launch_b_elementwise(st, P->A, P->AT, u->all, u->mavg_d, 0, u->sv_d, u->rsx,
                                        u->rx, u->rsy, u->ry));
    HIPCHECK(pdlp::launch_b_spmv_plain(st, P->A, u->all.ablk_inst, u->all.alist, u->all.na,
                                       u->mavg_d, u->rx, u->rax));
    HIPCHECK(pdlp::launch_b_spmv_plain(st, P->AT, u->all.tblk_inst, u->all.tlist, u->all.nt,
                                       u->mavg_d, u->ry, u->raty));
    HIPCHECK(pdlp::launch_b_elementwise(st, P->A, P->AT, u->all, u->many_d, 2, u->zero_d,
                                        nullptr, u->rsx, nullptr, u->rsy));
    sync(u);  // the pinned staging arrays are rewritten by the next call
}

void replay_from_start(pdlp_unroll *u) {
    const pdlp_problem *P = u->b->P;
    hipStream_t st = stream_of(u);
    HIPCHECK(pdlp::launch_clamp0(st, (int)u->N, P->lvs, P->uvs, u->rx));
    HIPCHECK(pdlp::launch_fill(st, u->M, u->ry, 0.0));
    HIPCHECK(pdlp::launch_spmv_plain(st, P->A, u->rx, u->rax));
    HIPCHECK(pdlp::launch_spmv_plain(st, P->AT, u->ry, u->raty));
    HIPCHECK(pdlp::launch_fill(st, u->N, u->rsx, 0.0));
    HIPCHECK(pdlp::launch_fill(st, u->M, u->rsy, 0.0));
}

void replay_from_checkpoint(pdlp_unroll *u, int64_t slot) {
    const pdlp_problem *P = u->b->P;
    hipStream_t st = stream_of(u);
    const int64_t N = u->N, M = u->M;
    const double *base = u->rec.ck + (size_t)slot * 2 * (size_t)(N + M);
    HIPCHECK(pdlp::launch_copy(st, N, base, u->rx));
    HIPCHECK(pdlp::launch_copy(st, M, base + N, u->ry));
    HIPCHECK(pdlp::launch_copy(st, N, base + N + M, u->rsx));
    HIPCHECK(pdlp::launch_copy(st, M, base + 2 * N + M, u->rsy));
    HIPCHECK(pdlp::launch_spmv_plain(st, P->A, u->rx, u->rax));
    HIPCHECK(pdlp::launch_spmv_plain(st, P->AT, u->ry, u->raty));
}

void replay_steps(pdlp_unroll *u, int64_t s0, int64_t s1, bool store, unsigned long long *sig) {
    const pdlp_problem *P = u->b->P;
    hipStream_t st = stream_of(u);
    const int64_t N = u->N, M = u->M;
    for (int64_t s = s0; s < s1; ++s) {
        const size_t o = (size_t)(s - s0);
        HIPCHECK(pdlp::launch_u_step(st, P->A, P->AT, P->scaled(), step_args(u, s), u->rx, u->ry,
                                     u->rax, u->raty, u->rxn, u->ryn, u->raxn, u->ratyn, u->rsx,
                                     u->rsy, store ? u->seg_w + o * N : nullptr,
                                     store ? u->seg_y + o * M : nullptr,
                                     store ? u->seg_p + o * N : nullptr,
                                     store ? u->seg_q + o * M : nullptr, sig));
        std::swap(u->rx, u->rxn);
        std::swap(u->ry, u->ryn);
        std::swap(u->rax, u->raxn);
        std::swap(u->raty, u->ratyn);
        if (!u->rst[s].empty()) apply_restarts(u, s);
    }
}

void download(pdlp_unroll *u, double *host, const double *dev, int64_t len) {
    if (!host || len <= 0) return;
    HIPCHECK(hipMemcpyAsync(host, dev, sizeof(double) * len, hipMemcpyDeviceToHost,
                            stream_of(u)));
}

// Original-unit data -> the problem's original copies and scaled data.
void set_data(pdlp_unroll *u, const double *c, const double *lc, const double *uc,
              const double *val, Mem mem) {
    pdlp_problem *P = u->b->P;
    hipStream_t st = stream_of(u);
    const int64_t N = u->N, M = u->M;
    if (mem == Mem::host) {
        if (c)
            for (int64_t j = 0; j < N; ++j)
                if (!std::isfinite(c[j]))
                    invalid("non-finite objective coefficient " + std::to_string(j));
        if (val)
            for (int64_t e = 0; e < u->NZ; ++e)
                if (!std::isfinite(val[e])) invalid("non-finite matrix value " + std::to_string(e));
        if (lc || uc) {
            std::vector<double> l(M), h(M);
            HIPCHECK(hipMemcpy(l.data(), P->lc, sizeof(double) * M, hipMemcpyDeviceToHost));
            HIPCHECK(hipMemcpy(h.data(), P->uc, sizeof(double) * M, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < M; ++i) {
                const double a = lc ? lc[i] : l[i], z = uc ? uc[i] : h[i];
                if (std::isnan(a) || std::isnan(z) || a == INFINITY || z == -INFINITY || a > z)
                    invalid("bad constraint bounds in row " + std::to_string(i));
            }
        }
    } else if (c || lc || uc || val) {
        if (!u->bad_d) {
            u->bad_d = u->arena->dev<unsigned long long>(1);
            u->bad_h = u->arena->host<unsigned long long>(1);
        }
        HIPCHECK(hipMemsetAsync(u->bad_d, 0, sizeof(unsigned long long), st));
        HIPCHECK(pdlp::launch_u_check_data(st, c ? N : 0, (lc || uc) ? M : 0, val ? u->NZ : 0, c,
                                           lc, uc, val, P->lc, P->uc, u->bad_d));
        HIPCHECK(hipMemcpyAsync(u->bad_h, u->bad_d, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        sync(u);
        if (*u->bad_h)
            invalid(std::to_string(*u->bad_h) +
                    " invalid entries (non-finite objective or matrix values, or bounds with "
                    "NaN, lc = +inf, uc = -inf or lc > uc)");
    }
    if (c) copy_in(u, P->c, c, N, mem);
    if (lc) copy_in(u, P->lc, lc, M, mem);
    if (uc) copy_in(u, P->uc, uc, M, mem);
    if (c || lc || uc)
        HIPCHECK(pdlp::launch_scale_vectors(st, (int)M, (int)N, P->d1, P->d2, P->c, P->lc, P->uc,
                                            P->lv, P->uv, P->cs, P->lcs, P->ucs, P->lvs, P->uvs));
    if (val && u->NZ > 0) {
        copy_in(u, u->val_orig, val, u->NZ, mem);
        HIPCHECK(pdlp::launch_u_scale_values(st, P->A, u->val_orig, P->d1, P->d2, u->a2t,
                                             P->A.val, P->AT.val));
        refresh_block_gathers(P, st);
    }
    sync(u);
}

void ensure_tangent(pdlp_unroll *u) {
    if (u->tan_arena) return;
    u->tan_arena = new Arena();
    Arena &a = *u->tan_arena;
    const int64_t N = u->N, M = u->M;
    double **vn[] = {&u->dcs, &u->dir_c, &u->tdx, &u->tdxn, &u->tdaty, &u->tdatyn, &u->tdsx,
                     &u->tn1, &u->tn2};
    double **vm[] = {&u->dlcs, &u->ducs, &u->dir_l, &u->dir_u, &u->tdy, &u->tdyn, &u->tdax,
                     &u->tdaxn, &u->tdsy, &u->tm1, &u->tm2};
    for (auto p : vn) *p = a.dev<double>(N);
    for (auto p : vm) *p = a.dev<double>(M);
    u->dav = a.dev<double>(u->NZ);
    u->datv = a.dev<double>(u->NZ);
    u->dir_v = a.dev<double>(u->NZ);
}

// Tangent of the recorded map along a direction in original units (null
// parts are zero): dc~ = D2 dc, (dlc~, duc~) = D1 (dlc, duc), dA~_ij =
// D1_i dA_ij D2_j; the replay runs beside it; dx = D2 dx~_K.
void tangent(pdlp_unroll *u, const double *dc, const double *dlc, const double *duc,
             const double *dval, double *dx, Mem mem) {
    if (!u->recorded) invalid("no recorded forward pass");
    ensure_tangent(u);
    const pdlp_problem *P = u->b->P;
    hipStream_t st = stream_of(u);
    const int64_t N = u->N, M = u->M, K = u->rec.K;
    const double t0 = now_s();
    struct Dir {
        double *dst;
        const double *src;
        int64_t len;
    } dirs[] = {{u->dir_c, dc, N}, {u->dir_l, dlc, M}, {u->dir_u, duc, M}, {u->dir_v, dval, u->NZ}};
    for (auto &d : dirs) {
        if (d.src) copy_in(u, d.dst, d.src, d.len, mem);
        else HIPCHECK(pdlp::launch_fill(st, d.len, d.dst, 0.0));
    }
    HIPCHECK(pdlp::launch_scale_mul(st, N, u->dir_c, P->d2, u->dcs));
    HIPCHECK(pdlp::launch_scale_mul(st, M, u->dir_l, P->d1, u->dlcs));
    HIPCHECK(pdlp::launch_scale_mul(st, M, u->dir_u, P->d1, u->ducs));
    if (u->NZ > 0)
        HIPCHECK(pdlp::launch_u_scale_values(st, P->A, u->dir_v, P->d1, P->d2, u->a2t, u->dav,
                                             u->datv));
    // the direction as matrices with the pattern of A~ and A~^T (no sorted copies)
    DCsr dA = P->A, dAT = P->AT;
    dA.val = u->dav;
    dAT.val = u->datv;
    dA.scol = dAT.scol = nullptr;
    dA.sval = dAT.sval = nullptr;
    dA.slot = dAT.slot = nullptr;
    dA.sblk = dAT.sblk = nullptr;
    replay_from_start(u);
    for (double *p : {u->tdx, u->tdaty, u->tdsx}) HIPCHECK(pdlp::launch_fill(st, N, p, 0.0));
    for (double *p : {u->tdy, u->tdsy}) HIPCHECK(pdlp::launch_fill(st, M, p, 0.0));
    HIPCHECK(pdlp::launch_spmv_plain(st, dA, u->rx, u->tdax));  // d(A~ x_0) = dA~ x_0
    for (int64_t s = 0; s < K; ++s) {
        HIPCHECK(pdlp::launch_u_tangent_step(
            st, P->A, P->AT, dA, dAT, P->scaled(), step_args(u, s), u->dcs, u->dlcs, u->ducs,
            u->rx, u->ry, u->rax, u->raty, u->rxn, u->ryn, u->raxn, u->ratyn, u->rsx, u->rsy,
            u->tdx, u->tdy, u->tdax, u->tdaty, u->tdxn, u->tdyn, u->tdaxn, u->tdatyn, u->tdsx,
            u->tdsy, u->tm1, u->tm2, u->tn1, u->tn2));
        std::swap(u->rx, u->rxn);
        std::swap(u->ry, u->ryn);
        std::swap(u->rax, u->raxn);
        std::swap(u->raty, u->ratyn);
        std::swap(u->tdx, u->tdxn);
        std::swap(u->tdy, u->tdyn);
        std::swap(u->tdax, u->tdaxn);
        std::swap(u->tdaty, u->tdatyn);
        if (!u->rst[s].empty()) {
            apply_restarts(u, s);  // values; leaves this step's masks in mavg_d, many_d, sv_d
            HIPCHECK(pdlp::launch_b_elementwise(st, P->A, P->AT, u->all, u->mavg_d, 0, u->sv_d,
                                                u->tdsx, u->tdx, u->tdsy, u->tdy));
            // product tangents of the current points (unchanged where nothing restarted)
            HIPCHECK(pdlp::launch_spmv_plain(st, dA, u->rx, u->tm1));
            HIPCHECK(pdlp::launch_spmv_plain(st, P->A, u->tdx, u->tm2));
            HIPCHECK(pdlp::launch_u_add(st, M, u->tm1, u->tm2, u->tdax));
            HIPCHECK(pdlp::launch_spmv_plain(st, dAT, u->ry, u->tn1));
            HIPCHECK(pdlp::launch_spmv_plain(st, P->AT, u->tdy, u->tn2));
            HIPCHECK(pdlp::launch_u_add(st, N, u->tn1, u->tn2, u->tdaty));
            HIPCHECK(pdlp::launch_b_elementwise(st, P->A, P->AT, u->all, u->many_d, 2, u->zero_d,
                                                nullptr, u->tdsx, nullptr, u->tdsy));
        }
    }
    HIPCHECK(pdlp::launch_scale_mul(st, N, u->tdx, P->d2, u->tmp_n));
    sync(u);
    u->stats.tangent_seconds = now_s() - t0;
    copy_out(u, dx, u->tmp_n, N, mem);
    sync(u);
}

// Creation from host arrays (pdlp_unroll_create and, after staging device
// arrays on the host, pdlp_unroll_create_device).
pdlp_unroll *unroll_new(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                        const int32_t *row_ptr, const int32_t *col, const double *val,
                        const double *c, const double *lc, const double *uc, const double *lv,
                        const double *uv, const pdlp_params *params, void *hip_stream) {
    auto *u = new pdlp_unroll();
    try {
        u->b = make_batch(count, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, nullptr,
                          params, hip_stream, true);
        u->arena = new Arena();
        pdlp_problem *P = u->b->P;
        u->N = P->n;
        u->M = P->m;
        u->NZ = P->nnz;
        hipStream_t st = P->stream;
        // A entry -> position in A^T (columns of A^T keep increasing row order)
        std::vector<int32_t> rp((size_t)u->M + 1), cl((size_t)u->NZ), trp((size_t)u->N + 1),
            a2t((size_t)u->NZ);
        HIPCHECK(hipMemcpy(rp.data(), P->A.row_ptr, sizeof(int32_t) * rp.size(),
                           hipMemcpyDeviceToHost));
        if (u->NZ > 0)
            HIPCHECK(hipMemcpy(cl.data(), P->A.col, sizeof(int32_t) * cl.size(),
                               hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(trp.data(), P->AT.row_ptr, sizeof(int32_t) * trp.size(),
                           hipMemcpyDeviceToHost));
        std::vector<int32_t> next(trp.begin(), trp.end() - 1);
        for (int64_t r = 0; r < u->M; ++r)
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) a2t[e] = next[cl[e]]++;
        Arena &a = *u->arena;
        u->val_orig = a.dev<double>(u->NZ);
        u->a2t = a.dev<int32_t>(u->NZ);
        if (u->NZ > 0) {
            HIPCHECK(hipMemcpyAsync(u->a2t, a2t.data(), sizeof(int32_t) * u->NZ,
                                    hipMemcpyHostToDevice, st));
            HIPCHECK(hipMemcpyAsync(u->val_orig, val, sizeof(double) * u->NZ,
                                    hipMemcpyHostToDevice, st));
            HIPCHECK(pdlp::launch_u_scale_values(st, P->A, u->val_orig, P->d1, P->d2, u->a2t,
                                                 P->A.val, P->AT.val));
            refresh_block_gathers(P, st);
        }
        // identity lists: every instance and block in order
        const BatchMaps &bm = u->b->bm;
        std::vector<int32_t> il(u->b->B), al(bm.nA), tl(bm.nT), cll(bm.nA + bm.nT);
        for (size_t k = 0; k < il.size(); ++k) il[k] = (int32_t)k;
        for (size_t k = 0; k < al.size(); ++k) al[k] = (int32_t)k;
        for (size_t k = 0; k < tl.size(); ++k) tl[k] = (int32_t)k;
        for (size_t k = 0; k < cll.size(); ++k) cll[k] = (int32_t)k;
        int32_t *d_i = a.dev<int32_t>(il.size()), *d_a = a.dev<int32_t>(al.size());
        int32_t *d_t = a.dev<int32_t>(tl.size()), *d_c = a.dev<int32_t>(cll.size());
        HIPCHECK(hipMemcpyAsync(d_i, il.data(), sizeof(int32_t) * il.size(), hipMemcpyHostToDevice, st));
        if (!al.empty())
            HIPCHECK(hipMemcpyAsync(d_a, al.data(), sizeof(int32_t) * al.size(), hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(d_t, tl.data(), sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(d_c, cll.data(), sizeof(int32_t) * cll.size(), hipMemcpyHostToDevice, st));
        u->all = bm;
        u->all.ni = (int32_t)il.size();
        u->all.na = (int32_t)al.size();
        u->all.nt = (int32_t)tl.size();
        u->all.nc = (int32_t)cll.size();
        u->all.ilist = d_i;
        u->all.alist = d_a;
        u->all.tlist = d_t;
        u->all.clist = d_c;
        HIPCHECK(hipStreamSynchronize(st));
    } catch (...) {
        delete u;
        throw;
    }
    return u;
}

}  // namespace

extern "C" {

int pdlp_unroll_create(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                       const int32_t *row_ptr, const int32_t *col, const double *val,
                       const double *c, const double *lc, const double *uc, const double *lv,
                       const double *uv, const pdlp_params *params, void *hip_stream,
                       pdlp_unroll **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        *out = unroll_new(count, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, params,
                          hip_stream);
    });
}

int pdlp_unroll_create_device(int32_t count, const int32_t *m, const int32_t *n,
                              const int64_t *nnz, const int32_t *row_ptr, const int32_t *col,
                              const double *val, const double *c, const double *lc,
                              const double *uc, const double *lv, const double *uv,
                              const pdlp_params *params, void *hip_stream, pdlp_unroll **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        const StagedBatch h = stage_batch(count, m, n, nnz, row_ptr, col, val, c, lc, uc, lv,
                                          uv, hip_stream);
        *out = unroll_new(count, m, n, nnz, h.row_ptr.data(), h.col.data(), h.val.data(),
                          h.c.data(), h.lc.data(), h.uc.data(), h.lv.data(), h.uv.data(),
                          params, hip_stream);
    });
}

void pdlp_unroll_destroy(pdlp_unroll *u) { delete u; }

int pdlp_unroll_set_data(pdlp_unroll *u, const double *c, const double *lc, const double *uc,
                         const double *val) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        set_data(u, c, lc, uc, val, Mem::host);
    });
}

int pdlp_unroll_set_data_device(pdlp_unroll *u, const double *c, const double *lc,
                                const double *uc, const double *val, void *hip_stream) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        join_caller(u, static_cast<hipStream_t>(hip_stream));
        set_data(u, c, lc, uc, val, Mem::device);
    });
}

int pdlp_unroll_tangent(pdlp_unroll *u, const double *dc, const double *dlc, const double *duc,
                        const double *dval, double *dx) {
    return guarded([&] {
        if (!u || !dx) invalid("NULL argument");
        tangent(u, dc, dlc, duc, dval, dx, Mem::host);
    });
}

int pdlp_unroll_tangent_device(pdlp_unroll *u, const double *dc, const double *dlc,
                               const double *duc, const double *dval, double *dx,
                               void *hip_stream) {
    return guarded([&] {
        if (!u || !dx) invalid("NULL argument");
        join_caller(u, static_cast<hipStream_t>(hip_stream));
        tangent(u, dc, dlc, duc, dval, dx, Mem::device);
    });
}

}  // extern "C"

namespace {

void forward(pdlp_unroll *u, const pdlp_params *params, int64_t K, int32_t ckpt, double *x,
             Mem mem) {
    {
        if (!u) invalid("unroll is NULL");
        if (K < 0 || ckpt < 1) invalid("need K >= 0 and ckpt >= 1");
        pdlp_params prm;
        pdlp_params_default(&prm);
        if (params) prm = *params;
        check_params(prm);
        if (prm.restart_period > 0) invalid("the Algorithm 5 mode is not available for unrolling");
        const double t0 = now_s();
        const int B = u->b->B;
        const int64_t N = u->N, M = u->M;
        u->recorded = false;
        delete u->tape_arena;
        u->tape_arena = new Arena();
        Arena &ta = *u->tape_arena;
        BatchRecord &rec = u->rec;
        rec.K = K;
        rec.ckpt = ckpt;
        rec.nck = K > 0 ? (int32_t)((K - 1) / ckpt + 1) : 1;
        rec.eta = ta.dev<double>((size_t)B * K);
        rec.omega = ta.dev<double>((size_t)B * K);
        rec.ck = ta.dev<double>((size_t)rec.nck * 2 * (size_t)(N + M));
        rec.rtype.assign((size_t)B * K, 0);
        batch_record(u->b, prm, rec);
        // host copies of the decisions, sums of step sizes, restart lists
        u->eta_h.assign((size_t)B * K, 0.0);
        u->omega_h.assign((size_t)B * K, 0.0);
        if (K > 0) {
            HIPCHECK(hipMemcpy(u->eta_h.data(), rec.eta, sizeof(double) * B * K,
                               hipMemcpyDeviceToHost));
            HIPCHECK(hipMemcpy(u->omega_h.data(), rec.omega, sizeof(double) * B * K,
                               hipMemcpyDeviceToHost));
        }
        u->seta_h.assign((size_t)B * K, 0.0);
        u->rst.assign(K, {});
        int64_t nrst = 0;
        for (int i = 0; i < B; ++i) {
            double S = 0.0;
            for (int64_t s = 0; s < K; ++s) {
                const size_t q = (size_t)i * K + s;
                S += u->eta_h[q];
                u->seta_h[q] = S;
                if (rec.rtype[q]) {
                    u->rst[s].push_back({i, rec.rtype[q]});
                    S = 0.0;
                    ++nrst;
                }
            }
        }
        ensure_work(u, ckpt);
        const pdlp_problem *P = u->b->P;
        HIPCHECK(pdlp::launch_scale_mul(stream_of(u), N, batch_current_x(u->b), P->d2, u->tmp_n));
        sync(u);
        u->stats.K = K;
        u->stats.ckpt = ckpt;
        u->stats.restarts = nrst;
        u->stats.forward_seconds = now_s() - t0;
        copy_out(u, x, u->tmp_n, N, mem);
        sync(u);
        u->recorded = true;
    }
}

void backward(pdlp_unroll *u, const double *gx, double *gc, double *glc, double *guc,
              double *gval, Mem mem);

}  // namespace

extern "C" {

int pdlp_unroll_forward(pdlp_unroll *u, const pdlp_params *params, int64_t K, int32_t ckpt,
                        double *x) {
    return guarded([&] { forward(u, params, K, ckpt, x, Mem::host); });
}

int pdlp_unroll_forward_device(pdlp_unroll *u, const pdlp_params *params, int64_t K,
                               int32_t ckpt, double *x, void *hip_stream) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        join_caller(u, static_cast<hipStream_t>(hip_stream));
        forward(u, params, K, ckpt, x, Mem::device);
    });
}

int pdlp_unroll_backward(pdlp_unroll *u, const double *gx, double *gc, double *glc, double *guc,
                         double *gval) {
    return guarded([&] { backward(u, gx, gc, glc, guc, gval, Mem::host); });
}

int pdlp_unroll_backward_device(pdlp_unroll *u, const double *gx, double *gc, double *glc,
                                double *guc, double *gval, void *hip_stream) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        join_caller(u, static_cast<hipStream_t>(hip_stream));
        backward(u, gx, gc, glc, guc, gval, Mem::device);
    });
}

int pdlp_unroll_replay(pdlp_unroll *u, double *x, int64_t *signature) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        if (!u->recorded) invalid("no recorded forward pass");
        const double t0 = now_s();
        const int B = u->b->B;
        hipStream_t st = stream_of(u);
        HIPCHECK(hipMemsetAsync(u->sig_d, 0, sizeof(unsigned long long) * B, st));
        replay_from_start(u);
        replay_steps(u, 0, u->rec.K, false, u->sig_d);
        HIPCHECK(pdlp::launch_scale_mul(st, u->N, u->rx, u->b->P->d2, u->tmp_n));
        sync(u);
        u->stats.replay_seconds = now_s() - t0;
        download(u, x, u->tmp_n, u->N);
        HIPCHECK(hipMemcpyAsync(u->sig_h, u->sig_d, sizeof(unsigned long long) * B,
                                hipMemcpyDeviceToHost, st));
        sync(u);
        if (signature)
            for (int i = 0; i < B; ++i) signature[i] = (int64_t)u->sig_h[i];
    });
}

}  // extern "C"

namespace {

void backward(pdlp_unroll *u, const double *gx, double *gc, double *glc, double *guc,
              double *gval, Mem mem) {
    {
        if (!u || !gx) invalid("NULL argument");
        if (!u->recorded) invalid("no recorded forward pass");
        const pdlp_problem *P = u->b->P;
        hipStream_t st = stream_of(u);
        const int64_t N = u->N, M = u->M, K = u->rec.K;
        const int32_t ck = u->rec.ckpt;
        const int B = u->b->B;
        copy_in(u, u->gx_d, gx, N, mem);
        sync(u);
        const double t0 = now_s();
        double t_replay = 0.0, t_rev = 0.0;
        HIPCHECK(pdlp::launch_scale_mul(st, N, u->gx_d, P->d2, u->xb));
        double *zn[] = {u->sxb, u->gc};
        for (auto p : zn) HIPCHECK(pdlp::launch_fill(st, N, p, 0.0));
        double *zm[] = {u->yb, u->syb, u->glc, u->guc};
        for (auto p : zm) HIPCHECK(pdlp::launch_fill(st, M, p, 0.0));
        HIPCHECK(pdlp::launch_fill(st, u->NZ, u->gval, 0.0));
        const int64_t nseg = K > 0 ? (K - 1) / ck + 1 : 0;
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t s0 = seg * ck, s1 = std::min<int64_t>(K, s0 + ck);
            const double ta = now_s();
            replay_from_checkpoint(u, seg);
            replay_steps(u, s0, s1, true, nullptr);
            sync(u);
            const double tb = now_s();
            for (int64_t s = s1 - 1; s >= s0; --s) {
                if (!u->rst[s].empty()) {
                    for (int i = 0; i < B; ++i) u->rt_h[i] = 0;
                    for (auto &e : u->rst[s]) {
                        u->rt_h[e.first] = e.second;
                        u->sv_h[e.first] = u->seta_h[(size_t)e.first * K + s];
                    }
                    upload_i32(u, u->rt_d, u->rt_h);
                    HIPCHECK(hipMemcpyAsync(u->sv_d, u->sv_h, sizeof(double) * B,
                                            hipMemcpyHostToDevice, st));
                    HIPCHECK(pdlp::launch_u_restart_adj(st, P->A, P->AT, u->all, u->rt_d, u->sv_d,
                                                        u->xb, u->yb, u->sxb, u->syb));
                    sync(u);  // staging arrays are rewritten at the next restart
                }
                const size_t o = (size_t)(s - s0);
                HIPCHECK(pdlp::launch_u_reverse(st, P->A, P->AT, step_args(u, s), u->seg_w + o * N,
                                                u->seg_y + o * M, u->seg_p + o * N,
                                                u->seg_q + o * M, u->xb, u->yb, u->sxb, u->syb,
                                                u->yhb, u->vb, u->gc, u->glc, u->guc, u->gval));
            }
            sync(u);
            t_replay += tb - ta;
            t_rev += now_s() - tb;
        }
        HIPCHECK(pdlp::launch_u_finish(st, P->A, N, P->d1, P->d2, P->lc, P->uc, u->gc, u->glc,
                                       u->guc, u->gval, u->oc, u->olc, u->ouc, u->oval));
        sync(u);
        u->stats.backward_seconds = now_s() - t0;
        u->stats.backward_replay_seconds = t_replay;
        u->stats.backward_reverse_seconds = t_rev;
        copy_out(u, gc, u->oc, N, mem);
        copy_out(u, glc, u->olc, M, mem);
        copy_out(u, guc, u->ouc, M, mem);
        copy_out(u, gval, u->oval, u->NZ, mem);
        sync(u);
    }
}

}  // namespace

extern "C" {


int pdlp_unroll_get_tape(const pdlp_unroll *u, double *eta, double *omega, int32_t *restart) {
    return guarded([&] {
        if (!u) invalid("unroll is NULL");
        if (!u->recorded) invalid("no recorded forward pass");
        const size_t n = u->eta_h.size();
        if (eta) std::memcpy(eta, u->eta_h.data(), sizeof(double) * n);
        if (omega) std::memcpy(omega, u->omega_h.data(), sizeof(double) * n);
        if (restart) std::memcpy(restart, u->rec.rtype.data(), sizeof(int32_t) * n);
    });
}

int pdlp_unroll_get_stats(const pdlp_unroll *u, pdlp_unroll_stats *stats) {
    return guarded([&] {
        if (!u || !stats) invalid("NULL argument");
        *stats = u->stats;
    });
}

}  // extern "C"
