// Batched PDLP: many independent LPs solved together on one device.
//
// The instances are packed block-diagonally into one problem (rows and
// columns in instance order, caller labels kept), so Ruiz and Pock-Chambolle
// scaling, which act per row and per column, are exactly those of each
// instance alone.  Each instance has its own device control block: step
// size, primal weight, counters and the accept/reject flags of Algorithm 2.
// One launch of each step kernel serves every instance; a row block belongs
// to one instance, reads that instance's control block and skips itself when
// the instance is idle, finished or has reached its block target.
//
// The host runs Algorithm 1 per instance at the boundaries of iteration
// blocks.  In one round every unfinished instance runs to its own next
// boundary (next multiple of the check cadence, the first count where
// restart condition (iii) holds, or the iteration cap); the round ends when
// all have arrived.  The checks of the round (average, normalized duality
// gaps, termination, restart with the primal-weight update) then run for all
// instances at once with per-instance masks.  Decisions, counters and
// readings are those of the single-LP driver; feasibility polishing and warm
// starts are not offered for batches.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "pdlp_batch.h"

using namespace pdlp::host;
using pdlp::BatchMaps;
using pdlp::Ctrl;
using pdlp::DCsr;
using pdlp::GapState;
using pdlp::Iter;
using pdlp::Vecs;

namespace {

// Active-set steps per normalized-duality-gap evaluation (at most), enqueued
// in chunks; the host stops once every evaluation of the launch has converged.
constexpr int kBatchGapSteps = 32;
constexpr int kBatchGapChunk = 6;
// XCDs of the device: workgroup w of a launch runs on XCD w mod kXcds.
constexpr int kXcds = 8;

}  // namespace

// Device buffers of a batch solve, sized by the packed problem.
struct pdlp::host::BatchWork {
    Arena arena;
    Iter it{};
    double *x0, *y0, *xb, *yb, *axb, *atyb, *xp, *yp, *xo, *yo, *ro;
    double *cx, *cy, *cax, *caty;  // infeasibility candidate and its products
    Ctrl *ctrl_d, *ctrl_h;
    double *part_dual, *part_ps, *part_pf, *part_chk;
    GapState *gs_d, *gs_h;
    double *out_d, *out_h;
    int32_t *mask_d, *mask_h;  // kMasks arrays of B
    int32_t *sel_d, *sel_h;
    double *sv_d, *sv_h, *om_d, *om_h, *zero_d;
    int32_t *list_d, *list_h;  // ilist | alist | tlist | clist of the running instances
    int32_t *slot_d, *slot_h;  // checkpoint slot per instance (-1: none) of a recorded run
};

pdlp_batch::~pdlp_batch() {
    delete W;
    delete P;
}

namespace {

enum { MASK_CHK = 0, MASK_KKT, MASK_RST, MASK_RST_AVG, MASK_INF, kMasks };
// per-instance values pulled at once: 7 of the termination test, or
// kCertVals for each of the three infeasibility candidates
constexpr int kOutVals = 3 * pdlp::kCertVals > 7 ? 3 * pdlp::kCertVals : 7;

BatchWork *make_work(pdlp_batch *b) {
    pdlp_problem *P = b->P;
    const int64_t M = P->m, N = P->n;
    const int B = b->B;
    const int ncb = b->bm.nA + b->bm.nT;
    auto *W = new BatchWork();
    try {
        Arena &a = W->arena;
        for (int k = 0; k < 2; ++k) {
            W->it.X[k] = a.dev<double>(N);
            W->it.ATY[k] = a.dev<double>(N);
            W->it.Y[k] = a.dev<double>(M);
            W->it.AX[k] = a.dev<double>(M);
        }
        W->it.sx = a.dev<double>(N);
        W->it.sy = a.dev<double>(M);
        double **vn[] = {&W->x0, &W->xb, &W->atyb, &W->xp, &W->xo, &W->ro, &W->cx, &W->caty};
        for (auto p : vn) *p = a.dev<double>(N);
        double **vm[] = {&W->y0, &W->yb, &W->axb, &W->yp, &W->yo, &W->cy, &W->cax};
        for (auto p : vm) *p = a.dev<double>(M);
        W->ctrl_d = a.dev<Ctrl>(B);
        W->ctrl_h = a.host<Ctrl>(B);
        W->part_dual = a.dev<double>(2 * (size_t)std::max(b->bm.nA, 1));
        W->part_ps = a.dev<double>(std::max(b->bm.nT, 1));
        W->part_pf = a.dev<double>(std::max(b->bm.nT, 1));
        W->part_chk = a.dev<double>(7 * (size_t)std::max(ncb, 1));
        W->gs_d = a.dev<GapState>(3 * (size_t)B);
        W->gs_h = a.host<GapState>(3 * (size_t)B);
        W->out_d = a.dev<double>(kOutVals * (size_t)B);
        W->out_h = a.host<double>(kOutVals * (size_t)B);
        W->mask_d = a.dev<int32_t>(kMasks * (size_t)B);
        W->mask_h = a.host<int32_t>(kMasks * (size_t)B);
        W->sel_d = a.dev<int32_t>(B);
        W->sel_h = a.host<int32_t>(B);
        W->sv_d = a.dev<double>(B);
        W->sv_h = a.host<double>(B);
        W->om_d = a.dev<double>(B);
        W->om_h = a.host<double>(B);
        W->zero_d = a.dev<double>(B);
        // instance list + per-XCD interleaved block lists (padding at most kXcds-fold)
        const size_t nl = (size_t)B + 2 * (size_t)kXcds * ((size_t)b->bm.nA + b->bm.nT);
        W->list_d = a.dev<int32_t>(nl);
        W->list_h = a.host<int32_t>(nl);
        W->slot_d = a.dev<int32_t>(B);
        W->slot_h = a.host<int32_t>(B);
        HIPCHECK(pdlp::launch_fill(P->stream, B, W->zero_d, 0.0));
        HIPCHECK(hipStreamSynchronize(P->stream));
    } catch (...) {
        delete W;
        throw;
    }
    return W;
}

// Per-instance solver state kept on the host.
struct Inst {
    int status = -1;  // -1 while running, else a PDLP_STATUS_* value
    long long n_outer = 0, kkt_passes = 1, r_i = 0, r_ii = 0, r_iii = 0;
    double mu_ref = INFINITY, mu_c_prev = INFINITY;
    bool have = false;  // a candidate has been evaluated for termination
    int out_sel = 0;    // its buffers: 0 current iterate, 1 average
    // flags of the current round
    bool full = false, art = false, capchk = false, chk = false, use_cur = false;
    int cert_src = 0;   // infeasibility certificate: candidate 1..3
    pdlp::CertOut cert{};
    double mu_c = 0.0;
};

struct KktHost {
    double pres_abs, pres_rel, dres_abs, dres_rel, pobj, dobj, gap;
};

KktHost kkt_from(const double *v, double off) {
    KktHost k;
    k.pres_abs = v[0];
    k.pres_rel = v[1];
    k.dres_abs = v[2];
    k.dres_rel = v[3];
    k.pobj = v[4] + off;
    k.dobj = v[5] + off;
    const double den = std::fabs(k.pobj) + std::fabs(k.dobj);
    k.gap = den > 0.0 ? std::fabs(k.pobj - k.dobj) / den : 0.0;
    if (v[6] > 0.0) k.gap = NAN;
    return k;
}

bool met(const pdlp_params &prm, const KktHost &k) {
    return k.pres_rel <= prm.eps_feas && k.dres_rel <= prm.eps_feas && k.gap <= prm.eps_gap;
}

class BatchSolver {
  public:
    BatchSolver(pdlp_batch *b, const pdlp_params &prm, BatchRecord *rec = nullptr)
        : b_(b), P_(b->P), W_(*b->W), prm_(prm), rec_(rec) {}

    // Exactly K accepted steps per instance with restart checks and no
    // termination test (the loop of pdlp_iterate_k), recording the decisions.
    void run_record() {
        const long long K = rec_->K;
        init();
        take_checkpoints(true);
        for (auto &st : inst_)
            if (K == 0) st.status = PDLP_STATUS_ITERATION_LIMIT;
        while (any_running()) {
            set_active(false);
            run_round(K);
            for (int i = 0; i < B(); ++i)
                if (inst_[i].status == PDLP_STATUS_NUMERICAL_ERROR)
                    throw LibError(PDLP_ERR_STATE, "numerical error in instance " +
                                                       std::to_string(i) + " at step " +
                                                       std::to_string(W_.ctrl_h[i].k));
            check_round(K);
            take_checkpoints(false);
            for (int i = 0; i < B(); ++i) {
                if (inst_[i].status == PDLP_STATUS_NUMERICAL_ERROR)
                    throw LibError(PDLP_ERR_STATE,
                                   "numerical error in instance " + std::to_string(i));
                if (inst_[i].status < 0 && W_.ctrl_h[i].k >= K)
                    inst_[i].status = PDLP_STATUS_ITERATION_LIMIT;
            }
        }
    }

    void run(pdlp_result *res, double *x_host, double *y_host, double *r_host) {
        const double t0 = now_s();
        rc_mode_ = prm_.reduced_cost_mode >= 0 ? prm_.reduced_cost_mode : 1;
        init();
        const double t_setup = now_s() - t0;
        const long long max_k = prm_.max_iters;
        // termination check at k = 0
        for (int i = 0; i < B(); ++i) mask(MASK_KKT)[i] = 1, W_.sel_h[i] = 0;
        eval_kkt();
        for (int i = 0; i < B(); ++i) {
            inst_[i].have = true;
            inst_[i].out_sel = 0;
            if (met(prm_, kkt_[i])) inst_[i].status = PDLP_STATUS_OPTIMAL;
            else if (max_k == 0) inst_[i].status = PDLP_STATUS_ITERATION_LIMIT;
        }
        pdlp_batch_stats &st = b_->stats;
        std::memset(&st, 0, sizeof st);
        st.setup_seconds = t_setup;
        while (any_running()) {
            if (now_s() - t0 >= prm_.time_limit) {
                for (auto &s : inst_)
                    if (s.status < 0) s.status = PDLP_STATUS_TIME_LIMIT;
                break;
            }
            set_active(false);
            const double ta = now_s();
            run_round(max_k);
            const double tb = now_s();
            check_round(max_k);
            st.rounds += 1;
            st.step_seconds += tb - ta;
            st.check_seconds += now_s() - tb;
        }
        finish(res, x_host, y_host, r_host, now_s() - t0, t_setup);
        for (int i = 0; i < B(); ++i) {
            st.max_iterations = std::max<int64_t>(st.max_iterations, res[i].iterations);
            st.total_iterations += res[i].iterations;
        }
        st.seconds = now_s() - t0;
    }

  private:
    pdlp_batch *b_;
    pdlp_problem *P_;
    BatchWork &W_;
    pdlp_params prm_;
    BatchRecord *rec_ = nullptr;

    // Checkpoints of a recorded run: every running instance whose step count
    // is a multiple of the cadence (and below K) stores its state, after the
    // restart of that boundary; at the start (all = true) every instance.
    void take_checkpoints(bool all) {
        if (!rec_) return;
        bool any = false;
        for (int i = 0; i < B(); ++i) {
            const long long k = W_.ctrl_h[i].k;
            const bool due = all || (inst_[i].status < 0 && k > 0 && k < rec_->K &&
                                     k % rec_->ckpt == 0);
            W_.slot_h[i] = due ? (int32_t)(k / rec_->ckpt) : -1;
            any = any || due;
        }
        if (!any) return;
        HIPCHECK(hipMemcpyAsync(W_.slot_d, W_.slot_h, sizeof(int32_t) * B(),
                                hipMemcpyHostToDevice, s()));
        HIPCHECK(pdlp::launch_b_checkpoint(s(), P_->A, P_->AT, bm_, W_.slot_d, W_.it.X[0],
                                           W_.it.Y[0], W_.it.sx, W_.it.sy, rec_->ck, P_->n,
                                           P_->m));
        sync();
    }
    int rc_mode_ = 1;
    std::vector<Inst> inst_;
    std::vector<KktHost> kkt_;
    BatchMaps bm_;       // maps with the lists of the instances launches serve
    int listed_ = -1;    // running instances when the lists were built (-1: all)
    // Step attempts replayed from graphs once the running set has stayed the
    // same for two rounds (capturing for sets that change every round costs
    // more than it saves).
    pdlp::host::AttemptGraphs graphs_;
    int rounds_on_lists_ = 0;

    // Lists of the instances the launches serve and of their blocks: every
    // instance (all = true) or the running ones.  Rebuilt when that set
    // changes.  With at least kXcds instances, each is assigned to one XCD
    // (greedy by block count) and the block lists are interleaved so that
    // position p of a list serves an instance of XCD p mod kXcds (padding -1).
    void set_active(bool all) {
        int running = 0;
        for (const auto &st : inst_) running += st.status < 0;
        const int want = all ? -1 : running;
        if (want == listed_ && bm_.ilist) return;
        const BatchMaps &base = b_->bm;
        const int B = b_->B, nT = base.nT;
        const std::vector<int32_t> &ao = b_->aoff, &to = b_->toff;
        std::vector<int32_t> il;
        for (int i = 0; i < B; ++i)
            if (all || inst_[i].status < 0) il.push_back(i);
        const int nx = (int)il.size() >= kXcds ? kXcds : 1;
        // instance -> XCD, heaviest first onto the least loaded XCD
        std::vector<int32_t> order(il);
        auto nblk = [&](int i) { return (ao[i + 1] - ao[i]) + (to[i + 1] - to[i]); };
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return nblk(a) > nblk(b); });
        std::vector<std::vector<int32_t>> sub_a(nx), sub_t(nx), sub_c(nx);
        std::vector<long long> load(nx, 0);
        for (int i : order) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[k] += nblk(i);
            for (int q = ao[i]; q < ao[i + 1]; ++q) sub_a[k].push_back(q);
            for (int q = to[i]; q < to[i + 1]; ++q) sub_t[k].push_back(q);
            for (int q = to[i]; q < to[i + 1]; ++q) sub_c[k].push_back(q);
            for (int q = ao[i]; q < ao[i + 1]; ++q) sub_c[k].push_back(nT + q);
        }
        auto interleave = [&](const std::vector<std::vector<int32_t>> &sub, int32_t *dst) {
            size_t mx = 0;
            for (const auto &v : sub) mx = std::max(mx, v.size());
            size_t len = 0;
            for (size_t t = 0; t < mx; ++t)
                for (int k = 0; k < nx; ++k) {
                    const int32_t e = t < sub[k].size() ? sub[k][t] : -1;
                    dst[t * nx + k] = e;
                    if (e >= 0) len = t * nx + k + 1;
                }
            return (int32_t)len;
        };
        int32_t *h = W_.list_h;
        const size_t oi = 0, oa = (size_t)B, ot = oa + (size_t)kXcds * base.nA,
                     oc = ot + (size_t)kXcds * nT;
        std::copy(il.begin(), il.end(), h + oi);
        const int32_t na = interleave(sub_a, h + oa);
        const int32_t nt = interleave(sub_t, h + ot);
        const int32_t nc = interleave(sub_c, h + oc);
        const size_t off[4] = {oi, oa, ot, oc};
        const size_t len[4] = {il.size(), (size_t)na, (size_t)nt, (size_t)nc};
        for (int q = 0; q < 4; ++q)
            if (len[q] > 0)
                HIPCHECK(hipMemcpyAsync(W_.list_d + off[q], W_.list_h + off[q],
                                        sizeof(int32_t) * len[q], hipMemcpyHostToDevice, s()));
        sync();
        bm_ = base;
        if (rec_) {
            bm_.tape_eta = rec_->eta;
            bm_.tape_omega = rec_->omega;
            bm_.tape_K = rec_->K;
        }
        bm_.ni = (int32_t)il.size();
        bm_.na = na;
        bm_.nt = nt;
        bm_.nc = nc;
        bm_.ilist = W_.list_d + oi;
        bm_.alist = W_.list_d + oa;
        bm_.tlist = W_.list_d + ot;
        bm_.clist = W_.list_d + oc;
        listed_ = want;
        graphs_.reset();       // the captured launches carry the old list sizes
        rounds_on_lists_ = 0;
    }

    // Normalized duality gaps of up to three evaluations (slots of gs) for the
    // instances of mask; the active-set steps run in chunks until all converged.
    struct GapArgs {
        const double *x, *y, *ax, *aty, *xr, *yr;
        int slot;
    };
    void gaps(const GapArgs *g, int ng, int mask_k) {
        const Vecs v = P_->scaled();
        const int32_t *md = mask_dev(mask_k);
        for (int q = 0; q < ng; ++q)
            HIPCHECK(pdlp::launch_b_gap_begin(s(), P_->A, P_->AT, bm_, md, v, g[q].x, g[q].y,
                                              g[q].ax, g[q].aty, g[q].xr, g[q].yr, W_.om_d,
                                              W_.part_chk, W_.gs_d + (size_t)g[q].slot * B()));
        for (int first = 0; first < kBatchGapSteps; first += kBatchGapChunk) {
            for (int q = 0; q < ng; ++q)
                HIPCHECK(pdlp::launch_b_gap_steps(s(), P_->A, P_->AT, bm_, md, v, g[q].x, g[q].y,
                                                  g[q].ax, g[q].aty, W_.part_chk,
                                                  W_.gs_d + (size_t)g[q].slot * B(), first,
                                                  kBatchGapChunk, kBatchGapSteps));
            pull_gaps(g[0].slot, g[ng - 1].slot - g[0].slot + 1);
            bool open = false;
            for (int q = 0; q < ng && !open; ++q)
                for (int i = 0; i < B() && !open; ++i)
                    open = mask(mask_k)[i] && W_.gs_h[(size_t)g[q].slot * B() + i].done == 0;
            if (!open) break;
        }
        pdlp_batch_stats &st = b_->stats;
        for (int q = 0; q < ng; ++q)
            for (int i = 0; i < B(); ++i) {
                if (!mask(mask_k)[i]) continue;
                const GapState &gsi = W_.gs_h[(size_t)g[q].slot * B() + i];
                st.gap_evals += 1;
                st.gap_steps += gsi.nsteps;
                st.gap_capped += gsi.nsteps > 0 && !gsi.exact;
            }
    }

    int B() const { return b_->B; }
    hipStream_t s() const { return P_->stream; }
    int32_t *mask(int k) const { return W_.mask_h + (size_t)k * b_->B; }
    const int32_t *mask_dev(int k) const { return W_.mask_d + (size_t)k * b_->B; }
    bool any_running() const {
        for (const auto &s : inst_)
            if (s.status < 0) return true;
        return false;
    }
    const double *X() const { return W_.it.X[0]; }
    const double *Y() const { return W_.it.Y[0]; }

    void sync() { HIPCHECK(hipStreamSynchronize(s())); }
    void push_ctrl() {
        HIPCHECK(hipMemcpyAsync(W_.ctrl_d, W_.ctrl_h, sizeof(Ctrl) * B(), hipMemcpyHostToDevice,
                                s()));
        sync();
    }
    void pull_ctrl() {
        HIPCHECK(hipMemcpyAsync(W_.ctrl_h, W_.ctrl_d, sizeof(Ctrl) * B(), hipMemcpyDeviceToHost,
                                s()));
        sync();
    }
    void push_masks() {
        HIPCHECK(hipMemcpyAsync(W_.mask_d, W_.mask_h, sizeof(int32_t) * kMasks * B(),
                                hipMemcpyHostToDevice, s()));
        HIPCHECK(hipMemcpyAsync(W_.sel_d, W_.sel_h, sizeof(int32_t) * B(), hipMemcpyHostToDevice,
                                s()));
        sync();
    }
    void push_doubles(double *d, const double *h) {
        HIPCHECK(hipMemcpyAsync(d, h, sizeof(double) * B(), hipMemcpyHostToDevice, s()));
        sync();
    }
    void pull_out(int nv) {
        HIPCHECK(hipMemcpyAsync(W_.out_h, W_.out_d, sizeof(double) * nv * B(),
                                hipMemcpyDeviceToHost, s()));
        sync();
    }
    void pull_gaps(int first_slot, int slots) {
        const size_t o = (size_t)first_slot * B();
        HIPCHECK(hipMemcpyAsync(W_.gs_h + o, W_.gs_d + o, sizeof(GapState) * slots * B(),
                                hipMemcpyDeviceToHost, s()));
        sync();
    }

    // Algorithm 1 initialization per instance (the single-LP readings:
    // eta_hat = 1 / max |scaled A entry|, omega = ||c|| / ||Combine(lc, uc)||,
    // x = proj_X(0), y = 0).
    void init() {
        const Vecs v = P_->scaled();
        inst_.assign(B(), Inst());
        kkt_.assign(B(), KktHost{});
        listed_ = -2;
        set_active(true);
        const BatchMaps &bm = bm_;
        HIPCHECK(pdlp::launch_b_norms(s(), P_->A, P_->AT, bm, nullptr, 3, nullptr, nullptr, nullptr,
                                      nullptr, v, W_.part_chk, 1u, W_.out_d));
        pull_out(2);
        std::vector<double> amax(B());
        for (int i = 0; i < B(); ++i) amax[i] = W_.out_h[2 * i];
        HIPCHECK(pdlp::launch_b_norms(s(), P_->A, P_->AT, bm, nullptr, 2, nullptr, nullptr, nullptr,
                                      nullptr, v, W_.part_chk, 0u, W_.out_d));
        pull_out(2);
        std::memset(W_.ctrl_h, 0, sizeof(Ctrl) * B());
        for (int i = 0; i < B(); ++i) {
            const double nc = std::sqrt(W_.out_h[2 * i]), nb = std::sqrt(W_.out_h[2 * i + 1]);
            Ctrl &c = W_.ctrl_h[i];
            c.omega = (nc > 0.0 && nb > 0.0) ? nc / nb : 1.0;
            c.eta = c.eta_hat = amax[i] > 0.0 ? 1.0 / amax[i] : 1.0;
            c.red_exp = prm_.red_exp;
            c.grow_exp = prm_.grow_exp;
            c.need_primal = 1;
        }
        const int64_t M = P_->m, N = P_->n;
        HIPCHECK(pdlp::launch_clamp0(s(), (int)N, P_->lvs, P_->uvs, W_.it.X[0]));
        HIPCHECK(pdlp::launch_fill(s(), M, W_.it.Y[0], 0.0));
        HIPCHECK(pdlp::launch_spmv_plain(s(), P_->A, W_.it.X[0], W_.it.AX[0]));
        HIPCHECK(pdlp::launch_spmv_plain(s(), P_->AT, W_.it.Y[0], W_.it.ATY[0]));
        HIPCHECK(pdlp::launch_copy(s(), N, W_.it.X[0], W_.x0));
        HIPCHECK(pdlp::launch_copy(s(), M, W_.it.Y[0], W_.y0));
        HIPCHECK(pdlp::launch_fill(s(), N, W_.it.sx, 0.0));
        HIPCHECK(pdlp::launch_fill(s(), M, W_.it.sy, 0.0));
        sync();
    }

    // Termination sums for the instances of MASK_KKT at the points chosen by sel.
    void eval_kkt() {
        push_masks();
        const double *p0[4] = {W_.it.X[0], W_.it.Y[0], W_.it.AX[0], W_.it.ATY[0]};
        const double *p1[4] = {W_.xb, W_.yb, W_.axb, W_.atyb};
        const Vecs orig{P_->c, P_->lc, P_->uc, P_->lv, P_->uv};
        HIPCHECK(pdlp::launch_b_kkt(s(), P_->A, P_->AT, bm_, mask_dev(MASK_KKT), W_.sel_d, p0, p1,
                                    P_->d1, P_->d2, orig, rc_mode_, W_.part_chk, W_.out_d, nullptr,
                                    nullptr, nullptr));
        pull_out(7);
        for (int i = 0; i < B(); ++i)
            if (mask(MASK_KKT)[i]) kkt_[i] = kkt_from(W_.out_h + 7 * i, b_->obj_offset[i]);
    }

    // Every running instance advances to its next block boundary.
    void run_round(long long max_k) {
        const long long ce = prm_.check_every;
        long long rem = 0;
        for (int i = 0; i < B(); ++i) {
            Ctrl &c = W_.ctrl_h[i];
            c.block_acc = 0;
            c.run_at = 0;
            c.cur = 0;
            c.pending_sy = 0;
            if (inst_[i].status >= 0) {
                c.block_target = 0;
                c.stop = 1;
                c.need_primal = 0;
                continue;
            }
            long long kb = (c.k / ce + 1) * ce;
            if (rec_) kb = std::min<long long>(kb, (c.k / rec_->ckpt + 1) * rec_->ckpt);
            kb = std::min(kb, next_art(c.k, c.t, prm_.beta_art, max_k));
            kb = std::min(kb, max_k);
            c.block_target = kb - c.k;
            c.stop = 0;
            c.need_primal = 1;
            rem = std::max(rem, c.block_target);
        }
        push_ctrl();
        const BatchMaps &bm = bm_;
        const Vecs v = P_->scaled();
        auto attempt = [&](hipStream_t st) {
            HIPCHECK(pdlp::launch_b_attempt(st, P_->A, P_->AT, v, W_.it, W_.ctrl_d, bm,
                                            W_.part_dual, W_.part_ps, W_.part_pf));
        };
        const bool use_graphs = prm_.graphs && ++rounds_on_lists_ > 2;
        if (use_graphs && !graphs_.ready()) graphs_.capture(attempt);
        // primal candidates of the first attempt (later ones come from the products)
        HIPCHECK(pdlp::launch_b_primal(s(), P_->AT, v, W_.it, W_.ctrl_d, bm,
                                       W_.part_ps));
        long long tried = 0;
        for (int i = 0; i < B(); ++i) tried += W_.ctrl_h[i].attempts;
        while (rem > 0) {
            long long n_att = rem + rem / 8 + 1;
            if (n_att > 4096) n_att = 4096;
            b_->stats.attempt_launches += n_att;
            if (use_graphs)
                graphs_.launch(s(), n_att);
            else
                for (long long a = 0; a < n_att; ++a) attempt(s());
            pull_ctrl();
            rem = 0;
            long long now = 0;
            for (int i = 0; i < B(); ++i) {
                const Ctrl &c = W_.ctrl_h[i];
                now += c.attempts;
                if (inst_[i].status < 0 && !c.stop) rem = std::max(rem, c.block_target - c.block_acc);
            }
            // every launched attempt decides each running instance once
            if (rem > 0 && now == tried)
                throw LibError(PDLP_ERR_STATE, "batched step attempts made no decision");
            tried = now;
            if (rem == 0) {
                // instances still running with nothing left cannot exist: stop is set
                // exactly when block_acc reaches the target
                break;
            }
        }
        HIPCHECK(pdlp::launch_b_settle(s(), P_->A, P_->AT, W_.it, W_.ctrl_d, bm));
        sync();
        for (int i = 0; i < B(); ++i) {
            Ctrl &c = W_.ctrl_h[i];
            c.cur = 0;
            c.pending_sy = 0;
            if (inst_[i].status >= 0) continue;
            inst_[i].kkt_passes += c.block_acc;
            if (c.numerr) inst_[i].status = PDLP_STATUS_NUMERICAL_ERROR;
        }
    }

    // Periodic checks of Section 3 for the instances at a boundary.
    // Infeasibility candidate c (0 difference of the current and previous
    // iterate, 1 current iterate, 2 average) of the instances in mask mk,
    // projected onto Xbar x Y, with its products.
    struct CertPoint {
        const double *px, *py, *pax, *paty;
    };
    // When no instance of the mask has a variable with an infinite bound
    // (Xbar = {0}), the x part and its product are skipped: null pointers
    // read as zeros.
    CertPoint cert_point(int c, const int32_t *mk, bool xs) {
        const BatchMaps &bm = bm_;
        const Vecs orig{P_->c, P_->lc, P_->uc, P_->lv, P_->uv};
        double *px = xs ? W_.cx : nullptr, *pax = xs ? W_.cax : nullptr;
        if (xs || c == 0)
            HIPCHECK(pdlp::launch_b_cert_point(s(), P_->A, P_->AT, bm, mk, c, W_.it, W_.xb, orig,
                                               px, W_.cy));
        if (xs)
            HIPCHECK(pdlp::launch_b_spmv_plain(s(), P_->A, bm.ablk_inst, bm.alist, bm.na, mk,
                                               W_.cx, W_.cax));
        if (c == 0) {
            HIPCHECK(pdlp::launch_b_spmv_plain(s(), P_->AT, bm.tblk_inst, bm.tlist, bm.nt, mk,
                                               W_.cy, W_.caty));
            return {px, W_.cy, pax, W_.caty};
        }
        if (c == 1) return {px, W_.it.Y[0], pax, W_.it.ATY[0]};
        return {px, W_.yb, pax, W_.atyb};
    }
    bool masked_ray_cols(int mk) {
        for (int i = 0; i < B(); ++i)
            if (mask(mk)[i] && b_->ray_cols[i] > 0) return true;
        return false;
    }

    // Appendix D tests on the three candidates of the instances in
    // MASK_INF (the single-LP order: primal infeasibility on each candidate,
    // then dual infeasibility); an instance at its iteration cap that is not
    // declared infeasible stops with ITERATION_LIMIT.
    void detect_infeasible() {
        push_masks();
        const int32_t *mk = mask_dev(MASK_INF);
        const Vecs orig{P_->c, P_->lc, P_->uc, P_->lv, P_->uv};
        const size_t nv = pdlp::kCertVals;
        const bool xs = masked_ray_cols(MASK_INF);
        for (int c = 0; c < 3; ++c) {
            const CertPoint q = cert_point(c, mk, xs);
            HIPCHECK(pdlp::launch_b_cert(s(), P_->A, P_->AT, bm_, mk, q.px, q.py, q.pax, q.paty,
                                         P_->d1, P_->d2, orig, W_.part_chk,
                                         W_.out_d + (size_t)c * nv * B()));
        }
        pull_out(3 * (int)nv);
        const double eps = prm_.eps_infeasible;
        for (int i = 0; i < B(); ++i) {
            if (!mask(MASK_INF)[i]) continue;
            Inst &st = inst_[i];
            st.kkt_passes += 3;
            for (int pass = 0; pass < 2 && st.status < 0; ++pass) {
                for (int c = 0; c < 3; ++c) {
                    const double *v = W_.out_h + ((size_t)c * B() + i) * nv;
                    const pdlp::CertOut o{v[0], v[1], v[2], v[3], v[4]};
                    if (o.nonfinite > 0.0) continue;
                    const bool ok = pass == 0 ? (std::isfinite(o.pobj) && o.pobj > 0.0 &&
                                                 o.pres <= eps * o.pobj)
                                              : (std::isfinite(o.dobj) && o.dobj < 0.0 &&
                                                 o.dres <= eps * std::fabs(o.dobj));
                    if (!ok) continue;
                    st.status = pass == 0 ? PDLP_STATUS_PRIMAL_INFEASIBLE
                                          : PDLP_STATUS_DUAL_INFEASIBLE;
                    st.cert_src = c + 1;
                    st.cert = o;
                    break;
                }
            }
            if (st.status < 0 && st.capchk) st.status = PDLP_STATUS_ITERATION_LIMIT;
            if (st.status >= 0) st.chk = false;
        }
    }

    void check_round(long long max_k) {
        const BatchMaps &bm = bm_;
        const Vecs v = P_->scaled();
        bool any = false;
        for (int i = 0; i < B(); ++i) {
            Inst &st = inst_[i];
            const Ctrl &c = W_.ctrl_h[i];
            st.chk = false;
            for (int k = 0; k < kMasks; ++k) mask(k)[i] = 0;
            if (st.status >= 0) continue;
            st.full = (c.k % prm_.check_every) == 0;
            st.art = (double)c.t >= prm_.beta_art * (double)c.k;
            st.capchk = !rec_ && c.k == max_k;
            st.chk = st.full || st.art || st.capchk;
            mask(MASK_CHK)[i] = st.chk;
            W_.sv_h[i] = c.seta > 0.0 ? c.seta : 1.0;
            W_.om_h[i] = c.omega;
            any = any || st.chk;
        }
        if (!any) return;
        push_masks();
        push_doubles(W_.sv_d, W_.sv_h);
        push_doubles(W_.om_d, W_.om_h);
        const DCsr &A = P_->A, &AT = P_->AT;
        const int32_t *mchk = mask_dev(MASK_CHK);
        // average and its products
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, mchk, 0, W_.sv_d, W_.it.sx, W_.xb,
                                            W_.it.sy, W_.yb));
        HIPCHECK(pdlp::launch_b_spmv_plain(s(), A, bm.ablk_inst, bm.alist, bm.na, mchk, W_.xb,
                                           W_.axb));
        HIPCHECK(pdlp::launch_b_spmv_plain(s(), AT, bm.tblk_inst, bm.tlist, bm.nt, mchk, W_.yb,
                                           W_.atyb));
        // mu(z, z0) and mu(z_bar, z0)
        const GapArgs g2[2] = {
            {W_.it.X[0], W_.it.Y[0], W_.it.AX[0], W_.it.ATY[0], W_.x0, W_.y0, 0},
            {W_.xb, W_.yb, W_.axb, W_.atyb, W_.x0, W_.y0, 1}};
        gaps(g2, 2, MASK_CHK);
        bool any_kkt = false;
        for (int i = 0; i < B(); ++i) {
            Inst &st = inst_[i];
            if (!st.chk) continue;
            st.kkt_passes += 1;
            const double mu_cur = W_.gs_h[i].mu, mu_avg = W_.gs_h[B() + i].mu;
            if (!std::isfinite(mu_cur) || !std::isfinite(mu_avg)) {
                st.status = PDLP_STATUS_NUMERICAL_ERROR;
                st.chk = false;
                continue;
            }
            st.use_cur = mu_cur < mu_avg;  // a tie goes to the average
            st.mu_c = st.use_cur ? mu_cur : mu_avg;
            W_.sel_h[i] = st.use_cur ? 0 : 1;
            if (!rec_ && (st.full || st.capchk)) {
                mask(MASK_KKT)[i] = 1;
                any_kkt = true;
            }
        }
        if (any_kkt) {
            bool any_inf = false;
            eval_kkt();
            for (int i = 0; i < B(); ++i) {
                Inst &st = inst_[i];
                if (!mask(MASK_KKT)[i]) continue;
                st.have = true;
                st.out_sel = W_.sel_h[i];
                if (prm_.verbose)
                    std::fprintf(stderr, "[pdlp batch %d] k=%lld gap=%.2e pres=%.2e dres=%.2e\n", i,
                                 W_.ctrl_h[i].k, kkt_[i].gap, kkt_[i].pres_rel, kkt_[i].dres_rel);
                if (!std::isfinite(kkt_[i].gap)) {
                    st.status = PDLP_STATUS_NUMERICAL_ERROR;
                } else if (met(prm_, kkt_[i])) {
                    st.status = PDLP_STATUS_OPTIMAL;
                } else if (prm_.detect_infeasibility) {
                    mask(MASK_INF)[i] = 1;
                    any_inf = true;
                } else if (st.capchk) {
                    st.status = PDLP_STATUS_ITERATION_LIMIT;
                }
                if (st.status >= 0) st.chk = false;
            }
            if (any_inf) detect_infeasible();
        }
        // restart decisions (criteria (i)-(iii))
        bool any_rst = false;
        for (int i = 0; i < B(); ++i) {
            Inst &st = inst_[i];
            if (!st.chk) continue;
            int why = 0;
            if (!prm_.adaptive_restarts || st.n_outer == 0) {
                if (st.art) why = 3;
            } else {
                if (st.full && st.mu_c <= prm_.beta_suff * st.mu_ref) why = 1;
                else if (st.full && st.mu_c <= prm_.beta_nec * st.mu_ref && st.mu_c > st.mu_c_prev)
                    why = 2;
                else if (st.art) why = 3;
            }
            if (!why) {
                if (st.full) st.mu_c_prev = st.mu_c;
                continue;
            }
            st.r_i += why == 1;
            st.r_ii += why == 2;
            st.r_iii += why == 3;
            if (rec_) {
                const long long k = W_.ctrl_h[i].k;
                if (k >= 1 && k <= rec_->K) rec_->rtype[(size_t)i * rec_->K + (k - 1)] = st.use_cur ? 1 : 2;
            }
            mask(MASK_RST)[i] = 1;
            mask(MASK_RST_AVG)[i] = !st.use_cur;
            any_rst = true;
        }
        if (!any_rst) return;
        push_masks();
        const int32_t *mr = mask_dev(MASK_RST), *ma = mask_dev(MASK_RST_AVG);
        Iter &it = W_.it;
        // z_prev0 = z0; z = z0 = candidate (with its products)
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, mr, 1, nullptr, W_.x0, W_.xp, W_.y0,
                                            W_.yp));
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, ma, 1, nullptr, W_.xb, it.X[0], W_.yb,
                                            it.Y[0]));
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, ma, 1, nullptr, W_.atyb, it.ATY[0],
                                            W_.axb, it.AX[0]));
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, mr, 1, nullptr, it.X[0], W_.x0,
                                            it.Y[0], W_.y0));
        // primal weight update (Algorithm 3)
        HIPCHECK(pdlp::launch_b_norms(s(), A, AT, bm, mr, 0, W_.x0, W_.xp, W_.y0, W_.yp, v,
                                      W_.part_chk, 0u, W_.out_d));
        pull_out(2);
        const double ez = prm_.eps_zero;
        for (int i = 0; i < B(); ++i) {
            if (!mask(MASK_RST)[i]) continue;
            Inst &st = inst_[i];
            Ctrl &c = W_.ctrl_h[i];
            const double dx = std::sqrt(W_.out_h[2 * i]), dy = std::sqrt(W_.out_h[2 * i + 1]);
            if (dx > ez && dx < 1.0 / ez && dy > ez && dy < 1.0 / ez)
                c.omega = std::exp(prm_.theta * std::log(dy / dx) +
                                   (1.0 - prm_.theta) * std::log(c.omega));
            st.n_outer += 1;
            c.t = 0;
            c.seta = 0.0;
            W_.om_h[i] = c.omega;
        }
        push_doubles(W_.om_d, W_.om_h);
        HIPCHECK(pdlp::launch_b_elementwise(s(), A, AT, bm, mr, 2, W_.zero_d, nullptr, it.sx,
                                            nullptr, it.sy));
        // mu_ref = mu(z0, z_prev0) under the new primal weight
        const GapArgs g1[1] = {{W_.x0, W_.y0, it.AX[0], it.ATY[0], W_.xp, W_.yp, 2}};
        gaps(g1, 1, MASK_RST);
        for (int i = 0; i < B(); ++i) {
            if (!mask(MASK_RST)[i]) continue;
            inst_[i].mu_ref = W_.gs_h[2 * (size_t)B() + i].mu;
            inst_[i].mu_c_prev = INFINITY;
        }
    }

    // Final evaluation on each instance's output point, unscaled outputs.
    void finish(pdlp_result *res, double *x_host, double *y_host, double *r_host, double secs,
                double setup) {
        set_active(true);
        for (int i = 0; i < B(); ++i) {
            const Inst &st = inst_[i];
            mask(MASK_KKT)[i] = 1;
            const bool cand = st.have && st.status != PDLP_STATUS_NUMERICAL_ERROR;
            W_.sel_h[i] = cand ? st.out_sel : 0;
        }
        push_masks();
        const double *p0[4] = {W_.it.X[0], W_.it.Y[0], W_.it.AX[0], W_.it.ATY[0]};
        const double *p1[4] = {W_.xb, W_.yb, W_.axb, W_.atyb};
        const Vecs orig{P_->c, P_->lc, P_->uc, P_->lv, P_->uv};
        HIPCHECK(pdlp::launch_b_kkt(s(), P_->A, P_->AT, bm_, mask_dev(MASK_KKT), W_.sel_d, p0,
                                    p1, P_->d1, P_->d2, orig, rc_mode_, W_.part_chk, W_.out_d,
                                    W_.ro, W_.xo, W_.yo));
        pull_out(7);
        std::vector<double> kout(W_.out_h, W_.out_h + 7 * (size_t)B());
        // certificates of the instances declared infeasible replace their outputs
        for (int c = 0; c < 3; ++c) {
            bool any = false;
            for (int i = 0; i < B(); ++i) {
                const Inst &st = inst_[i];
                const bool inf = st.status == PDLP_STATUS_PRIMAL_INFEASIBLE ||
                                 st.status == PDLP_STATUS_DUAL_INFEASIBLE;
                mask(MASK_INF)[i] = inf && st.cert_src == c + 1;
                any = any || mask(MASK_INF)[i];
            }
            if (!any) continue;
            push_masks();
            const int32_t *mk = mask_dev(MASK_INF);
            const CertPoint q = cert_point(c, mk, masked_ray_cols(MASK_INF));
            HIPCHECK(pdlp::launch_b_cert_out(s(), P_->A, P_->AT, bm_, mk, q.px, q.py, q.paty,
                                             P_->d1, P_->d2, orig, W_.xo, W_.yo, W_.ro));
        }
        const int64_t M = P_->m, N = P_->n;
        if (x_host && N > 0)
            HIPCHECK(hipMemcpyAsync(x_host, W_.xo, sizeof(double) * N, hipMemcpyDeviceToHost, s()));
        if (y_host && M > 0)
            HIPCHECK(hipMemcpyAsync(y_host, W_.yo, sizeof(double) * M, hipMemcpyDeviceToHost, s()));
        if (r_host && N > 0)
            HIPCHECK(hipMemcpyAsync(r_host, W_.ro, sizeof(double) * N, hipMemcpyDeviceToHost, s()));
        sync();
        for (int i = 0; i < B(); ++i) {
            const Inst &st = inst_[i];
            const Ctrl &c = W_.ctrl_h[i];
            const KktHost k = kkt_from(kout.data() + 7 * i, b_->obj_offset[i]);
            pdlp_result &r = res[i];
            std::memset(&r, 0, sizeof r);
            r.status = st.status >= 0 ? st.status : PDLP_STATUS_ITERATION_LIMIT;
            r.iterations = c.k;
            r.attempts = c.attempts;
            r.kkt_passes = st.kkt_passes;
            r.restarts_i = st.r_i;
            r.restarts_ii = st.r_ii;
            r.restarts_iii = st.r_iii;
            r.restarts = st.r_i + st.r_ii + st.r_iii;
            r.primal_obj = k.pobj;
            r.dual_obj = k.dobj;
            r.rel_gap = k.gap;
            r.primal_res_abs = k.pres_abs;
            r.primal_res_rel = k.pres_rel;
            r.dual_res_abs = k.dres_abs;
            r.dual_res_rel = k.dres_rel;
            r.omega = c.omega;
            r.eta = c.eta_hat;
            if (st.cert_src) {
                const bool pinf = st.status == PDLP_STATUS_PRIMAL_INFEASIBLE;
                r.certificate = st.cert_src;
                r.certificate_objective = pinf ? st.cert.pobj : st.cert.dobj;
                r.certificate_residual = pinf ? st.cert.pres : st.cert.dres;
            }
            r.seconds = secs;
            r.seconds_setup = setup;
        }
    }
};

void build_maps(pdlp_batch *b) {
    pdlp_problem *P = b->P;
    const int B = b->B;
    const std::vector<int32_t> &ba = P->blkA, &bt = P->blkT;
    const int nA = (int)ba.size() - 1, nT = (int)bt.size() - 1;
    std::vector<int32_t> ainst(std::max(nA, 1)), tinst(std::max(nT, 1)), aoff(B + 1), toff(B + 1);
    auto inst_of = [](const std::vector<int32_t> &off, int32_t r) {
        return (int32_t)(std::upper_bound(off.begin(), off.end(), r) - off.begin()) - 1;
    };
    for (int k = 0; k < nA; ++k) ainst[k] = inst_of(b->roff, ba[k]);
    for (int k = 0; k < nT; ++k) tinst[k] = inst_of(b->coff, bt[k]);
    for (int i = 0; i <= B; ++i) {
        aoff[i] = (int32_t)(std::lower_bound(ba.begin(), ba.end() - 1, b->roff[i]) - ba.begin());
        toff[i] = (int32_t)(std::lower_bound(bt.begin(), bt.end() - 1, b->coff[i]) - bt.begin());
    }
    aoff[B] = nA;
    toff[B] = nT;
    // every block lies inside its instance
    for (int k = 0; k < nA; ++k)
        if (ba[k + 1] > b->roff[ainst[k] + 1] || k < aoff[ainst[k]] || k >= aoff[ainst[k] + 1])
            throw LibError(PDLP_ERR_HIP, "internal: row block crosses an instance boundary");
    for (int k = 0; k < nT; ++k)
        if (bt[k + 1] > b->coff[tinst[k] + 1] || k < toff[tinst[k]] || k >= toff[tinst[k] + 1])
            throw LibError(PDLP_ERR_HIP, "internal: column block crosses an instance boundary");
    Arena &a = b->arena;
    int32_t *d_ai = a.dev<int32_t>(ainst.size()), *d_ti = a.dev<int32_t>(tinst.size());
    int32_t *d_ao = a.dev<int32_t>(B + 1), *d_to = a.dev<int32_t>(B + 1);
    hipStream_t s = P->stream;
    HIPCHECK(hipMemcpyAsync(d_ai, ainst.data(), sizeof(int32_t) * ainst.size(), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(d_ti, tinst.data(), sizeof(int32_t) * tinst.size(), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(d_ao, aoff.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(d_to, toff.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
    b->aoff = aoff;
    b->toff = toff;
    b->bm.B = B;
    b->bm.nA = nA;
    b->bm.nT = nT;
    b->bm.ablk_inst = d_ai;
    b->bm.tblk_inst = d_ti;
    b->bm.ablk_off = d_ao;
    b->bm.tblk_off = d_to;
}

}  // namespace

void pdlp::host::batch_totals(int32_t count, const int32_t *m, const int32_t *n,
                               const int64_t *nnz, int64_t &M, int64_t &N, int64_t &NZ) {
    if (count < 1) invalid("count must be >= 1");
    if (!m || !n || !nnz) invalid("NULL size array");
    M = N = NZ = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (m[i] < 0 || n[i] < 1 || nnz[i] < 0)
            invalid("instance " + std::to_string(i) + ": need m >= 0, n >= 1, nnz >= 0");
        M += m[i];
        N += n[i];
        NZ += nnz[i];
    }
    const int64_t lim = std::numeric_limits<int32_t>::max();
    if (M >= lim || N >= lim || NZ >= lim) invalid("batch totals must stay below 2^31");
}

pdlp::host::StagedBatch pdlp::host::stage_batch(int32_t count, const int32_t *m,
                                                const int32_t *n, const int64_t *nnz,
                                                const int32_t *row_ptr, const int32_t *col,
                                                const double *val, const double *c,
                                                const double *lc, const double *uc,
                                                const double *lv, const double *uv,
                                                void *hip_stream) {
    int64_t M = 0, N = 0, NZ = 0;
    batch_totals(count, m, n, nnz, M, N, NZ);
    if (!row_ptr || (NZ > 0 && (!col || !val)) || !c || (M > 0 && (!lc || !uc)) || !lv || !uv)
        invalid("NULL input array");
    StagedBatch h;
    h.row_ptr.resize((size_t)(M + count));
    h.col.resize((size_t)NZ);
    h.val.resize((size_t)NZ);
    h.c.resize((size_t)N);
    h.lc.resize((size_t)M);
    h.uc.resize((size_t)M);
    h.lv.resize((size_t)N);
    h.uv.resize((size_t)N);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto get = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
    };
    get(h.row_ptr.data(), row_ptr, sizeof(int32_t) * h.row_ptr.size());
    get(h.col.data(), col, sizeof(int32_t) * h.col.size());
    get(h.val.data(), val, sizeof(double) * h.val.size());
    get(h.c.data(), c, sizeof(double) * h.c.size());
    get(h.lc.data(), lc, sizeof(double) * h.lc.size());
    get(h.uc.data(), uc, sizeof(double) * h.uc.size());
    get(h.lv.data(), lv, sizeof(double) * h.lv.size());
    get(h.uv.data(), uv, sizeof(double) * h.uv.size());
    HIPCHECK(hipStreamSynchronize(s));
    return h;
}

pdlp_batch *pdlp::host::make_batch(int32_t count, const int32_t *m, const int32_t *n,
                                   const int64_t *nnz, const int32_t *row_ptr,
                                   const int32_t *col, const double *val, const double *c,
                                   const double *lc, const double *uc, const double *lv,
                                   const double *uv, const double *obj_offset,
                                   const pdlp_params *params, void *hip_stream, bool sort_gathers) {
    int64_t M = 0, N = 0, NZ = 0;
    batch_totals(count, m, n, nnz, M, N, NZ);
    if (!row_ptr || (NZ > 0 && (!col || !val)) || !c || (M > 0 && (!lc || !uc)) || !lv || !uv)
        invalid("NULL input array");
    // per-instance checks, then pack: global row pointers and column labels
    std::vector<int32_t> rp((size_t)M + 1), cg((size_t)NZ);
    std::vector<int32_t> roff(count + 1), coff(count + 1);
    std::vector<int32_t> row_breaks, col_breaks;
    int64_t r0 = 0, c0 = 0, e0 = 0, p0 = 0;
    rp[0] = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int32_t *rpi = row_ptr + p0;
        try {
            validate(m[i], n[i], nnz[i], rpi, NZ > 0 ? col + e0 : nullptr,
                     NZ > 0 ? val + e0 : nullptr, c + c0, M > 0 ? lc + r0 : nullptr,
                     M > 0 ? uc + r0 : nullptr, lv + c0, uv + c0);
        } catch (const LibError &e) {
            throw LibError(e.code, "instance " + std::to_string(i) + ": " + e.what());
        }
        for (int64_t e = 0; e < nnz[i]; ++e) cg[e0 + e] = (int32_t)(col[e0 + e] + c0);
        for (int32_t r = 0; r < m[i]; ++r) rp[r0 + r + 1] = (int32_t)(e0 + rpi[r + 1]);
        roff[i] = (int32_t)r0;
        coff[i] = (int32_t)c0;
        row_breaks.push_back((int32_t)r0);
        col_breaks.push_back((int32_t)c0);
        r0 += m[i];
        c0 += n[i];
        e0 += nnz[i];
        p0 += (int64_t)m[i] + 1;
    }
    roff[count] = (int32_t)M;
    coff[count] = (int32_t)N;
    auto *b = new pdlp_batch();
    try {
        b->B = count;
        b->m.assign(m, m + count);
        b->n.assign(n, n + count);
        b->roff = roff;
        b->coff = coff;
        b->obj_offset.assign(count, 0.0);
        b->ray_cols.assign(count, 0);
        for (int32_t i = 0; i < count; ++i)
            for (int64_t j = coff[i]; j < coff[i + 1]; ++j)
                b->ray_cols[i] += !std::isfinite(lv[j]) || !std::isfinite(uv[j]);
        if (obj_offset)
            for (int32_t i = 0; i < count; ++i) {
                if (!std::isfinite(obj_offset[i])) invalid("objective offset must be finite");
                b->obj_offset[i] = obj_offset[i];
            }
        b->P = create_problem((int32_t)M, (int32_t)N, NZ, rp.data(), cg.data(), val, c, lc, uc,
                              lv, uv, 0.0, params, hip_stream, &row_breaks, &col_breaks, true);
        if (sort_gathers && (!params || params->sorted_gathers)) sort_block_gathers(b->P);
        build_maps(b);
    } catch (...) {
        delete b;
        throw;
    }
    return b;
}

void pdlp::host::batch_record(pdlp_batch *b, const pdlp_params &prm, BatchRecord &rec) {
    if (!b->W) b->W = make_work(b);
    BatchSolver solver(b, prm, &rec);
    solver.run_record();
}

const double *pdlp::host::batch_current_x(const pdlp_batch *b) {
    return b->W ? b->W->it.X[0] : nullptr;
}

extern "C" {

int pdlp_batch_create(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                      const int32_t *row_ptr, const int32_t *col, const double *val,
                      const double *c, const double *lc, const double *uc, const double *lv,
                      const double *uv, const double *obj_offset, const pdlp_params *params,
                      void *hip_stream, pdlp_batch **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        *out = make_batch(count, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset,
                          params, hip_stream, true);
    });
}

int pdlp_batch_create_device(int32_t count, const int32_t *m, const int32_t *n,
                             const int64_t *nnz, const int32_t *row_ptr, const int32_t *col,
                             const double *val, const double *c, const double *lc,
                             const double *uc, const double *lv, const double *uv,
                             const double *obj_offset, const pdlp_params *params,
                             void *hip_stream, pdlp_batch **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        const StagedBatch h = stage_batch(count, m, n, nnz, row_ptr, col, val, c, lc, uc, lv,
                                          uv, hip_stream);
        *out = make_batch(count, m, n, nnz, h.row_ptr.data(), h.col.data(), h.val.data(),
                          h.c.data(), h.lc.data(), h.uc.data(), h.lv.data(), h.uv.data(),
                          obj_offset, params, hip_stream, true);
    });
}

void pdlp_batch_destroy(pdlp_batch *b) { delete b; }

int pdlp_batch_dims(const pdlp_batch *b, int32_t *count, int64_t *m_total, int64_t *n_total,
                    int64_t *nnz_total) {
    return guarded([&] {
        if (!b) invalid("batch is NULL");
        if (count) *count = b->B;
        if (m_total) *m_total = b->P->m;
        if (n_total) *n_total = b->P->n;
        if (nnz_total) *nnz_total = b->P->nnz;
    });
}

int pdlp_batch_get_stats(const pdlp_batch *b, pdlp_batch_stats *stats) {
    return guarded([&] {
        if (!b || !stats) invalid("NULL argument");
        *stats = b->stats;
    });
}

int pdlp_batch_solve(pdlp_batch *b, const pdlp_params *params, pdlp_result *results, double *x,
                     double *y, double *r) {
    return guarded([&] {
        if (!b || !results) invalid("NULL argument");
        pdlp_params prm;
        pdlp_params_default(&prm);
        if (params) prm = *params;
        check_params(prm);
        if (prm.polish) invalid("feasibility polishing is not available for batches");
        if (prm.restart_period > 0) invalid("the Algorithm 5 mode is not available for batches");
        if (!b->W) b->W = make_work(b);
        BatchSolver solver(b, prm);
        solver.run(results, x, y, r);
    });
}

}  // extern "C"
