// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer run of the
// library's host code (test infrastructure only).  It is linked against a
// build of libpdlp.so whose host code is instrumented (device code is not:
// GPU sanitizers are not used) and calls every entry point of the C ABI on
// small synthetic LPs, so that the host-side engine -- validation, the
// relabelling sorts, block partitions, the two-phase layout, graph capture,
// the batch lists, the unrolled map's bookkeeping -- runs under the
// sanitizers.  Results are only checked for being produced (return codes,
// finite values); the parity tests compare them with the oracle.
//
//   pdlp_host_sanitize cpu       only calls that must fail before any GPU work
//   pdlp_host_sanitize gpu       everything (needs a GPU)
//   pdlp_host_sanitize overflow  a caller mistake the library's validation must
//                                trip over on the host: c one entry short (shows
//                                that the instrumentation is live; no GPU work)
//
// Exit status 0 when every call behaved; the sanitizers abort on the first
// memory or undefined-behaviour error.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pdlp.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, pdlp_last_error());
        ++failures;
    }
}

#define OK(call) expect((call) == PDLP_OK, #call)
#define ERR(call, code) expect((call) == (code), #call " -> " #code)

// splitmix64
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double unif() { return (double)(next() >> 11) * 0x1.0p-53; }
    int below(int k) { return (int)(next() % (uint64_t)k); }
};

struct Lp {
    int32_t m = 0, n = 0;
    std::vector<int32_t> rp, col;
    std::vector<double> val, c, lc, uc, lv, uv;
    int64_t nnz() const { return (int64_t)col.size(); }
};

// A feasible, bounded LP: per_col distinct rows per column (values in
// [-1, 1]), a point x* in the box, rows of every kind around A x*, and
// variables boxed except a few free or one-sided ones with zero cost.
Lp feasible_lp(int32_t m, int32_t n, int per_col, uint64_t seed) {
    Rng r{seed};
    Lp lp;
    lp.m = m;
    lp.n = n;
    std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)m);
    std::vector<int32_t> pick;
    for (int32_t j = 0; j < n; ++j) {
        pick.clear();
        const int k = m > 0 ? std::min(per_col, (int)m) : 0;
        while ((int)pick.size() < k) {
            const int32_t i = r.below(m);
            bool dup = false;
            for (int32_t p : pick) dup |= p == i;
            if (!dup) pick.push_back(i);
        }
        for (int32_t i : pick) rows[(size_t)i].push_back({j, 2.0 * r.unif() - 1.0});
    }
    lp.rp.push_back(0);
    for (auto &row : rows) {
        for (auto &e : row) {
            lp.col.push_back(e.first);
            lp.val.push_back(e.second);
        }
        lp.rp.push_back((int32_t)lp.col.size());
    }
    std::vector<double> xs((size_t)n);
    lp.c.resize((size_t)n);
    lp.lv.assign((size_t)n, 0.0);
    lp.uv.assign((size_t)n, 1.0);
    for (int32_t j = 0; j < n; ++j) {
        xs[(size_t)j] = r.unif();
        lp.c[(size_t)j] = 2.0 * r.unif() - 1.0;
        if (j % 17 == 5) {  // free, no cost
            lp.lv[(size_t)j] = -HUGE_VAL;
            lp.uv[(size_t)j] = HUGE_VAL;
            lp.c[(size_t)j] = 0.0;
        } else if (j % 17 == 9) {  // one-sided, cost keeps it bounded
            lp.uv[(size_t)j] = HUGE_VAL;
            lp.c[(size_t)j] = std::fabs(lp.c[(size_t)j]) + 0.1;
        }
    }
    lp.lc.resize((size_t)m);
    lp.uc.resize((size_t)m);
    for (int32_t i = 0; i < m; ++i) {
        double ax = 0.0;
        for (int32_t e = lp.rp[(size_t)i]; e < lp.rp[(size_t)i + 1]; ++e)
            ax += lp.val[(size_t)e] * xs[(size_t)lp.col[(size_t)e]];
        switch (i % 5) {
            case 0: lp.lc[(size_t)i] = lp.uc[(size_t)i] = ax; break;
            case 1: lp.lc[(size_t)i] = -HUGE_VAL; lp.uc[(size_t)i] = ax + 0.5 * r.unif(); break;
            case 2: lp.lc[(size_t)i] = ax - 0.5 * r.unif(); lp.uc[(size_t)i] = HUGE_VAL; break;
            case 3: lp.lc[(size_t)i] = ax - 0.3; lp.uc[(size_t)i] = ax + 0.3; break;
            default: lp.lc[(size_t)i] = -HUGE_VAL; lp.uc[(size_t)i] = HUGE_VAL; break;
        }
    }
    return lp;
}

// x >= 0 with sum_j x_j <= -1: primal infeasible.
Lp infeasible_lp() {
    Lp lp;
    lp.m = 1;
    lp.n = 3;
    lp.rp = {0, 3};
    lp.col = {0, 1, 2};
    lp.val = {1.0, 1.0, 1.0};
    lp.c = {1.0, 2.0, 3.0};
    lp.lc = {-HUGE_VAL};
    lp.uc = {-1.0};
    lp.lv = {0.0, 0.0, 0.0};
    lp.uv = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
    return lp;
}

pdlp_problem *create(const Lp &lp, const pdlp_params *prm) {
    pdlp_problem *p = nullptr;
    OK(pdlp_problem_create(lp.m, lp.n, lp.nnz(), lp.rp.data(), lp.col.data(), lp.val.data(),
                           lp.c.data(), lp.lc.data(), lp.uc.data(), lp.lv.data(), lp.uv.data(),
                           0.25, prm, nullptr, &p));
    return p;
}

// Calls that must be refused before anything reaches the GPU.
void rejections() {
    const Lp good = feasible_lp(40, 60, 3, 1);
    pdlp_problem *p = nullptr;
    auto try_lp = [&](const Lp &lp, const char *what, const pdlp_params *prm = nullptr) {
        p = nullptr;
        const int rc = pdlp_problem_create(lp.m, lp.n, lp.nnz(), lp.rp.data(), lp.col.data(),
                                           lp.val.data(), lp.c.data(), lp.lc.data(),
                                           lp.uc.data(), lp.lv.data(), lp.uv.data(), 0.0,
                                           prm, nullptr, &p);
        expect(rc == PDLP_ERR_INVALID_ARGUMENT && p == nullptr, what);
    };
    Lp bad = good;
    bad.col[1] = bad.col[0];
    try_lp(bad, "duplicate column");
    bad = good;
    bad.col[2] = good.n;
    try_lp(bad, "column out of range");
    bad = good;
    bad.val[3] = NAN;
    try_lp(bad, "NaN value");
    bad = good;
    bad.lc[0] = bad.uc[0] + 1.0;
    try_lp(bad, "lc > uc");
    bad = good;
    bad.lv[1] = HUGE_VAL;
    try_lp(bad, "lower bound +inf");
    bad = good;
    bad.rp[5] = bad.rp[4] - 1;
    try_lp(bad, "row_ptr decreasing");
    bad = good;
    bad.rp[0] = 1;
    try_lp(bad, "row_ptr[0]");
    ERR(pdlp_problem_create(-1, 3, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, 0.0, nullptr, nullptr, &p),
        PDLP_ERR_INVALID_ARGUMENT);
    ERR(pdlp_problem_create(2, 3, 1, good.rp.data(), nullptr, nullptr, good.c.data(), nullptr,
                            nullptr, good.lv.data(), good.uv.data(), 0.0, nullptr, nullptr, &p),
        PDLP_ERR_INVALID_ARGUMENT);
    pdlp_params prm;
    pdlp_params_default(&prm);
    prm.stream_block = 7;
    try_lp(good, "stream_block out of range", &prm);
    // batches: per-instance checks name the instance
    const int32_t ms[2] = {good.m, good.m}, ns[2] = {good.n, 0};
    const int64_t zs[2] = {good.nnz(), good.nnz()};
    pdlp_batch *b = nullptr;
    ERR(pdlp_batch_create(2, ms, ns, zs, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr, nullptr, nullptr, nullptr, &b),
        PDLP_ERR_INVALID_ARGUMENT);
    expect(std::strstr(pdlp_last_error(), "instance 1") != nullptr, "batch error names instance");
    ERR(pdlp_batch_create_device(0, ms, ns, zs, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &b),
        PDLP_ERR_INVALID_ARGUMENT);
    pdlp_unroll *u = nullptr;
    ERR(pdlp_unroll_create_device(2, ms, ns, zs, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, &u),
        PDLP_ERR_INVALID_ARGUMENT);
    ERR(pdlp_solve(nullptr, nullptr, nullptr, nullptr, nullptr), PDLP_ERR_INVALID_ARGUMENT);
    ERR(pdlp_iterate_k(nullptr, 1, nullptr), PDLP_ERR_INVALID_ARGUMENT);
    ERR(pdlp_batch_solve(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr),
        PDLP_ERR_INVALID_ARGUMENT);
    ERR(pdlp_unroll_forward(nullptr, nullptr, 3, 1, nullptr), PDLP_ERR_INVALID_ARGUMENT);
}

bool finite(const std::vector<double> &v) {
    for (double a : v)
        if (!std::isfinite(a)) return false;
    return true;
}

void single_problem(const Lp &lp, pdlp_params prm, bool polish) {
    pdlp_problem *p = create(lp, &prm);
    if (!p) return;
    int32_t m = 0, n = 0, blk = 0, med = 0;
    int64_t nnz = 0;
    OK(pdlp_problem_dims(p, &m, &n, &nnz));
    expect(m == lp.m && n == lp.n && nnz == lp.nnz(), "dims");
    OK(pdlp_problem_schedule(p, &blk, &med));
    std::vector<double> d1((size_t)m), d2((size_t)n), sv((size_t)nnz), sc((size_t)n),
        slc((size_t)m), suc((size_t)m), slv((size_t)n), suv((size_t)n);
    OK(pdlp_problem_get_scaled(p, d1.data(), d2.data(), sv.data(), sc.data(), slc.data(),
                               suc.data(), slv.data(), suv.data()));
    std::vector<double> xin((size_t)n, 0.5), yin((size_t)m, -0.25), ax((size_t)m), aty((size_t)n);
    double ms = 0.0;
    for (int t = 0; t < 2; ++t)
        for (int scaled = 0; scaled < 2; ++scaled) {
            OK(pdlp_spmv(p, t, scaled, t ? yin.data() : xin.data(), t ? aty.data() : ax.data(),
                         2, &ms));
        }
    expect(finite(ax) && finite(aty), "spmv finite");
    // allocation-free product on caller device buffers
    double *xd = nullptr, *od = nullptr;
    if (hipMalloc((void **)&xd, sizeof(double) * (size_t)(m + n)) == hipSuccess &&
        hipMalloc((void **)&od, sizeof(double) * (size_t)(m + n)) == hipSuccess) {
        (void)hipMemcpy(xd, xin.data(), sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
        OK(pdlp_spmv_noalloc(p, 0, 1, xd, od, nullptr));
        OK(pdlp_spmv_noalloc(p, 1, 0, xd, od, nullptr));
        (void)hipDeviceSynchronize();
    } else {
        expect(false, "hipMalloc");
    }
    (void)hipFree(xd);
    (void)hipFree(od);
    // solve
    std::vector<double> x((size_t)n), y((size_t)m), r((size_t)n);
    pdlp_result res;
    std::memset(&res, 0, sizeof(res));
    res.x = x.data();
    res.y = y.data();
    res.r = r.data();
    prm.polish = polish;
    OK(pdlp_solve(p, &prm, nullptr, nullptr, &res));
    expect(finite(x) && finite(y), "solution finite");
    // warm start from the solution
    pdlp_result res2;
    std::memset(&res2, 0, sizeof(res2));
    OK(pdlp_solve(p, &prm, x.data(), y.data(), &res2));
    // state: iterate, export, import, continue, kernel statistics
    pdlp_params sp = prm;
    sp.profile = 1;
    pdlp_state *s = nullptr;
    OK(pdlp_state_create(p, &sp, &s));
    if (s) {
        pdlp_iter_info info;
        OK(pdlp_iterate_k(s, 70, &info));
        std::vector<double> bx((size_t)n), by((size_t)m), bax((size_t)m), baty((size_t)n),
            bx0((size_t)n), by0((size_t)m), bsx((size_t)n), bsy((size_t)m);
        pdlp_state_blob blob;
        std::memset(&blob, 0, sizeof(blob));
        blob.x = bx.data();
        blob.y = by.data();
        blob.ax = bax.data();
        blob.aty = baty.data();
        blob.x0 = bx0.data();
        blob.y0 = by0.data();
        blob.sx = bsx.data();
        blob.sy = bsy.data();
        OK(pdlp_state_get(s, &blob));
        OK(pdlp_state_set(s, &blob));
        double mu = 0.0;
        OK(pdlp_norm_gap(p, bx.data(), by.data(), bax.data(), baty.data(), bx0.data(),
                         by0.data(), blob.omega, &mu));
        expect(std::isfinite(mu), "norm gap finite");
        pdlp_result rs;
        std::memset(&rs, 0, sizeof(rs));
        OK(pdlp_state_solve(s, 200, &rs));
        pdlp_kernel_stats ks;
        OK(pdlp_state_kernel_stats(s, &ks, 1));
        pdlp_state_destroy(s);
    }
    pdlp_problem_destroy(p);
}

void batch(const std::vector<Lp> &lps, pdlp_params prm) {
    std::vector<int32_t> m, n, rp, col;
    std::vector<int64_t> nnz;
    std::vector<double> val, c, lc, uc, lv, uv, off;
    for (const Lp &lp : lps) {
        m.push_back(lp.m);
        n.push_back(lp.n);
        nnz.push_back(lp.nnz());
        rp.insert(rp.end(), lp.rp.begin(), lp.rp.end());
        col.insert(col.end(), lp.col.begin(), lp.col.end());
        val.insert(val.end(), lp.val.begin(), lp.val.end());
        c.insert(c.end(), lp.c.begin(), lp.c.end());
        lc.insert(lc.end(), lp.lc.begin(), lp.lc.end());
        uc.insert(uc.end(), lp.uc.begin(), lp.uc.end());
        lv.insert(lv.end(), lp.lv.begin(), lp.lv.end());
        uv.insert(uv.end(), lp.uv.begin(), lp.uv.end());
        off.push_back(1.5);
    }
    const int32_t cnt = (int32_t)lps.size();
    pdlp_batch *b = nullptr;
    OK(pdlp_batch_create(cnt, m.data(), n.data(), nnz.data(), rp.data(), col.data(), val.data(),
                         c.data(), lc.data(), uc.data(), lv.data(), uv.data(), off.data(), &prm,
                         nullptr, &b));
    if (!b) return;
    int32_t bc = 0;
    int64_t M = 0, N = 0, NZ = 0;
    OK(pdlp_batch_dims(b, &bc, &M, &N, &NZ));
    std::vector<pdlp_result> res((size_t)cnt);
    std::memset(res.data(), 0, sizeof(pdlp_result) * res.size());
    std::vector<double> x((size_t)N), y((size_t)M), r((size_t)N);
    pdlp_params sp = prm;
    sp.max_iters = 3000;
    OK(pdlp_batch_solve(b, &sp, res.data(), x.data(), y.data(), r.data()));
    expect(finite(x) && finite(y), "batch solution finite");
    sp.graphs = 0;
    OK(pdlp_batch_solve(b, &sp, res.data(), nullptr, nullptr, nullptr));
    pdlp_batch_stats st;
    OK(pdlp_batch_get_stats(b, &st));
    pdlp_batch_destroy(b);
    // the same arrays from device memory
    std::vector<void *> dev;
    auto alloc = [&](size_t bytes) -> void * {
        void *d = nullptr;
        if (hipMalloc(&d, bytes ? bytes : 8) != hipSuccess) {
            expect(false, "hipMalloc");
            return nullptr;
        }
        dev.push_back(d);
        return d;
    };
    auto put = [&](const void *src, size_t bytes) -> void * {
        void *d = alloc(bytes);
        if (d && bytes) (void)hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
        return d;
    };
    void *drp = put(rp.data(), 4 * rp.size()), *dcol = put(col.data(), 4 * col.size());
    void *dval = put(val.data(), 8 * val.size()), *dc = put(c.data(), 8 * c.size());
    void *dlc = put(lc.data(), 8 * lc.size()), *duc = put(uc.data(), 8 * uc.size());
    void *dlv = put(lv.data(), 8 * lv.size()), *duv = put(uv.data(), 8 * uv.size());
    OK(pdlp_batch_create_device(cnt, m.data(), n.data(), nnz.data(), (const int32_t *)drp,
                                (const int32_t *)dcol, (const double *)dval, (const double *)dc,
                                (const double *)dlc, (const double *)duc, (const double *)dlv,
                                (const double *)duv, off.data(), &prm, nullptr, &b));
    if (b) {
        OK(pdlp_batch_solve(b, &sp, res.data(), x.data(), y.data(), r.data()));
        pdlp_batch_destroy(b);
    }
    // the unrolled map: forward, replay, backward, tangent, tape, device variants
    pdlp_unroll *u = nullptr;
    OK(pdlp_unroll_create_device(cnt, m.data(), n.data(), nnz.data(), (const int32_t *)drp,
                                 (const int32_t *)dcol, (const double *)dval, (const double *)dc,
                                 (const double *)dlc, (const double *)duc, (const double *)dlv,
                                 (const double *)duv, &prm, nullptr, &u));
    if (u) {
        const int64_t K = 90;
        OK(pdlp_unroll_forward(u, &prm, K, 25, x.data()));
        std::vector<int64_t> sig((size_t)cnt);
        OK(pdlp_unroll_replay(u, x.data(), sig.data()));
        std::vector<double> gx((size_t)N, 1.0), gc((size_t)N), glc((size_t)M), guc((size_t)M),
            gval((size_t)NZ), dx((size_t)N);
        OK(pdlp_unroll_backward(u, gx.data(), gc.data(), glc.data(), guc.data(), gval.data()));
        expect(finite(gc) && finite(gval), "gradients finite");
        OK(pdlp_unroll_tangent(u, c.data(), nullptr, nullptr, val.data(), dx.data()));
        std::vector<double> eta((size_t)(cnt * K)), om((size_t)(cnt * K));
        std::vector<int32_t> rst((size_t)(cnt * K));
        OK(pdlp_unroll_get_tape(u, eta.data(), om.data(), rst.data()));
        pdlp_unroll_stats us;
        OK(pdlp_unroll_get_stats(u, &us));
        OK(pdlp_unroll_set_data(u, c.data(), nullptr, nullptr, val.data()));
        OK(pdlp_unroll_set_data_device(u, (const double *)dc, (const double *)dlc,
                                       (const double *)duc, (const double *)dval, nullptr));
        void *dgx = put(gx.data(), 8 * gx.size());
        void *dxo = alloc(8 * (size_t)N), *dgc = alloc(8 * (size_t)N), *ddx = alloc(8 * (size_t)N);
        void *dgl = alloc(8 * (size_t)M), *dgu = alloc(8 * (size_t)M);
        void *dgv = alloc(8 * (size_t)NZ);
        OK(pdlp_unroll_forward_device(u, &prm, K, 25, (double *)dxo, nullptr));
        OK(pdlp_unroll_backward_device(u, (const double *)dgx, (double *)dgc, (double *)dgl,
                                       (double *)dgu, (double *)dgv, nullptr));
        OK(pdlp_unroll_tangent_device(u, (const double *)dc, nullptr, nullptr,
                                      (const double *)dval, (double *)ddx, nullptr));
        (void)hipDeviceSynchronize();
        pdlp_unroll_destroy(u);
    }
    (void)hipDeviceSynchronize();
    for (void *d : dev) (void)hipFree(d);
}

}  // namespace

int main(int argc, char **argv) {
    const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
    if (argc > 1 && std::strcmp(argv[1], "overflow") == 0) {
        Lp lp = feasible_lp(40, 60, 3, 1);
        std::vector<double> c_short(lp.c.begin(), lp.c.end() - 1);
        pdlp_problem *p = nullptr;
        const int rc = pdlp_problem_create(lp.m, lp.n, lp.nnz(), lp.rp.data(), lp.col.data(),
                                           lp.val.data(), c_short.data(), lp.lc.data(),
                                           lp.uc.data(), lp.lv.data(), lp.uv.data(), 0.0,
                                           nullptr, nullptr, &p);
        std::printf("[sanitize] short c not detected (rc %d)\n", rc);
        return 0;
    }
    std::printf("[sanitize] rejections\n");
    std::fflush(stdout);
    rejections();
    if (gpu) {
        pdlp_params prm;
        pdlp_params_default(&prm);
        prm.eps_feas = prm.eps_gap = 1e-5;
        prm.max_iters = 4000;
        const Lp a = feasible_lp(300, 500, 4, 11);
        std::printf("[sanitize] single problem, default schedule\n");
        std::fflush(stdout);
        single_problem(a, prm, false);
        std::printf("[sanitize] single problem, polishing, two-phase product, no relabelling\n");
        std::fflush(stdout);
        pdlp_params p2 = prm;
        p2.segmented_gathers = 1;
        p2.reorder = 0;
        single_problem(feasible_lp(2000, 3000, 5, 12), p2, true);
        std::printf("[sanitize] single problem, autotuned schedule, eager launches\n");
        std::fflush(stdout);
        pdlp_params p3 = prm;
        p3.stream_block = -1;
        p3.graphs = 0;
        single_problem(feasible_lp(1500, 2500, 6, 13), p3, false);
        std::printf("[sanitize] infeasible problem, Algorithm 5 mode\n");
        std::fflush(stdout);
        single_problem(infeasible_lp(), prm, false);
        pdlp_params p5 = prm;
        p5.restart_period = 16;
        p5.fixed_step_size = 0.5;
        p5.fixed_primal_weight = 1.0;
        single_problem(feasible_lp(100, 150, 3, 14), p5, false);
        std::printf("[sanitize] batch and unrolled map\n");
        std::fflush(stdout);
        std::vector<Lp> lps = {feasible_lp(200, 300, 4, 21), feasible_lp(0, 5, 0, 22),
                               feasible_lp(900, 1200, 8, 23), infeasible_lp()};
        batch(lps, prm);
        pdlp_params pb = prm;
        pb.stream_block = -1;
        pb.sorted_gathers = 0;
        batch(lps, pb);
    }
    std::printf("[sanitize] done, %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
