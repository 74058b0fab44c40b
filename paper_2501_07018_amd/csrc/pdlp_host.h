// Host-side plumbing shared by the single-LP and the batched drivers of the
// gfx950 PDLP library: error handling, device allocations, the problem object
// and problem creation.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "pdlp.h"
#include "pdlp_internal.h"

namespace pdlp {
namespace host {

extern thread_local std::string g_last_error;

struct LibError : std::runtime_error {
    int code;
    LibError(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] inline void hip_fail(hipError_t e, const char *what, int line) {
    const int code = (e == hipErrorOutOfMemory) ? PDLP_ERR_OUT_OF_MEMORY : PDLP_ERR_HIP;
    throw LibError(code, std::string(what) + " failed (line " + std::to_string(line) +
                             "): " + hipGetErrorString(e));
}

#define HIPCHECK(expr)                                       \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) hip_fail(e_, #expr, __LINE__); \
    } while (0)

[[noreturn]] inline void invalid(const std::string &msg) { throw LibError(PDLP_ERR_INVALID_ARGUMENT, msg); }

// Device allocations owned by an object, freed together.
struct Arena {
    std::vector<void *> ptrs;
    std::vector<void *> pinned;
    template <class T>
    T *dev(size_t count) {
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw LibError(e == hipErrorOutOfMemory ? PDLP_ERR_OUT_OF_MEMORY : PDLP_ERR_HIP,
                           "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                               hipGetErrorString(e));
        }
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
    template <class T>
    T *host(size_t count) {
        void *p = nullptr;
        HIPCHECK(hipHostMalloc(&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
        pinned.push_back(p);
        return static_cast<T *>(p);
    }
    void release(void *p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            (void)hipFree(p);
            ptrs.erase(it);
        }
    }
    ~Arena() {
        for (void *p : ptrs) (void)hipFree(p);
        for (void *p : pinned) (void)hipHostFree(p);
    }
};

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

inline int red_grid(int64_t len) {
    int64_t g = (len + pdlp::kThreads - 1) / pdlp::kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

template <class F>
int guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return PDLP_OK;
    } catch (const LibError &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return PDLP_ERR_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return PDLP_ERR_HIP;
    }
}

// Replays of a fixed launch sequence from HIP graphs: the sequence of one
// step attempt is captured for 64, 8 and 1 attempts, and n attempts are
// enqueued as graph launches of those sizes (greedily), i.e. exactly the
// launches an eager loop would make.  Capture runs on a private stream
// (capturing executes nothing); replays go to the caller's stream.
//
// Lifetime rules: a capture either installs all three executable graphs or
// none (a failure ends the capture, frees what it made and leaves the object
// empty); replaced executable graphs are not destroyed while the owner runs
// but kept until the object is destroyed, which first waits for the last
// replay stream, so no executable graph is freed while work or a runtime
// record of a replay may still refer to it.
struct AttemptGraphs {
    hipStream_t cap = nullptr;
    hipStream_t replay = nullptr;  // stream of the last replay
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    std::vector<hipGraphExec_t> retired;
    static constexpr long long kSizes[3] = {64, 8, 1};
    bool ready() const { return exec[0] && exec[1] && exec[2]; }
    void reset() {
        for (auto &e : exec)
            if (e) {
                retired.push_back(e);
                e = nullptr;
            }
    }
    template <class F>
    void capture(F &&attempt) {
        reset();
        if (!cap) HIPCHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraphExec_t made[3] = {nullptr, nullptr, nullptr};
        try {
            for (int g = 0; g < 3; ++g) {
                HIPCHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
                try {
                    for (long long a = 0; a < kSizes[g]; ++a) attempt(cap);
                } catch (...) {
                    hipGraph_t junk = nullptr;
                    (void)hipStreamEndCapture(cap, &junk);
                    if (junk) (void)hipGraphDestroy(junk);
                    (void)hipGetLastError();
                    throw;
                }
                hipGraph_t graph = nullptr;
                HIPCHECK(hipStreamEndCapture(cap, &graph));
                if (!graph) throw LibError(PDLP_ERR_HIP, "graph capture returned no graph");
                size_t nodes = 0;
                const hipError_t en = hipGraphGetNodes(graph, nullptr, &nodes);
                hipError_t e = en;
                if (en == hipSuccess && nodes == 0) {
                    (void)hipGraphDestroy(graph);
                    throw LibError(PDLP_ERR_STATE, "captured step attempt is empty");
                }
                if (en == hipSuccess) e = hipGraphInstantiate(&made[g], graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                HIPCHECK(e);
            }
        } catch (...) {
            for (auto &e : made)
                if (e) (void)hipGraphExecDestroy(e);
            throw;
        }
        for (int g = 0; g < 3; ++g) exec[g] = made[g];
    }
    void launch(hipStream_t s, long long n) {
        if (!ready()) throw LibError(PDLP_ERR_STATE, "graph replay without a complete capture");
        replay = s;
        for (int g = 0; g < 3; ++g)
            for (; n >= kSizes[g]; n -= kSizes[g]) HIPCHECK(hipGraphLaunch(exec[g], s));
    }
    ~AttemptGraphs() {
        if (replay) (void)hipStreamSynchronize(replay);
        reset();
        for (auto e : retired) (void)hipGraphExecDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

inline void check_params(const pdlp_params &p) {
    if (!(p.check_every >= 1)) invalid("check_every must be >= 1");
    if (p.ruiz_iters < 0) invalid("ruiz_iters must be >= 0");
    if (!(p.eps_feas >= 0.0) || !(p.eps_gap >= 0.0)) invalid("tolerances must be >= 0");
    if (p.max_iters < 0) invalid("max_iters must be >= 0");
    if (!(p.theta >= 0.0 && p.theta <= 1.0)) invalid("theta must lie in [0, 1]");
    if (!(p.beta_art > 0.0)) invalid("beta_art must be > 0");
    if (p.detect_infeasibility && !(p.eps_infeasible >= 0.0))
        invalid("eps_infeasible must be >= 0");
    if (p.restart_period < 0) invalid("restart_period must be >= 0");
    if (p.stream_block != 0 && p.stream_block != -1 &&
        !(p.stream_block >= 64 && p.stream_block <= pdlp::kStage))
        invalid("stream_block must be 0, -1 or in [64, 2048]");
    if (p.sorted_gathers != 0 && p.sorted_gathers != 1) invalid("sorted_gathers must be 0 or 1");
    if (p.segmented_gathers < -1 || p.segmented_gathers > 1)
        invalid("segmented_gathers must be -1, 0 or 1");
    if (p.restart_period > 0) {
        if (!(p.fixed_step_size > 0.0) || !std::isfinite(p.fixed_step_size))
            invalid("restart_period > 0 needs a finite fixed_step_size > 0");
        if (!(p.fixed_primal_weight > 0.0) || !std::isfinite(p.fixed_primal_weight))
            invalid("restart_period > 0 needs a finite fixed_primal_weight > 0");
        if (p.polish) invalid("restart_period > 0 excludes polishing");
    }
}

// Input checks of a problem (conventions of the C ABI); throws
// INVALID_ARGUMENT with a message naming the offending row or column.
void validate(int32_t m, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
              const double *val, const double *c, const double *lc, const double *uc,
              const double *lv, const double *uv);

// Smallest k' > k with (double)(t + k' - k) >= beta * (double)k' (restart
// condition (iii) of Section 3), capped at cap.
long long next_art(long long k, long long t, double beta, long long cap);

}  // namespace host
}  // namespace pdlp

// Device copy of a problem (the C ABI's opaque pdlp_problem).
struct pdlp_problem {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    int device = 0;  // the GPU holding the problem (current at creation)
    int32_t stage = pdlp::kStage;  // nonzeros per stream block (the schedule in use)
    hipStream_t stream = nullptr;
    pdlp::host::Arena arena;
    pdlp::DCsr A, AT;
    pdlp::SegCsr segT;  // two-phase layout of A^T (built for long y; S = 0 otherwise)
    double *d1 = nullptr, *d2 = nullptr;                                // scaling
    double *c = nullptr, *lc = nullptr, *uc = nullptr, *lv = nullptr, *uv = nullptr;  // original
    double *cs = nullptr, *lcs = nullptr, *ucs = nullptr, *lvs = nullptr, *uvs = nullptr;
    double *zero_n = nullptr;                                            // c = 0 (primal polish)
    double *lc0 = nullptr, *uc0 = nullptr, *lv0 = nullptr, *uv0 = nullptr;  // finite bounds -> 0
    double obj_offset = 0.0;
    int64_t ray_cols = 0;        // variables with an infinite bound (recession cone Xbar_j != {0})
    double *red_part = nullptr;  // partials of generic reductions
    int red_cap = 0;
    // internal row/column labels: row_order[new] = caller's row, col_order likewise;
    // orig_pos[new entry] = caller's entry index
    int32_t *row_order = nullptr, *col_order = nullptr, *orig_pos = nullptr;
    std::vector<int32_t> blkA, blkT;  // host copies of the row-block partitions
    int64_t *sperm[2] = {nullptr, nullptr};  // A, A^T: source entry of each sorted-copy entry
    double *res_d = nullptr, *res_h = nullptr;  // small reduction results
    pdlp_params scale_params;

    pdlp::Vecs scaled() const { return pdlp::Vecs{cs, lcs, ucs, lvs, uvs}; }
};

// Problem creation shared by single problems and batches (row_breaks /
// col_breaks: first rows / columns of the instances of a batch, which row
// blocks may not straddle; a batch keeps the caller's labels).
// Column-sorted copies of the short-row blocks (DCsr::scol/sval/slot) of a
// created problem, from its current scaled values.
void sort_block_gathers(pdlp_problem *P);
// Copy the current values of A and A^T into their sorted copies (after the
// values changed), on stream s.
void refresh_block_gathers(pdlp_problem *P, hipStream_t s);
pdlp_problem *create_problem(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col, const double *val, const double *c,
                             const double *lc, const double *uc, const double *lv,
                             const double *uv, double obj_offset, const pdlp_params *params,
                             void *hip_stream, const std::vector<int32_t> *row_breaks,
                             const std::vector<int32_t> *col_breaks, bool validated = false);
