// Batch object shared by the batched solver and the unrolled (differentiable)
// driver.  Nothing here is part of the C ABI.
#pragma once

#include <vector>

#include "pdlp_host.h"

namespace pdlp {
namespace host {

struct BatchWork;  // device work buffers of a batch solve (pdlp_batch.hip)

// Record of a batched Algorithm 1 run of exactly K accepted steps per
// instance without termination tests: the decisions of every accepted step
// (written by the step-decision kernel) and checkpoints of the state.
struct BatchRecord {
    int64_t K = 0;
    int32_t ckpt = 25;          // checkpoint every ckpt accepted steps (k = 0, ckpt, ...)
    double *eta = nullptr;      // device [B * K]: step size of accepted step k of instance i
    double *omega = nullptr;    // device [B * K]: primal weight it used
    std::vector<int32_t> rtype; // host [B * K]: restart right after step k (0, 1 current, 2 average)
    double *ck = nullptr;       // device [nck * 2 (N + M)]: slot c = state at k = c ckpt
    int32_t nck = 0;            //   (post-restart), laid out x | y | Sx | Sy
};

// Checks the per-instance sizes of a batch (count >= 1; m >= 0, n >= 1,
// nnz >= 0 each) and returns their totals, each below 2^31.
void batch_totals(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                  int64_t &M, int64_t &N, int64_t &NZ);

// Host copies of a batch's concatenated instance arrays given in GPU memory
// (the *_create_device calls): lengths from the host size arrays m, n, nnz;
// copied on hip_stream after the work already queued there, and waited for.
struct StagedBatch {
    std::vector<int32_t> row_ptr, col;
    std::vector<double> val, c, lc, uc, lv, uv;
};
StagedBatch stage_batch(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                        const int32_t *row_ptr, const int32_t *col, const double *val,
                        const double *c, const double *lc, const double *uc, const double *lv,
                        const double *uv, void *hip_stream);

// Packs `count` instances (arrays concatenated in instance order, local
// column labels) into a batch; validates every instance.  sort_gathers adds
// the column-sorted block copies of the matrices (refresh_block_gathers
// after any later change of the matrix values).
pdlp_batch *make_batch(int32_t count, const int32_t *m, const int32_t *n, const int64_t *nnz,
                       const int32_t *row_ptr, const int32_t *col, const double *val,
                       const double *c, const double *lc, const double *uc, const double *lv,
                       const double *uv, const double *obj_offset, const pdlp_params *params,
                       void *hip_stream, bool sort_gathers);

// Runs K accepted steps of Algorithm 1 (restart checks, no termination) on
// every instance from (proj_X(0), 0), filling `rec`; the final iterate is
// left in the batch's work buffers (batch_current_x).  Throws on a
// numerical error.
void batch_record(pdlp_batch *b, const pdlp_params &prm, BatchRecord &rec);
const double *batch_current_x(const pdlp_batch *b);

}  // namespace host
}  // namespace pdlp

struct pdlp_batch {
    int32_t B = 0;
    std::vector<int32_t> m, n, roff, coff;
    std::vector<double> obj_offset;
    std::vector<int64_t> ray_cols;    // per instance: variables with an infinite bound
    pdlp_problem *P = nullptr;
    pdlp::host::Arena arena;
    pdlp::BatchMaps bm;
    std::vector<int32_t> aoff, toff;  // host copies of the block ranges per instance
    pdlp::host::BatchWork *W = nullptr;
    pdlp_batch_stats stats{};  // of the last solve
    ~pdlp_batch();
};
