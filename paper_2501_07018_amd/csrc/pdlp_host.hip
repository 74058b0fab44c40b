// Host driver and C ABI of the gfx950 PDLP library.
//
// The host runs the control logic of Algorithm 1 at iteration-block
// boundaries; the device runs every per-element step.  Block boundaries
// are the accepted-step counts where something other than a plain PDHG step
// must happen: multiples of the check cadence (restart criteria (i), (ii)
// and termination, Section 3 "Periodic checks"), the first count where
// condition (iii) t >= beta_art k holds (it depends only on t and k, so it is
// known in advance), feasibility-polishing points (Algorithm 4) and the
// iteration cap.  Inside a block the step attempts (Algorithm 2) run on the
// device with their accept/reject decision in the device control block.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "pdlp_host.h"

// Workgroups of the persistent CSR stream kernels (8 per CU on 256 CUs).
#ifndef PDLP_STREAM_GRID_CAP
#define PDLP_STREAM_GRID_CAP 2048
#endif

namespace pdlp {
namespace host {
thread_local std::string g_last_error;
}  // namespace host
}  // namespace pdlp

using namespace pdlp::host;

namespace {

using pdlp::Ctrl;
using pdlp::DCsr;
using pdlp::GapState;
using pdlp::Iter;
using pdlp::KktOut;
using pdlp::kThreads;
using pdlp::Vecs;


// Row blocks of the CSR stream kernels (see DCsr): stream blocks of rows
// with at most kMedRow nonzeros that fit the LDS stage, wave blocks of up
// to kWaveRows medium rows, and single long rows.
// `breaks` (sorted, optional) lists rows at which a block must start: the
// first rows of the instances of a batch.
std::vector<int32_t> make_blocks(const int32_t *rp, int32_t rows,
                                 const std::vector<int32_t> *breaks, int32_t stage,
                                 int32_t max_rows = pdlp::kMaxBlockRows,
                                 int32_t med_row = pdlp::kMedRow) {
    std::vector<int32_t> blk;
    blk.push_back(0);
    int32_t r = 0;
    size_t bi = 0;
    auto L = [&](int32_t i) { return rp[i + 1] - rp[i]; };
    while (r < rows) {
        while (breaks && bi < breaks->size() && (*breaks)[bi] <= r) ++bi;
        const int32_t lim = (breaks && bi < breaks->size()) ? (*breaks)[bi] : rows;
        const int32_t len = L(r);
        if (len > pdlp::kWaveMax) {
            ++r;
        } else if (len > med_row) {
            const int32_t start = r;
            while (r < lim && r - start < pdlp::kWaveRows && L(r) > med_row &&
                   L(r) <= pdlp::kWaveMax)
                ++r;
        } else {
            const int32_t start = r;
            int64_t nz = 0;
            while (r < lim && r - start < max_rows) {
                const int32_t l = L(r);
                if (l > med_row || nz + l > stage) break;
                nz += l;
                ++r;
            }
        }
        blk.push_back(r);
    }
    return blk;
}

// [hot-path layout begin]
// (The labels decide which cache lines the products gather from, so this
// region is part of what the recorded traffic figures were taken on.)

// Host threads for the labelling sorts: at most 16, about one per 2^20 items.
template <class F>
void parallel_for(int64_t len, F &&f) {
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t t = std::max<int64_t>(1, std::min<int64_t>({16, hw, len >> 20}));
    if (t == 1) {
        f(0, len);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t k = 0; k < t; ++k) th.emplace_back(f, len * k / t, len * (k + 1) / t);
    for (auto &x : th) x.join();
}

// Sort by (key, index); the indices are distinct, so the order is total and
// the result does not depend on the thread count.  Chunks are sorted in
// parallel, then merged pairwise.
template <class K>
void parallel_sort(std::vector<std::pair<K, int32_t>> &kv) {
    const int64_t len = (int64_t)kv.size();
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t t = std::max<int64_t>(1, std::min<int64_t>({16, hw, len >> 20}));
    if (t == 1) {
        std::sort(kv.begin(), kv.end());
        return;
    }
    std::vector<int64_t> cut((size_t)t + 1);
    for (int64_t k = 0; k <= t; ++k) cut[(size_t)k] = len * k / t;
    {
        std::vector<std::thread> th;
        for (int64_t k = 0; k < t; ++k)
            th.emplace_back([&, k] { std::sort(kv.begin() + cut[k], kv.begin() + cut[k + 1]); });
        for (auto &x : th) x.join();
    }
    for (int64_t w = 1; w < t; w *= 2) {
        std::vector<std::thread> th;
        for (int64_t k = 0; k + w < t; k += 2 * w) {
            const int64_t a = cut[(size_t)k], b = cut[(size_t)(k + w)],
                          c = cut[(size_t)std::min(t, k + 2 * w)];
            th.emplace_back([&kv, a, b, c] {
                std::inplace_merge(kv.begin() + a, kv.begin() + b, kv.begin() + c);
            });
        }
        for (auto &x : th) x.join();
    }
}

// Stable order of indices by decreasing count (counting sort): order[new] = old.
std::vector<int32_t> order_by_count(const std::vector<int32_t> &cnt, bool reorder) {
    const int32_t len = (int32_t)cnt.size();
    std::vector<int32_t> order(len);
    if (!reorder) {
        for (int32_t i = 0; i < len; ++i) order[i] = i;
        return order;
    }
    int32_t mx = 0;
    for (int32_t c : cnt) mx = std::max(mx, c);
    std::vector<int64_t> start((size_t)mx + 2, 0);
    for (int32_t c : cnt) start[(size_t)(mx - c) + 1] += 1;
    for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
    for (int32_t i = 0; i < len; ++i) order[start[(size_t)(mx - cnt[i])]++] = i;
    return order;
}

// Row labels: rows longer than kMedRow first, by decreasing length; then the
// stream rows ordered by the three smallest new labels of their columns --
// with columns labelled by decreasing degree, the hottest columns of the
// row.  Rows that share hot columns then sit next to each other, so a row
// of A^T (a column of A) gathers from fewer cache lines of y.  Ties fall
// back to the caller's order, so the labels are deterministic.  (Mixing row
// lengths inside a stream block was measured not to slow the products.)
std::vector<int32_t> order_rows(const std::vector<int32_t> &rlen, const int32_t *rp,
                                const int32_t *col, const std::vector<int32_t> &new_col,
                                bool reorder) {
    std::vector<int32_t> order = order_by_count(rlen, reorder);
    if (!reorder) return order;
    const int32_t m = (int32_t)rlen.size();
    constexpr uint64_t kNone = (1ull << 25) - 1;
    // key: 25 bits of each of the two hottest labels, 14 of the third (labels < 2^25,
    // beyond that the key only groups rows coarser)
    auto key_of = [&](int32_t i) -> uint64_t {
        uint64_t k[3] = {kNone, kNone, kNone};
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            uint64_t v = std::min<uint64_t>((uint64_t)new_col[col[e]], kNone - 1);
            if (v < k[2]) {
                k[2] = v;
                if (k[2] < k[1]) std::swap(k[1], k[2]);
                if (k[1] < k[0]) std::swap(k[0], k[1]);
            }
        }
        return (k[0] << 39) | (k[1] << 14) | (k[2] >> 11);
    };
    int32_t lo = 0;
    while (lo < m) {
        int32_t hi = lo;
        const int32_t len = rlen[order[lo]];
        const bool stream = len <= pdlp::kMedRow;   // one group for all stream rows
        while (hi < m && (stream ? rlen[order[hi]] <= pdlp::kMedRow : rlen[order[hi]] == len)) ++hi;
        if (stream && hi - lo > 1) {
            std::vector<std::pair<uint64_t, int32_t>> kv((size_t)(hi - lo));
            parallel_for(hi - lo, [&](int64_t a, int64_t b) {
                for (int64_t q = a; q < b; ++q) kv[(size_t)q] = {key_of(order[lo + q]), order[lo + q]};
            });
            parallel_sort(kv);
            for (int32_t q = lo; q < hi; ++q) order[q] = kv[(size_t)(q - lo)].second;
        }
        lo = hi;
    }
    return order;
}

// Column labels: decreasing degree (hot columns first, and at low labels,
// where the rows' keys above look); inside a class of equal degree, by the
// smallest new label of the column's rows.  The cold columns (degree at most
// kColdDeg, most of them of degree 1 or 2) form one class, ordered by that
// first row alone, so that all cold columns of a row sit next to each other
// and a row of A gathers them from one run of cache lines of x.
constexpr int32_t kColdDeg = 8;
std::vector<int32_t> order_cols(const std::vector<int32_t> &cdeg, const int32_t *rp,
                                const int32_t *col, int32_t m,
                                const std::vector<int32_t> &new_row, bool reorder) {
    std::vector<int32_t> order = order_by_count(cdeg, reorder);
    if (!reorder) return order;
    const int32_t n = (int32_t)cdeg.size();
    std::vector<int32_t> first(n, std::numeric_limits<int32_t>::max());
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) first[col[e]] = std::min(first[col[e]], new_row[i]);
    int32_t lo = 0;
    while (lo < n) {
        int32_t hi = lo;
        const int32_t d = cdeg[order[lo]];
        if (d <= kColdDeg)
            hi = n;   // degrees decrease along order: the rest are all cold
        else
            while (hi < n && cdeg[order[hi]] == d) ++hi;
        if (hi - lo > 1) {
            std::vector<std::pair<int32_t, int32_t>> kv((size_t)(hi - lo));
            for (int32_t q = lo; q < hi; ++q) kv[(size_t)(q - lo)] = {first[order[q]], order[q]};
            parallel_sort(kv);
            for (int32_t q = lo; q < hi; ++q) order[q] = kv[(size_t)(q - lo)].second;
        }
        lo = hi;
    }
    return order;
}

// Two-phase layout (pdlp::SegCsr) of M for products with a gathered vector
// of M.cols entries.  Segments: S = 8 * ceil(cols / 2^18 / 8) (at most 128)
// contiguous index ranges balanced by nonzeros (each at most 2^19 indices
// unless the balance needs more), segment s belonging to XCD s mod 8.
// Pairs: a row of at most kMedRow nonzeros gives one pair per nonzero in
// stored order; a longer row one pair per segment it touches, in segment
// order, its entries in stored order.  Phase-2 blocks: consecutive rows with
// at most kStage pairs and kMaxBlockRows rows.  Q order: single-entry pairs
// first, then the others; inside each class by segment, then block, then
// position in the block.  Phase-1 work of segment s (chunks of at most
// kStage singles, then blocks of G) is listed for XCD s mod 8.  Values are
// taken from M.val on the device (call after scaling).
void build_segmented(pdlp_problem *P, const DCsr &M, pdlp::SegCsr &sg) {
    hipStream_t s = P->stream;
    const int32_t R = M.rows, C = M.cols;
    const int64_t nnz = M.nnz;
    if (nnz == 0 || R == 0 || C == 0) return;
    std::vector<int32_t> rp((size_t)R + 1), col((size_t)nnz);
    HIPCHECK(hipMemcpyAsync(rp.data(), M.row_ptr, sizeof(int32_t) * rp.size(),
                            hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(col.data(), M.col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
#ifndef PDLP_SEG_LEN_LOG2
#define PDLP_SEG_LEN_LOG2 18
#endif
    constexpr int64_t kSegLen = 1 << PDLP_SEG_LEN_LOG2;
    constexpr int kMaxSeg = 128;
    int S = (int)std::min<int64_t>(kMaxSeg, (C + kSegLen - 1) / kSegLen);
    S = std::min(kMaxSeg, (S + 7) / 8 * 8);
    if (C < S) return;
    // segments balanced by nonzeros
    std::vector<int64_t> cnt((size_t)C, 0);
    for (int64_t e = 0; e < nnz; ++e) cnt[(size_t)col[(size_t)e]] += 1;
    std::vector<uint8_t> seg_of((size_t)C);
    {
        int64_t rem = nnz;
        int32_t i = 0;
        for (int k = 0; k < S; ++k) {
            const int32_t lo = i;
            if (k == S - 1) {
                i = C;
            } else {
                const int64_t target = rem / (S - k);
                const int64_t max_end =
                    std::min<int64_t>((int64_t)C - (S - 1 - k), (int64_t)i + 2 * kSegLen);
                int64_t e = 0;
                while (i < max_end && (e == 0 || e + cnt[(size_t)i] <= target)) e += cnt[(size_t)i++];
                rem -= e;
            }
            for (int32_t q = lo; q < i; ++q) seg_of[(size_t)q] = (uint8_t)k;
        }
    }
    // pairs in pair-space order (rows in order)
    std::vector<int32_t> prp((size_t)R + 1, 0);
    std::vector<uint8_t> pseg;
    std::vector<int32_t> pn;               // entries per pair
    std::vector<int32_t> ent((size_t)nnz); // entries in pair-space order
    pseg.reserve((size_t)nnz);
    pn.reserve((size_t)nnz);
    {
        std::vector<int32_t> sc((size_t)S), so((size_t)S);
        int64_t k = 0;
        for (int32_t r = 0; r < R; ++r) {
            const int32_t a = rp[(size_t)r], z = rp[(size_t)r + 1];
            if (z - a <= pdlp::kMedRow) {
                for (int32_t e = a; e < z; ++e) {
                    pseg.push_back(seg_of[(size_t)col[(size_t)e]]);
                    pn.push_back(1);
                    ent[(size_t)k++] = e;
                }
            } else {
                std::fill(sc.begin(), sc.end(), 0);
                for (int32_t e = a; e < z; ++e) sc[seg_of[(size_t)col[(size_t)e]]] += 1;
                int32_t acc = 0;
                for (int q = 0; q < S; ++q) {
                    so[(size_t)q] = acc;
                    acc += sc[(size_t)q];
                    if (sc[(size_t)q] > 0) {
                        pseg.push_back((uint8_t)q);
                        pn.push_back(sc[(size_t)q]);
                    }
                }
                for (int32_t e = a; e < z; ++e)
                    ent[(size_t)(k + so[seg_of[(size_t)col[(size_t)e]]]++)] = e;
                k += z - a;
            }
            prp[(size_t)r + 1] = (int32_t)pseg.size();
        }
    }
    const int64_t NP = (int64_t)pseg.size();
    std::vector<int64_t> pent((size_t)NP + 1, 0);
    for (int64_t p = 0; p < NP; ++p) pent[(size_t)p + 1] = pent[(size_t)p] + pn[(size_t)p];
    // phase-2 blocks
    std::vector<int32_t> blk2{0};
    for (int32_t r = 0; r < R;) {
        const int32_t first = r;
        while (r < R && r - first < pdlp::kMaxBlockRows &&
               prp[(size_t)r + 1] - prp[(size_t)first] <= pdlp::kStage)
            ++r;
        blk2.push_back(r);
    }
    const int32_t NB = (int32_t)blk2.size() - 1;
    // Q order, run starts and slots; class c = 0 single-entry pairs, 1 the others
    const int RS = 2 * S;  // runs per block
    std::vector<int64_t> ccount((size_t)RS, 0);
    for (int64_t p = 0; p < NP; ++p) ccount[(size_t)((pn[(size_t)p] > 1) * S + pseg[(size_t)p])] += 1;
    std::vector<int64_t> cstart((size_t)RS + 1, 0);
    for (int q = 0; q < RS; ++q) cstart[(size_t)q + 1] = cstart[(size_t)q] + ccount[(size_t)q];
    const int64_t N1 = cstart[(size_t)S];
    std::vector<int32_t> qoff(((size_t)NB + 1) * RS);
    std::vector<int64_t> next(cstart.begin(), cstart.end() - 1);
    std::vector<int32_t> pair_of_q((size_t)NP);
    std::vector<uint16_t> slot((size_t)NP);
    for (int32_t b = 0; b < NB; ++b) {
        for (int q = 0; q < RS; ++q) qoff[(size_t)b * RS + q] = (int32_t)next[(size_t)q];
        const int32_t p0 = prp[(size_t)blk2[(size_t)b]], p1 = prp[(size_t)blk2[(size_t)b + 1]];
        for (int32_t p = p0; p < p1; ++p) {
            const int64_t qi = next[(size_t)((pn[(size_t)p] > 1) * S + pseg[(size_t)p])]++;
            pair_of_q[(size_t)qi] = p;
            slot[(size_t)qi] = (uint16_t)(p - p0);
        }
    }
    for (int q = 0; q < RS; ++q) qoff[(size_t)NB * RS + q] = (int32_t)next[(size_t)q];
    // singles: gathered index and source entry
    std::vector<int32_t> c1((size_t)std::max<int64_t>(N1, 1));
    std::vector<int64_t> src1((size_t)std::max<int64_t>(N1, 1));
    for (int64_t qi = 0; qi < N1; ++qi) {
        const int32_t e = ent[(size_t)pent[(size_t)pair_of_q[(size_t)qi]]];
        c1[(size_t)qi] = col[(size_t)e];
        src1[(size_t)qi] = e;
    }
    // G: one row per multi-entry pair in Q order
    const int64_t N2 = NP - N1;
    const int64_t nnz2 = nnz - N1;
    std::vector<int32_t> grp((size_t)N2 + 1, 0), gcol((size_t)std::max<int64_t>(nnz2, 1));
    std::vector<int64_t> gsrc((size_t)std::max<int64_t>(nnz2, 1));
    {
        int64_t k = 0;
        for (int64_t t = 0; t < N2; ++t) {
            const int32_t p = pair_of_q[(size_t)(N1 + t)];
            for (int64_t u = pent[(size_t)p]; u < pent[(size_t)p + 1]; ++u) {
                const int32_t e = ent[(size_t)u];
                gcol[(size_t)k] = col[(size_t)e];
                gsrc[(size_t)k] = e;
                ++k;
            }
            grp[(size_t)t + 1] = (int32_t)k;
        }
    }
    std::vector<int32_t> gbreaks((size_t)S);
    for (int q = 0; q < S; ++q) gbreaks[(size_t)q] = (int32_t)(cstart[(size_t)S + q] - N1);
    std::vector<int32_t> gblk = make_blocks(grp.data(), (int32_t)N2, &gbreaks, pdlp::kStage);
    const int32_t GB = (int32_t)gblk.size() - 1;
    // phase-1 work items by XCD: per segment, its singles in equal chunks, then
    // its G blocks; each segment's chunks and blocks are padded (-1) to a
    // multiple of the XCD's workgroups (kWgPerXcd: the persistent grid of
    // 2048 on 8 XCDs), so that every workgroup of the XCD takes the same
    // number of chunks and of blocks of a segment and the XCD's workgroups
    // move from one segment to the next together (its L2 then holds one
    // segment of v at a time)
    constexpr int64_t kWgPerXcd = PDLP_STREAM_GRID_CAP / 8;
    std::vector<int32_t> chunks;
    std::vector<std::vector<int32_t>> lx(8);
    {
        auto pad = [&](std::vector<int32_t> &L) {
            while ((int64_t)L.size() % kWgPerXcd) L.push_back(-1);
        };
        int32_t gb = 0;
        for (int q = 0; q < S; ++q) {
            auto &L = lx[(size_t)(q % 8)];
            const int64_t lo = cstart[(size_t)q], hi = cstart[(size_t)q + 1];
            if (hi > lo) {
                int64_t nch = (hi - lo + pdlp::kStage - 1) / pdlp::kStage;
                nch = (nch + kWgPerXcd - 1) / kWgPerXcd * kWgPerXcd;
                const int64_t csz = (hi - lo + nch - 1) / nch;
                for (int64_t k = 0; k < nch; ++k) {
                    const int64_t a = std::min(hi, lo + k * csz), z = std::min(hi, a + csz);
                    if (z > a) {
                        L.push_back(-2 - (int32_t)(chunks.size() / 2));
                        chunks.push_back((int32_t)a);
                        chunks.push_back((int32_t)z);
                    } else {
                        L.push_back(-1);
                    }
                }
            }
            const int32_t gend = q + 1 < S ? gbreaks[(size_t)q + 1] : (int32_t)N2;
            const size_t before = L.size();
            for (; gb < GB && gblk[(size_t)gb] < gend; ++gb) L.push_back(gb);
            if (L.size() > before) pad(L);
        }
    }
    size_t T = 0;
    for (auto &v : lx) T = std::max(T, v.size());
    std::vector<int32_t> glist(8 * T, -1);
    for (size_t t = 0; t < T; ++t)
        for (int x = 0; x < 8; ++x)
            if (t < lx[(size_t)x].size()) glist[t * 8 + (size_t)x] = lx[(size_t)x][t];
    // upload
    Arena &a = P->arena;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    };
    sg.n1 = N1;
    int32_t *c1d = a.dev<int32_t>(std::max<int64_t>(N1, 1));
    double *v1d = a.dev<double>(std::max<int64_t>(N1, 1));
    up(c1d, c1.data(), sizeof(int32_t) * N1);
    sg.c1 = c1d;
    sg.v1 = v1d;
    int32_t *chd = a.dev<int32_t>(std::max<size_t>(chunks.size(), 1));
    up(chd, chunks.data(), sizeof(int32_t) * chunks.size());
    sg.chunk = chd;
    DCsr &G = sg.G;
    G.rows = (int32_t)N2;
    G.cols = C;
    G.nnz = nnz2;
    G.row_ptr = a.dev<int32_t>((size_t)N2 + 1);
    G.col = a.dev<int32_t>(std::max<int64_t>(nnz2, 1));
    G.val = a.dev<double>(std::max<int64_t>(nnz2, 1));
    G.nblk = GB;
    G.blk = a.dev<int32_t>(gblk.size());
    G.grid = 0;  // G is walked through glist only
    up(G.row_ptr, grp.data(), sizeof(int32_t) * grp.size());
    up(G.col, gcol.data(), sizeof(int32_t) * nnz2);
    up(G.blk, gblk.data(), sizeof(int32_t) * gblk.size());
    int32_t *gl = a.dev<int32_t>(std::max<size_t>(glist.size(), 1));
    up(gl, glist.data(), sizeof(int32_t) * glist.size());
    sg.glist = gl;
    sg.glen = (int32_t)glist.size();
    sg.grid1 = (int32_t)std::min<size_t>(glist.size(), PDLP_STREAM_GRID_CAP);
    sg.Q = a.dev<double>(NP);
    uint16_t *sl = a.dev<uint16_t>(NP);
    up(sl, slot.data(), sizeof(uint16_t) * NP);
    sg.slot = sl;
    int32_t *qo = a.dev<int32_t>(qoff.size());
    up(qo, qoff.data(), sizeof(int32_t) * qoff.size());
    sg.qoff = qo;
    DCsr &PP = sg.P;
    PP.rows = R;
    PP.cols = C;
    PP.nnz = NP;
    PP.row_ptr = a.dev<int32_t>((size_t)R + 1);
    up(PP.row_ptr, prp.data(), sizeof(int32_t) * prp.size());
    PP.nblk = NB;
    PP.blk = a.dev<int32_t>(blk2.size());
    up(PP.blk, blk2.data(), sizeof(int32_t) * blk2.size());
    PP.grid = std::min<int32_t>(NB, PDLP_STREAM_GRID_CAP);
    {
        Arena tmp;
        int64_t *src = tmp.dev<int64_t>(std::max<int64_t>(std::max(N1, nnz2), 1));
        if (N1 > 0) {
            up(src, src1.data(), sizeof(int64_t) * N1);
            HIPCHECK(pdlp::launch_take(s, N1, src, M.val, v1d));
            HIPCHECK(hipStreamSynchronize(s));
        }
        if (nnz2 > 0) {
            up(src, gsrc.data(), sizeof(int64_t) * nnz2);
            HIPCHECK(pdlp::launch_take(s, nnz2, src, M.val, G.val));
            HIPCHECK(hipStreamSynchronize(s));
        }
    }
    sg.S = S;
}

// [hot-path layout end]

}  // namespace

// ===================================================================== problem

void pdlp::host::validate(int32_t m, int32_t n, int64_t nnz, const int32_t *rp,
                          const int32_t *col, const double *val, const double *c,
                          const double *lc, const double *uc, const double *lv,
                          const double *uv) {
    if (m < 0 || n < 1) invalid("need m >= 0 and n >= 1");
    if (nnz < 0 || nnz > (int64_t)std::numeric_limits<int32_t>::max())
        invalid("nnz must lie in [0, 2^31)");
    if (!rp || (nnz > 0 && (!col || !val)) || !c || (m > 0 && (!lc || !uc)) || !lv || !uv)
        invalid("NULL input array");
    if (rp[0] != 0) invalid("row_ptr[0] must be 0");
    for (int32_t i = 0; i < m; ++i)
        if (rp[i + 1] < rp[i]) invalid("row_ptr must be nondecreasing (row " + std::to_string(i) + ")");
    if ((int64_t)rp[m] != nnz) invalid("row_ptr[m] must equal nnz");
    for (int32_t i = 0; i < m; ++i) {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n)
                invalid("column index out of range in row " + std::to_string(i));
            if (e > rp[i] && col[e] <= col[e - 1])
                invalid("columns must be strictly increasing within row " + std::to_string(i));
            if (!std::isfinite(val[e])) invalid("non-finite matrix value in row " + std::to_string(i));
        }
    }
    for (int32_t j = 0; j < n; ++j) {
        if (!std::isfinite(c[j])) invalid("non-finite objective coefficient " + std::to_string(j));
        if (std::isnan(lv[j]) || std::isnan(uv[j])) invalid("NaN variable bound");
        if (lv[j] == INFINITY || uv[j] == -INFINITY) invalid("variable bound of wrong infinity");
        if (lv[j] > uv[j]) invalid("lv > uv for variable " + std::to_string(j));
    }
    for (int32_t i = 0; i < m; ++i) {
        if (std::isnan(lc[i]) || std::isnan(uc[i])) invalid("NaN constraint bound");
        if (lc[i] == INFINITY || uc[i] == -INFINITY) invalid("constraint bound of wrong infinity");
        if (lc[i] > uc[i]) invalid("lc > uc for row " + std::to_string(i));
    }
}

namespace {

std::vector<int32_t> upload_blocks(pdlp_problem *P, Arena &arena, DCsr &M, const int32_t *rp_host,
                                   const std::vector<int32_t> *breaks, int32_t stage,
                                   int32_t med_row = pdlp::kMedRow) {
    std::vector<int32_t> blk =
        make_blocks(rp_host, M.rows, breaks, stage, pdlp::kMaxBlockRows, med_row);
    M.med_row = med_row;
    M.stage = stage;
    M.nblk = (int32_t)blk.size() - 1;
    M.blk = arena.dev<int32_t>(blk.size());
    HIPCHECK(hipMemcpyAsync(M.blk, blk.data(), blk.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, P->stream));
    M.grid = std::min<int32_t>(M.nblk, PDLP_STREAM_GRID_CAP);
    HIPCHECK(hipStreamSynchronize(P->stream));
    return blk;
}

// Block partition of M: kStage nonzeros per stream block (stream_block =
// 0), a fixed size, or autotuned (-1): each candidate partition times five
// plain products on the device after one warm-up, and the fastest is kept.
// (Measured: smaller blocks do not pay on the workloads here -- on the
// 1,000 x 2,000 LP 256-nonzero blocks cut the step time by 8% while the
// changed order of the norm partials cost 12% more steps, and the tail of
// the batch runs 1.5x slower with them.)
std::vector<int32_t> choose_blocks(pdlp_problem *P, DCsr &M, const int32_t *rp_host,
                                   const std::vector<int32_t> *breaks, int32_t stream_block) {
    if (stream_block > 0) return upload_blocks(P, P->arena, M, rp_host, breaks, stream_block);
    if (stream_block == 0 || M.nnz == 0)
        return upload_blocks(P, P->arena, M, rp_host, breaks, pdlp::kStage);
    Arena tmp;
    double *x = tmp.dev<double>(std::max(M.cols, 1));
    double *y = tmp.dev<double>(std::max(M.rows, 1));
    HIPCHECK(pdlp::launch_fill(P->stream, std::max(M.cols, 1), x, 1.0));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    int32_t best = pdlp::kStage;
    float best_ms = INFINITY;
    for (int32_t cand = 256; cand <= pdlp::kStage; cand *= 2) {
        Arena blk_arena;
        upload_blocks(P, blk_arena, M, rp_host, breaks, cand);
        HIPCHECK(pdlp::launch_spmv_plain(P->stream, M, x, y));
        HIPCHECK(hipEventRecord(e0, P->stream));
        for (int r = 0; r < 5; ++r) HIPCHECK(pdlp::launch_spmv_plain(P->stream, M, x, y));
        HIPCHECK(hipEventRecord(e1, P->stream));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return upload_blocks(P, P->arena, M, rp_host, breaks, best);
}

// A^T from the caller-order entries: a stable radix sort by new column label
// keeps, inside every row of A^T, the caller's row order (the summation
// order of a sequential A^T y); columns of A^T carry the new row labels.
void build_transpose(pdlp_problem *P, const int32_t *rp0, const int32_t *col0, const double *val0,
                     const int32_t *new_row, const int32_t *new_col) {
    hipStream_t s = P->stream;
    const int64_t nnz = P->nnz;
    DCsr &T = P->AT;
    T.rows = P->n;
    T.cols = P->m;
    T.nnz = nnz;
    T.row_ptr = P->arena.dev<int32_t>((size_t)P->n + 1);
    T.col = P->arena.dev<int32_t>(nnz);
    T.val = P->arena.dev<double>(nnz);
    if (nnz == 0) {
        HIPCHECK(hipMemsetAsync(T.row_ptr, 0, sizeof(int32_t) * ((size_t)P->n + 1), s));
        HIPCHECK(hipStreamSynchronize(s));
        return;
    }
    Arena tmp;
    int32_t *rowid = tmp.dev<int32_t>(nnz);
    uint32_t *keys_in = tmp.dev<uint32_t>(nnz);
    uint32_t *keys_out = tmp.dev<uint32_t>(nnz);
    int32_t *vals_in = tmp.dev<int32_t>(nnz);
    int32_t *vals_out = tmp.dev<int32_t>(nnz);
    HIPCHECK(pdlp::launch_row_ids_mapped(s, P->m, rp0, new_row, rowid));
    HIPCHECK(pdlp::launch_relabel(s, nnz, col0, new_col, keys_in));
    HIPCHECK(pdlp::launch_iota(s, nnz, vals_in));
    int key_bits = 1;
    while (key_bits < 31 && (1LL << key_bits) <= (long long)P->n) ++key_bits;
    int32_t *temp = tmp.dev<int32_t>((size_t)pdlp::radix_sort_temp_ints(nnz));
    uint32_t *keys[2] = {keys_in, keys_out};
    int32_t *vals[2] = {vals_in, vals_out};
    int which = 0;
    HIPCHECK(pdlp::radix_sort_pairs(s, nnz, key_bits, keys, vals, temp, &which));
    HIPCHECK(pdlp::launch_transpose_finish(s, nnz, P->n, reinterpret_cast<const int32_t *>(keys[which]),
                                           vals[which], rowid, val0, T.row_ptr, T.col, T.val));
    HIPCHECK(hipStreamSynchronize(s));
}

// host vector in caller order -> device vector in internal order (dst[i] = src[perm[i]])
void upload_perm(pdlp_problem *P, const double *host, int64_t len, const int32_t *perm,
                 double *dst) {
    if (len <= 0) return;
    Arena tmp;
    double *t = tmp.dev<double>(len);
    HIPCHECK(hipMemcpyAsync(t, host, sizeof(double) * len, hipMemcpyHostToDevice, P->stream));
    HIPCHECK(pdlp::launch_gather(P->stream, len, perm, t, dst));
    HIPCHECK(hipStreamSynchronize(P->stream));
}

// device vector in internal order -> host vector in caller order (host[perm[i]] = src[i])
void download_unperm(pdlp_problem *P, const double *src, int64_t len, const int32_t *perm,
                     double *host) {
    if (len <= 0 || !host) return;
    Arena tmp;
    double *t = tmp.dev<double>(len);
    HIPCHECK(pdlp::launch_scatter(P->stream, len, perm, src, t));
    HIPCHECK(hipMemcpyAsync(host, t, sizeof(double) * len, hipMemcpyDeviceToHost, P->stream));
    HIPCHECK(hipStreamSynchronize(P->stream));
}

double reduce_result(pdlp_problem *P, int idx = 0) {
    HIPCHECK(hipMemcpyAsync(P->res_h, P->res_d, 8 * sizeof(double), hipMemcpyDeviceToHost,
                            P->stream));
    HIPCHECK(hipStreamSynchronize(P->stream));
    return P->res_h[idx];
}

// Diagonal preconditioning (Section 3): ruiz_iters Ruiz rounds (infinity
// norms) then an optional Pock-Chambolle round (alpha = 1: 1-norms); in each
// round both factors come from the same current matrix, zero norms give 1.
// Row norms of A and of A^T (= column norms of A) are summed one lane per
// row in index order, so the scaled matrix matches a sequential reference.
void precondition(pdlp_problem *P, const pdlp_params &prm) {
    hipStream_t s = P->stream;
    const int m = P->m, n = P->n;
    HIPCHECK(pdlp::launch_fill(s, m, P->d1, 1.0));
    HIPCHECK(pdlp::launch_fill(s, n, P->d2, 1.0));
    Arena tmp;
    double *rn = tmp.dev<double>(m), *cn = tmp.dev<double>(n);
    const int rounds = prm.ruiz_iters + (prm.pock_chambolle ? 1 : 0);
    for (int round = 0; round < rounds; ++round) {
        const int use_inf = round < prm.ruiz_iters;
        HIPCHECK(pdlp::launch_row_norms(s, P->A, use_inf, rn));
        HIPCHECK(pdlp::launch_row_norms(s, P->AT, use_inf, cn));
        HIPCHECK(pdlp::launch_norm_to_factor(s, m, rn));
        HIPCHECK(pdlp::launch_norm_to_factor(s, n, cn));
        HIPCHECK(pdlp::launch_scale_matrix(s, P->A, rn, cn));
        HIPCHECK(pdlp::launch_scale_matrix(s, P->AT, cn, rn));
        HIPCHECK(pdlp::launch_div_inplace(s, m, P->d1, rn));
        HIPCHECK(pdlp::launch_div_inplace(s, n, P->d2, cn));
    }
    HIPCHECK(pdlp::launch_scale_vectors(s, m, n, P->d1, P->d2, P->c, P->lc, P->uc, P->lv, P->uv,
                                        P->cs, P->lcs, P->ucs, P->lvs, P->uvs));
    HIPCHECK(hipStreamSynchronize(s));
}

}  // namespace

// ====================================================================== engine

namespace {

enum { TERM_NONE = 0, TERM_FULL = 1, TERM_PRIMAL = 2, TERM_DUAL = 3 };
enum { RUN_OK = 0, RUN_LIMIT = 1, RUN_TIME = 2, RUN_NUMERR = 3, RUN_PINF = 4, RUN_DINF = 5,
       RUN_POLISHED = 10 };

// A~^T y as the step kernels compute it: the two-phase product when it is
// built, else the one-pass stream product.
hipError_t spmv_t(pdlp_problem *P, hipStream_t s, const double *y, double *out) {
    return P->segT.S ? pdlp::launch_seg_plain(s, P->segT, y, out)
                     : pdlp::launch_spmv_plain(s, P->AT, y, out);
}

// One PDLP run (the main run or a feasibility-polishing run) on the device.
struct Engine {
    pdlp_problem *P = nullptr;
    Vecs v{};
    int m = 0, n = 0;
    Arena arena;
    Iter it{};
    double *x0 = nullptr, *y0 = nullptr, *xb = nullptr, *yb = nullptr, *axb = nullptr,
           *atyb = nullptr, *xp = nullptr, *yp = nullptr;
    Ctrl *ctrl_d = nullptr, *ctrl_h = nullptr;
    double *part_dual = nullptr, *part_ps = nullptr, *part_pf = nullptr;
    int gd = 0, gps = 0, gpf = 0;
    GapState *gap_d = nullptr, *gap_h = nullptr;
    KktOut *kkt_d = nullptr, *kkt_h = nullptr;
    double *gap_part = nullptr;
    int ggrid = 0;
    // infeasibility candidate and its products (allocated at the first test)
    Arena cert_arena;
    double *cx = nullptr, *cy = nullptr, *cax = nullptr, *caty = nullptr;
    pdlp::CertOut *cert_d = nullptr, *cert_h = nullptr;
    double *zero_m = nullptr;  // y = 0 of the Algorithm 5 termination candidate
    // host-side counters of Algorithm 1
    long long n_outer = 0, kkt_passes = 0, restarts_i = 0, restarts_ii = 0, restarts_iii = 0;
    double mu_ref = INFINITY, mu_c_prev = INFINITY;
    // optional HIP-event timing of the step kernels
    bool profile = false;
    // step attempts replayed from graphs (not while profiling), captured for
    // the vectors in v (polishing swaps them)
    bool use_graphs = true;
    pdlp::host::AttemptGraphs graphs;
    Vecs graphs_v{};
    std::vector<hipEvent_t> ev;
    pdlp_kernel_stats kst{};

    Engine(pdlp_problem *p, Vecs vv) : P(p), v(vv), m(p->m), n(p->n) {
        for (int b = 0; b < 2; ++b) {
            it.X[b] = arena.dev<double>(n);
            it.ATY[b] = arena.dev<double>(n);
            it.Y[b] = arena.dev<double>(m);
            it.AX[b] = arena.dev<double>(m);
        }
        it.sx = arena.dev<double>(n);
        it.sy = arena.dev<double>(m);
        x0 = arena.dev<double>(n);
        xb = arena.dev<double>(n);
        atyb = arena.dev<double>(n);
        xp = arena.dev<double>(n);
        y0 = arena.dev<double>(m);
        yb = arena.dev<double>(m);
        axb = arena.dev<double>(m);
        yp = arena.dev<double>(m);
        ctrl_d = arena.dev<Ctrl>(1);
        ctrl_h = arena.host<Ctrl>(1);
        gd = P->A.grid;
        gpf = P->segT.S ? P->segT.P.grid : P->AT.grid;
        gps = red_grid(n);
        part_dual = arena.dev<double>(2 * (size_t)std::max(gd, 1));
        part_pf = arena.dev<double>(std::max(gpf, 1));
        part_ps = arena.dev<double>(gps);
        gap_d = arena.dev<GapState>(4);
        gap_h = arena.host<GapState>(4);
        kkt_d = arena.dev<KktOut>(1);
        kkt_h = arena.host<KktOut>(1);
        ggrid = red_grid((int64_t)m + n);
        gap_part = arena.dev<double>((size_t)ggrid * (2 * pdlp::kGapPts));
        std::memset(ctrl_h, 0, sizeof(Ctrl));
    }
    ~Engine() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }

    hipStream_t s() const { return P->stream; }
    double *X() const { return it.X[ctrl_h->cur]; }
    double *Y() const { return it.Y[ctrl_h->cur]; }
    double *AXc() const { return it.AX[ctrl_h->cur]; }
    double *ATYc() const { return it.ATY[ctrl_h->cur]; }

    void push() {
        HIPCHECK(hipMemcpyAsync(ctrl_d, ctrl_h, sizeof(Ctrl), hipMemcpyHostToDevice, s()));
    }
    void pull() {
        HIPCHECK(hipMemcpyAsync(ctrl_h, ctrl_d, sizeof(Ctrl), hipMemcpyDeviceToHost, s()));
        HIPCHECK(hipStreamSynchronize(s()));
    }

    double dist2(const double *a, const double *b, int64_t len) {
        HIPCHECK(pdlp::launch_dist2(s(), len, a, b, P->red_part, red_grid(len), P->res_d));
        return reduce_result(P);
    }

    // z = (x, y) from host-chosen device vectors; products computed here.
    void set_point(const double *x_src, const double *y_src) {
        Ctrl &c = *ctrl_h;
        c.cur = 0;
        HIPCHECK(pdlp::launch_copy(s(), n, x_src, it.X[0]));
        HIPCHECK(pdlp::launch_copy(s(), m, y_src, it.Y[0]));
        HIPCHECK(pdlp::launch_spmv_plain(s(), P->A, it.X[0], it.AX[0]));
        HIPCHECK(spmv_t(P, s(), it.Y[0], it.ATY[0]));
        HIPCHECK(pdlp::launch_copy(s(), n, it.X[0], x0));
        HIPCHECK(pdlp::launch_copy(s(), m, it.Y[0], y0));
        HIPCHECK(pdlp::launch_fill(s(), n, it.sx, 0.0));
        HIPCHECK(pdlp::launch_fill(s(), m, it.sy, 0.0));
    }

    // Algorithm 1 initialization.  Reading: ||A||_inf in eta_hat^{0,0} is the
    // largest absolute entry of the scaled matrix; the initial point is
    // (proj_X(0), 0) unless a warm start is given.
    void init(double omega, double eta_hat, const pdlp_params &prm) {
        Ctrl &c = *ctrl_h;
        std::memset(&c, 0, sizeof(Ctrl));
        c.eta = eta_hat;
        c.eta_hat = eta_hat;
        c.omega = omega;
        c.red_exp = prm.red_exp;
        c.grow_exp = prm.grow_exp;
        c.need_primal = 1;
        if (prm.restart_period > 0) {
            // Algorithm 5: constant step and primal weight
            c.fixed_step = 1;
            c.fixed_eta = c.eta = c.eta_hat = prm.fixed_step_size;
            c.omega = prm.fixed_primal_weight;
        }
        n_outer = 0;
        kkt_passes = 1;
        restarts_i = restarts_ii = restarts_iii = 0;
        mu_ref = INFINITY;
        mu_c_prev = INFINITY;
    }

    // One step attempt: four predicated launches (five with the two-phase
    // A^T y'); with profiling each launch records its own start/stop events
    // (kEv per attempt).
    static constexpr int kEv = 10;
    void enqueue_attempt_on(hipStream_t st) {
        HIPCHECK(pdlp::launch_primal(st, n, v, it, ctrl_d, part_ps, gps, nullptr));
        HIPCHECK(pdlp::launch_spmv_dual(st, P->A, v, it, ctrl_d, part_dual, nullptr));
        HIPCHECK(pdlp::launch_step_decide(st, ctrl_d, part_dual, gd, part_ps, gps, part_pf, gpf,
                                          nullptr));
        if (P->segT.S)
            HIPCHECK(pdlp::launch_seg_primal(st, P->segT, v, it, ctrl_d, part_pf, nullptr));
        else
            HIPCHECK(pdlp::launch_spmv_primal(st, P->AT, v, it, ctrl_d, part_pf, nullptr));
    }
    void enqueue_attempt(hipEvent_t *e) {
        HIPCHECK(pdlp::launch_primal(s(), n, v, it, ctrl_d, part_ps, gps, e ? e + 0 : nullptr));
        HIPCHECK(pdlp::launch_spmv_dual(s(), P->A, v, it, ctrl_d, part_dual, e ? e + 2 : nullptr));
        HIPCHECK(pdlp::launch_step_decide(s(), ctrl_d, part_dual, gd, part_ps, gps, part_pf, gpf,
                                          e ? e + 4 : nullptr));
        if (P->segT.S)
            HIPCHECK(pdlp::launch_seg_primal(s(), P->segT, v, it, ctrl_d, part_pf,
                                             e ? e + 6 : nullptr));
        else
            HIPCHECK(pdlp::launch_spmv_primal(s(), P->AT, v, it, ctrl_d, part_pf,
                                              e ? e + 6 : nullptr));
    }

    float ev_ms(int a, int b) {
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, ev[a], ev[b]));
        return t;
    }

    // Exactly `target` accepted steps (or a numerical error).
    void run_block(long long target) {
        Ctrl &c = *ctrl_h;
        c.block_target = target;
        c.block_acc = 0;
        c.stop = 0;
        c.need_primal = 1;
        c.run_at = 0;
        push();
        long long remaining = target;
        for (;;) {
            long long n_att = remaining + remaining / 8 + 1;
            if (n_att > 4096) n_att = 4096;
            const long long att0 = c.attempts, acc0 = c.block_acc;
            if (profile) {
                while ((long long)ev.size() < kEv * n_att) {
                    hipEvent_t e;
                    HIPCHECK(hipEventCreate(&e));
                    ev.push_back(e);
                }
            }
            if (profile || !use_graphs) {
                for (long long a = 0; a < n_att; ++a)
                    enqueue_attempt(profile ? &ev[kEv * a] : nullptr);
            } else {
                const bool same = graphs_v.c == v.c && graphs_v.lc == v.lc && graphs_v.uc == v.uc &&
                                  graphs_v.lv == v.lv && graphs_v.uv == v.uv;
                if (!graphs.ready() || !same) {
                    graphs.capture([&](hipStream_t st) { enqueue_attempt_on(st); });
                    graphs_v = v;
                }
                graphs.launch(s(), n_att);
            }
            pull();
            if (profile) {
                const long long ran = c.attempts - att0;
                for (long long a = 0; a < ran; ++a) {
                    const int b = (int)(kEv * a);
                    kst.standalone_primal_ms += ev_ms(b, b + 1);
                    kst.dual_ms += ev_ms(b + 2, b + 3);
                    kst.decide_ms += ev_ms(b + 4, b + 5);
                    kst.primal_ms += ev_ms(b + 6, b + 7);
                    if (P->segT.S) {
                        kst.primal_gather_ms += ev_ms(b + 6, b + 7);
                        kst.primal_ms += ev_ms(b + 8, b + 9);
                    }
                }
                kst.attempts += ran;
                kst.dual_launches += ran;
                kst.primal_launches += c.block_acc - acc0;
            }
            if (c.stop) break;
            remaining = target - c.block_acc;
        }
        kkt_passes += c.block_acc;
        if (c.pending_sy && !c.numerr) {
            HIPCHECK(pdlp::launch_flush_sy(s(), m, it, ctrl_d));
            c.pending_sy = 0;
        }
    }

    void average() {
        const double seta = ctrl_h->seta;
        HIPCHECK(pdlp::launch_average(s(), n, it.sx, seta, xb));
        HIPCHECK(pdlp::launch_average(s(), m, it.sy, seta, yb));
        HIPCHECK(pdlp::launch_spmv_plain(s(), P->A, xb, axb));
        HIPCHECK(spmv_t(P, s(), yb, atyb));
        kkt_passes += 1;
    }

    // Gap evaluations: the head of each (setup and the first active-set
    // steps) is enqueued at once; gap_fetch reads the states and enqueues the
    // tail (further steps, multisection, final segment) only for evaluations
    // that have not finished, instead of launches that would do nothing.
    struct GapArgs {
        const double *x, *y, *ax, *aty;
        bool live;
    };
    GapArgs gap_args[4] = {};
    void gap_enqueue(int slot, const double *x, const double *y, const double *ax,
                     const double *aty, const double *xr, const double *yr, double omega) {
        HIPCHECK(pdlp::launch_gap_head(s(), m, n, v, x, y, ax, aty, xr, yr, omega, gap_part,
                                       ggrid, gap_d + slot));
        gap_args[slot] = GapArgs{x, y, ax, aty, true};
    }
    void gap_fetch() {
        HIPCHECK(hipMemcpyAsync(gap_h, gap_d, 4 * sizeof(GapState), hipMemcpyDeviceToHost, s()));
        HIPCHECK(hipStreamSynchronize(s()));
        bool more = false;
        for (int k = 0; k < 4; ++k) {
            const GapArgs &g = gap_args[k];
            if (g.live && (gap_h[k].done == 0 || gap_h[k].done == 1)) {
                HIPCHECK(pdlp::launch_gap_tail(s(), m, n, v, g.x, g.y, g.ax, g.aty, gap_part,
                                               ggrid, gap_d + k));
                more = true;
            }
            gap_args[k].live = false;
        }
        if (more) {
            HIPCHECK(hipMemcpyAsync(gap_h, gap_d, 4 * sizeof(GapState), hipMemcpyDeviceToHost,
                                    s()));
            HIPCHECK(hipStreamSynchronize(s()));
        }
    }

    // Infeasibility candidate c (0 difference of the two latest iterates,
    // 1 current iterate, 2 average since the restart) projected onto
    // Xbar x Y, with its products, at (cpx, cpy, cpax, cpaty).  After an
    // accepted step the other buffer of the pair still holds the previous
    // iterate: the step that ends a block does not start the next primal
    // update.  The iterate's and the average's y already lie in Y (the dual
    // step and averaging keep it there), so their cached A^T y serve; x needs
    // its projection (boxed coordinates go to 0) and a fresh product.
    // Without a variable that has an infinite bound, Xbar = {0}: every x
    // candidate projects to 0 and the dual test cannot pass, so the x part
    // and its product are skipped (null pointers read as 0).
    const double *cpx = nullptr, *cpy = nullptr, *cpax = nullptr, *cpaty = nullptr;
    void cert_point(int c) {
        if (!cx) {
            cx = cert_arena.dev<double>(n);
            caty = cert_arena.dev<double>(n);
            cy = cert_arena.dev<double>(m);
            cax = cert_arena.dev<double>(m);
            cert_d = cert_arena.dev<pdlp::CertOut>(3);
            cert_h = cert_arena.host<pdlp::CertOut>(3);
        }
        const int cur = ctrl_h->cur;
        const bool xs = P->ray_cols > 0;
        if (c == 0) {
            HIPCHECK(pdlp::launch_cert_point(s(), m, xs ? n : 0, it.X[cur], it.X[cur ^ 1],
                                             it.Y[cur], it.Y[cur ^ 1], P->lc, P->uc, P->lv, P->uv,
                                             cx, cy));
            HIPCHECK(spmv_t(P, s(), cy, caty));
            cpy = cy;
            cpaty = caty;
        } else {
            if (xs)
                HIPCHECK(pdlp::launch_cert_point(s(), 0, n, c == 1 ? it.X[cur] : xb, nullptr,
                                                 nullptr, nullptr, P->lc, P->uc, P->lv, P->uv, cx,
                                                 nullptr));
            cpy = c == 1 ? it.Y[cur] : yb;
            cpaty = c == 1 ? it.ATY[cur] : atyb;
        }
        if (xs) HIPCHECK(pdlp::launch_spmv_plain(s(), P->A, cx, cax));
        cpx = xs ? cx : nullptr;
        cpax = xs ? cax : nullptr;
    }

    // Appendix D tests of the three candidates: primal infeasibility on each
    // in order, then dual infeasibility.  Returns RUN_PINF, RUN_DINF or 0 and
    // the certifying candidate (1-based) with its values.
    int infeasible(double eps, int &src, pdlp::CertOut &val) {
        for (int c = 0; c < 3; ++c) {
            cert_point(c);
            HIPCHECK(pdlp::launch_cert(s(), m, n, cpx, cpy, cpax, cpaty, P->d1, P->d2, P->c,
                                       P->lc, P->uc, P->lv, P->uv, P->red_part,
                                       red_grid((int64_t)m + n), cert_d + c));
        }
        HIPCHECK(hipMemcpyAsync(cert_h, cert_d, 3 * sizeof(pdlp::CertOut), hipMemcpyDeviceToHost,
                                s()));
        HIPCHECK(hipStreamSynchronize(s()));
        kkt_passes += 3;
        for (int pass = 0; pass < 2; ++pass) {
            for (int c = 0; c < 3; ++c) {
                const pdlp::CertOut &o = cert_h[c];
                if (o.nonfinite > 0.0) continue;
                const bool ok = pass == 0 ? (std::isfinite(o.pobj) && o.pobj > 0.0 &&
                                             o.pres <= eps * o.pobj)
                                          : (std::isfinite(o.dobj) && o.dobj < 0.0 &&
                                             o.dres <= eps * std::fabs(o.dobj));
                if (!ok) continue;
                src = c + 1;
                val = o;
                return pass == 0 ? RUN_PINF : RUN_DINF;
            }
        }
        return 0;
    }

    KktOut kkt(const double *x, const double *y, const double *ax, const double *aty, int mode,
               double *r_out = nullptr, double *x_out = nullptr, double *y_out = nullptr) {
        HIPCHECK(pdlp::launch_kkt(s(), m, n, x, y, ax, aty, P->d1, P->d2, P->c, P->lc, P->uc,
                                  P->lv, P->uv, mode, P->obj_offset, P->red_part,
                                  red_grid((int64_t)m + n), r_out, x_out, y_out, kkt_d));
        HIPCHECK(hipMemcpyAsync(kkt_h, kkt_d, sizeof(KktOut), hipMemcpyDeviceToHost, s()));
        HIPCHECK(hipStreamSynchronize(s()));
        return *kkt_h;
    }
};

struct Candidate {
    const double *x, *y, *ax, *aty;
};

struct RunOut {
    Candidate cand{};
    KktOut kkt{};
    bool have = false;
    int cert_src = 0;             // infeasibility certificate: candidate 1..3
    pdlp::CertOut cert{};
};

bool term_met(const pdlp_params &prm, int mode, const KktOut &k) {
    const double e = prm.eps_feas;
    if (mode == TERM_PRIMAL) return k.primal_res_rel <= e;
    if (mode == TERM_DUAL) return k.dual_res_rel <= e;
    return k.primal_res_rel <= e && k.dual_res_rel <= e && k.rel_gap <= prm.eps_gap;
}

int effective_rc_mode(const pdlp_params &prm) {
    if (prm.reduced_cost_mode >= 0) return prm.reduced_cost_mode;
    return prm.polish ? 0 : 1;
}


// Buffers of feasibility polishing, created on first use and kept.
struct PolishBufs {
    Engine *sub = nullptr;
    Arena *store = nullptr;
    double *pol_x = nullptr, *pol_ax = nullptr, *pol_y = nullptr, *pol_aty = nullptr;
    double *zero_m = nullptr;
    ~PolishBufs() {
        delete sub;
        delete store;
    }
};

struct Ctx {
    pdlp_problem *P;
    const pdlp_params *prm;
    double t_start;
    pdlp_result *res;
    PolishBufs *pb;
};

int run_loop(Ctx &X, Engine &E, long long max_k, int term_mode, bool allow_polish, RunOut &out);

// Feasibility polishing (Algorithm 4): primal feasibility LP (c = 0) from
// (x_bar, 0), then dual feasibility LP (finite bounds set to 0) from (0, y_bar),
// each for at most floor(k/8) accepted steps with the current omega and
// eta_hat, then the polished pair must meet the full termination criteria.
bool feasibility_polish(Ctx &X, Engine &E, RunOut &out) {
    pdlp_problem *P = X.P;
    const pdlp_params &prm = *X.prm;
    const long long cap = E.ctrl_h->k / 8;
    X.res->polish_attempts += 1;
    PolishBufs &B = *X.pb;
    if (!B.sub) {
        B.store = new Arena();
        B.pol_x = B.store->dev<double>(P->n);
        B.pol_aty = B.store->dev<double>(P->n);
        B.pol_y = B.store->dev<double>(P->m);
        B.pol_ax = B.store->dev<double>(P->m);
        B.zero_m = B.store->dev<double>(P->m);
        HIPCHECK(pdlp::launch_fill(P->stream, P->m, B.zero_m, 0.0));
        B.sub = new Engine(P, P->scaled());
    }
    Engine &S = *B.sub;
    S.profile = false;
    S.use_graphs = prm.graphs != 0;
    pdlp_params p2 = prm;
    p2.polish = 0;
    p2.reduced_cost_mode = 0;
    Ctx X2 = X;
    X2.prm = &p2;
    bool ok = false;
    // primal feasibility problem
    S.v = Vecs{P->zero_n, P->lcs, P->ucs, P->lvs, P->uvs};
    S.init(E.ctrl_h->omega, E.ctrl_h->eta_hat, prm);
    S.set_point(E.xb, B.zero_m);
    RunOut o1;
    int rc = run_loop(X2, S, cap, TERM_PRIMAL, false, o1);
    X.res->polish_iters += S.ctrl_h->k;
    E.kkt_passes += S.kkt_passes;
    if (rc == RUN_OK) {
        HIPCHECK(pdlp::launch_copy(P->stream, P->n, o1.cand.x, B.pol_x));
        HIPCHECK(pdlp::launch_copy(P->stream, P->m, o1.cand.ax, B.pol_ax));
        // dual feasibility problem
        S.v = Vecs{P->cs, P->lc0, P->uc0, P->lv0, P->uv0};
        S.init(E.ctrl_h->omega, E.ctrl_h->eta_hat, prm);
        S.set_point(P->zero_n, E.yb);
        RunOut o2;
        rc = run_loop(X2, S, cap, TERM_DUAL, false, o2);
        X.res->polish_iters += S.ctrl_h->k;
        E.kkt_passes += S.kkt_passes;
        if (rc == RUN_OK) {
            HIPCHECK(pdlp::launch_copy(P->stream, P->m, o2.cand.y, B.pol_y));
            HIPCHECK(pdlp::launch_copy(P->stream, P->n, o2.cand.aty, B.pol_aty));
            KktOut k = E.kkt(B.pol_x, B.pol_y, B.pol_ax, B.pol_aty, 0);
            if (term_met(prm, TERM_FULL, k)) {
                out.cand = Candidate{B.pol_x, B.pol_y, B.pol_ax, B.pol_aty};
                out.kkt = k;
                out.have = true;
                ok = true;
            }
        }
    }
    if (rc == RUN_TIME) return false;
    return ok;
}

// Check of Algorithm 5 (Appendix C): the termination test (at the usual
// cadence) on the point a restart would produce, (x average, 0), then, every
// restart_period steps, that restart (counted as (iii)); no gap
// evaluations, no primal weight update.  Returns a RUN_* status, or -1.
int fixed_period_check(Ctx &X, Engine &E, bool full, bool per, bool capchk, int term_mode,
                       int rc_mode, RunOut &out) {
    const pdlp_params &prm = *X.prm;
    Ctrl &C = *E.ctrl_h;
    const int m = E.m, n = E.n;
    if ((full || capchk) && term_mode != TERM_NONE) {
        if (!E.zero_m) {
            E.zero_m = E.cert_arena.dev<double>(std::max(m, 1));
            HIPCHECK(pdlp::launch_fill(E.s(), m, E.zero_m, 0.0));
        }
        out.cand = Candidate{E.xb, E.zero_m, E.axb, E.P->zero_n};
        out.kkt = E.kkt(out.cand.x, out.cand.y, out.cand.ax, out.cand.aty, rc_mode);
        out.have = true;
        if (!std::isfinite(out.kkt.rel_gap)) return RUN_NUMERR;
        if (term_met(prm, term_mode, out.kkt)) return RUN_OK;
        if (term_mode == TERM_FULL && prm.detect_infeasibility) {
            const int inf = E.infeasible(prm.eps_infeasible, out.cert_src, out.cert);
            if (inf) return inf;
        }
        if (capchk) return RUN_LIMIT;
    }
    if (!per) return -1;
    E.restarts_iii += 1;
    hipStream_t s = E.s();
    HIPCHECK(pdlp::launch_copy(s, n, E.xb, E.X()));
    HIPCHECK(pdlp::launch_copy(s, m, E.axb, E.AXc()));
    HIPCHECK(pdlp::launch_fill(s, m, E.Y(), 0.0));
    HIPCHECK(pdlp::launch_fill(s, n, E.ATYc(), 0.0));
    HIPCHECK(pdlp::launch_copy(s, n, E.X(), E.x0));
    HIPCHECK(pdlp::launch_fill(s, m, E.y0, 0.0));
    E.n_outer += 1;
    C.t = 0;
    C.seta = 0.0;
    HIPCHECK(pdlp::launch_fill(s, n, E.it.sx, 0.0));
    HIPCHECK(pdlp::launch_fill(s, m, E.it.sy, 0.0));
    return -1;
}

// Algorithm 1 with the periodic checks (same readings as the oracle: at
// n = 0 only (iii); mu_c_prev is the previous evaluation in the outer loop;
// restart = candidate, then omega update, then mu_ref under the new omega;
// ties in GetRestartCandidate go to the average).
int run_loop(Ctx &X, Engine &E, long long max_k, int term_mode, bool allow_polish, RunOut &out) {
    const pdlp_params &prm = *X.prm;
    Ctrl &C = *E.ctrl_h;
    const int rc_mode = effective_rc_mode(prm);
    const int m = E.m, n = E.n;
    long long next_polish = prm.polish_first > 0 ? prm.polish_first : 100;
    while (allow_polish && next_polish <= C.k) next_polish *= 2;

    if (term_mode != TERM_NONE && (C.k == 0 || C.k >= max_k)) {
        out.cand = Candidate{E.X(), E.Y(), E.AXc(), E.ATYc()};
        out.kkt = E.kkt(out.cand.x, out.cand.y, out.cand.ax, out.cand.aty, rc_mode);
        out.have = true;
        if (term_met(prm, term_mode, out.kkt)) return RUN_OK;
        if (C.k >= max_k) return RUN_LIMIT;
    }
    const bool per_mode = prm.restart_period > 0;
    if (per_mode) {
        // Algorithm 5 constants, also over a state imported with other values
        C.fixed_step = 1;
        C.fixed_eta = C.eta = C.eta_hat = prm.fixed_step_size;
        C.omega = prm.fixed_primal_weight;
    }
    while (C.k < max_k) {
        if (term_mode != TERM_NONE && now_s() - X.t_start >= prm.time_limit) return RUN_TIME;
        long long kb = (C.k / prm.check_every + 1) * prm.check_every;
        if (per_mode)
            kb = std::min(kb, C.k + std::max(1LL, (long long)prm.restart_period - C.t));
        else
            kb = std::min(kb, next_art(C.k, C.t, prm.beta_art, max_k));
        kb = std::min(kb, max_k);
        if (allow_polish && prm.polish) kb = std::min(kb, next_polish);
        E.run_block(kb - C.k);
        if (C.numerr) return RUN_NUMERR;
        struct CheckTimer {
            Engine &e;
            double t0;
            ~CheckTimer() { e.kst.check_ms += 1e3 * (now_s() - t0); }
        } check_timer{E, now_s()};

        const bool full = (C.k % prm.check_every) == 0;
        const bool art = !per_mode && (double)C.t >= prm.beta_art * (double)C.k;
        const bool per = per_mode && C.t >= prm.restart_period;
        const bool capchk = term_mode != TERM_NONE && C.k == max_k;
        const bool pol = !per_mode && allow_polish && prm.polish && C.k == next_polish;
        if (!(full || art || per || capchk || pol)) continue;

        E.average();
        if (per_mode) {
            const int rc = fixed_period_check(X, E, full, per, capchk, term_mode, rc_mode, out);
            if (rc >= 0) return rc;
            continue;
        }
        if (pol) {
            next_polish *= 2;
            KktOut kb_ = E.kkt(E.xb, E.yb, E.axb, E.atyb, 0);
            if (kb_.rel_gap < prm.eps_gap) {
                RunOut po;
                if (feasibility_polish(X, E, po)) {
                    out = po;
                    return RUN_POLISHED;
                }
            }
            if (now_s() - X.t_start >= prm.time_limit) return RUN_TIME;
            if (!(full || art || capchk)) continue;
        }
        E.gap_enqueue(0, E.X(), E.Y(), E.AXc(), E.ATYc(), E.x0, E.y0, C.omega);
        E.gap_enqueue(1, E.xb, E.yb, E.axb, E.atyb, E.x0, E.y0, C.omega);
        E.gap_fetch();
        const double mu_cur = E.gap_h[0].mu, mu_avg = E.gap_h[1].mu;
        if (!std::isfinite(mu_cur) || !std::isfinite(mu_avg)) return RUN_NUMERR;
        const bool use_cur = mu_cur < mu_avg;
        const double mu_c = use_cur ? mu_cur : mu_avg;
        Candidate cand = use_cur ? Candidate{E.X(), E.Y(), E.AXc(), E.ATYc()}
                                 : Candidate{E.xb, E.yb, E.axb, E.atyb};
        if ((full || capchk) && term_mode != TERM_NONE) {
            out.cand = cand;
            out.kkt = E.kkt(cand.x, cand.y, cand.ax, cand.aty, rc_mode);
            out.have = true;
            if (prm.verbose)
                std::fprintf(stderr,
                             "[pdlp] k=%lld n=%lld omega=%.3e eta=%.3e mu=%.3e pres=%.2e "
                             "dres=%.2e gap=%.2e obj=%.10e\n",
                             C.k, E.n_outer, C.omega, C.eta_hat, mu_c, out.kkt.primal_res_rel,
                             out.kkt.dual_res_rel, out.kkt.rel_gap, out.kkt.primal_obj);
            if (!std::isfinite(out.kkt.rel_gap)) return RUN_NUMERR;
            if (term_met(prm, term_mode, out.kkt)) return RUN_OK;
            if (term_mode == TERM_FULL && prm.detect_infeasibility) {
                const int inf = E.infeasible(prm.eps_infeasible, out.cert_src, out.cert);
                if (inf) return inf;
            }
            if (capchk) return RUN_LIMIT;
        }
        int why = 0;
        if (!prm.adaptive_restarts || E.n_outer == 0) {
            if (art) why = 3;
        } else {
            if (full && mu_c <= prm.beta_suff * E.mu_ref) why = 1;
            else if (full && mu_c <= prm.beta_nec * E.mu_ref && mu_c > E.mu_c_prev) why = 2;
            else if (art) why = 3;
        }
        if (!why) {
            if (full) E.mu_c_prev = mu_c;
            continue;
        }
        if (why == 1) E.restarts_i += 1;
        if (why == 2) E.restarts_ii += 1;
        if (why == 3) E.restarts_iii += 1;
        hipStream_t s = E.s();
        HIPCHECK(pdlp::launch_copy(s, n, E.x0, E.xp));
        HIPCHECK(pdlp::launch_copy(s, m, E.y0, E.yp));
        if (!use_cur) {
            HIPCHECK(pdlp::launch_copy(s, n, E.xb, E.X()));
            HIPCHECK(pdlp::launch_copy(s, m, E.yb, E.Y()));
            HIPCHECK(pdlp::launch_copy(s, m, E.axb, E.AXc()));
            HIPCHECK(pdlp::launch_copy(s, n, E.atyb, E.ATYc()));
        }
        HIPCHECK(pdlp::launch_copy(s, n, E.X(), E.x0));
        HIPCHECK(pdlp::launch_copy(s, m, E.Y(), E.y0));
        const double dx = std::sqrt(E.dist2(E.x0, E.xp, n));
        const double dy = std::sqrt(E.dist2(E.y0, E.yp, m));
        const double ez = prm.eps_zero;
        if (dx > ez && dx < 1.0 / ez && dy > ez && dy < 1.0 / ez)
            C.omega = std::exp(prm.theta * std::log(dy / dx) + (1.0 - prm.theta) * std::log(C.omega));
        E.n_outer += 1;
        C.t = 0;
        C.seta = 0.0;
        HIPCHECK(pdlp::launch_fill(s, n, E.it.sx, 0.0));
        HIPCHECK(pdlp::launch_fill(s, m, E.it.sy, 0.0));
        E.gap_enqueue(2, E.x0, E.y0, E.AXc(), E.ATYc(), E.xp, E.yp, C.omega);
        E.gap_fetch();
        E.mu_ref = E.gap_h[2].mu;
        E.mu_c_prev = INFINITY;
    }
    return RUN_LIMIT;
}

}  // namespace

long long pdlp::host::next_art(long long k, long long t, double beta, long long cap) {
    if (!(beta < 1.0)) {
        if (beta == 1.0 && t == k) return k + 1;
        return cap;
    }
    double est = (beta * (double)k - (double)t) / (1.0 - beta);
    long long d = (long long)std::ceil(est);
    if (d < 1) d = 1;
    d = std::max<long long>(1, d - 2);
    while ((double)(t + d) < beta * (double)(k + d)) ++d;
    return std::min(cap, k + d);
}

struct pdlp_state {
    pdlp_problem *P = nullptr;
    pdlp_params prm{};
    Engine *E = nullptr;
    PolishBufs pb;
    ~pdlp_state() { delete E; }
};

// ===================================================================== C ABI

namespace {


void engine_initialize(pdlp_state *S, const double *x0_host, const double *y0_host) {
    pdlp_problem *P = S->P;
    Engine &E = *S->E;
    hipStream_t s = P->stream;
    HIPCHECK(pdlp::launch_absmax(s, P->nnz, P->A.val, P->red_part, red_grid(P->nnz), P->res_d));
    const double amax = reduce_result(P);
    HIPCHECK(pdlp::launch_primal_weight_init(s, P->m, P->n, P->cs, P->lcs, P->ucs, P->red_part,
                                             red_grid(std::max(P->m, P->n)), P->res_d));
    const double cc = reduce_result(P, 0), bb = reduce_result(P, 1);
    const double nc = std::sqrt(cc), nb = std::sqrt(bb);
    const double omega = (nc > 0.0 && nb > 0.0) ? nc / nb : 1.0;
    const double eta_hat = amax > 0.0 ? 1.0 / amax : 1.0;
    E.init(omega, eta_hat, S->prm);
    Arena tmp;
    double *xs = tmp.dev<double>(P->n), *ys = tmp.dev<double>(P->m);
    if (x0_host && y0_host) {
        // warm start (unscaled) -> x~ = x / D2, y~ = y / D1, then project
        upload_perm(P, x0_host, P->n, P->col_order, xs);
        upload_perm(P, y0_host, P->m, P->row_order, ys);
        HIPCHECK(pdlp::launch_scale_div(s, P->n, xs, P->d2, xs));
        HIPCHECK(pdlp::launch_scale_div(s, P->m, ys, P->d1, ys));
    } else {
        HIPCHECK(pdlp::launch_clamp0(s, P->n, P->lvs, P->uvs, xs));
        HIPCHECK(pdlp::launch_fill(s, P->m, ys, 0.0));
    }
    E.set_point(xs, ys);
    HIPCHECK(hipStreamSynchronize(s));
}

// Block schedules scored on the solver's own steps (stream_block = -1,
// single problems): for each candidate (nonzeros per stream block, longest
// row of the stream class) the row blocks of A and A^T are rebuilt and the
// fused step kernels of pdlp_solve run 4 accepted steps from the initial
// point (first launches, graph capture), then 16 more, timed on the host
// around the block; the fastest candidate is kept.  A row no longer than the
// chosen length is summed in stored order by one lane, a longer one by a
// wave or a workgroup tree, so the choice can change the rounding of those
// rows' sums (never the method).
void autotune_schedules(pdlp_problem *P, const pdlp_params &prm, const int32_t *rp_a,
                        const int32_t *rp_t) {
    struct Cand {
        int32_t stage, med;
    };
    static constexpr Cand kCands[] = {{pdlp::kStage, pdlp::kMedRow}, {pdlp::kStage, 32},
                                      {pdlp::kStage, 128},          {1024, pdlp::kMedRow},
                                      {1024, 32},                   {512, pdlp::kMedRow}};
    pdlp_params p2 = prm;
    p2.profile = 0;
    double best = INFINITY;
    Cand pick = kCands[0];
    for (const Cand &c : kCands) {
        Arena blk_arena;
        upload_blocks(P, blk_arena, P->A, rp_a, nullptr, c.stage, c.med);
        upload_blocks(P, blk_arena, P->AT, rp_t, nullptr, c.stage, c.med);
        pdlp_state S;
        S.P = P;
        S.prm = p2;
        S.E = new Engine(P, P->scaled());
        S.E->use_graphs = p2.graphs != 0;
        engine_initialize(&S, nullptr, nullptr);
        S.E->run_block(4);
        const double t0 = now_s();
        S.E->run_block(16);
        HIPCHECK(hipStreamSynchronize(P->stream));
        const double t = now_s() - t0;
        if (t < best) {
            best = t;
            pick = c;
        }
    }
    P->blkA = upload_blocks(P, P->arena, P->A, rp_a, nullptr, pick.stage, pick.med);
    P->blkT = upload_blocks(P, P->arena, P->AT, rp_t, nullptr, pick.stage, pick.med);
    P->stage = pick.stage;
}

}  // namespace

extern "C" {

const char *pdlp_last_error(void) { return g_last_error.c_str(); }

int pdlp_problem_schedule(const pdlp_problem *p, int32_t *stream_block, int32_t *med_row) {
    return guarded([&] {
        if (!p) invalid("problem is NULL");
        if (stream_block) *stream_block = p->stage;
        if (med_row) *med_row = p->A.med_row;
    });
}

void pdlp_params_default(pdlp_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eps_feas = 1e-8;
    p->eps_gap = 1e-8;
    p->max_iters = 1000000;
    p->time_limit = 1e30;
    p->check_every = 64;
    p->ruiz_iters = 10;
    p->pock_chambolle = 1;
    p->polish = 0;
    p->polish_first = 100;
    p->reduced_cost_mode = -1;
    p->adaptive_restarts = 1;
    p->beta_suff = 0.1;
    p->beta_nec = 0.9;
    p->beta_art = 0.5;
    p->theta = 0.5;
    p->eps_zero = 1e-10;
    p->red_exp = 0.3;
    p->grow_exp = 0.6;
    p->verbose = 0;
    p->reorder = 1;
    p->detect_infeasibility = 1;
    p->eps_infeasible = 1e-9;
    p->restart_period = 0;
    p->fixed_step_size = 0.0;
    p->fixed_primal_weight = 1.0;
    p->graphs = 1;
    p->sorted_gathers = 1;
    p->segmented_gathers = -1;
}

}  // extern "C"

pdlp_problem *create_problem(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col, const double *val, const double *c,
                             const double *lc, const double *uc, const double *lv,
                             const double *uv, double obj_offset, const pdlp_params *params,
                             void *hip_stream, const std::vector<int32_t> *row_breaks,
                             const std::vector<int32_t> *col_breaks, bool validated) {
        if (!validated) validate(m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv);
        if (!std::isfinite(obj_offset)) invalid("objective offset must be finite");
        pdlp_params prm;
        pdlp_params_default(&prm);
        if (params) prm = *params;
        check_params(prm);
        if (row_breaks || col_breaks) prm.reorder = 0;
        auto *P = new pdlp_problem();
        try {
            P->m = m;
            P->n = n;
            P->nnz = nnz;
            HIPCHECK(hipGetDevice(&P->device));
            P->obj_offset = obj_offset;
            P->scale_params = prm;
            P->stream = static_cast<hipStream_t>(hip_stream);
            hipStream_t s = P->stream;
            Arena &a = P->arena;
            // internal labels: rows by decreasing length, columns by decreasing degree
            std::vector<int32_t> rlen(m), cdeg(n, 0);
            for (int32_t i = 0; i < m; ++i) rlen[i] = row_ptr[i + 1] - row_ptr[i];
            for (int64_t e = 0; e < nnz; ++e) cdeg[col[e]] += 1;
            // one round of co-clustering: columns by degree, rows by their hottest
            // columns, columns within a degree (the cold ones as one class) by
            // their first row, rows again
            const bool ro = prm.reorder != 0;
            std::vector<int32_t> col_order = order_by_count(cdeg, ro);
            std::vector<int32_t> new_row(m), new_col(n), new_rp((size_t)m + 1);
            for (int32_t j = 0; j < n; ++j) new_col[col_order[j]] = j;
            std::vector<int32_t> row_order = order_rows(rlen, row_ptr, col, new_col, ro);
            for (int32_t i = 0; i < m; ++i) new_row[row_order[i]] = i;
            if (ro) {
                col_order = order_cols(cdeg, row_ptr, col, m, new_row, ro);
                for (int32_t j = 0; j < n; ++j) new_col[col_order[j]] = j;
                row_order = order_rows(rlen, row_ptr, col, new_col, ro);
                for (int32_t i = 0; i < m; ++i) new_row[row_order[i]] = i;
            }
            new_rp[0] = 0;
            for (int32_t i = 0; i < m; ++i) new_rp[i + 1] = new_rp[i] + rlen[row_order[i]];
            P->row_order = a.dev<int32_t>(m);
            P->col_order = a.dev<int32_t>(n);
            P->orig_pos = a.dev<int32_t>(nnz);
            if (m > 0)
                HIPCHECK(hipMemcpyAsync(P->row_order, row_order.data(), sizeof(int32_t) * m,
                                        hipMemcpyHostToDevice, s));
            HIPCHECK(hipMemcpyAsync(P->col_order, col_order.data(), sizeof(int32_t) * n,
                                    hipMemcpyHostToDevice, s));
            DCsr &A = P->A;
            A.rows = m;
            A.cols = n;
            A.nnz = nnz;
            A.row_ptr = a.dev<int32_t>((size_t)m + 1);
            A.col = a.dev<int32_t>(nnz);
            A.val = a.dev<double>(nnz);
            HIPCHECK(hipMemcpyAsync(A.row_ptr, new_rp.data(), sizeof(int32_t) * ((size_t)m + 1),
                                    hipMemcpyHostToDevice, s));
            {
                // caller-order CSR on the device for the relabelling and the transpose
                Arena tmp;
                int32_t *rp0 = tmp.dev<int32_t>((size_t)m + 1), *col0 = tmp.dev<int32_t>(nnz);
                double *val0 = tmp.dev<double>(nnz);
                int32_t *nr = tmp.dev<int32_t>(m), *nc = tmp.dev<int32_t>(n);
                HIPCHECK(hipMemcpyAsync(rp0, row_ptr, sizeof(int32_t) * ((size_t)m + 1),
                                        hipMemcpyHostToDevice, s));
                if (nnz > 0) {
                    HIPCHECK(hipMemcpyAsync(col0, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
                    HIPCHECK(hipMemcpyAsync(val0, val, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
                }
                if (m > 0)
                    HIPCHECK(hipMemcpyAsync(nr, new_row.data(), sizeof(int32_t) * m,
                                            hipMemcpyHostToDevice, s));
                HIPCHECK(hipMemcpyAsync(nc, new_col.data(), sizeof(int32_t) * n,
                                        hipMemcpyHostToDevice, s));
                HIPCHECK(pdlp::launch_permute_rows(s, m, P->row_order, rp0, col0, val0, nc,
                                                   A.row_ptr, A.col, A.val, P->orig_pos));
                build_transpose(P, rp0, col0, val0, nr, nc);
            }
            double **vecs_n[] = {&P->c, &P->lv, &P->uv, &P->cs, &P->lvs, &P->uvs, &P->d2,
                                 &P->zero_n, &P->lv0, &P->uv0};
            for (auto pp : vecs_n) *pp = a.dev<double>(n);
            double **vecs_m[] = {&P->lc, &P->uc, &P->lcs, &P->ucs, &P->d1, &P->lc0, &P->uc0};
            for (auto pp : vecs_m) *pp = a.dev<double>(m);
            for (int32_t j = 0; j < n; ++j)
                P->ray_cols += !std::isfinite(lv[j]) || !std::isfinite(uv[j]);
            upload_perm(P, c, n, P->col_order, P->c);
            upload_perm(P, lv, n, P->col_order, P->lv);
            upload_perm(P, uv, n, P->col_order, P->uv);
            upload_perm(P, lc, m, P->row_order, P->lc);
            upload_perm(P, uc, m, P->row_order, P->uc);
            // dual-feasibility bounds: every finite bound set to 0 (Algorithm 4)
            {
                std::vector<double> t((size_t)std::max(m, n));
                auto zeroed = [&](const double *src, int64_t len, const int32_t *perm, double *dst) {
                    for (int64_t k = 0; k < len; ++k) t[k] = std::isfinite(src[k]) ? 0.0 : src[k];
                    upload_perm(P, t.data(), len, perm, dst);
                };
                zeroed(lv, n, P->col_order, P->lv0);
                zeroed(uv, n, P->col_order, P->uv0);
                zeroed(lc, m, P->row_order, P->lc0);
                zeroed(uc, m, P->row_order, P->uc0);
            }
            HIPCHECK(pdlp::launch_fill(s, n, P->zero_n, 0.0));
            P->red_cap = 1024 * 8;
            P->red_part = a.dev<double>(P->red_cap);
            P->res_d = a.dev<double>(8);
            P->res_h = a.host<double>(8);
            // a single problem autotunes on the solver's own steps once it is
            // scaled (autotune_schedules); until then it has the default blocks
            const bool single = !row_breaks && !col_breaks;
            const int32_t sb = (single && prm.stream_block == -1) ? 0 : prm.stream_block;
            P->blkA = choose_blocks(P, A, new_rp.data(), row_breaks, sb);
            P->stage = P->A.stage;
            std::vector<int32_t> trp((size_t)n + 1);
            HIPCHECK(hipMemcpy(trp.data(), P->AT.row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                               hipMemcpyDeviceToHost));
            P->blkT = choose_blocks(P, P->AT, trp.data(), col_breaks, sb);
            precondition(P, prm);
            const bool seg = prm.segmented_gathers == 1 ||
                             (prm.segmented_gathers < 0 && (int64_t)m * 8 > (int64_t)(32 << 20));
            if (seg && single) build_segmented(P, P->AT, P->segT);
            if (single && prm.stream_block == -1 && nnz > 0)
                autotune_schedules(P, prm, new_rp.data(), trp.data());
        } catch (...) {
            delete P;
            throw;
        }
        return P;
}

// Column-sorted copies of the short-row blocks of A and A^T (DCsr::scol,
// sval, slot, sblk) from the scaled values now on the device.  A block is
// sorted when that cuts the cache lines its waves gather from (distinct
// 128-byte lines per 64 consecutive entries, summed over the block) by at
// least a third; sorting a block whose columns are spread too thinly only
// adds the slot stream and scattered LDS stores.  The copies hold the
// scaled values of this moment: after a change of the matrix values,
// refresh_block_gathers copies them again.
void sort_block_gathers(pdlp_problem *P) {
    hipStream_t s = P->stream;
    for (int t = 0; t < 2; ++t) {
        DCsr &M = t == 0 ? P->A : P->AT;
        const std::vector<int32_t> &blk = t == 0 ? P->blkA : P->blkT;
        const int64_t nnz = M.nnz;
        if (nnz == 0 || M.nblk == 0) continue;
        std::vector<int32_t> rp((size_t)M.rows + 1), col((size_t)nnz);
        HIPCHECK(hipMemcpyAsync(rp.data(), M.row_ptr, sizeof(int32_t) * rp.size(),
                                hipMemcpyDeviceToHost, s));
        HIPCHECK(hipMemcpyAsync(col.data(), M.col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        std::vector<int32_t> scol((size_t)nnz);
        std::vector<uint16_t> slot((size_t)nnz);
        std::vector<int64_t> perm((size_t)nnz);
        std::vector<uint8_t> sblk((size_t)M.nblk, 0);
        // distinct 16-word lines in each run of 64 consecutive entries
        auto lines = [](const std::vector<std::pair<int32_t, int32_t>> &kv) {
            int64_t total = 0;
            std::vector<int32_t> g;
            for (size_t a = 0; a < kv.size(); a += 64) {
                g.clear();
                for (size_t q = a; q < std::min(kv.size(), a + 64); ++q) g.push_back(kv[q].first >> 4);
                std::sort(g.begin(), g.end());
                total += std::unique(g.begin(), g.end()) - g.begin();
            }
            return total;
        };
        parallel_for(M.nblk, [&](int64_t b0, int64_t b1) {
            std::vector<std::pair<int32_t, int32_t>> kv;
            for (int64_t b = b0; b < b1; ++b) {
                const int32_t r0 = blk[(size_t)b], r1 = blk[(size_t)b + 1];
                const int64_t e0 = rp[(size_t)r0], e1 = rp[(size_t)r1];
                const int64_t len = e1 - e0, len0 = rp[(size_t)r0 + 1] - e0;
                const bool stream = len <= pdlp::kStage && len0 <= M.med_row;
                kv.resize((size_t)len);
                for (int64_t q = 0; q < len; ++q) kv[(size_t)q] = {col[(size_t)(e0 + q)], (int32_t)q};
                bool use = false;
                if (stream && len > 64) {
                    const int64_t before = lines(kv);
                    std::sort(kv.begin(), kv.end());
                    use = 3 * lines(kv) <= 2 * before;
                }
                if (!use)
                    for (int64_t q = 0; q < len; ++q) kv[(size_t)q] = {col[(size_t)(e0 + q)], (int32_t)q};
                sblk[(size_t)b] = use;
                for (int64_t q = 0; q < len; ++q) {
                    const int64_t src = e0 + kv[(size_t)q].second;
                    scol[(size_t)(e0 + q)] = col[(size_t)src];
                    slot[(size_t)(e0 + q)] = (uint16_t)kv[(size_t)q].second;
                    perm[(size_t)(e0 + q)] = src;
                }
            }
        });
        int64_t *perm_d = P->arena.dev<int64_t>(nnz);
        int32_t *scol_d = P->arena.dev<int32_t>(nnz);
        double *sval_d = P->arena.dev<double>(nnz);
        uint16_t *slot_d = P->arena.dev<uint16_t>(nnz);
        uint8_t *sblk_d = P->arena.dev<uint8_t>(M.nblk);
        HIPCHECK(hipMemcpyAsync(sblk_d, sblk.data(), M.nblk, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(perm_d, perm.data(), sizeof(int64_t) * nnz, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(scol_d, scol.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(slot_d, slot.data(), sizeof(uint16_t) * nnz, hipMemcpyHostToDevice, s));
        HIPCHECK(pdlp::launch_take(s, nnz, perm_d, M.val, sval_d));
        HIPCHECK(hipStreamSynchronize(s));
        M.scol = scol_d;
        M.sval = sval_d;
        M.slot = slot_d;
        M.sblk = sblk_d;
        P->sperm[t] = perm_d;
    }
}

void refresh_block_gathers(pdlp_problem *P, hipStream_t s) {
    for (int t = 0; t < 2; ++t) {
        DCsr &M = t == 0 ? P->A : P->AT;
        if (M.sval && P->sperm[t])
            HIPCHECK(pdlp::launch_take(s, M.nnz, P->sperm[t], M.val, const_cast<double *>(M.sval)));
    }
}

extern "C" {

int pdlp_problem_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                        const int32_t *col, const double *val, const double *c, const double *lc,
                        const double *uc, const double *lv, const double *uv, double obj_offset,
                        const pdlp_params *params, void *hip_stream, pdlp_problem **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        *out = create_problem(m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, obj_offset, params,
                              hip_stream, nullptr, nullptr);
    });
}

int pdlp_problem_create_device(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col, const double *val, const double *c,
                               const double *lc, const double *uc, const double *lv,
                               const double *uv, double obj_offset, const pdlp_params *params,
                               void *hip_stream, pdlp_problem **out) {
    return guarded([&] {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        if (m < 0 || n < 1) invalid("need m >= 0 and n >= 1");
        if (nnz < 0 || nnz > (int64_t)std::numeric_limits<int32_t>::max())
            invalid("nnz must lie in [0, 2^31)");
        if (!row_ptr || (nnz > 0 && (!col || !val)) || !c || (m > 0 && (!lc || !uc)) || !lv || !uv)
            invalid("NULL input array");
        // validation and the labelling sorts run on the host: stage the
        // arrays there, after the work the caller queued on its stream
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        std::vector<int32_t> rp((size_t)m + 1), cl((size_t)nnz);
        std::vector<double> vl((size_t)nnz), cv(n), lcv(m), ucv(m), lvv(n), uvv(n);
        auto get = [&](void *dst, const void *src, size_t bytes) {
            if (bytes) HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
        };
        get(rp.data(), row_ptr, sizeof(int32_t) * rp.size());
        get(cl.data(), col, sizeof(int32_t) * cl.size());
        get(vl.data(), val, sizeof(double) * vl.size());
        get(cv.data(), c, sizeof(double) * cv.size());
        get(lcv.data(), lc, sizeof(double) * lcv.size());
        get(ucv.data(), uc, sizeof(double) * ucv.size());
        get(lvv.data(), lv, sizeof(double) * lvv.size());
        get(uvv.data(), uv, sizeof(double) * uvv.size());
        HIPCHECK(hipStreamSynchronize(s));
        *out = create_problem(m, n, nnz, rp.data(), cl.data(), vl.data(), cv.data(), lcv.data(),
                              ucv.data(), lvv.data(), uvv.data(), obj_offset, params, hip_stream,
                              nullptr, nullptr);
    });
}

void pdlp_problem_destroy(pdlp_problem *p) { delete p; }

int pdlp_problem_dims(const pdlp_problem *p, int32_t *m, int32_t *n, int64_t *nnz) {
    return guarded([&] {
        if (!p) invalid("problem is NULL");
        if (m) *m = p->m;
        if (n) *n = p->n;
        if (nnz) *nnz = p->nnz;
    });
}

int pdlp_problem_get_scaled(const pdlp_problem *pc, double *d1, double *d2, double *val, double *c,
                            double *lc, double *uc, double *lv, double *uv) {
    return guarded([&] {
        auto *p = const_cast<pdlp_problem *>(pc);
        if (!p) invalid("problem is NULL");
        download_unperm(p, p->d1, p->m, p->row_order, d1);
        download_unperm(p, p->d2, p->n, p->col_order, d2);
        download_unperm(p, p->cs, p->n, p->col_order, c);
        download_unperm(p, p->lcs, p->m, p->row_order, lc);
        download_unperm(p, p->ucs, p->m, p->row_order, uc);
        download_unperm(p, p->lvs, p->n, p->col_order, lv);
        download_unperm(p, p->uvs, p->n, p->col_order, uv);
        download_unperm(p, p->A.val, p->nnz, p->orig_pos, val);
    });
}

int pdlp_spmv(const pdlp_problem *pc, int32_t transpose, int32_t scaled, const double *x_host,
              double *out_host, int32_t repeat, double *ms) {
    return guarded([&] {
        auto *p = const_cast<pdlp_problem *>(pc);
        if (!p || !x_host || !out_host) invalid("NULL argument");
        if (repeat < 1) invalid("repeat must be >= 1");
        const DCsr &M = transpose ? p->AT : p->A;
        const int in_len = transpose ? p->m : p->n, out_len = transpose ? p->n : p->m;
        const double *din = transpose ? p->d1 : p->d2;   // original = D1^-1 A~ D2^-1
        const double *dout = transpose ? p->d2 : p->d1;
        hipStream_t s = p->stream;
        Arena tmp;
        double *xi = tmp.dev<double>(in_len), *yo = tmp.dev<double>(out_len);
        const int32_t *pin = transpose ? p->row_order : p->col_order;
        const int32_t *pout = transpose ? p->col_order : p->row_order;
        upload_perm(p, x_host, in_len, pin, xi);
        if (!scaled) HIPCHECK(pdlp::launch_scale_div(s, in_len, xi, din, xi));
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, s));
        for (int r = 0; r < repeat; ++r)
            HIPCHECK(transpose ? spmv_t(p, s, xi, yo) : pdlp::launch_spmv_plain(s, M, xi, yo));
        HIPCHECK(hipEventRecord(e1, s));
        HIPCHECK(hipEventSynchronize(e1));
        float el = 0.f;
        HIPCHECK(hipEventElapsedTime(&el, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ms) *ms = el / repeat;
        if (!scaled) HIPCHECK(pdlp::launch_scale_div(s, out_len, yo, dout, yo));
        download_unperm(p, yo, out_len, pout, out_host);
    });
}

int pdlp_norm_gap(const pdlp_problem *pc, const double *x, const double *y, const double *ax,
                  const double *aty, const double *xr, const double *yr, double omega,
                  double *mu) {
    return guarded([&] {
        auto *p = const_cast<pdlp_problem *>(pc);
        if (!p || !x || !aty || !xr || !mu || (p->m > 0 && (!y || !ax || !yr)))
            invalid("NULL argument");
        if (!(omega > 0.0)) invalid("omega must be > 0");
        hipStream_t s = p->stream;
        Arena tmp;
        const int m = p->m, n = p->n;
        double *d[6];
        const double *h[6] = {x, aty, xr, y, ax, yr};
        for (int i = 0; i < 6; ++i) {
            const int len = i < 3 ? n : m;
            d[i] = tmp.dev<double>(len);
            upload_perm(p, h[i], len, i < 3 ? p->col_order : p->row_order, d[i]);
        }
        const int grid = red_grid((int64_t)m + n);
        double *part = tmp.dev<double>((size_t)grid * 2 * pdlp::kGapPts);
        GapState *gs = tmp.dev<GapState>(1);
        HIPCHECK(pdlp::launch_gap(s, m, n, p->scaled(), d[0], d[3], d[4], d[1], d[2], d[5], omega,
                                  part, grid, gs));
        GapState hs;
        HIPCHECK(hipMemcpyAsync(&hs, gs, sizeof(GapState), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        *mu = hs.mu;
    });
}

int pdlp_state_create(pdlp_problem *p, const pdlp_params *params, pdlp_state **out) {
    return guarded([&] {
        if (!p || !out) invalid("NULL argument");
        *out = nullptr;
        auto *S = new pdlp_state();
        try {
            S->P = p;
            pdlp_params_default(&S->prm);
            if (params) S->prm = *params;
            check_params(S->prm);
            S->E = new Engine(p, p->scaled());
            S->E->profile = S->prm.profile != 0;
            S->E->use_graphs = S->prm.graphs != 0;
            engine_initialize(S, nullptr, nullptr);
        } catch (...) {
            delete S;
            throw;
        }
        *out = S;
    });
}

void pdlp_state_destroy(pdlp_state *s) { delete s; }

int pdlp_iterate_k(pdlp_state *S, int64_t k, pdlp_iter_info *info) {
    return guarded([&] {
        if (!S || k < 0) invalid("bad state or k < 0");
        Engine &E = *S->E;
        pdlp_result dummy;
        std::memset(&dummy, 0, sizeof dummy);
        Ctx X{S->P, &S->prm, now_s(), &dummy, &S->pb};
        RunOut out;
        const int rc = run_loop(X, E, E.ctrl_h->k + k, TERM_NONE, false, out);
        if (rc == RUN_NUMERR) throw LibError(PDLP_ERR_STATE, "numerical error during iterations");
        if (info) {
            const Ctrl &C = *E.ctrl_h;
            info->k = C.k;
            info->t = C.t;
            info->n_outer = E.n_outer;
            info->attempts = C.attempts;
            info->kkt_passes = E.kkt_passes;
            info->restarts_i = E.restarts_i;
            info->restarts_ii = E.restarts_ii;
            info->restarts_iii = E.restarts_iii;
            info->omega = C.omega;
            info->eta_hat = C.eta_hat;
            info->last_eta = C.eta_used;
            info->last_eta_bar = C.last_eta_bar;
            info->seta = C.seta;
            info->mu_ref = E.mu_ref;
            info->mu_c_prev = E.mu_c_prev;
        }
    });
}

int pdlp_state_get(const pdlp_state *S, pdlp_state_blob *b) {
    return guarded([&] {
        if (!S || !b) invalid("NULL argument");
        Engine &E = *S->E;
        const int m = E.m, n = E.n;
        pdlp_problem *P = S->P;
        download_unperm(P, E.X(), n, P->col_order, b->x);
        download_unperm(P, E.Y(), m, P->row_order, b->y);
        download_unperm(P, E.AXc(), m, P->row_order, b->ax);
        download_unperm(P, E.ATYc(), n, P->col_order, b->aty);
        download_unperm(P, E.x0, n, P->col_order, b->x0);
        download_unperm(P, E.y0, m, P->row_order, b->y0);
        download_unperm(P, E.it.sx, n, P->col_order, b->sx);
        download_unperm(P, E.it.sy, m, P->row_order, b->sy);
        const Ctrl &C = *E.ctrl_h;
        b->seta = C.seta;
        b->omega = C.omega;
        b->eta_hat = C.eta_hat;
        b->mu_ref = E.mu_ref;
        b->mu_c_prev = E.mu_c_prev;
        b->last_eta = C.eta_used;
        b->k = C.k;
        b->t = C.t;
        b->n_outer = E.n_outer;
        b->attempts = C.attempts;
        b->kkt_passes = E.kkt_passes;
        b->restarts_i = E.restarts_i;
        b->restarts_ii = E.restarts_ii;
        b->restarts_iii = E.restarts_iii;
    });
}

int pdlp_state_set(pdlp_state *S, const pdlp_state_blob *b) {
    return guarded([&] {
        if (!S || !b) invalid("NULL argument");
        Engine &E = *S->E;
        const int m = E.m, n = E.n;
        if (!b->x || !b->aty || !b->x0 || !b->sx || (m > 0 && (!b->y || !b->ax || !b->y0 || !b->sy)))
            invalid("state blob arrays must not be NULL");
        Ctrl &C = *E.ctrl_h;
        C.cur = 0;
        pdlp_problem *P = S->P;
        upload_perm(P, b->x, n, P->col_order, E.it.X[0]);
        upload_perm(P, b->y, m, P->row_order, E.it.Y[0]);
        upload_perm(P, b->ax, m, P->row_order, E.it.AX[0]);
        upload_perm(P, b->aty, n, P->col_order, E.it.ATY[0]);
        upload_perm(P, b->x0, n, P->col_order, E.x0);
        upload_perm(P, b->y0, m, P->row_order, E.y0);
        upload_perm(P, b->sx, n, P->col_order, E.it.sx);
        upload_perm(P, b->sy, m, P->row_order, E.it.sy);
        C.seta = b->seta;
        C.omega = b->omega;
        C.eta_hat = b->eta_hat;
        C.eta = b->eta_hat;
        C.eta_used = b->last_eta;
        C.k = b->k;
        C.t = b->t;
        C.attempts = b->attempts;
        C.pending_sy = 0;
        C.numerr = 0;
        E.mu_ref = b->mu_ref;
        E.mu_c_prev = b->mu_c_prev;
        E.n_outer = b->n_outer;
        E.kkt_passes = b->kkt_passes;
        E.restarts_i = b->restarts_i;
        E.restarts_ii = b->restarts_ii;
        E.restarts_iii = b->restarts_iii;
    });
}

}  // extern "C"


namespace {

// Run the solver of pdlp_solve on a state for at most k more accepted steps.
void state_solve(pdlp_state *S, long long k, pdlp_result *res, double t0, double setup_s) {
    pdlp_problem *p = S->P;
    Engine &E = *S->E;
    double *ux = res->x, *uy = res->y, *ur = res->r;
    std::memset(res, 0, sizeof(*res));
    res->x = ux;
    res->y = uy;
    res->r = ur;
    res->seconds_setup = setup_s;
    Ctx X{p, &S->prm, t0, res, &S->pb};
    RunOut out;
    const long long cap = std::min<long long>(S->prm.max_iters, E.ctrl_h->k + k);
    const int rc = run_loop(X, E, cap, TERM_FULL, S->prm.polish != 0, out);
    const int rc_mode = rc == RUN_POLISHED ? 0 : effective_rc_mode(S->prm);
    KktOut kk;
    if (ux || uy || ur || !out.have || rc == RUN_NUMERR) {
        if (!out.have || rc == RUN_NUMERR) out.cand = Candidate{E.X(), E.Y(), E.AXc(), E.ATYc()};
        Arena tmp;
        double *rx = tmp.dev<double>(p->n), *ry = tmp.dev<double>(p->m), *rr = tmp.dev<double>(p->n);
        kk = E.kkt(out.cand.x, out.cand.y, out.cand.ax, out.cand.aty, rc_mode, rr, rx, ry);
        if (rc == RUN_PINF || rc == RUN_DINF) {
            E.cert_point(out.cert_src - 1);
            HIPCHECK(pdlp::launch_cert_out(p->stream, p->m, p->n, E.cpx, E.cpy, E.cpaty, p->d1,
                                           p->d2, p->lv, p->uv, rx, ry, rr));
        }
        download_unperm(p, rx, p->n, p->col_order, ux);
        download_unperm(p, ry, p->m, p->row_order, uy);
        download_unperm(p, rr, p->n, p->col_order, ur);
    } else {
        kk = out.kkt;
    }
    res->status = rc == RUN_OK || rc == RUN_POLISHED ? PDLP_STATUS_OPTIMAL
                  : rc == RUN_TIME                   ? PDLP_STATUS_TIME_LIMIT
                  : rc == RUN_NUMERR                 ? PDLP_STATUS_NUMERICAL_ERROR
                  : rc == RUN_PINF                   ? PDLP_STATUS_PRIMAL_INFEASIBLE
                  : rc == RUN_DINF                   ? PDLP_STATUS_DUAL_INFEASIBLE
                                                     : PDLP_STATUS_ITERATION_LIMIT;
    if (rc == RUN_PINF || rc == RUN_DINF) {
        res->certificate = out.cert_src;
        res->certificate_objective = rc == RUN_PINF ? out.cert.pobj : out.cert.dobj;
        res->certificate_residual = rc == RUN_PINF ? out.cert.pres : out.cert.dres;
    }
    res->polished = rc == RUN_POLISHED;
    res->iterations = E.ctrl_h->k;
    res->attempts = E.ctrl_h->attempts;
    res->kkt_passes = E.kkt_passes;
    res->restarts_i = E.restarts_i;
    res->restarts_ii = E.restarts_ii;
    res->restarts_iii = E.restarts_iii;
    res->restarts = E.restarts_i + E.restarts_ii + E.restarts_iii;
    res->primal_obj = kk.primal_obj;
    res->dual_obj = kk.dual_obj;
    res->rel_gap = kk.rel_gap;
    res->primal_res_abs = kk.primal_res_abs;
    res->primal_res_rel = kk.primal_res_rel;
    res->dual_res_abs = kk.dual_res_abs;
    res->dual_res_rel = kk.dual_res_rel;
    res->omega = E.ctrl_h->omega;
    res->eta = E.ctrl_h->eta_hat;
    res->seconds = now_s() - t0;
}

}  // namespace

extern "C" {

int pdlp_solve(pdlp_problem *p, const pdlp_params *params, const double *x0_host,
               const double *y0_host, pdlp_result *res) {
    return guarded([&] {
        if (!p || !res) invalid("NULL argument");
        if ((x0_host == nullptr) != (y0_host == nullptr) && p->m > 0)
            invalid("warm start needs both x0 and y0");
        const double t0 = now_s();
        pdlp_state S;
        S.P = p;
        pdlp_params_default(&S.prm);
        if (params) S.prm = *params;
        check_params(S.prm);
        S.E = new Engine(p, p->scaled());
        S.E->profile = S.prm.profile != 0;
        S.E->use_graphs = S.prm.graphs != 0;
        engine_initialize(&S, x0_host, y0_host);
        const long long k = S.prm.max_iters;
        state_solve(&S, k, res, t0, now_s() - t0);
    });
}

int pdlp_state_solve(pdlp_state *S, int64_t k, pdlp_result *res) {
    return guarded([&] {
        if (!S || !res || k < 0) invalid("bad state, result or k < 0");
        state_solve(S, k, res, now_s(), 0.0);
    });
}

int pdlp_measure_device_rates(int64_t copy_bytes, int64_t gather_len, pdlp_device_rates *out) {
    return guarded([&] {
        if (!out || copy_bytes < (1 << 20) || gather_len < 1 || gather_len > (int64_t)UINT32_MAX)
            invalid("bad arguments");
        hipStream_t s = nullptr;
        Arena tmp;
        const int64_t len = copy_bytes / 16 * 2;  // doubles, even
        double *a = tmp.dev<double>(len), *b = tmp.dev<double>(len);
        HIPCHECK(pdlp::launch_fill(s, len, a, 1.0));
        const int64_t ng = 125000000;
        const int grid = 2048;
        uint32_t *idx = tmp.dev<uint32_t>(ng);
        double *x = tmp.dev<double>(gather_len), *o = tmp.dev<double>((size_t)grid * kThreads);
        HIPCHECK(pdlp::launch_fill(s, gather_len, x, 1.0));
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        auto best_ms = [&](auto &&launch) {
            float best = 1e30f;
            for (int rep = 0; rep < 5; ++rep) {
                HIPCHECK(hipEventRecord(e0, s));
                HIPCHECK(launch());
                HIPCHECK(hipEventRecord(e1, s));
                HIPCHECK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHECK(hipEventElapsedTime(&t, e0, e1));
                best = std::min(best, t);
            }
            return (double)best;
        };
        const double tc = best_ms([&] { return pdlp::launch_rate_copy(s, len, a, b); });
        out->copy_gbs = 2.0 * len * sizeof(double) / (tc * 1e-3) / 1e9;
        HIPCHECK(pdlp::launch_rate_idx(s, ng, (uint32_t)gather_len, idx));
        const double tg = best_ms([&] { return pdlp::launch_rate_gather(s, ng, idx, x, o, grid); });
        out->gather_gps = ng / (tg * 1e-3) / 1e9;
        HIPCHECK(pdlp::launch_rate_idx(s, ng, (uint32_t)std::min<int64_t>(gather_len, 131072), idx));
        const double tl = best_ms([&] { return pdlp::launch_rate_gather(s, ng, idx, x, o, grid); });
        out->gather_l2_gps = ng / (tl * 1e-3) / 1e9;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHECK(hipStreamSynchronize(s));
    });
}

int pdlp_state_kernel_stats(pdlp_state *S, pdlp_kernel_stats *st, int32_t reset) {
    return guarded([&] {
        if (!S || !st) invalid("NULL argument");
        *st = S->E->kst;
        if (reset) std::memset(&S->E->kst, 0, sizeof(pdlp_kernel_stats));
    });
}

}  // extern "C"

// --------------------------------------------- products without allocation
//
// Staging of pdlp_spmv_noalloc: a file-scope device array (one copy per GPU,
// held until the process ends).  Host code never passes the array's name to
// a kernel: its address on each device is looked up once, with that device
// current, and kept per device.
constexpr int64_t kNoAllocDoubles = int64_t(1) << 23;  // 64 MiB: m + n <= 8,388,608
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

double *scratch_on_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices)
        throw LibError(PDLP_ERR_HIP, "device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw LibError(PDLP_ERR_HIP, "no device address for the staging array");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int pdlp_spmv_noalloc(const pdlp_problem *pc, int32_t transpose, int32_t scaled,
                      const double *x_dev, double *out_dev, void *hip_stream) {
    return guarded([&] {
        auto *p = const_cast<pdlp_problem *>(pc);
        if (!p) invalid("NULL problem");
        const int64_t in_len = transpose ? p->m : p->n, out_len = transpose ? p->n : p->m;
        if ((in_len > 0 && !x_dev) || (out_len > 0 && !out_dev)) invalid("NULL vector");
        if (in_len + out_len > kNoAllocDoubles)
            invalid("pdlp_spmv_noalloc: m + n = " + std::to_string(in_len + out_len) +
                    " exceeds the staging capacity of " + std::to_string(kNoAllocDoubles) +
                    " doubles; use pdlp_spmv");
        int dev = 0;
        HIPCHECK(hipGetDevice(&dev));
        if (dev != p->device)
            invalid("pdlp_spmv_noalloc: make the problem's device (" + std::to_string(p->device) +
                    ") current");
        double *st = scratch_on_device(dev);
        hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : p->stream;
        const DCsr &M = transpose ? p->AT : p->A;
        const double *din = transpose ? p->d1 : p->d2;  // original = D1^-1 A~ D2^-1
        const double *dout = transpose ? p->d2 : p->d1;
        const int32_t *pin = transpose ? p->row_order : p->col_order;
        const int32_t *pout = transpose ? p->col_order : p->row_order;
        double *xi = st, *yo = st + in_len;
        HIPCHECK(pdlp::launch_gather(s, in_len, pin, x_dev, xi));
        if (!scaled) HIPCHECK(pdlp::launch_scale_div(s, in_len, xi, din, xi));
        HIPCHECK(transpose ? spmv_t(p, s, xi, yo) : pdlp::launch_spmv_plain(s, M, xi, yo));
        if (!scaled) HIPCHECK(pdlp::launch_scale_div(s, out_len, yo, dout, yo));
        HIPCHECK(pdlp::launch_scatter(s, out_len, pout, yo, out_dev));
    });
}

}  // extern "C"
