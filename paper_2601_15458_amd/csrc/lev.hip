// Batched Levenshtein distance, bit-parallel (Myers 1999 / Hyyro 2003 block
// form), for the distance batches of Alg. 1 (Sec. 2.1).
//
// Layout on the GPU.  A wavefront takes one work item: one pattern (a DP
// column of up to 2048 rows, i.e. 32 64-bit words) and up to 64 texts, one
// text per lane.  Every lane runs the whole column recurrence for its own
// pair, so no carry ever crosses lanes; the 64 texts share the pattern, whose
// match table Peq[word][symbol] sits in LDS (8 KB per wavefront).  A lane's
// vertical delta vectors (Pv, Mv) stay in VGPRs (4 per 64-row word).  The
// only per-symbol lookup is one LDS read per word, at an address that
// depends on the lane's text symbol.  A kernel variant is compiled for a
// number of words per pass (its class); longer patterns run as several
// passes, and the horizontal deltas leaving a pass (2 bits per text column)
// go through a per-lane buffer in the workspace.  The class comes from the
// tuning table (tune.hip) when it holds one for the set, else it is the
// smallest class that holds the longest pattern in one pass (at most 32).
//
// Per text symbol t and word k (Eq = Peq[k][t]; hin = horizontal delta
// entering the word from below-left, +1 for the top row):
//   Xv = Eq | Mv;  Eq' = Eq | [hin < 0];
//   Xh = (((Eq' & Pv) + Pv) ^ Pv) | Eq';
//   Ph = Mv | ~(Xh | Pv);  Mh = Pv & Xh;  hout = sign bit of Ph/Mh row;
//   Ph = (Ph << 1) | [hin > 0];  Mh = (Mh << 1) | [hin < 0];
//   Pv = Mh | ~(Xv | Ph);  Mv = Ph & Xv.
// The distance is m plus the sum of the horizontal deltas of the last row.
#include <algorithm>

#include "lev_core.hpp"

namespace msadp {


// ------------------------------------------------------------ all pairs
// Rows are ranks in length order.  The pattern of row r is the sequence of
// rank r, its texts are the ranks r+1 .. N-1 (no shorter than the pattern),
// in blocks of 64.  Items are numbered so that u = N-1-r grows with the item
// id: S(U) = sum_{u=1..U} ceil(u/64) items precede row U+1; item 0 is the
// longest pattern, so the largest items start first.

struct AllPairsArgs {
    Staged S;
    const int32_t *order;   // rank -> sequence
    uint16_t *out;          // condensed distances
    uint32_t *counter;
    uint32_t *hbuf;         // carry buffers (64 lanes * hstride dwords per wave), or null
    int64_t hstride;        // dwords per lane slot group
    int64_t n_items;
    int32_t sigma;
};

template <int WMAX>
__global__ void __launch_bounds__(64) k_lev_allpairs(AllPairsArgs a) {
    __shared__ uint64_t peq[WMAX * kSym];
    const int lane = lane_id();
    const int64_t N = a.S.n;
    uint32_t *hb = a.hbuf ? a.hbuf + (int64_t)blockIdx.x * a.hstride * kWave + lane : nullptr;
    for (;;) {
        const uint32_t it = next_item(a.counter);
        if ((int64_t)it >= a.n_items) break;
        const int64_t g = (int64_t)it;
        // find u with items_upto(u-1) <= g < items_upto(u)
        const int64_t u = triangle_row(g, N - 1);
        const int64_t blk = g - items_upto(u - 1);
        const int64_t r = N - 1 - u;
        const int64_t tpos = r + 1 + blk * 64 + lane;
        const bool valid = tpos < N;
        const int64_t tp = valid ? tpos : r + 1;
        const uint8_t *pat = a.S.codes + r * a.S.stride;
        const int m = a.S.len[r];
        const uint8_t *text = a.S.codes + tp * a.S.stride;
        const int n = a.S.len[tp];
        const int d = lev_item<WMAX>(peq, pat, m, a.sigma, text, n, valid, hb);
        if (valid) {
            int64_t i = a.order[r], j = a.order[tpos];
            if (i > j) { int64_t t = i; i = j; j = t; }
            a.out[i * N - i * (i + 1) / 2 + (j - i - 1)] = (uint16_t)d;
        }
    }
}

// --------------------------------------------------------- grouped pairs
struct Item {
    int64_t start;    // first position in the grouped pair list
    int32_t pattern;  // index into A
    int32_t count;    // pairs in this item (<= 64)
};

struct GroupedArgs {
    Staged A, B;
    const int32_t *ib;
    const int64_t *sorted;   // pair ids grouped by ia
    const Item *items;
    const int64_t *n_items;  // device count
    uint16_t *out;
    uint32_t *counter;
    uint32_t *hbuf;
    int64_t hstride;
    int32_t sigma;
};

template <int WMAX>
__global__ void __launch_bounds__(64) k_lev_grouped(GroupedArgs a) {
    __shared__ uint64_t peq[WMAX * kSym];
    const int lane = lane_id();
    const int64_t total = *a.n_items;
    uint32_t *hb = a.hbuf ? a.hbuf + (int64_t)blockIdx.x * a.hstride * kWave + lane : nullptr;
    for (;;) {
        const uint32_t it = next_item(a.counter);
        if ((int64_t)it >= total) break;
        const Item I = a.items[it];
        const bool valid = lane < I.count;
        const int64_t pid = a.sorted[I.start + (valid ? lane : 0)];
        const int32_t jb = a.ib[pid];
        const uint8_t *pat = a.A.codes + (int64_t)I.pattern * a.A.stride;
        const int m = a.A.len[I.pattern];
        const uint8_t *text = a.B.codes + (int64_t)jb * a.B.stride;
        const int n = a.B.len[jb];
        const int d = lev_item<WMAX>(peq, pat, m, a.sigma, text, n, valid, hb);
        if (valid) a.out[pid] = (uint16_t)d;
    }
}

__global__ void k_pair_hist(const int32_t *ia, const int32_t *ib, int64_t np, int32_t na,
                            int32_t nb, int64_t *counts, uint16_t *out, int32_t *st) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (x < 0 || x >= na || y < 0 || y >= nb) {
            set_status(st, MSA_DS_INDEX);
            if (out) out[p] = 0xFFFF;
            continue;
        }
        atomicAdd((unsigned long long *)&counts[x], 1ull);
    }
}

__global__ void k_pair_scatter(const int32_t *ia, const int32_t *ib, int64_t np, int32_t na,
                               int32_t nb, int64_t *cursor, int64_t *sorted) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (x < 0 || x >= na || y < 0 || y >= nb) continue;
        const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&cursor[x], 1ull);
        sorted[pos] = p;
    }
}

// nitems[g] = ceil(count_g / 64) where count_g = start[g+1] - start[g]
__global__ void k_item_counts(const int64_t *start, int32_t ng, int64_t *nitems) {
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ng) return;
    if (g == ng) { nitems[g] = 0; return; }
    nitems[g] = (start[g + 1] - start[g] + 63) / 64;
}

__global__ void k_make_items(const int64_t *start, const int64_t *item_start, int32_t ng,
                             Item *items, int64_t *n_items) {
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *n_items = item_start[ng];
    if (g >= ng) return;
    const int64_t c = start[g + 1] - start[g];
    const int64_t base = item_start[g];
    for (int64_t b = 0; b * 64 < c; ++b) {
        Item I;
        I.start = start[g] + b * 64;
        I.pattern = g;
        I.count = (int32_t)min<int64_t>(64, c - b * 64);
        items[base + b] = I;
    }
}

// ------------------------------------------------------------ host side
#define MSADP_LEV_CLASSES(X) X(4) X(8) X(16) X(20) X(24) X(28) X(32)

// Persistent grid of a kernel variant, cached per device (concurrent first
// calls compute the same value).
static int lev_grid(int wclass, bool grouped) {
    static std::atomic<int> cache[kMaxDevices][2][33];
    std::atomic<int> &slot = cache[current_device()][grouped][wclass];
    int g = slot.load(std::memory_order_relaxed);
    if (g == 0) {
        switch (wclass) {
#define MSADP_G(w) \
    case w: g = grouped ? persistent_grid(k_lev_grouped<w>) : persistent_grid(k_lev_allpairs<w>); break;
            MSADP_LEV_CLASSES(MSADP_G)
#undef MSADP_G
            default: g = device_cus();
        }
        slot.store(g, std::memory_order_relaxed);
    }
    return g;
}

static int64_t hbuf_stride(int32_t text_max) { return ((int64_t)text_max + 15) / 16; }

struct LevPlan {
    int64_t strideA, strideB, hstride;
    int grid, wclass;
};

template <class Alloc>
static void lev_layout(Alloc &al, const msa_seqs *A, const msa_seqs *B, int64_t n_pairs,
                       bool grouped) {
    al.template take<uint8_t>((size_t)A->n * staged_stride(A->max_len));
    al.template take<int32_t>((size_t)A->n + 1);
    if (grouped) {
        al.template take<uint8_t>((size_t)B->n * staged_stride(B->max_len));
        al.template take<int32_t>((size_t)B->n + 1);
        al.template take<int64_t>((size_t)A->n + 1);   // start
        al.template take<int64_t>((size_t)A->n + 1);   // cursor / item counts
        al.template take<int64_t>((size_t)n_pairs);    // sorted pair ids
        al.template take<Item>((size_t)n_pairs);       // items
        al.template take<int64_t>(1);                  // item count
    } else {
        al.template take<int32_t>((size_t)A->n);           // order
        al.template take<int32_t>((size_t)A->max_len + 1); // length histogram
    }
    al.template take<uint32_t>(1);  // work counter
    // carry buffer: sized for the largest need over all classes, so that a
    // tuning entry never outgrows a workspace sized beforehand
    size_t hb = 0;
    for (int c : kLevClasses)
        if (needs_passes(A->max_len, c))
            hb = std::max(hb, (size_t)lev_grid(c, grouped) * kWave * hbuf_stride(B->max_len));
    if (hb) al.template take<uint32_t>(hb);
}

// forced > 0 selects the class (autotuning), else the tuning table or the default.
static LevPlan plan_lev(const msa_seqs *A, const msa_seqs *B, bool grouped, int forced) {
    LevPlan p;
    p.strideA = staged_stride(A->max_len);
    p.strideB = staged_stride(B->max_len);
    const int words = (int)std::max<int64_t>(1, ((int64_t)A->max_len + 63) / 64);
    p.wclass = forced > 0 ? forced
                          : tuned_value(MSA_TUNE_LEV, A->sigma, words, wmax_class(A->max_len));
    p.grid = lev_grid(p.wclass, grouped);
    p.hstride = needs_passes(A->max_len, p.wclass) ? hbuf_stride(B->max_len) : 0;
    return p;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t lev_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    Sizer sz;
    lev_layout(sz, A, B, n_pairs, true);
    return sz.total();
}

int lev_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
              int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes, int32_t *d_status,
              hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0) return MSA_EINVAL;
    if (A->sigma != B->sigma) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || dist == nullptr || ws == nullptr) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL * 64) return MSA_ERANGE;
    const LevPlan pl = plan_lev(A, B, true, 0);
    Sizer sz;
    lev_layout(sz, A, B, n_pairs, true);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;

    Carve cv(ws, ws_bytes);
    Staged SA{cv.take<uint8_t>((size_t)A->n * pl.strideA), cv.take<int32_t>((size_t)A->n + 1),
              pl.strideA, A->n};
    Staged SB{cv.take<uint8_t>((size_t)B->n * pl.strideB), cv.take<int32_t>((size_t)B->n + 1),
              pl.strideB, B->n};
    int64_t *start = cv.take<int64_t>((size_t)A->n + 1);
    int64_t *cursor = cv.take<int64_t>((size_t)A->n + 1);
    int64_t *sorted = cv.take<int64_t>((size_t)n_pairs);
    Item *items = cv.take<Item>((size_t)n_pairs);
    int64_t *n_items = cv.take<int64_t>(1);
    uint32_t *counter = cv.take<uint32_t>(1);
    uint32_t *hbuf = pl.hstride ? cv.take<uint32_t>((size_t)pl.grid * kWave * pl.hstride) : nullptr;

    if ((rc = stage_set(A, nullptr, SA, d_status, s))) return rc;
    if ((rc = stage_set(B, nullptr, SB, d_status, s))) return rc;
    if ((rc = fill_i64(start, (int64_t)A->n + 1, 0, s))) return rc;
    const int64_t pg = std::min<int64_t>((n_pairs + 255) / 256, 8192);
    hipLaunchKernelGGL(k_pair_hist, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs, A->n,
                       B->n, start, dist, d_status);
    if ((rc = exclusive_scan_i64(start, (int64_t)A->n + 1, s))) return rc;
    if (hipMemcpyAsync(cursor, start, sizeof(int64_t) * ((size_t)A->n + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MSA_EDEVICE;
    hipLaunchKernelGGL(k_pair_scatter, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs,
                       A->n, B->n, cursor, sorted);
    const unsigned gg = (unsigned)((A->n + 1 + 255) / 256);
    hipLaunchKernelGGL(k_item_counts, dim3(gg), dim3(256), 0, s, start, A->n, cursor);
    if ((rc = exclusive_scan_i64(cursor, (int64_t)A->n + 1, s))) return rc;
    hipLaunchKernelGGL(k_make_items, dim3(gg), dim3(256), 0, s, start, cursor, A->n, items,
                       n_items);
    if ((rc = fill_i32((int32_t *)counter, 1, 0, s))) return rc;
    GroupedArgs ga{SA, SB, ib, sorted, items, n_items, dist, counter, hbuf, pl.hstride, A->sigma};
    switch (pl.wclass) {
#define MSADP_L(w) \
    case w: hipLaunchKernelGGL(k_lev_grouped<w>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        MSADP_LEV_CLASSES(MSADP_L)
#undef MSADP_L
        default: return MSA_EINVAL;
    }
    return launch_status();
}

size_t lev_allpairs_workspace_bytes(const msa_seqs *A) {
    if (check_seqs(A)) return 0;
    Sizer sz;
    lev_layout(sz, A, A, 0, false);
    return sz.total();
}

static int allpairs_impl(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                         int32_t *d_status, hipStream_t s, int forced) {
    int rc;
    if ((rc = check_seqs(A))) return rc;
    if (A->n < 2) return MSA_OK;
    if (condensed == nullptr || ws == nullptr) return MSA_EINVAL;
    const LevPlan pl = plan_lev(A, A, false, forced);
    Sizer sz;
    lev_layout(sz, A, A, 0, false);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    const int64_t n_items = items_upto((int64_t)A->n - 1);
    if (n_items > 0xffffffffLL) return MSA_ERANGE;

    Carve cv(ws, ws_bytes);
    Staged SA{cv.take<uint8_t>((size_t)A->n * pl.strideA), cv.take<int32_t>((size_t)A->n + 1),
              pl.strideA, A->n};
    int32_t *order = cv.take<int32_t>((size_t)A->n);
    int32_t *hist = cv.take<int32_t>((size_t)A->max_len + 1);
    uint32_t *counter = cv.take<uint32_t>(1);
    uint32_t *hbuf = pl.hstride ? cv.take<uint32_t>((size_t)pl.grid * kWave * pl.hstride) : nullptr;

    if ((rc = sort_by_length(A, SA.len, hist, order, d_status, s))) return rc;
    if ((rc = stage_set(A, order, SA, d_status, s))) return rc;
    if ((rc = fill_i32((int32_t *)counter, 1, 0, s))) return rc;
    AllPairsArgs aa{SA, order, condensed, counter, hbuf, pl.hstride, n_items, A->sigma};
    switch (pl.wclass) {
#define MSADP_L(w) \
    case w: hipLaunchKernelGGL(k_lev_allpairs<w>, dim3(pl.grid), dim3(64), 0, s, aa); break;
        MSADP_LEV_CLASSES(MSADP_L)
#undef MSADP_L
        default: return MSA_EINVAL;
    }
    return launch_status();
}

int lev_allpairs(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                 int32_t *d_status, hipStream_t s) {
    return allpairs_impl(A, condensed, ws, ws_bytes, d_status, s, 0);
}

int msa_autotune_lev(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                     int32_t reps, int32_t *best, float *best_ms, int32_t *d_status,
                     hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A))) return rc;
    if (best == nullptr || best_ms == nullptr || reps < 1 || A->n < 2) return MSA_EINVAL;
    const int words = (int)std::max<int64_t>(1, ((int64_t)A->max_len + 63) / 64);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MSA_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MSA_EDEVICE;
    }
    int bc = 0;
    float bms = 0.0f;
    rc = MSA_OK;
    for (int c : kLevClasses) {
        if (!class_within_passes(A->max_len, c)) continue;
        if ((rc = allpairs_impl(A, condensed, ws, ws_bytes, d_status, s, c))) break;   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        for (int r = 0; r < reps && rc == MSA_OK; ++r)
            rc = allpairs_impl(A, condensed, ws, ws_bytes, d_status, s, c);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        ms /= (float)reps;
        if (bc == 0 || ms < bms) {
            bc = c;
            bms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = bc;
    *best_ms = bms;
    return msa_tune_set(MSA_TUNE_LEV, A->sigma, words, bc);
}

}  // extern "C"
