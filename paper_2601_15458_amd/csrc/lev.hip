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
#include "lev_xl.hpp"

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
    for (uint32_t it = first_item();; it = later_item(a.counter)) {
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

// ------------------------------------------------------------ pair lists
// Two layouts for an explicit pair list, chosen per call:
//
//  * Shared pattern ("grouped"): pairs are grouped by their A sequence and a
//    wavefront takes up to 64 pairs of one group, whose match table sits once
//    in LDS.  Inside a group the pairs are ordered by text length, longest
//    first, and groups run longest pattern first, so a wavefront's texts have
//    nearly equal lengths and the largest items start first.  Good when every
//    sequence has many partners.
//  * One pattern per lane ("lanes"): each lane holds one pair, with the longer
//    sequence as its pattern (the distance is symmetric) and its own match
//    table in LDS.  Pairs are binned by pattern words and, inside a bin,
//    ordered by text length, longest first; a wavefront takes 64 consecutive
//    pairs of one bin.  For sparse lists (a few partners per sequence), where
//    shared-pattern wavefronts would leave most lanes idle.  It needs patterns
//    of at most 32 / sigma' words (sigma' = 4, 8 or 32 for sigma <= 4, <= 8,
//    <= 32): 512 rows of DNA.
struct Item {
    int64_t start;    // first position in the ordered pair list
    int32_t key;      // grouped: the pattern (index into A); lanes: pattern words
    int32_t count;    // pairs in this item (<= 64)
};

constexpr int kSwapBit = 62;   // lanes layout: the pattern is B's sequence
constexpr int64_t kPairMask = (1ll << kSwapBit) - 1;

struct GroupedArgs {
    Staged A, B;
    const int32_t *ib;
    const int64_t *sorted;   // pair ids grouped by ia, ordered inside groups
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
    for (uint32_t it = first_item();; it = later_item(a.counter)) {
        if ((int64_t)it >= total) break;
        const Item I = a.items[it];
        const bool valid = lane < I.count;
        const int64_t pid = a.sorted[I.start + (valid ? lane : 0)];
        const int32_t jb = a.ib[pid];
        const uint8_t *pat = a.A.codes + (int64_t)I.key * a.A.stride;
        const int m = a.A.len[I.key];
        const uint8_t *text = a.B.codes + (int64_t)jb * a.B.stride;
        const int n = a.B.len[jb];
        const int d = lev_item<WMAX>(peq, pat, m, a.sigma, text, n, valid, hb);
        if (valid) a.out[pid] = (uint16_t)d;
    }
}

struct LanesArgs {
    Staged A, B;             // staged with one common stride
    const int32_t *ia, *ib;
    const int64_t *sorted;   // pair ids (bit kSwapBit: B's sequence is the pattern)
    const Item *items;
    const int64_t *n_items;
    uint16_t *out;
    uint32_t *counter;
};

// WMAX words per pattern at most, SP = sigma' symbol rows per word (SP = 2:
// two bit planes per word, for alphabets of at most 4 symbols).
template <int WMAX, int SP>
__global__ void __launch_bounds__(64) k_lev_lanes(LanesArgs a) {
    __shared__ uint64_t tbl[WMAX * SP * kWave];
    const int lane = lane_id();
    const int64_t total = *a.n_items;
    for (uint32_t it = first_item();; it = later_item(a.counter)) {
        if ((int64_t)it >= total) break;
        const Item I = a.items[it];
        const bool valid = lane < I.count;
        const int64_t e = a.sorted[I.start + (valid ? lane : 0)];
        const int64_t pid = e & kPairMask;
        const bool swap = (e >> kSwapBit) & 1;
        const int32_t x = a.ia[pid], y = a.ib[pid];
        const uint8_t *sa = a.A.codes + (int64_t)x * a.A.stride;
        const uint8_t *sb = a.B.codes + (int64_t)y * a.B.stride;
        const int la = a.A.len[x], lb = a.B.len[y];
        const uint8_t *pat = swap ? sb : sa;
        const uint8_t *text = swap ? sa : sb;
        const int m = swap ? lb : la, n = swap ? la : lb;
        const int W = (int)uniform((uint32_t)I.key);
        const int nmax = (int)uniform((uint32_t)wave_max(valid ? n : 0));
        int d;
        if (W == 0) {
            d = n;                  // both sequences empty
        } else if (nmax == 0) {
            d = m;                  // every text empty
        } else {
            if constexpr (SP == 2) {
                build_lane_planes((uint4 *)tbl, pat, m, W);
                d = m + dispatch_planes<WMAX>(W, (lds_u128 *)tbl + lane, text, n, nmax,
                                              (m - 1) & 63);
            } else {
                build_lane_peq<SP>(tbl, pat, m, W);
                d = m + dispatch_lanes<WMAX, SP>(W, (lds_u64 *)tbl + lane, text, n, nmax,
                                                 (m - 1) & 63);
            }
        }
        if (valid) a.out[pid] = (uint16_t)d;
    }
}

__device__ __forceinline__ bool pair_ok(int32_t x, int32_t y, int32_t na, int32_t nb) {
    return x >= 0 && x < na && y >= 0 && y < nb;
}

// Across-lanes layout: a pair per group of G lanes, its pattern (the longer
// sequence; the distance is symmetric) spread over the group (lev_xl.hpp),
// 64 / G pairs per wavefront, in `order` (largest m * n first) when given.
// For long patterns with few partners each, where one pattern per lane does
// not fit and a shared pattern table would leave most lanes idle.
struct XlPairArgs {
    Staged A, B;             // staged with one common stride
    const int32_t *ia, *ib;
    const int32_t *order;    // launch order, or nullptr: index order
    int64_t n_pairs;
    uint16_t *out;
    uint32_t *counter;
    int32_t *st;
};

constexpr int kXlPairBlock = 256;   // four independent wavefronts per workgroup

template <int G, int WL, int NB>
__global__ void __launch_bounds__(kXlPairBlock) k_lev_xl(XlPairArgs a) {
    constexpr int kPpw = kWave / G;
    const int lane = lane_id(), grp = lane / G;
    for (uint32_t it = first_item();; it = later_item(a.counter)) {
        const int64_t p0 = (int64_t)it * kPpw;
        if (p0 >= a.n_pairs) break;
        const bool in = p0 + grp < a.n_pairs;
        const int64_t r = in ? p0 + grp : p0;
        const int64_t pid = a.order != nullptr ? a.order[r] : r;
        const int32_t x = a.ia[pid], y = a.ib[pid];
        const bool ok = pair_ok(x, y, a.A.n, a.B.n);
        const int32_t xs = ok ? x : 0, ys = ok ? y : 0;
        const uint8_t *sa = a.A.codes + (int64_t)xs * a.A.stride;
        const uint8_t *sb = a.B.codes + (int64_t)ys * a.B.stride;
        const int la = a.A.len[xs], lb = a.B.len[ys];
        const bool swap = lb > la;
        const int d = xl_distance<G, WL, NB>(swap ? sb : sa, swap ? lb : la, swap ? sa : sb,
                                             swap ? la : lb, a.A.stride - 16, in && ok);
        if (in && (lane & (G - 1)) == 0) {
            if (!ok) set_status(a.st, MSA_DS_INDEX);
            a.out[pid] = ok ? (uint16_t)d : (uint16_t)0xFFFF;
        }
    }
}

// grouped layout: pairs per A sequence
__global__ void k_pair_hist(const int32_t *ia, const int32_t *ib, int64_t np, int32_t na,
                            int32_t nb, int64_t *counts, uint16_t *out, int32_t *st) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (!pair_ok(x, y, na, nb)) {
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
        if (!pair_ok(x, y, na, nb)) continue;
        const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&cursor[x], 1ull);
        sorted[pos] = p;
    }
}

// One workgroup per group: a counting sort of the group's pairs into 64 text
// length buckets, longest first (the order inside a bucket is unspecified).
__global__ void __launch_bounds__(256) k_group_sort(const int64_t *start, const int64_t *sorted,
                                                    const int32_t *ib, const int32_t *lenB,
                                                    int32_t bmax, int64_t *sorted2) {
    __shared__ unsigned long long h[64];
    const int g = blockIdx.x, t = threadIdx.x;
    const int64_t s0 = start[g], c = start[g + 1] - s0;
    if (c <= 64) {   // one work item: its order does not matter
        for (int64_t i = t; i < c; i += blockDim.x) sorted2[s0 + i] = sorted[s0 + i];
        return;
    }
    if (t < 64) h[t] = 0;
    __syncthreads();
    for (int64_t i = t; i < c; i += blockDim.x) {
        const int32_t n = lenB[ib[sorted[s0 + i]]];
        atomicAdd(&h[63 - (int)((int64_t)n * 64 / ((int64_t)bmax + 1))], 1ull);
    }
    __syncthreads();
    if (t == 0) {
        unsigned long long acc = 0;
        for (int b = 0; b < 64; ++b) {
            const unsigned long long v = h[b];
            h[b] = acc;
            acc += v;
        }
    }
    __syncthreads();
    for (int64_t i = t; i < c; i += blockDim.x) {
        const int64_t pid = sorted[s0 + i];
        const int32_t n = lenB[ib[pid]];
        const unsigned long long pos =
            atomicAdd(&h[63 - (int)((int64_t)n * 64 / ((int64_t)bmax + 1))], 1ull);
        sorted2[s0 + (int64_t)pos] = pid;
    }
}

// nitems[r] = work items of the group at rank r, longest pattern first
// (order: ascending length ranks of A).
__global__ void k_rank_item_counts(const int64_t *start, const int32_t *order, int32_t ng,
                                   int64_t *nitems) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > ng) return;
    if (r == ng) {
        nitems[r] = 0;
        return;
    }
    const int32_t g = order[ng - 1 - r];
    nitems[r] = (start[g + 1] - start[g] + 63) / 64;
}

__global__ void k_rank_make_items(const int64_t *start, const int64_t *item_start,
                                  const int32_t *order, int32_t ng, Item *items,
                                  int64_t *n_items) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *n_items = item_start[ng];
    if (r >= ng) return;
    const int32_t g = order[ng - 1 - r];
    const int64_t c = start[g + 1] - start[g];
    const int64_t base = item_start[r];
    for (int64_t b = 0; b * 64 < c; ++b) {
        Item I;
        I.start = start[g] + b * 64;
        I.key = g;
        I.count = (int32_t)min<int64_t>(64, c - b * 64);
        items[base + b] = I;
    }
}

// lanes layout: key = (wmax - pattern words) * nb + (nb - 1 - text length / 4),
// so that ascending keys run the most pattern words first and, inside a
// words bin, the longest texts first.
__device__ __forceinline__ int32_t lanes_key(int la, int lb, int wmax, int nb, bool *swap) {
    *swap = lb > la;
    const int P = max(la, lb), T = min(la, lb);
    return (wmax - ((P + 63) >> 6)) * nb + (nb - 1 - (T >> 2));
}

// Lanes-layout binning, privatized: the keys are few (at most 9 x 129), so a
// global atomic per pair would queue thousands of adds on each counter.  A
// workgroup takes a fixed range of pairs, counts its keys in LDS and adds
// each nonzero count to the global counter once; the scatter recounts the
// same range, reserves each key's slots with one global add and places its
// pairs from an LDS cursor.
constexpr int kMaxLaneKeys = 9 * 129 + 1;
constexpr int kBinPairsPerBlock = 8192;

__global__ void __launch_bounds__(256) k_lanes_hist(const int32_t *ia, const int32_t *ib,
                                                    int64_t np, const int32_t *lenA,
                                                    const int32_t *lenB, int32_t na,
                                                    int32_t nb_seq, int32_t wmax, int32_t nb,
                                                    int64_t *counts, uint16_t *out,
                                                    int32_t *st) {
    __shared__ uint32_t h[kMaxLaneKeys];
    const int nkeys = (wmax + 1) * nb;
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * kBinPairsPerBlock;
    const int64_t p1 = min(np, p0 + kBinPairsPerBlock);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (!pair_ok(x, y, na, nb_seq)) {
            set_status(st, MSA_DS_INDEX);
            if (out) out[p] = 0xFFFF;
            continue;
        }
        bool sw;
        atomicAdd(&h[lanes_key(lenA[x], lenB[y], wmax, nb, &sw)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x)
        if (h[k]) atomicAdd((unsigned long long *)&counts[k], (unsigned long long)h[k]);
}

__global__ void __launch_bounds__(256) k_lanes_scatter(const int32_t *ia, const int32_t *ib,
                                                       int64_t np, const int32_t *lenA,
                                                       const int32_t *lenB, int32_t na,
                                                       int32_t nb_seq, int32_t wmax, int32_t nb,
                                                       int64_t *cursor, int64_t *sorted) {
    __shared__ uint32_t h[kMaxLaneKeys];
    __shared__ int64_t base[kMaxLaneKeys];
    const int nkeys = (wmax + 1) * nb;
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * kBinPairsPerBlock;
    const int64_t p1 = min(np, p0 + kBinPairsPerBlock);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (!pair_ok(x, y, na, nb_seq)) continue;
        bool sw;
        atomicAdd(&h[lanes_key(lenA[x], lenB[y], wmax, nb, &sw)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) {
        base[k] = h[k] ? (int64_t)atomicAdd((unsigned long long *)&cursor[k],
                                            (unsigned long long)h[k])
                       : 0;
        h[k] = 0;
    }
    __syncthreads();
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int32_t x = ia[p], y = ib[p];
        if (!pair_ok(x, y, na, nb_seq)) continue;
        bool sw;
        const int32_t key = lanes_key(lenA[x], lenB[y], wmax, nb, &sw);
        const int64_t pos = base[key] + atomicAdd(&h[key], 1u);
        sorted[pos] = p | ((int64_t)sw << kSwapBit);
    }
}

// Items of 64 consecutive pairs inside each words bin; start[] is the
// exclusive scan of the key counts ((wmax + 1) * nb + 1 entries).
constexpr int kLanesMaxWords = 8;
__global__ void k_lanes_items(const int64_t *start, int32_t wmax, int32_t nb, Item *items,
                              int64_t *n_items) {
    __shared__ int64_t base[kLanesMaxWords + 2];
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int b = 0; b <= wmax; ++b) {
            base[b] = acc;
            acc += (start[(b + 1) * nb] - start[b * nb] + 63) / 64;
        }
        base[wmax + 1] = acc;
        if (blockIdx.x == 0) *n_items = acc;
    }
    __syncthreads();
    const int64_t total = base[wmax + 1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int b = 0;
        while (base[b + 1] <= i) ++b;
        const int64_t s0 = start[b * nb], c = start[(b + 1) * nb] - s0, k = i - base[b];
        Item I;
        I.start = s0 + k * 64;
        I.key = wmax - b;
        I.count = (int32_t)min<int64_t>(64, c - k * 64);
        items[i] = I;
    }
}

// ------------------------------------------------------------ host side
#define MSADP_LEV_CLASSES(X) X(4) X(8) X(16) X(20) X(24) X(28) X(32)
// Lanes-layout variants: (most pattern words, sigma').
#define MSADP_LANES_CLASSES(X) X(8, 2) X(4, 8) X(1, 32)

enum { kAllPairsKernel = 0, kGroupedKernel = 1, kLanesKernel = 2 };

// Persistent grid of a kernel variant, cached per device (concurrent first
// calls compute the same value).  Lanes variants are keyed by their words.
static int lev_grid(int wclass, int kind) {
    static std::atomic<int> cache[kMaxDevices][3][33];
    std::atomic<int> &slot = cache[current_device()][kind][wclass];
    int g = slot.load(std::memory_order_relaxed);
    if (g == 0) {
        if (kind == kLanesKernel) {
            switch (wclass) {
#define MSADP_G(w, sp) \
    case w: g = persistent_grid(k_lev_lanes<w, sp>); break;
                MSADP_LANES_CLASSES(MSADP_G)
#undef MSADP_G
                default: g = device_cus();
            }
        } else {
            switch (wclass) {
#define MSADP_G(w)                                                                      \
    case w:                                                                             \
        g = kind == kGroupedKernel ? persistent_grid(k_lev_grouped<w>)                  \
                                   : persistent_grid(k_lev_allpairs<w>);                \
        break;
                MSADP_LEV_CLASSES(MSADP_G)
#undef MSADP_G
                default: g = device_cus();
            }
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
    al.template take<int32_t>((size_t)A->n);           // order
    al.template take<int32_t>((size_t)A->max_len + 1); // length histogram
    al.template take<uint32_t>(1);  // work counter
    // carry buffer: sized for the largest need over all classes, so that a
    // tuning entry never outgrows a workspace sized beforehand
    size_t hb = 0;
    for (int c : kLevClasses)
        if (needs_passes(A->max_len, c))
            hb = std::max(hb, (size_t)lev_grid(c, grouped ? kGroupedKernel : kAllPairsKernel) *
                                  kWave * hbuf_stride(B->max_len));
    if (hb) al.template take<uint32_t>(hb);
}

// forced > 0 selects the class (autotuning), forced < 0 the default, else
// the tuning table or the default.
static LevPlan plan_lev(const msa_seqs *A, const msa_seqs *B, bool grouped, int forced) {
    LevPlan p;
    p.strideA = staged_stride(A->max_len);
    p.strideB = staged_stride(B->max_len);
    const int words = (int)std::max<int64_t>(1, ((int64_t)A->max_len + 63) / 64);
    const int dflt = wmax_class(A->max_len);
    p.wclass = forced > 0 ? forced
               : forced < 0 ? dflt
                            : tuned_value(MSA_TUNE_LEV, A->sigma, words, dflt);
    p.grid = lev_grid(p.wclass, grouped ? kGroupedKernel : kAllPairsKernel);
    p.hstride = needs_passes(A->max_len, p.wclass) ? hbuf_stride(B->max_len) : 0;
    return p;
}

// ------------------------------------------------ pair-list planning
// Two descriptions of one set (same device pointers and sizes) are staged once.
static bool same_set(const msa_seqs *A, const msa_seqs *B) {
    return A->codes == B->codes && A->offsets == B->offsets && A->n == B->n &&
           A->sigma == B->sigma && A->max_len == B->max_len && A->packed_2bit == B->packed_2bit;
}

// The lanes variant for the alphabet, and whether patterns of up to the
// longer set's max_len fit it.
static bool lanes_fit(const msa_seqs *A, const msa_seqs *B, int *wmax, int *sp) {
    *sp = A->sigma <= 4 ? 2 : A->sigma <= 8 ? 8 : 32;   // 2: bit planes
    *wmax = A->sigma <= 4 ? 8 : 32 / *sp;
    return std::max(A->max_len, B->max_len) <= 64 * *wmax;
}

static int pair_words_bin(const msa_seqs *A, const msa_seqs *B) {
    return (int)std::max<int64_t>(1, ((int64_t)std::max(A->max_len, B->max_len) + 63) / 64);
}

// Workspace pieces of the grouped layout (pointers are null with a Sizer).
struct GroupedWs {
    Staged SA, SB;
    int32_t *order, *hist;
    int64_t *start, *cursor, *sorted, *sorted2, *n_items;
    Item *items;
    uint32_t *counter, *hbuf;
};

static int64_t grouped_item_bound(const msa_seqs *A, int64_t n_pairs) {
    return std::min<int64_t>(n_pairs, n_pairs / 64 + A->n) + 1;
}

template <class Alloc>
static GroupedWs carve_grouped(Alloc &al, const msa_seqs *A, const msa_seqs *B, int64_t n_pairs,
                               const LevPlan &pl, bool all_classes) {
    GroupedWs w;
    w.SA = Staged{al.template take<uint8_t>((size_t)A->n * pl.strideA),
                  al.template take<int32_t>((size_t)A->n + 1), pl.strideA, A->n};
    if (same_set(A, B)) {
        w.SB = w.SA;
    } else {
        w.SB = Staged{al.template take<uint8_t>((size_t)B->n * pl.strideB),
                      al.template take<int32_t>((size_t)B->n + 1), pl.strideB, B->n};
    }
    w.order = al.template take<int32_t>((size_t)A->n);
    w.hist = al.template take<int32_t>((size_t)A->max_len + 1);
    w.start = al.template take<int64_t>((size_t)A->n + 1);
    w.cursor = al.template take<int64_t>((size_t)A->n + 1);
    w.sorted = al.template take<int64_t>((size_t)n_pairs);
    w.sorted2 = al.template take<int64_t>((size_t)n_pairs);
    w.items = al.template take<Item>((size_t)grouped_item_bound(A, n_pairs));
    w.n_items = al.template take<int64_t>(1);
    w.counter = al.template take<uint32_t>(1);
    // carry buffer: with all_classes, the largest need over every class, so
    // that a tuning entry never outgrows a workspace sized beforehand
    size_t hb = 0;
    if (all_classes) {
        for (int c : kLevClasses)
            if (needs_passes(A->max_len, c))
                hb = std::max(hb, (size_t)lev_grid(c, kGroupedKernel) * kWave *
                                      hbuf_stride(B->max_len));
    } else if (pl.hstride) {
        hb = (size_t)pl.grid * kWave * pl.hstride;
    }
    w.hbuf = hb ? al.template take<uint32_t>(hb) : nullptr;
    return w;
}

struct LanesWs {
    Staged SA, SB;
    int64_t *counts, *cursor, *sorted, *n_items;
    Item *items;
    uint32_t *counter;
};

template <class Alloc>
static LanesWs carve_lanes(Alloc &al, const msa_seqs *A, const msa_seqs *B, int64_t n_pairs,
                           int wmax) {
    LanesWs w;
    const int64_t stride = staged_stride(std::max(A->max_len, B->max_len));
    w.SA = Staged{al.template take<uint8_t>((size_t)A->n * stride),
                  al.template take<int32_t>((size_t)A->n + 1), stride, A->n};
    if (same_set(A, B)) {
        w.SB = w.SA;
    } else {
        w.SB = Staged{al.template take<uint8_t>((size_t)B->n * stride),
                      al.template take<int32_t>((size_t)B->n + 1), stride, B->n};
    }
    const int nb = 16 * wmax + 1;
    w.counts = al.template take<int64_t>((size_t)(wmax + 1) * nb + 1);
    w.cursor = al.template take<int64_t>((size_t)(wmax + 1) * nb + 1);
    w.sorted = al.template take<int64_t>((size_t)n_pairs);
    w.items = al.template take<Item>((size_t)(n_pairs / 64 + wmax + 2));
    w.n_items = al.template take<int64_t>(1);
    w.counter = al.template take<uint32_t>(1);
    return w;
}

// Group shape of the across-lanes layout for patterns of up to `words`
// 64-bit words: one word per lane in the least power of two (at least 8)
// of lanes that holds them, else 64 lanes of 2, 3 or 4 words; false beyond
// 256 words.
struct XlPairShape {
    int g, wl, nb;
};

static bool xl_shape_for(int words, int sigma, XlPairShape *x) {
    x->nb = xl_planes(sigma);
    if (words <= 64) {
        x->wl = 1;
        x->g = 8;
        while (x->g < words) x->g <<= 1;
        return true;
    }
    x->g = kWave;
    x->wl = (words + 63) / 64;
    return x->wl <= 4;
}

static bool xl_pairs_shape(const msa_seqs *A, const msa_seqs *B, XlPairShape *x) {
    return xl_shape_for(pair_words_bin(A, B), A->sigma, x);
}

template <int NB>
static const void *xl_pair_kernel_nb(int g, int wl) {
    if (wl == 1) {
        switch (g) {
            case 8: return (const void *)&k_lev_xl<8, 1, NB>;
            case 16: return (const void *)&k_lev_xl<16, 1, NB>;
            case 32: return (const void *)&k_lev_xl<32, 1, NB>;
            default: return (const void *)&k_lev_xl<64, 1, NB>;
        }
    }
    switch (wl) {
        case 2: return (const void *)&k_lev_xl<64, 2, NB>;
        case 3: return (const void *)&k_lev_xl<64, 3, NB>;
        default: return (const void *)&k_lev_xl<64, 4, NB>;
    }
}

static const void *xl_pair_kernel(const XlPairShape &x) {
    return x.nb == 2 ? xl_pair_kernel_nb<2>(x.g, x.wl) : xl_pair_kernel_nb<5>(x.g, x.wl);
}

static int xl_pair_grid(const XlPairShape &x) {
    static std::atomic<int> cache[kMaxDevices][4][4][2];
    int gi = 0;
    while ((8 << gi) < x.g) ++gi;
    std::atomic<int> &slot = cache[current_device()][gi][x.wl - 1][x.nb == 2 ? 0 : 1];
    int v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, xl_pair_kernel(x),
                                                         kXlPairBlock, 0) != hipSuccess ||
            blocks < 1)
            blocks = 1;
        v = device_cus() * blocks;
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}

struct XlPairWs {
    Staged SA, SB;
    int32_t *order;
    uint32_t *counter;
};

template <class Alloc>
static XlPairWs carve_xl_pairs(Alloc &al, const msa_seqs *A, const msa_seqs *B,
                               int64_t n_pairs) {
    XlPairWs w;
    const int64_t stride = staged_stride(std::max(A->max_len, B->max_len));
    w.SA = Staged{al.template take<uint8_t>((size_t)A->n * stride),
                  al.template take<int32_t>((size_t)A->n + 1), stride, A->n};
    if (same_set(A, B)) {
        w.SB = w.SA;
    } else {
        w.SB = Staged{al.template take<uint8_t>((size_t)B->n * stride),
                      al.template take<int32_t>((size_t)B->n + 1), stride, B->n};
    }
    w.order = al.template take<int32_t>((size_t)std::min<int64_t>(n_pairs, kLptMaxPairs));
    w.counter = al.template take<uint32_t>(1);
    return w;
}

static int run_xl_pairs(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                        const int32_t *ib, int64_t n_pairs, uint16_t *dist, void *ws,
                        size_t ws_bytes, const XlPairShape &x, int32_t *d_status,
                        hipStream_t s) {
    int rc;
    Carve cv(ws, ws_bytes);
    const XlPairWs w = carve_xl_pairs(cv, A, B, n_pairs);
    if (!cv.ok()) return MSA_ENOSPC;
    if (A->n == 0 || B->n == 0) {   // every index is out of range
        const int64_t pg = std::min<int64_t>((n_pairs + 255) / 256, 8192);
        hipLaunchKernelGGL(k_pair_hist, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs,
                           A->n, B->n, (int64_t *)nullptr, dist, d_status);
        return launch_status();
    }
    if ((rc = stage_set(A, nullptr, w.SA, d_status, s))) return rc;
    if (!same_set(A, B) && (rc = stage_set(B, nullptr, w.SB, d_status, s))) return rc;
    const bool lpt = n_pairs <= kLptMaxPairs;
    if (lpt)
        hipLaunchKernelGGL(k_lpt_order<kLptTile>, dim3((unsigned)((n_pairs + 255) / 256)),
                           dim3(256), 0, s, w.SA, w.SB, ia, ib, n_pairs, w.order);
    if ((rc = fill_i32((int32_t *)w.counter, 1, 0, s))) return rc;
    XlPairArgs xa{w.SA, w.SB, ia, ib, lpt ? w.order : nullptr, n_pairs, dist, w.counter,
                  d_status};
    void *args[] = {&xa};
    if (hipLaunchKernel(xl_pair_kernel(x), dim3(xl_pair_grid(x)), dim3(kXlPairBlock), args, 0,
                        s) != hipSuccess)
        return MSA_EDEVICE;
    return launch_status();
}

int lev_xl_staged(const Staged &A, const Staged &B, int32_t sigma, int32_t max_len,
                  const int32_t *ia, const int32_t *ib, int64_t n_pairs, uint16_t *dist,
                  uint32_t *counter, int32_t *d_status, hipStream_t s) {
    XlPairShape x;
    if (!xl_shape_for((int)std::max<int64_t>(1, ((int64_t)max_len + 63) / 64), sigma, &x))
        return MSA_ERANGE;
    if (n_pairs <= 0) return MSA_OK;
    if (A.stride != B.stride) return MSA_EINVAL;
    const int64_t waves = (n_pairs + kWave / x.g - 1) / (kWave / x.g);
    const int64_t grid = (waves + kXlPairBlock / kWave - 1) / (kXlPairBlock / kWave);
    XlPairArgs xa{A, B, ia, ib, nullptr, n_pairs, dist, counter, d_status};
    void *args[] = {&xa};
    if (hipLaunchKernel(xl_pair_kernel(x), dim3((unsigned)grid), dim3(kXlPairBlock), args, 0,
                        s) != hipSuccess)
        return MSA_EDEVICE;
    return launch_status();
}

// The pair-list layout: forced (1 = lanes, 2 = across lanes, 64 = grouped;
// autotuning), else (forced == 0) the tuning table, else the default: lanes
// whenever the patterns fit it; across lanes for longer patterns with fewer
// than kXlPartners pairs per A sequence on average; else grouped.  A value
// whose layout does not fit the sets falls back to the default.
constexpr int kLayoutXl = 2;
constexpr int64_t kXlPartners = 16;

static int default_layout(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    int wmax, sp;
    XlPairShape x;
    if (lanes_fit(A, B, &wmax, &sp)) return 1;
    if (xl_pairs_shape(A, B, &x) && n_pairs < kXlPartners * std::max<int64_t>(1, A->n))
        return kLayoutXl;
    return kWave;
}

// Workspace of a pair list: enough for every layout that fits the sets and,
// in the grouped one, for the carry buffers of every word class (so that no
// tuning entry can outgrow it).  untuned: only what the default layout and
// class need.
static size_t pairs_ws_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs,
                             bool untuned) {
    int wmax, sp;
    XlPairShape x;
    const bool fit = lanes_fit(A, B, &wmax, &sp);
    const bool xl = xl_pairs_shape(A, B, &x);
    const int dflt = default_layout(A, B, n_pairs);
    size_t total = 0;
    if (!untuned || dflt == kWave) {
        Sizer sg;
        const LevPlan pl = plan_lev(A, B, true, untuned ? -1 : 0);
        carve_grouped(sg, A, B, n_pairs, pl, !untuned);
        total = sg.total();
    }
    if (fit && (!untuned || dflt == 1)) {
        Sizer sl;
        carve_lanes(sl, A, B, n_pairs, wmax);
        total = std::max(total, sl.total());
    }
    if (xl && (!untuned || dflt == kLayoutXl)) {
        Sizer sx;
        carve_xl_pairs(sx, A, B, n_pairs);
        total = std::max(total, sx.total());
    }
    return total;
}

static int run_grouped(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                       int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes,
                       bool untuned, int32_t *d_status, hipStream_t s) {
    int rc;
    const LevPlan pl = plan_lev(A, B, true, untuned ? -1 : 0);
    Carve cv(ws, ws_bytes);
    const GroupedWs w = carve_grouped(cv, A, B, n_pairs, pl, false);
    if (!cv.ok()) return MSA_ENOSPC;
    // A's length ranks (the staged lengths are written again, identically, by
    // the staging below)
    if ((rc = sort_by_length(A, w.SA.len, w.hist, w.order, d_status, s))) return rc;
    if ((rc = stage_set(A, nullptr, w.SA, d_status, s))) return rc;
    if (!same_set(A, B) && (rc = stage_set(B, nullptr, w.SB, d_status, s))) return rc;
    if ((rc = fill_i64(w.start, (int64_t)A->n + 1, 0, s))) return rc;
    const int64_t pg = std::min<int64_t>((n_pairs + 255) / 256, 8192);
    hipLaunchKernelGGL(k_pair_hist, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs, A->n,
                       B->n, w.start, dist, d_status);
    if ((rc = exclusive_scan_i64(w.start, (int64_t)A->n + 1, s))) return rc;
    if (hipMemcpyAsync(w.cursor, w.start, sizeof(int64_t) * ((size_t)A->n + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MSA_EDEVICE;
    hipLaunchKernelGGL(k_pair_scatter, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs,
                       A->n, B->n, w.cursor, w.sorted);
    if (A->n > 0)
        hipLaunchKernelGGL(k_group_sort, dim3((unsigned)A->n), dim3(256), 0, s, w.start,
                           w.sorted, ib, w.SB.len, B->max_len, w.sorted2);
    const unsigned gg = (unsigned)((A->n + 1 + 255) / 256);
    hipLaunchKernelGGL(k_rank_item_counts, dim3(gg), dim3(256), 0, s, w.start, w.order, A->n,
                       w.cursor);
    if ((rc = exclusive_scan_i64(w.cursor, (int64_t)A->n + 1, s))) return rc;
    hipLaunchKernelGGL(k_rank_make_items, dim3(gg), dim3(256), 0, s, w.start, w.cursor, w.order,
                       A->n, w.items, w.n_items);
    if ((rc = fill_i32((int32_t *)w.counter, 1, 0, s))) return rc;
    GroupedArgs ga{w.SA,   w.SB,   ib,       w.sorted2,  w.items, w.n_items,
                   dist,   w.counter, w.hbuf, pl.hstride, A->sigma};
    switch (pl.wclass) {
#define MSADP_L(wc) \
    case wc: hipLaunchKernelGGL(k_lev_grouped<wc>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        MSADP_LEV_CLASSES(MSADP_L)
#undef MSADP_L
        default: return MSA_EINVAL;
    }
    return launch_status();
}

static int run_lanes(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                     int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes, int wmax,
                     int32_t *d_status, hipStream_t s) {
    int rc;
    Carve cv(ws, ws_bytes);
    const LanesWs w = carve_lanes(cv, A, B, n_pairs, wmax);
    if (!cv.ok()) return MSA_ENOSPC;
    const int nb = 16 * wmax + 1;
    const int64_t nkeys = (int64_t)(wmax + 1) * nb;
    if ((rc = stage_set(A, nullptr, w.SA, d_status, s))) return rc;
    if (!same_set(A, B) && (rc = stage_set(B, nullptr, w.SB, d_status, s))) return rc;
    if ((rc = fill_i64(w.counts, nkeys + 1, 0, s))) return rc;
    const int64_t pg = (n_pairs + kBinPairsPerBlock - 1) / kBinPairsPerBlock;
    hipLaunchKernelGGL(k_lanes_hist, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs,
                       w.SA.len, w.SB.len, A->n, B->n, wmax, nb, w.counts, dist, d_status);
    if ((rc = exclusive_scan_i64(w.counts, nkeys + 1, s))) return rc;
    if (hipMemcpyAsync(w.cursor, w.counts, sizeof(int64_t) * (size_t)(nkeys + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MSA_EDEVICE;
    hipLaunchKernelGGL(k_lanes_scatter, dim3((unsigned)pg), dim3(256), 0, s, ia, ib, n_pairs,
                       w.SA.len, w.SB.len, A->n, B->n, wmax, nb, w.cursor, w.sorted);
    const int64_t ig = std::max<int64_t>(1, std::min<int64_t>((n_pairs / 64 + 255) / 256, 1024));
    hipLaunchKernelGGL(k_lanes_items, dim3((unsigned)ig), dim3(256), 0, s, w.counts, wmax, nb,
                       w.items, w.n_items);
    if ((rc = fill_i32((int32_t *)w.counter, 1, 0, s))) return rc;
    LanesArgs la{w.SA, w.SB, ia, ib, w.sorted, w.items, w.n_items, dist, w.counter};
    switch (wmax) {
#define MSADP_L(wc, sp)                                                                     \
    case wc:                                                                                \
        hipLaunchKernelGGL((k_lev_lanes<wc, sp>), dim3(lev_grid(wc, kLanesKernel)), dim3(64), 0, \
                           s, la);                                                          \
        break;
        MSADP_LANES_CLASSES(MSADP_L)
#undef MSADP_L
        default: return MSA_EINVAL;
    }
    return launch_status();
}

// The layout of a lev_batch call (see default_layout).
static int pairs_layout(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs, int forced,
                        int *wmax, XlPairShape *x) {
    int sp;
    const bool fit = lanes_fit(A, B, wmax, &sp);
    const bool xl = xl_pairs_shape(A, B, x);
    const int dflt = default_layout(A, B, n_pairs);
    const int v = forced > 0    ? forced
                  : forced == 0 ? tuned_value(MSA_TUNE_PAIRS, A->sigma, pair_words_bin(A, B), dflt)
                                : dflt;
    if (v == 1 && fit) return 1;
    if (v == kLayoutXl && xl) return kLayoutXl;
    if (v == kWave) return kWave;
    return dflt;
}

size_t lev_batch_ws_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs, bool untuned) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    return pairs_ws_bytes(A, B, n_pairs, untuned);
}

int lev_batch_impl(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                   int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes,
                   int32_t *d_status, hipStream_t s, int forced) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0) return MSA_EINVAL;
    if (A->sigma != B->sigma) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || dist == nullptr || ws == nullptr) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL * 64) return MSA_ERANGE;
    const bool untuned = forced < 0;
    if (ws_bytes < pairs_ws_bytes(A, B, n_pairs, untuned)) return MSA_ENOSPC;
    int wmax;
    XlPairShape x;
    const int layout = pairs_layout(A, B, n_pairs, forced, &wmax, &x);
    if (layout == 1)
        return run_lanes(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, wmax, d_status, s);
    if (layout == kLayoutXl)
        return run_xl_pairs(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, x, d_status, s);
    return run_grouped(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, untuned, d_status, s);
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t lev_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    return lev_batch_ws_bytes(A, B, n_pairs, false);
}

int lev_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
              int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes, int32_t *d_status,
              hipStream_t s) {
    return lev_batch_impl(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, d_status, s, 0);
}

int msa_autotune_pairs(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                       const int32_t *ib, int64_t n_pairs, uint16_t *dist, void *ws,
                       size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                       int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (best == nullptr || best_ms == nullptr || reps < 1 || n_pairs < 1) return MSA_EINVAL;
    int wmax, sp;
    XlPairShape x;
    const bool fit = lanes_fit(A, B, &wmax, &sp);
    const bool xl = xl_pairs_shape(A, B, &x);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MSA_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MSA_EDEVICE;
    }
    int bv = 0;
    float bms = 0.0f;
    rc = MSA_OK;
    for (int v : {kWave, 1, kLayoutXl}) {
        if ((v == 1 && !fit) || (v == kLayoutXl && !xl)) continue;
        if ((rc = lev_batch_impl(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, d_status, s, v)))
            break;   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        for (int r = 0; r < reps && rc == MSA_OK; ++r)
            rc = lev_batch_impl(A, B, ia, ib, n_pairs, dist, ws, ws_bytes, d_status, s, v);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        ms /= (float)reps;
        if (bv == 0 || ms < bms) {
            bv = v;
            bms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = bv;
    *best_ms = bms;
    return msa_tune_set(MSA_TUNE_PAIRS, A->sigma, pair_words_bin(A, B), bv);
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
