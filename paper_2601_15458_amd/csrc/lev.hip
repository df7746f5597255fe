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
// depends on the lane's text symbol.  Patterns longer than 2048 rows run as
// several passes of 32 words; the horizontal deltas leaving a pass (2 bits
// per text column) go through a per-lane buffer in the workspace.
//
// Per text symbol t and word k (Eq = Peq[k][t]; hin = horizontal delta
// entering the word from below-left, +1 for the top row):
//   Xv = Eq | Mv;  Eq' = Eq | [hin < 0];
//   Xh = (((Eq' & Pv) + Pv) ^ Pv) | Eq';
//   Ph = Mv | ~(Xh | Pv);  Mh = Pv & Xh;  hout = sign bit of Ph/Mh row;
//   Ph = (Ph << 1) | [hin > 0];  Mh = (Mh << 1) | [hin < 0];
//   Pv = Mh | ~(Xv | Ph);  Mv = Ph & Xv.
// The distance is m plus the sum of the horizontal deltas of the last row.
#include "common.hpp"

namespace msadp {

constexpr int kMaxWords = 32;  // 64-bit words per pass (2048 rows)
constexpr int kSym = 32;       // symbol stride of the Peq table

typedef const __attribute__((address_space(3))) uint64_t lds_u64;

struct Lut {
    static constexpr uint8_t XOR_OR = MSADP_LUT((A ^ B) | C);     // Xh
    static constexpr uint8_t PH = MSADP_LUT(C | ~(A | B));        // Ph = Mv | ~(Xh | Pv)
    static constexpr uint8_t PV = MSADP_LUT(A | ~(B | C));        // Pv = Mh | ~(Xv | Ph)
};

// Build this wavefront's Peq table for pattern words [w0, w0 + nw):
// peq[k * kSym + c] has bit i set iff pattern[(w0 + k) * 64 + i] == c.
__device__ __forceinline__ void build_peq(uint64_t *peq, const uint8_t *pat, int m, int w0,
                                          int nw, int sigma) {
    const int lane = lane_id();
    for (int k = 0; k < nw; ++k) {
        const int i = (w0 + k) * 64 + lane;
        const int c = i < m ? (int)pat[i] : 255;
        uint64_t mine = 0;
        for (int s = 0; s < sigma; ++s) {
            const uint64_t bal = __ballot(c == s);
            if (lane == s) mine = bal;
        }
        if (lane < kSym) peq[k * kSym + lane] = mine;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pass of W words over the lane's text.
//   CIN: the horizontal deltas entering word 0 come from `hbuf` (2 bits per
//        column: bit 2q = +1, bit 2q+1 = -1), else they are +1 (top row).
//   cout: write the deltas leaving the last word to `hbuf` instead of adding
//        them to the score.  `b` is the bit of the last row in word W-1.
template <int W, bool CIN>
__device__ __forceinline__ int lev_pass(lds_u64 *peq, const uint8_t *text, int n, int nmax,
                                        int b, bool cout, uint32_t *hbuf) {
    uint32_t pl[W], ph[W], ml[W], mh[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        pl[k] = ph[k] = ~0u;
        ml[k] = mh[k] = 0u;
    }
    int score = 0;
    const uint4 *tp = (const uint4 *)text;
    uint4 cur = tp[0];
    for (int j0 = 0; j0 < nmax; j0 += 16) {
        uint4 nxt = cur;
        if (j0 + 16 < nmax) nxt = tp[(j0 >> 4) + 1];
        uint32_t cw = CIN ? hbuf[(j0 >> 4) * kWave] : 0x55555555u;
        uint32_t ow = 0;
        uint32_t c0 = cur.x, c1 = cur.y, c2 = cur.z, c3 = cur.w;
        const int steps = min(16, nmax - j0);
        for (int jj = 0; jj < steps; ++jj) {
            const uint32_t t = c0 & 0xFFu;
            c0 = __builtin_amdgcn_alignbyte(c1, c0, 1);
            c1 = __builtin_amdgcn_alignbyte(c2, c1, 1);
            c2 = __builtin_amdgcn_alignbyte(c3, c2, 1);
            c3 >>= 8;
            // carry into word 0, kept as "bit 31 of the previous word's hi half"
            uint32_t cph = cw << 31;
            uint32_t cmh = (cw & 2u) << 30;
            cw >>= 2;
            lds_u64 *pe = peq + t;   // this lane's symbol row of the table
            uint32_t dp = 0, dn = 0;
            // Eq of word k+2 is requested while word k computes; the
            // scheduling barriers keep each word's temporaries short-lived.
            uint64_t eq0 = pe[0], eq1 = W > 1 ? pe[kSym] : 0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const uint64_t e = (k & 1) ? eq1 : eq0;
                if (k + 2 < W) {
                    if (k & 1) eq1 = pe[(k + 2) * kSym];
                    else eq0 = pe[(k + 2) * kSym];
                }
                const uint32_t el = (uint32_t)e, eh = (uint32_t)(e >> 32);
                const uint32_t elm = el | (cmh >> 31);
                const uint32_t xvl = el | ml[k], xvh = eh | mh[k];
                // 64-bit (Eq' & Pv) + Pv as an add with carry on 32-bit halves
                unsigned int cy, cy2;
                const uint32_t sl = __builtin_addc(elm & pl[k], pl[k], 0u, &cy);
                const uint32_t sh = __builtin_addc(eh & ph[k], ph[k], cy, &cy2);
                const uint32_t xhl = bop3<Lut::XOR_OR>(sl, pl[k], elm);
                const uint32_t xhh = bop3<Lut::XOR_OR>(sh, ph[k], eh);
                const uint32_t phl = bop3<Lut::PH>(xhl, pl[k], ml[k]);
                const uint32_t phh = bop3<Lut::PH>(xhh, ph[k], mh[k]);
                const uint32_t mhl = pl[k] & xhl, mhh = ph[k] & xhh;
                if (k == W - 1) {
                    const uint64_t P = ((uint64_t)phh << 32) | phl;
                    const uint64_t M = ((uint64_t)mhh << 32) | mhl;
                    dp = (uint32_t)(P >> b) & 1u;
                    dn = (uint32_t)(M >> b) & 1u;
                }
                const uint32_t Phl = shl1_carry(phl, cph), Phh = shl1_carry(phh, phl);
                const uint32_t Mhl = shl1_carry(mhl, cmh), Mhh = shl1_carry(mhh, mhl);
                cph = phh;
                cmh = mhh;
                pl[k] = bop3<Lut::PV>(Mhl, xvl, Phl);
                ph[k] = bop3<Lut::PV>(Mhh, xvh, Phh);
                ml[k] = Phl & xvl;
                mh[k] = Phh & xvh;
                // Tie the carries for word k+1 to word k's finished state so
                // the compiler cannot run the carry chain ahead of the state
                // updates (which would keep ~6 extra VGPRs per word alive).
                asm volatile("" : "+v"(cph), "+v"(cmh), "+v"(pl[k]), "+v"(ph[k]), "+v"(ml[k]),
                             "+v"(mh[k]));
            }
            if (cout) {
                ow |= (dp | (dn << 1)) << (2 * jj);
            } else {
                const int d = (int)dp - (int)dn;
                score += (j0 + jj < n) ? d : 0;
            }
        }
        if (cout) hbuf[(j0 >> 4) * kWave] = ow;
        cur = nxt;
    }
    return score;
}

template <int WMAX, int W = 1>
__device__ __forceinline__ int dispatch_first(int w, lds_u64 *peq, const uint8_t *text, int n,
                                              int nmax, int b, bool cout, uint32_t *hbuf) {
    if constexpr (W > WMAX) {
        return 0;
    } else {
        if (w == W) return lev_pass<W, false>(peq, text, n, nmax, b, cout, hbuf);
        return dispatch_first<WMAX, W + 1>(w, peq, text, n, nmax, b, cout, hbuf);
    }
}

// Distance between this wavefront's pattern (pat, m) and each lane's text
// (text, n; lanes with valid == false still take part but their result is
// ignored).  `hbuf` is this lane's carry buffer (used when m > 2048).
template <int WMAX>
__device__ __forceinline__ int lev_item(uint64_t *peq, const uint8_t *pat, int m, int sigma,
                                        const uint8_t *text, int n, bool valid, uint32_t *hbuf) {
    const int nmax = (int)uniform((uint32_t)wave_max(valid ? n : 0));
    if (m == 0) return n;
    if (nmax == 0) return m;
    const int words = (m + 63) >> 6;
    const int passes = (words + kMaxWords - 1) / kMaxWords;
    const int w_first = words - (passes - 1) * kMaxWords;
    const int b_last = (m - 1) & 63;
    build_peq(peq, pat, m, 0, w_first, sigma);
    lds_u64 *tbl = (lds_u64 *)peq;
    int s = dispatch_first<WMAX>(w_first, tbl, text, n, nmax, passes == 1 ? b_last : 63,
                                 passes > 1, hbuf);
    if constexpr (WMAX == kMaxWords)
    for (int p = 1; p < passes; ++p) {
        const int w0 = w_first + (p - 1) * kMaxWords;
        build_peq(peq, pat, m, w0, kMaxWords, sigma);
        const bool last = (p == passes - 1);
        s = lev_pass<kMaxWords, true>(tbl, text, n, nmax, last ? b_last : 63, !last, hbuf);
    }
    return m + s;
}

__device__ __forceinline__ uint32_t next_item(uint32_t *counter) {
    uint32_t it = 0;
    if (lane_id() == 0) it = atomicAdd(counter, 1u);
    return uniform(__shfl(it, 0, kWave));
}

// ------------------------------------------------------------ all pairs
// Rows are ranks in length order.  The pattern of row r is the sequence of
// rank r, its texts are the ranks r+1 .. N-1 (no shorter than the pattern),
// in blocks of 64.  Items are numbered so that u = N-1-r grows with the item
// id: S(U) = sum_{u=1..U} ceil(u/64) items precede row U+1; item 0 is the
// longest pattern, so the largest items start first.
__host__ __device__ inline int64_t items_upto(int64_t U) {
    const int64_t Q = U >> 6, s = U & 63;
    return 32 * Q * (Q + 1) + s * (Q + 1);
}

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
    __shared__ uint64_t peq[kMaxWords * kSym];
    const int lane = lane_id();
    const int64_t N = a.S.n;
    uint32_t *hb = a.hbuf ? a.hbuf + (int64_t)blockIdx.x * a.hstride * kWave + lane : nullptr;
    for (;;) {
        const uint32_t it = next_item(a.counter);
        if ((int64_t)it >= a.n_items) break;
        const int64_t g = (int64_t)it;
        // find u with items_upto(u-1) <= g < items_upto(u)
        int64_t lo = 1, hi = N - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (items_upto(mid) > g) hi = mid; else lo = mid + 1;
        }
        const int64_t u = lo;
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
    __shared__ uint64_t peq[kMaxWords * kSym];
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
static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

// Pattern words per pass that a kernel variant is compiled for; a variant
// holds 4 VGPRs of state per word, so small patterns get more wavefronts.
static int wmax_class(int32_t pat_max) {
    const int w = (pat_max + 63) / 64;
    if (w <= 4) return 4;
    if (w <= 8) return 8;
    if (w <= 16) return 16;
    if (w <= 24) return 24;
    return kMaxWords;
}

template <class K>
static int persistent_grid(K kernel) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 64, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return device_cus() * blocks;
}

static int lev_grid(int wclass, bool grouped) {
    static int cache[2][33];
    int &g = cache[grouped][wclass];
    if (g == 0) {
        switch (wclass) {
#define MSADP_G(w) \
    case w: g = grouped ? persistent_grid(k_lev_grouped<w>) : persistent_grid(k_lev_allpairs<w>); break;
            MSADP_G(4) MSADP_G(8) MSADP_G(16) MSADP_G(24) MSADP_G(32)
#undef MSADP_G
            default: g = device_cus();
        }
    }
    return g;
}

static int64_t hbuf_stride(int32_t text_max) { return ((int64_t)text_max + 15) / 16; }

static bool needs_passes(int32_t pat_max) { return pat_max > kMaxWords * 64; }

struct LevPlan {
    int64_t strideA, strideB, hstride;
    int grid, wclass;
};

template <class Alloc>
static void lev_layout(Alloc &al, const msa_seqs *A, const msa_seqs *B, int64_t n_pairs,
                       const LevPlan &pl, bool grouped) {
    al.template take<uint8_t>((size_t)A->n * pl.strideA);
    al.template take<int32_t>((size_t)A->n + 1);
    if (grouped) {
        al.template take<uint8_t>((size_t)B->n * pl.strideB);
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
    if (pl.hstride) al.template take<uint32_t>((size_t)pl.grid * kWave * pl.hstride);
}

static LevPlan plan_grouped(const msa_seqs *A, const msa_seqs *B) {
    LevPlan p;
    p.strideA = staged_stride(A->max_len);
    p.strideB = staged_stride(B->max_len);
    p.wclass = wmax_class(A->max_len);
    p.grid = lev_grid(p.wclass, true);
    p.hstride = needs_passes(A->max_len) ? hbuf_stride(B->max_len) : 0;
    return p;
}

static LevPlan plan_allpairs(const msa_seqs *A) {
    LevPlan p;
    p.strideA = p.strideB = staged_stride(A->max_len);
    p.wclass = wmax_class(A->max_len);
    p.grid = lev_grid(p.wclass, false);
    p.hstride = needs_passes(A->max_len) ? hbuf_stride(A->max_len) : 0;
    return p;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t lev_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    Sizer sz;
    lev_layout(sz, A, B, n_pairs, plan_grouped(A, B), true);
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
    const LevPlan pl = plan_grouped(A, B);
    Sizer sz;
    lev_layout(sz, A, B, n_pairs, pl, true);
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
        case 4: hipLaunchKernelGGL(k_lev_grouped<4>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        case 8: hipLaunchKernelGGL(k_lev_grouped<8>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        case 16: hipLaunchKernelGGL(k_lev_grouped<16>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        case 24: hipLaunchKernelGGL(k_lev_grouped<24>, dim3(pl.grid), dim3(64), 0, s, ga); break;
        default: hipLaunchKernelGGL(k_lev_grouped<32>, dim3(pl.grid), dim3(64), 0, s, ga); break;
    }
    return launch_status();
}

size_t lev_allpairs_workspace_bytes(const msa_seqs *A) {
    if (check_seqs(A)) return 0;
    Sizer sz;
    lev_layout(sz, A, A, 0, plan_allpairs(A), false);
    return sz.total();
}

int lev_allpairs(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                 int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A))) return rc;
    if (A->n < 2) return MSA_OK;
    if (condensed == nullptr || ws == nullptr) return MSA_EINVAL;
    const LevPlan pl = plan_allpairs(A);
    Sizer sz;
    lev_layout(sz, A, A, 0, pl, false);
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
        case 4: hipLaunchKernelGGL(k_lev_allpairs<4>, dim3(pl.grid), dim3(64), 0, s, aa); break;
        case 8: hipLaunchKernelGGL(k_lev_allpairs<8>, dim3(pl.grid), dim3(64), 0, s, aa); break;
        case 16: hipLaunchKernelGGL(k_lev_allpairs<16>, dim3(pl.grid), dim3(64), 0, s, aa); break;
        case 24: hipLaunchKernelGGL(k_lev_allpairs<24>, dim3(pl.grid), dim3(64), 0, s, aa); break;
        default: hipLaunchKernelGGL(k_lev_allpairs<32>, dim3(pl.grid), dim3(64), 0, s, aa); break;
    }
    return launch_status();
}

}  // extern "C"
