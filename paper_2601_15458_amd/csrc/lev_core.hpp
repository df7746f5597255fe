// Bit-parallel Levenshtein core shared by the all-pairs, pair-list and
// tree-level kernels (see lev.hip for the method and the layout).
#pragma once

#include "common.hpp"

namespace msadp {

constexpr int kMaxWords = 32;  // most 64-bit words per pass (2048 rows)
constexpr int kSym = 32;       // symbol stride of the Peq table

typedef const __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint64_t lds_w64;
typedef __attribute__((address_space(3))) uint32_t lds_w32;

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
//        them to the score.  `b` is the bit of the last row in word W-1 (it
//        may differ between lanes).
//   TS, KS: the match word of symbol t and word k is peq[t * TS + k * KS]
//        (a wavefront's shared table: 1, kSym; a lane's own table, with peq
//        already offset to the lane: kWave, sigma' * kWave).
template <int W, bool CIN, int TS = 1, int KS = kSym>
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
        const int steps = (int)uniform((uint32_t)min(16, nmax - j0));
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
            lds_u64 *pe = peq + t * TS;   // this lane's symbol row of the table
            uint32_t dp = 0, dn = 0;
            // Eq of word k+2 is requested while word k computes; the
            // scheduling barriers keep each word's temporaries short-lived.
            uint64_t eq0 = pe[0], eq1 = W > 1 ? pe[KS] : 0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const uint64_t e = (k & 1) ? eq1 : eq0;
                if (k + 2 < W) {
                    if (k & 1) eq1 = pe[(k + 2) * KS];
                    else eq0 = pe[(k + 2) * KS];
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
            // both outputs every column (no branch in the loop): the carry
            // word is stored only when cout, the score used only by a last pass
            ow |= (dp | (dn << 1)) << (2 * jj);
            score += (j0 + jj < n) ? (int)dp - (int)dn : 0;
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

// A lane's own match table for its pattern (pat, m; words [0, nw)), for
// wavefronts whose lanes hold different patterns: tbl[(k * SP + c) * kWave +
// lane] has bit i set iff pat[k * 64 + i] == c, for c < SP (symbols >= SP
// never occur).  Rows past m hold the staged zero padding: they only feed
// rows below the last one, which no result reads.  Each lane ORs one bit per
// pattern symbol into its own entries (no two lanes share an entry).
template <int SP>
__device__ __forceinline__ void build_lane_peq(uint64_t *tbl, const uint8_t *pat, int m,
                                               int nw) {
    const int lane = lane_id();
    lds_w64 *t64 = (lds_w64 *)tbl;
    for (int k = 0; k < nw; ++k) {
#pragma unroll
        for (int c = 0; c < SP; ++c) t64[(k * SP + c) * kWave + lane] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint4 *pp = (const uint4 *)pat;
    for (int k = 0; k < nw; ++k) {
        // 32-bit halves: entry e of the table is dwords 2e (rows 0-31), 2e+1
        lds_w32 *row = (lds_w32 *)(t64 + k * SP * kWave + lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int chunk = k * 4 + q;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (chunk * 16 < m) v = pp[chunk];
            const uint32_t d4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int w = 0; w < 4; ++w) {
#pragma unroll
                for (int by = 0; by < 4; ++by) {
                    const int i = q * 16 + w * 4 + by;   // row within the word
                    const uint32_t c = (d4[w] >> (8 * by)) & 0xFFu;
                    __hip_atomic_fetch_or(row + c * (2 * kWave) + (i >> 5), 1u << (i & 31),
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Two-bit alphabets (sigma <= 4): a lane's pattern as two bit planes per
// word instead of four match masks (half the LDS, so twice the wavefronts
// per CU).  tbl[k * kWave + lane] = (plane 0 lo, hi, plane 1 lo, hi) of word
// k, plane b holding bit b of each row's symbol.  Built in registers: the
// bit b of the four symbols of a dword is gathered into four adjacent bits
// by one multiply (bits at 0, 8, 16, 24 times 2^28 + 2^21 + 2^14 + 2^7 land
// at 28 .. 31 with no carries between the partial products).
__device__ __forceinline__ void build_lane_planes(uint4 *tbl, const uint8_t *pat, int m, int nw) {
    const int lane = lane_id();
    const uint4 *pp = (const uint4 *)pat;
    for (int k = 0; k < nw; ++k) {
        uint32_t p0l = 0, p0h = 0, p1l = 0, p1h = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int chunk = k * 4 + q;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (chunk * 16 < m) v = pp[chunk];
            const uint32_t d4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t b0 = ((d4[w] & 0x01010101u) * 0x10204080u) >> 28;
                const uint32_t b1 = (((d4[w] >> 1) & 0x01010101u) * 0x10204080u) >> 28;
                const int sh = 4 * ((q * 4 + w) & 7);   // row 4 (4q + w) within its half
                if (q < 2) {
                    p0l |= b0 << sh;
                    p1l |= b1 << sh;
                } else {
                    p0h |= b0 << sh;
                    p1h |= b1 << sh;
                }
            }
        }
        tbl[k * kWave + lane] = make_uint4(p0l, p0h, p1l, p1h);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) u32x4 lds_u128;

// lev_pass for a lane's bit-plane table (first and only pass; see lev_pass).
// The match mask of symbol t is ~((P0 ^ s0) | (P1 ^ s1)) with sb = all ones
// where bit b of t is 1 (a sign-extended bit field).  Holding the planes in
// registers instead of LDS was tried: 148 VGPRs for 8 words, 3 wavefronts
// per SIMD instead of 5, and slower.
template <int W>
__device__ __forceinline__ int lev_pass_planes(lds_u128 *tbl, const uint8_t *text, int n,
                                               int nmax, int b) {
    constexpr uint8_t kNorXor = MSADP_LUT(~(A | (B ^ C)));
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
        uint32_t c0 = cur.x, c1 = cur.y, c2 = cur.z, c3 = cur.w;
        const int steps = (int)uniform((uint32_t)min(16, nmax - j0));
        for (int j4 = 0; j4 < steps; j4 += 4) {
            const uint32_t wd = c0;      // symbols j4 .. j4 + 3, one byte each
            c0 = c1;
            c1 = c2;
            c2 = c3;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
            const int jj = j4 + u;
            if (jj >= steps) break;      // uniform
            // s0, s1: all ones where bit 0, 1 of the text symbol is set
            const uint32_t s0 = (uint32_t)((int32_t)(wd << (31 - 8 * u)) >> 31);
            const uint32_t s1 = (uint32_t)((int32_t)(wd << (30 - 8 * u)) >> 31);
            uint32_t cph = 1u << 31, cmh = 0u;   // top row: +1
            uint32_t dp = 0, dn = 0;
            u32x4 q0 = tbl[0], q1 = {0u, 0u, 0u, 0u};
            if (W > 1) q1 = tbl[kWave];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const u32x4 q = (k & 1) ? q1 : q0;
                if (k + 2 < W) {
                    if (k & 1) q1 = tbl[(k + 2) * kWave];
                    else q0 = tbl[(k + 2) * kWave];
                }
                const uint32_t el = bop3<kNorXor>(q.x ^ s0, q.z, s1);
                const uint32_t eh = bop3<kNorXor>(q.y ^ s0, q.w, s1);
                const uint32_t elm = el | (cmh >> 31);
                const uint32_t xvl = el | ml[k], xvh = eh | mh[k];
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
                asm volatile("" : "+v"(cph), "+v"(cmh), "+v"(pl[k]), "+v"(ph[k]), "+v"(ml[k]),
                             "+v"(mh[k]));
            }
            score += (j0 + jj < n) ? (int)dp - (int)dn : 0;
            }
        }
        cur = nxt;
    }
    return score;
}

template <int WMAX, int W = 1>
__device__ __forceinline__ int dispatch_planes(int w, lds_u128 *tbl, const uint8_t *text, int n,
                                               int nmax, int b) {
    if constexpr (W > WMAX) {
        return 0;
    } else {
        if (w == W) return lev_pass_planes<W>(tbl, text, n, nmax, b);
        return dispatch_planes<WMAX, W + 1>(w, tbl, text, n, nmax, b);
    }
}

template <int WMAX, int SP, int W = 1>
__device__ __forceinline__ int dispatch_lanes(int w, lds_u64 *tbl, const uint8_t *text, int n,
                                              int nmax, int b) {
    if constexpr (W > WMAX) {
        return 0;
    } else {
        if (w == W)
            return lev_pass<W, false, kWave, SP * kWave>(tbl, text, n, nmax, b, false, nullptr);
        return dispatch_lanes<WMAX, SP, W + 1>(w, tbl, text, n, nmax, b);
    }
}

// Distance between this wavefront's pattern (pat, m) and each lane's text
// (text, n; lanes with valid == false still take part but their result is
// ignored).  A pattern of more than WMAX words runs as several passes (the
// first takes the remainder, the others WMAX words each); `hbuf` is this
// lane's carry buffer between passes (needed when m > 64 * WMAX).  peq holds
// WMAX words of the table.
template <int WMAX>
__device__ __forceinline__ int lev_item(uint64_t *peq, const uint8_t *pat, int m, int sigma,
                                        const uint8_t *text, int n, bool valid, uint32_t *hbuf) {
    const int nmax = (int)uniform((uint32_t)wave_max(valid ? n : 0));
    if (m == 0) return n;
    if (nmax == 0) return m;
    const int words = (m + 63) >> 6;
    const int passes = (words + WMAX - 1) / WMAX;
    const int w_first = words - (passes - 1) * WMAX;
    const int b_last = (m - 1) & 63;
    build_peq(peq, pat, m, 0, w_first, sigma);
    lds_u64 *tbl = (lds_u64 *)peq;
    int s = dispatch_first<WMAX>(w_first, tbl, text, n, nmax, passes == 1 ? b_last : 63,
                                 passes > 1, hbuf);
    for (int p = 1; p < passes; ++p) {
        const int w0 = w_first + (p - 1) * WMAX;
        build_peq(peq, pat, m, w0, WMAX, sigma);
        const bool last = (p == passes - 1);
        s = lev_pass<WMAX, true>(tbl, text, n, nmax, last ? b_last : 63, !last, hbuf);
    }
    return m + s;
}

// Next work item of a persistent kernel.  Every lane executes the atomic
// (lane 0 adds 1, the others 0) so the loop holds no lane-conditional
// branch; the compiler may otherwise restructure a lane-0 branch around the
// loop back edge and let the other lanes re-enter without lane 0.
__device__ __forceinline__ uint32_t next_item(uint32_t *counter) {
    const uint32_t lane0 = lane_id() == 0 ? 1u : 0u;
    const uint32_t it = atomicAdd(counter, lane0);
    return uniform(__builtin_amdgcn_readlane(it, 0));
}

// Work items of a persistent kernel: wavefront w of the grid starts with
// item w, with no atomic, and takes later items from the counter (offset by
// the grid's wavefront count).  Every wavefront that finds no work then exits
// without touching the counter: atomics on one address serialize (about
// 12 ns each), so a launch whose few items all went to the first wavefronts
// used to cost 60-100 us in fetches that found nothing.
//   for (uint32_t it = first_item();; it = later_item(counter)) {
//       if (it >= total) break;
//       ...
//   }
__device__ __forceinline__ uint32_t first_item() {
    return uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
}

__device__ __forceinline__ uint32_t later_item(uint32_t *counter) {
    return gridDim.x * (blockDim.x / kWave) + next_item(counter);
}

__host__ __device__ inline int64_t items_upto(int64_t U) {
    // sum_{u=1..U} ceil(u/64): work items of a triangle whose rows hold 1..U texts
    const int64_t Q = U >> 6, s = U & 63;
    return 32 * Q * (Q + 1) + s * (Q + 1);
}

// Smallest u >= 1 with items_upto(u) > g (u in [1, hi]).
__device__ __forceinline__ int64_t triangle_row(int64_t g, int64_t hi) {
    int64_t lo = 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (items_upto(mid) > g) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Pattern words per pass that a kernel variant is compiled for; a variant
// holds 4 VGPRs of state per word, so small patterns get more wavefronts.
// The tree build uses the classes of wmax_class; the pair kernels also have
// 20 and 28, which a tuning entry may select.
inline int wmax_class(int32_t pat_max) {
    const int w = (pat_max + 63) / 64;
    if (w <= 4) return 4;
    if (w <= 8) return 8;
    if (w <= 16) return 16;
    if (w <= 24) return 24;
    return kMaxWords;
}

constexpr int kLevClasses[] = {4, 8, 16, 20, 24, 28, 32};

inline bool is_lev_class(int c) {
    for (int x : kLevClasses)
        if (x == c) return true;
    return false;
}

// Variants of the tree build's medoid and pole kernels.
constexpr int kTreeClasses[] = {4, 8, 16, 20, 24, 32};

inline bool is_tree_class(int c) {
    for (int x : kTreeClasses)
        if (x == c) return true;
    return false;
}

// A tuned class may take at most this many passes over the longest pattern
// (the default's count, and at least two).
inline bool class_within_passes(int32_t pat_max, int c) {
    const int words = pat_max > 64 ? (pat_max + 63) / 64 : 1;
    const int dflt = wmax_class(pat_max);
    const int max_passes = (words + dflt - 1) / dflt > 2 ? (words + dflt - 1) / dflt : 2;
    return (words + c - 1) / c <= max_passes;
}

// Passes of a class over patterns of up to pat_max rows need a carry buffer.
inline bool needs_passes(int32_t pat_max, int wclass) { return pat_max > wclass * 64; }

// Workgroups of one wavefront that fit on the device at once for `kernel`.
template <class K>
inline int persistent_grid(K kernel) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 64, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return device_cus() * blocks;
}

}  // namespace msadp
