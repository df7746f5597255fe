// Bit-parallel Levenshtein with a pattern's words spread across lanes.
//
// A group of G consecutive lanes computes one pair (pattern, text).  Lane r
// of the group holds pattern words [r WL, r WL + WL) (64 rows each) as NB
// bit planes in registers: plane b has bit i set iff bit b of row i's symbol
// is set, so a word's match mask for symbol c is the AND over b of
// (plane b XNOR bit b of c).  The rows run the column recurrence of Myers'
// bit-vector algorithm as extended to several words by Hyyrö (the same
// vectors as lev_core.hpp): word k of column j needs the horizontal delta
// leaving the bottom row of word k - 1 in the same column, so the lanes are
// skewed by one column each: at step t lane r works on column t - r, and
// what it sends down (the +1 and -1 carries of its last word, and the text
// symbol it used) reaches lane r + 1 one step later through a one-lane DPP
// wavefront shift.  Lane 0 of a group reads the text and feeds the top row
// (+1 into every column).
//
// A lane works only on its columns 0 .. n-1: the step runs under the lane
// mask of (t - r) < n, so a lane's vector state is the initial column before
// its first step and the last column after its last one.  The distance is
// then read from the last column instead of summing the bottom row over the
// columns: D(m, n) = n + sum over the pattern's rows of the last column's
// vertical deltas (+1 where Pv is set, -1 where Mv is), a popcount per lane
// and a sum over the group once per pair.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace msadp {

constexpr int kDppWaveShr1x = 0x138;   // DPP wave_shr:1: lane i reads lane i - 1

struct XlLut {
    static constexpr uint8_t XOR_OR = MSADP_LUT((A ^ B) | C);
    static constexpr uint8_t PH = MSADP_LUT(C | ~(A | B));
    static constexpr uint8_t PV = MSADP_LUT(A | ~(B | C));
    static constexpr uint8_t OR_XOR = MSADP_LUT(A | (B ^ C));
    static constexpr uint8_t NOR_XOR = MSADP_LUT(~(A | (B ^ C)));
};

// Bit plane count of an alphabet: symbols are codes 0 .. sigma - 1.
__host__ __device__ inline int xl_planes(int sigma) { return sigma <= 4 ? 2 : 5; }

// A tree build's use of the across-lanes passes, as one tuning value:
// (WL << 28) | (pole cap << 14) | sum cap.  WL = words per lane (1 or 2);
// a cap is the largest cluster whose passes of that kind run across lanes
// (0: none, kXlCapAll: every cluster).
constexpr int kXlCapAll = (1 << 14) - 1;
inline int xl_value(int wl, int sum_cap, int pole_cap) {
    return (wl << 28) | (pole_cap << 14) | sum_cap;
}
inline int xl_value_wl(int v) { return v >> 28; }
inline int32_t xl_cap_of(int c) { return c == kXlCapAll ? (int32_t)(1 << 30) : (int32_t)c; }
inline int32_t xl_value_sum_cap(int v) { return xl_cap_of(v & kXlCapAll); }
inline int32_t xl_value_pole_cap(int v) { return xl_cap_of((v >> 14) & kXlCapAll); }
inline bool xl_value_valid(int v) {
    return v > 0 && (xl_value_wl(v) == 1 || xl_value_wl(v) == 2);
}
inline int xl_default_value() { return xl_value(2, 128, kXlCapAll); }
// What the tree autotuner tries: off, poles only, and both kinds up to a cap.
constexpr int kXlCandidates[] = {
    (1 << 28),                                         // off
    (1 << 28) | (kXlCapAll << 14),                     // pole passes only
    (1 << 28) | (kXlCapAll << 14) | 32,  (2 << 28) | (kXlCapAll << 14) | 32,
    (1 << 28) | (kXlCapAll << 14) | 64,  (2 << 28) | (kXlCapAll << 14) | 64,
    (1 << 28) | (kXlCapAll << 14) | 128, (2 << 28) | (kXlCapAll << 14) | 128,
    (1 << 28) | (kXlCapAll << 14) | 256, (2 << 28) | (kXlCapAll << 14) | 256,
    (1 << 28) | (kXlCapAll << 14) | kXlCapAll,
};

// Planes of pattern word k (rows 64 k .. 64 k + 63; lo = rows 0-31 of the
// word, hi = rows 32-63).  Rows at or past m read the staged zero padding or
// are not loaded (16-byte chunks that start at or past m): they lie below the
// pattern's last row, which is all that any result reads.  Bit b of the four
// symbols of a dword is gathered into four adjacent bits by one multiply
// (bits at 0, 8, 16, 24 times 2^28 + 2^21 + 2^14 + 2^7 land at 28 .. 31 and
// no two partial products meet).
template <int NB>
__device__ __forceinline__ void xl_word_planes(const uint8_t *pat, int m, int k,
                                               uint32_t (&lo)[NB], uint32_t (&hi)[NB]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) lo[b] = hi[b] = 0u;
    const uint4 *pp = (const uint4 *)pat + 4 * k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if ((4 * k + q) * 16 < m) v = pp[q];
        const uint32_t d4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int sh = 4 * ((4 * q + w) & 7);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint32_t bits = (((d4[w] >> b) & 0x01010101u) * 0x10204080u) >> 28;
                if (q < 2) lo[b] |= bits << sh;
                else hi[b] |= bits << sh;
            }
        }
    }
}

// Match mask half of one word: ~OR over b of (plane b ^ s_b), s_b = all ones
// where bit b of the symbol is set.
template <int NB>
__device__ __forceinline__ uint32_t xl_eq(const uint32_t (&pl)[NB], const uint32_t (&s)[NB]) {
    if constexpr (NB == 1) {
        return ~(pl[0] ^ s[0]);
    } else {
        uint32_t x = pl[0] ^ s[0];
#pragma unroll
        for (int b = 1; b < NB - 1; ++b) x = bop3<XlLut::OR_XOR>(x, pl[b], s[b]);
        return bop3<XlLut::NOR_XOR>(x, pl[NB - 1], s[NB - 1]);
    }
}

// Sum of v over the G lanes of each group (every lane of the group gets it).
template <int G>
__device__ __forceinline__ int xl_group_sum(int v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Segmented reduction over the groups of a wavefront: every lane of group g
// holds (slot, v), groups of one slot are contiguous, and slot -1 marks a
// group with nothing to add.  Returns, in the lanes of each run's first
// group, the run's sum (MAX = false) or maximum, and sets head there.  All
// lanes must call it.
template <int G, bool MAX>
__device__ __forceinline__ uint64_t xl_segment(int64_t slot, uint64_t v, bool &head) {
    constexpr int kGroups = kWave / G;
    const int grp = lane_id() / G;
#pragma unroll
    for (int o = 1; o < kGroups; o <<= 1) {
        const int64_t os = __shfl_down(slot, o * G, kWave);
        const uint64_t ov = __shfl_down(v, o * G, kWave);
        if (grp + o < kGroups && os == slot) v = MAX ? (ov > v ? ov : v) : v + ov;
    }
    const int64_t ps = __shfl_up(slot, G, kWave);
    head = slot >= 0 && (grp == 0 || ps != slot);
    return v;
}

// Distance of this group's pair: pattern row `pat` (m symbols, staged with
// zero padding), text row `text` (n symbols; 16-byte aligned, readable up to
// byte tlim + 16).  Every lane of the wavefront must call it (the steps run
// in lockstep across groups); lanes of a group without a pair pass
// live = false.  Needs m <= 64 G WL.  Returns D(pattern, text) in every lane
// of a live group.
template <int G, int WL, int NB>
__device__ __forceinline__ int xl_distance(const uint8_t *pat, int m, const uint8_t *text, int n,
                                           int64_t tlim, bool live) {
    const int r = lane_id() & (G - 1);
    const bool first = r == 0;
    const int words = live ? (m + 63) >> 6 : 0;
    const int used = (words + WL - 1) / WL;
    uint32_t qlo[WL][NB], qhi[WL][NB];
    uint32_t pl[WL], ph[WL], ml[WL], mh[WL];
#pragma unroll
    for (int s = 0; s < WL; ++s) {
        const int k = r * WL + s;
        if (k < words) {
            xl_word_planes<NB>(pat, m, k, qlo[s], qhi[s]);
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) qlo[s][b] = qhi[s][b] = 0u;
        }
        pl[s] = ph[s] = ~0u;
        ml[s] = mh[s] = 0u;
    }
    const uint32_t nl = (live && r < used) ? (uint32_t)n : 0u;
    // steps, rounded up to whole 16-symbol blocks: past the last column of
    // every group no lane is active, and a step only moves the packets
    const int T = (int)uniform(
        (uint32_t)wave_max(live && n > 0 && used > 0 ? (n + used - 1 + 15) & ~15 : 0));
    // A block of 16 steps in which every lane of a pattern word is inside
    // its columns (t0 >= G - 1 and t0 + 16 <= the shortest text of the
    // wavefront) runs with no lane mask: the lanes past a group's pattern
    // then compute values that only flow into other such lanes (or into a
    // group's lane 0, which reads the text instead) and whose rows the
    // final count masks out.
    const int nmin = -wave_max(live && used > 0 ? -n : INT32_MIN + 1);
    uint32_t oph = 0u, opk = 0u;
    auto step = [&](uint32_t fresh, int t, auto masked) {
        // lane 0 of the wavefront has no source (it is a group's first
        // lane, which does not read these)
        const uint32_t rph = __builtin_amdgcn_mov_dpp((int)oph, kDppWaveShr1x, 0xF, 0xF, true);
        const uint32_t rpk = __builtin_amdgcn_mov_dpp((int)opk, kDppWaveShr1x, 0xF, 0xF, true);
        if (!decltype(masked)::value || (uint32_t)(t - r) < nl) {
            // carries in: bit 31 of cph (+1) and of cmh (-1); the symbol
            // rides in the low bits of the -1 packet
            uint32_t cph = first ? 0x80000000u : rph;
            uint32_t cmh = first ? fresh : rpk;
            const uint32_t pk = cmh;
            uint32_t sb[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) sb[b] = (uint32_t)__builtin_amdgcn_sbfe((int)pk, b, 1);
#pragma unroll
            for (int s = 0; s < WL; ++s) {
                const uint32_t el = xl_eq<NB>(qlo[s], sb);
                const uint32_t eh = xl_eq<NB>(qhi[s], sb);
                const uint32_t elm = el | (cmh >> 31);
                const uint32_t xvl = el | ml[s], xvh = eh | mh[s];
                unsigned int cy, cy2;
                const uint32_t sl = __builtin_addc(elm & pl[s], pl[s], 0u, &cy);
                const uint32_t sh = __builtin_addc(eh & ph[s], ph[s], cy, &cy2);
                const uint32_t xhl = bop3<XlLut::XOR_OR>(sl, pl[s], elm);
                const uint32_t xhh = bop3<XlLut::XOR_OR>(sh, ph[s], eh);
                const uint32_t phl = bop3<XlLut::PH>(xhl, pl[s], ml[s]);
                const uint32_t phh = bop3<XlLut::PH>(xhh, ph[s], mh[s]);
                const uint32_t mhl = pl[s] & xhl, mhh = ph[s] & xhh;
                const uint32_t Phl = shl1_carry(phl, cph), Phh = shl1_carry(phh, phl);
                const uint32_t Mhl = shl1_carry(mhl, cmh), Mhh = shl1_carry(mhh, mhl);
                cph = phh;
                cmh = mhh;
                pl[s] = bop3<XlLut::PV>(Mhl, xvl, Phl);
                ph[s] = bop3<XlLut::PV>(Mhh, xvh, Phh);
                ml[s] = Phl & xvl;
                mh[s] = Phh & xvh;
            }
            oph = cph;
            opk = (cmh & 0x80000000u) | (pk & 0x7FFFFFFFu);
        }
    };
    const uint4 *tp = (const uint4 *)text;
    uint4 cur = tp[0];
    for (int t0 = 0; t0 < T; t0 += 16) {
        const int64_t off = min<int64_t>((int64_t)t0 + 16, tlim);
        const uint4 nxt = tp[off >> 4];
        const uint32_t cw[4] = {cur.x, cur.y, cur.z, cur.w};
        if (t0 >= G - 1 && t0 + 16 <= nmin) {   // uniform
#pragma unroll
            for (int u = 0; u < 16; ++u)
                step((cw[u >> 2] >> (8 * (u & 3))) & 0xFFu, t0 + u, std::false_type{});
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u)
                step((cw[u >> 2] >> (8 * (u & 3))) & 0xFFu, t0 + u, std::true_type{});
        }
        cur = nxt;
    }
    // the last column's vertical deltas over the pattern's rows
    int c = 0;
#pragma unroll
    for (int s = 0; s < WL; ++s) {
        const int k = r * WL + s;
        const int rows = k < words ? min(m - 64 * k, 64) : 0;
        const uint32_t mlo = rows >= 32 ? ~0u : (1u << rows) - 1u;
        const uint32_t mhi = rows >= 64 ? ~0u : rows > 32 ? (1u << (rows - 32)) - 1u : 0u;
        c += __popc(pl[s] & mlo) + __popc(ph[s] & mhi) - __popc(ml[s] & mlo) -
             __popc(mh[s] & mhi);
    }
    return n + xl_group_sum<G>(c);
}

// Distances of pairs (ia[p], ib[p]) of two sets already staged with one
// common stride, one pair per group of lanes (the across-lanes layout), in
// one launch of just enough wavefronts for the pairs, each taking its pairs
// as its first work item (`counter` may hold any value).  MSA_ERANGE when
// patterns of max_len rows do not fit the layout (lev.hip).
int lev_xl_staged(const Staged &A, const Staged &B, int32_t sigma, int32_t max_len,
                  const int32_t *ia, const int32_t *ib, int64_t n_pairs, uint16_t *dist,
                  uint32_t *counter, int32_t *d_status, hipStream_t s);

}  // namespace msadp
