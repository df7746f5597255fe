// Exact banded Levenshtein distance (Ukkonen's band, verified): the distance
// batches of Alg. 1 for long, similar pairs, where the full DP matrix is
// mostly cells no optimal path visits.
//
// Band.  An alignment of cost C of a (m rows) against b (n columns) only
// visits diagonals d = j - i with |d| + |d - (n - m)| <= C.  With a threshold
// K >= |n - m| the band dlo <= d <= dhi, dlo = min(0, n-m) - e, dhi =
// max(0, n-m) + e, e = floor((K - |n - m|) / 2), therefore holds every
// alignment of cost <= K.  Cells outside the band are never computed; the
// boundary of the computed region takes values that are costs of real
// alignments (a row entering the region at the left starts with vertical
// deltas +1, a row above it that has left the region continues with
// horizontal deltas +1), so every computed value is the cost of some
// alignment and is at least the true distance, and a value <= K is exact: the
// optimal path then lies in the band and the band recurrence reproduces it.
// A pair whose banded value exceeds K is recomputed with 2K, up to kmax.
//
// Layout.  One wavefront per pair.  The pattern is cut into 64-row words;
// word g is live on the columns where one of its rows is in the band,
// [64 g + dlo, 64 g + 63 + dhi], and runs column j at step j + g (one step
// behind word g - 1, whose horizontal delta on its bottom row it needs).
// Lane p takes words p, p + 64, p + 128, ... in turn: their live steps do not
// overlap while the band is narrower than 4096 diagonals, so one wavefront
// covers any pattern length.  Each step every lane passes (horizontal delta,
// bottom-row value) to the next lane by a one-lane DPP wavefront rotation
// (lane 63 feeds lane 0 of the next cycle of words).  The text and the
// pattern's match table Peq[word][symbol] sit in LDS.  The value of the last
// row at the last column is the distance.
#include "common.hpp"
#include "lev_core.hpp"

namespace msadp {

constexpr int kBandMaxK = 4000;        // band widths up to K + 1 < 4096 diagonals
constexpr int kDppWaveRor1 = 0x13C;    // DPP: rotate the wavefront right by one lane
constexpr uint32_t kBandNone = 0xFFFFu;

struct BandArgs {
    Staged A, B;
    const int32_t *ia, *ib;
    uint16_t *out;
    int32_t *k_used;         // per pair: the K that verified it (may be null)
    int32_t k0, kmax, sigma;
    int32_t *st;
};

// Words [0, W) of the pattern: tbl[g * sigma + c] has bit i set iff
// pat[64 g + i] == c (rows past m never match).
__device__ __forceinline__ void band_peq(uint64_t *tbl, const uint8_t *pat, int m, int W,
                                         int sigma) {
    const int lane = lane_id();
    for (int g = 0; g < W; ++g) {
        const int i = 64 * g + lane;
        const int c = i < m ? (int)pat[i] : 255;
        uint64_t mine = 0;
        for (int s = 0; s < sigma; ++s) {
            const uint64_t bal = __ballot(c == s);
            if (lane == s) mine = bal;
        }
        if (lane < sigma) tbl[g * sigma + lane] = mine;
    }
}

// One banded pass with threshold K; returns the distance bound at (m, n)
// (valid in every lane).
//
// The value is assembled without carrying absolute values between lanes:
// with jlo(g) the first column of word g, the row above word g + 1 before
// column jlo(g + 1) holds (the row above word g before jlo(g)) + 64 + the
// bottom-row deltas of word g over columns jlo(g) .. jlo(g + 1) - 1, and the
// last word adds its rows and its last-row deltas up to column n - 1.  So
// each lane sums, over its words, the deltas of the columns before the next
// word starts; the distance is m plus the sum over all lanes (the top row
// holds jlo(0) = 0).
//
// The match word of a column is read from LDS one step ahead and its text
// symbol two steps ahead, into two alternating registers (two steps per loop
// trip), so that no LDS read sits on the step's dependent chain
// (DPP packet -> word update -> packet).
__device__ int band_pass(const uint64_t *tbl, const uint8_t *text, int m, int n, int W,
                         int sigma, int K) {
    const int lane = lane_id();
    const int dd = n - m;
    // at least one diagonal either side, so that consecutive words' bands
    // overlap (a wider band than K needs is always safe)
    const int e = max(1, (K - (dd < 0 ? -dd : dd)) >> 1);
    const int dlo = min(0, dd) - e, dhi = max(0, dd) + e;
    const int last_bit = (m - 1) & 63;
    auto lo_of = [&](int gg) { return max(0, 64 * gg + dlo); };
    auto hi_of = [&](int gg) { return min(n - 1, 64 * gg + 63 + dhi); };
    auto txt = [&](int jj) { return (int)text[min(max(jj, 0), n - 1)]; };
    int g = lane;                                   // this lane's current word
    int jlo = 0, jhi = -1, jhi_above = -1, jnext = 0, b = 63;
    auto take_word = [&]() {
        jlo = lo_of(g);
        jhi = g < W ? hi_of(g) : -1;
        jhi_above = g > 0 ? hi_of(g - 1) : -1;
        jnext = g < W - 1 ? lo_of(g + 1) : n;       // the columns this word sums
        b = g == W - 1 ? last_bit : 63;
    };
    take_word();
    uint32_t pl = ~0u, ph = ~0u, ml = 0u, mh = 0u;  // Pv, Mv of the current word
    int acc = 0;                                    // summed bottom-row deltas
    uint32_t pk = 0;                                // packet: h as (+1 bit, -1 bit)
    int sym_next = txt(1 - g);
    uint64_t eqA = tbl[min(g, W - 1) * sigma + txt(-g)], eqB = 0;
    const int steps = (n - 1) + (W - 1) + 1;
    // one step: uses eq_cur (column s - g), loads the next column's word
    // into eq_load and the symbol two columns ahead
    auto step = [&](int s, const uint64_t eq_cur, uint64_t &eq_load) {
        const uint32_t pin = __builtin_amdgcn_update_dpp(0u, pk, kDppWaveRor1, 0xF, 0xF, false);
        int j = s - g;
        if (j > jhi && g < W) {
            // this word's band is done: take the lane's next word, live at
            // least 97 steps later (the prefetch refills meanwhile)
            g += 64;
            take_word();
            pl = ph = ~0u;
            ml = mh = 0u;
            j = s - g;
        }
        eq_load = tbl[min(g, W - 1) * sigma + sym_next];
        sym_next = txt(j + 2);
        const bool live = g < W && j >= jlo && j <= jhi;
        // horizontal delta entering from the row above the word: from word
        // g - 1 while column j lies in its band, else +1 (the top row, or a
        // row that has left the band)
        const bool from_above = j <= jhi_above;
        const uint32_t hp_in = from_above ? (pin & 1u) : 1u;
        const uint32_t hn_in = from_above ? ((pin >> 1) & 1u) : 0u;
        const uint32_t el = (uint32_t)eq_cur, eh = (uint32_t)(eq_cur >> 32);
        const uint32_t cph = hp_in << 31, cmh = hn_in << 31;
        const uint32_t elm = el | hn_in;
        const uint32_t xvl = el | ml, xvh = eh | mh;
        unsigned int cy, cy2;
        const uint32_t sl = __builtin_addc(elm & pl, pl, 0u, &cy);
        const uint32_t sh = __builtin_addc(eh & ph, ph, cy, &cy2);
        const uint32_t xhl = bop3<Lut::XOR_OR>(sl, pl, elm);
        const uint32_t xhh = bop3<Lut::XOR_OR>(sh, ph, eh);
        const uint32_t phl = bop3<Lut::PH>(xhl, pl, ml);
        const uint32_t phh = bop3<Lut::PH>(xhh, ph, mh);
        const uint32_t mhl = pl & xhl, mhh = ph & xhh;
        const uint32_t Phl = shl1_carry(phl, cph), Phh = shl1_carry(phh, phl);
        const uint32_t Mhl = shl1_carry(mhl, cmh), Mhh = shl1_carry(mhh, mhl);
        const uint64_t P = ((uint64_t)phh << 32) | phl, Mw = ((uint64_t)mhh << 32) | mhl;
        const int dp = (int)((P >> b) & 1u), dn = (int)((Mw >> b) & 1u);
        acc += (live && j < jnext) ? dp - dn : 0;
        pl = live ? bop3<Lut::PV>(Mhl, xvl, Phl) : pl;
        ph = live ? bop3<Lut::PV>(Mhh, xvh, Phh) : ph;
        ml = live ? Phl & xvl : ml;
        mh = live ? Phh & xvh : mh;
        // bottom row's delta (bit 63; the last word feeds nobody)
        pk = (phh >> 31) | ((mhh >> 31) << 1);
    };
    int s = 0;
    for (; s + 1 < steps; s += 2) {
        step(s, eqA, eqB);
        step(s + 1, eqB, eqA);
    }
    if (s < steps) step(s, eqA, eqB);
    // m plus every lane's sum (a wavefront reduction)
    int v = acc;
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return m + v;
}

__global__ void __launch_bounds__(64) k_lev_band(BandArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int64_t p = blockIdx.x;
    const int lane = lane_id();
    const int32_t x = a.ia[p], y = a.ib[p];
    if (x < 0 || x >= a.A.n || y < 0 || y >= a.B.n) {
        if (lane == 0) {
            set_status(a.st, MSA_DS_INDEX);
            a.out[p] = (uint16_t)kBandNone;
        }
        return;
    }
    const int m = a.A.len[x], n = a.B.len[y];
    int d;
    int kv = 0;
    if (m == 0 || n == 0) {
        d = m + n;
    } else {
        const int W = (m + 63) >> 6;
        uint64_t *tbl = (uint64_t *)smem;
        uint8_t *text = smem + (size_t)W * a.sigma * 8;
        const uint8_t *tg = a.B.codes + (int64_t)y * a.B.stride;
        for (int k = lane; k < n; k += 64) text[k] = tg[k];
        band_peq(tbl, a.A.codes + (int64_t)x * a.A.stride, m, W, a.sigma);
        __syncthreads();
        const int dd = m > n ? m - n : n - m;
        int K = min(max(a.k0, dd + 2), a.kmax);
        d = (int)kBandNone;
        if (K >= dd) {   // else the distance (at least |m - n|) exceeds kmax
            for (;;) {
                const int v = band_pass(tbl, text, m, n, W, a.sigma, K);
                if (v <= K) {
                    d = v;
                    kv = K;
                    break;
                }
                if (K >= a.kmax) break;
                K = min(2 * K, a.kmax);
            }
        }
    }
    if (lane == 0) {
        a.out[p] = (uint16_t)(d <= a.kmax ? d : (int)kBandNone);
        if (a.k_used) a.k_used[p] = d <= a.kmax ? kv : -1;
    }
}

struct BandWs {
    Staged SA, SB;
};

template <class Alloc>
static BandWs carve_band(Alloc &al, const msa_seqs *A, const msa_seqs *B) {
    BandWs w;
    const int64_t sa = staged_stride(A->max_len), sb = staged_stride(B->max_len);
    w.SA = Staged{al.template take<uint8_t>((size_t)A->n * sa),
                  al.template take<int32_t>((size_t)A->n + 1), sa, A->n};
    w.SB = Staged{al.template take<uint8_t>((size_t)B->n * sb),
                  al.template take<int32_t>((size_t)B->n + 1), sb, B->n};
    return w;
}

static size_t band_lds_bytes(const msa_seqs *A, const msa_seqs *B) {
    const size_t W = ((size_t)A->max_len + 63) / 64;
    return W * (size_t)A->sigma * 8 + (((size_t)B->max_len + 15) / 16) * 16;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t lev_band_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    Sizer sz;
    carve_band(sz, A, B);
    return sz.total();
}

int lev_band(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
             int64_t n_pairs, int32_t k0, int32_t kmax, uint16_t *dist, int32_t *k_used,
             void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0 || A->sigma != B->sigma) return MSA_EINVAL;
    if (k0 < 1 || kmax < k0 || kmax > kBandMaxK) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || dist == nullptr || ws == nullptr) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL) return MSA_ERANGE;
    const size_t lds = band_lds_bytes(A, B);
    if (lds > 65536) return MSA_ERANGE;
    Sizer sz;
    carve_band(sz, A, B);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    const BandWs w = carve_band(cv, A, B);
    if ((rc = stage_set(A, nullptr, w.SA, d_status, s))) return rc;
    if ((rc = stage_set(B, nullptr, w.SB, d_status, s))) return rc;
    BandArgs ba{w.SA, w.SB, ia, ib, dist, k_used, k0, kmax, A->sigma, d_status};
    hipLaunchKernelGGL(k_lev_band, dim3((unsigned)n_pairs), dim3(64), (unsigned)lds, s, ba);
    return launch_status();
}

}  // extern "C"
