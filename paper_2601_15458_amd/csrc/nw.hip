// Needleman-Wunsch fill and traceback with unit costs (the pairwise aligner
// of the merge, Sec. 2.2 step 2), bit-parallel.
//
// With match 0 / mismatch 1 / gap 1 the NW score matrix is the Levenshtein
// matrix, so the fill runs the same bit-vector recurrence as lev.hip, here
// one 32-row word per lane.  Per cell it also emits the backward-walk choice
// (diagonal > up > left) as two bits derived from the bit vectors:
//   M (diagonal) iff a_i == b_j or D[i][j] == D[i-1][j-1] + 1, i.e.
//       M = Eq | ~D0 with D0 = Xh | Mv (diagonal delta zero);
//   U (up)       iff not M and D[i][j] == D[i-1][j] + 1, i.e. the new Pv;
//   else left.
//
// Fill layout.  A pair gets one workgroup; global lane g = 64*w + l holds
// pattern word g (rows 32g+1 .. 32g+32).  Lanes run skewed: lane g handles
// text column j one step after lane g-1 did, so the horizontal delta leaving
// word g-1 and the text symbol of column j reach lane g by a one-lane
// wavefront shift (DPP).  Between wavefronts the same packet goes through an
// LDS ring; wavefront w runs R + 64 steps behind w-1 and all wavefronts meet
// at a barrier every R steps, which orders every ring write before its read.
// R (16, 32 or 64) comes from the tuning table (tune.hip), default 32.
// The equality mask of a word is rebuilt per column from the word's symbol
// bit planes (no lookup table).  Codes are stored by anti-diagonal: the entry
// of (column j, word g) is record (j + g) * W + g, so at every step one
// wavefront writes 64 consecutive 8-byte records (M plane, U plane).
#include "common.hpp"

namespace msadp {

// Schedule of a fill with R steps between workgroup barriers.
template <int R>
struct Round {
    static constexpr int kRound = R;            // steps between workgroup barriers
    static constexpr int kLag = 64 + R;         // step lag between consecutive wavefronts
    static constexpr int kRing = 4 * R;         // ring entries per wavefront boundary
    static_assert(kLag >= 63 + kRound, "ring handoff needs a barrier in between");
    static_assert(kRing >= kLag - 63 + kRound, "ring too small");
    static_assert((kRing & (kRing - 1)) == 0, "ring size is a power of two");
};
constexpr int kMaxFillWaves = 16;
constexpr int kDefaultRound = 32;

__host__ __device__ inline int64_t tb_words(int32_t m) { return ((int64_t)m + 31) / 32; }

__host__ __device__ inline int64_t tb_bytes(int32_t m, int32_t n) {
    if (m <= 0 || n <= 0) return 0;
    const int64_t W = tb_words(m);
    return (n + W - 1) * W * 8;
}

struct NwLut {
    static constexpr uint8_t NOTA_OR_B = MSADP_LUT(~A | B);          // Eq' = ~neq | hn
    static constexpr uint8_t NOTA_OR_B2 = MSADP_LUT(~A | B);         // Xv = ~neq | Mv
    static constexpr uint8_t XOR_OR = MSADP_LUT((A ^ B) | C);        // Xh
    static constexpr uint8_t PH = MSADP_LUT(C | ~(A | B));           // Ph = Mv | ~(Xh | Pv)
    static constexpr uint8_t PV = MSADP_LUT(A | ~(B | C));           // Pv = Mh | ~(Xv | Ph)
    static constexpr uint8_t MCODE = MSADP_LUT(~(A & (B | C)));      // M = ~neq | ~(Xh | Mv)
    static constexpr uint8_t ACC_XOR = MSADP_LUT(A | (B ^ C));       // neq |= plane ^ mask
};

struct FillArgs {
    Staged A, B;
    const int32_t *ia, *ib;
    int32_t *score;
    uint8_t *tb;
    const int64_t *tb_off;
    int32_t *st;
    int32_t planes;   // bits per symbol code
    const int32_t *order;   // launch order (longest pair first), or null
};

// DPP control: shift the whole wavefront right by one lane.
constexpr int kDppWaveShr1 = 0x138;

typedef __attribute__((address_space(1))) uint64_t global_u64;

// State of one lane of the fill between steps.
struct FillLane {
    uint32_t Pv, Mv;       // vertical delta vectors of the lane's word
    uint32_t xout;         // packet sent to the next lane: symbol << 8 | hn << 1 | hp
    uint32_t accp, accn;   // +1 / -1 horizontal deltas leaving the last row
    uint64_t raddr;        // byte address of the lane's record at the current step
};

// One round of kRound steps of a wavefront.  kSteady: every lane's column
// j = t - shift lies in [0, n) for the whole round, so no step needs a
// range check.  kLast: the wavefront holding the pattern's last word (it
// counts the score's deltas and feeds no ring; the others feed the ring and
// count nothing).
template <int P, int R, bool kSteady, bool kLast>
__device__ __forceinline__ void fill_round(FillLane &L, const uint32_t (&plane)[P],
                                           uint32_t bpos, uint32_t feed, int t0, int shift,
                                           int n, bool word_ok, uint64_t rec_step,
                                           uint32_t *ring_out, int lane) {
    constexpr int kRing = Round<R>::kRing;
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const uint32_t sin = __builtin_amdgcn_readlane(feed, s);
        const uint32_t xin = __builtin_amdgcn_update_dpp(sin, L.xout, kDppWaveShr1, 0xF, 0xF,
                                                          false);
        const uint32_t tc = (xin >> 8) & 0xFFu;
        const uint32_t hp = xin & 1u, hn = (xin >> 1) & 1u;
        // neq: bit i set iff pattern row i differs from tc
        uint32_t neq = plane[0] ^ (uint32_t)(-(int32_t)(tc & 1u));
#pragma unroll
        for (int b = 1; b < P; ++b)
            neq = bop3<NwLut::ACC_XOR>(neq, plane[b], (uint32_t)(-(int32_t)((tc >> b) & 1u)));
        const uint32_t Pv = L.Pv, Mv = L.Mv;
        const uint32_t eqm = bop3<NwLut::NOTA_OR_B>(neq, hn, 0u);
        const uint32_t xv = bop3<NwLut::NOTA_OR_B2>(neq, Mv, 0u);
        const uint32_t sum = (eqm & Pv) + Pv;
        const uint32_t xh = bop3<NwLut::XOR_OR>(sum, Pv, eqm);
        const uint32_t ph = bop3<NwLut::PH>(xh, Pv, Mv);
        const uint32_t mh = Pv & xh;
        const uint32_t mcode = bop3<NwLut::MCODE>(neq, xh, Mv);
        const uint32_t hpo = __builtin_amdgcn_ubfe(ph, bpos, 1);
        const uint32_t hno = __builtin_amdgcn_ubfe(mh, bpos, 1);
        L.xout = (xin & 0xFF00u) | hpo | (hno << 1);
        const uint32_t Ph = (ph << 1) | hp, Mh = (mh << 1) | hn;
        const uint32_t pv_new = bop3<NwLut::PV>(Mh, xv, Ph);
        const uint32_t mv_new = Ph & xv;
        const int j = t0 + s - shift;
        const bool in = kSteady || (j >= 0 && j < n);
        // a lane keeps its initial column state until its first column
        L.Pv = kSteady || j >= 0 ? pv_new : Pv;
        L.Mv = kSteady || j >= 0 ? mv_new : Mv;
        // record (M plane, U plane) as one 8-byte store
        if ((!kLast || word_ok) && in)
            *(global_u64 *)L.raddr = ((uint64_t)L.Pv << 32) | mcode;
        if (kLast) {
            if (in) {
                L.accp += hpo;
                L.accn += hno;
            }
        } else if (lane == 63 && in) {
            ring_out[j & (kRing - 1)] = L.xout;
        }
        L.raddr += rec_step;
    }
}

template <int P, int R>
__device__ void nw_fill_pair(const FillArgs &a, int64_t p, uint32_t *ring) {
    constexpr int kRound = Round<R>::kRound, kLag = Round<R>::kLag, kRing = Round<R>::kRing;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int32_t x = a.ia[p], y = a.ib[p];
    if (x < 0 || x >= a.A.n || y < 0 || y >= a.B.n) {
        if (threadIdx.x == 0) set_status(a.st, MSA_DS_INDEX);
        return;
    }
    const int m = a.A.len[x], n = a.B.len[y];
    if (m == 0 || n == 0) {
        if (threadIdx.x == 0 && a.score) a.score[p] = m + n;
        return;
    }
    const int64_t W = tb_words(m);
    const int nw = (int)((W + 63) >> 6);
    if (a.tb_off[p + 1] - a.tb_off[p] < tb_bytes(m, n)) {
        if (threadIdx.x == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    if (w >= nw) return;   // wavefronts past the last word leave at once
    const int g = 64 * w + lane;
    const bool word_ok = g < W;

    // symbol bit planes of this lane's 32 pattern rows
    uint32_t plane[P];
#pragma unroll
    for (int b = 0; b < P; ++b) plane[b] = 0;
    if (word_ok) {
        const uint8_t *pat = a.A.codes + (int64_t)x * a.A.stride + 32 * g;
        const uint4 q0 = ((const uint4 *)pat)[0], q1 = ((const uint4 *)pat)[1];
        const uint32_t qs[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        const int rows = min(32, m - 32 * g);
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const uint32_t c = (qs[i >> 2] >> (8 * (i & 3))) & 0xFFu;
            if (i < rows) {
#pragma unroll
                for (int b = 0; b < P; ++b) plane[b] |= ((c >> b) & 1u) << i;
            }
        }
    }
    const uint32_t bpos = (g == W - 1) ? (uint32_t)((m - 1) & 31) : 31u;
    const uint8_t *text = a.B.codes + (int64_t)y * a.B.stride;
    uint8_t *tbp = a.tb + a.tb_off[p];
    uint32_t *ring_in = ring + (w - 1) * kRing;   // written by wavefront w-1
    uint32_t *ring_out = ring + w * kRing;

    const int total = n + 63 + kLag * (nw - 1);
    const int rounds = (total + kRound - 1) / kRound;
    const int shift = kLag * w + lane;       // column j = t - shift
    // record index at step t: (j + g) * W + g with j + g = t - (kLag - 64) * w;
    // the address advances by W records a step (unsigned wrap-around keeps
    // the start, which may lie before the region, exact)
    const int64_t rec0 = -(int64_t)(kLag - 64) * w * W + g;
    FillLane L{~0u, 0u, 0u, 0u, 0u,
               (uint64_t)(uintptr_t)tbp + (uint64_t)(rec0 * (int64_t)sizeof(uint2))};
    const uint64_t rec_step = (uint64_t)W * sizeof(uint2);
    const bool last = w == nw - 1;
    for (int rnd = 0; rnd < rounds; ++rnd) {
        const int t0 = rnd * kRound;
        // feed[l] = packet entering lane 0 at step t0 + l (l < kRound)
        // The barrier comes first: ring entries read here were written in an
        // earlier round (at least kLag - 63 - kRound steps before).
        __syncthreads();
        uint32_t feed = 0;
        {
            const int jj = t0 + lane - kLag * w;   // column reaching lane 0 at step t0 + lane
            if (lane < kRound && jj >= 0 && jj < n) {
                if (w == 0) feed = ((uint32_t)text[jj] << 8) | 1u;
                else feed = ring_in[jj & (kRing - 1)];
            }
        }
        // columns of the round: lane 63 at its first step to lane 0 at its last
        const bool steady = t0 - kLag * w - 63 >= 0 && t0 + kRound - 1 - kLag * w < n;
        if (steady) {
            if (last)
                fill_round<P, R, true, true>(L, plane, bpos, feed, t0, shift, n, word_ok,
                                             rec_step, ring_out, lane);
            else
                fill_round<P, R, true, false>(L, plane, bpos, feed, t0, shift, n, word_ok,
                                              rec_step, ring_out, lane);
        } else {
            if (last)
                fill_round<P, R, false, true>(L, plane, bpos, feed, t0, shift, n, word_ok,
                                              rec_step, ring_out, lane);
            else
                fill_round<P, R, false, false>(L, plane, bpos, feed, t0, shift, n, word_ok,
                                               rec_step, ring_out, lane);
        }
    }
    if (g == W - 1 && a.score) a.score[p] = m + (int)L.accp - (int)L.accn;
}

template <int P, int R>
__global__ void __launch_bounds__(1024) k_nw_fill(FillArgs a) {
    __shared__ uint32_t ring[kMaxFillWaves * Round<R>::kRing];
    nw_fill_pair<P, R>(a, a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x, ring);
}

// ------------------------------------------------------------ traceback
struct TbArgs {
    msa_seqs A, B;
    const int32_t *ia, *ib;
    const uint8_t *tb;
    const int64_t *tb_off;
    uint8_t *ops;
    const int64_t *ops_off;
    int32_t *ops_len;
    int32_t *st;
};

// One wavefront per pair.  The walk is uniform across the wavefront; the
// wavefront caches a tile of records: lane l holds records (s_hi - l,
// g_hi - q) for q < 4.  Ops are emitted backwards, 64 per store, at the end
// of the pair's region, then moved to its start.
__global__ void __launch_bounds__(64) k_nw_traceback(TbArgs a) {
    const int64_t p = blockIdx.x;
    const int lane = lane_id();
    const int32_t x = a.ia[p], y = a.ib[p];
    if (x < 0 || x >= a.A.n || y < 0 || y >= a.B.n) {
        if (lane == 0) set_status(a.st, MSA_DS_INDEX);
        return;
    }
    const int64_t m = a.A.offsets[x + 1] - a.A.offsets[x];
    const int64_t n = a.B.offsets[y + 1] - a.B.offsets[y];
    if (m < 0 || n < 0 || m > a.A.max_len || n > a.B.max_len) {
        if (lane == 0) set_status(a.st, MSA_DS_LENGTH);
        return;
    }
    const int64_t cap = a.ops_off[p + 1] - a.ops_off[p];
    if (cap < m + n || a.tb_off[p + 1] - a.tb_off[p] < tb_bytes((int32_t)m, (int32_t)n)) {
        if (lane == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    uint8_t *out = a.ops + a.ops_off[p];
    const uint2 *rec = (const uint2 *)(a.tb + a.tb_off[p]);
    // lengths are below 2^16, so every coordinate fits 32 bits
    const int32_t W = (int32_t)tb_words((int32_t)m);
    const int32_t nn = (int32_t)n;
    int32_t i = (int32_t)m, j = (int32_t)n;
    int64_t emitted = 0;
    uint32_t obuf = 0;
    // The tile: records of anti-diagonals s_hi - l (lane l) for words g_hi - k,
    // reloaded when the walk leaves it.  (Loading the next tile ahead of
    // time, halfway through the current one, measured slower.)
    int32_t s_hi = -1000000, g_hi = -1000000;
    uint2 tile[4];
    // one op: recorded in lane (emitted mod 64), stored 64 at a time
    auto emit = [&](uint32_t op) {
        obuf = lane == (int)(emitted & 63) ? op : obuf;
        ++emitted;
        if ((emitted & 63) == 0) out[cap - emitted + (63 - lane)] = (uint8_t)obuf;
    };
    // Inside the matrix: the step's record comes from the tile, and the
    // choice is made with selects rather than branches.
    while (i > 0 && j > 0) {
        const int32_t g = (i - 1) >> 5;
        const int32_t sp = (j - 1) + g;
        if (s_hi - sp < 0 || s_hi - sp >= 64 || g_hi - g < 0 || g_hi - g >= 4) {
            s_hi = sp;
            g_hi = g;
            const int64_t sl = s_hi - lane;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t gk = g_hi - k;
                // record (sl, gk) exists iff its column j' = sl - gk is in [0, n)
                const int64_t jc = sl - gk;
                tile[k] = (gk >= 0 && jc >= 0 && jc < nn) ? rec[sl * W + gk] : make_uint2(0, 0);
            }
            // wait for the tile here, so that the common path carries no
            // wait (on this GPU a vector-memory wait would also wait for the
            // pending op stores)
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        }
        const int L = s_hi - sp, q = g_hi - g;
        const uint32_t m0 = __builtin_amdgcn_readlane(tile[0].x, L);
        const uint32_t m1 = __builtin_amdgcn_readlane(tile[1].x, L);
        const uint32_t m2 = __builtin_amdgcn_readlane(tile[2].x, L);
        const uint32_t m3 = __builtin_amdgcn_readlane(tile[3].x, L);
        const uint32_t u0 = __builtin_amdgcn_readlane(tile[0].y, L);
        const uint32_t u1 = __builtin_amdgcn_readlane(tile[1].y, L);
        const uint32_t u2 = __builtin_amdgcn_readlane(tile[2].y, L);
        const uint32_t u3 = __builtin_amdgcn_readlane(tile[3].y, L);
        const uint32_t mw = q == 0 ? m0 : q == 1 ? m1 : q == 2 ? m2 : m3;
        const uint32_t uw = q == 0 ? u0 : q == 1 ? u1 : q == 2 ? u2 : u3;
        const uint32_t bit = (uint32_t)((i - 1) & 31);
        const uint32_t diag = (mw >> bit) & 1u, up = (uw >> bit) & 1u;
        const uint32_t op = diag ? 0u : (up ? 1u : 2u);
        i -= (op != 2u) ? 1 : 0;
        j -= (op != 1u) ? 1 : 0;
        emit(op);
    }
    // on the first row or column only gaps remain
    for (; i > 0; --i) emit(1u);
    for (; j > 0; --j) emit(2u);
    const int rem = (int)(emitted & 63);
    if (rem && lane < rem) out[cap - emitted + (rem - 1 - lane)] = (uint8_t)obuf;
    // the alignment now sits in out[cap - emitted .. cap); move it to the front
    // Chunks move from low to high addresses and the destination lies below
    // the source, so no chunk overwrites bytes that are still to be read.
    const int64_t src0 = cap - emitted;
    if (src0 > 0) {
        __threadfence();
        for (int64_t c = 0; c < emitted; c += 64) {
            const int64_t k = c + lane;
            uint8_t v = 0;
            if (k < emitted) v = out[src0 + k];
            if (k < emitted) out[k] = v;
        }
    }
    if (lane == 0) a.ops_len[p] = (int32_t)emitted;
}

static int bits_for(int sigma) {
    int b = 1;
    while ((1 << b) < sigma) ++b;
    return b;
}

struct NwPlan {
    int64_t strideA, strideB;
};

template <class Alloc>
static void nw_layout(Alloc &al, const msa_seqs *A, const msa_seqs *B, const NwPlan &pl,
                      int64_t n_pairs) {
    al.template take<uint8_t>((size_t)A->n * pl.strideA);
    al.template take<int32_t>((size_t)A->n + 1);
    al.template take<uint8_t>((size_t)B->n * pl.strideB);
    al.template take<int32_t>((size_t)B->n + 1);
    // launch order; sized min(n_pairs, kLptMaxPairs) so that a workspace
    // sized for a batch also holds any smaller one
    al.template take<int32_t>((size_t)std::min<int64_t>(n_pairs, kLptMaxPairs));
}

static NwPlan plan_nw(const msa_seqs *A, const msa_seqs *B) {
    NwPlan p;
    // staged pattern rows are read 32 symbols past each word start
    p.strideA = staged_stride(A->max_len) + 32;
    p.strideB = staged_stride(B->max_len);
    return p;
}

template <int R>
static void launch_fill(int planes, dim3 grid, dim3 block, const FillArgs &fa, hipStream_t s) {
    switch (planes) {
        case 1: hipLaunchKernelGGL((k_nw_fill<1, R>), grid, block, 0, s, fa); break;
        case 2: hipLaunchKernelGGL((k_nw_fill<2, R>), grid, block, 0, s, fa); break;
        case 3: hipLaunchKernelGGL((k_nw_fill<3, R>), grid, block, 0, s, fa); break;
        case 4: hipLaunchKernelGGL((k_nw_fill<4, R>), grid, block, 0, s, fa); break;
        default: hipLaunchKernelGGL((k_nw_fill<5, R>), grid, block, 0, s, fa); break;
    }
}

// forced > 0 selects R (autotuning), else the tuning table or the default.
static int nw_batch_impl(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                         const int32_t *ib, int64_t n_pairs, int32_t *score, uint8_t *tb,
                         const int64_t *tb_offsets, void *ws, size_t ws_bytes, int32_t *d_status,
                         hipStream_t s, int forced) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0) return MSA_EINVAL;
    if (A->sigma != B->sigma) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || tb_offsets == nullptr || ws == nullptr) return MSA_EINVAL;
    if (tb == nullptr && (A->max_len > 0 && B->max_len > 0)) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL) return MSA_ERANGE;
    const int64_t W = tb_words(A->max_len);
    if ((W + 63) / 64 > kMaxFillWaves) return MSA_ERANGE;   // patterns up to 32768 rows
    const NwPlan pl = plan_nw(A, B);
    Sizer sz;
    nw_layout(sz, A, B, pl, n_pairs);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    Staged SA{cv.take<uint8_t>((size_t)A->n * pl.strideA), cv.take<int32_t>((size_t)A->n + 1),
              pl.strideA, A->n};
    Staged SB{cv.take<uint8_t>((size_t)B->n * pl.strideB), cv.take<int32_t>((size_t)B->n + 1),
              pl.strideB, B->n};
    int32_t *order = cv.take<int32_t>((size_t)std::min<int64_t>(n_pairs, kLptMaxPairs));
    if (n_pairs > kLptMaxPairs) order = nullptr;
    if ((rc = stage_set(A, nullptr, SA, d_status, s))) return rc;
    if ((rc = stage_set(B, nullptr, SB, d_status, s))) return rc;
    const int waves = (int)std::max<int64_t>(1, (W + 63) / 64);
    if (order)
        hipLaunchKernelGGL(k_lpt_order<kLptTile>, dim3((unsigned)((n_pairs + 255) / 256)),
                           dim3(256), 0, s, SA, SB, ia, ib, n_pairs, order);
    FillArgs fa{SA, SB, ia, ib, score, tb, tb_offsets, d_status, bits_for(A->sigma), order};
    dim3 grid((unsigned)n_pairs), block(64 * waves);
    const int R = forced > 0 ? forced : tuned_value(MSA_TUNE_NW, A->sigma, waves, kDefaultRound);
    switch (R) {
        case 16: launch_fill<16>(fa.planes, grid, block, fa, s); break;
        case 32: launch_fill<32>(fa.planes, grid, block, fa, s); break;
        case 64: launch_fill<64>(fa.planes, grid, block, fa, s); break;
        default: return MSA_EINVAL;
    }
    return launch_status();
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t nw_tb_bytes(int32_t m, int32_t n) { return (size_t)tb_bytes(m, n); }

size_t nw_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    Sizer sz;
    nw_layout(sz, A, B, plan_nw(A, B), n_pairs);
    return sz.total();
}

int nw_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
             int64_t n_pairs, int32_t *score, uint8_t *tb, const int64_t *tb_offsets, void *ws,
             size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    return nw_batch_impl(A, B, ia, ib, n_pairs, score, tb, tb_offsets, ws, ws_bytes, d_status,
                         s, 0);
}

int msa_autotune_nw(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                    int64_t n_pairs, int32_t *score, uint8_t *tb, const int64_t *tb_offsets,
                    void *ws, size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                    int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (best == nullptr || best_ms == nullptr || reps < 1 || n_pairs < 1) return MSA_EINVAL;
    const int waves = (int)std::max<int64_t>(1, (tb_words(A->max_len) + 63) / 64);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MSA_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MSA_EDEVICE;
    }
    int br = 0;
    float bms = 0.0f;
    rc = MSA_OK;
    for (int R : {16, 32, 64}) {
        if ((rc = nw_batch_impl(A, B, ia, ib, n_pairs, score, tb, tb_offsets, ws, ws_bytes,
                                d_status, s, R)))
            break;   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        for (int r = 0; r < reps && rc == MSA_OK; ++r)
            rc = nw_batch_impl(A, B, ia, ib, n_pairs, score, tb, tb_offsets, ws, ws_bytes,
                               d_status, s, R);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        ms /= (float)reps;
        if (br == 0 || ms < bms) {
            br = R;
            bms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = br;
    *best_ms = bms;
    return msa_tune_set(MSA_TUNE_NW, A->sigma, waves, br);
}

int nw_traceback(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                 int64_t n_pairs, const uint8_t *tb, const int64_t *tb_offsets, uint8_t *ops,
                 const int64_t *ops_offsets, int32_t *ops_len, int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || tb_offsets == nullptr || ops == nullptr ||
        ops_offsets == nullptr || ops_len == nullptr)
        return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL) return MSA_ERANGE;
    TbArgs ta{*A, *B, ia, ib, tb, tb_offsets, ops, ops_offsets, ops_len, d_status};
    hipLaunchKernelGGL(k_nw_traceback, dim3((unsigned)n_pairs), dim3(64), 0, s, ta);
    return launch_status();
}

}  // extern "C"
