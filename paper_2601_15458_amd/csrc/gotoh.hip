// Needleman-Wunsch with a substitution score matrix and affine gaps, the cost
// model of the paper's experiments (Sec. 2.4: substitution matrices, gap
// opening charged ten times the extension).  A run of k gap symbols scores
// -(open + k * ext); the aligner maximizes the sum of substitution scores of
// aligned pairs minus the gap-run penalties.  Gotoh's recurrences:
//   E[i][j] = max(E[i][j-1] - ext, H[i][j-1] - open - ext)     (ends with I)
//   F[i][j] = max(F[i-1][j] - ext, H[i-1][j] - open - ext)     (ends with D)
//   H[i][j] = max(H[i-1][j-1] + sub[a_i][b_j], E[i][j], F[i][j])
// with H[i][0] = F[i][0] = -(open + i ext), H[0][j] = E[0][j] = -(open + j ext).
// The fill keeps X + (i + j) ext for X in {H, E, F}: then both extension
// branches compare without a subtraction (E[i][j] + (i+j) ext =
// max(E[i][j-1] + (i+j-1) ext, H[i][j-1] + (i+j-1) ext - open), likewise F),
// the diagonal gains 2 ext (folded into the score table), the borders are
// -open, and every difference the codes compare is unchanged.  The score is
// the shifted H[m][n] minus (m + n) ext.
//
// Fill layout.  One workgroup per pair; global lane g = 64 w + l owns the 16
// rows 16g+1 .. 16g+16 of a and keeps their H and E of the previous column
// in registers.  Lanes run skewed: lane g handles column j one step after
// lane g-1, which hands down (by a one-lane DPP wavefront shift) the H of its
// bottom row and a packet with b_j and the gap state of that row:
// min(H - F, open + 1), enough to rebuild every comparison F takes part in
// (when H - F > open the extension branch loses whatever F is).  Between
// wavefronts the same two words go through an LDS ring; wavefront w runs
// kLag steps behind w-1 and all wavefronts meet at a barrier every kRound
// steps, which orders each ring write before its read.
//
// Codes.  Per cell one byte, four signs u = sign(x) + 1 in {0, 1, 2} as the
// 2-bit fields of u0 + 4 u1 + 16 u2 + 64 u3 (at most 170):
//   u0: hd - max(E, F)      (hd = H[i-1][j-1] + sub: the diagonal)
//   u1: F - E
//   u2: (H[i][j-1] - open - ext) - (E[i][j-1] - ext)    (E opens / extends)
//   u3: (H[i-1][j] - open - ext) - (F[i-1][j] - ext)    (F opens / extends)
// which is everything the backward walk needs: the diagonal reaches H iff
// u0 >= 1; F reaches H iff u1 >= 1 and u0 <= 1; a gap run may open at the
// cell iff its digit is >= 1 and extend iff it is <= 1.  Codes are
// stored by anti-diagonal: record (j + g) * G + g (G = lanes of the pair)
// holds the 16 bytes of lane g at column j, so at every step a wavefront
// writes 64 consecutive 16-byte records.
//
// Walk (gotoh_traceback): among the best-scoring alignments, the one whose
// op string read backwards is smallest with M < D < I.  From (m, n), with
// `last` the op chosen at the step before (the op that follows in forward
// order): after M or at the start, take M if the diagonal reaches H, else D
// if F does, else I; after D (coming from (i+1, j)), take M if the
// diagonal reaches H[i][j] and F[i+1][j] opens from it, else D if F[i+1][j]
// extends F[i][j], else I; after I (coming from (i, j+1)), take M if the
// diagonal reaches H[i][j] and E[i][j+1] opens from it, else D if F reaches
// H[i][j] and E[i][j+1] opens from it, else I.  On the first row or column
// only I or D remain.
#include "common.hpp"

namespace msadp {

constexpr int kGRows = 16;                 // rows per lane
constexpr int kGRound = 32;                // steps between workgroup barriers
constexpr int kGLag = 64 + kGRound;        // step lag between consecutive wavefronts
constexpr int kGRing = 4 * kGRound;        // ring entries per wavefront boundary
constexpr int kGMaxWaves = 16;
constexpr int kGMaxRows = kGRows * kWave * kGMaxWaves;   // 16384
constexpr int kSubStride = 32;             // row stride of the score table (host copy)
constexpr int kLdsSubRow = 64;             // entries per b row of the table in LDS
constexpr int32_t kNegInf = -(1 << 30);
constexpr int32_t kMaxSub = 2048;          // |sub| and open + ext at most this
static_assert(kGLag >= 63 + kGRound, "ring handoff needs a barrier in between");
static_assert(kGRing >= kGLag - 63 + kGRound, "ring too small");

__host__ __device__ inline int64_t gotoh_lanes(int32_t m) { return ((int64_t)m + kGRows - 1) / kGRows; }

__host__ __device__ inline int64_t gotoh_tb_size(int32_t m, int32_t n) {
    if (m <= 0 || n <= 0) return 0;
    const int64_t G = gotoh_lanes(m);
    return (n + G - 1) * G * kGRows;
}

struct GotohArgs {
    Staged A, B;
    const int32_t *ia, *ib;
    const int32_t *sub;      // sigma x sigma scores, row stride kSubStride (device)
    int32_t open, ext;
    int32_t *score;
    uint8_t *tb;
    const int64_t *tb_off;
    int32_t *st;
    const int32_t *order;    // launch order (longest pair first), or null
};

constexpr int kGDppWaveShr1 = 0x138;   // DPP: shift the wavefront right by one lane

// Code records are written through a global-address-space pointer: a flat
// store would count against the LDS wait counter too, and every LDS read of
// the score table would then wait for the step's store to complete.
typedef unsigned int gu32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) gu32x4 g_uint4;

// sign(x - y) in {-1, 0, 1}: one subtraction and one v_med3_i32 (written
// out, so that the compiler does not turn it into two compares and selects)
__device__ __forceinline__ int32_t sign_of(int32_t x, int32_t y) {
    int32_t d = x - y, s;
    asm volatile("v_med3_i32 %0, %1, -1, 1" : "=v"(s) : "v"(d));
    return s;
}

// LDS byte address of row r's score at a step: byte 0 of the lane's packed
// row symbols (each already times 4) and byte 1 the column symbol, i.e.
// b * 256 + 4 a in one v_perm_b32 (selectors 0-3: bytes of `rows`, 4: byte 0
// of `pk`, 12: zero)
__device__ __forceinline__ uint32_t sub_addr(uint32_t pk, uint32_t rows, int r) {
    return __builtin_amdgcn_perm(pk, rows, 0x0C0C0400u | (uint32_t)(r & 3));
}

// a << sh + b in one instruction (v_lshl_add_u32), exact in wrapping
// 32-bit arithmetic for signed a and b
template <int SH>
__device__ __forceinline__ uint32_t lshl_add(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(SH), "v"(b));
    return r;
}

struct GotohLane {
    int32_t H[kGRows];      // H[i][j-1] of the lane's rows (plus (i + j - 1) ext)
    int32_t E[kGRows];      // E[i][j-1] (plus (i + j - 1) ext)
    int32_t htop;           // H of the row above the lane at the previous column
    int32_t outH;           // H of the lane's bottom row at the current column
    uint32_t outP;          // packet: symbol | min(H - F, open + 1) << 8
};

// One round of kGRound steps.  kSteady: every lane's column lies in [0, n)
// for the whole round (no range checks).
template <bool kSteady>
__device__ __forceinline__ void gotoh_round(GotohLane &L, const uint32_t (&roff)[kGRows / 4],
                                            const char *sub_lds, uint32_t feedH,
                                            uint32_t feedP, int t0, int shift, int n,
                                            int32_t open, bool rec_ok,
                                            g_uint4 *rec, int64_t rec_step, uint2 *ring_out,
                                            int lane) {
    // two steps per loop iteration: a row's new H and E then alternate
    // between two registers instead of being copied back at every step
#pragma unroll 2
    for (int s = 0; s < kGRound; ++s) {
        const uint32_t sinH = __builtin_amdgcn_readlane(feedH, s);
        const uint32_t sinP = __builtin_amdgcn_readlane(feedP, s);
        const int32_t htop = (int32_t)__builtin_amdgcn_update_dpp(sinH, (uint32_t)L.outH,
                                                                  kGDppWaveShr1, 0xF, 0xF, false);
        const uint32_t pk = __builtin_amdgcn_update_dpp(sinP, L.outP, kGDppWaveShr1, 0xF, 0xF,
                                                        false);
        const int jj = t0 + s - shift;
        const bool in = kSteady || (jj >= 0 && jj < n);
        const int32_t sym = (int32_t)(pk & 0xFFu);
        // the packed row symbols go through an empty asm each step, so that
        // nothing derived from them is hoisted out of the step loop into
        // registers that would spill
        uint32_t rs[kGRows / 4] = {roff[0], roff[1], roff[2], roff[3]};
        asm volatile("" : "+v"(rs[0]), "+v"(rs[1]), "+v"(rs[2]), "+v"(rs[3]));
        // the step's 16 scores are read before the row chain starts, so that
        // one LDS round trip is waited for per step instead of one per row
        // (the empty asm statements below keep later loads from moving)
        int32_t svs[kGRows];
#pragma unroll
        for (int r = 0; r < kGRows; ++r)
            svs[r] = *(const int32_t *)(sub_lds + sub_addr(pk, rs[r >> 2], r));
        int32_t up_h = htop;
        int32_t up_f = htop - (int32_t)(pk >> 8);
        int32_t diag = L.htop;
        // each byte gets its +85 (the +1 of every field) from the start value
        uint32_t code[kGRows / 4] = {0x55555555u, 0x55555555u, 0x55555555u, 0x55555555u};
        // outside [0, n) a lane keeps its state (its first column is still
        // to come, or its last is done)
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int32_t sv = svs[r];
            int32_t hprev = L.H[r], eprev = L.E[r];
            // tie the row's inputs to the row above's result, so that the
            // compiler does not compute every row's E ahead of the chain
            // (which would hold ~4 more registers per row)
            asm volatile("" : "+v"(hprev), "+v"(eprev) : "v"(up_h));
            const int32_t e_ext = eprev, e_opn = hprev - open;
            const int32_t e = max(e_ext, e_opn);
            const int32_t f_ext = up_f, f_opn = up_h - open;
            const int32_t f = max(f_ext, f_opn);
            const int32_t hd = diag + sv;
            const int32_t mef = max(e, f);
            const int32_t h = max(hd, mef);
            // four signs as 2-bit fields (sign + 1): c = s0 + 4 s1 + 16 s2 +
            // 64 s3 in [-85, 85], added into the code word at the row's byte;
            // the words start at 85 per byte, so every byte ends in [0, 170]
            // and the wrapping sum carries nothing between bytes.  Shifts and
            // adds only: v_mul_lo_u32 issues at a quarter of the rate.
            const uint32_t c =
                lshl_add<2>((uint32_t)sign_of(f, e), (uint32_t)sign_of(hd, mef));
            const uint32_t c2 = lshl_add<4>((uint32_t)sign_of(e_opn, e_ext), c);
            const uint32_t c3 = lshl_add<6>((uint32_t)sign_of(f_opn, f_ext), c2);
            switch (r & 3) {   // resolved at compile time (the row loop is unrolled)
                case 0: code[r >> 2] = lshl_add<0>(c3, code[r >> 2]); break;
                case 1: code[r >> 2] = lshl_add<8>(c3, code[r >> 2]); break;
                case 2: code[r >> 2] = lshl_add<16>(c3, code[r >> 2]); break;
                default: code[r >> 2] = lshl_add<24>(c3, code[r >> 2]); break;
            }
            // the code is formed here, not sunk into the (conditional) store,
            // which would keep every row's six compared values alive
            asm volatile("" : "+v"(code[r >> 2]));
            diag = hprev;   // H[i][j-1] is the diagonal of row i+1
            L.H[r] = in ? h : hprev;
            L.E[r] = in ? e : eprev;
            up_h = h;
            up_f = f;
        }
        // bottom row's H and the gap-state packet for the next lane
        const int32_t dF = min(up_h - up_f, open + 1);
        if (in) {
            L.htop = htop;
            L.outH = up_h;
            L.outP = (uint32_t)sym | ((uint32_t)dF << 8);
            if (rec_ok) *rec = gu32x4{code[0], code[1], code[2], code[3]};
            if (lane == 63) ring_out[jj & (kGRing - 1)] = make_uint2((uint32_t)L.outH, L.outP);
        }
        rec = (g_uint4 *)((uintptr_t)rec + (uintptr_t)rec_step);
    }
}

__global__ void __launch_bounds__(1024) k_gotoh_fill(GotohArgs a) {
    __shared__ int32_t sub_lds[kSubStride * kLdsSubRow];
    __shared__ uint2 ring[kGMaxWaves * kGRing];
    const int64_t p = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // transposed, with the diagonal's 2 ext of the shifted recurrences:
    // sub_lds[b * kLdsSubRow + a] = sub[a][b] + 2 ext, at byte b * 256 + 4 a
    // (entries a >= kSubStride of a row are never read)
    for (int e = threadIdx.x; e < kSubStride * kSubStride; e += blockDim.x)
        sub_lds[(e % kSubStride) * kLdsSubRow + e / kSubStride] = a.sub[e] + 2 * a.ext;
    __syncthreads();
    const int32_t x = a.ia[p], y = a.ib[p];
    if (x < 0 || x >= a.A.n || y < 0 || y >= a.B.n) {
        if (threadIdx.x == 0) set_status(a.st, MSA_DS_INDEX);
        return;
    }
    const int m = a.A.len[x], n = a.B.len[y];
    if (m == 0 || n == 0) {
        if (threadIdx.x == 0 && a.score)
            a.score[p] = (m + n) == 0 ? 0 : -(a.open + (m + n) * a.ext);
        return;
    }
    if (m > kGMaxRows) {
        if (threadIdx.x == 0) set_status(a.st, MSA_DS_LENGTH);
        return;
    }
    if (a.tb_off[p + 1] - a.tb_off[p] < gotoh_tb_size(m, n)) {
        if (threadIdx.x == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    const int64_t G = gotoh_lanes(m);
    const int nwv = (int)((G + 63) >> 6);
    if (w >= nwv) return;   // wavefronts past the last lane leave at once (before any barrier)
    const int g = 64 * w + lane;
    const bool lane_ok = g < G;
    const int32_t open = a.open, ext = a.ext;

    // the lane's 16 pattern symbols times 4, four per register (one byte
    // each; staged symbols are below 32, so the shift carries nothing between
    // bytes): row r's score at column j is at LDS byte b_j * 256 + byte r
    uint32_t roff[kGRows / 4];
    {
        uint4 q = make_uint4(0, 0, 0, 0);
        if (lane_ok) q = *(const uint4 *)(a.A.codes + (int64_t)x * a.A.stride + kGRows * g);
        roff[0] = q.x << 2;
        roff[1] = q.y << 2;
        roff[2] = q.z << 2;
        roff[3] = q.w << 2;
    }
    // column 0 in the shifted form: H = -open below row 0, H[0][0] = 0
    GotohLane L;
    const int32_t row0 = kGRows * g;   // the row above the lane
#pragma unroll
    for (int r = 0; r < kGRows; ++r) {
        L.H[r] = -open;
        L.E[r] = kNegInf;
    }
    L.htop = row0 == 0 ? 0 : -open;
    L.outH = 0;
    L.outP = 0;
    const int r_last = (m - 1) - kGRows * (int)((m - 1) / kGRows);
    const bool score_lane = g == (m - 1) / kGRows;

    const uint8_t *text = a.B.codes + (int64_t)y * a.B.stride;
    uint8_t *tbp = a.tb + a.tb_off[p];
    uint2 *ring_in = ring + (w - 1) * kGRing;
    uint2 *ring_out = ring + w * kGRing;
    const int total = n + 63 + kGLag * (nwv - 1);
    const int rounds = (total + kGRound - 1) / kGRound;
    const int shift = kGLag * w + lane;   // column jj = t - shift
    // record of step t: (jj + g) * G + g with jj + g = t - (kGLag - 64) w; it
    // advances by G records a step (unsigned wrap-around keeps the start,
    // which may lie before the region, exact)
    const int64_t rec0 = -(int64_t)(kGLag - 64) * w * G + g;
    g_uint4 *rec = (g_uint4 *)((uintptr_t)tbp + (uintptr_t)(rec0 * (int64_t)sizeof(uint4)));
    const int64_t rec_step = G * (int64_t)sizeof(uint4);
    for (int rnd = 0; rnd < rounds; ++rnd) {
        const int t0 = rnd * kGRound;
        // feed[l]: the words entering lane 0 at step t0 + l (l < kGRound);
        // ring entries read here were written at least kGLag - 63 - kGRound
        // steps earlier, before an earlier barrier
        __syncthreads();
        uint32_t feedH = 0, feedP = 0;
        {
            const int jj = t0 + lane - kGLag * w;
            if (lane < kGRound && jj >= 0 && jj < n) {
                if (w == 0) {
                    feedH = (uint32_t)(-open);   // row 0, shifted
                    feedP = (uint32_t)text[jj] | ((uint32_t)(open + 1) << 8);
                } else {
                    const uint2 v = ring_in[jj & (kGRing - 1)];
                    feedH = v.x;
                    feedP = v.y;
                }
            }
        }
        const bool steady = t0 - kGLag * w - 63 >= 0 && t0 + kGRound - 1 - kGLag * w < n;
        if (steady)
            gotoh_round<true>(L, roff, (const char *)sub_lds, feedH, feedP, t0, shift, n, open,
                              lane_ok, rec, rec_step, ring_out, lane);
        else
            gotoh_round<false>(L, roff, (const char *)sub_lds, feedH, feedP, t0, shift, n, open,
                               lane_ok, rec, rec_step, ring_out, lane);
        rec = (g_uint4 *)((uintptr_t)rec + (uintptr_t)(kGRound * rec_step));
    }
    // the lane state stopped at the last column: H[m][n] is row r_last's H,
    // less the (m + n) ext of the shifted form
    if (score_lane && a.score) {
        int32_t sc = 0;
#pragma unroll
        for (int r = 0; r < kGRows; ++r) sc = r == r_last ? L.H[r] : sc;
        a.score[p] = sc - (m + n) * ext;
    }
}

// ------------------------------------------------------------ traceback
struct GotohTbArgs {
    msa_seqs A, B;
    const int32_t *ia, *ib;
    const uint8_t *tb;
    const int64_t *tb_off;
    uint8_t *ops;
    const int64_t *ops_off;
    int32_t *ops_len;
    int32_t *st;
};

// One wavefront per pair, the walk uniform across it.  The wavefront caches
// a tile of records: lane l holds records (s_hi - l, g_hi - q), q < 2.  Ops
// are emitted backwards, 64 per store, at the end of the pair's region,
// then moved to its start.
__global__ void __launch_bounds__(64) k_gotoh_traceback(GotohTbArgs a) {
    const int64_t p = blockIdx.x;
    const int lane = lane_id();
    const int32_t x = a.ia[p], y = a.ib[p];
    if (x < 0 || x >= a.A.n || y < 0 || y >= a.B.n) {
        if (lane == 0) set_status(a.st, MSA_DS_INDEX);
        return;
    }
    const int64_t m = a.A.offsets[x + 1] - a.A.offsets[x];
    const int64_t n = a.B.offsets[y + 1] - a.B.offsets[y];
    if (m < 0 || n < 0 || m > a.A.max_len || n > a.B.max_len || m > kGMaxRows) {
        if (lane == 0) set_status(a.st, MSA_DS_LENGTH);
        return;
    }
    const int64_t cap = a.ops_off[p + 1] - a.ops_off[p];
    if (cap < m + n || a.tb_off[p + 1] - a.tb_off[p] < gotoh_tb_size((int32_t)m, (int32_t)n)) {
        if (lane == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    uint8_t *out = a.ops + a.ops_off[p];
    const uint4 *rec = (const uint4 *)(a.tb + a.tb_off[p]);
    const int32_t G = (int32_t)gotoh_lanes((int32_t)m);
    const int32_t nn = (int32_t)n;
    int32_t i = (int32_t)m, j = (int32_t)n;
    int64_t emitted = 0;
    uint32_t obuf = 0;
    int32_t s_hi = -1000000, g_hi = -1000000;
    uint4 tile[2];
    auto emit = [&](uint32_t op) {
        obuf = lane == (int)(emitted & 63) ? op : obuf;
        ++emitted;
        if ((emitted & 63) == 0) out[cap - emitted + (63 - lane)] = (uint8_t)obuf;
    };
    uint32_t last = 0;    // op chosen at the previous step (0 also at the start)
    uint32_t nextc = 0;   // code byte of the cell visited at the previous step
    while (i > 0 && j > 0) {
        const int32_t g = (i - 1) >> 4;
        const int32_t sp = (j - 1) + g;
        if (s_hi - sp < 0 || s_hi - sp >= 64 || g_hi - g < 0 || g_hi - g >= 2) {
            s_hi = sp;
            g_hi = g;
            const int64_t sl = s_hi - lane;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int64_t gq = g_hi - q;
                // record (sl, gq) exists iff its column sl - gq is in [0, n)
                const int64_t jc = sl - gq;
                tile[q] = (gq >= 0 && jc >= 0 && jc < nn) ? rec[sl * G + gq] : make_uint4(0, 0, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the tile is complete
        }
        const int Ls = s_hi - sp, q = g_hi - g;
        const int r = (i - 1) & 15;
        const uint32_t d0 = __builtin_amdgcn_readlane(tile[0].x, Ls);
        const uint32_t d1 = __builtin_amdgcn_readlane(tile[0].y, Ls);
        const uint32_t d2 = __builtin_amdgcn_readlane(tile[0].z, Ls);
        const uint32_t d3 = __builtin_amdgcn_readlane(tile[0].w, Ls);
        const uint32_t e0 = __builtin_amdgcn_readlane(tile[1].x, Ls);
        const uint32_t e1 = __builtin_amdgcn_readlane(tile[1].y, Ls);
        const uint32_t e2 = __builtin_amdgcn_readlane(tile[1].z, Ls);
        const uint32_t e3 = __builtin_amdgcn_readlane(tile[1].w, Ls);
        const int dw = r >> 2;
        const uint32_t w0 = dw == 0 ? d0 : dw == 1 ? d1 : dw == 2 ? d2 : d3;
        const uint32_t w1 = dw == 0 ? e0 : dw == 1 ? e1 : dw == 2 ? e2 : e3;
        const uint32_t c = ((q == 0 ? w0 : w1) >> (8 * (r & 3))) & 0xFFu;
        const uint32_t u0 = c & 3u, u1 = (c >> 2) & 3u;
        const bool hM = u0 >= 1u;                // the diagonal reaches H
        const bool hD = u1 >= 1u && u0 <= 1u;    // F reaches H
        const uint32_t ne = (nextc >> 4) & 3u, nf = nextc >> 6;
        uint32_t op;
        if (last == 1u) {          // after D: F[i+1][j] opens (nf >= 1) or extends (nf <= 1)
            op = (hM && nf >= 1u) ? 0u : (nf <= 1u ? 1u : 2u);
        } else if (last == 2u) {   // after I: E[i][j+1] opens (ne >= 1) or extends
            op = (hM && ne >= 1u) ? 0u : ((hD && ne >= 1u) ? 1u : 2u);
        } else {
            op = hM ? 0u : (hD ? 1u : 2u);
        }
        emit(op);
        i -= (op != 2u) ? 1 : 0;
        j -= (op != 1u) ? 1 : 0;
        last = op;
        nextc = c;
    }
    while (i > 0) {
        emit(1u);
        --i;
    }
    while (j > 0) {
        emit(2u);
        --j;
    }
    const int64_t rem = emitted & 63;
    if (rem && lane < rem) out[cap - emitted + (rem - 1 - lane)] = (uint8_t)obuf;
    // the alignment sits in out[cap - emitted .. cap); move it to the front.
    // Chunks move from low to high addresses and the destination lies below
    // the source, so no chunk overwrites bytes that are still to be read.
    const int64_t src0 = cap - emitted;
    if (src0 > 0) {
        __threadfence();
        for (int64_t c0 = 0; c0 < emitted; c0 += 64) {
            const int64_t k = c0 + lane;
            uint8_t v = 0;
            if (k < emitted) v = out[src0 + k];
            if (k < emitted) out[k] = v;
        }
    }
    if (lane == 0) a.ops_len[p] = (int32_t)emitted;
}

static int gotoh_check_costs(const int32_t *sub, int32_t sigma, int32_t open, int32_t ext) {
    if (sub == nullptr || open < 0 || ext < 0 || open + ext > kMaxSub) return MSA_EINVAL;
    for (int k = 0; k < sigma * sigma; ++k)
        if (sub[k] < -kMaxSub || sub[k] > kMaxSub) return MSA_EINVAL;
    return MSA_OK;
}

struct GotohWs {
    Staged SA, SB;
    int32_t *sub;
    int32_t *order;
};

template <class Alloc>
static GotohWs carve_gotoh(Alloc &al, const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    GotohWs w;
    const int64_t sa = staged_stride(A->max_len), sb = staged_stride(B->max_len);
    w.SA = Staged{al.template take<uint8_t>((size_t)A->n * sa),
                  al.template take<int32_t>((size_t)A->n + 1), sa, A->n};
    w.SB = Staged{al.template take<uint8_t>((size_t)B->n * sb),
                  al.template take<int32_t>((size_t)B->n + 1), sb, B->n};
    w.sub = al.template take<int32_t>(kSubStride * kSubStride);
    // launch order; min(n_pairs, kLptMaxPairs) entries, so that a workspace
    // sized for a batch also holds any smaller one
    w.order = al.template take<int32_t>((size_t)std::min<int64_t>(n_pairs, kLptMaxPairs));
    if (n_pairs > kLptMaxPairs) w.order = nullptr;
    return w;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t gotoh_tb_bytes(int32_t m, int32_t n) {
    if (m < 0 || n < 0) return 0;
    return (size_t)gotoh_tb_size(m, n);
}

size_t gotoh_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs) {
    if (check_seqs(A) || check_seqs(B) || n_pairs < 0) return 0;
    Sizer sz;
    carve_gotoh(sz, A, B, n_pairs);
    return sz.total();
}

int gotoh_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                int64_t n_pairs, const int32_t *sub, int32_t open, int32_t ext, int32_t *score,
                uint8_t *tb, const int64_t *tb_offsets, void *ws, size_t ws_bytes,
                int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0 || A->sigma != B->sigma) return MSA_EINVAL;
    if ((rc = gotoh_check_costs(sub, A->sigma, open, ext))) return rc;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || tb_offsets == nullptr || ws == nullptr) return MSA_EINVAL;
    if (tb == nullptr && (A->max_len > 0 && B->max_len > 0)) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL) return MSA_ERANGE;
    if (A->max_len > kGMaxRows) return MSA_ERANGE;
    Sizer sz;
    carve_gotoh(sz, A, B, n_pairs);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    const GotohWs w = carve_gotoh(cv, A, B, n_pairs);
    // the score table, padded to a row stride of kSubStride
    int32_t table[kSubStride * kSubStride] = {};
    for (int x = 0; x < A->sigma; ++x)
        for (int y = 0; y < A->sigma; ++y) table[x * kSubStride + y] = sub[x * A->sigma + y];
    if (hipMemcpyAsync(w.sub, table, sizeof(table), hipMemcpyHostToDevice, s) != hipSuccess)
        return MSA_EDEVICE;
    if ((rc = stage_set(A, nullptr, w.SA, d_status, s))) return rc;
    if ((rc = stage_set(B, nullptr, w.SB, d_status, s))) return rc;
    const int waves = (int)std::max<int64_t>(1, (gotoh_lanes(A->max_len) + 63) / 64);
    if (w.order)
        hipLaunchKernelGGL(k_lpt_order<kLptTile>, dim3((unsigned)((n_pairs + 255) / 256)),
                           dim3(256), 0, s, w.SA, w.SB, ia, ib, n_pairs, w.order);
    GotohArgs ga{w.SA, w.SB, ia, ib, w.sub, open, ext, score, tb, tb_offsets, d_status, w.order};
    hipLaunchKernelGGL(k_gotoh_fill, dim3((unsigned)n_pairs), dim3(64 * waves), 0, s, ga);
    return launch_status();
}

int gotoh_traceback(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                    int64_t n_pairs, const uint8_t *tb, const int64_t *tb_offsets, uint8_t *ops,
                    const int64_t *ops_offsets, int32_t *ops_len, int32_t *d_status,
                    hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || tb_offsets == nullptr || ops == nullptr ||
        ops_offsets == nullptr || ops_len == nullptr)
        return MSA_EINVAL;
    if (tb == nullptr && (A->max_len > 0 && B->max_len > 0)) return MSA_EINVAL;
    if (n_pairs > 0x7fffffffLL) return MSA_ERANGE;
    if (A->max_len > kGMaxRows) return MSA_ERANGE;
    GotohTbArgs ta{*A, *B, ia, ib, tb, tb_offsets, ops, ops_offsets, ops_len, d_status};
    hipLaunchKernelGGL(k_gotoh_traceback, dim3((unsigned)n_pairs), dim3(64), 0, s, ta);
    return launch_status();
}

}  // extern "C"
