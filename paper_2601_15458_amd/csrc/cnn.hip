// Learned surrogate of the Levenshtein distance: a 1D-CNN sequence embedder
// (4 conv layers of width 128, kernel 5, ReLU between, masked mean pool),
// trained so that the Euclidean distance of two embeddings approximates
// lev(a, b) / mean length.  BF16 weights and activations, FP32 accumulation
// on the matrix cores (v_mfma_f32_16x16x32_bf16), FP32 master weights and
// Adam state.
//
// Layout.  A batch's sequences are laid end to end as rows (one row per
// position, channels contiguous), each sequence framed by 2 zero rows on
// either side; kLead zero rows precede the first sequence and at least
// kLead + 127 follow the last.  A convolution output row r then reads the
// contiguous span X[(r - 2) * Cin .. (r - 2) * Cin + K * Cin), which makes
// every layer an implicit GEMM with rows x (K * Cin) times (K * Cin) x 128:
//   forward:        Z_l  = span(H_{l-1}) . W_l          (+ bias, ReLU, mask)
//   input gradient: dH   = span(dZ_l) . flip(W_l)^T     (x ReLU'(H), mask)
//   weight gradient dW_l = span(H_{l-1})^T . dZ_l       (reduction over rows)
// Padding rows are written as zeros by every epilogue, so the spans of the
// next layer see each sequence's zero padding.
#include <vector>

#include "common.hpp"

namespace msadp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint16_t bf16_t;   // storage type

constexpr int kW = 128;      // channels
constexpr int kKer = 5;      // kernel width
constexpr int kLayers = 4;
constexpr int kIn = 8;       // one-hot channels (sigma <= 8)
constexpr int kLead = 8;     // zero rows before the first sequence
constexpr int kRowTiles = 4; // 16-row MFMA tiles per wavefront in the conv GEMM
constexpr int kTile = 8 * 16 * kRowTiles;   // rows per GEMM workgroup (8 wavefronts)
// Rows per workgroup for R row tiles per wavefront (the one-hot layer, two
// K-steps only, takes R = 1: fewer registers, more wavefronts in flight).
__host__ __device__ constexpr int conv_tile(int R) { return 8 * 16 * R; }
constexpr int kRowTiles0 = 1;

__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? kIn : kW; }
__host__ __device__ constexpr int kd_of(int l) { return kKer * cin_of(l); }              // 40 / 640
__host__ __device__ constexpr int kdp_of(int l) { return (kd_of(l) + 31) / 32 * 32; }   // 64 / 640

// ------------------------------------------------------------ parameters
// One device blob; offsets in floats (bf16 copies use the same byte offsets).
struct ParamLayout {
    size_t w[kLayers], b[kLayers];              // fp32 master [128][kdp], [128]
    size_t mw[kLayers], mb[kLayers], vw[kLayers], vb[kLayers];
    size_t gw[kLayers], gb[kLayers];            // fp32 gradients
    size_t wt[kLayers];                         // bf16 forward [128][kdp] (byte offsets)
    size_t wbt[kLayers];                        // bf16 input-gradient [cin][640]
    size_t bytes;
};

static ParamLayout param_layout() {
    ParamLayout p{};
    size_t off = 0;   // bytes
    auto take = [&](size_t bytes) {
        off = (off + 255) / 256 * 256;
        size_t o = off;
        off += bytes;
        return o;
    };
    for (int l = 0; l < kLayers; ++l) {
        const size_t nw = (size_t)kW * kdp_of(l);
        p.w[l] = take(4 * nw);
        p.b[l] = take(4 * kW);
        p.mw[l] = take(4 * nw);
        p.mb[l] = take(4 * kW);
        p.vw[l] = take(4 * nw);
        p.vb[l] = take(4 * kW);
        p.gw[l] = take(4 * nw);
        p.gb[l] = take(4 * kW);
        p.wt[l] = take(2 * nw);
        p.wbt[l] = take(2 * (size_t)cin_of(l) * kKer * kW);
    }
    p.bytes = take(0) + 256;
    return p;
}

template <class T>
__host__ __device__ inline T *at(void *base, size_t off) { return (T *)((uint8_t *)base + off); }

__device__ inline bf16_t to_bf16(float f) {
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ inline float from_bf16(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Forward weights Wt[co][k*cin + ci] and input-gradient weights
// Wbt[ci][k'*128 + co] = W[K-1-k'][ci][co] from the fp32 master.
__global__ void k_pack_weights(void *P, ParamLayout pl) {
    for (int l = 0; l < kLayers; ++l) {
        const int kdp = kdp_of(l), cin = cin_of(l);
        const float *w = at<float>(P, pl.w[l]);
        bf16_t *wt = at<bf16_t>(P, pl.wt[l]);
        bf16_t *wbt = at<bf16_t>(P, pl.wbt[l]);
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kW * kdp;
             i += gridDim.x * blockDim.x) {
            wt[i] = to_bf16(w[i]);
            const int co = i / kdp, kk = i % kdp;
            if (kk < kd_of(l)) {
                const int k = kk / cin, ci = kk % cin;
                wbt[(size_t)ci * kKer * kW + (kKer - 1 - k) * kW + co] = to_bf16(w[i]);
            }
        }
    }
}

// ------------------------------------------------------------ batch layout
struct Batch {
    const uint8_t *codes;    // staged rows of the sequence set
    const int32_t *len;
    int64_t stride;
    const int32_t *idx;      // sequences of the batch
    int32_t nb;
    int64_t rows;            // data + framing rows (excludes lead/tail)
    int64_t *roff;           // [nb + 1] first row of each sequence's frame
    int32_t *rowseq;         // [rows] batch index of a data row, -1 for framing
};

__global__ void k_frame_lengths(Batch b, int32_t *st) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= b.nb; i += gridDim.x * blockDim.x)
        b.roff[i] = i < b.nb ? (int64_t)b.len[b.idx[i]] + 4 : 0;
}

__global__ void k_frame_rows(Batch b, int32_t *st) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && b.roff[b.nb] != b.rows)
        set_status(st, MSA_DS_CAPACITY);
    for (int i = blockIdx.x; i < b.nb; i += gridDim.x) {
        const int64_t r0 = b.roff[i];
        const int32_t L = b.len[b.idx[i]];
        if (r0 + L + 4 > b.rows) continue;
        for (int64_t t = threadIdx.x; t < L + 4; t += blockDim.x)
            b.rowseq[r0 + t] = (t >= 2 && t < L + 2) ? i : -1;
    }
}

// One-hot input rows (8 channels, bf16).
__global__ void k_onehot(Batch b, bf16_t *H0) {
    for (int i = blockIdx.x; i < b.nb; i += gridDim.x) {
        const int64_t r0 = b.roff[i];
        const int32_t s = b.idx[i], L = b.len[s];
        const uint8_t *x = b.codes + (int64_t)s * b.stride;
        for (int64_t t = threadIdx.x; t < (int64_t)(L + 4) * kIn; t += blockDim.x) {
            const int64_t row = t / kIn, c = t % kIn;
            const bool data = row >= 2 && row < L + 2;
            const float v = (data && x[row - 2] == c) ? 1.0f : 0.0f;
            H0[(kLead + r0 + row) * kIn + c] = to_bf16(v);
        }
    }
}

// ------------------------------------------------------------ conv GEMM
enum { kEpiRelu = 0, kEpiLinearF32 = 1, kEpiGradRelu = 2 };

struct ConvArgs {
    const bf16_t *X;         // input rows (lead included), cin channels
    const bf16_t *Wt;        // [128][kdp]
    const float *bias;
    const int32_t *rowseq;
    int64_t rows;
    void *out;               // output rows (lead included), 128 channels
    const bf16_t *relu_ref;  // rows whose sign gates the input gradient
};

// Workgroup = 8 wavefronts = kTile output rows x 128 channels; wavefront w
// owns rows [16 R w, 16 R (w + 1)), R = kRowTiles: R x 8 tiles of 16 x 16, K
// in steps of 32.  Each weight fragment read from LDS feeds R MFMAs, so R
// sets the LDS bytes per FLOP (the LDS read rate, not the matrix unit, is
// what limits the GEMM at R = 2).
// The A fragments (8 consecutive span elements of one row) are 16-byte
// global loads; the weights' K slice of each step, shared by the eight
// wavefronts, is staged in LDS ([co][32], padded) and read as 16-byte
// fragments.  Global loads run two steps ahead of the MFMAs, the LDS slice
// one step (two LDS buffers, one barrier a step).
constexpr int kBp = 40;   // LDS pitch of a staged weight row (32 + 8)
constexpr int kOp = 136;  // LDS pitch of a staged output row (128 + 8)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Lane i of every 16-lane row receives lane (i + N) mod 16 of the same row
// (DPP row rotate right by 16 - N).
template <int N>
__device__ __forceinline__ uint32_t row_rotl(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x120 + (16 - N), 0xF, 0xF, false);
}

// A fragment of tap N from the tap-0 fragments of a tile (lo) and of the
// tile below it (hi): in the 16 x 32 fragment, lane i of each 16-lane row
// holds span row i, and tap N reads span row i + N, which is lane i + N of
// lo, or lane i + N - 16 of hi once that passes the tile.
template <int N>
__device__ __forceinline__ bf16x8 shift_rows(bf16x8 lo, bf16x8 hi, int li) {
    const u32x4 a = __builtin_bit_cast(u32x4, lo), b = __builtin_bit_cast(u32x4, hi);
    const bool from_lo = li < 16 - N;
    u32x4 r;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t x = row_rotl<N>(a[d]), y = row_rotl<N>(b[d]);
        r[d] = from_lo ? x : y;
    }
    return __builtin_bit_cast(bf16x8, r);
}

// DPP controls: row_shl:1 (lane i of a 16-lane row takes lane i + 1) and
// row_shr:n (lane i takes lane i - n); lanes with no source keep `old`.
constexpr int kDppRowShl1 = 0x101;
constexpr int kDppRowShr = 0x110;

template <int N>
__device__ __forceinline__ float shr_rows(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowShr + N, 0xF,
                                                      0xF, false));
}

__device__ __forceinline__ bf16x8 tap_rows(bf16x8 lo, bf16x8 hi, int tap, int li) {
    switch (tap) {
    case 1: return shift_rows<1>(lo, hi, li);
    case 2: return shift_rows<2>(lo, hi, li);
    case 3: return shift_rows<3>(lo, hi, li);
    case 4: return shift_rows<4>(lo, hi, li);
    default: return lo;
    }
}

template <int CIN, int KDP, int EPI, int RT = kRowTiles>
__global__ void __launch_bounds__(512) k_conv(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) bf16_t sb[2][kW * kBp];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * conv_tile(RT) + 16 * RT * w;
    f32x4 acc[RT][8];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    const int kq = 8 * (lane >> 4);   // this lane's first K element of a step
    const int li = lane & 15;
    const bf16_t *arow[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
        arow[i] = a.X + (kLead + row0 + 16 * i + li - 2) * CIN + kq;
    // staging role: weight row co = t / 4, quarter q = t % 4 (8 of the 32 K)
    const int sco = threadIdx.x >> 2, sq = (threadIdx.x & 3) * 8;
    const bf16_t *wsrc = a.Wt + (size_t)sco * KDP + sq;
    // K order: 32-channel column blocks outer, kernel taps inner, so the five
    // taps of a block re-read the same input columns (one row apart) while
    // they are still in the L1 cache
    constexpr int kSteps = KDP / 32;
    constexpr int kTaps = CIN >= 32 ? kKer : kSteps;   // K steps per column block
    auto k_of = [](int step) { return CIN >= 32 ? (step % kTaps) * CIN + (step / kTaps) * 32 : step * 32; };
    // Loads run two steps ahead (slot = step & 1; the loop is unrolled, so
    // the slots are fixed registers): the weight quarter a thread stages and
    // (one-hot layer) the A fragments of step s + 2 are requested while step
    // s computes.  For the 128-channel layers the five taps of a column block
    // read the same rows shifted by one, so the block's tap-0 fragments (the
    // wavefront's tiles plus the 16 rows below them) are loaded once, a
    // column block ahead, and taps 1-4 are rotated out of them across lanes.
    constexpr bool kShift = CIN >= 32;
    constexpr int kBlocks = kShift ? kSteps / kKer : 1;
    const bf16_t *ahalo = a.X + (kLead + row0 + 16 * RT + li - 2) * CIN + kq;
    uint4 wq[2];
    bf16x8 aq[2][RT];
    bf16x8 tq[2][RT + 1];
#pragma unroll
    for (int s0 = 0; s0 < 2 && s0 < kSteps; ++s0) wq[s0] = *(const uint4 *)(wsrc + k_of(s0));
    if constexpr (kShift) {
#pragma unroll
        for (int i = 0; i < RT; ++i) tq[0][i] = *(const bf16x8 *)(arow[i]);
        tq[0][RT] = *(const bf16x8 *)(ahalo);
    } else {
#pragma unroll
        for (int s0 = 0; s0 < 2 && s0 < kSteps; ++s0)
#pragma unroll
            for (int i = 0; i < RT; ++i) aq[s0][i] = *(const bf16x8 *)(arow[i] + k_of(s0));
    }
    *(uint4 *)(sb[0] + sco * kBp + sq) = wq[0];
    __syncthreads();
#pragma unroll
    for (int step = 0; step < kSteps; ++step) {
        const int cur = step & 1;
        bf16x8 af[RT];
        if constexpr (kShift) {
            const int cb = step / kKer, tap = step % kKer;
            if (tap == 0 && cb + 1 < kBlocks) {
                const int nb = (cb + 1) & 1, k1 = (cb + 1) * 32;
#pragma unroll
                for (int i = 0; i < RT; ++i) tq[nb][i] = *(const bf16x8 *)(arow[i] + k1);
                tq[nb][RT] = *(const bf16x8 *)(ahalo + k1);
            }
#pragma unroll
            for (int i = 0; i < RT; ++i) af[i] = tap_rows(tq[cb & 1][i], tq[cb & 1][i + 1], tap, li);
        } else {
#pragma unroll
            for (int i = 0; i < RT; ++i) af[i] = aq[cur][i];
        }
        const uint4 wstage = wq[cur ^ 1];          // weights of step + 1
        if (step + 2 < kSteps) {
            const int k2 = k_of(step + 2);
            wq[cur] = *(const uint4 *)(wsrc + k2);
            if constexpr (!kShift) {
#pragma unroll
                for (int i = 0; i < RT; ++i) aq[cur][i] = *(const bf16x8 *)(arow[i] + k2);
            }
        }
        bf16x8 bfr[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) bfr[j] = *(const bf16x8 *)(sb[cur] + (16 * j + li) * kBp + kq);
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
        if (step + 1 < kSteps) *(uint4 *)(sb[cur ^ 1] + sco * kBp + sq) = wstage;
        __syncthreads();
    }
    // The weights are the first MFMA operand, so tile (i, j) is the
    // transposed output: the lane holds channels 16 j + 4 (lane / 16) + r,
    // r = 0..3, of row 16 i + lane % 16, stored as one 4-channel piece.
    if constexpr (EPI == kEpiLinearF32) {
        // Last layer: only its mean over each sequence is used, so the rows
        // are summed here.  Within each 16-row tile (one 16-lane DPP row per
        // channel group) a segmented inclusive scan keyed by the sequence id
        // leaves the sum of each sequence's rows of the tile in the lane of
        // its last row, which alone is stored (k_pool adds the tiles).
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int64_t row = row0 + 16 * i + li;
            const int sid = row < a.rows ? a.rowseq[row] : -1;
            const int below = __builtin_amdgcn_update_dpp(-3, sid, kDppRowShl1, 0xF, 0xF, false);
            const bool last = sid >= 0 && below != sid;
            // all-ones where the lane n above holds the same sequence: the
            // sums are masked with it, so every lane runs every DPP move (a
            // lane that skipped one would hand 0 to the lane below it)
            int same[4];
            same[0] = -(int)(__builtin_amdgcn_update_dpp(-2, sid, kDppRowShr + 1, 0xF, 0xF, false) == sid);
            same[1] = -(int)(__builtin_amdgcn_update_dpp(-2, sid, kDppRowShr + 2, 0xF, 0xF, false) == sid);
            same[2] = -(int)(__builtin_amdgcn_update_dpp(-2, sid, kDppRowShr + 4, 0xF, 0xF, false) == sid);
            same[3] = -(int)(__builtin_amdgcn_update_dpp(-2, sid, kDppRowShr + 8, 0xF, 0xF, false) == sid);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c0 = 16 * j + 4 * (lane >> 4);
                const float4 b4 = *(const float4 *)(a.bias + c0);
                const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = __int_as_float(__float_as_int(acc[i][j][r] + bb[r]) & -(int)(sid >= 0));
                    v[r] += __int_as_float(__float_as_int(shr_rows<1>(v[r])) & same[0]);
                    v[r] += __int_as_float(__float_as_int(shr_rows<2>(v[r])) & same[1]);
                    v[r] += __int_as_float(__float_as_int(shr_rows<4>(v[r])) & same[2]);
                    v[r] += __int_as_float(__float_as_int(shr_rows<8>(v[r])) & same[3]);
                }
                if (last)
                    *(float4 *)((float *)a.out + (kLead + row) * kW + c0) =
                        make_float4(v[0], v[1], v[2], v[3]);
            }
        }
        return;
    }
    // bf16 outputs: each 16-row tile goes through the wavefront's LDS slice
    // so that the stores are whole rows (4 rows of 256 bytes per store)
    // instead of 8-byte pieces spread over 16 rows.
    __shared__ __attribute__((aligned(16))) bf16_t so[8][16 * kOp];
    bf16_t *sw = so[w];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int64_t rbase = row0 + 16 * i;
        const int64_t row = rbase + li;                  // < the allocated rows
        const bool data = row < a.rows && a.rowseq[row] >= 0;
        if (EPI == kEpiGradRelu) {
            // the gating rows come in the same way, whole rows into the slice
            // (each lane then reads and overwrites only its own pieces)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int rr = 4 * k + (lane >> 4), c = 8 * (lane & 15);
                *(uint4 *)(sw + rr * kOp + c) =
                    *(const uint4 *)(a.relu_ref + (kLead + rbase + rr) * kW + c);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c0 = 16 * j + 4 * (lane >> 4);
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = acc[i][j][r];
            {
                float z[4];
                if (EPI == kEpiRelu) {
                    const float4 b4 = *(const float4 *)(a.bias + c0);
                    const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float y = v[r] + bb[r];
                        z[r] = data && y > 0.0f ? y : 0.0f;
                    }
                } else {
                    const uint2 ref = *(const uint2 *)(sw + li * kOp + c0);
                    const uint32_t rr[2] = {ref.x, ref.y};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bf16_t h = (bf16_t)(rr[r >> 1] >> (16 * (r & 1)));
                        z[r] = data && from_bf16(h) > 0.0f ? v[r] : 0.0f;
                    }
                }
                const uint32_t p0 = (uint32_t)to_bf16(z[0]) | ((uint32_t)to_bf16(z[1]) << 16);
                const uint32_t p1 = (uint32_t)to_bf16(z[2]) | ((uint32_t)to_bf16(z[3]) << 16);
                *(uint2 *)(sw + li * kOp + c0) = make_uint2(p0, p1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int rr = 4 * k + (lane >> 4), c = 8 * (lane & 15);
            const uint4 piece = *(const uint4 *)(sw + rr * kOp + c);
            if (rbase + rr < a.rows)
                *(uint4 *)((bf16_t *)a.out + (kLead + rbase + rr) * kW + c) = piece;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Weight gradient: gW[co][kk] += sum over rows r of dZ[r][co] * span(H)[r][kk],
// with kk = k * CIN + ci and span(H)[r][kk] = H[r + k - 2][ci]; blockIdx.x = 0
// also adds the bias gradient gb[co] += sum over rows of dZ[r][co].
// The reduction runs over rows, which the matrix cores take 32 at a time
// (8 consecutive rows per lane, row-major tiles being channel-contiguous), so
// the fragments come from LDS through the transposing read
// ds_read_b64_tr_b16: within each group of 16 lanes, lane 4j + q names 4
// consecutive channels (4q .. 4q + 3 of a 16-channel tile) of row j, and
// lane i receives channel i of the 4 rows.  Each 64-row step stages dZ rows
// and H rows (shifted by k - 2, with a two-row halo either side for the
// one-hot layer) row-major with 16-byte writes.  blockIdx.x = k covers
// kk in [128 k, 128 k + 128) for CIN = 128; one block holds the one-hot
// layer's 40 columns (5 taps x 8).  Workgroup = 4 wavefronts, wavefront w
// owns co in [32 w, 32 w + 32) x the block's kk.
constexpr int kWgChunk = 4096;      // rows per workgroup (128-channel layers)
constexpr int kWgChunk0 = 2048;     // rows per workgroup (one-hot layer: one column block)
constexpr int kStep = 64;      // rows staged per step
constexpr int kPitch = 144;    // LDS row pitch of the 128-channel tiles (288 bytes)
constexpr int kHalo = 2;

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16;

// Rows r .. r + 3 of one channel per lane (see above); p = this lane's address.
__device__ __forceinline__ v4i16 read_tr(const bf16_t *p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16 *)(bf16_t *)p);
}

__device__ __forceinline__ bf16x8 join_frag(v4i16 lo, v4i16 hi) {
    const v4i16 both[2] = {lo, hi};
    return __builtin_bit_cast(bf16x8, both);
}

template <int CIN, int KDP>
__global__ void __launch_bounds__(256) k_conv_wgrad(const bf16_t *H, const bf16_t *dZ,
                                                    int64_t rows, float *part, float *part_b) {
    // this chunk's partial sums: part[chunk][co][kk], part_b[chunk][co]
    float *gW = part + (size_t)blockIdx.y * kW * KDP;
    float *gb = part_b + (size_t)blockIdx.y * kW;
    constexpr int NT = (KDP < 128 ? KDP : 128) / 16;   // 16-column tiles per block
    constexpr int KD = kKer * CIN;
    constexpr int kHRows = CIN == kW ? kStep : kStep + 2 * kHalo;
    constexpr int kHPitch = CIN == kW ? kPitch : CIN;
    __shared__ __attribute__((aligned(16))) bf16_t sdz[kStep * kPitch];
    __shared__ __attribute__((aligned(16))) bf16_t sh[kHRows * kHPitch + 8];   // + zero slot
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4, t = lane & 15;
    const int kb = blockIdx.x;
    const int kk0 = kb * 128;
    constexpr int64_t kChunk = CIN == kW ? kWgChunk : kWgChunk0;
    const int64_t r_begin = (int64_t)blockIdx.y * kChunk;
    const int64_t r_end = min(rows, r_begin + kChunk);
    bf16_t *zero_slot = sh + kHRows * kHPitch;
    if (threadIdx.x < 8) zero_slot[threadIdx.x] = 0;
    f32x4 acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    float bsum = 0.0f;
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kStep) {
        __syncthreads();
        // dZ rows r0 .. r0 + 63, 16 channels per thread and pass (rows at or
        // past the chunk end read as zero)
        for (int e = threadIdx.x; e < kStep * 16; e += blockDim.x) {
            const int rr = e >> 4, c = (e & 15) * 8;
            const bool live = r0 + rr < r_end;
            const uint4 v = live ? *(const uint4 *)(dZ + (kLead + r0 + rr) * kW + c)
                                 : make_uint4(0, 0, 0, 0);
            *(uint4 *)(sdz + rr * kPitch + c) = v;
        }
        if (CIN == kW) {
            // H rows r0 + kb - 2 + rr (inside the framed buffer: lead rows
            // before the first row, tail rows after the last)
            for (int e = threadIdx.x; e < kStep * 16; e += blockDim.x) {
                const int rr = e >> 4, c = (e & 15) * 8;
                *(uint4 *)(sh + rr * kPitch + c) =
                    *(const uint4 *)(H + (kLead + r0 + kb - 2 + rr) * kW + c);
            }
        } else {
            // H rows r0 - 2 .. r0 + 65, one 16-byte row per thread
            for (int rr = threadIdx.x; rr < kHRows; rr += blockDim.x)
                *(uint4 *)(sh + rr * CIN) = *(const uint4 *)(H + (kLead + r0 - kHalo + rr) * CIN);
        }
        __syncthreads();
        if (kb == 0 && threadIdx.x < kW) {
#pragma unroll 8
            for (int rr = 0; rr < kStep; ++rr) bsum += from_bf16(sdz[rr * kPitch + threadIdx.x]);
        }
#pragma unroll
        for (int ks = 0; ks < kStep; ks += 32) {
            const int rb = ks + 8 * g + (t >> 2);   // this lane's row of the first read
            bf16x8 af[2], bfr[NT];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16_t *p = sdz + rb * kPitch + 32 * w + 16 * i + 4 * (t & 3);
                af[i] = join_frag(read_tr(p), read_tr(p + 4 * kPitch));
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const bf16_t *p;
                int step4;
                if (CIN == kW) {
                    p = sh + rb * kPitch + 16 * n + 4 * (t & 3);
                    step4 = 4 * kPitch;
                } else {
                    // columns kk0 + 16 n + 4 (t & 3) .. + 3 share one tap k
                    const int kk = kk0 + 16 * n + 4 * (t & 3);
                    const int k = kk / CIN, ci = kk % CIN;
                    p = kk < KD ? sh + (rb + k - 2 + kHalo) * CIN + ci : zero_slot;
                    step4 = kk < KD ? 4 * CIN : 0;
                }
                bfr[n] = join_frag(read_tr(p), read_tr(p + step4));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[i][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[n], acc[i][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int kk = kk0 + 16 * n + t;
            if (kk >= KDP) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 32 * w + 16 * i + 4 * g + r;
                gW[(size_t)co * KDP + kk] = acc[i][n][r];
            }
        }
    if (kb == 0 && threadIdx.x < kW) gb[threadIdx.x] = bsum;
}

// Weight gradient of the 128-channel layers with every tap from one staging
// of the rows: a workgroup takes a 4096-row chunk and one half of the output
// channels (64 co) against all 640 columns kk = k * 128 + ci, so a row's H is
// read twice and its dZ once (each half reads its own 64 channels).  Each
// 64-row step stages the chunk's 64 dZ rows (the half's channels) and the 68
// H rows r0 - 2 .. r0 + 65 that the five taps need; the next step's rows are
// loaded into registers while the current one computes.  Eight wavefronts:
// wavefront w owns the half's 4 co tiles x column tiles 5 w .. 5 w + 4 (20
// matrix tiles, 80 accumulators).  The chunk's sums go to its own slice of
// a partial buffer (no atomics); every workgroup also sums its 64 channels
// of dZ over the chunk's rows (bias gradient).
constexpr int kWgRows = 4096;
constexpr int kHRows2 = kStep + 2 * kHalo;   // 68
constexpr int kZPitch = 72;                  // LDS row pitch of the 64-channel dZ tile

__global__ void __launch_bounds__(512) k_conv_wgrad_h(const bf16_t *H, const bf16_t *dZ,
                                                      int64_t rows, float *part,
                                                      float *part_b) {
    constexpr int KDP = kKer * kW;   // 640
    __shared__ __attribute__((aligned(16))) bf16_t sdz[kStep * kZPitch];
    __shared__ __attribute__((aligned(16))) bf16_t sh[kHRows2 * kPitch];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4, t = lane & 15;
    const int tid = threadIdx.x;
    const int half = blockIdx.x;
    const int64_t r_begin = (int64_t)blockIdx.y * kWgRows;
    const int64_t r_end = min(rows, r_begin + kWgRows);
    const int cz = 64 * half;        // first dZ channel (co) of the half
    const int kt0 = 5 * w;           // first column tile (of 40)
    f32x4 acc[4][5];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 5; ++u) acc[i][u] = f32x4{0, 0, 0, 0};
    float bsum = 0.0f;
    // 16-byte pieces of a step: dZ 64 rows x 8, H 68 rows x 16
    uint4 pz, ph[3];
    auto load = [&](int64_t r0) {
        {
            const int rr = tid >> 3, c = (tid & 7) * 8;
            pz = r0 + rr < r_end ? *(const uint4 *)(dZ + (kLead + r0 + rr) * kW + cz + c)
                                 : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 512 * q, rr = e >> 4, c = (e & 15) * 8;
            // rows r0 - 2 .. r0 + 65 lie inside the framed buffer (lead and
            // tail rows); dZ rows past the chunk are zero, so the H rows they
            // meet contribute nothing
            ph[q] = e < kHRows2 * 16 ? *(const uint4 *)(H + (kLead + r0 - kHalo + rr) * kW + c)
                                     : make_uint4(0, 0, 0, 0);
        }
    };
    load(r_begin);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kStep) {
        __syncthreads();
        *(uint4 *)(sdz + (tid >> 3) * kZPitch + (tid & 7) * 8) = pz;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int e = tid + 512 * q, rr = e >> 4, c = (e & 15) * 8;
            if (e < kHRows2 * 16) *(uint4 *)(sh + rr * kPitch + c) = ph[q];
        }
        __syncthreads();
        if (r0 + kStep < r_end) load(r0 + kStep);
        if (tid < 64) {
#pragma unroll 8
            for (int rr = 0; rr < kStep; ++rr) bsum += from_bf16(sdz[rr * kZPitch + tid]);
        }
#pragma unroll
        for (int ks = 0; ks < kStep; ks += 32) {
            const int rb = ks + 8 * g + (t >> 2);   // this lane's row of the first read
            bf16x8 af[4], bfr[5];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bf16_t *p = sdz + rb * kZPitch + 16 * i + 4 * (t & 3);
                af[i] = join_frag(read_tr(p), read_tr(p + 4 * kZPitch));
            }
#pragma unroll
            for (int u = 0; u < 5; ++u) {
                const int kk = 16 * (kt0 + u);
                const int k = kk >> 7, ci0 = kk & (kW - 1);   // tap, first channel
                const bf16_t *p = sh + (rb + k) * kPitch + ci0 + 4 * (t & 3);
                bfr[u] = join_frag(read_tr(p), read_tr(p + 4 * kPitch));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int u = 0; u < 5; ++u)
                    acc[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[u], acc[i][u],
                                                                        0, 0, 0);
        }
    }
    float *gW = part + (size_t)blockIdx.y * kW * KDP;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int kk = 16 * (kt0 + u) + t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = cz + 16 * i + 4 * g + r;
                gW[(size_t)co * KDP + kk] = acc[i][u][r];
            }
        }
    if (tid < 64) part_b[(size_t)blockIdx.y * kW + cz + tid] = bsum;
}

// gW = sum of the chunks' partial sums, chunk 0 first (a fixed order, so equal
// inputs give equal bits); the same for the bias.
__global__ void k_wgrad_reduce(const float *part, const float *part_b, int32_t chunks,
                               int32_t n, float *gW, float *gb) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n + kW; i += gridDim.x * blockDim.x) {
        const bool bias = i >= n;
        const float *src = bias ? part_b + (i - n) : part + i;
        const int64_t stride = bias ? kW : n;
        float sum = 0.0f;
#pragma unroll 8
        for (int c = 0; c < chunks; ++c) sum += src[(int64_t)c * stride];
        if (bias) gb[i - n] = sum;
        else gW[i] = sum;
    }
}

// ------------------------------------------------------------ pool, loss
// Mean over each sequence's rows.  The last layer stored, for every 16-row
// tile (tiles start at multiples of 16) that holds rows of the sequence, the
// sum of those rows at the row of the tile where the sequence's rows end:
// min(last data row, tile end).  The tiles are added in order.
__global__ void __launch_bounds__(128) k_pool(Batch b, const float *Z4, float *E) {
    const int c = threadIdx.x;
    for (int i = blockIdx.x; i < b.nb; i += gridDim.x) {
        const int64_t r0 = b.roff[i] + 2;
        const int32_t L = b.len[b.idx[i]];
        float s = 0.0f;
        if (L > 0) {
            const int64_t r1 = r0 + L - 1;
            for (int64_t t = r0 / 16; t <= r1 / 16; ++t) {
                const int64_t e = r1 < 16 * t + 15 ? r1 : 16 * t + 15;
                s += Z4[(kLead + e) * kW + c];
            }
        }
        E[(int64_t)i * kW + c] = L > 0 ? s / (float)L : 0.0f;
    }
}

// One wavefront per pair: pred = ||E[a] - E[b]||, r = pred - y; the pair's
// gradient row G[p] = 2 r / (P pred) (E[a] - E[b]) (added to dE[a],
// subtracted from dE[b] by k_seq_grad) and r2[p] = r^2 / P.
__global__ void __launch_bounds__(64) k_pair_loss(const float *E, const int32_t *pa,
                                                 const int32_t *pb, const float *label,
                                                 int32_t P, float *G, float *r2) {
    const int lane = lane_id();
    const int p = blockIdx.x;
    const int a = pa[p], bq = pb[p];
    const float d0 = E[(int64_t)a * kW + lane] - E[(int64_t)bq * kW + lane];
    const float d1 = E[(int64_t)a * kW + lane + 64] - E[(int64_t)bq * kW + lane + 64];
    float ss = d0 * d0 + d1 * d1;
    for (int o = 32; o >= 1; o >>= 1) ss += __shfl_xor(ss, o, kWave);
    const float pred = sqrtf(ss);
    const float r = pred - label[p];
    const float scale = pred > 0.0f ? 2.0f * r / ((float)P * pred) : 0.0f;
    G[(int64_t)p * kW + lane] = scale * d0;
    G[(int64_t)p * kW + lane + 64] = scale * d1;
    if (lane == 0) r2[p] = r * r / (float)P;
}

// The pairs of each batch sequence, as entries 2p (the sequence is a) and
// 2p + 1 (it is b) in a CSR list: counts, then a scatter (any order).
__global__ void k_pair_count(const int32_t *pa, const int32_t *pb, int32_t P, int32_t *cnt) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        atomicAdd(&cnt[pa[p]], 1);
        atomicAdd(&cnt[pb[p]], 1);
    }
}

__global__ void k_pair_fill(const int32_t *pa, const int32_t *pb, int32_t P, int64_t *cursor,
                            int32_t *list) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        list[atomicAdd((unsigned long long *)&cursor[pa[p]], 1ull)] = 2 * p;
        list[atomicAdd((unsigned long long *)&cursor[pb[p]], 1ull)] = 2 * p + 1;
    }
}

// dE[i] = sum of +G[p] (entries 2p) and -G[p] (entries 2p + 1) of sequence
// i's list, taken in increasing entry order whatever order the scatter left
// (one wavefront per sequence; lists hold a few entries).
__global__ void __launch_bounds__(64) k_seq_grad(const int64_t *start, const int32_t *list,
                                                const float *G, int32_t nb, float *dE) {
    const int lane = lane_id();
    for (int i = blockIdx.x; i < nb; i += gridDim.x) {
        const int64_t s0 = start[i];
        const int32_t k = (int32_t)(start[i + 1] - s0);
        float a0 = 0.0f, a1 = 0.0f;
        int32_t prev = -1;
        for (int32_t r = 0; r < k; ++r) {
            int32_t mn = 0x7fffffff;
            for (int32_t e = lane; e < k; e += 64) {
                const int32_t v = list[s0 + e];
                mn = (v > prev && v < mn) ? v : mn;
            }
            for (int o = 32; o >= 1; o >>= 1) mn = min(mn, __shfl_xor(mn, o, kWave));
            const int32_t pq = mn >> 1;
            const float sg = (mn & 1) ? -1.0f : 1.0f;
            a0 += sg * G[(int64_t)pq * kW + lane];
            a1 += sg * G[(int64_t)pq * kW + lane + 64];
            prev = mn;
        }
        dE[(int64_t)i * kW + lane] = a0;
        dE[(int64_t)i * kW + lane + 64] = a1;
    }
}

// loss = sum of r2 in a fixed order: strided per-thread sums, then a tree.
__global__ void __launch_bounds__(1024) k_sum_fixed(const float *x, int32_t n, float *out) {
    __shared__ float part[1024];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 1024) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// Regression target of a pair: lev(a, b) / ((|a| + |b|) / 2).
__global__ void k_labels(Batch b, const int32_t *pa, const int32_t *pb, const uint16_t *dist,
                         int32_t P, float *label) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const float la = (float)b.len[b.idx[pa[p]]], lb = (float)b.len[b.idx[pb[p]]];
        label[p] = la + lb > 0.0f ? (float)dist[p] / (0.5f * (la + lb)) : 0.0f;
    }
}

// Mean-pool backward: dZ4[r][c] = dE[seq][c] / L on data rows, 0 elsewhere.
// Thread = 8 channels of one row (one 16-byte store); a workgroup covers 16
// rows per trip.
__global__ void __launch_bounds__(128) k_pool_bwd(Batch b, const float *dE, bf16_t *dZ4) {
    const int c = (threadIdx.x & 15) * 8;
    for (int64_t r = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 4); r < b.rows;
         r += (int64_t)gridDim.x * 8) {
        const int32_t i = b.rowseq[r];
        float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (i >= 0) {
            const float L = (float)b.len[b.idx[i]];
            const float4 e0 = *(const float4 *)(dE + (int64_t)i * kW + c);
            const float4 e1 = *(const float4 *)(dE + (int64_t)i * kW + c + 4);
            const float e[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = e[k] / L;
        }
        uint4 o;
        o.x = (uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
        o.y = (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
        o.z = (uint32_t)to_bf16(v[4]) | ((uint32_t)to_bf16(v[5]) << 16);
        o.w = (uint32_t)to_bf16(v[6]) | ((uint32_t)to_bf16(v[7]) << 16);
        *(uint4 *)(dZ4 + (kLead + r) * kW + c) = o;
    }
}

// Adam (Kingma & Ba) on one flat array.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_widen_i32(const int32_t *a, int64_t n, int64_t *b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}


// ------------------------------------------------------------ host side
struct CnnWork {
    Batch b;
    bf16_t *h[kLayers];      // H0 (8 ch), H1..H3 (128 ch)
    float *z4;               // last layer output (fp32)
    bf16_t *dz;              // gradient rows (two buffers)
    bf16_t *dz2;
    float *E, *dE, *loss, *label;
    float *part, *part_b;    // weight-gradient partial sums per row chunk
    float *G, *r2;           // per-pair gradient rows and squared errors
    int32_t *cnt, *list;     // pairs of each batch sequence (CSR)
    int64_t *pstart, *pcur;
    int64_t alloc_rows;
};

static int64_t wgrad_chunks(int64_t rows) { return (rows + kWgRows - 1) / kWgRows; }
static int64_t wgrad_chunks0(int64_t rows) { return (rows + kWgChunk0 - 1) / kWgChunk0; }
static size_t wgrad_part_floats(int64_t rows) {
    return std::max((size_t)wgrad_chunks(rows) * kW * kd_of(1),
                    (size_t)wgrad_chunks0(rows) * kW * kdp_of(0));
}

// Tail: the last tile's overhang plus the longest span (8 rows) past it.
constexpr int kTail = 64;
static int64_t alloc_rows_for(int64_t rows) {
    return kLead + (rows + kTile - 1) / kTile * kTile + kTail;
}

template <class Alloc>
static void cnn_layout(Alloc &al, int32_t nb, int64_t rows, const msa_seqs *S, bool train,
                       int32_t n_pairs) {
    const int64_t ar = alloc_rows_for(rows);
    al.template take<uint8_t>((size_t)S->n * staged_stride(S->max_len));
    al.template take<int32_t>((size_t)S->n + 1);
    al.template take<int64_t>((size_t)nb + 1);
    al.template take<int32_t>((size_t)rows + 1);
    al.template take<bf16_t>((size_t)ar * kIn);
    for (int l = 1; l < kLayers; ++l) al.template take<bf16_t>((size_t)ar * kW);
    al.template take<float>((size_t)ar * kW);
    al.template take<float>((size_t)nb * kW);
    if (train) {
        al.template take<bf16_t>((size_t)ar * kW);
        al.template take<bf16_t>((size_t)ar * kW);
        al.template take<float>((size_t)nb * kW);
        al.template take<float>(1);
        al.template take<float>((size_t)n_pairs);
        al.template take<float>(wgrad_part_floats(rows));
        al.template take<float>((size_t)std::max(wgrad_chunks(rows), wgrad_chunks0(rows)) * kW);
        al.template take<float>((size_t)n_pairs * kW);
        al.template take<float>((size_t)n_pairs);
        al.template take<int32_t>((size_t)nb + 1);
        al.template take<int32_t>(2 * (size_t)n_pairs);
        al.template take<int64_t>((size_t)nb + 1);
        al.template take<int64_t>((size_t)nb + 1);
    }
}

static int zero(void *p, size_t bytes, hipStream_t s) {
    return fill_i32((int32_t *)p, (int64_t)(bytes / 4), 0, s);
}

// Zero the lead rows and every row from `rows` to the end of the buffer.
static int zero_frame(void *p, size_t row_bytes, int64_t alloc_rows, int64_t rows, hipStream_t s) {
    int rc;
    if ((rc = zero(p, row_bytes * kLead, s))) return rc;
    return zero((uint8_t *)p + row_bytes * (kLead + rows), row_bytes * (alloc_rows - kLead - rows), s);
}

static int cnn_forward(void *P, const ParamLayout &pl, CnnWork &w, hipStream_t s) {
    const Batch &b = w.b;
    const unsigned tiles = (unsigned)((b.rows + kTile - 1) / kTile);
    int rc;
    // the GEMMs write every row in [0, rows); only the lead and tail rows,
    // which spans read but no epilogue writes, need zeros
    if ((rc = zero_frame(w.h[0], kIn * 2, w.alloc_rows, b.rows, s))) return rc;
    for (int l = 1; l < kLayers; ++l)
        if ((rc = zero_frame(w.h[l], kW * 2, w.alloc_rows, b.rows, s))) return rc;
    hipLaunchKernelGGL(k_onehot, dim3((unsigned)std::min(b.nb, 65535)), dim3(256), 0, s, b, w.h[0]);
    ConvArgs c{};
    c.rowseq = b.rowseq;
    c.rows = b.rows;
    for (int l = 0; l < kLayers; ++l) {
        c.X = w.h[l];
        c.Wt = at<bf16_t>(P, pl.wt[l]);
        c.bias = at<float>(P, pl.b[l]);
        if (l == 0) {
            c.out = w.h[1];
            hipLaunchKernelGGL((k_conv<kIn, kdp_of(0), kEpiRelu, kRowTiles0>),
                               dim3((unsigned)((b.rows + conv_tile(kRowTiles0) - 1) / conv_tile(kRowTiles0))),
                               dim3(512), 0, s, c);
        } else if (l < kLayers - 1) {
            c.out = w.h[l + 1];
            hipLaunchKernelGGL((k_conv<kW, kdp_of(1), kEpiRelu>), dim3(tiles), dim3(512), 0, s, c);
        } else {
            c.out = w.z4;
            hipLaunchKernelGGL((k_conv<kW, kdp_of(1), kEpiLinearF32>), dim3(tiles), dim3(512), 0, s, c);
        }
    }
    hipLaunchKernelGGL(k_pool, dim3((unsigned)std::min(b.nb, 65535)), dim3(128), 0, s, b, w.z4, w.E);
    return launch_status();
}

static int cnn_backward(void *P, const ParamLayout &pl, CnnWork &w, hipStream_t s) {
    const Batch &b = w.b;
    const unsigned tiles = (unsigned)((b.rows + kTile - 1) / kTile);
    const unsigned chunks = (unsigned)wgrad_chunks(b.rows);
    const unsigned chunks0 = (unsigned)wgrad_chunks0(b.rows);
    int rc;
    if ((rc = zero_frame(w.dz, kW * 2, w.alloc_rows, b.rows, s))) return rc;
    if ((rc = zero_frame(w.dz2, kW * 2, w.alloc_rows, b.rows, s))) return rc;
    hipLaunchKernelGGL(k_pool_bwd, dim3((unsigned)std::min<int64_t>((b.rows + 7) / 8, 65535)),
                       dim3(128), 0, s, b, w.dE, w.dz);
    bf16_t *dz = w.dz, *dzn = w.dz2;
    for (int l = kLayers - 1; l >= 0; --l) {
        float *gw = at<float>(P, pl.gw[l]);
        float *gb = at<float>(P, pl.gb[l]);
        if (l == 0) {
            hipLaunchKernelGGL((k_conv_wgrad<kIn, kdp_of(0)>), dim3(1, chunks0), dim3(256), 0, s,
                               w.h[0], dz, b.rows, w.part, w.part_b);
            hipLaunchKernelGGL(k_wgrad_reduce, dim3((kW * kdp_of(0) + kW + 255) / 256), dim3(256),
                               0, s, w.part, w.part_b, (int32_t)chunks0, kW * kdp_of(0), gw, gb);
        } else {
            hipLaunchKernelGGL(k_conv_wgrad_h, dim3(2, chunks), dim3(512), 0, s, w.h[l], dz,
                               b.rows, w.part, w.part_b);
            hipLaunchKernelGGL(k_wgrad_reduce, dim3((kW * kdp_of(1) + kW + 255) / 256), dim3(256),
                               0, s, w.part, w.part_b, (int32_t)chunks, kW * kdp_of(1), gw, gb);
        }
        if (l > 0) {
            ConvArgs c{};
            c.X = dz;
            c.Wt = at<bf16_t>(P, pl.wbt[l]);
            c.rowseq = b.rowseq;
            c.rows = b.rows;
            c.out = dzn;
            c.relu_ref = w.h[l];
            hipLaunchKernelGGL((k_conv<kW, kKer * kW, kEpiGradRelu>), dim3(tiles), dim3(512), 0, s, c);
            std::swap(dz, dzn);
        }
    }
    return launch_status();
}

static int setup(const msa_seqs *S, const int32_t *idx, int32_t nb, int64_t total_len, bool train,
                 int32_t n_pairs, void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s,
                 CnnWork &w) {
    int rc;
    const int64_t rows = total_len + 4 * (int64_t)nb;
    Sizer sz;
    cnn_layout(sz, nb, rows, S, train, n_pairs);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    Staged st{cv.take<uint8_t>((size_t)S->n * staged_stride(S->max_len)),
              cv.take<int32_t>((size_t)S->n + 1), staged_stride(S->max_len), S->n};
    w.b.codes = st.codes;
    w.b.len = st.len;
    w.b.stride = st.stride;
    w.b.idx = idx;
    w.b.nb = nb;
    w.b.rows = rows;
    w.b.roff = cv.take<int64_t>((size_t)nb + 1);
    w.b.rowseq = cv.take<int32_t>((size_t)rows + 1);
    w.alloc_rows = alloc_rows_for(rows);
    w.h[0] = cv.take<bf16_t>((size_t)w.alloc_rows * kIn);
    for (int l = 1; l < kLayers; ++l) w.h[l] = cv.take<bf16_t>((size_t)w.alloc_rows * kW);
    w.z4 = cv.take<float>((size_t)w.alloc_rows * kW);
    w.E = cv.take<float>((size_t)nb * kW);
    if (train) {
        w.dz = cv.take<bf16_t>((size_t)w.alloc_rows * kW);
        w.dz2 = cv.take<bf16_t>((size_t)w.alloc_rows * kW);
        w.dE = cv.take<float>((size_t)nb * kW);
        w.loss = cv.take<float>(1);
        w.label = cv.take<float>((size_t)n_pairs);
        w.part = cv.take<float>(wgrad_part_floats(rows));
        w.part_b = cv.take<float>((size_t)std::max(wgrad_chunks(rows), wgrad_chunks0(rows)) * kW);
        w.G = cv.take<float>((size_t)n_pairs * kW);
        w.r2 = cv.take<float>((size_t)n_pairs);
        w.cnt = cv.take<int32_t>((size_t)nb + 1);
        w.list = cv.take<int32_t>(2 * (size_t)n_pairs);
        w.pstart = cv.take<int64_t>((size_t)nb + 1);
        w.pcur = cv.take<int64_t>((size_t)nb + 1);
    }
    if ((rc = stage_set(S, nullptr, st, d_status, s))) return rc;
    hipLaunchKernelGGL(k_frame_lengths, dim3((nb + 256) / 256), dim3(256), 0, s, w.b, d_status);
    if ((rc = exclusive_scan_i64(w.b.roff, (int64_t)nb + 1, s))) return rc;
    hipLaunchKernelGGL(k_frame_rows, dim3((unsigned)std::min(nb, 65535)), dim3(256), 0, s, w.b,
                       d_status);
    return launch_status();
}

static int check_cnn_args(const msa_seqs *S, const int32_t *idx, int32_t nb, int64_t total_len) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (S->sigma > kIn) return MSA_ERANGE;
    if (idx == nullptr || nb < 1 || total_len < 0) return MSA_EINVAL;
    return MSA_OK;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t cnn_param_bytes(void) { return param_layout().bytes; }

int cnn_set_params(void *P, const float *w_host, const float *b_host, hipStream_t s) {
    if (P == nullptr || w_host == nullptr || b_host == nullptr) return MSA_EINVAL;
    const ParamLayout pl = param_layout();
    if (zero(P, pl.bytes / 4 * 4, s)) return MSA_EDEVICE;
    // host layout: per layer W[k][ci][co] then b[co]; device master [co][k*cin + ci]
    size_t wo = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = cin_of(l), kdp = kdp_of(l);
        const int cin_host = l == 0 ? 0 : kW;   // layer 0 host cin = sigma, padded below
        (void)cin_host;
        std::vector<float> m((size_t)kW * kdp, 0.0f);
        for (int k = 0; k < kKer; ++k)
            for (int ci = 0; ci < cin; ++ci)
                for (int co = 0; co < kW; ++co)
                    m[(size_t)co * kdp + k * cin + ci] = w_host[wo + ((size_t)k * cin + ci) * kW + co];
        wo += (size_t)kKer * cin * kW;
        if (hipMemcpy(at<float>(P, pl.w[l]), m.data(), 4 * m.size(), hipMemcpyHostToDevice) ||
            hipMemcpy(at<float>(P, pl.b[l]), b_host + (size_t)l * kW, 4 * kW, hipMemcpyHostToDevice))
            return MSA_EDEVICE;
    }
    hipLaunchKernelGGL(k_pack_weights, dim3(256), dim3(256), 0, s, P, pl);
    return launch_status();
}

int cnn_get_params(const void *Pc, float *w_host, float *b_host, float *gw_host, float *gb_host,
                   hipStream_t s) {
    if (Pc == nullptr) return MSA_EINVAL;
    void *P = (void *)Pc;
    const ParamLayout pl = param_layout();
    if (hipStreamSynchronize(s)) return MSA_EDEVICE;
    size_t wo = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = cin_of(l), kdp = kdp_of(l);
        std::vector<float> m((size_t)kW * kdp), g((size_t)kW * kdp);
        if (hipMemcpy(m.data(), at<float>(P, pl.w[l]), 4 * m.size(), hipMemcpyDeviceToHost) ||
            hipMemcpy(g.data(), at<float>(P, pl.gw[l]), 4 * g.size(), hipMemcpyDeviceToHost))
            return MSA_EDEVICE;
        for (int k = 0; k < kKer; ++k)
            for (int ci = 0; ci < cin; ++ci)
                for (int co = 0; co < kW; ++co) {
                    const size_t h = wo + ((size_t)k * cin + ci) * kW + co;
                    if (w_host) w_host[h] = m[(size_t)co * kdp + k * cin + ci];
                    if (gw_host) gw_host[h] = g[(size_t)co * kdp + k * cin + ci];
                }
        wo += (size_t)kKer * cin * kW;
        if ((b_host && hipMemcpy(b_host + (size_t)l * kW, at<float>(P, pl.b[l]), 4 * kW,
                                 hipMemcpyDeviceToHost)) ||
            (gb_host && hipMemcpy(gb_host + (size_t)l * kW, at<float>(P, pl.gb[l]), 4 * kW,
                                  hipMemcpyDeviceToHost)))
            return MSA_EDEVICE;
    }
    return MSA_OK;
}

size_t cnn_workspace_bytes(const msa_seqs *S, int32_t n_idx, int64_t total_len,
                           int32_t n_pairs) {
    if (check_cnn_args(S, (const int32_t *)16, n_idx, total_len) || n_pairs < 0) return 0;
    Sizer sz;
    cnn_layout(sz, n_idx, total_len + 4 * (int64_t)n_idx, S, n_pairs > 0, n_pairs);
    return sz.total();
}

int cnn_embed(const void *P, const msa_seqs *S, const int32_t *idx, int32_t n_idx,
              int64_t total_len, float *emb, void *ws, size_t ws_bytes, int32_t *d_status,
              hipStream_t s) {
    int rc;
    if ((rc = check_cnn_args(S, idx, n_idx, total_len))) return rc;
    if (P == nullptr || emb == nullptr || ws == nullptr) return MSA_EINVAL;
    const ParamLayout pl = param_layout();
    CnnWork w{};
    if ((rc = setup(S, idx, n_idx, total_len, false, 0, ws, ws_bytes, d_status, s, w))) return rc;
    if ((rc = cnn_forward((void *)P, pl, w, s))) return rc;
    if (hipMemcpyAsync(emb, w.E, 4 * (size_t)n_idx * kW, hipMemcpyDeviceToDevice, s))
        return MSA_EDEVICE;
    return MSA_OK;
}

int cnn_train_step(void *P, const msa_seqs *S, const int32_t *idx, int32_t n_idx,
                   int64_t total_len, const int32_t *pa, const int32_t *pb, const uint16_t *dist,
                   int32_t n_pairs, float lr, int32_t step, float *loss, void *ws,
                   size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_cnn_args(S, idx, n_idx, total_len))) return rc;
    if (P == nullptr || pa == nullptr || pb == nullptr || dist == nullptr || n_pairs < 1 ||
        ws == nullptr || step < 1)
        return MSA_EINVAL;
    const ParamLayout pl = param_layout();
    CnnWork w{};
    if ((rc = setup(S, idx, n_idx, total_len, true, n_pairs, ws, ws_bytes, d_status, s, w)))
        return rc;
    hipLaunchKernelGGL(k_labels, dim3((n_pairs + 255) / 256), dim3(256), 0, s, w.b, pa, pb, dist,
                       n_pairs, w.label);
    if ((rc = cnn_forward(P, pl, w, s))) return rc;
    // pair loss and embedding gradient, summed in fixed orders
    hipLaunchKernelGGL(k_pair_loss, dim3(n_pairs), dim3(64), 0, s, w.E, pa, pb, w.label, n_pairs,
                       w.G, w.r2);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, s, w.r2, n_pairs, w.loss);
    if ((rc = fill_i32(w.cnt, (int64_t)n_idx + 1, 0, s))) return rc;
    const unsigned pg = (unsigned)std::min((n_pairs + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pair_count, dim3(pg), dim3(256), 0, s, pa, pb, n_pairs, w.cnt);
    hipLaunchKernelGGL(k_widen_i32, dim3((n_idx + 1 + 255) / 256), dim3(256), 0, s, w.cnt,
                       (int64_t)n_idx + 1, w.pstart);
    if ((rc = exclusive_scan_i64(w.pstart, (int64_t)n_idx + 1, s))) return rc;
    if (hipMemcpyAsync(w.pcur, w.pstart, sizeof(int64_t) * ((size_t)n_idx + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MSA_EDEVICE;
    hipLaunchKernelGGL(k_pair_fill, dim3(pg), dim3(256), 0, s, pa, pb, n_pairs, w.pcur, w.list);
    hipLaunchKernelGGL(k_seq_grad, dim3((unsigned)std::min(n_idx, 65535)), dim3(64), 0, s,
                       w.pstart, w.list, w.G, n_idx, w.dE);
    if ((rc = cnn_backward(P, pl, w, s))) return rc;
    if (lr > 0.0f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
        for (int l = 0; l < kLayers; ++l) {
            hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, s, at<float>(P, pl.w[l]),
                               at<float>(P, pl.gw[l]), at<float>(P, pl.mw[l]),
                               at<float>(P, pl.vw[l]), (int64_t)kW * kdp_of(l), lr, b1, b2, eps,
                               c1, c2);
            hipLaunchKernelGGL(k_adam, dim3(1), dim3(128), 0, s, at<float>(P, pl.b[l]),
                               at<float>(P, pl.gb[l]), at<float>(P, pl.mb[l]),
                               at<float>(P, pl.vb[l]), (int64_t)kW, lr, b1, b2, eps, c1, c2);
        }
        hipLaunchKernelGGL(k_pack_weights, dim3(256), dim3(256), 0, s, P, pl);
    }
    if (loss && hipMemcpyAsync(loss, w.loss, 4, hipMemcpyDeviceToDevice, s)) return MSA_EDEVICE;
    return launch_status();
}

}  // extern "C"
