// Alignment-quality metrics of Sec. 2.3 (and the width and stretch columns of
// Table 2) over a finished alignment: rows x width symbol codes, one code
// reserved for the gap.
//
//   1. k_qual_planes: each row becomes bit planes over 32-column words, one
//      gap plane and NB symbol planes (bit b of the code), stored word-major
//      ([plane][word][row]) so that the lanes of a wavefront, which take
//      consecutive rows, read consecutive words.  Columns past the width are
//      gaps with code 0 in every row, so they count as equal gap-gap columns;
//      the row dimension is padded to a multiple of 64 with rows of such
//      columns, so no load needs a bounds check.
//   2. k_qual_tri / k_qual_list: per pair of rows and word, the columns that
//      differ are the OR over the symbol planes of x ^ y (two gaps have equal
//      codes), the columns with a residue in both rows are ~(gx | gy), and
//      three population counts add the Hamming distance, the aligned columns
//      and the aligned columns that differ.  The triangle variant gives a
//      wavefront 16 rows i (staged in LDS, read as broadcasts) against 64
//      rows j (one per lane), so each loaded word of row j serves 16 pairs.
//   3. k_qual_reduce + k_qual_final: the per-pair ratios (p-score over the
//      aligned columns, Hamming over Levenshtein) and per-row gap fractions
//      summed in a fixed order (fixed grid, tree reduction per block, block
//      partials folded in a fixed pattern), so repeated calls agree bit for bit.
#include <algorithm>

#include "common.hpp"

namespace msadp {
namespace {

constexpr int kQualThreads = 256;
constexpr int kQualRows = 16;         // rows i per wavefront item (triangle)
constexpr int kQualGroups = kQualRows / 4;   // 16-byte groups of 4 rows
constexpr int kReduceBlocks = 2048;   // enough wavefronts to hide load latency
constexpr int kMaxPlanes = 6;         // codes up to 63

inline int planes_of(int32_t gap_code) {
    int nb = 1;
    while ((1 << nb) <= gap_code) ++nb;
    return nb;
}

inline int64_t words_of(int32_t width) { return ((int64_t)width + 31) / 32; }

inline int64_t rows_pad_of(int32_t rows) { return ((int64_t)rows + 63) / 64 * 64; }

struct QualArgs {
    const uint8_t *msa;
    int32_t rows, width, gap;
    int64_t words;
    int64_t rows_pad;         // rows rounded up to a multiple of 64
    uint32_t *planes;         // [1 + NB][words][rows_pad]
    int32_t *st;
};

__device__ __forceinline__ const uint32_t *plane(const QualArgs &a, int b) {
    return a.planes + (int64_t)b * a.words * a.rows_pad;
}

// One wavefront per (row, 64 columns): lane l reads column 64 k + l (one
// coalesced 64-byte load), and one ballot per plane gives two words.
__global__ void __launch_bounds__(kQualThreads) k_qual_planes(QualArgs a, int nb) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t chunks = (a.words + 1) / 2;             // 64-column chunks per row
    const int64_t total = chunks * a.rows_pad;
    const int64_t wave = (int64_t)blockIdx.x * (kQualThreads / kWave) +
                         (int64_t)uniform(threadIdx.x / kWave);
    const int64_t nwaves = (int64_t)gridDim.x * (kQualThreads / kWave);
    for (int64_t t = wave; t < total; t += nwaves) {
        const int64_t k = t / a.rows_pad, r = t % a.rows_pad;    // uniform
        const int64_t col = 64 * k + lane;
        const bool in = r < a.rows && col < a.width;
        const uint32_t code = in ? a.msa[r * (int64_t)a.width + col] : 0u;
        if (in && code > (uint32_t)a.gap) set_status(a.st, MSA_DS_SYMBOL);
        const uint64_t g = __ballot(!in || code == (uint32_t)a.gap);
        const int64_t o = 2 * k * a.rows_pad + r;            // word 2k of row r
        const bool second = 2 * k + 1 < a.words;
        if (lane == 0) a.planes[o] = (uint32_t)g;
        if (lane == 1 && second) a.planes[o + a.rows_pad] = (uint32_t)(g >> 32);
        for (int b = 0; b < nb; ++b) {
            const uint64_t m = __ballot((code >> b) & 1u);
            uint32_t *pb = a.planes + (int64_t)(b + 1) * a.words * a.rows_pad + o;
            if (lane == 0) pb[0] = (uint32_t)m;
            if (lane == 1 && second) pb[a.rows_pad] = (uint32_t)(m >> 32);
        }
    }
}

struct PairOut {
    int32_t *hamming, *aligned, *mismatched;
};

// Counts of one word of rows x and y: differ, both residues, differing residues.
template <int NB>
__device__ __forceinline__ void word_counts(uint32_t gx, const uint32_t (&sx)[NB], uint32_t gy,
                                            const uint32_t (&sy)[NB], int32_t &h, int32_t &al,
                                            int32_t &mm) {
    uint32_t diff = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) diff |= sx[b] ^ sy[b];
    const uint32_t both = ~(gx | gy);
    h += __builtin_popcount(diff);
    al += __builtin_popcount(both);
    mm += __builtin_popcount(diff & both);
}

// All pairs i < j of the rows, stored at the condensed index
// i * rows - i (i + 1) / 2 + (j - i - 1).  Item = (16 rows i, 64 rows j).
constexpr int kQualChunk = 64;        // words of the rows i staged in LDS at a time

template <int NB>
__global__ void __launch_bounds__(kQualThreads) k_qual_tri(QualArgs a,
                                                           const uint32_t *__restrict__ pl,
                                                           PairOut o) {
    // The rows i of a wavefront's item, kQualChunk words at a time, staged
    // in the wavefront's own LDS slice: [plane][word][group] -> 4 rows'
    // words (consecutive in the word-major layout: one 16-byte load each).
    __shared__ uint4 si[kQualThreads / kWave][NB + 1][kQualChunk][kQualGroups];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t wave = (int64_t)blockIdx.x * (kQualThreads / kWave) + (int64_t)uniform(wv);
    const int64_t nwaves = (int64_t)gridDim.x * (kQualThreads / kWave);
    const int64_t ni = (a.rows + kQualRows - 1) / kQualRows, nj = (a.rows + kWave - 1) / kWave;
    const int64_t n = a.rows;
    const int64_t ps = a.words * a.rows_pad;              // plane stride
    for (int64_t it = wave; it < ni * nj; it += nwaves) {
        const int64_t i0 = (it / nj) * kQualRows, j0 = (it % nj) * kWave;   // uniform
        if (j0 + kWave - 1 <= i0) continue;              // no j above these rows i (uniform)
        const int64_t j = j0 + lane;                     // < rows_pad
        int32_t h[kQualRows] = {}, al[kQualRows] = {}, mm[kQualRows] = {};
        const uint32_t *pj = pl + j;
        for (int64_t w0 = 0; w0 < a.words; w0 += kQualChunk) {
            const int cw = (int)(a.words - w0 < kQualChunk ? a.words - w0 : kQualChunk);
            // reads of the previous chunk are done before it is overwritten
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int e = lane; e < (NB + 1) * cw * kQualGroups; e += kWave) {
                const int q = e % kQualGroups, bw = e / kQualGroups;
                const int b = bw / cw, w = bw % cw;      // i0 + 15 < rows_pad
                si[wv][b][w][q] =
                    *(const uint4 *)(pl + b * ps + (w0 + w) * a.rows_pad + i0 + 4 * q);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
            for (int w = 0; w < cw; ++w, pj += a.rows_pad) {
                const uint32_t gy = pj[0];
                uint32_t sy[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) sy[b] = pj[(b + 1) * ps];
#pragma unroll
                for (int q = 0; q < kQualGroups; ++q) {
                    const uint4 g4 = si[wv][0][w][q];       // same address in every lane
                    uint4 s4[NB];
#pragma unroll
                    for (int b = 0; b < NB; ++b) s4[b] = si[wv][b + 1][w][q];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int r = 4 * q + k;
                        const uint32_t gx = k == 0 ? g4.x : k == 1 ? g4.y : k == 2 ? g4.z : g4.w;
                        uint32_t sx[NB];
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            sx[b] = k == 0 ? s4[b].x : k == 1 ? s4[b].y : k == 2 ? s4[b].z : s4[b].w;
                        word_counts<NB>(gx, sx, gy, sy, h[r], al[r], mm[r]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kQualRows; ++r) {
            const int64_t i = i0 + r;
            if (i < n && j < n && i < j) {
                const int64_t c = i * n - i * (i + 1) / 2 + (j - i - 1);
                o.hamming[c] = h[r];
                o.aligned[c] = al[r];
                o.mismatched[c] = mm[r];
            }
        }
    }
}

// Explicit pairs (ia[p], ib[p]), one per thread.
template <int NB>
__global__ void __launch_bounds__(kQualThreads) k_qual_list(QualArgs a, const int32_t *ia,
                                                            const int32_t *ib, int64_t n_pairs,
                                                            PairOut o) {
    const int64_t n = a.rows;
    for (int64_t p = (int64_t)blockIdx.x * kQualThreads + threadIdx.x; p < n_pairs;
         p += (int64_t)gridDim.x * kQualThreads) {
        int64_t x = ia[p], y = ib[p];
        const bool ok = x >= 0 && x < n && y >= 0 && y < n;
        if (!ok) {
            set_status(a.st, MSA_DS_INDEX);
            x = y = 0;
        }
        int32_t h = 0, al = 0, mm = 0;
        for (int64_t w = 0; w < a.words; ++w) {
            const int64_t base = w * a.rows_pad;
            uint32_t sx[NB], sy[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                sx[b] = plane(a, b + 1)[base + x];
                sy[b] = plane(a, b + 1)[base + y];
            }
            word_counts<NB>(plane(a, 0)[base + x], sx, plane(a, 0)[base + y], sy, h, al, mm);
        }
        o.hamming[p] = h;
        o.aligned[p] = al;
        o.mismatched[p] = mm;
    }
}

// Per-block partials: [0] sum of gap fractions, [1] p sum, [2] p min,
// [3] p max, [4] p count, [5] distortion sum, [6] distortion count.
constexpr int kPart = 7;

__global__ void __launch_bounds__(kQualThreads) k_qual_reduce(QualArgs a, const int32_t *hamming,
                                                              const int32_t *aligned,
                                                              const int32_t *mismatched,
                                                              const uint16_t *lev, int64_t n_pairs,
                                                              double *part) {
    __shared__ double red[kPart][kQualThreads];
    const int t = threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kQualThreads;
    double v[kPart] = {0.0, 0.0, __builtin_inf(), -__builtin_inf(), 0.0, 0.0, 0.0};
    // gap fraction of each row, from the gap plane (padding columns removed)
    const int32_t pad = (int32_t)(a.words * 32 - a.width);
    for (int64_t r = (int64_t)blockIdx.x * kQualThreads + t; a.width > 0 && r < a.rows;
         r += stride) {
        int32_t g = 0;
        for (int64_t w = 0; w < a.words; ++w)
            g += __builtin_popcount(plane(a, 0)[w * a.rows_pad + r]);
        v[0] += (double)(g - pad) / (double)a.width;
    }
    for (int64_t p = (int64_t)blockIdx.x * kQualThreads + t; p < n_pairs; p += stride) {
        const int32_t al = aligned[p];
        if (al > 0) {
            const double q = (double)mismatched[p] / (double)al;
            v[1] += q;
            v[2] = q < v[2] ? q : v[2];
            v[3] = q > v[3] ? q : v[3];
            v[4] += 1.0;
        }
        const int32_t d = lev != nullptr ? (int32_t)lev[p] : 0;
        if (d > 0) {
            v[5] += (double)hamming[p] / (double)d;
            v[6] += 1.0;
        }
    }
#pragma unroll
    for (int k = 0; k < kPart; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int off = kQualThreads / 2; off >= 1; off >>= 1) {
        if (t < off) {
#pragma unroll
            for (int k = 0; k < kPart; ++k) {
                const double x = red[k][t], y = red[k][t + off];
                red[k][t] = k == 2 ? (y < x ? y : x) : k == 3 ? (y > x ? y : x) : x + y;
            }
        }
        __syncthreads();
    }
    if (t < kPart) part[(int64_t)blockIdx.x * kPart + t] = red[t][0];
}

// out: pct_gaps, p_min, p_avg, p_max, distortion, stretch, n_p_pairs, n_d_pairs.
// Combine two partial tuples (sums add, minimum, maximum).
__device__ __forceinline__ void combine(double (&v)[kPart], const double *q) {
    v[0] += q[0];
    v[1] += q[1];
    v[2] = q[2] < v[2] ? q[2] : v[2];
    v[3] = q[3] > v[3] ? q[3] : v[3];
    v[4] += q[4];
    v[5] += q[5];
    v[6] += q[6];
}

// One workgroup: thread t folds block partials t, t + 256, ... in order, then
// a fixed tree over the threads; the result does not depend on timing.
__global__ void __launch_bounds__(kQualThreads) k_qual_final(const double *part, int nblocks,
                                                             int32_t rows, int32_t width,
                                                             int32_t max_len, double *out) {
    __shared__ double red[kQualThreads][kPart];
    const int t = threadIdx.x;
    double v[kPart] = {0.0, 0.0, __builtin_inf(), -__builtin_inf(), 0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += kQualThreads) combine(v, part + (int64_t)b * kPart);
#pragma unroll
    for (int k = 0; k < kPart; ++k) red[t][k] = v[k];
    __syncthreads();
    for (int off = kQualThreads / 2; off >= 1; off >>= 1) {
        if (t < off) {
            double w[kPart];
#pragma unroll
            for (int k = 0; k < kPart; ++k) w[k] = red[t][k];
            combine(w, red[t + off]);
#pragma unroll
            for (int k = 0; k < kPart; ++k) red[t][k] = w[k];
        }
        __syncthreads();
    }
    if (t != 0) return;
#pragma unroll
    for (int k = 0; k < kPart; ++k) v[k] = red[0][k];
    const bool anyp = v[4] > 0.0, anyd = v[6] > 0.0;
    out[0] = rows > 0 && width > 0 ? 100.0 * v[0] / (double)rows : 0.0;
    out[1] = anyp ? v[2] : 0.0;
    out[2] = anyp ? v[1] / v[4] : 0.0;
    out[3] = anyp ? v[3] : 0.0;
    out[4] = anyd ? v[5] / v[6] : 0.0;
    out[5] = max_len > 0 ? (double)width / (double)max_len : 0.0;
    out[6] = v[4];
    out[7] = v[6];
}

size_t planes_bytes(int32_t rows, int32_t width, int32_t gap) {
    return (size_t)(1 + planes_of(gap)) * (size_t)words_of(width) * (size_t)rows_pad_of(rows) * 4;
}

int check_msa(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap) {
    if (rows < 0 || width < 0 || gap < 0 || gap >= (1 << kMaxPlanes)) return MSA_EINVAL;
    if (msa == nullptr && (int64_t)rows * width > 0) return MSA_EINVAL;
    return MSA_OK;
}

template <int NB>
void launch_pairs(const QualArgs &a, const int32_t *ia, const int32_t *ib, int64_t n_pairs,
                  PairOut o, hipStream_t s) {
    const unsigned grid = (unsigned)std::max(1, device_cus() * 16);
    if (ia == nullptr)
        hipLaunchKernelGGL(k_qual_tri<NB>, dim3(grid), dim3(kQualThreads), 0, s, a,
                           (const uint32_t *)a.planes, o);
    else
        hipLaunchKernelGGL(k_qual_list<NB>, dim3(grid), dim3(kQualThreads), 0, s, a, ia, ib,
                           n_pairs, o);
}

}  // namespace
}  // namespace msadp

using namespace msadp;

extern "C" size_t msa_quality_workspace_bytes(int32_t rows, int32_t width, int32_t gap_code) {
    if (rows < 0 || width < 0 || gap_code < 0 || gap_code >= (1 << kMaxPlanes)) return 0;
    Sizer sz;
    sz.take<uint32_t>(planes_bytes(rows, width, gap_code) / 4);
    sz.take<double>((size_t)kReduceBlocks * kPart);
    return sz.total();
}

static int qual_setup(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap_code, void *ws,
                      size_t ws_bytes, int32_t *d_status, hipStream_t s, QualArgs &a,
                      double **part) {
    if (ws == nullptr || ws_bytes < msa_quality_workspace_bytes(rows, width, gap_code))
        return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    a.msa = msa;
    a.rows = rows;
    a.width = width;
    a.gap = gap_code;
    a.words = words_of(width);
    a.rows_pad = rows_pad_of(rows);
    a.planes = cv.take<uint32_t>(planes_bytes(rows, width, gap_code) / 4);
    a.st = d_status;
    *part = cv.take<double>((size_t)kReduceBlocks * kPart);
    const int64_t tasks = (a.words + 1) / 2 * a.rows_pad;  // one wavefront each
    if (tasks > 0) {
        const int64_t per_block = kQualThreads / kWave;
        const unsigned grid = (unsigned)std::min<int64_t>((tasks + per_block - 1) / per_block,
                                                          (int64_t)device_cus() * 64);
        hipLaunchKernelGGL(k_qual_planes, dim3(grid), dim3(kQualThreads), 0, s, a,
                           planes_of(gap_code));
    }
    return MSA_OK;
}

extern "C" int msa_pair_counts(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap_code,
                               const int32_t *ia, const int32_t *ib, int64_t n_pairs,
                               int32_t *hamming, int32_t *aligned, int32_t *mismatched, void *ws,
                               size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    int rc = check_msa(msa, rows, width, gap_code);
    if (rc != MSA_OK) return rc;
    if (n_pairs < 0 || (ia == nullptr) != (ib == nullptr)) return MSA_EINVAL;
    if (ia == nullptr && n_pairs != (int64_t)rows * (rows - 1) / 2) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (rows == 0) return MSA_EINVAL;                    // a pair needs rows
    if (hamming == nullptr || aligned == nullptr || mismatched == nullptr) return MSA_EINVAL;
    QualArgs a{};
    double *part = nullptr;
    if ((rc = qual_setup(msa, rows, width, gap_code, ws, ws_bytes, d_status, s, a, &part)))
        return rc;
    const PairOut o{hamming, aligned, mismatched};
    switch (planes_of(gap_code)) {
        case 1: launch_pairs<1>(a, ia, ib, n_pairs, o, s); break;
        case 2: launch_pairs<2>(a, ia, ib, n_pairs, o, s); break;
        case 3: launch_pairs<3>(a, ia, ib, n_pairs, o, s); break;
        case 4: launch_pairs<4>(a, ia, ib, n_pairs, o, s); break;
        case 5: launch_pairs<5>(a, ia, ib, n_pairs, o, s); break;
        default: launch_pairs<6>(a, ia, ib, n_pairs, o, s); break;
    }
    return launch_status();
}

extern "C" int msa_quality(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap_code,
                           int32_t max_len, const int32_t *hamming, const int32_t *aligned,
                           const int32_t *mismatched, const uint16_t *lev, int64_t n_pairs,
                           double *out, void *ws, size_t ws_bytes, int32_t *d_status,
                           hipStream_t s) {
    int rc = check_msa(msa, rows, width, gap_code);
    if (rc != MSA_OK) return rc;
    if (n_pairs < 0 || out == nullptr || max_len < 0) return MSA_EINVAL;
    if (n_pairs > 0 && (hamming == nullptr || aligned == nullptr || mismatched == nullptr))
        return MSA_EINVAL;
    QualArgs a{};
    double *part = nullptr;
    if ((rc = qual_setup(msa, rows, width, gap_code, ws, ws_bytes, d_status, s, a, &part)))
        return rc;
    hipLaunchKernelGGL(k_qual_reduce, dim3(kReduceBlocks), dim3(kQualThreads), 0, s, a, hamming,
                       aligned, mismatched, lev, n_pairs, part);
    hipLaunchKernelGGL(k_qual_final, dim3(1), dim3(kQualThreads), 0, s, (const double *)part,
                       kReduceBlocks, rows, width, max_len, out);
    return launch_status();
}
