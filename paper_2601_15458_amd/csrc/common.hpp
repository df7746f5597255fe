// Internal helpers shared by the msadp device library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <atomic>

#include "msadp.h"

namespace msadp {

constexpr int kWave = 64;

// ---------------------------------------------------------------- bit ops
// gfx950 has a three-input bitwise instruction (v_bitop3_b32) whose 8-bit
// immediate is the truth table of f(S0, S1, S2) indexed by (S0 S1 S2) read
// as a 3-bit number.  LUT(expr) builds that table by evaluating the
// expression on the three canonical operand patterns 0xF0, 0xCC, 0xAA.
#define MSADP_LUT(expr) \
    ((uint8_t)([](uint32_t A, uint32_t B, uint32_t C) { return (expr); }(0xF0u, 0xCCu, 0xAAu)))

template <uint8_t L>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, L);
}

// (hi:lo) >> 31, low word: (hi << 1) | (lo >> 31)
__device__ __forceinline__ uint32_t shl1_carry(uint32_t hi, uint32_t lo) {
    return __builtin_amdgcn_alignbit(hi, lo, 31);
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) {
    if (st != nullptr) atomicCAS(st, 0, code);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// --------------------------------------------------------- staged sequences
// Every entry point first copies its input sequences into this layout: one
// row of `stride` bytes per sequence (one byte per symbol, zero padded), so
// kernels read aligned words regardless of the caller's offsets or packing.
struct Staged {
    uint8_t *codes;     // n * stride bytes
    int32_t *len;       // n lengths
    int64_t stride;     // bytes per row, multiple of 16, >= max_len + 16
    int32_t n;
};

inline int64_t staged_stride(int32_t max_len) { return ((int64_t)max_len + 16 + 15) / 16 * 16; }

// Launch order for batches that give each pair a workgroup of its own and
// hold about one such workgroup per CU: longest first (the largest m * n),
// so that the long pairs start at once and the short ones fill the CUs that
// free up (list scheduling, longest processing time first).  order[r] = the
// pair of rank r; equal sizes keep their index order; pairs with an index
// out of range count as empty (the fill reports them).  O(P^2) work, used
// for batches of at most kLptMaxPairs pairs (beyond that many pairs per CU
// even out and the index order is kept).
constexpr int64_t kLptMaxPairs = 8192;
constexpr int kLptTile = 1024;

__device__ __forceinline__ int64_t pair_cells(const Staged &A, const Staged &B,
                                              const int32_t *ia, const int32_t *ib, int64_t q) {
    const int32_t x = ia[q], y = ib[q];
    if (x < 0 || x >= A.n || y < 0 || y >= B.n) return 0;
    return (int64_t)A.len[x] * B.len[y];
}

template <int kTile>
__global__ void __launch_bounds__(256) k_lpt_order(Staged A, Staged B, const int32_t *ia,
                                                   const int32_t *ib, int64_t P,
                                                   int32_t *order) {
    __shared__ int64_t keys[kTile];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t kp = p < P ? pair_cells(A, B, ia, ib, p) : 0;
    int64_t rank = 0;
    for (int64_t base = 0; base < P; base += kTile) {
        const int64_t cnt = P - base < kTile ? P - base : kTile;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < cnt; i += 256) keys[i] = pair_cells(A, B, ia, ib, base + i);
        __syncthreads();
        for (int64_t i = 0; i < cnt; ++i) {
            const int64_t kq = keys[i];
            rank += (kq > kp || (kq == kp && base + i < p)) ? 1 : 0;
        }
    }
    if (p < P) order[rank] = (int32_t)p;
}

// ----------------------------------------------------------- host helpers
// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carve {
    uintptr_t base, cur, end;
    explicit Carve(void *p, size_t bytes)
        : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + bytes) {}
    template <class T>
    T *take(size_t count) {
        cur = (cur + 255) / 256 * 256;
        T *p = (T *)cur;
        cur += count * sizeof(T);
        return p;
    }
    size_t used() const { return (size_t)(cur - base) + 256; }
    bool ok() const { return cur <= end; }
};

// Size-only twin of Carve for the workspace queries.
struct Sizer {
    size_t cur = 0;
    template <class T>
    T *take(size_t count) {
        cur = (cur + 255) / 256 * 256;
        cur += count * sizeof(T);
        return nullptr;
    }
    size_t total() const { return cur + 256; }
};

int check_seqs(const msa_seqs *S);
// The current device (0 when it cannot be read) and its compute units.
constexpr int kMaxDevices = 64;
int current_device();
int device_cus();
int launch_status();

// staging (stage.hip)
int stage_set(const msa_seqs *S, const int32_t *order, Staged out, int32_t *d_status,
              hipStream_t s);
int sort_by_length(const msa_seqs *S, int32_t *len_tmp, int32_t *hist, int32_t *order,
                   int32_t *d_status, hipStream_t s);
int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
int exclusive_scan_i64(int64_t *data, int64_t n, hipStream_t s);
// lev_batch with a forced pair-list layout (1 = one pattern per lane, 64 =
// shared patterns; 0 = the tuning table or the default; -1 = the default
// layout and word class, tuning table not read) (lev.hip).
int lev_batch_impl(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                   int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes,
                   int32_t *d_status, hipStream_t s, int forced);
// Workspace of lev_batch_impl; untuned: for forced == -1 only.
size_t lev_batch_ws_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs, bool untuned);
// The tuning table's value for (kind, sigma, bin), or `fallback` (tune.hip).
int tuned_value(int kind, int sigma, int bin, int fallback);
// K disjoint root clusters for a tree build: cluster f holds the input
// indices mem[start[f] .. start[f+1]), m = start[K] in all (tree.hip).
struct Forest {
    int32_t K;
    const int32_t *mem;
    const int64_t *start;
    int64_t m;
};
int tree_build_forest(const msa_seqs *S, const Forest &fr, const msa_tree *T, int32_t *n_nodes,
                      void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

}  // namespace msadp
