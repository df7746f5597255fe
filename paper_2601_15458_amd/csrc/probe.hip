// Machine-rate probes: the measured counterparts of the vendor peaks that the
// roofline figures of the other kernels are priced against.
//
//   k_probe_valu   independent 32-bit xor/add chains (the instruction class
//                  of the bit-vector recurrences)
//   k_probe_mfma   independent accumulator chains of one MFMA shape (the
//                  bf16 and int8 shapes the CNN and the pair-distance
//                  kernels use, plus their 32x32 twins)
//   k_probe_copy   a streaming 16-byte-per-lane device copy (HBM)
//
// Each entry point reports the work one launch performs, so the caller only
// has to time the launch.
//
// This file is compiled with the MFMA VGPR form (-amdgpu-mfma-vgpr-form):
// with accumulators in AGPRs the register allocator rotates the 4-register
// 16x16 accumulators through accvgpr copies on every loop trip, and the
// loop would measure those copies rather than the matrix unit.
#include "common.hpp"

namespace msadp {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kValuPairs = 8;       // independent (a, b) chains per lane
constexpr int kValuUnroll = 8;      // chain steps per loop trip
// One chain step is two VALU instructions: a ^= b, then b += a.
constexpr int64_t kValuOpsPerTrip = 2 * kValuPairs * kValuUnroll;

__global__ __launch_bounds__(kProbeThreads) void k_probe_valu(int32_t iters, uint32_t *sink) {
    const uint32_t t = blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t a[kValuPairs], b[kValuPairs];
#pragma unroll
    for (int c = 0; c < kValuPairs; ++c) {
        a[c] = t * (2u * c + 1u);
        b[c] = t ^ (0x9E3779B9u * (c + 1u));
    }
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kValuUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kValuPairs; ++c) {
                a[c] ^= b[c];
                b[c] += a[c];
            }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kValuPairs; ++c) r ^= a[c] + b[c];
    sink[t] = r;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 pbf16x8;
typedef float pf32x4 __attribute__((ext_vector_type(4)));
typedef float pf32x16 __attribute__((ext_vector_type(16)));
typedef int32_t pi32x4 __attribute__((ext_vector_type(4)));
typedef int32_t pi32x16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaChains = 8;      // independent accumulators per wavefront
constexpr int kMfmaUnroll = 2;      // instructions per accumulator per loop trip

// One MFMA per call; the result feeds the same accumulator on the next trip.
template <int Kind>
struct MfmaShape;
template <>
struct MfmaShape<MSA_PROBE_MFMA_BF16_16X16X32> {
    typedef pbf16x8 In;
    typedef pf32x4 Acc;
    static constexpr int64_t kOps = 2LL * 16 * 16 * 32;
    static __device__ __forceinline__ Acc step(In x, In y, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
};
template <>
struct MfmaShape<MSA_PROBE_MFMA_BF16_32X32X16> {
    typedef pbf16x8 In;
    typedef pf32x16 Acc;
    static constexpr int64_t kOps = 2LL * 32 * 32 * 16;
    static __device__ __forceinline__ Acc step(In x, In y, Acc c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
    }
};
template <>
struct MfmaShape<MSA_PROBE_MFMA_I8_16X16X64> {
    typedef pi32x4 In;
    typedef pi32x4 Acc;
    static constexpr int64_t kOps = 2LL * 16 * 16 * 64;
    static __device__ __forceinline__ Acc step(In x, In y, Acc c) {
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, c, 0, 0, 0);
    }
};
template <>
struct MfmaShape<MSA_PROBE_MFMA_I8_32X32X32> {
    typedef pi32x4 In;
    typedef pi32x16 Acc;
    static constexpr int64_t kOps = 2LL * 32 * 32 * 32;
    static __device__ __forceinline__ Acc step(In x, In y, Acc c) {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(x, y, c, 0, 0, 0);
    }
};

template <int Kind>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int32_t iters, uint32_t *sink) {
    typedef MfmaShape<Kind> S;
    const uint32_t t = blockIdx.x * kProbeThreads + threadIdx.x;
    typename S::In x, y;
    // Operands depend on the lane so that nothing folds; their values do not
    // matter (the rate of a matrix instruction does not depend on its data).
    uint32_t wx[4], wy[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        wx[q] = (t * (2u * q + 1u)) & 0x3F803F80u;
        wy[q] = (t ^ (0x01010101u * q)) & 0x3F803F80u;
    }
    x = __builtin_bit_cast(typename S::In, wx);
    y = __builtin_bit_cast(typename S::In, wy);
    typename S::Acc acc[kMfmaChains];
#pragma unroll
    for (int c = 0; c < kMfmaChains; ++c) acc[c] = typename S::Acc{};
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kMfmaUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kMfmaChains; ++c) acc[c] = S::step(x, y, acc[c]);
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kMfmaChains; ++c) r ^= __builtin_bit_cast(uint32_t, acc[c][0]);
    sink[t] = r;
}

typedef uint32_t pu32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const pu32x4 *__restrict__ src,
                                                              pu32x4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    // Four independent 16-byte loads in flight per lane per trip.
    for (; i + 3 * stride < n; i += 4 * stride) {
        pu32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

template <int Kind>
int launch_mfma(int32_t blocks, int32_t iters, uint32_t *sink, int64_t *ops, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_mfma<Kind>, dim3(blocks), dim3(kProbeThreads), 0, s, iters, sink);
    if (hipGetLastError() != hipSuccess) return MSA_EDEVICE;
    *ops = MfmaShape<Kind>::kOps * kMfmaChains * kMfmaUnroll * (int64_t)iters * (blocks * (kProbeThreads / kWave));
    return MSA_OK;
}

}  // namespace
}  // namespace msadp

using namespace msadp;

extern "C" int msa_probe_valu(int32_t blocks, int32_t iters, uint32_t *sink, int64_t *ops,
                              hipStream_t s) {
    if (blocks <= 0 || iters <= 0 || sink == nullptr || ops == nullptr) return MSA_EINVAL;
    hipLaunchKernelGGL(k_probe_valu, dim3(blocks), dim3(kProbeThreads), 0, s, iters, sink);
    if (hipGetLastError() != hipSuccess) return MSA_EDEVICE;
    *ops = kValuOpsPerTrip * (int64_t)iters * blocks * kProbeThreads;
    return MSA_OK;
}

extern "C" int msa_probe_mfma(int32_t kind, int32_t blocks, int32_t iters, uint32_t *sink,
                              int64_t *ops, hipStream_t s) {
    if (blocks <= 0 || iters <= 0 || sink == nullptr || ops == nullptr) return MSA_EINVAL;
    switch (kind) {
    case MSA_PROBE_MFMA_BF16_16X16X32:
        return launch_mfma<MSA_PROBE_MFMA_BF16_16X16X32>(blocks, iters, sink, ops, s);
    case MSA_PROBE_MFMA_BF16_32X32X16:
        return launch_mfma<MSA_PROBE_MFMA_BF16_32X32X16>(blocks, iters, sink, ops, s);
    case MSA_PROBE_MFMA_I8_16X16X64:
        return launch_mfma<MSA_PROBE_MFMA_I8_16X16X64>(blocks, iters, sink, ops, s);
    case MSA_PROBE_MFMA_I8_32X32X32:
        return launch_mfma<MSA_PROBE_MFMA_I8_32X32X32>(blocks, iters, sink, ops, s);
    default:
        return MSA_EINVAL;
    }
}

extern "C" int msa_probe_copy(const void *src, void *dst, size_t bytes, int32_t blocks,
                              hipStream_t s) {
    if (src == nullptr || dst == nullptr || blocks <= 0) return MSA_EINVAL;
    if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0) return MSA_EINVAL;
    if (bytes == 0) return MSA_OK;
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(kProbeThreads), 0, s,
                       (const pu32x4 *)src, (pu32x4 *)dst, (int64_t)(bytes / 16));
    return hipGetLastError() == hipSuccess ? MSA_OK : MSA_EDEVICE;
}
