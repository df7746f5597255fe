// Staging, length binning and small device utilities.
//
// Encode/pack step of the path: the caller's CSR sequences (one byte per
// symbol, or four 2-bit symbols per byte) are copied into fixed-stride rows
// of one byte per symbol, validated on the way (codes < sigma, lengths in
// [0, max_len]).  For the all-pairs batch the rows are first ordered by
// length (a counting sort on the device) so that every wavefront later gets
// texts of nearly equal length.
#include "common.hpp"

namespace msadp {

int launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MSA_OK : MSA_EDEVICE;
}

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    return dev;
}

// Cached per device; concurrent first calls compute the same value.
int device_cus() {
    static std::atomic<int> cache[kMaxDevices];
    const int dev = current_device();
    int cus = cache[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[dev].store(cus, std::memory_order_relaxed);
    }
    return cus;
}

int check_seqs(const msa_seqs *S) {
    if (S == nullptr || S->offsets == nullptr) return MSA_EINVAL;
    if (S->n < 0) return MSA_EINVAL;
    if (S->sigma < 2 || S->sigma > 32) return MSA_EINVAL;
    if (S->packed_2bit != 0 && S->packed_2bit != 1) return MSA_EINVAL;
    if (S->packed_2bit && S->sigma > 4) return MSA_EINVAL;
    if (S->max_len < 0) return MSA_EINVAL;
    if (S->max_len > 65535) return MSA_ERANGE;
    if (S->n > 0 && S->max_len > 0 && S->codes == nullptr) return MSA_EINVAL;
    return MSA_OK;
}

__device__ __forceinline__ int32_t seq_len(const msa_seqs &S, int32_t k, int32_t *st) {
    int64_t L = S.offsets[k + 1] - S.offsets[k];
    if (L < 0 || L > S.max_len) {
        set_status(st, MSA_DS_LENGTH);
        return L < 0 ? 0 : S.max_len;
    }
    return (int32_t)L;
}

// One workgroup per staged row.  Row r receives sequence order[r] (or r).
__global__ void __launch_bounds__(256) k_stage(msa_seqs S, const int32_t *order, Staged out,
                                               int32_t *st) {
    const int32_t r = blockIdx.x;
    const int32_t k = order ? order[r] : r;
    const int32_t L = seq_len(S, k, st);
    const int64_t o = S.offsets[k];
    uint8_t *dst = out.codes + (int64_t)r * out.stride;
    const uint32_t sig = (uint32_t)S.sigma;
    for (int64_t p = threadIdx.x; p < out.stride; p += blockDim.x) {
        uint32_t c = 0;
        if (p < L) {
            const int64_t q = o + p;
            c = S.packed_2bit ? ((S.codes[q >> 2] >> (2 * (q & 3))) & 3u) : S.codes[q];
            if (c >= sig) {
                set_status(st, MSA_DS_SYMBOL);
                c = 0;
            }
        }
        dst[p] = (uint8_t)c;
    }
    if (threadIdx.x == 0) out.len[r] = L;
}

int stage_set(const msa_seqs *S, const int32_t *order, Staged out, int32_t *d_status,
              hipStream_t s) {
    if (S->n == 0) return MSA_OK;
    hipLaunchKernelGGL(k_stage, dim3(S->n), dim3(256), 0, s, *S, order, out, d_status);
    return launch_status();
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static dim3 grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return MSA_OK;
    hipLaunchKernelGGL(k_fill_i32, grid_for(n), dim3(256), 0, s, p, n, v);
    return launch_status();
}
int fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return MSA_OK;
    hipLaunchKernelGGL(k_fill_i64, grid_for(n), dim3(256), 0, s, p, n, v);
    return launch_status();
}

// Exclusive prefix sum of data[0..n) in place, one workgroup of 1024 threads:
// each thread sums a contiguous chunk, the chunk totals are scanned in LDS,
// then each thread rewrites its chunk.
__global__ void __launch_bounds__(1024) k_scan_i64(int64_t *data, int64_t n) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk, hi = min(n, lo + chunk);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += data[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t v = data[i];
        data[i] = run;
        run += v;
    }
}

int exclusive_scan_i64(int64_t *data, int64_t n, hipStream_t s) {
    if (n <= 0) return MSA_OK;
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, data, n);
    return launch_status();
}

__global__ void k_len_hist(msa_seqs S, int32_t *len, int32_t *hist, int32_t *st) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.n) return;
    int32_t L = seq_len(S, k, st);
    len[k] = L;
    atomicAdd(&hist[L], 1);
}

__global__ void __launch_bounds__(1024) k_scan_i32(int32_t *data, int32_t n) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int32_t chunk = (n + 1023) / 1024;
    const int32_t lo = t * chunk, hi = min(n, lo + chunk);
    int32_t sum = 0;
    for (int32_t i = lo; i < hi; ++i) sum += data[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int32_t i = lo; i < hi; ++i) {
        int32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

__global__ void k_len_scatter(int32_t n, const int32_t *len, int32_t *hist, int32_t *order) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t pos = atomicAdd(&hist[len[k]], 1);
    order[pos] = k;
}

// order[r] = the sequence at rank r when sequences are ordered by length
// (ascending; the order among equal lengths is unspecified).
int sort_by_length(const msa_seqs *S, int32_t *len_tmp, int32_t *hist, int32_t *order,
                   int32_t *d_status, hipStream_t s) {
    if (S->n == 0) return MSA_OK;
    int rc = fill_i32(hist, (int64_t)S->max_len + 1, 0, s);
    if (rc) return rc;
    dim3 g((S->n + 255) / 256);
    hipLaunchKernelGGL(k_len_hist, g, dim3(256), 0, s, *S, len_tmp, hist, d_status);
    hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, s, hist, S->max_len + 1);
    hipLaunchKernelGGL(k_len_scatter, g, dim3(256), 0, s, S->n, len_tmp, hist, order);
    return launch_status();
}

}  // namespace msadp

extern "C" {

const char *msa_strerror(int code) {
    switch (code) {
        case MSA_OK: return "ok";
        case MSA_EINVAL: return "invalid argument";
        case MSA_ERANGE: return "size out of supported range";
        case MSA_ENOSPC: return "workspace or output capacity too small";
        case MSA_EDEVICE: return "device launch or runtime failure";
        default: return "unknown error";
    }
}

int msa_version(void) { return 1; }

}  // extern "C"
