// lev_batch for callers that cannot allocate device memory: the workspace is
// a fixed device array of the library (`scratch`) instead of a caller buffer.
//
// In host code `scratch` names a host-side stand-in, not the device array;
// the device address is read once per device with hipGetSymbolAddress (with
// that device current) and only that address is handed to kernels and copies.
// Each GPU holds its own copy of the array until the process ends, and every
// call on one GPU shares it.
#include <mutex>

#include "common.hpp"

namespace msadp {

static __device__ __align__(256) uint8_t scratch[MSA_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch`, per device

// The current device's copy of `scratch`, looked up on its first use; null
// when the device cannot be read or the lookup fails.
void *scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}
}  // namespace

}  // namespace msadp

using namespace msadp;

extern "C" int lev_batch_noalloc(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                                 const int32_t *ib, int64_t n_pairs, uint16_t *dist,
                                 int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(A)) || (rc = check_seqs(B))) return rc;
    if (n_pairs < 0 || A->sigma != B->sigma) return MSA_EINVAL;
    if (n_pairs == 0) return MSA_OK;
    if (ia == nullptr || ib == nullptr || dist == nullptr) return MSA_EINVAL;
    // the default layout and word class (no tuning entry can then ask for
    // carry buffers beyond what this size check covered)
    if (lev_batch_ws_bytes(A, B, n_pairs, true) > (size_t)MSA_NOALLOC_SCRATCH_BYTES)
        return MSA_ENOSPC;
    void *ws = scratch_ptr();
    if (ws == nullptr) return MSA_EDEVICE;
    return lev_batch_impl(A, B, ia, ib, n_pairs, dist, ws, (size_t)MSA_NOALLOC_SCRATCH_BYTES,
                          d_status, s, -1);
}
