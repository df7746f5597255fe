// Bottom-up merge of partial alignments (Sec. 2.2) on the GPU.
//
// The tree from tree_build is walked by depth, deepest first.  Every node's
// alignment is a block of rows (its members, in perm order) in a matrix with
// one row per position; two such matrices alternate between levels.  For all
// nodes of one depth at once:
//   * leaves write their sequence into their row;
//   * internal nodes gather the aligned row of each child's center (the
//     child's Alg. 1 medoid), align the two rows with nw_batch/nw_traceback
//     (the gap is an ordinary symbol, code sigma), turn the ops into column
//     maps with a block scan, and widen both children's rows into the
//     parent's block: an all-gap column at every I op for L's rows and at
//     every D op for R's rows (steps 2-4 of Sec. 2.2).
// The host reads the children's widths once per level to size the batch.
#include <vector>
#include <algorithm>

#include "common.hpp"

namespace msadp {

struct MergeArgs {
    uint8_t *cur, *next;     // n x pitch matrices (rows = positions)
    int64_t pitch;
    int32_t width_cap;
    const int32_t *perm;     // position -> input index
    const int32_t *pos_of;   // input index -> position
    const int32_t *center;
    const int32_t *left, *right;
    const int64_t *mstart, *mcount;
    int32_t *width;          // per node (at most width_cap)
    int32_t *over;           // set to 1 when a node's width exceeds width_cap
    int32_t *st;
    uint8_t gap;
};

// Leaf rows: each member of a leaf gets its sequence.
__global__ void __launch_bounds__(256) k_write_leaves(MergeArgs a, Staged S, const int32_t *ids,
                                                      int32_t n_ids) {
    for (int32_t i = blockIdx.x; i < n_ids; i += gridDim.x) {
        const int32_t v = ids[i];
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        int32_t w = 0;
        for (int64_t r = 0; r < k; ++r) {
            const int32_t s = a.perm[ms + r];
            const int32_t L = S.len[s];
            w = max(w, L);
            uint8_t *dst = a.next + (ms + r) * a.pitch;
            const uint8_t *src = S.codes + (int64_t)s * S.stride;
            for (int32_t c = threadIdx.x; c < L && c < a.width_cap; c += blockDim.x) dst[c] = src[c];
        }
        // copies of one sequence share the width; pad shorter rows (none
        // arise for distinct inputs) with gaps
        for (int64_t r = 0; r < k; ++r) {
            const int32_t s = a.perm[ms + r];
            uint8_t *dst = a.next + (ms + r) * a.pitch;
            for (int32_t c = S.len[s] + threadIdx.x; c < w && c < a.width_cap; c += blockDim.x)
                dst[c] = a.gap;
        }
        if (threadIdx.x == 0) {
            if (w > a.width_cap) *a.over = 1;
            a.width[v] = min(w, a.width_cap);
        }
    }
}

// Aligned center rows of the children of each internal node into two CSR
// sets (offsets computed on the host from the children's widths).
__global__ void __launch_bounds__(256) k_gather_centers(MergeArgs a, const int32_t *ids,
                                                        int32_t n_ids, uint8_t *ca,
                                                        const int64_t *oa, uint8_t *cb,
                                                        const int64_t *ob) {
    for (int32_t i = blockIdx.x; i < n_ids; i += gridDim.x) {
        const int32_t v = ids[i];
        const int32_t L = a.left[v], R = a.right[v];
        const uint8_t *ra = a.cur + (int64_t)a.pos_of[a.center[L]] * a.pitch;
        const uint8_t *rb = a.cur + (int64_t)a.pos_of[a.center[R]] * a.pitch;
        const int64_t wa = oa[i + 1] - oa[i], wb = ob[i + 1] - ob[i];
        for (int64_t c = threadIdx.x; c < wa; c += blockDim.x) ca[oa[i] + c] = ra[c];
        for (int64_t c = threadIdx.x; c < wb; c += blockDim.x) cb[ob[i] + c] = rb[c];
    }
}

// Column maps of each merge: for output column c, the source column of the
// L rows (or -1 for a new gap column) and of the R rows.
__global__ void __launch_bounds__(256) k_merge_maps(MergeArgs a, const int32_t *ids, int32_t n_ids,
                                                    const uint8_t *ops, const int64_t *ops_off,
                                                    const int32_t *ops_len, int16_t *map_l,
                                                    int16_t *map_r, const int64_t *map_off) {
    __shared__ int32_t sl[256], sr[256];
    __shared__ int32_t base_l, base_r;
    for (int32_t i = blockIdx.x; i < n_ids; i += gridDim.x) {
        const int32_t v = ids[i];
        const int32_t W = ops_len[i];
        const uint8_t *o = ops + ops_off[i];
        if (threadIdx.x == 0) {
            base_l = 0;
            base_r = 0;
            if (W > a.width_cap) *a.over = 1;
            a.width[v] = min(W, a.width_cap);
        }
        __syncthreads();
        for (int32_t c0 = 0; c0 < W; c0 += blockDim.x) {
            const int32_t c = c0 + threadIdx.x;
            const int op = c < W ? o[c] : 1;   // op 0 = M, 1 = D, 2 = I
            const int fl = (c < W && op != 2) ? 1 : 0;   // consumes an L column
            const int fr = (c < W && op != 1) ? 1 : 0;   // consumes an R column
            sl[threadIdx.x] = fl;
            sr[threadIdx.x] = fr;
            __syncthreads();
            for (int off = 1; off < 256; off <<= 1) {
                const int32_t tl = threadIdx.x >= off ? sl[threadIdx.x - off] : 0;
                const int32_t tr = threadIdx.x >= off ? sr[threadIdx.x - off] : 0;
                __syncthreads();
                sl[threadIdx.x] += tl;
                sr[threadIdx.x] += tr;
                __syncthreads();
            }
            if (c < W) {
                map_l[map_off[i] + c] = (int16_t)(fl ? base_l + sl[threadIdx.x] - 1 : -1);
                map_r[map_off[i] + c] = (int16_t)(fr ? base_r + sr[threadIdx.x] - 1 : -1);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                base_l += sl[255];
                base_r += sr[255];
            }
            __syncthreads();
        }
    }
}

// Widen and join: one workgroup per row of the level's internal nodes.
__global__ void __launch_bounds__(256) k_merge_rows(MergeArgs a, const int32_t *row_node,
                                                    const int32_t *row_pos, int64_t n_rows,
                                                    const int32_t *ids, const int16_t *map_l,
                                                    const int16_t *map_r, const int64_t *map_off) {
    for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
        const int32_t i = row_node[r];
        const int32_t v = ids[i];
        const int64_t p = row_pos[r];
        const int32_t L = a.left[v];
        const bool in_left = p < a.mstart[L] + a.mcount[L];
        const int16_t *map = (in_left ? map_l : map_r) + map_off[i];
        const int32_t W = a.width[v];
        const uint8_t *src = a.cur + p * a.pitch;
        uint8_t *dst = a.next + p * a.pitch;
        for (int32_t c = threadIdx.x; c < W; c += blockDim.x) {
            const int32_t m = map[c];
            dst[c] = m < 0 ? a.gap : src[m];
        }
    }
}

__global__ void k_pos_of(const int32_t *perm, int32_t n, int32_t *pos_of) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) pos_of[perm[p]] = p;
}

__global__ void __launch_bounds__(256) k_msa_out(const uint8_t *cur, int64_t pitch,
                                                 const int32_t *pos_of, int32_t n, int32_t W,
                                                 uint8_t *out, int64_t out_pitch) {
    for (int32_t s = blockIdx.x; s < n; s += gridDim.x) {
        const uint8_t *src = cur + (int64_t)pos_of[s] * pitch;
        for (int32_t c = threadIdx.x; c < W; c += blockDim.x) out[(int64_t)s * out_pitch + c] = src[c];
    }
}

struct MergePlan {
    int64_t pitch, stride;
    size_t nw_ws;
};

static MergePlan plan_merge(const msa_seqs *S, int32_t width_cap) {
    MergePlan p;
    p.pitch = ((int64_t)width_cap + 15) / 16 * 16;
    p.stride = staged_stride(S->max_len);
    msa_seqs g{};
    g.codes = (const uint8_t *)16;
    g.offsets = (const int64_t *)16;
    g.n = S->n;
    g.sigma = S->sigma + 1;
    g.max_len = width_cap;
    p.nw_ws = nw_workspace_bytes(&g, &g, S->n);
    return p;
}

template <class Alloc>
static void merge_layout(Alloc &al, const msa_seqs *S, int32_t n_nodes, int32_t width_cap,
                         size_t tb_cap, const MergePlan &p) {
    const size_t n = (size_t)S->n;
    al.template take<uint8_t>(n * p.stride);           // staged sequences
    al.template take<int32_t>(n + 1);
    al.template take<uint8_t>(n * p.pitch);            // matrix A
    al.template take<uint8_t>(n * p.pitch);            // matrix B
    al.template take<int32_t>((size_t)n_nodes);        // widths
    al.template take<int32_t>(1);                      // width overflow flag
    al.template take<int32_t>(n);                      // pos_of
    al.template take<int32_t>(n);                      // node ids of a level
    al.template take<uint8_t>(n * (size_t)width_cap / 2 + 16);  // center rows A
    al.template take<uint8_t>(n * (size_t)width_cap / 2 + 16);  // center rows B
    al.template take<int64_t>(n + 1);                  // offsets A
    al.template take<int64_t>(n + 1);                  // offsets B
    al.template take<int32_t>(n);                      // iota
    al.template take<uint8_t>(tb_cap);                 // traceback codes
    al.template take<int64_t>(n + 1);                  // tb offsets
    al.template take<uint8_t>(n * (size_t)width_cap);  // ops (<= n/2 merges of <= 2 cap)
    al.template take<int64_t>(n + 1);                  // ops offsets
    al.template take<int32_t>(n);                      // ops lengths
    al.template take<int16_t>(n * (size_t)width_cap);  // map L
    al.template take<int16_t>(n * (size_t)width_cap);  // map R
    al.template take<int64_t>(n + 1);                  // map offsets
    al.template take<int32_t>(n);                      // row -> node
    al.template take<int32_t>(n);                      // row -> position
    al.template take<uint8_t>(p.nw_ws);                // nw_batch workspace
}

}  // namespace msadp

using namespace msadp;

extern "C" {

size_t msa_merge_workspace_bytes(const msa_seqs *S, int32_t n_nodes, int32_t width_cap,
                                 size_t tb_cap) {
    if (check_seqs(S) || n_nodes < 0 || width_cap < 1 || width_cap > 32768) return 0;
    Sizer sz;
    merge_layout(sz, S, n_nodes, width_cap, tb_cap, plan_merge(S, width_cap));
    return sz.total();
}

int msa_merge(const msa_seqs *S, const msa_tree *T, int32_t n_nodes, int32_t width_cap,
              size_t tb_cap, uint8_t *msa, int64_t msa_pitch, int32_t *width_out, void *ws,
              size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (T == nullptr || width_out == nullptr || msa == nullptr || ws == nullptr) return MSA_EINVAL;
    if (S->sigma + 1 > 32) return MSA_ERANGE;
    if (width_cap < 1 || width_cap > 32768 || msa_pitch < width_cap) return MSA_EINVAL;
    if (S->n == 0 || n_nodes < 1) return MSA_EINVAL;
    if (S->max_len > width_cap) return MSA_ENOSPC;
    const MergePlan pl = plan_merge(S, width_cap);
    Sizer sz;
    merge_layout(sz, S, n_nodes, width_cap, tb_cap, pl);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    const size_t n = (size_t)S->n;
    Carve cv(ws, ws_bytes);
    Staged SS{cv.take<uint8_t>(n * pl.stride), cv.take<int32_t>(n + 1), pl.stride, S->n};
    uint8_t *mat0 = cv.take<uint8_t>(n * pl.pitch);
    uint8_t *mat1 = cv.take<uint8_t>(n * pl.pitch);
    int32_t *width = cv.take<int32_t>((size_t)n_nodes);
    int32_t *over = cv.take<int32_t>(1);
    int32_t *pos_of = cv.take<int32_t>(n);
    int32_t *ids = cv.take<int32_t>(n);
    uint8_t *ca = cv.take<uint8_t>(n * (size_t)width_cap / 2 + 16);
    uint8_t *cb = cv.take<uint8_t>(n * (size_t)width_cap / 2 + 16);
    int64_t *oa = cv.take<int64_t>(n + 1);
    int64_t *ob = cv.take<int64_t>(n + 1);
    int32_t *iota = cv.take<int32_t>(n);
    uint8_t *tb = cv.take<uint8_t>(tb_cap);
    int64_t *tb_off = cv.take<int64_t>(n + 1);
    uint8_t *ops = cv.take<uint8_t>(n * (size_t)width_cap);
    int64_t *ops_off = cv.take<int64_t>(n + 1);
    int32_t *ops_len = cv.take<int32_t>(n);
    int16_t *map_l = cv.take<int16_t>(n * (size_t)width_cap);
    int16_t *map_r = cv.take<int16_t>(n * (size_t)width_cap);
    int64_t *map_off = cv.take<int64_t>(n + 1);
    int32_t *row_node = cv.take<int32_t>(n);
    int32_t *row_pos = cv.take<int32_t>(n);
    uint8_t *nw_ws = cv.take<uint8_t>(pl.nw_ws);

    // host copy of the tree shape
    std::vector<int32_t> left(n_nodes), right(n_nodes), depth(n_nodes);
    std::vector<int64_t> mstart(n_nodes), mcount(n_nodes);
    if (hipMemcpyAsync(left.data(), T->left, 4 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
        hipMemcpyAsync(right.data(), T->right, 4 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
        hipMemcpyAsync(depth.data(), T->depth, 4 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
        hipMemcpyAsync(mstart.data(), T->mstart, 8 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
        hipMemcpyAsync(mcount.data(), T->mcount, 8 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
        hipStreamSynchronize(s))
        return MSA_EDEVICE;
    int32_t dmax = 0;
    for (int32_t v = 0; v < n_nodes; ++v) {
        if (depth[v] < 0 || (v > 0 && depth[v] < depth[v - 1])) return MSA_EINVAL;
        dmax = std::max(dmax, depth[v]);
    }
    {
        std::vector<int32_t> io(n);
        for (size_t i = 0; i < n; ++i) io[i] = (int32_t)i;
        if (hipMemcpyAsync(iota, io.data(), 4 * n, hipMemcpyHostToDevice, s)) return MSA_EDEVICE;
        if (hipStreamSynchronize(s)) return MSA_EDEVICE;
    }
    if ((rc = stage_set(S, nullptr, SS, d_status, s))) return rc;
    hipLaunchKernelGGL(k_pos_of, dim3((S->n + 255) / 256), dim3(256), 0, s, T->perm, S->n, pos_of);

    MergeArgs a{};
    a.pitch = pl.pitch;
    a.width_cap = width_cap;
    a.perm = T->perm;
    a.pos_of = pos_of;
    a.center = T->center;
    a.left = T->left;
    a.right = T->right;
    a.mstart = T->mstart;
    a.mcount = T->mcount;
    a.width = width;
    a.over = over;
    a.st = d_status;
    if ((rc = fill_i32(over, 1, 0, s))) return rc;
    a.gap = (uint8_t)S->sigma;
    uint8_t *cur = mat0, *next = mat1;
    std::vector<int32_t> wv(n_nodes, 0);

    int32_t vend = n_nodes;
    for (int32_t d = dmax; d >= 0; --d) {
        int32_t vbeg = vend;
        while (vbeg > 0 && depth[vbeg - 1] == d) --vbeg;
        std::vector<int32_t> leaves, inner;
        for (int32_t v = vbeg; v < vend; ++v) (left[v] < 0 ? leaves : inner).push_back(v);
        a.cur = cur;
        a.next = next;
        if (!leaves.empty()) {
            if (hipMemcpyAsync(ids, leaves.data(), 4 * leaves.size(), hipMemcpyHostToDevice, s))
                return MSA_EDEVICE;
            hipLaunchKernelGGL(k_write_leaves, dim3((unsigned)std::min<size_t>(leaves.size(), 4096)),
                               dim3(256), 0, s, a, SS, ids, (int32_t)leaves.size());
            if ((rc = launch_status())) return rc;
        }
        if (!inner.empty()) {
            // children's widths, known from the previous level
            if (hipMemcpyAsync(wv.data(), width, 4 * (size_t)n_nodes, hipMemcpyDeviceToHost, s) ||
                hipStreamSynchronize(s))
                return MSA_EDEVICE;
            const size_t ni = inner.size();
            std::vector<int64_t> hoa(ni + 1, 0), hob(ni + 1, 0), htb(ni + 1, 0), hops(ni + 1, 0);
            int32_t maxa = 0, maxb = 0;
            int64_t rows = 0;
            for (size_t i = 0; i < ni; ++i) {
                const int32_t wa = wv[left[inner[i]]], wb = wv[right[inner[i]]];
                if (wa > width_cap || wb > width_cap) return MSA_ENOSPC;
                maxa = std::max(maxa, wa);
                maxb = std::max(maxb, wb);
                hoa[i + 1] = hoa[i] + wa;
                hob[i + 1] = hob[i] + wb;
                htb[i + 1] = htb[i] + ((int64_t)nw_tb_bytes(wa, wb) + 255) / 256 * 256;
                hops[i + 1] = hops[i] + wa + wb;
                rows += mcount[inner[i]];
            }
            if ((size_t)htb[ni] > tb_cap) return MSA_ENOSPC;
            std::vector<int32_t> hrn((size_t)rows), hrp((size_t)rows);
            {
                int64_t r = 0;
                for (size_t i = 0; i < ni; ++i)
                    for (int64_t k = 0; k < mcount[inner[i]]; ++k, ++r) {
                        hrn[r] = (int32_t)i;
                        hrp[r] = (int32_t)(mstart[inner[i]] + k);
                    }
            }
            std::vector<int64_t> hmo(ni + 1, 0);
            for (size_t i = 0; i < ni; ++i) hmo[i + 1] = hmo[i] + hops[i + 1] - hops[i];
            if (hipMemcpyAsync(ids, inner.data(), 4 * ni, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(oa, hoa.data(), 8 * (ni + 1), hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(ob, hob.data(), 8 * (ni + 1), hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(tb_off, htb.data(), 8 * (ni + 1), hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(ops_off, hops.data(), 8 * (ni + 1), hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(map_off, hmo.data(), 8 * (ni + 1), hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(row_node, hrn.data(), 4 * (size_t)rows, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(row_pos, hrp.data(), 4 * (size_t)rows, hipMemcpyHostToDevice, s))
                return MSA_EDEVICE;
            const unsigned g = (unsigned)std::min<size_t>(ni, 4096);
            hipLaunchKernelGGL(k_gather_centers, dim3(g), dim3(256), 0, s, a, ids, (int32_t)ni, ca,
                               oa, cb, ob);
            msa_seqs A{ca, oa, (int32_t)ni, S->sigma + 1, std::max(maxa, 1), 0};
            msa_seqs B{cb, ob, (int32_t)ni, S->sigma + 1, std::max(maxb, 1), 0};
            if ((rc = nw_batch(&A, &B, iota, iota, (int64_t)ni, nullptr, tb, tb_off, nw_ws,
                               pl.nw_ws, d_status, s)))
                return rc;
            if ((rc = nw_traceback(&A, &B, iota, iota, (int64_t)ni, tb, tb_off, ops, ops_off,
                                   ops_len, d_status, s)))
                return rc;
            hipLaunchKernelGGL(k_merge_maps, dim3(g), dim3(256), 0, s, a, ids, (int32_t)ni, ops,
                               ops_off, ops_len, map_l, map_r, map_off);
            hipLaunchKernelGGL(k_merge_rows, dim3((unsigned)std::min<int64_t>(rows, 65536)),
                               dim3(256), 0, s, a, row_node, row_pos, rows, ids, map_l, map_r,
                               map_off);
            if ((rc = launch_status())) return rc;
        }
        // keep this level's host vectors alive until their copies have run;
        // a width beyond width_cap ends the merge with MSA_ENOSPC
        int32_t over_h = 0;
        if (hipMemcpyAsync(&over_h, over, 4, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
            return MSA_EDEVICE;
        if (over_h) return MSA_ENOSPC;
        std::swap(cur, next);
        vend = vbeg;
    }
    if (hipMemcpyAsync(wv.data(), width, 4, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
        return MSA_EDEVICE;
    const int32_t W = wv[0];
    if (W > width_cap) return MSA_ENOSPC;
    hipLaunchKernelGGL(k_msa_out, dim3((unsigned)std::min<int32_t>(S->n, 65536)), dim3(256), 0, s,
                       cur, pl.pitch, pos_of, S->n, W, msa, msa_pitch);
    if ((rc = launch_status())) return rc;
    *width_out = W;
    return MSA_OK;
}

}  // extern "C"
