// Insertion of new sequences into an existing Alg. 1 tree.  Sec. 5 of the
// paper names online updates (new sequences added to the clusters, the
// guide tree and the alignment) as future work without a procedure; the
// reading built here:
//   1. route: every new x starts at the root and, at an internal node with
//      poles l and r, goes to the left child if f(l, x) <= f(r, x), else to
//      the right one (Alg. 1's split rule), down to a leaf;
//   2. re-partition: each leaf that received new sequences is replaced by
//      Alg. 1 (full median) on its old and new members;
//   3. renumber: the updated tree gets breadth-first ids from the root (a
//      level's children after the level, in parent order, L before R), and
//      member ranges as in tree_build (L's range, then R's).
// Internal nodes keep their center and poles.  The alignment of the grown
// set is msa_merge along the new tree.
//
// Routing runs level-synchronously: one distance launch per tree depth on the
// (pole, x) pairs of the sequences still above a leaf, a pair per group of
// lanes on the set staged once per call (lev_batch for patterns beyond that
// layout).  The grown leaves are
// re-partitioned together, as a forest, by the level passes of tree.hip.
// The splice walks the combined tree breadth-first inside one workgroup
// (a block scan per chunk of a level), then sums member counts bottom-up and
// places ranges top-down, level by level.
#include "common.hpp"
#include "lev_xl.hpp"

namespace msadp {

struct OldTree {
    const int32_t *left, *right, *center, *lpole, *rpole, *perm;
    const int64_t *mstart, *mcount;
    int32_t n_nodes;
    int32_t n_old;           // perm entries
};

// A leaf's member range lies inside the old perm.
__device__ __forceinline__ bool range_ok(const OldTree &t, int32_t v) {
    const int64_t ms = t.mstart[v], k = t.mcount[v];
    return ms >= 0 && k >= 1 && ms + k <= t.n_old;
}

__global__ void __launch_bounds__(256) k_route_init(int32_t *cur, int32_t n_new) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_new) cur[k] = 0;
}

// The (l, x) and (r, x) pairs of every new sequence above a leaf, compacted
// through a counter (slot order is free: each slot names its sequence).
// Out-of-range node ids or poles set MSA_DS_INDEX and end that route.
__global__ void __launch_bounds__(256) k_route_pairs(OldTree t, int32_t n_old, int32_t *cur,
                                                    int32_t n_new, uint32_t *cnt,
                                                    int32_t *slot_k, int32_t *ia, int32_t *ib,
                                                    int32_t *st) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_new) return;
    const int32_t v = cur[k];
    if (v < 0) return;
    if (v >= t.n_nodes) {
        set_status(st, MSA_DS_INDEX);
        cur[k] = -1;
        return;
    }
    if (t.left[v] < 0) return;
    const int32_t l = t.lpole[v], r = t.rpole[v], L = t.left[v], R = t.right[v];
    if (l < 0 || l >= n_old || r < 0 || r >= n_old || L >= t.n_nodes || R < 0 ||
        R >= t.n_nodes) {
        set_status(st, MSA_DS_INDEX);
        cur[k] = -1;
        return;
    }
    const uint32_t slot = atomicAdd(cnt, 1u);
    slot_k[slot] = k;
    ia[2 * slot] = l;
    ia[2 * slot + 1] = r;
    ib[2 * slot] = ib[2 * slot + 1] = n_old + k;
}

__global__ void __launch_bounds__(256) k_route_step(OldTree t, int32_t *cur,
                                                   const int32_t *slot_k, const uint16_t *dist,
                                                   int32_t n_slots) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_slots) return;
    const int32_t k = slot_k[j], v = cur[k];
    cur[k] = dist[2 * j] <= dist[2 * j + 1] ? t.left[v] : t.right[v];
}

// New arrivals per leaf (routes that failed count nowhere).
__global__ void __launch_bounds__(256) k_leaf_count(const int32_t *cur, int32_t n_new,
                                                   int32_t *arrivals) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_new && cur[k] >= 0) atomicAdd(&arrivals[cur[k]], 1);
}

// Exclusive scan of n int64 in place (one workgroup); a[n] = the total.
__global__ void __launch_bounds__(1024) k_scan_i64(int64_t *a, int32_t n) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int32_t chunk = (n + 1023) / 1024;
    const int32_t lo = min(n, t * chunk), hi = min(n, lo + chunk);
    int64_t sum = 0;
    for (int32_t i = lo; i < hi; ++i) sum += a[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int32_t i = lo; i < hi; ++i) {
        const int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (t == 1023) a[n] = part[1023];
}

// Forest root f of every grown leaf v: which leaf, and its size.
__global__ void __launch_bounds__(256) k_forest_sizes(OldTree t, const int32_t *arrivals,
                                                     const int32_t *froot, int32_t *fleaf,
                                                     int64_t *fsize) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= t.n_nodes || arrivals[v] == 0) return;
    const int32_t f = froot[v];
    fleaf[f] = v;
    // a leaf with a broken range keeps only its arrivals
    fsize[f] = (range_ok(t, v) ? t.mcount[v] : 0) + arrivals[v];
}

// Members of forest root f: the leaf's old members, then its arrivals.
__global__ void __launch_bounds__(256) k_forest_old(OldTree t, const int32_t *fleaf,
                                                   const int64_t *fstart, int32_t K,
                                                   int32_t *fmem, int32_t *st) {
    for (int32_t f = blockIdx.x; f < K; f += gridDim.x) {
        const int32_t v = fleaf[f];
        if (!range_ok(t, v)) {
            if (threadIdx.x == 0) set_status(st, MSA_DS_INDEX);
            continue;
        }
        const int64_t ms = t.mstart[v], k = t.mcount[v], dst = fstart[f];
        for (int64_t i = threadIdx.x; i < k; i += blockDim.x) fmem[dst + i] = t.perm[ms + i];
    }
}

__global__ void __launch_bounds__(256) k_forest_new(OldTree t, const int32_t *cur, int32_t n_new,
                                                   int32_t n_old, const int32_t *froot,
                                                   const int64_t *fstart, int32_t *fill,
                                                   int32_t *fmem) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_new || cur[k] < 0) return;
    const int32_t v = cur[k], f = froot[v];
    const int32_t at = atomicAdd(&fill[f], 1);
    fmem[fstart[f] + (range_ok(t, v) ? t.mcount[v] : 0) + at] = n_old + k;
}

struct SpliceArgs {
    OldTree o;
    const int32_t *froot;    // [o.n_nodes + 1] exclusive scan of grown-leaf flags
    // the re-partitioned forest (roots 0 .. K-1 replace the grown leaves)
    const int32_t *fl, *fr, *fc, *flp, *frp, *fperm;
    const int64_t *fms, *fmc;
    int32_t K, nf;
    int32_t *bfs;            // [U]: unified node of each new id
    int32_t *lvl;            // [U + 1]: first new id of each depth
    msa_tree out;
    int32_t cap;             // node capacity of out
    int32_t n;               // perm entries of out
    int32_t *total;          // node count written here
    int32_t *st;
};

// Unified ids: old nodes keep theirs; forest node u >= K becomes
// o.n_nodes + u - K; forest root f is the grown leaf it replaces.
struct UView {
    int32_t l, r, c, lp, rp;
    const int32_t *mem;      // members of a leaf (in range order)
    int64_t nmem;            // 0 when the old range is broken
};

__device__ __forceinline__ bool grown(const SpliceArgs &a, int32_t v) {
    return a.froot[v + 1] > a.froot[v];
}

__device__ __forceinline__ int32_t forest_uid(const SpliceArgs &a, int32_t u) {
    return u < 0 ? -1 : a.o.n_nodes + u - a.K;
}

__device__ UView view(const SpliceArgs &a, int32_t w) {
    UView x;
    int32_t u = -1;                       // forest node behind w, if any
    if (w < a.o.n_nodes) {
        if (grown(a, w)) u = a.froot[w];
    } else {
        u = w - a.o.n_nodes + a.K;
    }
    if (u < 0) {
        x.l = a.o.left[w];
        x.r = a.o.right[w];
        x.c = a.o.center[w];
        x.lp = a.o.lpole[w];
        x.rp = a.o.rpole[w];
        const bool ok = range_ok(a.o, w);
        x.mem = a.o.perm + (ok ? a.o.mstart[w] : 0);
        x.nmem = ok ? a.o.mcount[w] : 0;
    } else {
        x.l = forest_uid(a, a.fl[u]);
        x.r = forest_uid(a, a.fr[u]);
        x.c = a.fc[u];
        x.lp = a.flp[u];
        x.rp = a.frp[u];
        x.mem = a.fperm + a.fms[u];
        x.nmem = a.fmc[u];
    }
    return x;
}

// Count of set flags among threads 0 .. t of the 1024-thread block (an
// inclusive prefix), and the block's total: a ballot prefix inside each
// wavefront and the 16 wavefronts' counts through LDS.  wsum holds two
// buffers of 16, used alternately (buf), so that one barrier per call
// orders every write before its reads and after the previous call's.
constexpr int kSpliceWaves = 1024 / kWave;

__device__ __forceinline__ int32_t block_count(bool f, int32_t (*wsum)[kSpliceWaves], int &buf,
                                               int32_t &total) {
    const int t = threadIdx.x, w = t / kWave;
    const uint64_t m = __ballot(f);
    const int32_t below = (int32_t)__builtin_amdgcn_mbcnt_hi(
        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if ((t & (kWave - 1)) == 0) wsum[buf][w] = __popcll(m);
    __syncthreads();
    int32_t before = 0, tot = 0;
#pragma unroll
    for (int x = 0; x < kSpliceWaves; ++x) {
        const int32_t c = wsum[buf][x];
        tot += c;
        before += x < w ? c : 0;
    }
    buf ^= 1;
    total = tot;
    return before + below + (f ? 1 : 0);
}

// Exclusive scan of n int32 flags (an entry counts when it is > 0) into
// out, one workgroup of 1024 threads; in == out allowed (every entry is read
// and written by the same thread); out[n] = the total.  Entries go in tiles
// of 1024, thread t taking entry t of each (coalesced), the loads of
// kScanTiles tiles issued together; block_count gives each entry its offset
// within its tile and a running total carries from tile to tile.
constexpr int kScanTiles = 8;

__global__ void __launch_bounds__(1024) k_scan_flags(const int32_t *in, int32_t *out, int32_t n) {
    __shared__ int32_t wsum[2][kSpliceWaves];
    const int t = threadIdx.x;
    int buf = 0;
    int32_t run = 0;   // flags before the current tile (the same in every thread)
    for (int64_t base = 0; base < n; base += 1024 * kScanTiles) {
        bool f[kScanTiles];
#pragma unroll
        for (int k = 0; k < kScanTiles; ++k) {
            const int64_t i = base + 1024 * k + t;
            f[k] = i < n && in[i] > 0;
        }
#pragma unroll
        for (int k = 0; k < kScanTiles; ++k) {
            const int64_t i = base + 1024 * k + t;
            int32_t tile_total;
            const int32_t incl = block_count(f[k], wsum, buf, tile_total);
            if (i < n) out[i] = run + incl - (f[k] ? 1 : 0);
            run += tile_total;
        }
    }
    if (t == 0) out[n] = run;
}

__global__ void __launch_bounds__(1024) k_splice(SpliceArgs a) {
    __shared__ int32_t wsum[2][kSpliceWaves];
    __shared__ int32_t s_bad;
    const int t = threadIdx.x;
    const int32_t U = a.o.n_nodes + a.nf - a.K;
    if (t == 0) {
        a.bfs[0] = 0;
        a.out.parent[0] = -1;
        a.out.depth[0] = 0;
        s_bad = 0;
    }
    __syncthreads();
    // breadth-first ids, one level at a time; `next` (the next free id) is
    // the same in every thread
    int32_t lo = 0, hi = 1, d = 0;
    int buf = 0;
    while (lo < hi) {
        if (t == 0) a.lvl[d] = lo;
        int32_t next = hi;
        for (int32_t base = lo; base < hi; base += 1024) {
            const int32_t j = base + t;
            UView x{};
            const bool in = j < hi;
            if (in) x = view(a, a.bfs[j]);
            const int32_t c = (in && x.l >= 0) ? 2 : 0;
            int32_t splits;
            const int32_t incl = 2 * block_count(c != 0, wsum, buf, splits);
            const int32_t chunk = 2 * splits;
            if (in) {
                const int32_t at = next + incl - c;
                const bool fits = at + c <= U && at + c <= a.cap;
                if (c && !fits) s_bad = 1;
                a.out.center[j] = x.c;
                a.out.lpole[j] = c ? x.lp : -1;
                a.out.rpole[j] = c ? x.rp : -1;
                if (c && fits) {
                    a.bfs[at] = x.l;
                    a.bfs[at + 1] = x.r;
                    a.out.left[j] = at;
                    a.out.right[j] = at + 1;
                    a.out.parent[at] = a.out.parent[at + 1] = j;
                    a.out.depth[at] = a.out.depth[at + 1] = d + 1;
                } else {
                    a.out.left[j] = a.out.right[j] = -1;
                }
            }
            next += chunk;
        }
        // every thread's writes of the level (bfs, s_bad) before the next
        // level reads them
        __syncthreads();
        if (s_bad) break;
        lo = hi;
        hi = min(next, min(U, a.cap));
        ++d;
    }
    if (s_bad || hi != U) {
        if (t == 0) {
            set_status(a.st, MSA_DS_INDEX);
            *a.total = 0;
        }
        return;
    }
    if (t == 0) {
        a.lvl[d] = hi;
        *a.total = hi;
    }
    __syncthreads();
    // member counts, deepest level first
    for (int32_t e = d - 1; e >= 0; --e) {
        for (int32_t j = a.lvl[e] + t; j < a.lvl[e + 1]; j += 1024) {
            const int32_t L = a.out.left[j];
            a.out.mcount[j] = L >= 0 ? a.out.mcount[L] + a.out.mcount[a.out.right[j]]
                                     : view(a, a.bfs[j]).nmem;
        }
        __syncthreads();
    }
    // member ranges, root first
    if (t == 0) a.out.mstart[0] = 0;
    __syncthreads();
    for (int32_t e = 0; e < d; ++e) {
        for (int32_t j = a.lvl[e] + t; j < a.lvl[e + 1]; j += 1024) {
            const int32_t L = a.out.left[j];
            if (L < 0) continue;
            a.out.mstart[L] = a.out.mstart[j];
            a.out.mstart[a.out.right[j]] = a.out.mstart[j] + a.out.mcount[L];
        }
        __syncthreads();
    }
    // leaves copy their members (a broken old range leaves a short count)
    if (t == 0 && a.out.mcount[0] != a.n) set_status(a.st, MSA_DS_INDEX);
    for (int32_t j = t; j < hi; j += 1024) {
        if (a.out.left[j] >= 0) continue;
        const UView x = view(a, a.bfs[j]);
        const int64_t dst = a.out.mstart[j];
        if (dst < 0 || dst + x.nmem > a.n) continue;
        for (int64_t i = 0; i < x.nmem; ++i) a.out.perm[dst + i] = x.mem[i];
    }
}

struct InsertWs {
    int32_t *cur, *slot_k, *ia, *ib;
    uint16_t *dist;
    uint32_t *cnt;
    int32_t *arrivals, *froot, *fleaf, *fill, *fmem;
    int64_t *fstart;
    int32_t *fparent, *fleft, *fright, *fcenter, *flpole, *frpole, *fdepth, *fperm;
    int64_t *fmstart, *fmcount;
    int32_t *bfs, *lvl, *total;
    // routing distances: the set staged once for the across-lanes kernel
    // (xl), else lev_batch's workspace
    bool xl;
    Staged SS;
    uint32_t *xl_counter;
    void *lev_ws, *tree_ws;
    size_t lev_bytes, tree_bytes;
};

// Whether the routing rounds can run across lanes: patterns of up to 256
// 64-bit words (the across-lanes layout's limit).
static bool insert_xl(const msa_seqs *S) { return ((int64_t)S->max_len + 63) / 64 <= 256; }

template <class Alloc>
static void insert_layout(Alloc &al, const msa_seqs *S, int32_t n_old, int32_t n_nodes_old,
                          InsertWs &w) {
    const size_t n = (size_t)S->n, nn = (size_t)(S->n - n_old), no = (size_t)n_nodes_old;
    const size_t cap = 2 * n;
    w.cur = al.template take<int32_t>(nn);
    w.slot_k = al.template take<int32_t>(nn);
    w.ia = al.template take<int32_t>(2 * nn);
    w.ib = al.template take<int32_t>(2 * nn);
    w.dist = al.template take<uint16_t>(2 * nn);
    w.cnt = al.template take<uint32_t>(1);
    w.arrivals = al.template take<int32_t>(no);
    w.froot = al.template take<int32_t>(no + 1);
    w.fleaf = al.template take<int32_t>(nn);
    w.fill = al.template take<int32_t>(nn);
    w.fstart = al.template take<int64_t>(nn + 1);
    w.fmem = al.template take<int32_t>(n);
    w.fparent = al.template take<int32_t>(cap);
    w.fleft = al.template take<int32_t>(cap);
    w.fright = al.template take<int32_t>(cap);
    w.fcenter = al.template take<int32_t>(cap);
    w.flpole = al.template take<int32_t>(cap);
    w.frpole = al.template take<int32_t>(cap);
    w.fdepth = al.template take<int32_t>(cap);
    w.fmstart = al.template take<int64_t>(cap);
    w.fmcount = al.template take<int64_t>(cap);
    w.fperm = al.template take<int32_t>(n);
    w.bfs = al.template take<int32_t>(cap);
    w.lvl = al.template take<int32_t>(cap + 1);
    w.total = al.template take<int32_t>(1);
    w.xl = insert_xl(S);
    if (w.xl) {
        const int64_t stride = staged_stride(S->max_len);
        w.SS = Staged{al.template take<uint8_t>(n * (size_t)stride),
                      al.template take<int32_t>(n + 1), stride, S->n};
        w.xl_counter = al.template take<uint32_t>(1);
        w.lev_bytes = 0;
        w.lev_ws = nullptr;
    } else {
        w.lev_bytes = nn ? lev_batch_ws_bytes(S, S, 2 * (int64_t)nn, false) : 0;
        w.lev_ws = al.template take<uint8_t>(w.lev_bytes);
    }
    w.tree_bytes = tree_workspace_bytes(S);
    w.tree_ws = al.template take<uint8_t>(w.tree_bytes);
}

static int insert_args(const msa_seqs *S, int32_t n_old, const msa_tree *T_old,
                       int32_t n_nodes_old) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (n_old < 1 || n_old > S->n || n_nodes_old < 1 || n_nodes_old > 2 * n_old - 1)
        return MSA_EINVAL;
    if (S->n >= (1 << 24)) return MSA_ERANGE;
    if (T_old == nullptr || !T_old->left || !T_old->right || !T_old->center || !T_old->lpole ||
        !T_old->rpole || !T_old->mstart || !T_old->mcount || !T_old->perm)
        return MSA_EINVAL;
    return MSA_OK;
}

static int read_i32(const int32_t *d, int32_t *h, hipStream_t s) {
    if (hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MSA_EDEVICE;
    return MSA_OK;
}

static unsigned blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace msadp

extern "C" {

size_t tree_insert_workspace_bytes(const msa_seqs *S, int32_t n_old, int32_t n_nodes_old) {
    using namespace msadp;
    if (S == nullptr || check_seqs(S) || n_old < 1 || n_old > S->n || n_nodes_old < 1)
        return 0;
    Sizer sz;
    InsertWs w{};
    insert_layout(sz, S, n_old, n_nodes_old, w);
    return sz.total();
}

int tree_insert(const msa_seqs *S, int32_t n_old, const msa_tree *T_old, int32_t n_nodes_old,
                const msa_tree *T_new, int32_t *n_nodes_new, void *ws, size_t ws_bytes,
                int32_t *d_status, hipStream_t s) {
    using namespace msadp;
    int rc;
    if (n_nodes_new == nullptr || T_new == nullptr) return MSA_EINVAL;
    *n_nodes_new = 0;
    if ((rc = insert_args(S, n_old, T_old, n_nodes_old))) return rc;
    if (!T_new->parent || !T_new->left || !T_new->right || !T_new->center || !T_new->lpole ||
        !T_new->rpole || !T_new->depth || !T_new->mstart || !T_new->mcount || !T_new->perm ||
        ws == nullptr || d_status == nullptr)
        return MSA_EINVAL;
    Sizer sz;
    InsertWs w{};
    insert_layout(sz, S, n_old, n_nodes_old, w);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    Carve cv(ws, ws_bytes);
    insert_layout(cv, S, n_old, n_nodes_old, w);
    const int32_t n_new = S->n - n_old;
    const OldTree ot{T_old->left, T_old->right, T_old->center, T_old->lpole, T_old->rpole,
                     T_old->perm, T_old->mstart, T_old->mcount, n_nodes_old, n_old};

    // 1. routing, one tree depth per round
    if (n_new > 0) {
        // each round's pairs are a few per new sequence: one launch sized to
        // them on the set staged once, a pair per group of lanes
        if (w.xl && (rc = stage_set(S, nullptr, w.SS, d_status, s))) return rc;
        hipLaunchKernelGGL(k_route_init, dim3(blocks(n_new)), dim3(256), 0, s, w.cur, n_new);
        for (int32_t round = 0;; ++round) {
            if (round > n_nodes_old) return MSA_EINVAL;   // a child cycle in T_old
            if ((rc = fill_i32((int32_t *)w.cnt, 1, 0, s))) return rc;
            hipLaunchKernelGGL(k_route_pairs, dim3(blocks(n_new)), dim3(256), 0, s, ot, n_old,
                               w.cur, n_new, w.cnt, w.slot_k, w.ia, w.ib, d_status);
            if ((rc = launch_status())) return rc;
            int32_t h = 0;
            if ((rc = read_i32((const int32_t *)w.cnt, &h, s))) return rc;
            if (h == 0) break;
            if (w.xl) {
                if ((rc = lev_xl_staged(w.SS, w.SS, S->sigma, S->max_len, w.ia, w.ib,
                                        2 * (int64_t)h, w.dist, w.xl_counter, d_status, s)))
                    return rc;
            } else if ((rc = lev_batch_impl(S, S, w.ia, w.ib, 2 * (int64_t)h, w.dist, w.lev_ws,
                                            w.lev_bytes, d_status, s, 0))) {
                return rc;
            }
            hipLaunchKernelGGL(k_route_step, dim3(blocks(h)), dim3(256), 0, s, ot, w.cur,
                               w.slot_k, w.dist, h);
        }
    }
    // 2. grown leaves become forest roots, re-partitioned by Alg. 1
    if ((rc = fill_i32(w.arrivals, n_nodes_old, 0, s))) return rc;
    if (n_new > 0)
        hipLaunchKernelGGL(k_leaf_count, dim3(blocks(n_new)), dim3(256), 0, s, w.cur, n_new,
                           w.arrivals);
    hipLaunchKernelGGL(k_scan_flags, dim3(1), dim3(1024), 0, s, w.arrivals, w.froot, n_nodes_old);
    if ((rc = launch_status())) return rc;
    int32_t K = 0, nf = 0;
    if ((rc = read_i32(w.froot + n_nodes_old, &K, s))) return rc;
    const msa_tree TF{w.fparent, w.fleft, w.fright, w.fcenter, w.flpole, w.frpole, w.fdepth,
                      w.fmstart, w.fmcount, w.fperm};
    if (K > 0) {
        hipLaunchKernelGGL(k_forest_sizes, dim3(blocks(n_nodes_old)), dim3(256), 0, s, ot,
                           w.arrivals, w.froot, w.fleaf, w.fstart);
        hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, w.fstart, K);
        if ((rc = fill_i32(w.fill, K, 0, s))) return rc;
        hipLaunchKernelGGL(k_forest_old, dim3((unsigned)std::min(K, 4096)), dim3(256), 0, s, ot,
                           w.fleaf, w.fstart, K, w.fmem, d_status);
        hipLaunchKernelGGL(k_forest_new, dim3(blocks(n_new)), dim3(256), 0, s, ot, w.cur, n_new,
                           n_old, w.froot, w.fstart, w.fill, w.fmem);
        if ((rc = launch_status())) return rc;
        int64_t m = 0;
        if (hipMemcpyAsync(&m, w.fstart + K, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MSA_EDEVICE;
        const Forest fr{K, w.fmem, w.fstart, m};
        if ((rc = tree_build_forest(S, fr, &TF, &nf, w.tree_ws, w.tree_bytes, d_status, s)))
            return rc;
    }
    // 3. splice and renumber
    const int64_t U = (int64_t)n_nodes_old + nf - K;
    if (U < 1 || U > 2 * (int64_t)S->n - 1) return MSA_EINVAL;
    SpliceArgs a{};
    a.o = ot;
    a.froot = w.froot;
    a.fl = w.fleft; a.fr = w.fright; a.fc = w.fcenter; a.flp = w.flpole; a.frp = w.frpole;
    a.fperm = w.fperm; a.fms = w.fmstart; a.fmc = w.fmcount;
    a.K = K;
    a.nf = nf;
    a.bfs = w.bfs;
    a.lvl = w.lvl;
    a.out = *T_new;
    a.cap = 2 * S->n - 1;
    a.n = S->n;
    a.total = w.total;
    a.st = d_status;
    hipLaunchKernelGGL(k_splice, dim3(1), dim3(1024), 0, s, a);
    if ((rc = launch_status())) return rc;
    int32_t total = 0;
    if ((rc = read_i32(w.total, &total, s))) return rc;
    *n_nodes_new = total;
    return MSA_OK;
}

}  // extern "C"
