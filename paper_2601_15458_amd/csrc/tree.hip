// Alg. 1 (Partition, Sec. 2.1) on the GPU, one tree level at a time.
//
// All clusters of one depth are split together.  Per level:
//   1. medoid: row sums S[x] = sum_y f(x, y) over every pair of every
//      cluster (the triangle of each cluster, each distance added to both
//      ends), then c = the member with the least sum;
//   2. l = argmax_x f(c, x) (in the pruned mode without a pass of its own:
//      the candidate pass also keeps each candidate's farthest member);
//   3. r = argmax_x f(l, x) (f(l, .) kept);
//   4. f(r, .); 5. stable split: L = {x : f(l,x) <= f(r,x)}, R = the rest;
//   6. children numbered breadth-first (L before R) after the level.
// Ties: the least sum / the largest distance with the lowest input index
// wins, encoded in 64-bit keys so that one min/max decides both.  A cluster
// whose radius max_x f(c, x) is 0 (copies of one sequence) stays a leaf.
//
// Sequences are staged once in length order; a cluster's members stay in
// that order through the stable splits, so the 64 texts of a wavefront have
// nearly equal lengths.  The distance passes are the persistent bit-parallel
// kernels of lev_core.hpp with per-level work lists derived on the device.
// Every size a level needs lives in device memory, so the level's ~20
// launches can be captured once into a HIP graph and replayed per level;
// the host reads one 4-byte split count per level to know when to stop.
#include "lev_core.hpp"
#include "lev_xl.hpp"

namespace msadp {

enum { kMedoid = 0, kPoleMax = 1, kPoleMaxStore = 2, kPoleStore = 3, kCandSum = 4,
       kPivotSum = 5 };

// Surrogate-pruned medoid: clusters above exact_below members get exact row
// sums for their topk best-ranked members only.  The embeddings are
// quantized once per call to int8 codes with one power-of-two scale 2^s for
// the whole set: with M = max |e| over every coordinate, s = 6 - floor(log2 M)
// clamped to [kEmbShiftMin, kEmbShiftMax] (M below 2^(6 - kEmbShiftMax): s =
// kEmbShiftMax), so M 2^s lies in [64, 128); a coordinate's code is
// rint(e 2^s) clamped to +-127.  The surrogate distance of two members is
// then sqrt(D) 2^-s with D = |c_x - c_y|^2 an exact integer (below 2^24,
// exact in float32; its Gram part runs on the int8 matrix cores), in float32:
// the square root (correctly rounded), the scaling (exact), the cap at
// kEmbCap and the rounding of 2^16 times it to an integer.  Exact integers
// up to one float32 square root make the ranking reproducible, and the row
// sums are integers.
constexpr int kMaxTopk = 1024;
constexpr uint32_t kMaxEmbOffset = 1u << 31;   // 2^15 in units of 2^-16
constexpr float kEmbScale = 65536.0f;   // fixed point of embedding distances (2^16)
constexpr float kEmbCap = 32768.0f;     // embedding distances saturate here
constexpr int kEmbDim = 128;
constexpr int kEmbShiftMin = -20, kEmbShiftMax = 40;
constexpr float kEmbCodeMax = 127.0f;

struct TreeArgs {
    Staged S;
    const int32_t *order;    // rank -> input index
    const int32_t *rank_of;  // input index -> rank
    int32_t *perm;           // position -> rank (current level)
    int32_t *perm_next;
    int32_t *parent, *left, *right, *center, *lpole, *rpole, *depth;
    int64_t *mstart, *mcount;
    int32_t *desc;           // [0] level start, [1] level end, [2] splits of last level
    int64_t *cnt;            // per cluster item count of the next pass (nq + 1)
    int64_t *items;          // exclusive prefix of cnt (read by the pass)
    int64_t *pitems;         // exclusive prefix of the pairs given to k_tree_xl (nq + 1)
    uint64_t *key;           // per cluster min/max key
    int32_t *pat;            // per cluster pattern rank of the current pass
    int32_t *nleft;          // per cluster |L| (or -1 when it stays a leaf)
    int64_t *split;          // per cluster 1 if split -> exclusive prefix
    uint64_t *rowsum;        // per position
    int32_t *dl, *dr;        // per position f(l, x), f(r, x)
    uint32_t *counter;       // [0] k_tree_lev's work counter, [1] k_tree_xl's
    uint32_t *hbuf;
    int64_t hstride;
    int32_t *st;             // device status
    int32_t sigma;
    int32_t n;
    // surrogate-pruned medoid (emb == nullptr: exact medoid)
    const float *emb;        // [n][128] by input index
    int8_t *embq;            // [n][128] int8 codes by input index
    int32_t *embn;           // [n] squared norms of the codes
    uint32_t *emb_max;       // [2]: bits of max |e|, quantization shift s
    uint32_t emb_q0;         // calibration offset added to every surrogate distance
    int32_t pivots;          // sampled median: pivots per cluster (0: not sampled)
    // clusters of at most this many members take their medoid / candidate /
    // pivot passes (xl_sum) and their pole passes (xl_pole) in k_tree_xl
    int32_t xl_sum, xl_pole;
    int32_t topk;
    int32_t exact_below;     // clusters of at most this many members: all are candidates
    int64_t *ncand;          // per cluster candidate count (nq + 1)
    int64_t *coff;           // exclusive prefix of ncand: the cluster's first candidate
    int32_t *cand;           // [n] candidate ranks, cluster by cluster
    uint64_t *candsum;       // [n] exact row sums of the candidates
    // [n] per candidate y the largest far key (f(y, x) << 32 | ~order(x))
    // over the cluster's members x, y itself included
    uint64_t *candkey;
};

constexpr int kClusterGrid = 2048;

__device__ __forceinline__ int32_t level_clusters(const int32_t *desc) { return desc[1] - desc[0]; }

// largest q in [0, nq) with prefix[q] <= g
__device__ __forceinline__ int32_t find_cluster(const int64_t *prefix, int32_t nq, int64_t g) {
    int32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Tiles of 64 x 64 members (I <= J) over the upper triangle of a cluster of
// k members, row by row: tile_rows_before(I, nb) tiles precede row I.
__host__ __device__ inline int64_t tile_rows_before(int64_t I, int64_t nb) {
    return I * nb - I * (I - 1) / 2;
}

__host__ __device__ inline int64_t emb_tiles(int64_t k) {
    const int64_t nb = (k + 63) / 64;
    return k >= 2 ? nb * (nb + 1) / 2 : 0;
}

// Key of the farthest member: the larger distance wins, then the lower input
// index (the tie rule of the poles).
__device__ __forceinline__ uint64_t far_key(int d, int32_t order_y) {
    return ((uint64_t)(uint32_t)d << 32) | (0xFFFFFFFFu - (uint32_t)order_y);
}

// The median is pruned (a ranking picks its candidates): by the embedding
// or by sampled pivots.
__device__ __forceinline__ bool ranked(const TreeArgs &a) {
    return a.emb != nullptr || a.pivots > 0;
}

// Pivot order of the sampled median: MurmurHash3's 32-bit finalizer
// (Appleby), a bijection of the input index, so no two members tie.
__device__ __forceinline__ uint32_t pivot_hash(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Level start: reset per-node fields, member sums and the medoid work list.
__global__ void __launch_bounds__(256) k_level_init(TreeArgs a) {
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int32_t v = lvl + q;
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        // at most max(exact_below, topk) members: every member is a
        // candidate and no ranking is needed
        const bool pruned = ranked(a) && k > a.exact_below && k > a.topk;
        if (threadIdx.x == 0) {
            a.left[v] = a.right[v] = a.lpole[v] = a.rpole[v] = -1;
            a.key[q] = ~0ull;
            if (a.emb != nullptr) {
                a.cnt[q] = pruned ? emb_tiles(k) : 0;
                a.ncand[q] = pruned ? a.topk : k;
            } else if (a.pivots > 0) {
                // first the pivots; the candidates' count is set after them
                a.cnt[q] = 0;
                a.ncand[q] = pruned ? min<int64_t>(a.pivots, k) : k;
            } else {
                a.cnt[q] = k >= 2 ? items_upto(k - 1) : 0;
            }
            a.nleft[q] = -1;
            a.split[q] = 0;
        }
        // the sampled median picks its pivots by the least hash: the hash
        // stands in the estimate slot until the pivot pass
        const bool hashed = pruned && a.pivots > 0;
        for (int64_t i = threadIdx.x; i < k; i += blockDim.x)
            a.rowsum[ms + i] = hashed ? pivot_hash((uint32_t)a.order[a.perm[ms + i]]) : 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.cnt[nq] = 0;
        a.split[nq] = 0;
        if (ranked(a)) a.ncand[nq] = 0;
    }
}

// out[i] = sum of in[0 .. i) for i <= nq (one workgroup; in == out allowed).
__global__ void __launch_bounds__(1024) k_scan_level(const int64_t *in, int64_t *out,
                                                     const int32_t *desc) {
    __shared__ int64_t part[1024];
    const int64_t n = (int64_t)level_clusters(desc) + 1;
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk, hi = min(n, lo + chunk);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += in[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = in[i];
        out[i] = run;
        run += v;
    }
}

// Classes of distance passes, for the split of their work between the kernels.
enum { kClsMedoid = 0, kClsSum = 1, kClsPole = 2 };

// Work of one distance pass, split by cluster size: a cluster of at most the
// class's cap members (xl_sum or xl_pole) goes to k_tree_xl as pairs, a
// larger one to k_tree_lev as cnt[q] items (cnt as set by the kernel that
// chose the pass's patterns; 0 = no work).  Pairs per cluster of k members:
// the medoid triangle k (k - 1) / 2; a candidate or pivot pass (cnt = count
// x ceil(k / 64) items) count x k, or the triangle when every member is a
// candidate; a pole pass k.  items and pitems get the
// exclusive prefixes, q = 0 .. nq (one workgroup).  It also clears both
// kernels' work counters for the pass.
__global__ void __launch_bounds__(1024) k_scan_work(TreeArgs a, int cls) {
    __shared__ int64_t part[2][1024];
    if (threadIdx.x < 2) a.counter[threadIdx.x] = 0;
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    const int64_t n = (int64_t)nq + 1;
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = min<int64_t>(n, t * chunk), hi = min<int64_t>(n, lo + chunk);
    const int64_t cap = cls == kClsPole ? a.xl_pole : a.xl_sum;
    auto work = [&](int64_t q, int64_t &it, int64_t &pr) {
        it = pr = 0;
        if (q >= nq) return;
        const int64_t c = a.cnt[q];
        if (c == 0) return;
        const int64_t k = a.mcount[lvl + q];
        // a candidate pass over a cluster whose every member is a candidate
        // (at most topk or exact_below members) takes its triangle: each
        // distance once, credited to both members
        const bool all_cand = cls == kClsSum && (k <= a.exact_below || k <= a.topk);
        if (k > cap) {
            it = all_cand ? items_upto(k - 1) : c;
            return;
        }
        pr = cls == kClsMedoid || all_cand ? k * (k - 1) / 2
             : cls == kClsSum              ? c / ((k + 63) / 64) * k
                                           : k;
    };
    int64_t si = 0, sp = 0;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t it, pr;
        work(i, it, pr);
        si += it;
        sp += pr;
    }
    part[0][t] = si;
    part[1][t] = sp;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v0 = t >= off ? part[0][t - off] : 0;
        const int64_t v1 = t >= off ? part[1][t - off] : 0;
        __syncthreads();
        part[0][t] += v0;
        part[1][t] += v1;
        __syncthreads();
    }
    int64_t ri = part[0][t] - si, rp = part[1][t] - sp;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t it, pr;
        work(i, it, pr);
        a.items[i] = ri;
        a.pitems[i] = rp;
        ri += it;
        rp += pr;
    }
}

// The distance passes of a level.
template <int WMAX, int MODE>
__global__ void __launch_bounds__(64) k_tree_lev(TreeArgs a) {
    __shared__ uint64_t peq[WMAX * kSym];
    const int lane = lane_id();
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    const int64_t total = a.items[nq];
    // A level never holds more work than n patterns against all n members
    // (the medoid triangle is half of that; a candidate or pivot pass over
    // every member of a cluster is all of it).
    if (nq < 1 || nq > a.n || total < 0 || total > (int64_t)a.n * ((a.n + 63) / 64)) {
        if (blockIdx.x == 0 && lane == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    uint32_t *hb = a.hbuf ? a.hbuf + (int64_t)blockIdx.x * a.hstride * kWave + lane : nullptr;
    for (uint32_t it = first_item();; it = later_item(a.counter)) {
        if ((int64_t)it >= total) break;
        const int32_t q = find_cluster(a.items, nq, it);
        const int64_t local = (int64_t)it - a.items[q];
        const int32_t v = lvl + q;
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        int64_t tpos, prow_pos = -1;
        int32_t prow;
        int64_t cslot = 0;
        int64_t tend = ms + k;                   // texts are positions [.., tend)
        // a candidate pass over a cluster whose every member is a candidate
        // (candidate i = member i) takes the medoid triangle: each distance
        // once, credited to both members
        const bool tri = MODE == kMedoid ||
                         (MODE == kCandSum && (k <= a.exact_below || k <= a.topk));
        if (tri) {
            // Member u (the longer of each pair: members are in length order)
            // is the pattern of members 0 .. u-1, which cost fewer bit
            // columns than the other way round and round up fewer rows; the
            // members with the most texts come first.
            const int64_t r = items_upto(k - 1) - 1 - local;
            const int64_t u = triangle_row(r, k - 1);
            const int64_t blk = r - items_upto(u - 1);
            prow_pos = ms + u;
            prow = a.perm[prow_pos];
            tpos = ms + blk * 64 + lane;
            tend = ms + u;
            cslot = a.coff[q] + u;
        } else if (MODE == kCandSum || MODE == kPivotSum) {
            const int64_t nblk = (k + 63) / 64;
            const int64_t j = local / nblk, blk = local % nblk;
            cslot = a.coff[q] + j;
            prow = a.cand[cslot];
            tpos = ms + blk * 64 + lane;
        } else {
            prow = a.pat[q];
            tpos = ms + local * 64 + lane;
        }
        const bool valid = tpos < tend;
        const int32_t trow = a.perm[valid ? tpos : ms];
        const int d = lev_item<WMAX>(peq, a.S.codes + (int64_t)prow * a.S.stride, a.S.len[prow],
                                     a.sigma, a.S.codes + (int64_t)trow * a.S.stride,
                                     a.S.len[trow], valid, hb);
        // The epilogue has no lane-dependent branch (see next_item): lanes
        // without a pair write to the spare slot n or add zero.
        const int64_t slot = valid ? tpos : (int64_t)a.n;
        // the far key of the pattern row over this item's texts
        const uint64_t key = valid ? far_key(d, a.order[trow]) : 0ull;
        if (MODE == kMedoid) {
            atomicAdd((unsigned long long *)&a.rowsum[slot],
                      (unsigned long long)(valid ? d : 0));
            const uint64_t s = wave_sum_u64(valid ? (uint64_t)d : 0ull);
            atomicAdd((unsigned long long *)&a.rowsum[prow_pos],
                      (unsigned long long)(lane == 0 ? s : 0ull));
        }
        if (MODE == kPoleMax || MODE == kPoleMaxStore) {
            const uint64_t m = wave_max_u64(key);
            atomicMax((unsigned long long *)&a.key[q], (unsigned long long)m);
        }
        if (MODE == kCandSum) {
            const uint64_t s = wave_sum_u64(valid ? (uint64_t)d : 0ull);
            atomicAdd((unsigned long long *)&a.candsum[cslot],
                      (unsigned long long)(lane == 0 ? s : 0ull));
            const uint64_t m = wave_max_u64(key);
            atomicMax((unsigned long long *)&a.candkey[cslot],
                      (unsigned long long)(lane == 0 ? m : 0ull));
            if (tri) {   // uniform: the texts' side of the triangle pairs
                const int64_t ts = a.coff[q] + ((valid ? tpos : ms) - ms);
                atomicAdd((unsigned long long *)&a.candsum[ts],
                          (unsigned long long)(valid ? d : 0));
                atomicMax((unsigned long long *)&a.candkey[ts],
                          (unsigned long long)(valid ? far_key(d, a.order[prow]) : 0ull));
            }
        }
        if (MODE == kPivotSum)
            atomicAdd((unsigned long long *)&a.rowsum[slot], (unsigned long long)(valid ? d : 0));
        if (MODE == kPoleMaxStore) a.dl[slot] = d;
        if (MODE == kPoleStore) a.dr[slot] = d;
    }
}

// The same distance passes for the clusters k_scan_work gave to pairs: one
// pair per group of G lanes (lev_xl.hpp), kWave / G consecutive pairs of the
// pitems numbering per work item, so one wavefront serves several small
// clusters at once, and a pair takes about n + G steps instead of the n
// times pattern-words steps of one lane.  The group's lane 0 adds the
// pair's distance where the pass keeps it.
// Workgroups of four independent wavefronts (a quarter of the workgroups to
// dispatch for the same resident wavefronts).
constexpr int kXlBlock = 256;

template <int G, int WL, int NB>
__global__ void __launch_bounds__(kXlBlock) k_tree_xl(TreeArgs a, int mode) {
    constexpr int kPpw = kWave / G;
    const int lane = lane_id(), grp = lane / G;
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    const int64_t total = a.pitems[nq];
    // a pair list never exceeds n members times the largest cluster it holds
    const int64_t cap = max(a.xl_sum, a.xl_pole);
    if (nq < 1 || nq > a.n || total < 0 || total > (int64_t)a.n * cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    for (uint32_t it = first_item();; it = later_item(a.counter + 1)) {
        const int64_t p0 = (int64_t)it * kPpw;
        if (p0 >= total) break;
        const bool live = p0 + grp < total;
        const int64_t p = live ? p0 + grp : p0;
        const int32_t q = find_cluster(a.pitems, nq, p);
        const int64_t L = p - a.pitems[q];
        const int32_t v = lvl + q;
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        int64_t tpos, ppos = 0, cslot = 0, tslot = 0;
        int32_t prow;
        // candidate pass of a cluster whose members are all candidates
        // (candidate i = member i): its triangle, as the medoid pass
        const bool tri = mode == kMedoid ||
                         (mode == kCandSum && (k <= a.exact_below || k <= a.topk));
        if (tri) {
            // triangle pair L = u (u - 1) / 2 + t, t < u: member u (the
            // longer one, members being in length order) is the pattern
            int64_t u = (int64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)L)) * 0.5f);
            while (u > 1 && u * (u - 1) / 2 > L) --u;
            while ((u + 1) * u / 2 <= L) ++u;
            ppos = ms + u;
            prow = a.perm[ppos];
            tpos = ms + (L - u * (u - 1) / 2);
            cslot = a.coff[q] + u;
            tslot = a.coff[q] + (tpos - ms);
        } else if (mode == kCandSum || mode == kPivotSum) {
            const int64_t jj = L / k;
            cslot = a.coff[q] + jj;
            prow = a.cand[cslot];
            tpos = ms + (L - jj * k);
        } else {
            prow = a.pat[q];
            tpos = ms + L;
        }
        const int32_t trow = a.perm[tpos];
        // the longer sequence of the pair is the pattern (the distance is
        // symmetric): the group's lanes hold the set's longest pattern
        // anyway, and the steps follow the shorter one
        const int32_t lp = a.S.len[prow], lt = a.S.len[trow];
        const bool sw = lt > lp;
        const int32_t xr = sw ? trow : prow, yr = sw ? prow : trow;
        const int d = xl_distance<G, WL, NB>(a.S.codes + (int64_t)xr * a.S.stride, sw ? lt : lp,
                                             a.S.codes + (int64_t)yr * a.S.stride, sw ? lp : lt,
                                             a.S.stride - 16, live);
        // Pairs of one cluster (pole keys), one candidate (candidate sums and
        // keys) or one pattern member (medoid sums of the longer member) are
        // consecutive: their values are first combined across the
        // wavefront's groups, so each run costs one atomic, not one per pair.
        const bool lead = live && (lane & (G - 1)) == 0;
        const uint64_t fk = far_key(d, a.order[trow]);
        bool head = false;
        if (mode == kMedoid) {
            const uint64_t sp = xl_segment<G, false>(live ? ppos : -1, (uint64_t)d, head);
            if (lead) atomicAdd((unsigned long long *)&a.rowsum[tpos], (unsigned long long)d);
            if (lead && head) atomicAdd((unsigned long long *)&a.rowsum[ppos], (unsigned long long)sp);
        } else if (mode == kPivotSum) {
            if (lead) atomicAdd((unsigned long long *)&a.rowsum[tpos], (unsigned long long)d);
        } else if (mode == kCandSum) {
            const uint64_t ss = xl_segment<G, false>(live ? cslot : -1, (uint64_t)d, head);
            const uint64_t sk = xl_segment<G, true>(live ? cslot : -1, fk, head);
            if (lead && head) {
                atomicAdd((unsigned long long *)&a.candsum[cslot], (unsigned long long)ss);
                atomicMax((unsigned long long *)&a.candkey[cslot], (unsigned long long)sk);
            }
            if (lead && tri) {   // the other member of a triangle pair
                atomicAdd((unsigned long long *)&a.candsum[tslot], (unsigned long long)d);
                atomicMax((unsigned long long *)&a.candkey[tslot],
                          (unsigned long long)far_key(d, a.order[prow]));
            }
        } else {
            if (mode == kPoleMax || mode == kPoleMaxStore) {
                const uint64_t sk = xl_segment<G, true>(live ? q : -1, fk, head);
                if (lead && head)
                    atomicMax((unsigned long long *)&a.key[q], (unsigned long long)sk);
            }
            if (lead && mode == kPoleMaxStore) a.dl[tpos] = d;
            if (lead && mode == kPoleStore) a.dr[tpos] = d;
        }
    }
}

// c = member with the least row sum (lowest input index on ties).
__global__ void __launch_bounds__(256) k_pick_center(TreeArgs a) {
    __shared__ uint64_t red[256];
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int32_t v = lvl + q;
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        uint64_t best = ~0ull;
        for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
            const int32_t orig = a.order[a.perm[ms + i]];
            const uint64_t key = (a.rowsum[ms + i] << 24) | (uint64_t)orig;
            best = key < best ? key : best;
        }
        red[threadIdx.x] = best;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if (threadIdx.x < o) {
                const uint64_t w = red[threadIdx.x + o];
                if (w < red[threadIdx.x]) red[threadIdx.x] = w;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int32_t c = (int32_t)(red[0] & 0xFFFFFFull);
            a.center[v] = c;
            a.pat[q] = a.rank_of[c];
            a.key[q] = 0;
            a.cnt[q] = k >= 2 ? (k + 63) / 64 : 0;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[nq] = 0;
}

// After a pole pass: decode the argmax into the next pattern.  `which` 0:
// l (a zero radius turns the cluster into a leaf), 1: r.
__global__ void k_pick_pole(TreeArgs a, int which) {
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const int32_t v = lvl + q;
        const int64_t k = a.mcount[v];
        if (a.cnt[q] == 0) continue;            // no work in the last pass: a leaf
        const uint64_t key = a.key[q];
        const int32_t far = (int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
        const uint32_t dmax = (uint32_t)(key >> 32);
        a.key[q] = 0;
        if (which == 0 && dmax == 0) {
            a.cnt[q] = 0;
            continue;
        }
        if (which == 0) a.lpole[v] = far; else a.rpole[v] = far;
        a.pat[q] = a.rank_of[far];
        a.cnt[q] = (k + 63) / 64;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[nq] = 0;
}

// Stable split of every cluster that has both poles: L = f(l,x) <= f(r,x).
// One workgroup per cluster: a count of L, then chunks of 256 members whose
// destinations come from a ballot prefix inside each wavefront and the
// wavefronts' counts (double-buffered, so one barrier per chunk).
constexpr int kSplitThreads = 256;
constexpr int kSplitWaves = kSplitThreads / kWave;

__global__ void __launch_bounds__(kSplitThreads) k_split(TreeArgs a) {
    __shared__ int32_t sc[kSplitThreads];
    __shared__ int32_t wsum[2][kSplitWaves];
    const int t = threadIdx.x, w = t / kWave;
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int32_t v = lvl + q;
        if (a.rpole[v] < 0) continue;   // uniform per block
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        int32_t cnt = 0;
        for (int64_t i = t; i < k; i += kSplitThreads) cnt += a.dl[ms + i] <= a.dr[ms + i];
        sc[t] = cnt;
        __syncthreads();
        for (int o = kSplitThreads / 2; o >= 1; o >>= 1) {
            if (t < o) sc[t] += sc[t + o];
            __syncthreads();
        }
        const int32_t nl = sc[0];
        int64_t base_l = 0, base_r = nl;   // the same in every thread
        int buf = 0;
        for (int64_t c0 = 0; c0 < k; c0 += kSplitThreads) {
            const int64_t i = c0 + t;
            const bool f = i < k && a.dl[ms + i] <= a.dr[ms + i];
            const uint64_t m = __ballot(f);
            const int before_w = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if ((t & (kWave - 1)) == 0) wsum[buf][w] = __popcll(m);
            __syncthreads();
            int32_t before_l = before_w, chunk_l = 0;
#pragma unroll
            for (int x = 0; x < kSplitWaves; ++x) {
                const int32_t c = wsum[buf][x];
                chunk_l += c;
                before_l += x < w ? c : 0;
            }
            if (i < k) {
                const int64_t dst = f ? ms + base_l + before_l
                                      : ms + base_r + (t - before_l);
                a.perm_next[dst] = a.perm[ms + i];
            }
            base_l += chunk_l;
            base_r += min<int64_t>(kSplitThreads, k - c0) - chunk_l;
            buf ^= 1;
        }
        if (t == 0) {
            a.nleft[q] = nl;
            a.split[q] = 1;
        }
        __syncthreads();   // sc and wsum are reused by the next cluster
    }
}

__global__ void k_make_children(TreeArgs a) {
    const int32_t lvl = a.desc[0], end = a.desc[1], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        if (a.nleft[q] < 0) continue;
        const int32_t v = lvl + q;
        const int32_t c0 = end + 2 * (int32_t)a.split[q], c1 = c0 + 1;
        const int64_t ms = a.mstart[v], k = a.mcount[v], nl = a.nleft[q];
        a.left[v] = c0;
        a.right[v] = c1;
        a.parent[c0] = a.parent[c1] = v;
        a.depth[c0] = a.depth[c1] = a.depth[v] + 1;
        a.mstart[c0] = ms;
        a.mcount[c0] = nl;
        a.mstart[c1] = ms + nl;
        a.mcount[c1] = k - nl;
    }
}

__global__ void k_next_level(TreeArgs a) {
    const int32_t nq = level_clusters(a.desc);
    const int32_t s = (int32_t)a.split[nq];
    a.desc[2] = s;
    a.desc[0] = a.desc[1];
    a.desc[1] = a.desc[1] + 2 * s;
}

__global__ void k_tree_root(TreeArgs a) {
    a.parent[0] = -1;
    a.depth[0] = 0;
    a.mstart[0] = 0;
    a.mcount[0] = a.n;
    a.desc[0] = 0;
    a.desc[1] = 1;
    a.desc[2] = 0;
}

// Level 0 of a forest: K root clusters whose members (input indices) fill
// positions fstart[f] .. fstart[f+1) of mem, one cluster after another.
__global__ void __launch_bounds__(256) k_forest_root(TreeArgs a, int32_t K, const int32_t *mem,
                                                    const int64_t *fstart, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        const int32_t x = mem[i];
        const bool ok = x >= 0 && x < a.n;
        if (!ok) set_status(a.st, MSA_DS_INDEX);
        a.perm[i] = a.rank_of[ok ? x : 0];
    }
    if (i < K) {
        a.parent[i] = -1;
        a.depth[i] = 0;
        a.mstart[i] = fstart[i];
        a.mcount[i] = fstart[i + 1] - fstart[i];
    }
    if (i == 0) {
        a.desc[0] = 0;
        a.desc[1] = K;
        a.desc[2] = 0;
    }
}

__global__ void k_rank_of(const int32_t *order, int32_t n, int32_t *rank_of, int32_t *perm) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    rank_of[order[r]] = r;
    perm[r] = r;
}

__global__ void k_perm_out(const int32_t *order, const int32_t *perm, int32_t n, int32_t *out) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = order[perm[r]];
}

// Members of a given tree: perm (input indices) to ranks; out-of-range
// entries are reported and read as rank 0.
__global__ void k_perm_in(const int32_t *perm_in, const int32_t *rank_of, int32_t n,
                          int32_t *perm, int32_t *st) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t x = perm_in[i];
    const bool ok = x >= 0 && x < n;
    if (!ok) set_status(st, MSA_DS_INDEX);
    perm[i] = rank_of[ok ? x : 0];
}

__global__ void k_set_desc(int32_t *desc, int32_t lo, int32_t hi) {
    desc[0] = lo;
    desc[1] = hi;
    desc[2] = 0;
}

// Quantization of the embeddings (see kEmbShiftMin above).  maxbits = the
// bit pattern of M = max |e| (a non-negative float orders like its bits).
__device__ __forceinline__ int emb_shift_of(uint32_t maxbits) {
    // M < 2^(6 - kEmbShiftMax), zero and subnormals included: the largest shift
    if (maxbits < ((uint32_t)(127 + 6 - kEmbShiftMax) << 23)) return kEmbShiftMax;
    const int L = (int)(maxbits >> 23) - 127;   // floor(log2 M) of a normal M
    return min(max(6 - L, kEmbShiftMin), kEmbShiftMax);
}

// 2^e for e in [-kEmbShiftMax, 16 - kEmbShiftMin] (a normal float).
__device__ __forceinline__ float pow2f(int e) { return __uint_as_float((uint32_t)(127 + e) << 23); }

__global__ void k_emb_reset(uint32_t *emb_max) {
    emb_max[0] = 0;
    emb_max[1] = 0;
}

// emb_max[0] = bits of max |e| over the n x 128 coordinates.
__global__ void __launch_bounds__(256) k_emb_absmax(const float *emb, int64_t count,
                                                   uint32_t *emb_max) {
    uint32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(emb[i]) & 0x7FFFFFFFu);
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, kWave));
    if (lane_id() == 0) atomicMax(emb_max, m);
}

// Codes and squared code norms; a thread quantizes 4 coordinates of a row.
__global__ void __launch_bounds__(256) k_emb_quantize(const float *emb, int32_t n,
                                                     const uint32_t *emb_max, int8_t *embq,
                                                     int32_t *embn, int32_t *st) {
    const uint32_t mb = emb_max[0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && mb >= 0x7F800000u) set_status(st, MSA_DS_VALUE);
    const float scale = pow2f(emb_shift_of(mb));
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // n * 32 threads
    const int64_t row = t >> 5;
    int32_t sq = 0;
    if (row < n) {
        const float4 e = ((const float4 *)emb)[t];
        const float ev[4] = {e.x, e.y, e.z, e.w};
        uint32_t packed = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float v = fminf(fmaxf(rintf(ev[c] * scale), -kEmbCodeMax), kEmbCodeMax);
            const int32_t code = (int32_t)v;
            sq += code * code;
            packed |= ((uint32_t)code & 0xFFu) << (8 * c);
        }
        ((uint32_t *)embq)[t] = packed;
    }
    for (int o = 16; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 32);
    if (row < n && (t & 31) == 0) embn[row] = sq;
}

typedef int32_t v4i32 __attribute__((ext_vector_type(4)));

// Correctly rounded float32 square root of an integer 0 <= x < 2^24.  The
// hardware square root r lies within one unit in the last place of the
// exact one (true on every such integer), so the answer is r or a
// neighbour: with m and p the floats below and above r, x <= m r means
// sqrt(x) is below the midpoint of m and r, and x > p r that it is above
// the midpoint of r and p; both products of 24-bit significands are exact
// inside the fused multiply-add, and an integer x never falls strictly
// between m r and that midpoint (nor between p r and the other one), so
// the sign tests decide exactly.  x = 0 gives r = 0 and neither test fires.
__device__ __forceinline__ float sqrt_int_rn(float x) {
    const float r = __builtin_amdgcn_sqrtf(x);
    const float m = __uint_as_float(__float_as_uint(r) - 1u);
    const float p = __uint_as_float(__float_as_uint(r) + 1u);
    const bool down = __builtin_fmaf(-m, r, x) <= 0.0f;
    const bool upw = __builtin_fmaf(-p, r, x) > 0.0f;
    return down ? m : (upw ? p : r);
}

// Row sums of one row tile of the Gram block: G[ta][tb][r] pairs x member
// 16 ta + 4 g + r with y member 16 tb + l16 of their blocks.
template <bool kCols>
__device__ __forceinline__ void emb_tile_epilogue(
    const v4i32 (&G)[4][4], int ta, int g, int l16, const int32_t *xn, const uint32_t *xl,
    const uint32_t *xm, const int32_t (&ny)[4], const uint32_t (&ly)[4], const uint32_t (&ym)[4],
    float qscale, uint64_t q0, uint64_t (&cs)[4], uint32_t (&cw)[4], uint64_t *red_r) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * ta + 4 * g + r;
        const int32_t nx = xn[row];
        const uint32_t lx = xl[row], mx = xm[row];
        uint64_t rs = 0;
        uint32_t rw = 0;
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
            const int32_t d2 = nx + ny[tb] - 2 * G[ta][tb][r];   // |c_x - c_y|^2, exact
            // min(sqrt 2^-s, 2^15) 2^16 = min(sqrt 2^(16-s), 2^31): power-of-two
            // scalings of normal floats are exact
            const float dq = sqrt_int_rn((float)d2) * qscale;
            const uint32_t qd = (uint32_t)rintf(fminf(dq, kEmbCap * kEmbScale));
            const uint32_t w = (lx + ly[tb]) & mx & ym[tb];
            rs += (uint64_t)qd * w;
            rw += w;
            if (kCols) {
                cs[tb] += (uint64_t)qd * w;
                cw[tb] += w;
            }
        }
        red_r[row * 17 + l16] = rs + q0 * rw;
    }
}

// Estimated medoid row sums from the embeddings.  The embedder is trained
// so that ||e_x - e_y|| predicts f(x, y) divided by the pair's mean length;
// with a linear recalibration of that prediction (offset emb_q0, the slope
// drops out of the ranking) the estimate of f(x, y) is proportional to
// (||e_x - e_y|| + offset) (|x| + |y|).  Every ordered pair of a cluster, x
// with itself included, adds it to the row sum of x.  One work item is a
// 64 x 64 tile (I, J) of the cluster's upper block triangle: the Gram block
// of the int8 codes of blocks I and J (128 coordinates) takes 32 int8 MFMAs
// (16 x 16 x 64, exact int32), then every pair's distance, weight and
// product; row sums go through LDS to one lane per member, and for I < J so
// do the column sums.  A diagonal tile visits every ordered pair of its
// block and adds row sums only.  The q0 part of a sum is q0 times the summed
// weights.
// Where tile `it` of the level lies, and what lane L needs of it: member L
// of block I (x) and of block J (y), by rank, input index, norm and length.
struct EmbTile {
    int64_t ms, k, I, J;
    int32_t xr, yr, xo, yo, xn, yn;
    bool xv, yv;
};

__device__ __forceinline__ EmbTile emb_locate(const TreeArgs &a, int32_t lvl, int32_t nq,
                                              int64_t it, int lane) {
    EmbTile t;
    const int32_t q = find_cluster(a.items, nq, it);
    const int64_t local = it - a.items[q];
    t.ms = a.mstart[lvl + q];
    t.k = a.mcount[lvl + q];
    const int64_t nb = (t.k + 63) / 64;
    int64_t lo = 0, hi = nb - 1;            // row I of the tile
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (tile_rows_before(mid, nb) <= local) lo = mid; else hi = mid - 1;
    }
    t.I = lo;
    t.J = lo + (local - tile_rows_before(lo, nb));
    const int64_t xi = t.I * 64 + lane, yi = t.J * 64 + lane;
    t.xv = xi < t.k;
    t.yv = yi < t.k;
    t.xr = a.perm[t.ms + (t.xv ? xi : 0)];
    t.yr = a.perm[t.ms + (t.yv ? yi : 0)];
    t.xo = a.order[t.xr];
    t.yo = a.order[t.yr];
    t.xn = a.embn[t.xo];
    t.yn = a.embn[t.yo];
    return t;
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_emb_rowsum(TreeArgs a) {
    __shared__ uint64_t red_r[64 * 17];    // row partials (16 per member, padded)
    __shared__ uint64_t red_c[64 * 4];     // column partials (4 per member)
    __shared__ int32_t xo_s[64], yo_s[64], xn_s[64];
    __shared__ uint32_t xl_s[64], xm_s[64];
    const int lane = lane_id();
    const int l16 = lane & 15, g = lane >> 4;
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    const int64_t total = a.items[nq];
    // Clusters of a level are disjoint, so their tiles number at most n(n+1)/2.
    if (nq < 1 || nq > a.n || total < 0 || total > (int64_t)a.n * (a.n + 1) / 2) {
        if (blockIdx.x == 0 && lane == 0) set_status(a.st, MSA_DS_CAPACITY);
        return;
    }
    const float qscale = pow2f(16 - emb_shift_of(a.emb_max[0]));   // 2^(16 - s)
    const uint64_t q0 = a.emb_q0;
    // Tiles cost the same, so they are dealt out statically (stride = grid);
    // the next tile's location and member data load while this one computes.
    int64_t it = blockIdx.x;
    EmbTile nxt{};
    if (it < total) nxt = emb_locate(a, lvl, nq, it, lane);
    while (it < total) {
        const EmbTile cur = nxt;
        const int64_t ms = cur.ms, I = cur.I, J = cur.J;
        const int64_t xi = I * 64 + lane, yi = J * 64 + lane;
        const bool xv = cur.xv, yv = cur.yv;
        xo_s[lane] = cur.xo;
        yo_s[lane] = cur.yo;
        xn_s[lane] = cur.xn;
        xl_s[lane] = (uint32_t)a.S.len[cur.xr];
        xm_s[lane] = xv ? ~0u : 0u;
        const int32_t yn_l = cur.yn;
        const uint32_t yl_l = (uint32_t)a.S.len[cur.yr], ym_l = yv ? ~0u : 0u;
        __syncthreads();
        // operands: A row i = x member 16 t + i, B column j = y member 16 t + j;
        // lane group g brings coordinates 16 g .. 16 g + 15 of each 64-wide K step
        v4i32 A[4][2], B[4][2];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4i32 *xp = (const v4i32 *)(a.embq + (int64_t)xo_s[16 * t + l16] * kEmbDim);
            const v4i32 *yp = (const v4i32 *)(a.embq + (int64_t)yo_s[16 * t + l16] * kEmbDim);
            A[t][0] = xp[g];
            A[t][1] = xp[4 + g];
            B[t][0] = yp[g];
            B[t][1] = yp[4 + g];
        }
        v4i32 G[4][4];
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) G[ta][tb] = v4i32{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = 0; tb < 4; ++tb)
                    G[ta][tb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[ta][kk], B[tb][kk],
                                                                      G[ta][tb], 0, 0, 0);
        const int64_t it_next = it + gridDim.x;
        if (it_next < total) nxt = emb_locate(a, lvl, nq, it_next, lane);   // uniform
        // this lane's y members 16 tb + l16: norm, length, validity
        int32_t ny[4];
        uint32_t ly[4], ym[4];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
            ny[tb] = __shfl(yn_l, 16 * tb + l16, kWave);
            ly[tb] = (uint32_t)__shfl((int)yl_l, 16 * tb + l16, kWave);
            ym[tb] = (uint32_t)__shfl((int)ym_l, 16 * tb + l16, kWave);
        }
        uint64_t cs[4] = {0, 0, 0, 0};
        uint32_t cw[4] = {0, 0, 0, 0};
        const bool cols = I != J;                // uniform per item
#pragma unroll
        for (int ta = 0; ta < 4; ++ta) {
            if (cols)
                emb_tile_epilogue<true>(G, ta, g, l16, xn_s, xl_s, xm_s, ny, ly, ym, qscale, q0,
                                        cs, cw, red_r);
            else
                emb_tile_epilogue<false>(G, ta, g, l16, xn_s, xl_s, xm_s, ny, ly, ym, qscale, q0,
                                         cs, cw, red_r);
        }
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) red_c[(16 * tb + l16) * 4 + g] = cs[tb] + q0 * cw[tb];
        __syncthreads();
        uint64_t rsum = 0, csum = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) rsum += red_r[lane * 17 + j];
#pragma unroll
        for (int j = 0; j < 4; ++j) csum += red_c[lane * 4 + j];
        // no lane-dependent branch around the atomics (see next_item)
        atomicAdd((unsigned long long *)&a.rowsum[xv ? ms + xi : (int64_t)a.n],
                  (unsigned long long)(xv ? rsum : 0ull));
        if (cols)
            atomicAdd((unsigned long long *)&a.rowsum[yv ? ms + yi : (int64_t)a.n],
                      (unsigned long long)(yv ? csum : 0ull));
        __syncthreads();
        it = it_next;
    }
}

__device__ __forceinline__ bool key_less(uint64_t s0, uint32_t i0, uint64_t s1, uint32_t i1) {
    return s0 < s1 || (s0 == s1 && i0 < i1);
}

// Ascending bitonic sort of n (a power of two, n <= kTopkSel) keys (e, i)
// in LDS by the whole block.
__device__ void block_sort_keys(uint64_t *e, uint32_t *id, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const bool swap = up ? key_less(e[hi], id[hi], e[lo], id[lo])
                                     : key_less(e[lo], id[lo], e[hi], id[hi]);
                if (swap) {
                    const uint64_t te = e[lo];
                    const uint32_t ti = id[lo];
                    e[lo] = e[hi];
                    id[lo] = id[hi];
                    e[hi] = te;
                    id[hi] = ti;
                }
            }
            __syncthreads();
        }
    }
}

constexpr int kTopkThreads = 256;
constexpr int kTopkSel = 2048;      // members a selection may collect in LDS
static_assert(kMaxTopk <= kTopkSel, "the pivots of a cluster are staged in the selection's LDS");

constexpr uint64_t kPivotFlag = 1ull << 63;

__device__ __forceinline__ uint64_t estimate(uint64_t v, bool sampled, int64_t ps) {
    if (!sampled) return v;
    const bool piv = (v & kPivotFlag) != 0;
    const uint64_t m = piv ? (uint64_t)ps : (uint64_t)(ps > 1 ? ps - 1 : 1);
    return (v & ~kPivotFlag) * m;
}

// Ranking keys (estimate, input index) of members i0 + u blockDim.x, u <
// kTopkUnroll, of the cluster at ms (k members); members past the cluster
// get the largest key, which no comparison selects.
constexpr int kTopkUnroll = 4;

__device__ __forceinline__ void member_keys(const TreeArgs &a, int64_t ms, int64_t k, int64_t i0,
                                            bool sampled, int64_t ps, uint64_t (&sv)[kTopkUnroll],
                                            uint32_t (&oi)[kTopkUnroll]) {
    uint64_t r[kTopkUnroll];
    int32_t pm[kTopkUnroll];
#pragma unroll
    for (int u = 0; u < kTopkUnroll; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        r[u] = i < k ? a.rowsum[ms + i] : 0ull;
        pm[u] = i < k ? a.perm[ms + i] : 0;
    }
#pragma unroll
    for (int u = 0; u < kTopkUnroll; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        oi[u] = i < k ? (uint32_t)a.order[pm[u]] : ~0u;
        sv[u] = i < k ? estimate(r[u], sampled, ps) : ~0ull;
    }
}

// Candidates of each cluster, from its first candidate slot on: every member
// of a cluster of at most max(exact_below, topk) members (one full row sum
// each, which keeps every work item 64 texts wide); otherwise the topk members
// with the least estimated row sum (lowest input index on ties).  Selection:
// each thread takes the least key of its strided share of the members; T =
// the topk-th least of those 256 keys bounds at least topk members (one per
// thread), so the topk least keys are among the members with key <= T, which
// are collected in LDS and sorted.  If topk exceeds the thread count or more
// than kTopkSel members fall under T, topk rounds of a block-wide minimum
// over the members above the last pick are taken instead.  Clears the
// candidates' sums and sets the work of the candidate-sum pass.
// Phase 0 (sampled median) picks the pivots instead, by the hash in the
// estimate slots, in pruned clusters only; it then clears those slots for
// the pivot pass and sets the candidates' count for phase 1.
__global__ void __launch_bounds__(kTopkThreads) k_topk(TreeArgs a, int phase) {
    // Phase 1 of the sampled median ranks by the mean distance to the pivots
    // other than the member itself: sum * s for a pivot, * max(s - 1, 1) for
    // the others (s = the cluster's pivots).
    const bool sampled = phase == 1 && a.emb == nullptr && a.pivots > 0;
    __shared__ uint64_t se[kTopkSel];
    __shared__ uint32_t si[kTopkSel];
    __shared__ uint32_t count;
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int32_t v = lvl + q;
        const int64_t ms = a.mstart[v], k = a.mcount[v];
        const bool small = k <= a.exact_below || k <= a.topk;
        const int64_t ps = min<int64_t>(a.pivots, k);
        if (phase == 0 && small) {         // uniform per block
            if (threadIdx.x == 0) a.cnt[q] = 0;
            continue;
        }
        const int64_t nc = a.ncand[q], base = a.coff[q];
        for (int64_t j = threadIdx.x; j < nc; j += blockDim.x) {
            a.candsum[base + j] = 0;
            a.candkey[base + j] = 0;
        }
        if (small) {
            for (int64_t i = threadIdx.x; i < k; i += blockDim.x) a.cand[base + i] = a.perm[ms + i];
        } else {
            bool done = false;
            if (nc <= kTopkThreads) {
                // least key of this thread's share (four members a round,
                // their loads issued together)
                uint64_t be = ~0ull;
                uint32_t bi = ~0u;
                for (int64_t i0 = threadIdx.x; i0 < k; i0 += kTopkUnroll * blockDim.x) {
                    uint64_t sv[kTopkUnroll];
                    uint32_t oi[kTopkUnroll];
                    member_keys(a, ms, k, i0, sampled, ps, sv, oi);
#pragma unroll
                    for (int u = 0; u < kTopkUnroll; ++u)
                        if (key_less(sv[u], oi[u], be, bi)) { be = sv[u]; bi = oi[u]; }
                }
                se[threadIdx.x] = be;
                si[threadIdx.x] = bi;
                if (threadIdx.x == 0) count = 0;
                __syncthreads();
                block_sort_keys(se, si, kTopkThreads);
                const uint64_t te = se[nc - 1];
                const uint32_t ti = si[nc - 1];
                __syncthreads();
                // every member with key <= (te, ti)
                for (int64_t i0 = threadIdx.x; i0 < k; i0 += kTopkUnroll * blockDim.x) {
                    uint64_t sv[kTopkUnroll];
                    uint32_t oi[kTopkUnroll];
                    member_keys(a, ms, k, i0, sampled, ps, sv, oi);
#pragma unroll
                    for (int u = 0; u < kTopkUnroll; ++u) {
                        if (!key_less(te, ti, sv[u], oi[u])) {
                            const uint32_t slot = atomicAdd(&count, 1u);
                            if (slot < (uint32_t)kTopkSel) {
                                se[slot] = sv[u];
                                si[slot] = oi[u];
                            }
                        }
                    }
                }
                __syncthreads();
                const uint32_t got = count;
                if (got <= (uint32_t)kTopkSel) {
                    int n2 = 1;
                    while (n2 < (int)got) n2 <<= 1;
                    for (int i = (int)got + threadIdx.x; i < n2; i += blockDim.x) {
                        se[i] = ~0ull;
                        si[i] = ~0u;
                    }
                    __syncthreads();
                    block_sort_keys(se, si, n2);
                    for (int64_t j = threadIdx.x; j < nc; j += blockDim.x)
                        a.cand[base + j] = a.rank_of[si[j]];
                    done = true;
                }
                __syncthreads();
            }
            if (!done) {
                uint64_t last_s = 0;
                uint32_t last_i = 0;
                bool have_last = false;
                for (int64_t j = 0; j < nc; ++j) {
                    uint64_t bs = ~0ull;
                    uint32_t bi = ~0u;
                    for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
                        const uint64_t sv = estimate(a.rowsum[ms + i], sampled, ps);
                        const uint32_t oi = (uint32_t)a.order[a.perm[ms + i]];
                        if (have_last && !key_less(last_s, last_i, sv, oi)) continue;
                        if (key_less(sv, oi, bs, bi)) { bs = sv; bi = oi; }
                    }
                    se[threadIdx.x] = bs;
                    si[threadIdx.x] = bi;
                    __syncthreads();
                    for (int o = kTopkThreads / 2; o >= 1; o >>= 1) {
                        if (threadIdx.x < o && key_less(se[threadIdx.x + o], si[threadIdx.x + o],
                                                        se[threadIdx.x], si[threadIdx.x])) {
                            se[threadIdx.x] = se[threadIdx.x + o];
                            si[threadIdx.x] = si[threadIdx.x + o];
                        }
                        __syncthreads();
                    }
                    last_s = se[0];
                    last_i = si[0];
                    have_last = true;
                    if (threadIdx.x == 0) a.cand[base + j] = a.rank_of[last_i];
                    __syncthreads();
                }
            }
        }
        if (threadIdx.x == 0) a.cnt[q] = k >= 2 ? nc * ((k + 63) / 64) : 0;
        if (phase == 0) {
            __syncthreads();               // every hash has been read
            // the pivots' ranks into LDS (nc <= kMaxTopk <= kTopkSel)
            for (int64_t j = threadIdx.x; j < nc; j += blockDim.x) si[j] = (uint32_t)a.cand[base + j];
            __syncthreads();
            // clear the estimates, keeping a pivot flag in the top bit
            // (four members a round: their loads overlap, and each pivot
            // read from LDS serves all four)
            for (int64_t i0 = threadIdx.x; i0 < k; i0 += kTopkUnroll * blockDim.x) {
                uint32_t r[kTopkUnroll];
                bool piv[kTopkUnroll];
#pragma unroll
                for (int u = 0; u < kTopkUnroll; ++u) {
                    const int64_t i = i0 + (int64_t)u * blockDim.x;
                    r[u] = i < k ? (uint32_t)a.perm[ms + i] : ~0u;
                    piv[u] = false;
                }
                for (int64_t j = 0; j < nc; ++j) {
                    const uint32_t c = si[j];
#pragma unroll
                    for (int u = 0; u < kTopkUnroll; ++u) piv[u] |= c == r[u];
                }
#pragma unroll
                for (int u = 0; u < kTopkUnroll; ++u) {
                    const int64_t i = i0 + (int64_t)u * blockDim.x;
                    if (i < k) a.rowsum[ms + i] = piv[u] ? kPivotFlag : 0ull;
                }
            }
            if (threadIdx.x == 0) a.ncand[q] = a.topk;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[nq] = 0;
}

// c = the candidate with the least exact row sum (lowest input index on ties).
__global__ void k_pick_center_cand(TreeArgs a) {
    const int32_t lvl = a.desc[0], nq = level_clusters(a.desc);
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const int32_t v = lvl + q;
        const int64_t k = a.mcount[v];
        const int64_t nc = a.ncand[q], base = a.coff[q];
        uint64_t bs = ~0ull;
        uint32_t bi = ~0u;
        int64_t bj = 0;
        for (int64_t j = 0; j < nc; ++j) {
            const uint64_t sv = a.candsum[base + j];
            const uint32_t oi = (uint32_t)a.order[a.cand[base + j]];
            if (key_less(sv, oi, bs, bi)) { bs = sv; bi = oi; bj = j; }
        }
        if (k == 1) bi = (uint32_t)a.order[a.perm[a.mstart[v]]];
        a.center[v] = (int32_t)bi;
        a.pat[q] = a.rank_of[bi];
        // c's far key, kept by the candidate pass: the first pole without a pass
        a.key[q] = nc > 0 && k >= 2 ? a.candkey[base + bj] : 0;
        a.cnt[q] = k >= 2 ? (k + 63) / 64 : 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[nq] = 0;
}

// Shape of k_tree_xl for a build: G lanes per pair, WL words per lane, NB
// bit planes; grid = its persistent grid; caps as in TreeArgs (0 and 0: off).
struct XlShape {
    int g = 0, wl = 0, nb = 0, grid = 0;
    int32_t sum_cap = 0, pole_cap = 0;
    bool on() const { return g > 0 && (sum_cap > 0 || pole_cap > 0); }
};

template <int WL, int NB>
static const void *xl_kernel_g(int g) {
    switch (g) {
        case 1: return (const void *)&k_tree_xl<1, WL, NB>;
        case 2: return (const void *)&k_tree_xl<2, WL, NB>;
        case 4: return (const void *)&k_tree_xl<4, WL, NB>;
        case 8: return (const void *)&k_tree_xl<8, WL, NB>;
        case 16: return (const void *)&k_tree_xl<16, WL, NB>;
        case 32: return (const void *)&k_tree_xl<32, WL, NB>;
        default: return (const void *)&k_tree_xl<64, WL, NB>;
    }
}

static const void *xl_kernel(int g, int wl, int nb) {
    if (wl == 1) return nb == 2 ? xl_kernel_g<1, 2>(g) : xl_kernel_g<1, 5>(g);
    return nb == 2 ? xl_kernel_g<2, 2>(g) : xl_kernel_g<2, 5>(g);
}

// One distance pass: its work split between k_tree_lev (large clusters) and
// k_tree_xl (small ones).
template <int WMAX, int MODE>
static void dist_pass(const TreeArgs &a, int grid, const XlShape &xl, hipStream_t s) {
    constexpr int cls = MODE == kMedoid ? kClsMedoid
                        : (MODE == kCandSum || MODE == kPivotSum) ? kClsSum
                                                                   : kClsPole;
    const int32_t cap = xl.on() ? (cls == kClsPole ? xl.pole_cap : xl.sum_cap) : 0;
    hipLaunchKernelGGL(k_scan_work, dim3(1), dim3(1024), 0, s, a, cls);
    // a cap above n sends every cluster across lanes: k_tree_lev would only
    // find no work
    if (cap <= a.n) hipLaunchKernelGGL((k_tree_lev<WMAX, MODE>), dim3(grid), dim3(kWave), 0, s, a);
    if (cap > 0) {
        TreeArgs aa = a;
        int mode = MODE;
        void *args[] = {&aa, &mode};
        (void)hipLaunchKernel(xl_kernel(xl.g, xl.wl, xl.nb), dim3(xl.grid), dim3(kXlBlock), args,
                              0, s);
    }
}

template <int WMAX>
static void launch_select(const TreeArgs &a, int grid, const XlShape &xl, int egrid,
                          hipStream_t s) {
    const dim3 cg(kClusterGrid), cb(256), tb(64);
    hipLaunchKernelGGL(k_level_init, cg, cb, 0, s, a);
    const bool exact = a.emb == nullptr && a.pivots == 0;
    if (exact) {
        dist_pass<WMAX, kMedoid>(a, grid, xl, s);
        hipLaunchKernelGGL(k_pick_center, cg, cb, 0, s, a);
    } else {
        if (a.emb != nullptr) {
            hipLaunchKernelGGL(k_scan_level, dim3(1), dim3(1024), 0, s, a.cnt, a.items, a.desc);
            hipLaunchKernelGGL(k_emb_rowsum, dim3(egrid), tb, 0, s, a);
        } else {
            // sampled median: pivots by hash, then every member's summed
            // distance to them is its estimate
            hipLaunchKernelGGL(k_scan_level, dim3(1), dim3(1024), 0, s, a.ncand, a.coff, a.desc);
            hipLaunchKernelGGL(k_topk, cg, dim3(kTopkThreads), 0, s, a, 0);
            dist_pass<WMAX, kPivotSum>(a, grid, xl, s);
        }
        hipLaunchKernelGGL(k_scan_level, dim3(1), dim3(1024), 0, s, a.ncand, a.coff, a.desc);
        hipLaunchKernelGGL(k_topk, cg, dim3(kTopkThreads), 0, s, a, 1);
        dist_pass<WMAX, kCandSum>(a, grid, xl, s);
        hipLaunchKernelGGL(k_pick_center_cand, dim3(256), dim3(256), 0, s, a);
    }
    // l = argmax f(c, x).  Pruned mode: c's far key is already in key[q]
    // from the candidate pass.
    if (exact) dist_pass<WMAX, kPoleMax>(a, grid, xl, s);
    hipLaunchKernelGGL(k_pick_pole, dim3(256), dim3(256), 0, s, a, 0);
    dist_pass<WMAX, kPoleMaxStore>(a, grid, xl, s);
    hipLaunchKernelGGL(k_pick_pole, dim3(256), dim3(256), 0, s, a, 1);
}

// One level of Alg. 1: c, l, r, then f(r, x), the split and the children.
template <int WMAX>
static void launch_passes(const TreeArgs &a, int grid, const XlShape &xl, int egrid,
                          hipStream_t s) {
    const dim3 cg(kClusterGrid), cb(256);
    launch_select<WMAX>(a, grid, xl, egrid, s);
    dist_pass<WMAX, kPoleStore>(a, grid, xl, s);
    (void)hipMemcpyAsync(a.perm_next, a.perm, sizeof(int32_t) * (size_t)a.n, hipMemcpyDeviceToDevice, s);
    hipLaunchKernelGGL(k_split, cg, cb, 0, s, a);
    hipLaunchKernelGGL(k_scan_level, dim3(1), dim3(1024), 0, s, a.split, a.split, a.desc);
    hipLaunchKernelGGL(k_make_children, dim3(256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_next_level, dim3(1), dim3(1), 0, s, a);
    (void)hipMemcpyAsync(a.perm, a.perm_next, sizeof(int32_t) * (size_t)a.n, hipMemcpyDeviceToDevice, s);
}

static void level_pass(const TreeArgs &a, int wclass, int grid, const XlShape &xl, int egrid,
                       hipStream_t s) {
    switch (wclass) {
        case 4: launch_passes<4>(a, grid, xl, egrid, s); break;
        case 8: launch_passes<8>(a, grid, xl, egrid, s); break;
        case 16: launch_passes<16>(a, grid, xl, egrid, s); break;
        case 20: launch_passes<20>(a, grid, xl, egrid, s); break;
        case 24: launch_passes<24>(a, grid, xl, egrid, s); break;
        default: launch_passes<32>(a, grid, xl, egrid, s); break;
    }
}

static void level_select(const TreeArgs &a, int wclass, int grid, const XlShape &xl, int egrid,
                         hipStream_t s) {
    switch (wclass) {
        case 4: launch_select<4>(a, grid, xl, egrid, s); break;
        case 8: launch_select<8>(a, grid, xl, egrid, s); break;
        case 16: launch_select<16>(a, grid, xl, egrid, s); break;
        case 20: launch_select<20>(a, grid, xl, egrid, s); break;
        case 24: launch_select<24>(a, grid, xl, egrid, s); break;
        default: launch_select<32>(a, grid, xl, egrid, s); break;
    }
}

// Persistent grids, cached per device (concurrent first calls compute the
// same value).
static int emb_grid() {
    static std::atomic<int> cache[kMaxDevices];
    std::atomic<int> &slot = cache[current_device()];
    int g = slot.load(std::memory_order_relaxed);
    if (g == 0) {
        g = persistent_grid(k_emb_rowsum);
        slot.store(g, std::memory_order_relaxed);
    }
    return g;
}

static int tree_grid(int wclass) {
    static std::atomic<int> cache[kMaxDevices][33];
    std::atomic<int> &slot = cache[current_device()][wclass];
    int g = slot.load(std::memory_order_relaxed);
    if (g == 0) {
        switch (wclass) {
            case 4: g = persistent_grid(k_tree_lev<4, kMedoid>); break;
            case 8: g = persistent_grid(k_tree_lev<8, kMedoid>); break;
            case 16: g = persistent_grid(k_tree_lev<16, kMedoid>); break;
            case 20: g = persistent_grid(k_tree_lev<20, kMedoid>); break;
            case 24: g = persistent_grid(k_tree_lev<24, kMedoid>); break;
            default: g = persistent_grid(k_tree_lev<32, kMedoid>); break;
        }
        slot.store(g, std::memory_order_relaxed);
    }
    return g;
}

static int xl_grid(int g, int wl, int nb) {
    static std::atomic<int> cache[kMaxDevices][7][2][2];
    int gi = 0;
    while ((1 << gi) < g) ++gi;
    std::atomic<int> &slot = cache[current_device()][gi][wl - 1][nb == 2 ? 0 : 1];
    int v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, xl_kernel(g, wl, nb), kXlBlock,
                                                         0) != hipSuccess ||
            blocks < 1)
            blocks = 1;
        v = device_cus() * blocks;
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}

struct TreePlan {
    int64_t stride, hstride;
    int wclass, grid;
    size_t hbuf_dwords;     // carry buffer: the largest any admissible class needs
    XlShape xl;
};

static int64_t tree_hstride(const msa_seqs *S, int wclass) {
    return needs_passes(S->max_len, wclass) ? ((int64_t)S->max_len + 15) / 16 : 0;
}

// Across-lanes passes of a build: the tuning table's entry for
// (MSA_TUNE_TREE_XL, sigma, pattern words) if valid, else the default.  G =
// the least power of two with G WL >= pattern words (at most 64).
static XlShape plan_xl(const msa_seqs *S, int forced_xl) {
    XlShape x;
    const int words = (int)std::max<int64_t>(1, ((int64_t)S->max_len + 63) / 64);
    int v = forced_xl > 0 ? forced_xl : tuned_value(MSA_TUNE_TREE_XL, S->sigma, words, 0);
    if (!xl_value_valid(v)) v = xl_default_value();
    const int wl = xl_value_wl(v);
    int g = 1;
    while (g * wl < words) g <<= 1;
    if (g > kWave) return x;
    x.g = g;
    x.wl = wl;
    x.nb = xl_planes(S->sigma);
    x.sum_cap = xl_value_sum_cap(v);
    x.pole_cap = xl_value_pole_cap(v);
    if (x.on()) x.grid = xl_grid(g, wl, x.nb);
    return x;
}

// forced > 0 selects the class (autotuning); else the tuning table's entry
// for (MSA_TUNE_TREE, sigma, pattern words) if it is an admissible class,
// else the default.  Admissible: a tree class within class_within_passes.
static TreePlan plan_tree(const msa_seqs *S, int forced, int forced_xl = 0) {
    TreePlan p;
    p.stride = staged_stride(S->max_len);
    const int words = (int)std::max<int64_t>(1, ((int64_t)S->max_len + 63) / 64);
    const int tuned = tuned_value(MSA_TUNE_TREE, S->sigma, words, 0);
    p.wclass = forced > 0 ? forced
               : (is_tree_class(tuned) && class_within_passes(S->max_len, tuned))
                   ? tuned
                   : wmax_class(S->max_len);
    p.grid = tree_grid(p.wclass);
    p.hstride = tree_hstride(S, p.wclass);
    p.hbuf_dwords = 0;
    for (int c : kTreeClasses) {
        if (!class_within_passes(S->max_len, c)) continue;
        p.hbuf_dwords = std::max(p.hbuf_dwords,
                                 (size_t)tree_grid(c) * kWave * (size_t)tree_hstride(S, c));
    }
    p.xl = plan_xl(S, forced_xl);
    return p;
}

template <class Alloc>
static void tree_layout(Alloc &al, const msa_seqs *S, const TreePlan &p) {
    const size_t n = (size_t)S->n;
    al.template take<uint8_t>(n * p.stride);
    al.template take<int32_t>(n + 1);           // staged lengths
    al.template take<int32_t>(n);               // order
    al.template take<int32_t>(n);               // rank_of
    al.template take<int32_t>((size_t)S->max_len + 1);
    al.template take<int32_t>(n);               // perm
    al.template take<int32_t>(n);               // perm_next
    al.template take<int32_t>(4);               // desc
    al.template take<int64_t>(n + 1);           // cnt
    al.template take<int64_t>(n + 1);           // items
    al.template take<uint64_t>(n + 1);          // key
    al.template take<int32_t>(n + 1);           // pat
    al.template take<int32_t>(n + 1);           // nleft
    al.template take<int64_t>(n + 1);           // split
    al.template take<uint64_t>(n + 1);          // rowsum (+ spare slot)
    al.template take<int32_t>(n + 1);           // dl
    al.template take<int32_t>(n + 1);           // dr
    al.template take<uint32_t>(2);              // counters
    if (p.hbuf_dwords) al.template take<uint32_t>(p.hbuf_dwords);
    al.template take<int64_t>(n + 1);           // candidate counts
    al.template take<int64_t>(n + 1);           // candidate offsets
    al.template take<int32_t>(n);               // candidates
    al.template take<uint64_t>(n);              // candidate sums
    al.template take<uint64_t>(n);              // candidate far keys
    al.template take<int32_t>(2 * n);           // child ids of an evaluated tree
    al.template take<int32_t>(2 * n);
    al.template take<int8_t>(n * kEmbDim);      // embedding codes
    al.template take<int32_t>(n);               // their squared norms
    al.template take<uint32_t>(2);              // max |e|, spare
    al.template take<int64_t>(n + 1);           // pitems
}

// Quantize the embeddings once per call (before any level).
static int quantize_embeddings(const TreeArgs &a, hipStream_t s) {
    if (a.emb == nullptr) return MSA_OK;
    const int64_t count = (int64_t)a.n * kEmbDim;
    hipLaunchKernelGGL(k_emb_reset, dim3(1), dim3(1), 0, s, a.emb_max);
    hipLaunchKernelGGL(k_emb_absmax, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 2048)),
                       dim3(256), 0, s, a.emb, count, a.emb_max);
    hipLaunchKernelGGL(k_emb_quantize, dim3((unsigned)(((int64_t)a.n * 32 + 255) / 256)),
                       dim3(256), 0, s, a.emb, a.n, (const uint32_t *)a.emb_max, a.embq, a.embn,
                       a.st);
    return launch_status();
}

}  // namespace msadp

using namespace msadp;

static int build_impl(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T,
                      int32_t *n_nodes, int32_t use_graph, void *ws, size_t ws_bytes,
                      int32_t *d_status, hipStream_t s, int forced,
                      const Forest *fr = nullptr, int32_t pivots = 0, int forced_xl = 0);

extern "C" {

size_t tree_workspace_bytes(const msa_seqs *S) {
    if (check_seqs(S)) return 0;
    Sizer sz;
    tree_layout(sz, S, plan_tree(S, 0));
    return sz.total();
}

static int build_impl(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T,
                      int32_t *n_nodes, int32_t use_graph, void *ws, size_t ws_bytes,
                      int32_t *d_status, hipStream_t s, int forced,
                      const Forest *fr, int32_t pivots, int forced_xl) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (T == nullptr || n_nodes == nullptr) return MSA_EINVAL;
    *n_nodes = 0;
    if (S->n == 0) return MSA_OK;
    if (S->n >= (1 << 24)) return MSA_ERANGE;
    if (!T->parent || !T->left || !T->right || !T->center || !T->lpole || !T->rpole ||
        !T->depth || !T->mstart || !T->mcount || !T->perm || ws == nullptr)
        return MSA_EINVAL;
    const TreePlan p = plan_tree(S, forced, forced_xl);
    Sizer sz;
    tree_layout(sz, S, p);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    const size_t n = (size_t)S->n;
    Carve cv(ws, ws_bytes);
    TreeArgs a{};
    a.S = Staged{cv.take<uint8_t>(n * p.stride), cv.take<int32_t>(n + 1), p.stride, S->n};
    int32_t *order = cv.take<int32_t>(n);
    int32_t *rank_of = cv.take<int32_t>(n);
    int32_t *hist = cv.take<int32_t>((size_t)S->max_len + 1);
    a.order = order;
    a.rank_of = rank_of;
    a.perm = cv.take<int32_t>(n);
    a.perm_next = cv.take<int32_t>(n);
    a.parent = T->parent; a.left = T->left; a.right = T->right; a.center = T->center;
    a.lpole = T->lpole; a.rpole = T->rpole; a.depth = T->depth;
    a.mstart = T->mstart; a.mcount = T->mcount;
    a.desc = cv.take<int32_t>(4);
    a.cnt = cv.take<int64_t>(n + 1);
    a.items = cv.take<int64_t>(n + 1);
    a.key = cv.take<uint64_t>(n + 1);
    a.pat = cv.take<int32_t>(n + 1);
    a.nleft = cv.take<int32_t>(n + 1);
    a.split = cv.take<int64_t>(n + 1);
    a.rowsum = cv.take<uint64_t>(n + 1);
    a.dl = cv.take<int32_t>(n + 1);
    a.dr = cv.take<int32_t>(n + 1);
    a.counter = cv.take<uint32_t>(2);
    a.hbuf = p.hbuf_dwords ? cv.take<uint32_t>(p.hbuf_dwords) : nullptr;
    a.hstride = p.hstride;
    a.ncand = cv.take<int64_t>(n + 1);
    a.coff = cv.take<int64_t>(n + 1);
    a.cand = cv.take<int32_t>(n);
    a.candsum = cv.take<uint64_t>(n);
    a.candkey = cv.take<uint64_t>(n);
    int32_t *eval_left = cv.take<int32_t>(2 * n);
    int32_t *eval_right = cv.take<int32_t>(2 * n);
    (void)eval_left;
    (void)eval_right;
    a.embq = cv.take<int8_t>(n * kEmbDim);
    a.embn = cv.take<int32_t>(n);
    a.emb_max = cv.take<uint32_t>(2);
    a.pitems = cv.take<int64_t>(n + 1);
    a.xl_sum = p.xl.on() ? p.xl.sum_cap : 0;
    a.xl_pole = p.xl.on() ? p.xl.pole_cap : 0;
    a.emb = emb;
    a.emb_q0 = emb_q0;
    a.pivots = pivots;
    a.topk = topk;
    a.exact_below = exact_below;
    a.sigma = S->sigma;
    a.n = S->n;
    a.st = d_status;

    if ((rc = sort_by_length(S, a.S.len, hist, order, d_status, s))) return rc;
    if ((rc = stage_set(S, order, a.S, d_status, s))) return rc;
    hipLaunchKernelGGL(k_rank_of, dim3((S->n + 255) / 256), dim3(256), 0, s, order, S->n, rank_of,
                       a.perm);
    int32_t total = 1;
    if (fr == nullptr) {
        hipLaunchKernelGGL(k_tree_root, dim3(1), dim3(1), 0, s, a);
    } else {
        const int64_t span = std::max<int64_t>(fr->m, fr->K);
        hipLaunchKernelGGL(k_forest_root, dim3((unsigned)((span + 255) / 256)), dim3(256), 0, s,
                           a, fr->K, fr->mem, fr->start, fr->m);
        total = fr->K;
    }
    if ((rc = launch_status())) return rc;
    if ((rc = quantize_embeddings(a, s))) return rc;

    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (use_graph) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return MSA_EDEVICE;
        level_pass(a, p.wclass, p.grid, p.xl, emb_grid(), s);
        if (hipStreamEndCapture(s, &graph) != hipSuccess) return MSA_EDEVICE;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return MSA_EDEVICE;
        }
    }
    int32_t host_desc[3] = {0, total, 0};
    rc = MSA_OK;
    for (int level = 0; level < S->n; ++level) {
        if (use_graph) {
            if (hipGraphLaunch(exec, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        } else {
            level_pass(a, p.wclass, p.grid, p.xl, emb_grid(), s);
        }
        if ((rc = launch_status())) break;
        if (hipMemcpyAsync(host_desc, a.desc, sizeof(host_desc), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        if (host_desc[2] == 0) break;
        total += 2 * host_desc[2];
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    hipLaunchKernelGGL(k_perm_out, dim3((S->n + 255) / 256), dim3(256), 0, s, order, a.perm, S->n,
                       T->perm);
    if ((rc = launch_status())) return rc;
    *n_nodes = total;
    return MSA_OK;
}

int tree_build(const msa_seqs *S, const msa_tree *T, int32_t *n_nodes, int32_t use_graph,
               void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    return build_impl(S, nullptr, 0, 0, 0, T, n_nodes, use_graph, ws, ws_bytes, d_status, s, 0);
}

int tree_build_pruned(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T, int32_t *n_nodes,
                      int32_t use_graph, void *ws, size_t ws_bytes, int32_t *d_status,
                      hipStream_t s) {
    if (emb == nullptr || topk < 1 || topk > kMaxTopk || exact_below < 0 ||
        emb_q0 > kMaxEmbOffset)
        return MSA_EINVAL;
    return build_impl(S, emb, emb_q0, topk, exact_below, T, n_nodes, use_graph, ws, ws_bytes,
                      d_status, s, 0);
}

int msa_autotune_tree(const msa_seqs *S, const msa_tree *T, int32_t *n_nodes, int32_t use_graph,
                      void *ws, size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                      int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (best == nullptr || best_ms == nullptr || reps < 1 || S->n < 2) return MSA_EINVAL;
    const int words = (int)std::max<int64_t>(1, ((int64_t)S->max_len + 63) / 64);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MSA_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MSA_EDEVICE;
    }
    int bc = 0;
    float bms = 0.0f;
    rc = MSA_OK;
    for (int c : kTreeClasses) {
        if (!class_within_passes(S->max_len, c)) continue;
        if ((rc = build_impl(S, nullptr, 0, 0, 0, T, n_nodes, use_graph, ws, ws_bytes, d_status,
                             s, c)))
            break;   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        for (int r = 0; r < reps && rc == MSA_OK; ++r)
            rc = build_impl(S, nullptr, 0, 0, 0, T, n_nodes, use_graph, ws, ws_bytes, d_status,
                            s, c);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        ms /= (float)reps;
        if (bc == 0 || ms < bms) {
            bc = c;
            bms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = bc;
    *best_ms = bms;
    return msa_tune_set(MSA_TUNE_TREE, S->sigma, words, bc);
}

int msa_autotune_tree_xl(const msa_seqs *S, int32_t pivots, int32_t topk, const msa_tree *T,
                         int32_t *n_nodes, int32_t use_graph, void *ws, size_t ws_bytes,
                         int32_t reps, int32_t *best, float *best_ms, int32_t *d_status,
                         hipStream_t s) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (best == nullptr || best_ms == nullptr || reps < 1 || S->n < 2 || pivots < 0 ||
        pivots > kMaxTopk || (pivots > 0 && (topk < 1 || topk > kMaxTopk)))
        return MSA_EINVAL;
    const int words = (int)std::max<int64_t>(1, ((int64_t)S->max_len + 63) / 64);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MSA_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MSA_EDEVICE;
    }
    int bv = 0;
    float bms = 0.0f;
    rc = MSA_OK;
    for (const int v : kXlCandidates) {
        auto run = [&]() {
            return build_impl(S, nullptr, 0, pivots > 0 ? topk : 0, 0, T, n_nodes, use_graph, ws,
                              ws_bytes, d_status, s, 0, nullptr, pivots, v);
        };
        if ((rc = run())) break;   // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MSA_EDEVICE; break; }
        for (int r = 0; r < reps && rc == MSA_OK; ++r) rc = run();
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MSA_EDEVICE;
            break;
        }
        ms /= (float)reps;
        if (bv == 0 || ms < bms) {
            bv = v;
            bms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = bv;
    *best_ms = bms;
    return msa_tune_set(MSA_TUNE_TREE_XL, S->sigma, words, bv);
}

int tree_build_sampled(const msa_seqs *S, int32_t pivots, int32_t topk, int32_t exact_below,
                       const msa_tree *T, int32_t *n_nodes, int32_t use_graph, void *ws,
                       size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    if (pivots < 1 || pivots > kMaxTopk || topk < 1 || topk > kMaxTopk || exact_below < 0)
        return MSA_EINVAL;
    return build_impl(S, nullptr, 0, topk, exact_below, T, n_nodes, use_graph, ws, ws_bytes,
                      d_status, s, 0, nullptr, pivots);
}

static int eval_impl(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t pivots,
                     int32_t topk, int32_t exact_below, const msa_tree *T, int32_t n_nodes,
                     int32_t *center, int32_t *lpole, int32_t *rpole, void *ws,
                     size_t ws_bytes, int32_t *d_status, hipStream_t s);

int tree_eval_centers(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T,
                      int32_t n_nodes, int32_t *center, int32_t *lpole, int32_t *rpole,
                      void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    if (emb != nullptr &&
        (topk < 1 || topk > kMaxTopk || exact_below < 0 || emb_q0 > kMaxEmbOffset))
        return MSA_EINVAL;
    return eval_impl(S, emb, emb_q0, 0, topk, exact_below, T, n_nodes, center, lpole, rpole, ws,
                     ws_bytes, d_status, s);
}

int tree_eval_centers_sampled(const msa_seqs *S, int32_t pivots, int32_t topk,
                              int32_t exact_below, const msa_tree *T, int32_t n_nodes,
                              int32_t *center, int32_t *lpole, int32_t *rpole, void *ws,
                              size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    if (pivots < 1 || pivots > kMaxTopk || topk < 1 || topk > kMaxTopk || exact_below < 0)
        return MSA_EINVAL;
    return eval_impl(S, nullptr, 0, pivots, topk, exact_below, T, n_nodes, center, lpole, rpole,
                     ws, ws_bytes, d_status, s);
}

static int eval_impl(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t pivots,
                     int32_t topk, int32_t exact_below, const msa_tree *T, int32_t n_nodes,
                     int32_t *center, int32_t *lpole, int32_t *rpole, void *ws,
                     size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    int rc;
    if ((rc = check_seqs(S))) return rc;
    if (T == nullptr || center == nullptr || lpole == nullptr || rpole == nullptr ||
        T->mstart == nullptr || T->mcount == nullptr || T->depth == nullptr ||
        T->perm == nullptr || ws == nullptr || n_nodes < 0)
        return MSA_EINVAL;
    if (S->n == 0 || n_nodes == 0) return n_nodes == 0 ? MSA_OK : MSA_EINVAL;
    if (S->n >= (1 << 24)) return MSA_ERANGE;
    if (n_nodes > 2 * S->n - 1) return MSA_EINVAL;
    const TreePlan p = plan_tree(S, 0);
    Sizer sz;
    tree_layout(sz, S, p);
    if (ws_bytes < sz.total()) return MSA_ENOSPC;
    // The node table is read back to find the levels and to check that the
    // clusters of one depth are disjoint ranges of perm.
    const size_t nn = (size_t)n_nodes;
    int32_t *h_depth = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *h_ms = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *h_mc = (int64_t *)malloc(nn * sizeof(int64_t));
    if (!h_depth || !h_ms || !h_mc) {
        free(h_depth); free(h_ms); free(h_mc);
        return MSA_EDEVICE;
    }
    rc = MSA_OK;
    if (hipMemcpyAsync(h_depth, T->depth, nn * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(h_ms, T->mstart, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(h_mc, T->mcount, nn * sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = MSA_EDEVICE;
    if (rc == MSA_OK && (h_depth[0] != 0 || h_ms[0] != 0 || h_mc[0] != S->n)) rc = MSA_EINVAL;
    for (size_t v = 0; rc == MSA_OK && v < nn; ++v) {
        if (h_mc[v] < 1 || h_ms[v] < 0 || h_ms[v] + h_mc[v] > S->n) rc = MSA_EINVAL;
        if (v > 0 && (h_depth[v] < h_depth[v - 1] || h_depth[v] > h_depth[v - 1] + 1))
            rc = MSA_EINVAL;
        // same depth: ranges in increasing, non-overlapping order
        if (v > 0 && h_depth[v] == h_depth[v - 1] && h_ms[v] < h_ms[v - 1] + h_mc[v - 1])
            rc = MSA_EINVAL;
    }
    if (rc) {
        free(h_depth); free(h_ms); free(h_mc);
        return rc;
    }
    const size_t n = (size_t)S->n;
    Carve cv(ws, ws_bytes);
    TreeArgs a{};
    a.S = Staged{cv.take<uint8_t>(n * p.stride), cv.take<int32_t>(n + 1), p.stride, S->n};
    int32_t *order = cv.take<int32_t>(n);
    int32_t *rank_of = cv.take<int32_t>(n);
    int32_t *hist = cv.take<int32_t>((size_t)S->max_len + 1);
    a.order = order;
    a.rank_of = rank_of;
    a.perm = cv.take<int32_t>(n);
    a.perm_next = cv.take<int32_t>(n);
    a.desc = cv.take<int32_t>(4);
    a.cnt = cv.take<int64_t>(n + 1);
    a.items = cv.take<int64_t>(n + 1);
    a.key = cv.take<uint64_t>(n + 1);
    a.pat = cv.take<int32_t>(n + 1);
    a.nleft = cv.take<int32_t>(n + 1);
    a.split = cv.take<int64_t>(n + 1);
    a.rowsum = cv.take<uint64_t>(n + 1);
    a.dl = cv.take<int32_t>(n + 1);
    a.dr = cv.take<int32_t>(n + 1);
    a.counter = cv.take<uint32_t>(2);
    a.hbuf = p.hbuf_dwords ? cv.take<uint32_t>(p.hbuf_dwords) : nullptr;
    a.hstride = p.hstride;
    a.ncand = cv.take<int64_t>(n + 1);
    a.coff = cv.take<int64_t>(n + 1);
    a.cand = cv.take<int32_t>(n);
    a.candsum = cv.take<uint64_t>(n);
    a.candkey = cv.take<uint64_t>(n);
    a.left = cv.take<int32_t>(2 * n);
    a.right = cv.take<int32_t>(2 * n);
    a.embq = cv.take<int8_t>(n * kEmbDim);
    a.embn = cv.take<int32_t>(n);
    a.emb_max = cv.take<uint32_t>(2);
    a.pitems = cv.take<int64_t>(n + 1);
    a.xl_sum = p.xl.on() ? p.xl.sum_cap : 0;
    a.xl_pole = p.xl.on() ? p.xl.pole_cap : 0;
    a.center = center;
    a.lpole = lpole;
    a.rpole = rpole;
    a.mstart = T->mstart;
    a.mcount = T->mcount;
    a.emb = emb;
    a.emb_q0 = emb_q0;
    a.pivots = pivots;
    a.topk = topk;
    a.exact_below = exact_below;
    a.sigma = S->sigma;
    a.n = S->n;
    a.st = d_status;

    if ((rc = sort_by_length(S, a.S.len, hist, order, d_status, s)) == MSA_OK &&
        (rc = stage_set(S, order, a.S, d_status, s)) == MSA_OK) {
        hipLaunchKernelGGL(k_rank_of, dim3((S->n + 255) / 256), dim3(256), 0, s, order, S->n,
                           rank_of, a.perm_next);
        hipLaunchKernelGGL(k_perm_in, dim3((S->n + 255) / 256), dim3(256), 0, s, T->perm,
                           rank_of, S->n, a.perm, d_status);
        rc = launch_status();
        if (rc == MSA_OK) rc = quantize_embeddings(a, s);
    }
    for (size_t lo = 0; rc == MSA_OK && lo < nn;) {
        size_t hi = lo + 1;
        while (hi < nn && h_depth[hi] == h_depth[lo]) ++hi;
        hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, s, a.desc, (int32_t)lo, (int32_t)hi);
        level_select(a, p.wclass, p.grid, p.xl, emb_grid(), s);
        rc = launch_status();
        lo = hi;
    }
    free(h_depth); free(h_ms); free(h_mc);
    return rc;
}

}  // extern "C"

// Alg. 1 on each of K disjoint member lists at once (the full median): the
// same level passes as tree_build, started from K roots.  Node ids are
// breadth-first over the forest (roots 0 .. K-1).  T holds up to 2m nodes
// and S->n perm entries (the first m are the forest's, as input indices).
int msadp::tree_build_forest(const msa_seqs *S, const Forest &fr, const msa_tree *T,
                             int32_t *n_nodes, void *ws, size_t ws_bytes, int32_t *d_status,
                             hipStream_t s) {
    if (fr.K < 1 || fr.m < fr.K || fr.m > S->n || fr.mem == nullptr || fr.start == nullptr)
        return MSA_EINVAL;
    return build_impl(S, nullptr, 0, 0, 0, T, n_nodes, 0, ws, ws_bytes, d_status, s, 0, &fr);
}
