/*
 * msadp: batched Levenshtein and Needleman-Wunsch dynamic programs on
 * MI355X (gfx950), for the guide-tree clustering and bottom-up alignment of
 * MuSAlS (Light, Prior, Daniels, Ishaq; arXiv 2601.15458).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sequences.  A sequence set is described by `msa_seqs`: symbol codes in
 * CSR form.  Sequence k occupies symbols [offsets[k], offsets[k+1]).  With
 * packed_2bit == 0 each symbol is one byte of `codes`; with packed_2bit == 1
 * (only for sigma <= 4) symbol p sits in bits 2*(p%4) .. 2*(p%4)+1 of byte
 * codes[p/4].  `codes` and `offsets` are DEVICE pointers; n, sigma, max_len
 * and packed_2bit are host values.  max_len must bound every length; the
 * library relies on it to size workspace and to pick kernels.
 *
 * Ownership.  The caller owns every buffer: inputs, outputs and workspace.
 * The library never allocates device memory on these paths and never frees
 * caller memory.  Workspace sizes come from the *_workspace_bytes queries.
 * All calls are asynchronous on the caller's stream `s`; results are valid
 * once the stream reaches them.
 *
 * Errors.  Functions return MSA_OK (0) or a negative code.  Errors detected
 * on the host (null pointers, negative counts, sigma outside [2, 32],
 * packed_2bit with sigma > 4, max_len outside [0, 65535], workspace too
 * small) return before anything is launched and leave outputs untouched.
 * MSA_EDEVICE reports a failed launch.  Errors only visible on the device
 * (a code >= sigma, an index outside [0, n), a length above max_len or a
 * negative length, an output capacity too small) are written to *d_status
 * (a device int32 the caller zeroes; the first error wins) when d_status is
 * non-null; the affected outputs are then unspecified.  n_pairs == 0 returns
 * MSA_OK without launching.  No exception crosses this interface.
 */
#ifndef MSADP_H
#define MSADP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MSA_OK = 0,
    MSA_EINVAL = -1,   /* bad argument                                   */
    MSA_ERANGE = -2,   /* a size outside what the entry point supports   */
    MSA_ENOSPC = -3,   /* workspace or output capacity too small         */
    MSA_EDEVICE = -4   /* a HIP launch or runtime call failed            */
};

/* Values written to *d_status by the device. */
enum {
    MSA_DS_OK = 0,
    MSA_DS_SYMBOL = 1,     /* a symbol code >= sigma                      */
    MSA_DS_INDEX = 2,      /* a sequence index outside [0, n)             */
    MSA_DS_LENGTH = 3,     /* a length < 0 or > max_len                   */
    MSA_DS_CAPACITY = 4,   /* an output region smaller than required      */
    MSA_DS_VALUE = 5       /* a non-finite embedding coordinate           */
};

typedef struct msa_seqs {
    const uint8_t *codes;     /* device: symbol codes (see packed_2bit)   */
    const int64_t *offsets;   /* device: n + 1 symbol offsets             */
    int32_t n;                /* number of sequences                      */
    int32_t sigma;            /* alphabet size, 2..32; codes 0..sigma-1   */
    int32_t max_len;          /* upper bound on every length, <= 65535    */
    int32_t packed_2bit;      /* 1: four 2-bit symbols per byte           */
} msa_seqs;

const char *msa_strerror(int code);
int msa_version(void);

/* ------------------------------------------------------------------ */
/* Levenshtein distance (the distance f of Alg. 1, Sec. 2.1; exact, not an
 * approximation, Sec. 2): unit-cost edit distance with insertions,
 * deletions and substitutions, D[m][n] of the Wagner-Fischer recurrence.
 * Computed bit-parallel: one bit per DP row, 64 rows per machine word.   */

/* Workspace for lev_batch over n_pairs pairs drawn from A and B. */
size_t lev_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs);

/* dist[p] = lev(A[ia[p]], B[ib[p]]) for p in [0, n_pairs) (A and B share
 * sigma; two descriptions of the same set are staged once).
 * ia, ib: device int32[n_pairs]; dist: device uint16[n_pairs].  Any order
 * of pairs is correct; the pairs are scheduled on the device in one
 * persistent launch, in one of three layouts (MSA_TUNE_PAIRS below):
 * pairs grouped by ia, 64 pairs of one pattern per wavefront, groups
 * longest pattern first and each group's texts longest first; or, when the
 * patterns are short enough, one pair per lane with the longer sequence as
 * its pattern, binned by pattern words and ordered by text length, longest
 * first (for sparse lists with few pairs per sequence); or one pair per
 * group of lanes, the longer sequence's 64-bit words spread over the group
 * and the carries between words passed lane to lane (patterns of up to
 * 16,384 rows; lists of at most 8192 pairs run largest m * n first).  A
 * pair with an index out of range sets MSA_DS_INDEX and dist[p] = 0xFFFF. */
int lev_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
              int64_t n_pairs, uint16_t *dist, void *ws, size_t ws_bytes,
              int32_t *d_status, hipStream_t s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lev_batch
 * with its workspace in a fixed device array of the library instead of a
 * caller buffer.  Same arguments (less the workspace), results and errors as
 * lev_batch, with the default layout and word class (the tuning table is not
 * read), and MSA_ENOSPC, before anything is launched, when that needs more
 * than MSA_NOALLOC_SCRATCH_BYTES of workspace (about 64 MiB; e.g. 100,000
 * sequences of up to 500 symbols with 1 M pairs fit).  It calls no
 * allocating routine.  Each GPU the library runs on holds its own copy of
 * the array until the process ends, set up on the first call on that device
 * (MSA_EDEVICE if that fails).  All calls on one GPU share the array: calls
 * that overlap on one GPU (other streams, other host threads) race and must
 * be serialized by the caller. */
#define MSA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lev_batch_noalloc(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                      const int32_t *ib, int64_t n_pairs, uint16_t *dist, int32_t *d_status,
                      hipStream_t s);

/* Exact banded Levenshtein for long, similar pairs (Ukkonen's band,
 * verified): dist[p] = lev(A[ia[p]], B[ib[p]]) whenever it is at most kmax,
 * else 0xFFFF (the caller recomputes such pairs with lev_batch).  Only the
 * cells of the diagonal band that holds every alignment of cost <= K are
 * computed, starting from K = max(k0, |m - n| + 2) and doubling up to kmax
 * while the banded value exceeds K (a banded value <= K is exact).
 * k_used[p] (device int32, may be null) receives the K that verified the
 * pair, or -1.  1 <= k0 <= kmax <= 4000; one wavefront per pair holds the
 * pattern's match table and the text in LDS: A->max_len / 64 * sigma * 8 +
 * B->max_len bytes, at most 64 KiB (MSA_ERANGE otherwise). */
size_t lev_band_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs);
int lev_band(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
             int64_t n_pairs, int32_t k0, int32_t kmax, uint16_t *dist, int32_t *k_used,
             void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* Workspace for lev_allpairs over the set A. */
size_t lev_allpairs_workspace_bytes(const msa_seqs *A);

/* All n(n-1)/2 distances of the set A (the root-level distance batch of
 * Alg. 1).  condensed: device uint16[n(n-1)/2]; the pair i < j is stored at
 * i*n - i*(i+1)/2 + (j - i - 1).  Sequences are binned by length on the
 * device and all pairs run in one persistent launch, longest first. */
int lev_allpairs(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                 int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Needleman-Wunsch global alignment with unit costs (match 0, mismatch 1,
 * gap 1), the pairwise aligner of the merge (Sec. 2.2, step 2: align the two
 * centers and note where gaps were added).  The fill records, per DP cell,
 * which predecessor the backward walk takes, in the order diagonal > up >
 * left; nw_traceback follows those codes from (m, n) to (0, 0).           */

/* Bytes of traceback codes for one pair with |a| = m, |b| = n (2 bits per
 * cell plus a small layout overhead; 0 when m == 0 or n == 0). */
size_t nw_tb_bytes(int32_t m, int32_t n);

/* Workspace for nw_batch over n_pairs pairs drawn from A and B. */
size_t nw_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs);

/* Fill for each pair p: score[p] = D[m][n] (int32) and the traceback codes
 * of pair p in tb[tb_offsets[p] .. tb_offsets[p+1]) (device int64[n_pairs+1],
 * each region at least nw_tb_bytes(m, n) bytes and 8-byte aligned).  The
 * code layout is private to nw_traceback.  score may be null. */
int nw_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
             int64_t n_pairs, int32_t *score, uint8_t *tb, const int64_t *tb_offsets,
             void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* Walk the codes written by nw_batch (same A, B, ia, ib, tb, tb_offsets).
 * For pair p the alignment is written in forward order to
 * ops[ops_offsets[p] ..] (device int64[n_pairs+1]; each region must hold
 * m + n bytes), one byte per column: 0 = M (a_i with b_j), 1 = D (a_i with a
 * gap), 2 = I (a gap with b_j); ops_len[p] receives the column count.
 * Columns with op I are the gap positions added to a, op D those added to b. */
int nw_traceback(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                 int64_t n_pairs, const uint8_t *tb, const int64_t *tb_offsets,
                 uint8_t *ops, const int64_t *ops_offsets, int32_t *ops_len,
                 int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Needleman-Wunsch with a substitution score matrix and affine gaps: the cost
 * model of the paper's experiments (Sec. 2.4: substitution matrices for
 * residues, gap opening charged ten times the extension; the matrix and
 * costs are the caller's).  Reading where the paper gives no formula: a run
 * of k gap symbols in one row scores -(open + k * ext), and the aligner
 * maximizes the sum of sub[a_i * sigma + b_j] over aligned pairs minus the
 * penalties of all gap runs (Gotoh's three-state recurrence).  Among the
 * best-scoring alignments the one returned is the one whose op string read
 * backwards is smallest with M < D < I (the order of the unit-cost walk).
 * sub: HOST int32[sigma * sigma] (row = symbol of a), |sub| <= 2048;
 * 0 <= open, 0 <= ext, open + ext <= 2048 (EINVAL otherwise); a pattern
 * (A sequence) of more than 16384 symbols returns MSA_ERANGE (A->max_len)
 * or sets MSA_DS_LENGTH.  Scores are int32 (exact for every admitted
 * input). */

/* Bytes of traceback codes for one pair (one byte per cell plus a small
 * layout overhead; 0 when m == 0 or n == 0). */
size_t gotoh_tb_bytes(int32_t m, int32_t n);

size_t gotoh_workspace_bytes(const msa_seqs *A, const msa_seqs *B, int64_t n_pairs);

/* Fill: score[p] (may be null) = the best score of pair (A[ia[p]], B[ib[p]])
 * and its traceback codes in tb[tb_offsets[p] ..] (each region at least
 * gotoh_tb_bytes(m, n) bytes, 16-byte aligned; layout private to
 * gotoh_traceback).  The score table is copied to the device before the
 * call returns. */
int gotoh_batch(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                int64_t n_pairs, const int32_t *sub, int32_t open, int32_t ext, int32_t *score,
                uint8_t *tb, const int64_t *tb_offsets, void *ws, size_t ws_bytes,
                int32_t *d_status, hipStream_t s);

/* The alignments of a gotoh_batch call (same A, B, ia, ib, tb, tb_offsets),
 * in the op format of nw_traceback (regions of m + n bytes). */
int gotoh_traceback(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                    int64_t n_pairs, const uint8_t *tb, const int64_t *tb_offsets, uint8_t *ops,
                    const int64_t *ops_offsets, int32_t *ops_len, int32_t *d_status,
                    hipStream_t s);

/* ------------------------------------------------------------------ */
/* Guide tree by Alg. 1 (Partition, Sec. 2.1): recursive split of the set
 * until every leaf holds one sequence.  Per cluster C: c = the member with
 * the least sum of distances to all members (the full geometric median);
 * l = argmax f(c, x); r = argmax f(l, x); L = {x : f(l,x) <= f(r,x)},
 * R = {x : f(r,x) < f(l,x)}.  Readings where the paper is silent: every
 * argmin/argmax keeps the lowest input index among equals; a cluster whose
 * radius max f(c, x) is 0 (copies of one sequence) stays a leaf.
 * Node ids are breadth-first (children of v are created when v splits, L
 * before R).  Node arrays (device, capacity 2n - 1): parent, left, right
 * (-1 if none), center, lpole, rpole (-1 for leaves), depth, mstart and
 * mcount (the node's members are perm[mstart .. mstart + mcount); a node's
 * range is its L child's range followed by its R child's).  perm (device,
 * n) lists input indices. */
typedef struct msa_tree {
    int32_t *parent, *left, *right, *center, *lpole, *rpole, *depth;
    int64_t *mstart, *mcount;
    int32_t *perm;
} msa_tree;

size_t tree_workspace_bytes(const msa_seqs *S);

/* Builds the tree of S into T; *n_nodes (host) receives the node count.
 * Levels run on the device; the stream is synchronized once per level to
 * read the number of splits.  use_graph != 0 records one level's launches
 * into a HIP graph and replays it per level (needs a non-default stream).
 * S->n must be below 2^24. */
int tree_build(const msa_seqs *S, const msa_tree *T, int32_t *n_nodes, int32_t use_graph,
               void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* The same tree build with the medoid step (Alg. 1, the geometric median
 * of each cluster) pruned by a surrogate; not a method of the paper, which
 * only allows the median to be taken over a subset to save time.  In a
 * cluster of more than exact_below members (>= 0), emb (device
 * float[n][128], row i = embedding of input i, e.g. from cnn_embed, whose
 * distances predict f divided by the pair's mean length) ranks every member
 * x by E(x) = sum over the cluster, y = x included, of
 * (q(x, y) + emb_q0) (|x| + |y|), with q the Euclidean distance of the
 * quantized embeddings, capped at 2^15, in units of 2^-16: with M = max |e|
 * over all n x 128 coordinates, s = 6 - floor(log2 M) limited to [-20, 40]
 * (40 when M < 2^-34), each coordinate's code is rint(e 2^s) limited to
 * +-127, and q = rint(min(sqrt(D) 2^-s, 2^15) 2^16) in float32 (correctly
 * rounded square root) with D the exact integer squared distance of the
 * codes; a non-finite coordinate sets MSA_DS_VALUE.
 * emb_q0 <= 2^31 is a calibration offset in the same units (the intercept over
 * the slope of a linear fit of the true normalized distance on the
 * predicted one, which shrinks a noisy predictor towards the length prior);
 * the topk members with the least (E, input index), 1 <= topk <= 1024, are
 * the candidates.  In a cluster of at most
 * exact_below members every member is a candidate.  The candidates get
 * exact Levenshtein row sums over the whole cluster and c is the one with
 * the least (lowest input index on ties).  Poles, split and every other
 * step stay exact, so clusters of at most max(topk, exact_below) members
 * get the same c as tree_build.  E is a 64-bit sum: it stays exact while
 * n * max(|x| + |y|) * max(q + emb_q0) < 2^64, e.g. for any n below 2^24
 * with lengths below 2^15 and distance plus offset below 2^8.  Same
 * outputs, workspace and errors as tree_build; EINVAL when emb is null or
 * topk, exact_below or emb_q0 is out of range. */
int tree_build_pruned(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T, int32_t *n_nodes,
                      int32_t use_graph, void *ws, size_t ws_bytes, int32_t *d_status,
                      hipStream_t s);

/* The tree build with the median taken over a smaller subset, which Sec.
 * 2.1 allows to save time.  In a cluster of k members, k > exact_below and
 * k > topk, the min(pivots, k) members with the least h(i) are the pivots,
 * h being MurmurHash3's 32-bit finalizer (Appleby) of the input index i
 * (h ^= h >> 16; h *= 0x85EBCA6B; h ^= h >> 13; h *= 0xC2B2AE35;
 * h ^= h >> 16: a bijection, so no two members tie); with s = min(pivots,
 * k), every member x gets E(x) = (sum over the pivots p of f(x, p)) times
 * s if x is a pivot and max(s - 1, 1) otherwise (so that a pivot's missing
 * self-term does not favour it: the ranking compares mean distances to the
 * pivots other than x), and the topk members with the least (E, input
 * index) are the candidates.  The candidates get exact row
 * sums over the cluster and c is the one with the least (lowest input index
 * on ties); poles and split stay exact.  A pruned cluster costs about
 * (pivots + topk) k distances instead of the medoid's k (k - 1) / 2.
 * 1 <= pivots <= 1024, 1 <= topk <= 1024, exact_below >= 0 (MSA_EINVAL
 * otherwise).  Same outputs, workspace and errors as tree_build. */
int tree_build_sampled(const msa_seqs *S, int32_t pivots, int32_t topk, int32_t exact_below,
                       const msa_tree *T, int32_t *n_nodes, int32_t use_graph, void *ws,
                       size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* Teacher-forced evaluation of the choice of c, l, r (Alg. 1) on the
 * clusters of a given tree: for every node v < n_nodes of T (as filled by
 * tree_build or tree_build_pruned over the same S; only depth, mstart,
 * mcount and perm are read), center[v], lpole[v] and rpole[v] (device
 * int32[n_nodes]) receive what the build picks for v's member set: with
 * emb == NULL the full geometric median, otherwise the pruned median of
 * tree_build_pruned (emb, emb_q0, topk, exact_below as there); poles are -1 for one member or
 * radius 0.  This is how a pruned choice is compared node by node with
 * the exact one.  The node table is copied to the host and checked
 * (breadth-first depths, disjoint in-range member ranges per depth:
 * EINVAL otherwise); perm entries outside [0, n) set MSA_DS_INDEX.
 * Workspace: tree_workspace_bytes(S).  Synchronizes the stream once. */
int tree_eval_centers(const msa_seqs *S, const float *emb, uint32_t emb_q0, int32_t topk,
                      int32_t exact_below, const msa_tree *T, int32_t n_nodes,
                      int32_t *center, int32_t *lpole, int32_t *rpole, void *ws,
                      size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* tree_eval_centers for the median of tree_build_sampled (same pivots,
 * topk and exact_below rules and errors). */
int tree_eval_centers_sampled(const msa_seqs *S, int32_t pivots, int32_t topk,
                              int32_t exact_below, const msa_tree *T, int32_t n_nodes,
                              int32_t *center, int32_t *lpole, int32_t *rpole, void *ws,
                              size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* Online insertion of new sequences into a tree (Sec. 5 names online
 * updates of the clusters, guide tree and alignment as future work and
 * gives no procedure; the reading here).  S holds n_old sequences (inputs
 * 0 .. n_old-1, the set T_old was built on by tree_build, n_nodes_old
 * nodes) followed by the new ones (inputs n_old .. S->n-1).
 *   1. Every new x starts at the root; at an internal node with poles l, r
 *      it goes to the left child if f(l, x) <= f(r, x), else to the right
 *      (Alg. 1's split rule), down to a leaf.  Internal nodes keep their
 *      center and poles.
 *   2. Each leaf that receives new sequences is replaced by Alg. 1 (the
 *      full median, tie rules as tree_build) on its old and new members.
 *   3. The result is renumbered breadth-first from the root (children after
 *      their level, in parent order, L before R), with member ranges and
 *      perm as tree_build lays them out.
 * T_new (device, capacity 2 S->n - 1 nodes and S->n perm entries, not
 * overlapping T_old) receives the tree of all S->n sequences and *n_nodes_new
 * (host) its node count; msa_merge(S, T_new, ...) then aligns the grown set.
 * Only left, right, center, lpole, rpole, mstart, mcount and perm of T_old
 * are read.  Routing computes one lev_batch of (pole, x) pairs per tree
 * depth and synchronizes the stream once per depth; the grown leaves are
 * re-partitioned together by the level passes of tree_build.  Members of a
 * leaf that holds copies of one sequence come in unspecified order.
 * Errors: MSA_EINVAL for n_old outside [1, S->n], n_nodes_old outside
 * [1, 2 n_old - 1], null pointers, or a child cycle in T_old; MSA_ERANGE for
 * S->n >= 2^24; MSA_ENOSPC for a workspace below
 * tree_insert_workspace_bytes(S, n_old, n_nodes_old).  Node or pole ids out
 * of range in T_old set MSA_DS_INDEX (*n_nodes_new is then 0 or the tree
 * incomplete). */
size_t tree_insert_workspace_bytes(const msa_seqs *S, int32_t n_old, int32_t n_nodes_old);
int tree_insert(const msa_seqs *S, int32_t n_old, const msa_tree *T_old, int32_t n_nodes_old,
                const msa_tree *T_new, int32_t *n_nodes_new, void *ws, size_t ws_bytes,
                int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Bottom-up merge (Sec. 2.2) over a tree from tree_build (T, n_nodes as
 * returned).  A leaf's alignment is its sequence.  For an internal node the
 * aligned rows of its children's centers (each child's Alg. 1 medoid) are
 * aligned by nw_batch/nw_traceback with the gap as an ordinary symbol (code
 * S->sigma, so S->sigma <= 31), then the L child's rows get an all-gap column
 * at every I op, the R child's rows one at every D op, and the rows are
 * joined, L's first.  Output: msa (device, S->n rows of msa_pitch bytes,
 * row i = sequence i, gap = S->sigma, columns >= *width undefined); *width
 * (host) = the final width.  width_cap bounds every node's width (<= 32768)
 * and tb_cap the traceback bytes of one tree level; exceeding either returns
 * MSA_ENOSPC.  The stream is synchronized once per tree level. */
size_t msa_merge_workspace_bytes(const msa_seqs *S, int32_t n_nodes, int32_t width_cap,
                                 size_t tb_cap);
int msa_merge(const msa_seqs *S, const msa_tree *T, int32_t n_nodes, int32_t width_cap,
              size_t tb_cap, uint8_t *msa, int64_t msa_pitch, int32_t *width, void *ws,
              size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Learned surrogate of f (not part of the paper; used to prune the exact
 * medoid work of Alg. 1).  A 1D-CNN embedder with a fixed shape: one-hot
 * input over 8 channels (sigma <= 8), 4 conv layers of width 128 and kernel
 * 5 with zero padding, ReLU after layers 1-3, mean over the sequence ->
 * 128-d embedding; trained so that ||e_a - e_b|| approximates
 * lev(a, b) / ((|a| + |b|) / 2) (mean squared error over pairs, Adam).
 * BF16 weights/activations, FP32 accumulation on the matrix cores, FP32
 * master weights and Adam state, all in one device blob of
 * cnn_param_bytes() bytes owned by the caller. */
size_t cnn_param_bytes(void);

/* Load weights from host: per layer l, W[k][cin_l][128] (cin_0 = 8, the
 * one-hot channels beyond sigma zero; cin_l = 128 after) concatenated over
 * layers, and b[l][128].  Resets the Adam state.  Synchronous. */
int cnn_set_params(void *params, const float *w_host, const float *b_host, hipStream_t s);

/* Copy master weights and the last step's gradients back to host (any of
 * the four pointers may be null).  Synchronizes the stream. */
int cnn_get_params(const void *params, float *w_host, float *b_host, float *gw_host,
                   float *gb_host, hipStream_t s);

/* Workspace of a batch of n_idx sequences of total length total_len
 * (n_pairs = 0 for inference). */
size_t cnn_workspace_bytes(const msa_seqs *S, int32_t n_idx, int64_t total_len, int32_t n_pairs);

/* Embeddings of the sequences S[idx[i]] (idx: device int32[n_idx];
 * total_len = their summed length, checked on the device): emb (device
 * float[n_idx][128]). */
int cnn_embed(const void *params, const msa_seqs *S, const int32_t *idx, int32_t n_idx,
              int64_t total_len, float *emb, void *ws, size_t ws_bytes, int32_t *d_status,
              hipStream_t s);

/* One training step on the pairs (idx[pa[p]], idx[pb[p]]) with exact
 * distances dist[p] (device uint16, e.g. from lev_batch): forward, loss,
 * backward, and an Adam update with learning rate lr at step `step` (>= 1);
 * lr == 0 computes gradients only.  *loss (device float) receives the mean
 * squared error before the update. */
int cnn_train_step(void *params, const msa_seqs *S, const int32_t *idx, int32_t n_idx,
                   int64_t total_len, const int32_t *pa, const int32_t *pb,
                   const uint16_t *dist, int32_t n_pairs, float lr, int32_t step, float *loss,
                   void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Tuning table (not in the paper): the launch variant of a kernel family
 * per (kind, alphabet size sigma, length bin), used in place of the
 * library's default.  Thread-safe; process-wide; empty at load.
 *   MSA_TUNE_LEV: bin = ceil(max_len / 64) of the pattern set (A of
 *     lev_batch / lev_allpairs); value = 64-bit words per pass of the
 *     kernel variant (4, 8, 16, 20, 24, 28, 32).  Fewer words per pass than
 *     the longest pattern needs means several passes; more words cost
 *     registers and so resident wavefronts.  Default: the smallest of
 *     4, 8, 16, 24, 32 that holds the longest pattern (32 beyond).
 *   MSA_TUNE_NW: bin = wavefronts per pair, ceil(ceil(max_len_A / 32) / 64);
 *     value = steps between the fill's workgroup barriers (16, 32, 64;
 *     default 32).
 *   MSA_TUNE_TREE: bin = ceil(max_len / 64) of the set of tree_build,
 *     tree_build_pruned and tree_eval_centers; value = 64-bit words per pass
 *     of their Levenshtein kernels (4, 8, 16, 20, 24, 32; default as for
 *     MSA_TUNE_LEV).  An entry that would take more passes than the default
 *     (and more than two) is ignored.
 *   MSA_TUNE_PAIRS: bin = ceil(max(A->max_len, B->max_len) / 64) of a
 *     lev_batch call; value = the layout: 1 (every lane holds its own pair
 *     and pattern, pairs binned by pattern words and text length), 2 (a
 *     pair per group of lanes: one 64-bit word per lane in the least power
 *     of two of at least 8 lanes holding the longest pattern, else 64 lanes
 *     of 2, 3 or 4 words) or 64 (pairs grouped by A sequence, a wavefront
 *     takes 64 pairs of one pattern).  1 needs patterns of at most
 *     32 / sigma' words (sigma' = 4, 8, 32 for sigma <= 4, <= 8, <= 32) and
 *     is the default when they fit; 2 needs at most 256 words and is the
 *     default for longer patterns when the list holds fewer than 16 pairs
 *     per A sequence; else 64.  An entry whose layout does not fit is
 *     ignored.
 *   MSA_TUNE_TREE_XL: bin as for MSA_TUNE_TREE; value = which distance
 *     passes of the tree builds run with one pair per group of lanes (the
 *     pattern's 64-bit words spread over the group, carries passed lane to
 *     lane), packing the pairs of several small clusters into one wavefront:
 *     (WL << 28) | (pole cap << 14) | sum cap, WL = words per lane (1 or 2),
 *     the group = the least power of two of lanes holding the longest
 *     pattern (at most 64); clusters of at most `sum cap` members take
 *     their medoid, pivot and candidate passes that way, clusters of at
 *     most `pole cap` their pole passes (cap 0: none, 16383: every
 *     cluster).  Default WL 2, sum cap 128, pole cap 16383; patterns of more
 *     than 64 WL words use the one-wavefront-per-pattern passes only.
 * Workspace sizes never depend on the table.  Results never depend on it
 * (every variant computes the same exact values). */
enum { MSA_TUNE_LEV = 0, MSA_TUNE_NW = 1, MSA_TUNE_TREE = 2, MSA_TUNE_PAIRS = 3,
       MSA_TUNE_TREE_XL = 4 };

/* Set one entry (EINVAL for an unknown kind, a key out of range or a value
 * that is not a variant of the kind). */
int msa_tune_set(int32_t kind, int32_t sigma, int32_t bin, int32_t value);
/* *value = the entry, or 0 when the table has none. */
int msa_tune_get(int32_t kind, int32_t sigma, int32_t bin, int32_t *value);
int msa_tune_clear(void);
/* The variants of a kind: values[0 .. *count) (ENOSPC if cap < *count). */
int msa_tune_candidates(int32_t kind, int32_t *values, int32_t cap, int32_t *count);
/* The table as JSON text {"arch": "<gfx name>", "entries": [[kind, sigma,
 * bin, value], ...]} into buf (host, cap bytes with the terminating zero;
 * *len = its length; ENOSPC when it does not fit). */
int msa_tune_export(char *buf, size_t cap, size_t *len);
/* Merge entries from text in the export format; EINVAL (table unchanged)
 * if the arch differs from the current device or an entry is invalid. */
int msa_tune_import(const char *json);

/* Autotuning: time every lev_allpairs variant that needs no more passes
 * than the default (at least two allowed) on the set A, reps timed runs
 * each after one warm-up (same arguments as lev_allpairs; the condensed
 * output holds the last run's exact distances), then store the fastest
 * for (MSA_TUNE_LEV, A->sigma, ceil(A->max_len / 64)).  *best = its words
 * per pass, *best_ms = its mean time per call.  Synchronizes the stream. */
int msa_autotune_lev(const msa_seqs *A, uint16_t *condensed, void *ws, size_t ws_bytes,
                     int32_t reps, int32_t *best, float *best_ms, int32_t *d_status,
                     hipStream_t s);
/* The same for nw_batch (same arguments as nw_batch): every barrier
 * interval, fastest stored for (MSA_TUNE_NW, A->sigma, wavefronts per pair
 * of A->max_len). */
int msa_autotune_nw(const msa_seqs *A, const msa_seqs *B, const int32_t *ia, const int32_t *ib,
                    int64_t n_pairs, int32_t *score, uint8_t *tb, const int64_t *tb_offsets,
                    void *ws, size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                    int32_t *d_status, hipStream_t s);
/* The same for the pair-list layout of lev_batch (same arguments as
 * lev_batch; dist holds the last run's exact distances): every layout the
 * patterns fit (64 always, 1 and 2 under the limits of MSA_TUNE_PAIRS),
 * fastest stored for (MSA_TUNE_PAIRS, A->sigma, ceil(max(A->max_len,
 * B->max_len) / 64)); *best = 1, 2 or 64.  n_pairs >= 1. */
int msa_autotune_pairs(const msa_seqs *A, const msa_seqs *B, const int32_t *ia,
                       const int32_t *ib, int64_t n_pairs, uint16_t *dist, void *ws,
                       size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                       int32_t *d_status, hipStream_t s);
/* The same for the exact tree_build (same arguments as tree_build; T and
 * *n_nodes hold the last run's tree): every class within the default's
 * passes (at least two), fastest stored for (MSA_TUNE_TREE, S->sigma,
 * ceil(S->max_len / 64)).  S->n >= 2. */
int msa_autotune_tree(const msa_seqs *S, const msa_tree *T, int32_t *n_nodes, int32_t use_graph,
                      void *ws, size_t ws_bytes, int32_t reps, int32_t *best, float *best_ms,
                      int32_t *d_status, hipStream_t s);

/* Time the tree build once per across-lanes variant (msa_tune_candidates of
 * MSA_TUNE_TREE_XL: off, pole passes only, and both kinds of pass up to
 * cluster caps of 32 .. 256 members or for every cluster, with one or two
 * words per lane) and store the fastest for (MSA_TUNE_TREE_XL, S->sigma,
 * ceil(S->max_len / 64)).  pivots > 0 times tree_build_sampled(S, pivots,
 * topk, 0, ...), pivots = 0 the exact tree_build.  Every variant builds the
 * same tree (left in T, *n_nodes).  Arguments otherwise as tree_build;
 * *best = the value stored, *best_ms = its time per build. */
int msa_autotune_tree_xl(const msa_seqs *S, int32_t pivots, int32_t topk, const msa_tree *T,
                         int32_t *n_nodes, int32_t use_graph, void *ws, size_t ws_bytes,
                         int32_t reps, int32_t *best, float *best_ms, int32_t *d_status,
                         hipStream_t s);

/* ------------------------------------------------------------------ */
/* Alignment quality (Sec. 2.3: percentage of gaps, p-score, distance
 * distortion; Table 2 also reports width and stretch).  msa: device,
 * rows x width row-major symbol codes as msa_merge writes them, every code
 * in [0, gap_code], gap_code <= 63 the gap symbol.  Readings where the
 * paper gives no formula: a column of two gaps counts as equal; the p-score
 * of a pair is (aligned columns whose residues differ) / (columns with a
 * residue in both rows), pairs with no such column left out, reported as
 * min / mean / max over pairs; the distortion of a pair is its Hamming
 * distance over the Levenshtein distance of the unaligned sequences, pairs
 * at distance 0 left out, averaged over pairs; % gaps = 100 x the mean
 * over rows of gaps / width; stretch = width / max_len.  A code above
 * gap_code sets MSA_DS_SYMBOL, a pair index outside [0, rows) MSA_DS_INDEX. */

/* Workspace for msa_pair_counts and msa_quality (0 for invalid sizes). */
size_t msa_quality_workspace_bytes(int32_t rows, int32_t width, int32_t gap_code);

/* Per pair p: hamming[p] = columns whose symbols differ, aligned[p] =
 * columns where neither row holds a gap, mismatched[p] = aligned columns
 * whose symbols differ (device int32[n_pairs] each).  Pairs (ia[p], ib[p])
 * (device int32), or with ia == ib == NULL every pair i < j of the rows at
 * the condensed index i*rows - i*(i+1)/2 + (j - i - 1), the order of
 * lev_allpairs (n_pairs must then be rows*(rows-1)/2). */
int msa_pair_counts(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap_code,
                    const int32_t *ia, const int32_t *ib, int64_t n_pairs, int32_t *hamming,
                    int32_t *aligned, int32_t *mismatched, void *ws, size_t ws_bytes,
                    int32_t *d_status, hipStream_t s);

/* The metrics from the counts of msa_pair_counts and lev[p] (device uint16,
 * the distance of pair p's unaligned sequences, e.g. lev_allpairs' output;
 * NULL skips the distortion).  out: device double[8] = {pct_gaps, p_min,
 * p_avg, p_max, distortion, stretch, pairs in the p-score, pairs in the
 * distortion}; a metric with no pair is 0.  The sums run in a fixed order,
 * so equal inputs give equal bits. */
int msa_quality(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap_code,
                int32_t max_len, const int32_t *hamming, const int32_t *aligned,
                const int32_t *mismatched, const uint16_t *lev, int64_t n_pairs, double *out,
                void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Machine-rate probes.  These compute nothing from the method: they are
 * the measured counterparts of the vendor peaks (VALU lane-ops/s, MFMA
 * operations/s, HBM bytes/s) against which the roofline fractions of the
 * kernels above are read.  Each launches one kernel of `blocks` workgroups
 * of 256 threads on s and returns at once; the caller times the launch.
 * They return MSA_EINVAL for blocks <= 0, iters <= 0, null pointers or an
 * unknown kind, and MSA_EDEVICE for a failed launch. */

/* Eight independent chains of 32-bit xor / add per lane (a ^= b; b += a),
 * iters trips of 128 VALU instructions each.  sink: device, blocks * 256 uint32 (written, its
 * values meaningless).  *ops (host) = lane-instructions of the launch. */
int msa_probe_valu(int32_t blocks, int32_t iters, uint32_t *sink, int64_t *ops, hipStream_t s);

enum {
    MSA_PROBE_MFMA_BF16_16X16X32 = 0,   /* v_mfma_f32_16x16x32_bf16 (the CNN) */
    MSA_PROBE_MFMA_BF16_32X32X16 = 1,   /* v_mfma_f32_32x32x16_bf16           */
    MSA_PROBE_MFMA_I8_16X16X64 = 2,     /* v_mfma_i32_16x16x64_i8 (pair dist.) */
    MSA_PROBE_MFMA_I8_32X32X32 = 3      /* v_mfma_i32_32x32x32_i8             */
};
/* Eight independent accumulators per wavefront, iters trips of sixteen
 * matrix instructions of the given kind (two per accumulator).  sink: as above.  *ops (host) =
 * 2 * M * N * K per instruction times the instructions of the launch. */
int msa_probe_mfma(int32_t kind, int32_t blocks, int32_t iters, uint32_t *sink, int64_t *ops,
                   hipStream_t s);

/* Streaming copy of `bytes` (a multiple of 16) from src to dst (device,
 * 16-byte aligned, not overlapping), 16 bytes per lane per access with
 * non-temporal loads and stores.  bytes == 0 launches nothing. */
int msa_probe_copy(const void *src, void *dst, size_t bytes, int32_t blocks, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif /* MSADP_H */
