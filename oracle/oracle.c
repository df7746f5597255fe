/*
 * CPU oracle for the pairwise dynamic programs of MuSAlS (arXiv 2601.15458).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by the smoke check and by the
 * benchmark's CPU-baseline leg.  It shares no code, header, table or helper
 * with the device library; it reads the same seeded inputs and nothing else.
 *
 * Everything here is the plain, slow textbook form of each definition:
 *   - Levenshtein distance: the Wagner-Fischer recurrence with two rolling
 *     rows (Sec. 2 and Alg. 1 use Levenshtein as the distance f; Sec. 2.4
 *     says exact Levenshtein, not an approximation).
 *   - Needleman-Wunsch with unit costs (match 0, mismatch 1, gap 1) over the
 *     full (m+1) x (n+1) score matrix, then a backward walk that at each cell
 *     takes the first of diagonal / up / left that reproduces the cell's
 *     value (Sec. 2.2 step 2 aligns the two centers and records the gap
 *     positions; the tie order diag > up > left is this project's reading,
 *     the paper names none).
 *   - Needleman-Wunsch with a substitution score matrix and affine gaps
 *     (Gotoh's three matrices in full), the cost model of Sec. 2.4, with
 *     the walk that returns the best-scoring alignment whose backward op
 *     string is smallest (M < D < I).
 *   - Alg. 1 (Partition) with the full geometric median (Sec. 2.1), and
 *     the same with the median taken over candidates that a learned
 *     embedding ranks first (a surrogate of this project, not the paper's)
 *     or that their summed distance to a few hashed members ranks first
 *     (the median over a smaller subset that Sec. 2.1 allows).
 *   - Insertion of new sequences into an existing tree (Sec. 5 names it
 *     as future work; the routing and re-partition rules are this
 *     project's reading, stated at orc_tree_insert).
 *   - The bottom-up merge of Sec. 2.2.
 *   - The column counts behind the alignment-quality metrics of Sec. 2.3
 *     (gaps per row; per pair of rows the Hamming distance, the columns
 *     where both rows hold a residue, and how many of those differ).
 * Pairs are independent, so OpenMP spreads them over host threads; that is
 * the only concession to speed.
 *
 * Symbols are uint8 codes; sequence k of a set is codes[off[k] .. off[k+1]).
 * Alignment ops: 0 = M (a_i with b_j), 1 = D (a_i with a gap),
 * 2 = I (a gap with b_j).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t imin3(int64_t x, int64_t y, int64_t z) {
    int64_t r = x < y ? x : y;
    return r < z ? r : z;
}

/* Levenshtein distance by Wagner-Fischer:
 *   D[i][0] = i, D[0][j] = j,
 *   D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a_i != b_j]).
 * Only two rows are kept; the result is D[m][n]. */
int64_t orc_lev(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n) {
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t j = 0; j <= n; ++j) prev[j] = j;
    for (int64_t i = 1; i <= m; ++i) {
        cur[0] = i;
        for (int64_t j = 1; j <= n; ++j) {
            int64_t sub = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0);
            cur[j] = imin3(prev[j] + 1, cur[j - 1] + 1, sub);
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    int64_t d = prev[n];
    free(prev);
    free(cur);
    return d;
}

/* out[p] = lev(A[ia[p]], B[ib[p]]) for every pair p. */
void orc_lev_pairs(const uint8_t *ca, const int64_t *oa, const uint8_t *cb,
                   const int64_t *ob, const int32_t *ia, const int32_t *ib,
                   int64_t n_pairs, int64_t *out) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const uint8_t *a = ca + oa[ia[p]];
        const uint8_t *b = cb + ob[ib[p]];
        out[p] = orc_lev(a, oa[ia[p] + 1] - oa[ia[p]], b, ob[ib[p] + 1] - ob[ib[p]]);
    }
}

/* Needleman-Wunsch, unit costs, full matrix, then the backward walk:
 * at (i, j) take M if D[i-1][j-1] + [a_i != b_j] == D[i][j], else D (up)
 * if D[i-1][j] + 1 == D[i][j], else I (left).  The op string is written in
 * forward order to ops[0 .. *ops_len).  Returns D[m][n]. */
int64_t orc_nw(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
               uint8_t *ops, int64_t *ops_len) {
    const int64_t w = n + 1;
    int32_t *D = (int32_t *)malloc(sizeof(int32_t) * (size_t)((m + 1) * w));
    for (int64_t j = 0; j <= n; ++j) D[j] = (int32_t)j;
    for (int64_t i = 1; i <= m; ++i) {
        D[i * w] = (int32_t)i;
        for (int64_t j = 1; j <= n; ++j) {
            int64_t sub = D[(i - 1) * w + j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0);
            D[i * w + j] = (int32_t)imin3(D[(i - 1) * w + j] + 1, D[i * w + j - 1] + 1, sub);
        }
    }
    int64_t score = D[m * w + n];
    if (ops != NULL) {
        int64_t i = m, j = n, k = 0;
        while (i > 0 || j > 0) {
            int32_t here = D[i * w + j];
            if (i > 0 && j > 0 &&
                D[(i - 1) * w + j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0) == here) {
                ops[k++] = 0; --i; --j;
            } else if (i > 0 && D[(i - 1) * w + j] + 1 == here) {
                ops[k++] = 1; --i;
            } else {
                ops[k++] = 2; --j;
            }
        }
        for (int64_t x = 0, y = k - 1; x < y; ++x, --y) {
            uint8_t t = ops[x]; ops[x] = ops[y]; ops[y] = t;
        }
        *ops_len = k;
    }
    free(D);
    return score;
}

/* NW over pairs; ops for pair p go to ops[ops_off[p] ..], its length to
 * ops_len[p] (ops may be NULL for scores only). */
void orc_nw_pairs(const uint8_t *ca, const int64_t *oa, const uint8_t *cb,
                  const int64_t *ob, const int32_t *ia, const int32_t *ib,
                  int64_t n_pairs, int64_t *score, uint8_t *ops,
                  const int64_t *ops_off, int64_t *ops_len) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const uint8_t *a = ca + oa[ia[p]];
        const uint8_t *b = cb + ob[ib[p]];
        int64_t m = oa[ia[p] + 1] - oa[ia[p]], n = ob[ib[p] + 1] - ob[ib[p]];
        score[p] = orc_nw(a, m, b, n, ops ? ops + ops_off[p] : NULL,
                          ops ? ops_len + p : NULL);
    }
}

/* ------------------------------------------------------------ affine NW
 * Global alignment under the cost model of the paper's experiments
 * (Sec. 2.4): a substitution score matrix for aligned residues and affine
 * gaps, opening charged ten times the extension there (the ratio is the
 * caller's here).  Reading, as the paper gives no formula: a run of k gap
 * symbols in one row scores -(open + k * ext), and the aligner maximizes
 *   sum over M columns of sub[a_i * sigma + b_j]  -  sum over gap runs of
 *   (open + ext * run length),
 * where a run is a maximal stretch of consecutive D ops or of consecutive I
 * ops.  Gotoh's three matrices, in full:
 *   E[i][j] = best prefix score of a[1..i], b[1..j] ending with I,
 *   F[i][j] = ... ending with D,  H[i][j] = ... ending with anything:
 *   E[i][j] = max(E[i][j-1] - ext, H[i][j-1] - open - ext)
 *   F[i][j] = max(F[i-1][j] - ext, H[i-1][j] - open - ext)
 *   H[i][j] = max(H[i-1][j-1] + sub[a_i][b_j], E[i][j], F[i][j])
 *   H[0][0] = 0;  H[i][0] = F[i][0] = -(open + i ext);
 *   H[0][j] = E[0][j] = -(open + j ext);  E[i][0], F[0][j] = -infinity.
 * The alignment returned is, among those of the best score, the one whose
 * op string read backwards is smallest with M < D < I (the order of the
 * unit-cost walk).  It is found by walking back from (m, n) and taking at
 * each step the least op through which some best-scoring prefix completes
 * the part already chosen.  `need` is the score the remaining prefix must
 * reach, counted with a bonus of `open` when the prefix ends in the same gap
 * op that the chosen part starts with (the two then form one run).  The
 * best prefix ending with M, D or I at (i, j) scores H[i-1][j-1] + sub, F,
 * E; a candidate completes iff that plus its bonus equals `need` (it can
 * never exceed it).  Scores here stay far inside int32 (|sub| and open +
 * ext at most 2048, lengths at most 65535). */
#define ORC_NEG_INF (-(1 << 30))

int64_t orc_gotoh(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                  const int32_t *sub, int32_t sigma, int32_t open, int32_t ext,
                  uint8_t *ops, int64_t *ops_len) {
    const int64_t w = n + 1;
    const size_t cells = (size_t)((m + 1) * w);
    int32_t *H = (int32_t *)malloc(sizeof(int32_t) * cells);
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * cells);
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * cells);
    H[0] = 0;
    E[0] = F[0] = ORC_NEG_INF;
    for (int64_t j = 1; j <= n; ++j) {
        H[j] = E[j] = -(open + (int32_t)j * ext);
        F[j] = ORC_NEG_INF;
    }
    for (int64_t i = 1; i <= m; ++i) {
        H[i * w] = F[i * w] = -(open + (int32_t)i * ext);
        E[i * w] = ORC_NEG_INF;
        for (int64_t j = 1; j <= n; ++j) {
            const int64_t c = i * w + j;
            const int32_t e1 = E[c - 1] - ext, e2 = H[c - 1] - open - ext;
            const int32_t f1 = F[c - w] - ext, f2 = H[c - w] - open - ext;
            E[c] = e1 > e2 ? e1 : e2;
            F[c] = f1 > f2 ? f1 : f2;
            int32_t h = H[c - w - 1] + sub[a[i - 1] * sigma + b[j - 1]];
            if (E[c] > h) h = E[c];
            if (F[c] > h) h = F[c];
            H[c] = h;
        }
    }
    const int64_t score = H[m * w + n];
    if (ops != NULL) {
        int64_t i = m, j = n, k = 0, need = score;
        int last = -1;   /* first op of the part already chosen (-1: none) */
        while (i > 0 || j > 0) {
            const int64_t c = i * w + j;
            const int64_t bd = last == 1 ? open : 0, bi = last == 2 ? open : 0;
            int op;
            if (i > 0 && j > 0 && H[c - w - 1] + sub[a[i - 1] * sigma + b[j - 1]] == need)
                op = 0;
            else if (i > 0 && F[c] + bd == need)
                op = 1;
            else
                op = 2;   /* E[c] + bi == need: the only op left */
            if (op == 0) {
                need -= sub[a[i - 1] * sigma + b[j - 1]];
                --i; --j;
            } else if (op == 1) {
                need = need - bd + open + ext;
                --i;
            } else {
                need = need - bi + open + ext;
                --j;
            }
            ops[k++] = (uint8_t)op;
            last = op;
        }
        for (int64_t x = 0, y = k - 1; x < y; ++x, --y) {
            uint8_t t = ops[x]; ops[x] = ops[y]; ops[y] = t;
        }
        *ops_len = k;
    }
    free(H);
    free(E);
    free(F);
    return score;
}

/* Affine NW over pairs (ops as for orc_nw_pairs; ops may be NULL). */
void orc_gotoh_pairs(const uint8_t *ca, const int64_t *oa, const uint8_t *cb,
                     const int64_t *ob, const int32_t *ia, const int32_t *ib,
                     int64_t n_pairs, const int32_t *sub, int32_t sigma, int32_t open,
                     int32_t ext, int64_t *score, uint8_t *ops, const int64_t *ops_off,
                     int64_t *ops_len) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const uint8_t *a = ca + oa[ia[p]];
        const uint8_t *b = cb + ob[ib[p]];
        int64_t m = oa[ia[p] + 1] - oa[ia[p]], n = ob[ib[p] + 1] - ob[ib[p]];
        score[p] = orc_gotoh(a, m, b, n, sub, sigma, open, ext,
                             ops ? ops + ops_off[p] : NULL, ops ? ops_len + p : NULL);
    }
}

/* ------------------------------------------------------------------ Alg. 1
 * Partition(C): if |C| > 1 then c = geometric median of C (the member with
 * the least sum of distances to the members of C), l = argmax_x f(c, x),
 * r = argmax_x f(l, x), L = {x : f(l,x) <= f(r,x)}, R = {x : f(r,x) < f(l,x)},
 * recurse on L and R.  Readings fixed here: every argmin/argmax scans members
 * in ascending index order and keeps the first optimum (lowest index); a
 * cluster whose radius max_x f(c, x) is 0 (only copies of one sequence)
 * becomes a leaf.
 *
 * Nodes are numbered breadth-first (children of node v are created when v is
 * split, L before R).  Members of every node are a contiguous range of
 * `perm`: a node's range is its L child's range followed by its R child's.
 * Per node: parent, left, right (-1 if none), center, lpole, rpole (-1 for
 * leaves), depth, mstart, mcount.  Returns the node count (<= 2n-1). */
typedef struct {
    int32_t parent, left, right, center, lpole, rpole, depth;
    int64_t mstart, mcount;
} orc_node;

static int64_t dist_of(const uint8_t *codes, const int64_t *off, int32_t x, int32_t y) {
    return orc_lev(codes + off[x], off[x + 1] - off[x], codes + off[y], off[y + 1] - off[y]);
}

/* Surrogate distance of two embeddings (128 floats each).  The embeddings of
 * the set are quantized once: with M the largest |e| over every coordinate
 * of every row, s = 40 if M < 2^-34 (zero included), else s = 6 -
 * floor(log2 M) limited to [-20, 40], so that M 2^s lies in [64, 128); each
 * coordinate becomes the integer rint(e 2^s) limited to [-127, 127].  The
 * distance of x and y is sqrt(D) 2^-s with D the squared Euclidean distance
 * of their integer vectors (exact), in float32: the square root of D
 * (correctly rounded; D < 2^24 is exact in float32), the product with 2^-s
 * (exact), the cap at 2^15, then 2^16 times that rounded to the nearest
 * integer (ties to even).  Rounding decides the candidate ranking, so both
 * sides take these float32 steps; everything before them is integer and the
 * sums after them are integers.  Embeddings are taken to be finite. */
#define EMB_DIM 128

static int emb_shift(const float *emb, int64_t count) {
    float M = 0.0f;
    for (int64_t i = 0; i < count; ++i) {
        const float a = fabsf(emb[i]);
        if (a > M) M = a;
    }
    if (!(M >= ldexpf(1.0f, 6 - 40))) return 40;
    int E;
    frexpf(M, &E);                 /* M = f 2^E with f in [0.5, 1): floor(log2 M) = E - 1 */
    const int s = 6 - (E - 1);
    return s < -20 ? -20 : (s > 40 ? 40 : s);
}

/* codes: int8[n][128]; returns s. */
int32_t orc_emb_quantize(const float *emb, int64_t n, int8_t *codes) {
    const int s = emb_shift(emb, n * EMB_DIM);
    const float scale = ldexpf(1.0f, s);
    for (int64_t i = 0; i < n * EMB_DIM; ++i) {
        float v = rintf(emb[i] * scale);
        if (v > 127.0f) v = 127.0f;
        if (v < -127.0f) v = -127.0f;
        codes[i] = (int8_t)v;
    }
    return s;
}

static uint64_t emb_dist_q(const int8_t *cx, const int8_t *cy, int shift) {
    int64_t D = 0;
    for (int c = 0; c < EMB_DIM; ++c) {
        const int64_t d = (int64_t)cx[c] - (int64_t)cy[c];
        D += d * d;
    }
    const float dist = sqrtf((float)D) * ldexpf(1.0f, -shift);
    return (uint64_t)rintf(fminf(dist, 32768.0f) * 65536.0f);
}

/* The estimate of f(x, y) behind the ranking, in units of 2^-17: the
 * embedder predicts f divided by the pair's mean length, so the distance
 * plus the calibration offset q0 (units of 2^-16) is scaled by |x| + |y|. */
static uint64_t emb_estimate(const int64_t *off, const int8_t *code, int shift, uint32_t q0,
                             int32_t x, int32_t y) {
    const uint64_t len = (uint64_t)((off[x + 1] - off[x]) + (off[y + 1] - off[y]));
    return (emb_dist_q(code + (int64_t)x * EMB_DIM, code + (int64_t)y * EMB_DIM, shift) + q0) *
           len;
}

/* f(C[x], C[y]) for every y of the cluster. */
static int64_t *dist_row(const uint8_t *codes, const int64_t *off, const int32_t *C, int64_t k,
                         int64_t x) {
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t y = 0; y < k; ++y) row[y] = dist_of(codes, off, C[x], C[y]);
    return row;
}

/* The pivot order of the sampled median: MurmurHash3's 32-bit finalizer
 * (Appleby), a bijection, of the input index; the pivots of a cluster are
 * its members with the least values. */
static uint32_t pivot_hash(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* The choice Alg. 1 makes for one cluster C (ascending input indices, k
 * members): out[0] = c, out[1] = l = argmax f(c, x), out[2] = r = argmax
 * f(l, x) (lowest index on ties; l = r = -1 when k = 1 or the radius
 * f(c, l) is 0).  emb == NULL and pivots == 0: c is the full geometric
 * median of C (Sec. 2.1).  Otherwise c is a pruned median: if C has more
 * than exact_below members, every member x gets an estimate E(x) and the
 * topk members with the least (E, input index) are the candidates, else
 * every member is one; c is the candidate with the least exact sum of f
 * over C (lowest input index on ties).  The estimate is either the sum over
 * C (x itself included) of emb_estimate (ecode != NULL), or, with pivots > 0,
 * the sum of f(x, p) over the s = min(pivots, k) members p of least
 * pivot_hash (the median over a smaller subset that Sec. 2.1 allows, with
 * the subset drawn by the hash), times s for a pivot and max(s - 1, 1) for
 * any other member: a pivot's sum lacks the term of itself, so the ranking
 * compares each member's mean distance to the pivots other than itself. */
static void select_impl(const uint8_t *codes, const int64_t *off, const int32_t *C, int64_t k,
                        const int8_t *ecode, int eshift, uint32_t emb_q0, int32_t topk,
                        int32_t exact_below, int32_t pivots, int32_t out[3]) {
    out[1] = out[2] = -1;
    if (k == 1) { out[0] = C[0]; return; }
    int64_t best = -1;
    int64_t *rowc;
    if (ecode == NULL && pivots <= 0) {
        /* geometric median over the whole cluster */
        int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k * k));
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t x = 0; x < k; ++x) {
            D[x * k + x] = 0;
            for (int64_t y = x + 1; y < k; ++y) {
                int64_t d = dist_of(codes, off, C[x], C[y]);
                D[x * k + y] = d;
                D[y * k + x] = d;
            }
        }
        int64_t best_sum = 0;
        for (int64_t x = 0; x < k; ++x) {
            int64_t s = 0;
            for (int64_t y = 0; y < k; ++y) s += D[x * k + y];
            if (best < 0 || s < best_sum) { best = x; best_sum = s; }
        }
        rowc = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        memcpy(rowc, D + best * k, sizeof(int64_t) * (size_t)k);
        free(D);
    } else {
        uint64_t *E = (uint64_t *)calloc((size_t)k, sizeof(uint64_t));
        if (ecode != NULL) {
            #pragma omp parallel for schedule(dynamic, 1)
            for (int64_t x = 0; x < k; ++x)
                for (int64_t y = 0; y < k; ++y)
                    E[x] += emb_estimate(off, ecode, eshift, emb_q0, C[x], C[y]);
        } else if (k > exact_below && k > topk) {
            char *piv = (char *)calloc((size_t)k, 1);
            const int64_t np = pivots < k ? pivots : k;
            for (int64_t j = 0; j < np; ++j) {
                int64_t p = -1;   /* least hash not yet taken */
                for (int64_t x = 0; x < k; ++x)
                    if (!piv[x] && (p < 0 || pivot_hash((uint32_t)C[x]) <
                                                 pivot_hash((uint32_t)C[p])))
                        p = x;
                if (p < 0) break;
                piv[p] = 1;
                int64_t *row = dist_row(codes, off, C, k, p);
                for (int64_t x = 0; x < k; ++x) E[x] += (uint64_t)row[x];
                free(row);
            }
            /* a pivot's sum has one term fewer (its distance to itself is
             * 0): compare means over the other pivots, scaled to integers,
             * E(x) * (np if x is a pivot else max(np - 1, 1)) */
            for (int64_t x = 0; x < k; ++x)
                E[x] *= (uint64_t)(piv[x] ? np : (np > 1 ? np - 1 : 1));
            free(piv);
        }
        char *taken = (char *)calloc((size_t)k, 1);
        int64_t best_sum = 0;
        const int64_t nc = k <= exact_below ? k : (k < topk ? k : topk);
        for (int64_t j = 0; j < nc; ++j) {
            int64_t cand = -1;   /* least (E, index) not yet taken */
            for (int64_t x = 0; x < k; ++x)
                if (!taken[x] && (cand < 0 || E[x] < E[cand])) cand = x;
            if (cand < 0) break;
            taken[cand] = 1;
            int64_t *row = dist_row(codes, off, C, k, cand);
            int64_t s = 0;
            for (int64_t y = 0; y < k; ++y) s += row[y];
            free(row);
            if (best < 0 || s < best_sum || (s == best_sum && cand < best)) {
                best = cand;
                best_sum = s;
            }
        }
        free(taken);
        free(E);
        rowc = dist_row(codes, off, C, k, best);
    }
    out[0] = C[best];
    int64_t lp = 0;
    for (int64_t x = 1; x < k; ++x) if (rowc[x] > rowc[lp]) lp = x;
    const int64_t radius = rowc[lp];
    free(rowc);
    if (radius == 0) return;   /* radius 0: the cluster stays a leaf */
    int64_t *rowl = dist_row(codes, off, C, k, lp);
    int64_t rp = 0;
    for (int64_t x = 1; x < k; ++x) if (rowl[x] > rowl[rp]) rp = x;
    free(rowl);
    out[1] = C[lp];
    out[2] = C[rp];
}

/* emb: float[n_emb][128] of the whole input set (the quantization scale
 * comes from all of it), or NULL for the full median. */
void orc_select(const uint8_t *codes, const int64_t *off, const int32_t *C, int64_t k,
                const float *emb, int64_t n_emb, uint32_t emb_q0, int32_t topk,
                int32_t exact_below, int32_t pivots, int32_t out[3]) {
    int8_t *ecode = NULL;
    int eshift = 0;
    if (emb != NULL) {
        ecode = (int8_t *)malloc((size_t)(n_emb * EMB_DIM));
        eshift = orc_emb_quantize(emb, n_emb, ecode);
    }
    select_impl(codes, off, C, k, ecode, eshift, emb_q0, topk, exact_below,
                emb != NULL ? 0 : pivots, out);
    free(ecode);
}

/* Alg. 1 (Partition) with the choice of orc_select, then the split
 * L = {x : f(l, x) <= f(r, x)}, R = the rest, both in ascending order, and
 * breadth-first node numbering (L before R). */
static int32_t tree_impl(const uint8_t *codes, const int64_t *off, int32_t n, const float *emb,
                         uint32_t emb_q0, int32_t topk, int32_t exact_below, int32_t pivots,
                         int32_t *parent, int32_t *left, int32_t *right,
                         int32_t *center, int32_t *lpole, int32_t *rpole, int32_t *depth,
                         int64_t *mstart, int64_t *mcount, int32_t *perm) {
    if (n <= 0) return 0;
    /* members[v]: ascending member list of node v */
    int32_t **members = (int32_t **)calloc((size_t)(2 * n), sizeof(int32_t *));
    int64_t *msize = (int64_t *)calloc((size_t)(2 * n), sizeof(int64_t));
    members[0] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) members[0][i] = i;
    msize[0] = n;
    parent[0] = -1; depth[0] = 0;
    int32_t n_nodes = 1;
    int8_t *ecode = NULL;
    int eshift = 0;
    if (emb != NULL) {
        ecode = (int8_t *)malloc((size_t)n * EMB_DIM);
        eshift = orc_emb_quantize(emb, n, ecode);
    }
    for (int32_t v = 0; v < n_nodes; ++v) {
        int64_t k = msize[v];
        int32_t *C = members[v];
        left[v] = right[v] = -1;
        int32_t clr[3];
        select_impl(codes, off, C, k, ecode, eshift, emb_q0, topk, exact_below, pivots, clr);
        center[v] = clr[0];
        lpole[v] = clr[1];
        rpole[v] = clr[2];
        if (clr[1] < 0) continue;
        int64_t lp = 0, rp = 0;
        for (int64_t x = 0; x < k; ++x) {
            if (C[x] == clr[1]) lp = x;
            if (C[x] == clr[2]) rp = x;
        }
        int64_t *rowl = dist_row(codes, off, C, k, lp);
        int64_t *rowr = dist_row(codes, off, C, k, rp);
        int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int64_t nl = 0, nr = 0;
        for (int64_t x = 0; x < k; ++x) {
            if (rowl[x] <= rowr[x]) L[nl++] = C[x];
            else R[nr++] = C[x];
        }
        free(rowl);
        free(rowr);
        int32_t a = n_nodes++, b = n_nodes++;
        members[a] = L; msize[a] = nl;
        members[b] = R; msize[b] = nr;
        parent[a] = parent[b] = v;
        depth[a] = depth[b] = depth[v] + 1;
        left[v] = a; right[v] = b;
    }
    /* member ranges: a node's range is its children's ranges in order */
    mstart[0] = 0;
    for (int32_t v = 0; v < n_nodes; ++v) {
        mcount[v] = msize[v];
        if (left[v] >= 0) {
            mstart[left[v]] = mstart[v];
            mstart[right[v]] = mstart[v] + msize[left[v]];
        } else {
            for (int64_t x = 0; x < msize[v]; ++x) perm[mstart[v] + x] = members[v][x];
        }
    }
    for (int32_t v = 0; v < n_nodes; ++v) free(members[v]);
    free(members);
    free(msize);
    free(ecode);
    return n_nodes;
}

int32_t orc_tree(const uint8_t *codes, const int64_t *off, int32_t n,
                 int32_t *parent, int32_t *left, int32_t *right, int32_t *center,
                 int32_t *lpole, int32_t *rpole, int32_t *depth,
                 int64_t *mstart, int64_t *mcount, int32_t *perm) {
    return tree_impl(codes, off, n, NULL, 0, 0, 0, 0, parent, left, right, center, lpole, rpole,
                     depth, mstart, mcount, perm);
}

/* Alg. 1 with the sampled median: in clusters of more than exact_below and
 * more than topk members, the topk members with the least summed distance
 * to `pivots` hashed members are the candidates (select_impl). */
int32_t orc_tree_sampled(const uint8_t *codes, const int64_t *off, int32_t n, int32_t pivots,
                         int32_t topk, int32_t exact_below, int32_t *parent, int32_t *left,
                         int32_t *right, int32_t *center, int32_t *lpole, int32_t *rpole,
                         int32_t *depth, int64_t *mstart, int64_t *mcount, int32_t *perm) {
    if (pivots < 1 || topk < 1 || exact_below < 0) return -1;
    return tree_impl(codes, off, n, NULL, 0, topk, exact_below, pivots, parent, left, right,
                     center, lpole, rpole, depth, mstart, mcount, perm);
}

/* ------------------------------------------------------- online insertion
 * Sec. 5 names adding new sequences to an existing clustering, guide tree
 * and alignment as future work and gives no procedure.  This project's
 * reading, kept as close to Alg. 1 as an update can be:
 *   1. Routing.  A new sequence x starts at the root.  At an internal node
 *      with poles l and r it goes to the left child if f(l, x) <= f(r, x)
 *      and to the right child otherwise (the split rule of Alg. 1), down to
 *      a leaf.  Internal nodes keep their center and poles.
 *   2. Re-partition.  Every leaf that receives new sequences is replaced by
 *      Alg. 1 (full median, same tie rules) run on its old members and its
 *      new ones together; leaves that receive none stay as they are.
 *   3. Numbering.  The result is renumbered breadth-first from the root
 *      (a level's children after the level, in the order of their parents,
 *      L before R), so the node table reads like one built by Alg. 1:
 *      depth from the root, a node's member range its L child's range
 *      followed by its R child's.
 * The alignment of the updated set is the merge of Sec. 2.2 along the
 * updated tree (orc_merge).
 *
 * Sequences 0 .. n_old-1 are the ones the tree `in_*` (n_nodes_old nodes,
 * perm over n_old positions) was built on; n_old .. n-1 are new.  Output
 * arrays hold up to 2n - 1 nodes and n perm entries.  Returns the node
 * count, or -1 on bad input. */
typedef struct {
    int32_t left, right, center, lpole, rpole;
    int32_t *mem;       /* members of a leaf, in range order */
    int64_t nmem;
} ins_node;

static void ins_grow(ins_node **nodes, int64_t *cap, int64_t need) {
    if (need <= *cap) return;
    int64_t c = *cap ? *cap : 16;
    while (c < need) c *= 2;
    *nodes = (ins_node *)realloc(*nodes, sizeof(ins_node) * (size_t)c);
    *cap = c;
}

int32_t orc_tree_insert(const uint8_t *codes, const int64_t *off, int32_t n, int32_t n_old,
                        int32_t n_nodes_old, const int32_t *in_left, const int32_t *in_right,
                        const int32_t *in_center, const int32_t *in_lpole,
                        const int32_t *in_rpole, const int64_t *in_mstart,
                        const int64_t *in_mcount, const int32_t *in_perm,
                        int32_t *parent, int32_t *left, int32_t *right, int32_t *center,
                        int32_t *lpole, int32_t *rpole, int32_t *depth,
                        int64_t *mstart, int64_t *mcount, int32_t *perm) {
    if (n_old < 1 || n < n_old || n_nodes_old < 1 || n_nodes_old > 2 * n_old - 1) return -1;
    int64_t cap = 0, nn = n_nodes_old;
    ins_node *T = NULL;
    ins_grow(&T, &cap, nn);
    for (int32_t v = 0; v < n_nodes_old; ++v) {
        T[v].left = in_left[v];
        T[v].right = in_right[v];
        T[v].center = in_center[v];
        T[v].lpole = in_lpole[v];
        T[v].rpole = in_rpole[v];
        T[v].mem = NULL;
        T[v].nmem = 0;
        if (in_left[v] < 0) {
            T[v].nmem = in_mcount[v];
            T[v].mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in_mcount[v] + (n - n_old)));
            for (int64_t i = 0; i < in_mcount[v]; ++i) T[v].mem[i] = in_perm[in_mstart[v] + i];
        }
    }
    /* 1. routing: new members are appended to their leaf in index order */
    for (int32_t x = n_old; x < n; ++x) {
        int32_t v = 0;
        for (int64_t steps = 0; T[v].left >= 0; ++steps) {
            if (steps > n_nodes_old) return -1;
            const int64_t dl = dist_of(codes, off, T[v].lpole, x);
            const int64_t dr = dist_of(codes, off, T[v].rpole, x);
            v = dl <= dr ? T[v].left : T[v].right;
        }
        T[v].mem[T[v].nmem++] = x;
    }
    /* 2. re-partition every leaf that grew: Alg. 1 on its members (sorted,
     * so that the lowest-index tie rule is the same on the subset) */
    for (int32_t v = 0; v < n_nodes_old; ++v) {
        if (T[v].left >= 0 || T[v].nmem == in_mcount[v]) continue;
        const int64_t k = T[v].nmem;
        int32_t *C = T[v].mem;
        for (int64_t i = 1; i < k; ++i)          /* insertion sort, ascending */
            for (int64_t j = i; j > 0 && C[j - 1] > C[j]; --j) {
                int32_t t = C[j]; C[j] = C[j - 1]; C[j - 1] = t;
            }
        int64_t tot = 0;
        for (int64_t i = 0; i < k; ++i) tot += off[C[i] + 1] - off[C[i]];
        uint8_t *sc = (uint8_t *)malloc((size_t)tot + 1);
        int64_t *so = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
        so[0] = 0;
        for (int64_t i = 0; i < k; ++i) {
            const int64_t len = off[C[i] + 1] - off[C[i]];
            memcpy(sc + so[i], codes + off[C[i]], (size_t)len);
            so[i + 1] = so[i] + len;
        }
        const int64_t cs = 2 * k;
        int32_t *sp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(7 * cs));
        int64_t *sm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * cs));
        int32_t *sperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int32_t *s_par = sp, *s_l = sp + cs, *s_r = sp + 2 * cs, *s_c = sp + 3 * cs;
        int32_t *s_lp = sp + 4 * cs, *s_rp = sp + 5 * cs, *s_d = sp + 6 * cs;
        int64_t *s_ms = sm, *s_mc = sm + cs;
        const int32_t sn = tree_impl(sc, so, (int32_t)k, NULL, 0, 0, 0, 0, s_par, s_l, s_r, s_c,
                                     s_lp, s_rp, s_d, s_ms, s_mc, sperm);
        /* subtree node u > 0 becomes node base + u - 1; its root is v */
        const int64_t base = nn;
        ins_grow(&T, &cap, nn + sn - 1);
        nn += sn - 1;
        for (int32_t u = 0; u < sn; ++u) {
            const int64_t w = u == 0 ? v : base + u - 1;
            T[w].left = s_l[u] < 0 ? -1 : (int32_t)(base + s_l[u] - 1);
            T[w].right = s_r[u] < 0 ? -1 : (int32_t)(base + s_r[u] - 1);
            T[w].center = C[s_c[u]];
            T[w].lpole = s_lp[u] < 0 ? -1 : C[s_lp[u]];
            T[w].rpole = s_rp[u] < 0 ? -1 : C[s_rp[u]];
            if (u > 0) { T[w].mem = NULL; T[w].nmem = 0; }
            if (s_l[u] < 0) {
                int32_t *mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)s_mc[u]);
                for (int64_t i = 0; i < s_mc[u]; ++i) mem[i] = C[sperm[s_ms[u] + i]];
                if (u == 0) free(T[w].mem);
                T[w].mem = mem;
                T[w].nmem = s_mc[u];
            }
        }
        if (sn > 1) { free(C); T[v].mem = NULL; T[v].nmem = 0; }
        free(sc); free(so); free(sp); free(sm); free(sperm);
    }
    /* 3. breadth-first renumbering, then member ranges and perm */
    int32_t *bfs = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
    int64_t head = 0, tail = 0;
    bfs[tail++] = 0;
    id[0] = 0;
    parent[0] = -1;
    depth[0] = 0;
    while (head < tail) {
        const int32_t j = (int32_t)head;
        const int32_t w = bfs[head++];
        center[j] = T[w].center;
        lpole[j] = T[w].lpole;
        rpole[j] = T[w].rpole;
        left[j] = right[j] = -1;
        if (T[w].left >= 0) {
            const int32_t a = (int32_t)tail, b = (int32_t)tail + 1;
            bfs[tail++] = T[w].left;
            bfs[tail++] = T[w].right;
            id[T[w].left] = a;
            id[T[w].right] = b;
            left[j] = a;
            right[j] = b;
            parent[a] = parent[b] = j;
            depth[a] = depth[b] = depth[j] + 1;
        }
    }
    const int32_t total = (int32_t)tail;
    for (int32_t j = total - 1; j >= 0; --j)
        mcount[j] = left[j] < 0 ? T[bfs[j]].nmem : mcount[left[j]] + mcount[right[j]];
    mstart[0] = 0;
    for (int32_t j = 0; j < total; ++j) {
        if (left[j] >= 0) {
            mstart[left[j]] = mstart[j];
            mstart[right[j]] = mstart[j] + mcount[left[j]];
        } else {
            const ins_node *t = &T[bfs[j]];
            for (int64_t i = 0; i < t->nmem; ++i) perm[mstart[j] + i] = t->mem[i];
        }
    }
    for (int64_t w = 0; w < nn; ++w) free(T[w].mem);
    free(T);
    free(bfs);
    free(id);
    return total;
}

/* The same with the surrogate-pruned median (emb: float[n][128]). */
int32_t orc_tree_pruned(const uint8_t *codes, const int64_t *off, int32_t n, const float *emb,
                        uint32_t emb_q0, int32_t topk, int32_t exact_below, int32_t *parent, int32_t *left, int32_t *right,
                        int32_t *center, int32_t *lpole, int32_t *rpole, int32_t *depth,
                        int64_t *mstart, int64_t *mcount, int32_t *perm) {
    if (emb == NULL || topk < 1 || exact_below < 0) return -1;
    return tree_impl(codes, off, n, emb, emb_q0, topk, exact_below, 0, parent, left, right, center, lpole,
                     rpole, depth,
                     mstart, mcount, perm);
}

/* Surrogate row sums E(x) of emb_estimate over an explicit member list
 * (for tests of the ranking step); emb: float[n_emb][128], the whole set. */
void orc_emb_rowsums(const int64_t *off, const float *emb, int64_t n_emb, uint32_t emb_q0,
                     const int32_t *members, int64_t k, uint64_t *E) {
    int8_t *ecode = (int8_t *)malloc((size_t)(n_emb * EMB_DIM));
    const int eshift = orc_emb_quantize(emb, n_emb, ecode);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t x = 0; x < k; ++x) {
        uint64_t s = 0;
        for (int64_t y = 0; y < k; ++y)
            s += emb_estimate(off, ecode, eshift, emb_q0, members[x], members[y]);
        E[x] = s;
    }
    free(ecode);
}

/* ------------------------------------------------------------------ merge
 * Bottom-up merge of Sec. 2.2 over the tree from orc_tree.  A leaf's
 * alignment is its sequence(s) (one row each, no gaps).  For an internal
 * node with children L and R: take the aligned row of center(L) in L's
 * alignment and the aligned row of center(R) in R's, align the two rows with
 * the unit-cost NW above treating the gap symbol `sigma` as an ordinary
 * symbol, then widen L's alignment with an all-gap column at every I op and
 * R's alignment with an all-gap column at every D op, and stack L's rows over
 * R's.  Rows of a node follow its `perm` range.  The final alignment is
 * written with row i = input sequence i; returns its width (-1 on error). */
int64_t orc_merge(const uint8_t *codes, const int64_t *off, int32_t n, int32_t sigma,
                  int32_t n_nodes, const int32_t *left, const int32_t *right,
                  const int32_t *center, const int64_t *mstart, const int64_t *mcount,
                  const int32_t *perm, uint8_t *msa_out, int64_t msa_cap) {
    uint8_t **aln = (uint8_t **)calloc((size_t)n_nodes, sizeof(uint8_t *));
    int64_t *width = (int64_t *)calloc((size_t)n_nodes, sizeof(int64_t));
    const uint8_t gap = (uint8_t)sigma;
    for (int32_t v = n_nodes - 1; v >= 0; --v) {
        int64_t rows = mcount[v];
        if (left[v] < 0) {
            int64_t W = 0;
            for (int64_t r = 0; r < rows; ++r) {
                int32_t s = perm[mstart[v] + r];
                if (off[s + 1] - off[s] > W) W = off[s + 1] - off[s];
            }
            aln[v] = (uint8_t *)malloc((size_t)(rows * W + 1));
            for (int64_t r = 0; r < rows; ++r) {
                int32_t s = perm[mstart[v] + r];
                int64_t len = off[s + 1] - off[s];
                memcpy(aln[v] + r * W, codes + off[s], (size_t)len);
                memset(aln[v] + r * W + len, gap, (size_t)(W - len));
            }
            width[v] = W;
            continue;
        }
        int32_t L = left[v], R = right[v];
        int64_t WL = width[L], WR = width[R];
        int64_t rl = -1, rr = -1;
        for (int64_t r = 0; r < mcount[L]; ++r) if (perm[mstart[L] + r] == center[L]) rl = r;
        for (int64_t r = 0; r < mcount[R]; ++r) if (perm[mstart[R] + r] == center[R]) rr = r;
        if (rl < 0 || rr < 0) return -1;
        uint8_t *ops = (uint8_t *)malloc((size_t)(WL + WR + 1));
        int64_t nops = 0;
        orc_nw(aln[L] + rl * WL, WL, aln[R] + rr * WR, WR, ops, &nops);
        uint8_t *out = (uint8_t *)malloc((size_t)(rows * nops + 1));
        for (int64_t r = 0; r < mcount[L]; ++r) {
            int64_t src = 0;
            for (int64_t c = 0; c < nops; ++c)
                out[r * nops + c] = (ops[c] == 2) ? gap : aln[L][r * WL + src++];
        }
        for (int64_t r = 0; r < mcount[R]; ++r) {
            int64_t src = 0;
            for (int64_t c = 0; c < nops; ++c)
                out[(mcount[L] + r) * nops + c] = (ops[c] == 1) ? gap : aln[R][r * WR + src++];
        }
        free(ops);
        free(aln[L]); aln[L] = NULL;
        free(aln[R]); aln[R] = NULL;
        aln[v] = out;
        width[v] = nops;
    }
    int64_t W = width[0];
    if ((int64_t)n * W > msa_cap) W = -1;
    else
        for (int64_t r = 0; r < n; ++r)
            memcpy(msa_out + (int64_t)perm[r] * W, aln[0] + r * W, (size_t)W);
    free(aln[0]);
    free(aln);
    free(width);
    return W;
}

/*
 * Alignment-quality counts (Sec. 2.3).  msa: rows x width row-major symbol
 * codes, `gap` the gap code.  Per row: the number of gap symbols.  Per pair
 * (ia[p], ib[p]): hamming = columns whose two symbols differ (a column of two
 * gaps counts as equal); aligned = columns where neither symbol is a gap
 * (the columns the p-score looks at); mismatched = aligned columns whose
 * symbols differ.  A plain column loop per row and per pair.
 */
void orc_msa_row_gaps(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap,
                      int32_t *gaps) {
    for (int32_t i = 0; i < rows; ++i) {
        int32_t g = 0;
        for (int32_t c = 0; c < width; ++c) g += msa[(int64_t)i * width + c] == gap;
        gaps[i] = g;
    }
}

void orc_msa_pair_counts(const uint8_t *msa, int32_t rows, int32_t width, int32_t gap,
                         const int32_t *ia, const int32_t *ib, int64_t n_pairs,
                         int32_t *hamming, int32_t *aligned, int32_t *mismatched) {
    (void)rows;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const uint8_t *x = msa + (int64_t)ia[p] * width;
        const uint8_t *y = msa + (int64_t)ib[p] * width;
        int32_t h = 0, al = 0, mm = 0;
        for (int32_t c = 0; c < width; ++c) {
            const int differ = x[c] != y[c];
            const int both = x[c] != gap && y[c] != gap;
            h += differ;
            al += both;
            mm += both && differ;
        }
        hamming[p] = h;
        aligned[p] = al;
        mismatched[p] = mm;
    }
}
