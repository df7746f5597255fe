"""ctypes face of the C oracle (test infrastructure only).

Inputs are numpy arrays in the CSR form produced by the input generators:
uint8 codes plus int64 offsets.  Nothing here imports the device library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or \
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        L.orc_lev.restype = C.c_int64
        L.orc_lev.argtypes = [P, C.c_int64, P, C.c_int64]
        L.orc_lev_pairs.restype = None
        L.orc_lev_pairs.argtypes = [P, P, P, P, P, P, C.c_int64, P]
        L.orc_nw.restype = C.c_int64
        L.orc_nw.argtypes = [P, C.c_int64, P, C.c_int64, P, P]
        L.orc_nw_pairs.restype = None
        L.orc_nw_pairs.argtypes = [P, P, P, P, P, P, C.c_int64, P, P, P, P]
        L.orc_gotoh.restype = C.c_int64
        L.orc_gotoh.argtypes = [P, C.c_int64, P, C.c_int64, P, C.c_int32, C.c_int32,
                                C.c_int32, P, P]
        L.orc_gotoh_pairs.restype = None
        L.orc_gotoh_pairs.argtypes = [P, P, P, P, P, P, C.c_int64, P, C.c_int32, C.c_int32,
                                      C.c_int32, P, P, P, P]
        L.orc_tree.restype = C.c_int32
        L.orc_tree.argtypes = [P, P, C.c_int32] + [P] * 10
        L.orc_tree_insert.restype = C.c_int32
        L.orc_tree_insert.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32] + [P] * 18
        L.orc_tree_pruned.restype = C.c_int32
        L.orc_tree_pruned.argtypes = [P, P, C.c_int32, P, C.c_uint32, C.c_int32, C.c_int32] + [P] * 10
        L.orc_select.restype = None
        L.orc_select.argtypes = [P, P, P, C.c_int64, P, C.c_int64, C.c_uint32, C.c_int32,
                                 C.c_int32, C.c_int32, P]
        L.orc_tree_sampled.restype = C.c_int32
        L.orc_tree_sampled.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32] + [P] * 10
        L.orc_emb_rowsums.restype = None
        L.orc_emb_rowsums.argtypes = [P, P, C.c_int64, C.c_uint32, P, C.c_int64, P]
        L.orc_emb_quantize.restype = C.c_int32
        L.orc_emb_quantize.argtypes = [P, C.c_int64, P]
        L.orc_merge.restype = C.c_int64
        L.orc_merge.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                C.c_int64]
        L.orc_msa_row_gaps.restype = None
        L.orc_msa_row_gaps.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_msa_pair_counts.restype = None
        L.orc_msa_pair_counts.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int64,
                                          P, P, P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _u8(x):
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    if isinstance(x, str):
        return np.frombuffer(x.encode(), dtype=np.uint8).copy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint8))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def lev(a, b) -> int:
    a, b = _u8(a), _u8(b)
    return int(lib().orc_lev(_p(a), len(a), _p(b), len(b)))


def lev_pairs(ca, oa, cb, ob, ia, ib) -> np.ndarray:
    ca, cb = _u8(ca), _u8(cb)
    oa = np.ascontiguousarray(oa, dtype=np.int64)
    ob = np.ascontiguousarray(ob, dtype=np.int64)
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    out = np.zeros(len(ia), dtype=np.int64)
    lib().orc_lev_pairs(_p(ca), _p(oa), _p(cb), _p(ob), _p(ia), _p(ib), len(ia), _p(out))
    return out


def nw(a, b):
    """(score, ops) for one pair; ops uint8 with 0=M, 1=D, 2=I."""
    a, b = _u8(a), _u8(b)
    ops = np.zeros(len(a) + len(b) + 1, dtype=np.uint8)
    n = np.zeros(1, dtype=np.int64)
    s = lib().orc_nw(_p(a), len(a), _p(b), len(b), _p(ops), _p(n))
    return int(s), ops[: int(n[0])].copy()


def nw_pairs(ca, oa, cb, ob, ia, ib, with_ops=True):
    """Scores (int64[P]) and, if asked, a list of op arrays."""
    ca, cb = _u8(ca), _u8(cb)
    oa = np.ascontiguousarray(oa, dtype=np.int64)
    ob = np.ascontiguousarray(ob, dtype=np.int64)
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    P = len(ia)
    score = np.zeros(P, dtype=np.int64)
    if not with_ops:
        lib().orc_nw_pairs(_p(ca), _p(oa), _p(cb), _p(ob), _p(ia), _p(ib), P, _p(score),
                           None, None, None)
        return score, None
    cap = (oa[ia + 1] - oa[ia]) + (ob[ib + 1] - ob[ib])
    ops_off = np.zeros(P + 1, dtype=np.int64)
    np.cumsum(cap, out=ops_off[1:])
    ops = np.zeros(max(int(ops_off[-1]), 1), dtype=np.uint8)
    ops_len = np.zeros(P, dtype=np.int64)
    lib().orc_nw_pairs(_p(ca), _p(oa), _p(cb), _p(ob), _p(ia), _p(ib), P, _p(score),
                       _p(ops), _p(ops_off), _p(ops_len))
    return score, [ops[ops_off[p]: ops_off[p] + ops_len[p]].copy() for p in range(P)]


def gotoh(a, b, sub, open_, ext):
    """(score, ops) of the affine-gap alignment of one pair (see orc_gotoh):
    sub is the sigma x sigma score matrix, a gap run of k scores -(open + k ext)."""
    a, b = _u8(a), _u8(b)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    sigma = sub.shape[0]
    ops = np.zeros(len(a) + len(b) + 1, dtype=np.uint8)
    n = np.zeros(1, dtype=np.int64)
    s = lib().orc_gotoh(_p(a), len(a), _p(b), len(b), _p(sub), sigma, int(open_), int(ext),
                        _p(ops), _p(n))
    return int(s), ops[: int(n[0])].copy()


def gotoh_pairs(ca, oa, cb, ob, ia, ib, sub, open_, ext, with_ops=True):
    """Scores (int64[P]) and, if asked, the op arrays of affine-gap alignments."""
    ca, cb = _u8(ca), _u8(cb)
    oa = np.ascontiguousarray(oa, dtype=np.int64)
    ob = np.ascontiguousarray(ob, dtype=np.int64)
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    sigma = sub.shape[0]
    P = len(ia)
    score = np.zeros(P, dtype=np.int64)
    if not with_ops:
        lib().orc_gotoh_pairs(_p(ca), _p(oa), _p(cb), _p(ob), _p(ia), _p(ib), P, _p(sub), sigma,
                              int(open_), int(ext), _p(score), None, None, None)
        return score, None
    cap = (oa[ia + 1] - oa[ia]) + (ob[ib + 1] - ob[ib])
    ops_off = np.zeros(P + 1, dtype=np.int64)
    np.cumsum(cap, out=ops_off[1:])
    ops = np.zeros(max(int(ops_off[-1]), 1), dtype=np.uint8)
    ops_len = np.zeros(P, dtype=np.int64)
    lib().orc_gotoh_pairs(_p(ca), _p(oa), _p(cb), _p(ob), _p(ia), _p(ib), P, _p(sub), sigma,
                          int(open_), int(ext), _p(score), _p(ops), _p(ops_off), _p(ops_len))
    return score, [ops[ops_off[p]: ops_off[p] + ops_len[p]].copy() for p in range(P)]


TREE_FIELDS = ("parent", "left", "right", "center", "lpole", "rpole", "depth",
               "mstart", "mcount")


def tree(codes, offsets):
    """Alg. 1 with the full geometric median; dict of per-node arrays + perm."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    cap = max(2 * n - 1, 1)
    arr = {f: np.zeros(cap, dtype=np.int64 if f in ("mstart", "mcount") else np.int32)
           for f in TREE_FIELDS}
    perm = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_tree(_p(codes), _p(offsets), n, *[_p(arr[f]) for f in TREE_FIELDS],
                       _p(perm))
    out = {f: arr[f][:k].copy() for f in TREE_FIELDS}
    out["perm"] = perm[:n].copy()
    out["n_nodes"] = int(k)
    return out




def tree_sampled(codes, offsets, pivots=8, topk=16, exact_below=0):
    """Alg. 1 with the sampled median (orc_tree_sampled)."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    cap = max(2 * n - 1, 1)
    arr = {f: np.zeros(cap, dtype=np.int64 if f in ("mstart", "mcount") else np.int32)
           for f in TREE_FIELDS}
    perm = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_tree_sampled(_p(codes), _p(offsets), n, int(pivots), int(topk),
                               int(exact_below), *[_p(arr[f]) for f in TREE_FIELDS], _p(perm))
    if k < 0:
        raise ValueError("oracle tree_sampled: bad arguments")
    out = {f: arr[f][:k].copy() for f in TREE_FIELDS}
    out["perm"] = perm[:n].copy()
    out["n_nodes"] = int(k)
    return out

def tree_insert(codes, offsets, n_old, t):
    """Online insertion (orc_tree_insert): sequences n_old.. of the set are
    routed into the tree ``t`` built on the first n_old, the leaves they
    reach are re-partitioned by Alg. 1, and the tree is renumbered
    breadth-first.  Returns a tree dict over the whole set."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    k0 = int(t["n_nodes"])
    src = {f: np.ascontiguousarray(t[f][:k0], dtype=np.int64 if f in ("mstart", "mcount")
                                   else np.int32) for f in TREE_FIELDS}
    src_perm = np.ascontiguousarray(t["perm"][:n_old], dtype=np.int32)
    cap = max(2 * n - 1, 1)
    arr = {f: np.zeros(cap, dtype=np.int64 if f in ("mstart", "mcount") else np.int32)
           for f in TREE_FIELDS}
    perm = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_tree_insert(_p(codes), _p(offsets), n, int(n_old), k0,
                              *[_p(src[f]) for f in ("left", "right", "center", "lpole",
                                                     "rpole", "mstart", "mcount")],
                              _p(src_perm), *[_p(arr[f]) for f in TREE_FIELDS], _p(perm))
    if k < 0:
        raise ValueError("oracle tree_insert: bad input")
    out = {f: arr[f][:k].copy() for f in TREE_FIELDS}
    out["perm"] = perm[:n].copy()
    out["n_nodes"] = int(k)
    return out

def tree_pruned(codes, offsets, emb, topk=16, exact_below=0, emb_q0=0):
    """Alg. 1 with the surrogate-pruned median (emb: float32 [n, 128]);
    clusters of at most exact_below members keep the full median; emb_q0 is
    the calibration offset added to every embedding distance (units 2^-16)."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    emb = np.ascontiguousarray(emb, dtype=np.float32)
    assert emb.shape == (n, 128)
    cap = max(2 * n - 1, 1)
    arr = {f: np.zeros(cap, dtype=np.int64 if f in ("mstart", "mcount") else np.int32)
           for f in TREE_FIELDS}
    perm = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_tree_pruned(_p(codes), _p(offsets), n, _p(emb), int(emb_q0), int(topk),
                              int(exact_below),
                              *[_p(arr[f]) for f in TREE_FIELDS], _p(perm))
    if k < 0:
        raise ValueError("bad arguments")
    out = {f: arr[f][:k].copy() for f in TREE_FIELDS}
    out["perm"] = perm[:n].copy()
    out["n_nodes"] = int(k)
    return out


def select(codes, offsets, members, emb=None, topk=16, exact_below=0, emb_q0=0, pivots=0):
    """(c, l, r) that Alg. 1 picks for the cluster `members` (input indices);
    emb=None and pivots=0: full geometric median; emb: the surrogate-pruned
    one; pivots > 0: the sampled one (candidates ranked by their summed
    distance to `pivots` hashed members)."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    mem = np.ascontiguousarray(np.sort(np.asarray(members)), dtype=np.int32)
    e = None if emb is None else np.ascontiguousarray(emb, dtype=np.float32)
    out = np.zeros(3, dtype=np.int32)
    lib().orc_select(_p(codes), _p(offsets), _p(mem), len(mem), None if e is None else _p(e),
                     0 if e is None else len(e), int(emb_q0), int(topk), int(exact_below),
                     int(pivots), _p(out))
    return tuple(int(x) for x in out)


def emb_rowsums(offsets, emb, members, emb_q0=0):
    """Surrogate row sums E(x) over the member list: the summed embedding
    distance (plus emb_q0) times the pair's summed length, units of 2^-16.
    emb holds the whole set (its quantization scale comes from every row)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    emb = np.ascontiguousarray(emb, dtype=np.float32)
    members = np.ascontiguousarray(members, dtype=np.int32)
    E = np.zeros(len(members), dtype=np.uint64)
    lib().orc_emb_rowsums(_p(offsets), _p(emb), len(emb), int(emb_q0), _p(members),
                          len(members), _p(E))
    return E


def emb_quantize(emb):
    """(int8 codes [n, 128], shift s): the quantization of the surrogate
    distance, code = rint(e 2^s) limited to +-127."""
    emb = np.ascontiguousarray(emb, dtype=np.float32)
    codes = np.zeros(emb.shape, dtype=np.int8)
    s = lib().orc_emb_quantize(_p(emb), len(emb), _p(codes))
    return codes, int(s)


def merge(codes, offsets, sigma, t):
    """Final alignment (n x W uint8, gap = sigma) for the tree ``t``."""
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    cap = n * int(offsets[-1] + 1)
    msa = np.zeros(max(cap, 1), dtype=np.uint8)
    W = lib().orc_merge(_p(codes), _p(offsets), n, sigma, t["n_nodes"],
                        _p(t["left"]), _p(t["right"]), _p(t["center"]),
                        _p(t["mstart"]), _p(t["mcount"]), _p(t["perm"]), _p(msa), cap)
    if W < 0:
        raise RuntimeError("oracle merge failed")
    return msa[: n * W].reshape(n, W).copy()


# ------------------------------------------------------- alignment quality
# Sec. 2.3 defines three metrics on a finished alignment; Table 2 adds width
# and stretch.  Readings where the text is short of a formula: the
# percentage of gaps is the mean over rows of gaps / width, times 100; the
# p-score of a pair is mismatched / aligned over the columns where both rows
# hold a residue (pairs with no such column are left out) and the table
# reports its minimum, mean and maximum over pairs; the distortion of a pair
# is its Hamming distance (two gaps count as equal) over the Levenshtein
# distance of the unaligned sequences (pairs at distance 0 are left out),
# averaged over pairs; stretch = width / longest sequence.
QUALITY_FIELDS = ("pct_gaps", "p_min", "p_avg", "p_max", "distortion", "stretch",
                  "n_p_pairs", "n_d_pairs")


def msa_row_gaps(msa, gap):
    msa = np.ascontiguousarray(msa, dtype=np.uint8)
    rows, width = msa.shape
    out = np.zeros(rows, dtype=np.int32)
    lib().orc_msa_row_gaps(_p(msa), rows, width, int(gap), _p(out))
    return out


def msa_pair_counts(msa, gap, ia, ib):
    """(hamming, aligned, mismatched) int32 arrays for the pairs (ia[p], ib[p])."""
    msa = np.ascontiguousarray(msa, dtype=np.uint8)
    rows, width = msa.shape
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    n = len(ia)
    h = np.zeros(n, dtype=np.int32)
    a = np.zeros(n, dtype=np.int32)
    m = np.zeros(n, dtype=np.int32)
    lib().orc_msa_pair_counts(_p(msa), rows, width, int(gap), _p(ia), _p(ib), n, _p(h), _p(a),
                              _p(m))
    return h, a, m


def msa_quality(msa, gap, max_len, ia, ib, lev):
    """The metrics of QUALITY_FIELDS over the pairs (ia, ib); lev[p] is the
    Levenshtein distance of the two unaligned sequences of pair p."""
    msa = np.ascontiguousarray(msa, dtype=np.uint8)
    rows, width = msa.shape
    gaps = msa_row_gaps(msa, gap)
    h, a, m = msa_pair_counts(msa, gap, ia, ib)
    lev = np.asarray(lev, dtype=np.int64)
    pct = 100.0 * sum(float(g) / width for g in gaps) / rows if rows and width else 0.0
    ps = [float(mm) / float(al) for mm, al in zip(m.tolist(), a.tolist()) if al > 0]
    ds = [float(hh) / float(d) for hh, d in zip(h.tolist(), lev.tolist()) if d > 0]
    return {"pct_gaps": pct,
            "p_min": min(ps) if ps else 0.0,
            "p_avg": sum(ps) / len(ps) if ps else 0.0,
            "p_max": max(ps) if ps else 0.0,
            "distortion": sum(ds) / len(ds) if ds else 0.0,
            "stretch": float(width) / max_len if max_len > 0 else 0.0,
            "n_p_pairs": len(ps), "n_d_pairs": len(ds)}
