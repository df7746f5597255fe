"""Pins of the CPU oracle's surrogate-pruned Alg. 1 (no GPU).

The pruned median replaces the full geometric median of a cluster by the
best of `topk` candidates that an embedding ranks first; everything else
(poles, split, numbering) is Alg. 1 as in the exact oracle."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

from test_oracle_tree import check_partition

TWO16 = float(1 << 16)


def _emb(seed, n, scale=0.1):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, 128)) * scale).astype(np.float32)


def _off(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)


def test_emb_distance_closed_form():
    e = np.zeros((2, 128), dtype=np.float32)
    e[1, 0], e[1, 1] = 3.0, 4.0                    # |(3, 4)| = 5; 2^4 (3, 4) are integers
    off = _off([7, 10])                            # |x| + |y| = 17
    E = orc.emb_rowsums(off, e, np.array([0, 1], dtype=np.int32))
    assert E.tolist() == [5 * 17 * (1 << 16)] * 2
    # a single member: the sum holds only d(x, x) = 0
    assert orc.emb_rowsums(off, e, np.array([1], dtype=np.int32)).tolist() == [0]
    # distances saturate at 2^15
    e[1, 0] = 1e6
    E = orc.emb_rowsums(off, e, np.array([0, 1], dtype=np.int32))
    assert E.tolist() == [17 * (1 << 31)] * 2


def _shift_by_definition(M):
    """s with M 2^s in [64, 128), limited to [-20, 40] (40 below 2^-34)."""
    import math
    if M < 2.0 ** -34:
        return 40
    mant, ex = math.frexp(float(M))              # M = mant 2^ex, mant in [0.5, 1)
    return int(min(max(6 - (ex - 1), -20), 40))


@pytest.mark.parametrize("scale", [0.0, 1e-12, 1e-3, 0.1, 1.0, 37.0, 3e5, 1e9])
def test_emb_quantization_rule(scale):
    """Codes are e 2^s rounded to the nearest integer (ties to even), limited
    to +-127, with one power-of-two scale for the set: the largest |e| lands
    in [64, 128) unless the shift hits its limits."""
    e = _emb(20, 40, scale=max(scale, 1e-30)) if scale else np.zeros((40, 128), np.float32)
    codes, s = orc.emb_quantize(e)
    M = float(np.abs(e).max())
    assert s == _shift_by_definition(M)
    want = np.clip(np.rint(e.astype(np.float64) * 2.0 ** s), -127, 127)   # exact in float64
    assert np.array_equal(codes.astype(np.int64), want.astype(np.int64))
    if 2.0 ** -34 <= M < 2.0 ** 27:
        assert 64 <= M * 2.0 ** s < 128
        assert np.abs(codes).max() >= 64
        err = np.abs(e.astype(np.float64) - codes * 2.0 ** -s)
        assert err.max() <= 2.0 ** -s               # half a step, a full one where clipped


def test_emb_distance_within_quantization_bound():
    """|E / (2^16 (|x| + |y|)) - ||e_x - e_y||| stays within the quantization
    error (every coordinate moves by at most one step 2^-s, so the distance by
    at most sqrt(128) 2^-s) plus the float32 square root and rounding."""
    e = _emb(7, 64, scale=1.0)
    s = _shift_by_definition(np.abs(e).max())
    off = _off(np.arange(64) + 1)
    for i in range(1, 64):
        E = orc.emb_rowsums(off, e, np.array([0, i], dtype=np.int32))
        x, y = e[0].astype(np.float64), e[i].astype(np.float64)
        d = np.linalg.norm(x - y)
        L = 1 + (i + 1)
        bound = np.sqrt(128) * 2.0 ** -s + (d + 1) * 2.0 ** -22
        assert abs(float(E[0]) / (TWO16 * L) - d) <= bound + 0.5 / TWO16


def test_emb_distance_stated_steps():
    """The oracle takes the stated steps: integer codes, the exact squared
    distance D of the codes (Python integers here), then in float32 sqrt(D),
    times 2^-s, the cap at 2^15, times 2^16 and the rounding."""
    e = _emb(8, 6, scale=0.7)
    off = _off(np.ones(6, dtype=np.int64))
    s = _shift_by_definition(np.abs(e).max())
    c = np.clip(np.rint(e.astype(np.float64) * 2.0 ** s), -127, 127).astype(np.int64)
    f = np.float32
    for i in range(1, 6):
        D = int(sum((int(c[0, k]) - int(c[i, k])) ** 2 for k in range(128)))
        dist = f(np.sqrt(f(D))) * f(2.0 ** -s)
        want = 2 * int(np.rint(f(min(dist, f(32768.0))) * f(TWO16)))
        got = orc.emb_rowsums(off, e, np.array([0, i], dtype=np.int32))
        assert int(got[0]) == want


def test_emb_distance_is_a_metric_on_codes():
    """Quantized distances are symmetric, zero on equal codes and obey the
    triangle inequality up to the rounding of three values."""
    e = _emb(21, 10, scale=0.3)
    e[7] = e[3]
    off = _off(np.ones(10, dtype=np.int64))
    q = np.zeros((10, 10))
    for x in range(10):
        for y in range(10):
            q[x, y] = int(orc.emb_rowsums(off, e, np.array([x, y], dtype=np.int32))[0]) / 2
    assert np.array_equal(q, q.T) and q[3, 7] == 0 and np.all(np.diag(q) == 0)
    for x in range(10):
        for y in range(10):
            for z in range(10):
                assert q[x, z] <= q[x, y] + q[y, z] + 2


def test_row_sums_are_sums_of_pairs():
    e = _emb(9, 12)
    off = _off(np.arange(12) * 3 + 2)
    mem = np.array([3, 0, 7, 11, 5], dtype=np.int32)
    E = orc.emb_rowsums(off, e, mem)
    for x in range(len(mem)):
        s = sum(int(orc.emb_rowsums(off, e, mem[[x, y]])[0]) for y in range(len(mem)) if y != x)
        assert int(E[x]) == s


def test_topk_covering_cluster_is_exact_median():
    """With every member a candidate the pruned median is the full one."""
    d = synth.tiny()
    t0 = orc.tree(d["codes"], d["offsets"])
    t1 = orc.tree_pruned(d["codes"], d["offsets"], _emb(10, 64), topk=64)
    for f in orc.TREE_FIELDS + ("perm",):
        assert (t0[f] == t1[f]).all(), f


def _members(t, v):
    return np.sort(t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]])


def test_center_follows_the_ranking():
    """topk = 1: the root center is the member the embedding puts in the
    middle (origin among points on a sphere), not the exact medoid."""
    codes, off = synth.random_set(33, 30, 20, 60, 4)
    e = _emb(11, 30, scale=1.0)
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    e[17] = 0.0
    t = orc.tree_pruned(codes, off, e, topk=1)
    assert t["center"][0] == 17
    exact = orc.tree(codes, off)
    assert exact["center"][0] != 17                 # the pin would be vacuous otherwise


def test_equal_estimates_take_lowest_indices():
    """All estimates equal: the candidates are the topk lowest indices and
    c is the one of them with the least exact row sum (lowest on ties)."""
    codes, off = synth.random_set(34, 25, 10, 40, 4)
    seqs = synth.from_csr(codes, off)
    t = orc.tree_pruned(codes, off, np.zeros((25, 128), np.float32), topk=3)
    sums = [sum(orc.lev(seqs[x], seqs[y]) for y in range(25)) for x in range(3)]
    assert t["center"][0] == int(np.argmin(sums))


def check_pruned(seqs, emb, topk, t):
    """Alg. 1 with the median taken over the embedding's candidates: c is
    among the members the float64 estimate ranks near the top, beats every
    member it ranks clearly inside the top topk, and the rest is exact."""
    n = len(seqs)
    assert t["n_nodes"] == 2 * n - 1
    assert sorted(t["perm"].tolist()) == list(range(n))
    for v in range(t["n_nodes"]):
        C = _members(t, v)
        if t["left"][v] < 0:
            assert len(C) == 1 and t["center"][v] == C[0]
            continue
        D = np.array([[orc.lev(seqs[x], seqs[y]) for y in C] for x in C])
        lens = np.array([len(seqs[x]) for x in C], dtype=np.float64)
        E = (np.linalg.norm(emb[C][:, None, :].astype(np.float64) -
                            emb[C][None, :, :].astype(np.float64), axis=2) *
             (lens[:, None] + lens[None, :])).sum(1)
        rank = np.argsort(E, kind="stable")
        c = int(np.where(C == t["center"][v])[0][0])
        pos = int(np.where(rank == c)[0][0])
        assert pos < topk + 2
        sure = rank[: max(topk - 2, 0)]
        assert all(D[c].sum() <= D[s].sum() for s in sure)
        l = int(np.argmax(D[c]))
        r = int(np.argmax(D[l]))
        assert t["lpole"][v] == C[l] and t["rpole"][v] == C[r]
        a, b = t["left"][v], t["right"][v]
        assert _members(t, a).tolist() == C[D[l] <= D[r]].tolist()
        assert _members(t, b).tolist() == C[D[r] < D[l]].tolist()


@pytest.mark.parametrize("topk", [1, 4, 16])
def test_pruned_partition_random_dna(topk):
    codes, off = synth.random_set(35, 48, 20, 70, 4)
    seqs = synth.from_csr(codes, off)
    emb = _emb(12, 48)
    check_pruned(seqs, emb, topk, orc.tree_pruned(codes, off, emb, topk=topk))


def test_pruned_exact_checker_agrees_on_full_topk():
    """The exact partition checker accepts a pruned tree whose candidates
    cover every cluster."""
    codes, off = synth.random_set(36, 20, 5, 30, 20)
    seqs = synth.from_csr(codes, off)
    check_partition(seqs, orc.tree_pruned(codes, off, _emb(13, 20), topk=20))


def test_select_reproduces_tree_choices():
    """orc_select on a node's member set gives the node's (c, l, r) in the
    tree built from it, exact and pruned."""
    codes, off = synth.random_set(37, 40, 10, 50, 4)
    emb = _emb(14, 40)
    for e, t in ((None, orc.tree(codes, off)), (emb, orc.tree_pruned(codes, off, emb, 4))):
        for v in range(t["n_nodes"]):
            C = _members(t, v)
            want = (int(t["center"][v]), int(t["lpole"][v]), int(t["rpole"][v]))
            assert orc.select(codes, off, C, e, 4) == want


def test_select_brute_force_median():
    codes, off = synth.random_set(38, 12, 3, 12, 3)
    seqs = synth.from_csr(codes, off)
    C = np.array([1, 4, 5, 8, 11])
    D = np.array([[orc.lev(seqs[x], seqs[y]) for y in C] for x in C])
    c = int(np.argmin(D.sum(1)))
    l = int(np.argmax(D[c]))
    r = int(np.argmax(D[l]))
    assert orc.select(codes, off, C) == (C[c], C[l], C[r])


def test_exact_below_covering_set_is_exact():
    """exact_below >= n: every cluster keeps the full median."""
    codes, off = synth.random_set(39, 40, 10, 50, 4)
    t0 = orc.tree(codes, off)
    t1 = orc.tree_pruned(codes, off, _emb(15, 40), topk=1, exact_below=40)
    for f in orc.TREE_FIELDS + ("perm",):
        assert (t0[f] == t1[f]).all(), f


def test_exact_below_splits_by_size():
    """Clusters of at most exact_below members take the exact choice, larger
    ones the ranked one."""
    codes, off = synth.random_set(40, 50, 10, 50, 4)
    emb = _emb(16, 50)
    t = orc.tree_pruned(codes, off, emb, topk=1, exact_below=12)
    for v in range(t["n_nodes"]):
        C = _members(t, v)
        want = orc.select(codes, off, C) if len(C) <= 12 else orc.select(codes, off, C, emb, 1)
        assert (int(t["center"][v]), int(t["lpole"][v]), int(t["rpole"][v])) == want


def test_calibration_offset_adds_length_prior():
    """emb_q0 adds (q0)(|x| + |y|) per ordered pair, x with itself included."""
    e = _emb(17, 6)
    off = _off([5, 9, 2, 7, 3, 4])
    mem = np.arange(6, dtype=np.int32)
    q0 = 12345
    E0 = orc.emb_rowsums(off, e, mem)
    E1 = orc.emb_rowsums(off, e, mem, emb_q0=q0)
    L = np.diff(off)
    for x in range(6):
        assert int(E1[x]) - int(E0[x]) == q0 * int((L[x] + L).sum())


def test_large_offset_ranks_shortest_first():
    """An offset far above every embedding distance leaves the length prior:
    the candidates are the topk shortest members (lowest index on ties)."""
    codes, off = synth.random_set(41, 40, 10, 60, 4)
    seqs = synth.from_csr(codes, off)
    L = np.diff(off)
    topk = 4
    t = orc.tree_pruned(codes, off, _emb(18, 40, scale=1e-3), topk=topk, emb_q0=1 << 30)
    cand = np.lexsort((np.arange(40), L))[:topk]
    sums = [sum(orc.lev(seqs[x], seqs[y]) for y in range(40)) for x in cand]
    best = min(zip(sums, cand))[1]
    assert t["center"][0] == best
