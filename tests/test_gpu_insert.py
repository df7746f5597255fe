"""Online insertion on the GPU (tree_insert) against the CPU oracle.

Small and mid-size cases compare every node array (perm up to the order
inside a leaf of copies) and the merged alignment byte for byte; the
100,000-sequence learned workload, too large for the oracle's tree, is
checked by properties that hold at any size: breadth-first numbering and
member ranges, and on sampled new sequences the split rule at every node of
their path (distances from the oracle) and Alg. 1's choice in the subtree
that re-partitioned their leaf.
"""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _sorted_copy_leaves(t):
    p = t["perm"].copy()
    for v in range(t["n_nodes"]):
        if t["left"][v] < 0 and t["mcount"][v] > 1:
            a, k = t["mstart"][v], t["mcount"][v]
            p[a:a + k].sort()
    return p


def _compare(got, want):
    assert got["n_nodes"] == want["n_nodes"], (got["n_nodes"], want["n_nodes"])
    for f in orc.TREE_FIELDS:
        g, w = got[f].astype(np.int64), want[f].astype(np.int64)
        bad = np.flatnonzero(g != w)
        assert len(bad) == 0, (f, bad[:5], g[bad[:5]], w[bad[:5]])
    assert np.array_equal(_sorted_copy_leaves(got), _sorted_copy_leaves(want))


def _run(seqs, n_old, sigma, check_msa=False):
    M = _msadp()
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    print(f"[insert] n_old={n_old} n_new={n - n_old} sigma={sigma}", flush=True)
    S_old = M.to_device(*synth.to_csr(seqs[:n_old]), sigma)
    old = M.tree_build(S_old)
    S = M.to_device(codes, off, sigma)
    t = M.tree_insert(S, n_old, old)
    got = t.host()
    want = orc.tree_insert(codes, off, n_old, orc.tree(*synth.to_csr(seqs[:n_old])))
    _compare(got, want)
    if check_msa:
        msa = M.msa_merge(S, t)
        ref = orc.merge(codes, off, sigma, want)
        assert msa.shape == ref.shape, (msa.shape, ref.shape)
        assert np.array_equal(msa, ref)
    return got


@pytest.mark.parametrize("seed,n_old,n_new,lo,hi,sigma", [
    (1, 60, 20, 5, 90, 4),       # DNA, ragged, several tiles of one word
    (2, 40, 40, 1, 30, 4),       # as many new as old, very short sequences
    (3, 50, 15, 20, 200, 20),    # protein alphabet, multi-word patterns
    (4, 30, 1, 100, 700, 4),     # one new sequence, patterns past 512 symbols
])
def test_insert_matches_oracle(seed, n_old, n_new, lo, hi, sigma):
    codes, off = synth.random_set(seed, n_old + n_new, lo, hi, sigma)
    _run(synth.from_csr(codes, off), n_old, sigma, check_msa=True)


def test_insert_nothing_keeps_the_tree():
    codes, off = synth.random_set(5, 50, 5, 60, 4)
    seqs = synth.from_csr(codes, off)
    got = _run(seqs, 50, 4)
    want = orc.tree(codes, off)
    _compare(got, want)


def test_insert_into_one_sequence_is_alg1():
    codes, off = synth.random_set(6, 45, 5, 60, 4)
    seqs = synth.from_csr(codes, off)
    got = _run(seqs, 1, 4, check_msa=True)
    _compare(got, orc.tree(codes, off))


def test_insert_copies_and_duplicates():
    """Copies of old sequences (their leaves stay leaves of copies), copies
    of one new sequence among themselves, and an empty sequence."""
    codes, off = synth.random_set(7, 40, 3, 50, 4)
    seqs = synth.from_csr(codes, off)
    rng = np.random.default_rng(7)
    extra = [seqs[i].copy() for i in (0, 5, 5, 39)]
    fresh = rng.integers(0, 4, size=30).astype(np.uint8)
    extra += [fresh, fresh.copy(), fresh.copy(), np.zeros(0, np.uint8)]
    _run(seqs + extra, 40, 4, check_msa=True)


def test_insert_family_subset_matches_oracle():
    """1,000 members of the learned workload's families (DNA, 100-500) with
    100 more inserted: every node and the alignment equal the oracle's."""
    d = synth.learned()
    rng = np.random.default_rng(41)
    idx = rng.choice(d["n"], size=1100, replace=False)
    seqs = synth.from_csr(d["codes"], d["offsets"])
    _run([seqs[i] for i in idx], 1000, 4, check_msa=True)


def _members(t, v):
    a, k = int(t["mstart"][v]), int(t["mcount"][v])
    return t["perm"][a:a + k]


def test_insert_full_workload_properties():
    """100,000 learned-workload sequences: 99,000 build the tree, 1,000 are
    inserted (seeded choice)."""
    M = _msadp()
    d = synth.learned()
    n = d["n"]
    rng = np.random.default_rng(42)
    new = np.sort(rng.choice(n, size=1000, replace=False))
    keep = np.setdiff1d(np.arange(n), new)
    seqs = synth.from_csr(d["codes"], d["offsets"])
    order = np.concatenate([keep, new])
    allseqs = [seqs[i] for i in order]
    n_old = len(keep)
    print(f"[insert] full workload: {n_old} old + {len(new)} new; device build", flush=True)
    S_old = M.to_device(*synth.to_csr(allseqs[:n_old]), 4)
    old = M.tree_build(S_old)
    codes, off = synth.to_csr(allseqs)
    S = M.to_device(codes, off, 4)
    t = M.tree_insert(S, n_old, old).host()
    print(f"[insert] {old['n_nodes']} -> {t['n_nodes']} nodes; checks", flush=True)
    nn = t["n_nodes"]
    left, right = t["left"].astype(np.int64), t["right"].astype(np.int64)
    internal = np.flatnonzero(left >= 0)
    # breadth-first: the k-th internal node has children 2k+1, 2k+2
    assert np.array_equal(left[internal], 2 * np.arange(len(internal)) + 1)
    assert np.array_equal(right[internal], left[internal] + 1)
    assert np.all(np.diff(t["depth"]) >= 0)
    assert np.array_equal(np.sort(t["perm"]), np.arange(n))
    ms, mc = t["mstart"], t["mcount"]
    assert ms[0] == 0 and mc[0] == n
    assert np.array_equal(ms[left[internal]], ms[internal])
    assert np.array_equal(ms[right[internal]], ms[internal] + mc[left[internal]])
    assert np.array_equal(mc[left[internal]] + mc[right[internal]], mc[internal])
    # old internal nodes keep their choice: the old tree's internal nodes,
    # matched by their (center, lpole, rpole), all appear
    old_clr = {(int(c), int(l), int(r)) for c, l, r, L in
               zip(old["center"], old["lpole"], old["rpole"], old["left"]) if L >= 0}
    new_clr = {(int(c), int(l), int(r)) for c, l, r, L in
               zip(t["center"], t["lpole"], t["rpole"], left) if L >= 0}
    assert old_clr <= new_clr
    # sampled new sequences: split rule on their whole path; Alg. 1's choice
    # below the deepest node that was internal in the old tree
    parent = t["parent"]
    pos = np.empty(n, np.int64)
    pos[t["perm"]] = np.arange(n)
    leaf_of = np.empty(n, np.int64)
    for v in np.flatnonzero(left < 0):
        leaf_of[_members(t, v)] = v
    for x in rng.choice(np.arange(n_old, n), size=40, replace=False):
        path = []
        v = int(leaf_of[x])
        while v >= 0:
            path.append(v)
            v = int(parent[v])
        path.reverse()
        for v in path[:-1]:
            l, r = int(t["lpole"][v]), int(t["rpole"][v])
            dl = orc.lev(allseqs[l], allseqs[x])
            dr = orc.lev(allseqs[r], allseqs[x])
            in_left = ms[left[v]] <= pos[x] < ms[left[v]] + mc[left[v]]
            assert in_left == (dl <= dr), (x, v)
        for v in path:
            clr = (int(t["center"][v]), int(t["lpole"][v]), int(t["rpole"][v]))
            if left[v] >= 0 and clr in old_clr:
                continue
            mem = np.sort(_members(t, v))
            k = len(mem)
            ia = np.repeat(np.arange(k), k).astype(np.int32)
            ib = np.tile(np.arange(k), k).astype(np.int32)
            sc, so = synth.to_csr([allseqs[i] for i in mem])
            D = orc.lev_pairs(sc, so, sc, so, ia, ib).reshape(k, k).astype(np.int64)
            c = int(np.argmin(D.sum(1)))
            lp = int(np.argmax(D[c]))
            if k == 1 or D[c, lp] == 0:
                assert clr == (int(mem[c]), -1, -1) and left[v] < 0
            else:
                rp = int(np.argmax(D[lp]))
                assert clr == (int(mem[c]), int(mem[lp]), int(mem[rp]))
