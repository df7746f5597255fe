"""Pins of the CPU oracle's online insertion (no GPU).

The paper leaves insertion as future work (Sec. 5); the oracle's reading is
stated at orc_tree_insert: route each new sequence by the poles' split rule,
re-partition the leaves that grew by Alg. 1, renumber breadth-first.  These
tests pin that reading with properties the result must have whatever the
code looks like: a one-sequence tree grows into Alg. 1 on everything, copies
land beside their originals, every split of the result obeys the split rule,
old internal nodes keep their choice, new nodes make the Alg. 1 choice on
their members, and the numbering is breadth-first.
"""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth


def _members(t, v):
    a, k = int(t["mstart"][v]), int(t["mcount"][v])
    return t["perm"][a:a + k]


def _dists(seqs, x, ys):
    c, o = synth.to_csr(seqs)
    ys = np.asarray(ys, np.int32)
    return orc.lev_pairs(c, o, c, o, np.full(len(ys), x, np.int32), ys).astype(np.int64)


def check_numbering(t, n):
    """Breadth-first numbering, member ranges, perm a permutation."""
    nn = t["n_nodes"]
    assert sorted(t["perm"].tolist()) == list(range(n))
    assert t["parent"][0] == -1 and t["depth"][0] == 0
    assert t["mstart"][0] == 0 and t["mcount"][0] == n
    internal = 0
    for v in range(nn):
        if v > 0:
            assert t["depth"][v] >= t["depth"][v - 1]
        if t["left"][v] >= 0:
            # the k-th internal node (in id order) has children 2k+1, 2k+2
            assert t["left"][v] == 2 * internal + 1 and t["right"][v] == 2 * internal + 2
            internal += 1
            L, R = t["left"][v], t["right"][v]
            assert t["parent"][L] == v and t["parent"][R] == v
            assert t["depth"][L] == t["depth"][v] + 1
            assert t["mstart"][L] == t["mstart"][v]
            assert t["mstart"][R] == t["mstart"][v] + t["mcount"][L]
            assert t["mcount"][L] + t["mcount"][R] == t["mcount"][v]
        else:
            assert t["right"][v] == -1 and t["lpole"][v] == -1 and t["rpole"][v] == -1


def check_splits(seqs, t):
    """Every internal node's L child holds exactly its members x with
    f(l, x) <= f(r, x) (Alg. 1's split rule, which routing also follows)."""
    for v in range(t["n_nodes"]):
        if t["left"][v] < 0:
            continue
        mem = _members(t, v)
        dl = _dists(seqs, int(t["lpole"][v]), mem)
        dr = _dists(seqs, int(t["rpole"][v]), mem)
        want_l = set(mem[dl <= dr].tolist())
        assert set(_members(t, t["left"][v]).tolist()) == want_l, v


def alg1_choice(seqs, mem):
    """(c, l, r) of Alg. 1 on a member list by brute force: full median,
    lowest index on ties; l = r = -1 for one member or radius 0."""
    mem = np.sort(np.asarray(mem))
    if len(mem) == 1:
        return int(mem[0]), -1, -1
    D = np.stack([_dists(seqs, int(x), mem) for x in mem])
    c = int(np.argmin(D.sum(1)))
    lp = int(np.argmax(D[c]))
    if D[c, lp] == 0:
        return int(mem[c]), -1, -1
    rp = int(np.argmax(D[lp]))
    return int(mem[c]), int(mem[lp]), int(mem[rp])


def check_choices(seqs, old, new, n_old):
    """Nodes whose old members form an old internal node keep its choice;
    every other node makes Alg. 1's choice on its own members (a re-built
    leaf), and is a leaf exactly when Alg. 1 leaves it one."""
    old_internal = {}
    for v in range(old["n_nodes"]):
        if old["left"][v] >= 0:
            key = frozenset(_members(old, v).tolist())
            old_internal[key] = (old["center"][v], old["lpole"][v], old["rpole"][v])
    for v in range(new["n_nodes"]):
        mem = _members(new, v)
        key = frozenset(int(x) for x in mem if x < n_old)
        got = (new["center"][v], new["lpole"][v], new["rpole"][v])
        if key in old_internal:
            assert got == old_internal[key], v
        else:
            c, l, r = alg1_choice(seqs, mem)
            assert got == (c, l, r), (v, got, (c, l, r))
            assert (new["left"][v] < 0) == (l < 0), v


def _tree_eq(a, b):
    if a["n_nodes"] != b["n_nodes"]:
        return False
    return all(np.array_equal(a[f], b[f]) for f in orc.TREE_FIELDS + ("perm",))


def _case(seed, n_old, n_new, lo, hi, sigma):
    codes, off = synth.random_set(seed, n_old + n_new, lo, hi, sigma)
    seqs = synth.from_csr(codes, off)
    old = orc.tree(*synth.to_csr(seqs[:n_old]))
    return seqs, codes, off, old


def test_no_new_sequences_keeps_the_tree():
    seqs, codes, off, old = _case(1, 30, 0, 5, 40, 4)
    assert _tree_eq(orc.tree_insert(codes, off, 30, old), old)


@pytest.mark.parametrize("seed,n,sigma", [(2, 25, 4), (3, 18, 20)])
def test_one_sequence_tree_grows_into_alg1(seed, n, sigma):
    """The root is the only leaf, so everything is re-partitioned by Alg. 1."""
    codes, off = synth.random_set(seed, n, 3, 30, sigma)
    seqs = synth.from_csr(codes, off)
    one = orc.tree(*synth.to_csr(seqs[:1]))
    assert _tree_eq(orc.tree_insert(codes, off, 1, one), orc.tree(codes, off))


def test_copies_join_their_originals():
    """A copy of an old sequence takes the same side at every split, so it
    lands in its original's leaf, which stays a leaf (radius 0): the node
    table keeps its shape and only member counts grow."""
    codes, off = synth.random_set(4, 30, 5, 40, 4)
    seqs = synth.from_csr(codes, off)
    old = orc.tree(codes, off)
    src = [3, 17, 17, 29]
    allseqs = seqs + [seqs[i].copy() for i in src]
    c2, o2 = synth.to_csr(allseqs)
    new = orc.tree_insert(c2, o2, 30, old)
    assert new["n_nodes"] == old["n_nodes"]
    for f in ("parent", "left", "right", "center", "lpole", "rpole", "depth"):
        assert np.array_equal(new[f], old[f]), f
    for k, s in enumerate(src):
        leaf = [v for v in range(new["n_nodes"])
                if new["left"][v] < 0 and s in _members(new, v)]
        assert len(leaf) == 1 and 30 + k in _members(new, leaf[0])
    check_numbering(new, len(allseqs))


@pytest.mark.parametrize("seed,n_old,n_new,lo,hi,sigma", [
    (5, 40, 12, 5, 30, 4),      # DNA, ragged
    (6, 24, 24, 1, 20, 4),      # as many new as old, very short sequences
    (7, 30, 10, 10, 40, 20),    # protein alphabet
])
def test_insertion_obeys_its_rules(seed, n_old, n_new, lo, hi, sigma):
    seqs, codes, off, old = _case(seed, n_old, n_new, lo, hi, sigma)
    new = orc.tree_insert(codes, off, n_old, old)
    check_numbering(new, n_old + n_new)
    check_splits(seqs, new)
    check_choices(seqs, old, new, n_old)


def test_family_members_follow_their_family():
    """Members of one family inserted into a tree of several families end
    up in leaves whose old members are from that family, mostly (a sanity
    check of the reading on the kind of data the method is for)."""
    rng = np.random.default_rng(8)
    seqs, fam = synth.families(rng, 4, 12, 4, lambda: 60, 0.05, 40, 80)
    order = rng.permutation(len(seqs))
    seqs = [seqs[i] for i in order]
    fam = np.asarray(fam)[order]
    n_old = 40
    old = orc.tree(*synth.to_csr(seqs[:n_old]))
    codes, off = synth.to_csr(seqs)
    new = orc.tree_insert(codes, off, n_old, old)
    check_splits(seqs, new)
    same = 0
    for x in range(n_old, len(seqs)):
        # the deepest node holding x and at least one old member
        v = 0
        while new["left"][v] >= 0:
            nxt = [c for c in (new["left"][v], new["right"][v]) if x in _members(new, c)][0]
            if not any(m < n_old for m in _members(new, nxt)):
                break
            v = nxt
        olds = [m for m in _members(new, v) if m < n_old]
        same += all(fam[m] == fam[x] for m in olds)
    assert same >= len(seqs) - n_old - 1
