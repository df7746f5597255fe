"""Pins of the CPU oracle's sampled median (no GPU).

Sec. 2.1 lets the median be taken over a smaller subset.  The oracle's
reading (orc_tree_sampled): in a cluster above topk and exact_below members,
the pivots are the members whose input index has the least MurmurHash3
finalizer value, every member is ranked by its summed distance to the
pivots, and the topk best-ranked members compete by their exact row sums.
Pinned by reductions to the full median (pivots or topk covering every
cluster) and by a brute-force re-derivation of every node's choice from
exact distances, with the finalizer written out from its published
definition.
"""

import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth


def fmix32(h):
    """MurmurHash3's 32-bit finalizer (Appleby), from its published form."""
    h &= 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return h


def _same(a, b):
    return a["n_nodes"] == b["n_nodes"] and all(
        np.array_equal(a[f], b[f]) for f in orc.TREE_FIELDS + ("perm",))


def test_finalizer_is_a_bijection_on_a_sample():
    vals = {fmix32(i) for i in range(1 << 16)}
    assert len(vals) == 1 << 16
    assert fmix32(0) == 0


@pytest.mark.parametrize("seed,n,sigma", [(1, 40, 4), (2, 30, 20)])
def test_enough_pivots_is_the_full_median(seed, n, sigma):
    """With at least as many pivots as members the estimate is the exact row
    sum, so the exact medoid is the first candidate: the full-median tree."""
    codes, off = synth.random_set(seed, n, 3, 40, sigma)
    full = orc.tree(codes, off)
    for topk in (1, 3):
        assert _same(orc.tree_sampled(codes, off, pivots=n, topk=topk), full)


def test_topk_or_exact_below_covering_gives_the_full_median():
    codes, off = synth.random_set(3, 36, 3, 40, 4)
    full = orc.tree(codes, off)
    assert _same(orc.tree_sampled(codes, off, pivots=2, topk=36), full)
    assert _same(orc.tree_sampled(codes, off, pivots=2, topk=4, exact_below=36), full)


def _choice(seqs, mem, pivots, topk, exact_below):
    """Brute force: exact distance matrix, pivots by the finalizer, ranking,
    candidates, centre, poles (lowest index on every tie)."""
    mem = np.sort(np.asarray(mem))
    k = len(mem)
    D = np.array([[orc.lev(seqs[x], seqs[y]) for y in mem] for x in mem], dtype=np.int64)
    if k == 1:
        return int(mem[0]), -1, -1
    rows = D.sum(1)
    if k > exact_below and k > topk:
        s = min(pivots, k)
        piv = sorted(range(k), key=lambda i: fmix32(int(mem[i])))[:s]
        # mean distance to the pivots other than x, as an exact fraction
        from fractions import Fraction
        E = [Fraction(int(D[i, piv].sum()), s - 1 if i in piv else s) if s > 1 or i not in piv
             else Fraction(0) for i in range(k)]
        cand = sorted(range(k), key=lambda i: (E[i], mem[i]))[:topk]
    else:
        cand = list(range(k))
    c = min(cand, key=lambda i: (rows[i], mem[i]))
    lp = int(np.argmax(D[c]))
    if D[c, lp] == 0:
        return int(mem[c]), -1, -1
    rp = int(np.argmax(D[lp]))
    return int(mem[c]), int(mem[lp]), int(mem[rp])


@pytest.mark.parametrize("pivots,topk,exact_below", [(2, 2, 0), (3, 1, 0), (4, 3, 8)])
def test_every_node_by_brute_force(pivots, topk, exact_below):
    codes, off = synth.random_set(4, 34, 2, 30, 4)
    seqs = synth.from_csr(codes, off)
    t = orc.tree_sampled(codes, off, pivots=pivots, topk=topk, exact_below=exact_below)
    for v in range(t["n_nodes"]):
        mem = t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]]
        got = (t["center"][v], t["lpole"][v], t["rpole"][v])
        assert got == _choice(seqs, mem, pivots, topk, exact_below), v
        assert orc.select(codes, off, mem, topk=topk, exact_below=exact_below,
                          pivots=pivots) == got
        if t["left"][v] >= 0:
            # the split stays exact
            L = set(t["perm"][t["mstart"][t["left"][v]]:
                              t["mstart"][t["left"][v]] + t["mcount"][t["left"][v]]].tolist())
            l, r = got[1], got[2]
            want = {int(x) for x in mem if orc.lev(seqs[l], seqs[x]) <= orc.lev(seqs[r], seqs[x])}
            assert L == want


def test_a_pivot_is_not_favoured_by_its_own_zero_distance():
    """Three sequences where the pivot's sum over all pivots (its own 0
    included) would rank it first, but its mean distance to the other
    pivots does not."""
    pivot_of = sorted(range(3), key=fmix32)
    a, b, c = pivot_of          # a has the least hash
    seqs = [None] * 3
    seqs[a] = np.array([0] * 10, np.uint8)               # far from both others
    seqs[b] = np.array([1] * 10, np.uint8)
    seqs[c] = np.array([1] * 9 + [2], np.uint8)
    codes, off = synth.to_csr(seqs)
    # one pivot (a): every estimate is the distance to a, so a itself ranks first
    assert orc.select(codes, off, [0, 1, 2], topk=1, pivots=1)[0] == a
    # two pivots (a, b): a's mean to b is 10, b's mean to a is 10, c's mean
    # to (a, b) is (10 + 1) / 2: c wins though it is no pivot
    assert orc.select(codes, off, [0, 1, 2], topk=1, pivots=2)[0] == c


def test_sampled_families_beat_shortest_first():
    """On families of mutated copies the sampled ranking finds the exact
    medoid among few candidates far more often than a length prior (the
    reason to have it); a sanity check of the reading, not a definition."""
    rng = np.random.default_rng(5)
    seqs, _ = synth.families(rng, 6, 30, 4, lambda: 120, 0.3, 60, 200)
    hit_s = hit_l = 0
    for f in range(6):
        mem = np.arange(30 * f, 30 * f + 30)
        D = np.array([[orc.lev(seqs[x], seqs[y]) for y in mem] for x in mem])
        med = int(mem[np.argmin(D.sum(1))])
        c, _, _ = _choice(seqs, mem, 16, 4, 0)
        hit_s += c == med
        order = sorted(mem, key=lambda i: (len(seqs[i]), i))[:4]
        hit_l += med in order
    assert hit_s >= 5 and hit_s > hit_l
