"""Pins of the CPU oracle's Levenshtein distance (no GPU needed).

The oracle is checked against facts that do not come from its own
recurrence: textbook values, the shortest edit sequence found by search, the
cheapest alignment found by enumeration, and metric properties.
"""
import itertools
import os

import numpy as np
import pytest

from brute import all_alignments, alignment_cost, edit_distance_bfs
from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lev_textbook.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip("\n"):
            continue
        a, b, d, _src = line.rstrip("\n").split("\t")
        rows.append((a, b, int(d)))
    return rows


@pytest.mark.parametrize("a,b,d", _golden())
def test_textbook_values(a, b, d):
    assert orc.lev(a.encode(), b.encode()) == d
    assert orc.lev(b.encode(), a.encode()) == d
    if len(a) <= 8 and len(b) <= 8:
        # the fixture itself is re-derived by enumerating every alignment
        best = min(alignment_cost(a, b, ops) for ops in all_alignments(len(a), len(b)))
        assert best == d


def test_shortest_edit_sequence_exhaustive_binary():
    # every pair of binary strings of length <= 3
    strs = [s for L in range(4) for s in itertools.product((0, 1), repeat=L)]
    for a in strs:
        for b in strs:
            assert orc.lev(bytes(a), bytes(b)) == edit_distance_bfs(a, b, (0, 1)), (a, b)


def test_shortest_edit_sequence_random_ternary():
    rng = np.random.default_rng(11)
    for _ in range(150):
        a = tuple(int(x) for x in rng.integers(0, 3, size=int(rng.integers(0, 5))))
        b = tuple(int(x) for x in rng.integers(0, 3, size=int(rng.integers(0, 5))))
        assert orc.lev(bytes(a), bytes(b)) == edit_distance_bfs(a, b, (0, 1, 2)), (a, b)


def test_cheapest_alignment_enumeration():
    rng = np.random.default_rng(12)
    for _ in range(120):
        a = rng.integers(0, 4, size=int(rng.integers(0, 7)))
        b = rng.integers(0, 4, size=int(rng.integers(0, 7)))
        best = min(alignment_cost(a, b, o) for o in all_alignments(len(a), len(b)))
        assert orc.lev(a, b) == best


@pytest.fixture(scope="module")
def tiny_matrix():
    d = synth.tiny()
    n = d["n"]
    ia, ib = np.triu_indices(n, 1)
    dist = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    M = np.zeros((n, n), dtype=np.int64)
    M[ia, ib] = dist
    M[ib, ia] = dist
    return d, M


def test_metric_properties_tiny(tiny_matrix):
    d, M = tiny_matrix
    n = d["n"]
    L = np.diff(d["offsets"])
    seqs = synth.from_csr(d["codes"], d["offsets"])
    # identity of indiscernibles on distinct inputs, and d(x, x) = 0
    for i in range(n):
        assert orc.lev(seqs[i], seqs[i]) == 0
    off = ~np.eye(n, dtype=bool)
    assert (M[off] > 0).all()
    # symmetry of the oracle itself (argument order swapped)
    ia, ib = np.triu_indices(n, 1)
    back = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ib, ia)
    assert (back == M[ia, ib]).all()
    # |m - n| <= d <= max(m, n)
    lo = np.abs(L[:, None] - L[None, :])
    hi = np.maximum(L[:, None], L[None, :])
    assert (M >= lo).all() and (M <= hi).all()
    # triangle inequality on every ordered triple
    for y in range(n):
        assert (M <= M[:, y][:, None] + M[y, :][None, :]).all()


def test_hamming_bound_and_append():
    rng = np.random.default_rng(13)
    for _ in range(200):
        m = int(rng.integers(1, 40))
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        b = a.copy()
        flip = rng.random(m) < 0.3
        b[flip] = (b[flip] + rng.integers(1, 4, size=int(flip.sum()))) % 4
        d = orc.lev(a, b)
        assert d <= int((a != b).sum())
        s = np.uint8(rng.integers(0, 4))
        assert abs(orc.lev(np.append(a, s), b) - d) <= 1
