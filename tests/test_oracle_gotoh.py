"""Pins of the CPU oracle's affine-gap alignment (Sec. 2.4's cost model:
a substitution score matrix and affine gaps) -- no GPU needed.

The oracle runs Gotoh's three-matrix recurrence and a backward walk; the
pins do not: they list every alignment of tiny pairs and score each one
directly, or use closed forms and reductions to simpler problems."""
import itertools

import numpy as np
import pytest

from brute import affine_score, alignment_cost, best_affine_alignment, render
from oracle import pyoracle as orc


def _rand_sub(rng, sigma, lo=-6, hi=6, sym=True):
    s = rng.integers(lo, hi + 1, size=(sigma, sigma))
    if sym:
        s = np.triu(s) + np.triu(s, 1).T
    return s.astype(np.int32)


@pytest.mark.parametrize("sym", [True, False])
def test_exhaustive_tiny_pairs_random_costs(sym):
    """Score = the best over every alignment, and the walk's alignment is
    the best one whose reversed op string is smallest (M < D < I), for random
    matrices (asymmetric too), open and extension costs, including zero
    open (plain linear gaps) and ties."""
    rng = np.random.default_rng(31 + sym)
    for t in range(500):
        sigma = int(rng.integers(2, 5))
        sub = _rand_sub(rng, sigma, sym=sym)
        open_ = int(rng.integers(0, 7))
        ext = int(rng.integers(0, 4))
        a = [int(x) for x in rng.integers(0, sigma, size=int(rng.integers(0, 6)))]
        b = [int(x) for x in rng.integers(0, sigma, size=int(rng.integers(0, 6)))]
        want_s, want_ops = best_affine_alignment(a, b, sub, open_, ext)
        s, ops = orc.gotoh(a, b, sub, open_, ext)
        assert s == want_s, (t, a, b, sub.tolist(), open_, ext)
        assert list(ops) == want_ops, (t, a, b, sub.tolist(), open_, ext)


def test_exhaustive_tiny_pairs_extreme_costs():
    """The same enumeration at the largest admitted magnitudes (|sub| up to
    2048, open + ext = 2048, either one zero) and the largest alphabet."""
    rng = np.random.default_rng(35)
    for t, (open_, ext) in enumerate([(0, 2048), (2048, 0), (48, 2000), (1000, 1000)] * 60):
        sigma = 32 if t % 2 else int(rng.integers(2, 5))
        sub = _rand_sub(rng, sigma, lo=-2048, hi=2048, sym=bool(t % 3))
        a = [int(x) for x in rng.integers(0, sigma, size=int(rng.integers(0, 6)))]
        b = [int(x) for x in rng.integers(0, sigma, size=int(rng.integers(0, 6)))]
        want_s, want_ops = best_affine_alignment(a, b, sub, open_, ext)
        s, ops = orc.gotoh(a, b, sub, open_, ext)
        assert s == want_s, (t, a, b, open_, ext)
        assert list(ops) == want_ops, (t, a, b, open_, ext)


def test_all_short_binary_pairs_tie_heavy_costs():
    """Costs chosen to make many alignments tie: match 0, mismatch -1,
    open 1, extension 1, every pair of binary strings up to length 4."""
    sub = np.array([[0, -1], [-1, 0]], np.int32)
    strs = [s for L in range(5) for s in itertools.product((0, 1), repeat=L)]
    for a in strs:
        for b in strs[::2]:
            ws, wo = best_affine_alignment(a, b, sub, 1, 1)
            s, o = orc.gotoh(a, b, sub, 1, 1)
            assert s == ws and list(o) == wo, (a, b)


def test_unit_costs_reduce_to_levenshtein_walk():
    """With sub = -[a != b], open 0, extension 1 the score is minus the
    Levenshtein distance, and the alignment is the unit-cost walk's."""
    rng = np.random.default_rng(32)
    sub = -(1 - np.eye(4, dtype=np.int32))
    for _ in range(200):
        a = rng.integers(0, 4, size=int(rng.integers(0, 60))).astype(np.uint8)
        b = rng.integers(0, 4, size=int(rng.integers(0, 60))).astype(np.uint8)
        s, o = orc.gotoh(a, b, sub, 0, 1)
        ws, wo = orc.nw(a, b)
        assert s == -ws == -orc.lev(a, b)
        assert np.array_equal(o, wo)


def test_closed_forms():
    sub = np.array([[5, -4], [-4, 5]], np.int32)
    # identical strings: all matches
    s, o = orc.gotoh([0, 1, 1, 0], [0, 1, 1, 0], sub, 10, 1)
    assert s == 20 and list(o) == [0, 0, 0, 0]
    # one side empty: a single run
    s, o = orc.gotoh([], [1, 0, 1], sub, 10, 1)
    assert s == -13 and list(o) == [2, 2, 2]
    s, o = orc.gotoh([1, 1], [], sub, 10, 1)
    assert s == -12 and list(o) == [1, 1]
    s, o = orc.gotoh([], [], sub, 10, 1)
    assert s == 0 and len(o) == 0
    # a block insertion of 3 is one run (10 + 3) whatever its position;
    # the smallest reversed op string puts it first
    a = [0, 1, 0, 1]
    b = [1, 1, 1, 0, 1, 0, 1]
    s, o = orc.gotoh(a, b, sub, 10, 1)
    assert s == 4 * 5 - 13
    assert affine_score(a, b, o, sub, 10, 1) == s


@pytest.mark.parametrize("sigma", [4, 20])
def test_invariants_random_pairs(sigma):
    """The op string consumes both sequences, scores exactly the result,
    de-gaps to the inputs, never pairs two gaps, and scores at least the
    unit-cost alignment's ops under the same costs."""
    rng = np.random.default_rng(33 + sigma)
    sub = _rand_sub(rng, sigma, -4, 11)
    np.fill_diagonal(sub, rng.integers(4, 12, size=sigma))
    for _ in range(40):
        a = rng.integers(0, sigma, size=int(rng.integers(0, 120))).astype(np.uint8)
        b = rng.integers(0, sigma, size=int(rng.integers(0, 120))).astype(np.uint8)
        s, o = orc.gotoh(a, b, sub, 10, 1)
        assert affine_score(a, b, o, sub, 10, 1) == s
        ra, rb = render(a, b, o, 255)
        assert [x for x in ra if x != 255] == list(a)
        assert [x for x in rb if x != 255] == list(b)
        assert not any(x == 255 and y == 255 for x, y in zip(ra, rb))
        _, unit_ops = orc.nw(a, b)
        assert s >= affine_score(a, b, unit_ops, sub, 10, 1)
        # symmetric matrix: swapping the sequences keeps the score
        assert orc.gotoh(b, a, sub, 10, 1)[0] == s


def test_pairs_batch_equals_single_calls():
    rng = np.random.default_rng(34)
    seqs = [rng.integers(0, 4, size=int(rng.integers(0, 50))).astype(np.uint8)
            for _ in range(12)]
    codes = np.concatenate(seqs)
    off = np.concatenate([[0], np.cumsum([len(x) for x in seqs])]).astype(np.int64)
    sub = _rand_sub(rng, 4, -3, 5)
    ia = rng.integers(0, 12, 30)
    ib = rng.integers(0, 12, 30)
    sc, ops = orc.gotoh_pairs(codes, off, codes, off, ia, ib, sub, 6, 2)
    for p in range(30):
        s, o = orc.gotoh(seqs[ia[p]], seqs[ib[p]], sub, 6, 2)
        assert sc[p] == s and np.array_equal(ops[p], o)
