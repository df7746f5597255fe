"""Pins of the CPU oracle's Needleman-Wunsch alignment (no GPU needed)."""
import numpy as np
import pytest

from brute import alignment_cost, best_alignment, render
from oracle import pyoracle as orc


def test_exhaustive_tiny_alignments():
    # The backward walk (diagonal, then up, then left) must return exactly the
    # minimum-cost alignment whose reversed op string is smallest with
    # M < D < I -- found here by listing every alignment.
    rng = np.random.default_rng(21)
    for _ in range(400):
        a = [int(x) for x in rng.integers(0, 3, size=int(rng.integers(0, 6)))]
        b = [int(x) for x in rng.integers(0, 3, size=int(rng.integers(0, 6)))]
        cost, ops = best_alignment(a, b)
        s, o = orc.nw(a, b)
        assert s == cost
        assert list(o) == ops, (a, b)


def test_all_short_binary_pairs():
    import itertools
    strs = [s for L in range(5) for s in itertools.product((0, 1), repeat=L)]
    for a in strs[::3]:
        for b in strs:
            cost, ops = best_alignment(a, b)
            s, o = orc.nw(a, b)
            assert s == cost and list(o) == ops


@pytest.mark.parametrize("sigma", [2, 4, 5, 20])
def test_alignment_invariants(sigma):
    rng = np.random.default_rng(22 + sigma)
    gap = 255
    for _ in range(60):
        a = rng.integers(0, sigma, size=int(rng.integers(0, 80))).astype(np.uint8)
        b = rng.integers(0, sigma, size=int(rng.integers(0, 80))).astype(np.uint8)
        s, ops = orc.nw(a, b)
        assert s == orc.lev(a, b)                      # same minimum as Levenshtein
        assert alignment_cost(a, b, ops) == s           # the path costs its score
        ra, rb = render(a, b, ops, gap)
        assert [x for x in ra if x != gap] == list(a)   # de-gapped rows are the inputs
        assert [x for x in rb if x != gap] == list(b)
        assert not any(x == gap and y == gap for x, y in zip(ra, rb))
        assert max(len(a), len(b)) <= len(ops) <= len(a) + len(b)


def test_empty_sides():
    s, o = orc.nw([], [1, 2, 3])
    assert s == 3 and list(o) == [2, 2, 2]
    s, o = orc.nw([1, 2], [])
    assert s == 2 and list(o) == [1, 1]
    s, o = orc.nw([], [])
    assert s == 0 and len(o) == 0
