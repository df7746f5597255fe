"""Brute-force characterisations used to pin the CPU oracle on tiny inputs.

These do not run the dynamic programme: they enumerate.  A plausible slip in
the oracle (an off-by-one, a swapped operand, a wrong tie order) makes one of
them disagree.
"""
from __future__ import annotations

from collections import deque
from functools import lru_cache


def edit_distance_bfs(a, b, alphabet):
    """Fewest single-symbol insertions, deletions and substitutions turning
    ``a`` into ``b`` (the definition of Levenshtein distance), by breadth-first
    search over strings.  Lengths never need to exceed max(|a|, |b|) + 1."""
    a, b = tuple(a), tuple(b)
    if a == b:
        return 0
    limit = max(len(a), len(b)) + 1
    seen = {a}
    q = deque([(a, 0)])
    while q:
        s, d = q.popleft()
        nxt = []
        for i in range(len(s)):
            nxt.append(s[:i] + s[i + 1:])
            for c in alphabet:
                if c != s[i]:
                    nxt.append(s[:i] + (c,) + s[i + 1:])
        if len(s) < limit:
            for i in range(len(s) + 1):
                for c in alphabet:
                    nxt.append(s[:i] + (c,) + s[i:])
        for t in nxt:
            if t == b:
                return d + 1
            if t not in seen:
                seen.add(t)
                q.append((t, d + 1))
    raise AssertionError("unreachable")


def all_alignments(m, n):
    """Every op string (0 = pair a_i with b_j, 1 = a_i with a gap, 2 = a gap
    with b_j) that consumes exactly m symbols of a and n of b."""
    @lru_cache(maxsize=None)
    def rec(i, j):
        if i == 0 and j == 0:
            return [()]
        out = []
        if i > 0 and j > 0:
            out += [p + (0,) for p in rec(i - 1, j - 1)]
        if i > 0:
            out += [p + (1,) for p in rec(i - 1, j)]
        if j > 0:
            out += [p + (2,) for p in rec(i, j - 1)]
        return out
    return rec(m, n)


def alignment_cost(a, b, ops):
    """Unit cost of an op string: mismatched pairs plus gaps."""
    i = j = cost = 0
    for o in ops:
        if o == 0:
            cost += a[i] != b[j]
            i += 1
            j += 1
        elif o == 1:
            cost += 1
            i += 1
        else:
            cost += 1
            j += 1
    return cost


def best_alignment(a, b):
    """(min cost, the min-cost op string whose reversal is lexicographically
    smallest with M < D < I).  Walking the cost matrix backwards and always
    preferring the diagonal, then up, then left gives exactly this string."""
    best = None
    for ops in all_alignments(len(a), len(b)):
        c = alignment_cost(a, b, ops)
        key = (c, tuple(reversed(ops)))
        if best is None or key < best[0]:
            best = (key, ops)
    return best[0][0], list(best[1])


def render(a, b, ops, gap):
    """The two gapped rows an op string describes."""
    ra, rb = [], []
    i = j = 0
    for o in ops:
        if o == 0:
            ra.append(a[i]); rb.append(b[j]); i += 1; j += 1
        elif o == 1:
            ra.append(a[i]); rb.append(gap); i += 1
        else:
            ra.append(gap); rb.append(b[j]); j += 1
    return ra, rb


def affine_score(a, b, ops, sub, open_, ext):
    """Score of an op string: substitution scores of the M columns minus
    (open + ext * length) for every maximal run of D ops or of I ops."""
    i = j = 0
    score = 0
    prev = None
    for o in ops:
        if o == 0:
            score += int(sub[a[i]][b[j]])
            i += 1
            j += 1
        else:
            score -= ext + (open_ if prev != o else 0)
            if o == 1:
                i += 1
            else:
                j += 1
        prev = o
    return score


def best_affine_alignment(a, b, sub, open_, ext):
    """(max affine score, the best-scoring op string whose reversal is
    lexicographically smallest with M < D < I), by listing every alignment."""
    best = None
    for ops in all_alignments(len(a), len(b)):
        key = (-affine_score(a, b, ops, sub, open_, ext), tuple(reversed(ops)))
        if best is None or key < best[0]:
            best = (key, ops)
    return -best[0][0], list(best[1])
