"""Pins of the alignment-quality oracle (Sec. 2.3 metrics; Table 2 shapes):
a hand-worked pair, the shapes the paper prints, closed forms, identities
from the rows' gap masks, and the bounds a true alignment must meet."""
import os

import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "quality_table2.txt")
A, C, G, T, GAP = 0, 1, 2, 3, 4


def test_hand_worked_pair():
    # x = A C - G T - A, y = A G - G - T A (column 3 is gap-gap)
    x = [A, C, GAP, G, T, GAP, A]
    y = [A, G, GAP, G, GAP, T, A]
    msa = np.array([x, y], np.uint8)
    h, al, mm = orc.msa_pair_counts(msa, GAP, [0], [1])
    # differing columns: C/G, T/-, -/T; residue in both rows: A/A C/G G/G A/A
    assert (h[0], al[0], mm[0]) == (3, 4, 1)
    assert list(orc.msa_row_gaps(msa, GAP)) == [2, 2]
    q = orc.msa_quality(msa, GAP, 5, [0], [1], [2])
    assert q["p_min"] == q["p_avg"] == q["p_max"] == 0.25
    assert q["distortion"] == 1.5                 # Hamming 3 over the given distance 2
    assert q["pct_gaps"] == pytest.approx(100.0 * 2 / 7, rel=1e-14)
    assert q["stretch"] == 7 / 5


def _golden():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, mean, mx, width, stretch, pct, src = line.rstrip("\n").split("\t")
        rows.append((name, float(mean), int(mx), int(width), float(stretch), float(pct)))
    return rows


def _msa_with_lengths(lengths, width, sigma, gap, rng):
    """Rows of the given residue counts, the gaps scattered at random."""
    msa = np.full((len(lengths), width), gap, np.uint8)
    for i, L in enumerate(lengths):
        cols = np.sort(rng.choice(width, size=L, replace=False))
        msa[i, cols] = rng.integers(0, sigma, size=L)
    return msa


@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[0])
def test_table2_shapes(row):
    name, mean, mx, width, stretch, pct = row
    rng = np.random.default_rng(7)
    n = 100                                          # 100 rows: the mean is an integer sum
    total = int(round(mean * n))
    rest = total - mx                                # one longest sequence, the rest even
    lengths = np.full(n, rest // (n - 1))
    lengths[: rest - lengths[:-1].sum()] += 1
    lengths[-1] = mx
    assert lengths.sum() == total and lengths.max() == mx and lengths.min() > 0
    msa = _msa_with_lengths(lengths, width, 20, 20, rng)
    q = orc.msa_quality(msa, 20, mx, [], [], [])
    assert round(q["pct_gaps"], 2) == pct, (name, q["pct_gaps"])
    assert round(q["stretch"], 2) == stretch, (name, q["stretch"])


def test_pct_gaps_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(20):
        rows, width = int(rng.integers(1, 40)), int(rng.integers(1, 300))
        lengths = rng.integers(0, width + 1, size=rows)
        msa = _msa_with_lengths(lengths, width, 4, GAP, rng)
        q = orc.msa_quality(msa, GAP, max(1, int(lengths.max())), [], [], [])
        assert q["pct_gaps"] == pytest.approx(100.0 * (1.0 - lengths.mean() / width), rel=1e-12)
        assert list(orc.msa_row_gaps(msa, GAP)) == list(width - lengths)


def test_counts_against_gap_masks():
    # aligned = width - (columns with one gap) - (columns with two gaps) and
    # hamming = mismatched + (columns with one gap), from bit masks of the rows
    rng = np.random.default_rng(4)
    rows, width = 30, 257
    msa = _msa_with_lengths(rng.integers(0, width + 1, size=rows), width, 4, GAP, rng)
    ia, ib = np.triu_indices(rows, 1)
    h, al, mm = orc.msa_pair_counts(msa, GAP, ia, ib)
    g = msa == GAP
    for p, (i, j) in enumerate(zip(ia, ib)):
        one = int(np.count_nonzero(g[i] ^ g[j]))
        two = int(np.count_nonzero(g[i] & g[j]))
        assert al[p] == width - one - two
        assert h[p] == mm[p] + one
        assert mm[p] <= al[p]


def _degap(row, gap):
    return row[row != gap]


def test_distortion_bounds_on_merged_alignment():
    # every pair of rows of an alignment is an alignment of the two
    # sequences, whose cost (the Hamming distance) is at least their
    # Levenshtein distance: distortion >= 1 pair by pair
    d = synth.tiny()
    t = orc.tree(d["codes"], d["offsets"])
    msa = orc.merge(d["codes"], d["offsets"], d["sigma"], t)
    gap = d["sigma"]
    n = d["n"]
    ia, ib = np.triu_indices(n, 1)
    lev = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    h, al, mm = orc.msa_pair_counts(msa, gap, ia, ib)
    assert (h >= lev).all()
    q = orc.msa_quality(msa, gap, int(np.diff(d["offsets"]).max()), ia, ib, lev)
    assert q["distortion"] >= 1.0
    assert 0.0 <= q["p_min"] <= q["p_avg"] <= q["p_max"] <= 1.0
    for i in range(n):
        s = d["codes"][d["offsets"][i]:d["offsets"][i + 1]]
        assert np.array_equal(_degap(msa[i], gap), s)


def test_distortion_one_for_optimal_pairwise_alignments():
    # a 2-row alignment of minimum cost has Hamming distance = Levenshtein
    d = synth.tiny()
    n = d["n"]
    ia = np.arange(0, n - 1, 3)
    ib = ia + 1
    scores, ops = orc.nw_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    gap = d["sigma"]
    for p in range(len(ia)):
        a = list(d["codes"][d["offsets"][ia[p]]:d["offsets"][ia[p] + 1]])
        b = list(d["codes"][d["offsets"][ib[p]]:d["offsets"][ib[p] + 1]])
        ra, rb = [], []
        for op in ops[p]:
            ra.append(a.pop(0) if op in (0, 1) else gap)
            rb.append(b.pop(0) if op in (0, 2) else gap)
        msa = np.array([ra, rb], np.uint8)
        q = orc.msa_quality(msa, gap, len(ra), [0], [1], [scores[p]])
        if scores[p] > 0:
            assert q["distortion"] == 1.0


def test_hand_worked_three_rows():
    # x = A C - G T - A, y = A G - G - T A, z = T G - C T - -
    # (x,y): differ C/G T/- -/T; residues in both: cols 0 1 3 6; C/G differs
    # (x,z): differ A/T C/G G/C A/-; both: cols 0 1 3 4; three differ
    # (y,z): differ A/T G/C -/T T/- A/-; both: cols 0 1 3; two differ
    x = [A, C, GAP, G, T, GAP, A]
    y = [A, G, GAP, G, GAP, T, A]
    z = [T, G, GAP, C, T, GAP, GAP]
    msa = np.array([x, y, z], np.uint8)
    ia, ib = [0, 0, 1], [1, 2, 2]
    h, al, mm = orc.msa_pair_counts(msa, GAP, ia, ib)
    assert list(h) == [3, 4, 5] and list(al) == [4, 4, 3] and list(mm) == [1, 3, 2]
    q = orc.msa_quality(msa, GAP, 6, ia, ib, [2, 3, 4])
    # the p-score is averaged over pairs (not pooled: 6 / 11 would differ)
    assert q["p_avg"] == pytest.approx((1 / 4 + 3 / 4 + 2 / 3) / 3, rel=1e-15)
    assert (q["p_min"], q["p_max"]) == (0.25, 0.75)
    assert q["distortion"] == pytest.approx((3 / 2 + 4 / 3 + 5 / 4) / 3, rel=1e-15)
    assert q["pct_gaps"] == pytest.approx(100.0 * (2 + 2 + 3) / 21, rel=1e-14)
    assert (q["n_p_pairs"], q["n_d_pairs"]) == (3, 3)
