"""Levenshtein on the GPU against the CPU oracle, bit for bit."""
import itertools

import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu

BOUNDARY = [0, 1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 1000, 1600, 2000, 2047, 2048,
            2049, 4095, 4096, 4097]


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def lanes_fit(sigma, max_len):
    """Whether lev_batch's one-pattern-per-lane layout holds these patterns."""
    sp = 4 if sigma <= 4 else 8 if sigma <= 8 else 32
    return max_len <= 64 * (32 // sp)


def xl_fit(max_len):
    """Whether lev_batch's across-lanes layout holds these patterns (at most
    64 lanes of 4 words)."""
    return (max_len + 63) // 64 <= 256


def _check_pairs(codes_a, off_a, codes_b, off_b, sigma, ia, ib, packed=False, same=False):
    """lev_batch in every pair layout that fits (64 lanes per pattern table,
    one pattern per lane, a pattern across a group of lanes) against the
    oracle, bit for bit."""
    M = _msadp()
    if packed:
        A = M.to_device(M.pack_2bit_host(codes_a), off_a, sigma, packed_2bit=True)
        B = A if same else M.to_device(M.pack_2bit_host(codes_b), off_b, sigma, packed_2bit=True)
    else:
        A = M.to_device(codes_a, off_a, sigma)
        B = A if same else M.to_device(codes_b, off_b, sigma)
    want = orc.lev_pairs(codes_a, off_a, codes_b, off_b, ia, ib)
    ml = max(A.max_len, B.max_len)
    layouts = [64] + ([1] if lanes_fit(sigma, ml) else []) + ([2] if xl_fit(ml) else [])
    try:
        for v in layouts:
            M.tune_set(M.MSA_TUNE_PAIRS, sigma, M.pairs_words_bin(A, B), v)
            got = M.lev_batch(A, B, ia, ib).cpu().numpy().astype(np.int64)
            bad = np.flatnonzero(got != want)
            assert len(bad) == 0, (f"layout {v}: {len(bad)} mismatches, first {bad[:5]} "
                                   f"got {got[bad[:5]]} want {want[bad[:5]]}")
    finally:
        M.tune_clear()
    return layouts


def test_word_boundary_lengths_all_pairings():
    rng = np.random.default_rng(101)
    seqs = [rng.integers(0, 4, size=L).astype(np.uint8) for L in BOUNDARY]
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    _check_pairs(codes, off, codes, off, 4, ia.ravel(), ib.ravel())


def test_related_long_pairs_cross_pass_boundary():
    # patterns above 2048 rows run in several passes; similar pairs make the
    # carries between passes non-trivial
    rng = np.random.default_rng(102)
    seqs = []
    for L in (2047, 2048, 2049, 3000, 4096, 4097, 6000):
        a = rng.integers(0, 4, size=L).astype(np.uint8)
        seqs.append(a)
        seqs.append(synth.mutate(rng, a, 4, 0.05, 0.01, 0.01))
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    _check_pairs(codes, off, codes, off, 4, ia.ravel(), ib.ravel())


def test_all_binary_strings_up_to_length_8():
    # every ordered pair of the 511 binary strings of length 0..8 (261,121 pairs)
    strs = [s for L in range(9) for s in itertools.product((0, 1), repeat=L)]
    seqs = [np.array(s, dtype=np.uint8) for s in strs]
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    _check_pairs(codes, off, codes, off, 2, ia.ravel(), ib.ravel())


@pytest.mark.parametrize("sigma", [2, 4, 5, 20, 32])
def test_random_alphabets_and_ragged_lengths(sigma):
    codes, off = synth.random_set(200 + sigma, 150, 0, 700, sigma)
    rng = np.random.default_rng(sigma)
    ia = rng.integers(0, 150, size=3000)
    ib = rng.integers(0, 150, size=3000)
    _check_pairs(codes, off, codes, off, sigma, ia, ib)


def test_packed_2bit_input():
    codes, off = synth.random_set(301, 80, 0, 300, 4)
    # odd offsets make sequences start mid-byte
    rng = np.random.default_rng(3)
    ia = rng.integers(0, 80, size=2000)
    ib = rng.integers(0, 80, size=2000)
    _check_pairs(codes, off, codes, off, 4, ia, ib, packed=True)


LANE_BOUNDARY = [0, 1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 447,
                 448, 449, 511, 512]


@pytest.mark.parametrize("same", [False, True])
def test_lanes_layout_word_boundaries(same):
    """Patterns up to 512 rows (8 words: the per-lane layout for DNA), every
    ordered pairing, so both the A and the B sequence serve as pattern."""
    rng = np.random.default_rng(111)
    seqs = [rng.integers(0, 4, size=L).astype(np.uint8) for L in LANE_BOUNDARY]
    seqs += [synth.mutate(rng, s, 4, 0.1, 0.02, 0.02)[:512] for s in seqs[8:]]
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert _check_pairs(codes, off, codes, off, 4, ia.ravel(), ib.ravel(), same=same) == [64, 1, 2]


@pytest.mark.parametrize("sigma,hi", [(2, 512), (3, 500), (5, 256), (8, 256), (9, 64), (20, 64),
                                      (32, 64)])
def test_lanes_layout_alphabets(sigma, hi):
    """Each per-lane variant (sigma' = 4, 8, 32) at its longest patterns,
    two different sets (patterns drawn from either)."""
    ca, oa = synth.random_set(900 + sigma, 120, 0, hi, sigma)
    cb, ob = synth.random_set(950 + sigma, 90, 0, hi, sigma)
    rng = np.random.default_rng(sigma)
    ia = rng.integers(0, 120, size=5000)
    ib = rng.integers(0, 90, size=5000)
    assert _check_pairs(ca, oa, cb, ob, sigma, ia, ib) == [64, 1, 2]


def test_sparse_pairs_learned_workload_sampled():
    """The 2 M training-label batch over the 100,000-sequence DNA set (lengths
    100-500, about 20 pairs per sequence), in the layout lev_batch picks by
    default (one pattern per lane); 30,000 sampled pairs recomputed by the
    oracle, length bounds on every pair."""
    from paper_2601_15458_amd import learned
    M = _msadp()
    d = synth.learned()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    ia, ib = learned.sample_pairs(d["family"], 2_000_000, seed=11)
    got = M.lev_batch(S, S, ia, ib).cpu().numpy().astype(np.int64)
    L = np.diff(d["offsets"])
    assert (got >= np.abs(L[ia] - L[ib])).all() and (got <= np.maximum(L[ia], L[ib])).all()
    pick = np.random.default_rng(5).choice(len(ia), 30000, replace=False)
    want = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia[pick], ib[pick])
    assert (got[pick] == want).all()


def test_random_pair_list_allpairs_set():
    """8,386,560 random pairs of the 4096-sequence set (shared-pattern
    layout: about 2000 pairs per pattern): 20,000 sampled pairs recomputed by
    the oracle, and every pair equal to lev_allpairs' entry."""
    M = _msadp()
    d = synth.allpairs()
    n = d["n"]
    A = M.to_device(d["codes"], d["offsets"], d["sigma"])
    rng = np.random.default_rng(8)
    ia = rng.integers(0, n, size=n * (n - 1) // 2).astype(np.int32)
    ib = rng.integers(0, n, size=n * (n - 1) // 2).astype(np.int32)
    got = M.lev_batch(A, A, ia, ib).cpu().numpy().astype(np.int64)
    pick = rng.choice(len(ia), 20000, replace=False)
    want = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia[pick], ib[pick])
    assert (got[pick] == want).all()
    cond = M.lev_allpairs(A).cpu().numpy().astype(np.int64)
    i, j = np.minimum(ia, ib).astype(np.int64), np.maximum(ia, ib).astype(np.int64)
    off = i != j
    idx = i[off] * n - i[off] * (i[off] + 1) // 2 + (j[off] - i[off] - 1)
    assert (got[off] == cond[idx]).all() and (got[~off] == 0).all()


def test_autotune_pairs_picks_a_layout():
    M = _msadp()
    codes, off = synth.random_set(77, 500, 100, 500, 4)
    A = M.to_device(codes, off, 4)
    rng = np.random.default_rng(9)
    ia, ib = rng.integers(0, 500, 20000), rng.integers(0, 500, 20000)
    lb = M.LevBatch(A, A, ia, ib)
    try:
        best, ms = M.autotune_pairs(lb, reps=2)
        assert best in (1, 2, 64) and ms > 0
        assert M.tune_get(M.MSA_TUNE_PAIRS, 4, M.pairs_words_bin(A, A)) == best
        want = orc.lev_pairs(codes, off, codes, off, ia, ib)
        assert (lb().cpu().numpy().astype(np.int64) == want).all()
    finally:
        M.tune_clear()


def test_tiny_workload_allpairs_and_batch():
    M = _msadp()
    d = synth.tiny()
    A = M.to_device(d["codes"], d["offsets"], d["sigma"])
    got = M.lev_allpairs(A).cpu().numpy().astype(np.int64)
    n = d["n"]
    ia, ib = np.triu_indices(n, 1)
    want = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    assert (got == want).all()
    got2 = M.lev_batch(A, A, ia, ib).cpu().numpy().astype(np.int64)
    assert (got2 == want).all()


def test_allpairs_ragged_small_sets():
    M = _msadp()
    for n, seed in [(2, 1), (3, 2), (65, 3), (130, 4)]:
        codes, off = synth.random_set(seed, n, 0, 200, 4)
        A = M.to_device(codes, off, 4)
        got = M.lev_allpairs(A).cpu().numpy().astype(np.int64)
        ia, ib = np.triu_indices(n, 1)
        want = orc.lev_pairs(codes, off, codes, off, ia, ib)
        assert (got == want).all(), n


def test_allpairs_workload_full_size_sampled():
    """The 4096-sequence all-pairs batch as the benchmark runs it; a seeded
    sample of pairs plus every pair that touches one of the 8 shortest or 8
    longest sequences (65,520 pairs) is recomputed by the oracle."""
    M = _msadp()
    d = synth.allpairs()
    n = d["n"]
    A = M.to_device(d["codes"], d["offsets"], d["sigma"])
    got = M.lev_allpairs(A).cpu().numpy().astype(np.int64)
    L = np.diff(d["offsets"])
    order = np.argsort(L, kind="stable")
    ext = np.concatenate([order[:8], order[-8:]])
    rng = np.random.default_rng(77)
    ia = list(rng.integers(0, n, size=1500))
    ib = list(rng.integers(0, n, size=1500))
    ia, ib = np.array(ia), np.array(ib)
    keep = ia != ib
    ia, ib = ia[keep], ib[keep]
    # every pair touching an extreme sequence, each unordered pair once
    ex_i, ex_j = [], []
    ext_set = set(int(x) for x in ext)
    for x in ext:
        for y in range(n):
            if y != x and not (y in ext_set and y < x):
                ex_i.append(x)
                ex_j.append(y)
    assert len(ex_i) == 16 * (n - 1) - 16 * 15 // 2
    ia = np.concatenate([ia, ex_i])
    ib = np.concatenate([ib, ex_j])
    i, j = np.minimum(ia, ib), np.maximum(ia, ib)
    idx = i * n - i * (i + 1) // 2 + (j - i - 1)
    want = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    assert (got[idx] == want).all()
    # properties at full size: bounds by length difference and maximum length
    ii, jj = np.triu_indices(n, 1)
    assert (got >= np.abs(L[ii] - L[jj])).all() and (got <= np.maximum(L[ii], L[jj])).all()


def test_device_detected_errors():
    M = _msadp()
    codes = np.array([0, 1, 2, 7, 1], dtype=np.uint8)    # 7 >= sigma
    off = np.array([0, 2, 5], dtype=np.int64)
    A = M.to_device(codes, off, 4)
    with pytest.raises(RuntimeError, match="symbol"):
        M.lev_batch(A, A, [0], [1])
    codes = np.array([0, 1, 2, 3, 1], dtype=np.uint8)
    A = M.to_device(codes, off, 4)
    with pytest.raises(RuntimeError, match="index"):
        M.lev_batch(A, A, [0], [5])
    # every layout flags the bad pair and leaves 0xFFFF in its slot
    for v in (64, 1, 2):
        M.tune_set(M.MSA_TUNE_PAIRS, 4, 1, v)
        try:
            got = M.lev_batch(A, A, [0, 1, -1], [1, 0, 0], check=False).cpu().numpy()
        finally:
            M.tune_clear()
        assert got[2] == 0xFFFF and got[0] == got[1] == orc.lev_pairs(
            codes, off, codes, off, np.array([0]), np.array([1]))[0]


@pytest.mark.parametrize("sigma,lens", [
    (4, (1, 63, 64, 65, 500, 4095, 4096, 4097, 8191, 8192, 12000, 16384)),   # 1-4 words per lane
    (20, (5, 64, 700, 2049, 5000)),                                          # five bit planes
])
def test_across_lanes_layout_long_patterns(sigma, lens):
    """A pattern across 8-64 lanes of one to four words each (up to the
    16,384-row limit), related and unrelated texts, few pairs per sequence,
    against the oracle."""
    M = _msadp()
    rng = np.random.default_rng(103 + sigma)
    seqs = []
    for L in lens:
        a = rng.integers(0, sigma, size=L).astype(np.uint8)
        seqs += [a, synth.mutate(rng, a, sigma, 0.08, 0.02, 0.02)]
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia = np.concatenate([np.arange(0, n, 2), np.arange(n), [0, n - 1]])
    ib = np.concatenate([np.arange(1, n, 2), rng.permutation(n), [n - 1, n - 1]])
    A = M.to_device(codes, off, sigma)
    want = orc.lev_pairs(codes, off, codes, off, ia, ib)
    M.tune_clear()
    got = M.lev_batch(A, A, ia, ib).cpu().numpy().astype(np.int64)   # the default: across lanes
    assert np.array_equal(got, want)


def test_across_lanes_layout_long_pair_workload():
    """The 512 pairs of 5-10 kbp DNA (10 % divergence) through lev_batch's
    default layout for them (a pair per 64 lanes of 2-3 words): every
    distance equal to the oracle's."""
    M = _msadp()
    d = synth.nw_long()
    P = d["n_pairs"]
    A = M.to_device(d["a_codes"], d["a_offsets"], 4)
    B = M.to_device(d["b_codes"], d["b_offsets"], 4)
    ia = ib = np.arange(P)
    print("[lev] long pairs: device", flush=True)
    got = M.lev_batch(A, B, ia, ib).cpu().numpy().astype(np.int64)
    print("[lev] long pairs: oracle", flush=True)
    want = orc.lev_pairs(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"], ia, ib)
    assert np.array_equal(got, want)
