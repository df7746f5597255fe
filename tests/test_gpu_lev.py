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


def _check_pairs(codes_a, off_a, codes_b, off_b, sigma, ia, ib, packed=False):
    M = _msadp()
    if packed:
        A = M.to_device(M.pack_2bit_host(codes_a), off_a, sigma, packed_2bit=True)
        B = M.to_device(M.pack_2bit_host(codes_b), off_b, sigma, packed_2bit=True)
    else:
        A = M.to_device(codes_a, off_a, sigma)
        B = M.to_device(codes_b, off_b, sigma)
    got = M.lev_batch(A, B, ia, ib).cpu().numpy().astype(np.int64)
    want = orc.lev_pairs(codes_a, off_a, codes_b, off_b, ia, ib)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"


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
    sample of pairs plus every pair of the 8 shortest and 8 longest
    sequences is recomputed by the oracle."""
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
    for x in ext:
        for y in range(0, n, 97):
            ia.append(x)
            ib.append(y)
    ia, ib = np.array(ia), np.array(ib)
    keep = ia != ib
    ia, ib = ia[keep], ib[keep]
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
