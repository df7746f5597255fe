"""Needleman-Wunsch fill + traceback on the GPU against the CPU oracle."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _run(codes_a, off_a, codes_b, off_b, sigma, ia, ib):
    M = _msadp()
    A = M.to_device(codes_a, off_a, sigma)
    B = M.to_device(codes_b, off_b, sigma)
    r = M.nw_batch(A, B, ia, ib)
    ops, ops_off, ops_len = M.nw_traceback(A, B, r)
    return r.score.cpu().numpy().astype(np.int64), M.split_ops(ops, ops_off, ops_len)


def _check(codes_a, off_a, codes_b, off_b, sigma, ia, ib):
    score, ops = _run(codes_a, off_a, codes_b, off_b, sigma, ia, ib)
    ws, wops = orc.nw_pairs(codes_a, off_a, codes_b, off_b, ia, ib)
    assert (score == ws).all(), np.flatnonzero(score != ws)[:5]
    for p in range(len(ia)):
        assert np.array_equal(ops[p], wops[p]), (p, len(ops[p]), len(wops[p]))


def test_all_binary_strings_up_to_length_5():
    # every ordered pair of the 63 binary strings of length 0..5: scores and
    # the walked alignments (ties everywhere on a binary alphabet)
    import itertools
    strs = [s for L in range(6) for s in itertools.product((0, 1), repeat=L)]
    codes, off = synth.to_csr([np.array(s, dtype=np.uint8) for s in strs])
    n = len(strs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    _check(codes, off, codes, off, 2, ia.ravel(), ib.ravel())


@pytest.mark.parametrize("sigma", [2, 4, 5, 21])
def test_random_pairs(sigma):
    codes, off = synth.random_set(400 + sigma, 60, 0, 500, sigma)
    rng = np.random.default_rng(sigma)
    ia = rng.integers(0, 60, size=200)
    ib = rng.integers(0, 60, size=200)
    _check(codes, off, codes, off, sigma, ia, ib)


def test_word_and_wavefront_boundaries():
    # pattern lengths around 32-row words and 64-word wavefronts (2048 rows)
    rng = np.random.default_rng(5)
    lens = [1, 2, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 4096, 4097, 6200]
    A = [rng.integers(0, 4, size=L).astype(np.uint8) for L in lens]
    B = [synth.mutate(rng, a, 4, 0.08, 0.01, 0.01) if len(a) > 3 else
         rng.integers(0, 4, size=3).astype(np.uint8) for a in A]
    B += [rng.integers(0, 4, size=L).astype(np.uint8) for L in (1, 5, 100)]
    ca, oa = synth.to_csr(A)
    cb, ob = synth.to_csr(B)
    ia, ib = [], []
    for x in range(len(A)):
        for y in (x, len(A), len(A) + 1, len(A) + 2):
            ia.append(x)
            ib.append(y)
    _check(ca, oa, cb, ob, 4, np.array(ia), np.array(ib))


def test_texts_of_maximum_length():
    """Texts at the library's 65,535-symbol limit (and one above it, which
    is refused on the host), with one and two wavefronts per pattern."""
    M = _msadp()
    rng = np.random.default_rng(12)
    A = [rng.integers(0, 4, size=L).astype(np.uint8) for L in (40, 2100)]
    B = [rng.integers(0, 4, size=L).astype(np.uint8) for L in (65535, 65000)]
    B.append(synth.mutate(rng, np.tile(A[1], 30), 4, 0.05, 0.01, 0.01)[:65535])
    ca, oa = synth.to_csr(A)
    cb, ob = synth.to_csr(B)
    _check(ca, oa, cb, ob, 4, np.array([0, 1, 0, 1]), np.array([0, 1, 2, 2]))
    cl, ol = synth.to_csr([rng.integers(0, 4, size=65536).astype(np.uint8)])
    with pytest.raises(M.MsaError) as ex:
        M.nw_batch(M.to_device(ca, oa, 4), M.to_device(cl, ol, 4), np.array([0]), np.array([0]))
    assert ex.value.code == M.MSA_ERANGE


def test_empty_sides():
    A = [np.zeros(0, np.uint8), np.array([1, 2], np.uint8), np.array([3], np.uint8)]
    ca, oa = synth.to_csr(A)
    ia = np.array([0, 1, 0, 2, 1])
    ib = np.array([1, 0, 0, 2, 1])
    _check(ca, oa, ca, oa, 4, ia, ib)


def test_gapped_rows_alphabet_with_gap():
    # rows of partial alignments: symbols 0..3 plus the gap symbol 4
    rng = np.random.default_rng(9)
    rows = []
    for _ in range(40):
        L = int(rng.integers(150, 320))
        r = rng.integers(0, 4, size=L).astype(np.uint8)
        r[rng.random(L) < 0.2] = 4
        rows.append(r)
    c, o = synth.to_csr(rows)
    ia = np.arange(0, 40, 2)
    ib = np.arange(1, 40, 2)
    _check(c, o, c, o, 5, ia, ib)


def test_long_pairs_workload_full_parity():
    """The 512-pair long-DNA batch as the benchmark runs it (lengths
    5000-10000, 3.1e10 cells): every score and every alignment is checked
    against its defining properties and recomputed by the oracle (scores by
    Wagner-Fischer, alignments by the full-matrix walk, in chunks of 64
    pairs to bound the oracle's memory)."""
    M = _msadp()
    d = synth.nw_long()
    P = d["n_pairs"]
    A = M.to_device(d["a_codes"], d["a_offsets"], 4)
    B = M.to_device(d["b_codes"], d["b_offsets"], 4)
    ia = np.arange(P)
    r = M.nw_batch(A, B, ia, ia)
    ops, ops_off, ops_len = M.nw_traceback(A, B, r)
    score = r.score.cpu().numpy().astype(np.int64)
    allops = M.split_ops(ops, ops_off, ops_len)
    sa = synth.from_csr(d["a_codes"], d["a_offsets"])
    sb = synth.from_csr(d["b_codes"], d["b_offsets"])
    for p in range(P):
        o = allops[p]
        a, b = sa[p], sb[p]
        # the op string consumes both sequences and costs exactly the score
        assert (o != 2).sum() == len(a) and (o != 1).sum() == len(b)
        ai = np.cumsum(o != 2) - 1
        bj = np.cumsum(o != 1) - 1
        m_cols = o == 0
        cost = int((a[ai[m_cols]] != b[bj[m_cols]]).sum() + (~m_cols).sum())
        assert cost == score[p], p
    want = orc.lev_pairs(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"], ia, ia)
    assert np.array_equal(score, want)
    for c0 in range(0, P, 64):
        chunk = np.arange(c0, min(P, c0 + 64))
        print(f"[nw_long] oracle alignments {c0}..{chunk[-1]}", flush=True)
        ws, wops = orc.nw_pairs(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"],
                                chunk, chunk)
        for k, p in enumerate(chunk):
            assert score[p] == ws[k], p
            assert np.array_equal(allops[p], wops[k]), p
