"""Affine-gap Needleman-Wunsch (Sec. 2.4's cost model) on the GPU against the
CPU oracle: scores and alignments bit for bit."""
import itertools

import numpy as np
import pytest

from brute import affine_score
from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def dna_scores():
    """Stand-in nucleotide matrix: +5 for a match, -4 for a mismatch."""
    return np.where(np.eye(4, dtype=bool), 5, -4).astype(np.int32)


def protein_scores(seed=7):
    """Stand-in for a protein substitution matrix (the real tables are not
    available here): symmetric, diagonal 4..11, off-diagonal -4..3."""
    rng = np.random.default_rng(seed)
    s = rng.integers(-4, 4, size=(20, 20))
    s = np.triu(s) + np.triu(s, 1).T
    np.fill_diagonal(s, rng.integers(4, 12, size=20))
    return s.astype(np.int32)


def _check(codes_a, off_a, codes_b, off_b, sigma, ia, ib, sub, open_, ext):
    M = _msadp()
    A = M.to_device(codes_a, off_a, sigma)
    B = M.to_device(codes_b, off_b, sigma)
    print(f"[gotoh] {len(ia)} pairs sigma={sigma} open={open_} ext={ext}", flush=True)
    sc, ops = M.gotoh(A, B, ia, ib, sub, open_, ext)
    ws, wops = orc.gotoh_pairs(codes_a, off_a, codes_b, off_b, ia, ib, sub, open_, ext)
    bad = np.flatnonzero(sc != ws)
    assert len(bad) == 0, (bad[:5], sc[bad[:5]], ws[bad[:5]])
    for p in range(len(ia)):
        assert np.array_equal(ops[p], wops[p]), p
    return sc, ops


def test_all_short_ternary_pairs_random_costs():
    """Every pair of ternary strings up to length 3 (and a sample up to 4)
    under several random matrices, open and extension costs (zero too)."""
    strs = [s for L in range(4) for s in itertools.product(range(3), repeat=L)]
    strs += [s for s in itertools.product(range(3), repeat=4)][::5]
    seqs = [np.array(s, np.uint8) for s in strs]
    codes, off = synth.to_csr(seqs)
    n = len(seqs)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()
    rng = np.random.default_rng(1)
    for open_, ext in [(0, 1), (3, 1), (5, 2), (1, 0), (0, 0)]:
        sub = rng.integers(-3, 4, size=(3, 3)).astype(np.int32)
        _check(codes, off, codes, off, 3, ia, ib, sub, open_, ext)


@pytest.mark.parametrize("kind", ["dna", "protein"])
def test_block_and_wavefront_boundaries(kind):
    """Pattern lengths around the 16-row lane blocks and the 1024-row
    wavefronts, related and unrelated texts of ragged lengths."""
    rng = np.random.default_rng(2 if kind == "dna" else 3)
    sigma = 4 if kind == "dna" else 20
    sub = dna_scores() if kind == "dna" else protein_scores()
    lens = [1, 2, 15, 16, 17, 31, 33, 1023, 1024, 1025, 1040, 2047, 2049, 3000]
    seqs_a, seqs_b = [], []
    for L in lens:
        a = rng.integers(0, sigma, size=L).astype(np.uint8)
        seqs_a.append(a)
        seqs_b.append(synth.mutate(rng, a, sigma, 0.1, 0.03, 0.03))
        seqs_a.append(a)
        seqs_b.append(rng.integers(0, sigma, size=int(rng.integers(1, 300))).astype(np.uint8))
    ca, oa = synth.to_csr(seqs_a)
    cb, ob = synth.to_csr(seqs_b)
    P = len(seqs_a)
    _check(ca, oa, cb, ob, sigma, np.arange(P), np.arange(P), sub, 10, 1)


def test_extreme_costs_and_alphabet():
    """Costs at the admitted limits (|sub| up to 2048, open + ext = 2048, a
    zero open or extension), the largest alphabet (symbol 31 on both sides),
    patterns over several wavefronts and a 65,535-symbol text: the fill's
    values (offset by (i + j) ext) reach their widest range here."""
    rng = np.random.default_rng(11)
    sigma = 32
    sub = rng.integers(-2048, 2049, size=(sigma, sigma)).astype(np.int32)
    sub[sigma - 1, sigma - 1] = 2048
    seqs_a, seqs_b = [], []
    for L in (1, 17, 1025, 2100, 3100):
        a = rng.integers(0, sigma, size=L).astype(np.uint8)
        a[-1] = sigma - 1
        seqs_a.append(a)
        seqs_b.append(synth.mutate(rng, a, sigma, 0.1, 0.03, 0.03))
        seqs_a.append(a)
        seqs_b.append(rng.integers(0, sigma, size=int(rng.integers(1, 700))).astype(np.uint8))
    seqs_a.append(rng.integers(0, sigma, size=40).astype(np.uint8))
    seqs_b.append(rng.integers(0, sigma, size=65535).astype(np.uint8))
    ca, oa = synth.to_csr(seqs_a)
    cb, ob = synth.to_csr(seqs_b)
    P = len(seqs_a)
    for open_, ext in [(0, 2048), (2048, 0), (48, 2000), (1000, 1000)]:
        _check(ca, oa, cb, ob, sigma, np.arange(P), np.arange(P), sub, open_, ext)


def test_longest_patterns_sixteen_wavefronts():
    """16,384-row patterns (16 wavefronts of one workgroup) against short and
    related texts; one row more is refused on the host."""
    M = _msadp()
    rng = np.random.default_rng(4)
    a = rng.integers(0, 4, size=16384).astype(np.uint8)
    seqs_b = [rng.integers(0, 4, size=40).astype(np.uint8),
              synth.mutate(rng, a, 4, 0.05, 0.01, 0.01)[:2000]]
    ca, oa = synth.to_csr([a])
    cb, ob = synth.to_csr(seqs_b)
    _check(ca, oa, cb, ob, 4, np.array([0, 0]), np.array([0, 1]), dna_scores(), 10, 1)
    ca2, oa2 = synth.to_csr([np.zeros(16385, np.uint8)])
    A = M.to_device(ca2, oa2, 4)
    B = M.to_device(cb, ob, 4)
    with pytest.raises(M.MsaError) as e:
        M.gotoh(A, B, [0], [0], dna_scores(), 10, 1)
    assert e.value.code == M.MSA_ERANGE


def test_unit_costs_equal_unit_cost_aligner():
    """With sub = -[a != b], open 0, extension 1 the score is minus the
    unit-cost NW score and the alignment is nw_traceback's (two entry points
    of the library agree)."""
    M = _msadp()
    codes, off = synth.random_set(5, 60, 0, 400, 4)
    rng = np.random.default_rng(5)
    ia, ib = rng.integers(0, 60, 200), rng.integers(0, 60, 200)
    A = M.to_device(codes, off, 4)
    sub = -(1 - np.eye(4, dtype=np.int32))
    sc, ops = M.gotoh(A, A, ia, ib, sub, 0, 1)
    r = M.nw_batch(A, A, ia, ib)
    nops = M.split_ops(*M.nw_traceback(A, A, r))
    assert np.array_equal(sc, -r.score.cpu().numpy().astype(np.int64))
    for p in range(200):
        assert np.array_equal(ops[p], nops[p]), p


def test_empty_sequences_and_bad_arguments():
    M = _msadp()
    seqs = [np.zeros(0, np.uint8), np.array([1, 2, 3], np.uint8), np.array([0], np.uint8)]
    codes, off = synth.to_csr(seqs)
    ia = np.array([0, 0, 1, 2, 1])
    ib = np.array([0, 1, 0, 1, 1])
    sc, ops = _check(codes, off, codes, off, 4, ia, ib, dna_scores(), 10, 1)
    assert sc[0] == 0 and sc[1] == -13 and sc[2] == -13
    A = M.to_device(codes, off, 4)
    for sub, o, e in [(dna_scores() * 1000, 10, 1), (dna_scores(), -1, 1),
                      (dna_scores(), 2000, 100)]:
        with pytest.raises(M.MsaError) as err:
            M.gotoh(A, A, [0], [1], sub, o, e)
        assert err.value.code == M.MSA_EINVAL
    with pytest.raises(RuntimeError, match="index"):
        M.gotoh(A, A, [0], [7], dna_scores(), 10, 1)


def _affine_scores_np(a, b, ops, sub, open_, ext):
    """Vectorized affine_score of one op string (numpy)."""
    ops = np.asarray(ops)
    ai = np.cumsum(ops != 2) - 1
    bj = np.cumsum(ops != 1) - 1
    mcol = ops == 0
    s = int(sub[a[ai[mcol]], b[bj[mcol]]].sum())
    gaps = ops != 0
    n_gap = int(gaps.sum())
    starts = gaps & np.concatenate([[True], ops[1:] != ops[:-1]])
    return s - n_gap * ext - int(starts.sum()) * open_


def test_long_pairs_workload():
    """The 512-pair long-DNA batch (5-10 kbp, 10 % divergence) under the
    nucleotide stand-in matrix, open 10, extension 1: every alignment scores
    exactly its reported score and de-gaps to the inputs; 48 seeded pairs are
    recomputed by the oracle (12 bytes a cell there), in chunks."""
    M = _msadp()
    d = synth.nw_long()
    P = d["n_pairs"]
    A = M.to_device(d["a_codes"], d["a_offsets"], 4)
    B = M.to_device(d["b_codes"], d["b_offsets"], 4)
    sub = dna_scores()
    sc, ops = M.gotoh(A, B, np.arange(P), np.arange(P), sub, 10, 1)
    sa = synth.from_csr(d["a_codes"], d["a_offsets"])
    sb = synth.from_csr(d["b_codes"], d["b_offsets"])
    for p in range(P):
        o = ops[p]
        assert (o != 2).sum() == len(sa[p]) and (o != 1).sum() == len(sb[p])
        assert _affine_scores_np(sa[p], sb[p], o, sub, 10, 1) == sc[p], p
    pick = np.random.default_rng(6).choice(P, 48, replace=False)
    for c0 in range(0, 48, 8):
        ch = pick[c0:c0 + 8]
        print(f"[gotoh long] oracle pairs {c0}..{c0 + 7}", flush=True)
        ws, wops = orc.gotoh_pairs(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"],
                                   ch, ch, sub, 10, 1)
        for k, p in enumerate(ch):
            assert sc[p] == ws[k] and np.array_equal(ops[p], wops[k]), p
