"""Exact banded Levenshtein (lev_band) against the CPU oracle: every distance
up to kmax equal to Wagner-Fischer's, and 0xFFFF exactly for the pairs above."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _check(ca, oa, cb, ob, sigma, ia, ib, k0, kmax):
    M = _msadp()
    A = M.to_device(ca, oa, sigma)
    B = M.to_device(cb, ob, sigma)
    print(f"[band] {len(ia)} pairs k0={k0} kmax={kmax}", flush=True)
    got, ku = M.lev_band(A, B, ia, ib, k0, kmax)
    got = got.cpu().numpy().astype(np.int64)
    ku = ku.cpu().numpy()
    want = orc.lev_pairs(ca, oa, cb, ob, ia, ib)
    exp = np.where(want <= kmax, want, M.BAND_NONE)
    bad = np.flatnonzero(got != exp)
    assert len(bad) == 0, (bad[:5], got[bad[:5]], exp[bad[:5]])
    ok = want <= kmax
    # the verifying threshold covers the distance and |m - n|
    assert (ku[ok] >= want[ok]).all() and (ku[~ok] == -1).all()
    return got, ku, want


def test_related_pairs_around_word_and_cycle_boundaries():
    """Pattern lengths around 64-row words and around 64 words (the lanes
    take a second word), related texts with indels and unrelated ones."""
    rng = np.random.default_rng(1)
    seqs_a, seqs_b = [], []
    for L in [1, 2, 63, 64, 65, 127, 128, 129, 1000, 4095, 4096, 4097, 4160, 5000, 9000]:
        a = rng.integers(0, 4, size=L).astype(np.uint8)
        for d in (0.0, 0.02, 0.1, 0.3):
            seqs_a.append(a)
            seqs_b.append(synth.mutate(rng, a, 4, 0.8 * d, 0.1 * d, 0.1 * d))
        seqs_a.append(a)
        seqs_b.append(rng.integers(0, 4, size=int(rng.integers(1, 2 * L + 2))).astype(np.uint8))
    ca, oa = synth.to_csr(seqs_a)
    cb, ob = synth.to_csr(seqs_b)
    P = len(seqs_a)
    _check(ca, oa, cb, ob, 4, np.arange(P), np.arange(P), 64, 4000)


@pytest.mark.parametrize("k0,kmax", [(1, 4000), (8, 100), (1000, 1000), (3000, 4000)])
def test_threshold_doubling_and_cap(k0, kmax):
    """From tiny starting bands (many doublings) to a fixed band; pairs above
    kmax come back as 0xFFFF."""
    rng = np.random.default_rng(2 + k0)
    seqs_a, seqs_b = [], []
    for _ in range(60):
        L = int(rng.integers(0, 3000))
        a = rng.integers(0, 4, size=L).astype(np.uint8)
        d = float(rng.choice([0.0, 0.01, 0.05, 0.2, 0.6]))
        seqs_a.append(a)
        seqs_b.append(synth.mutate(rng, a, 4, 0.8 * d, 0.1 * d, 0.1 * d))
    ca, oa = synth.to_csr(seqs_a)
    cb, ob = synth.to_csr(seqs_b)
    _check(ca, oa, cb, ob, 4, np.arange(60), np.arange(60), k0, kmax)


@pytest.mark.parametrize("sigma", [2, 20, 32])
def test_alphabets_and_empty(sigma):
    codes, off = synth.random_set(30 + sigma, 80, 0, 600, sigma)
    rng = np.random.default_rng(sigma)
    ia, ib = rng.integers(0, 80, 400), rng.integers(0, 80, 400)
    _check(codes, off, codes, off, sigma, ia, ib, 16, 4000)


def test_long_pairs_workload_all_pairs():
    """The 512-pair long-DNA batch (5-10 kbp, 10 % divergence): every
    distance equal to Wagner-Fischer's, all verified inside the band."""
    d = synth.nw_long()
    P = d["n_pairs"]
    got, ku, want = _check(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"], 4,
                           np.arange(P), np.arange(P), 1024, 4000)
    assert (got == want).all()


def test_device_index_error():
    M = _msadp()
    codes, off = synth.random_set(40, 10, 5, 50, 4)
    A = M.to_device(codes, off, 4)
    with pytest.raises(RuntimeError, match="index"):
        M.lev_band(A, A, [0], [10])
    with pytest.raises(M.MsaError) as e:
        M.lev_band(A, A, [0], [1], 10, 5000)
    assert e.value.code == M.MSA_EINVAL
