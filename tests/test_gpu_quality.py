"""Alignment-quality metrics on the GPU (msa_pair_counts, msa_quality)
against the CPU oracle: counts bit-exact, metrics to 1e-12 relative (the
sums run in another order), min / max exact."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _random_msa(rows, width, gap, seed, gap_frac=0.4):
    """Seeded rows of residue codes [0, gap) with about gap_frac gaps."""
    rng = np.random.default_rng(seed)
    msa = rng.integers(0, max(gap, 1), size=(rows, width), dtype=np.int64).astype(np.uint8)
    msa[rng.random((rows, width)) < gap_frac] = gap
    return msa


def _check_metrics(got, want):
    for f in ("pct_gaps", "p_avg", "distortion", "stretch"):
        assert got[f] == pytest.approx(want[f], rel=1e-12, abs=1e-300), f
    for f in ("p_min", "p_max", "n_p_pairs", "n_d_pairs"):
        assert got[f] == want[f], f


@pytest.mark.parametrize("rows,width,gap", [
    (2, 1, 4), (5, 31, 4), (65, 32, 4), (66, 33, 4), (130, 100, 20), (67, 1000, 4),
    (40, 257, 1), (33, 95, 63), (3, 0, 4), (1, 50, 4),
])
def test_counts_and_metrics_random(rows, width, gap):
    M = _msadp()
    msa = _random_msa(rows, width, gap, seed=rows * 1000 + width + gap)
    Q = M.Quality(msa, gap)
    h, al, mm = (t.cpu().numpy() for t in Q.pair_counts())
    ia, ib = np.triu_indices(rows, 1)
    wh, wal, wmm = orc.msa_pair_counts(msa, gap, ia, ib)
    assert np.array_equal(h, wh) and np.array_equal(al, wal) and np.array_equal(mm, wmm)
    # explicit pairs, both orders and repeats
    rng = np.random.default_rng(rows + width)
    xa = rng.integers(0, rows, size=300)
    xb = rng.integers(0, rows, size=300)
    lh, lal, lmm = (t.cpu().numpy() for t in Q.pair_counts(xa, xb))
    wh2, wal2, wmm2 = orc.msa_pair_counts(msa, gap, xa, xb)
    assert np.array_equal(lh, wh2) and np.array_equal(lal, wal2) and np.array_equal(lmm, wmm2)
    # metrics with stand-in distances (any positive uint16 works for the sums)
    lev = rng.integers(0, 40, size=len(ia)).astype(np.uint16)
    import torch
    counts = Q.pair_counts()
    got = Q.metrics(counts, max_len=max(1, width), lev=torch.from_numpy(lev).cuda())
    want = orc.msa_quality(msa, gap, max(1, width), ia, ib, lev)
    _check_metrics(got, want)
    again = Q.metrics(counts, max_len=max(1, width), lev=torch.from_numpy(lev).cuda())
    assert again == got                                      # fixed summation order


def test_merged_alignment_with_device_distances():
    # the whole path on the small set: tree, merge, all-pairs distances,
    # counts and metrics; every pair's Hamming distance bounds its
    # Levenshtein distance from above
    M = _msadp()
    d = synth.tiny()
    A = M.to_device(d["codes"], d["offsets"], d["sigma"])
    tree, msa = M.align(A)
    lev = M.lev_allpairs(A)
    Q = M.Quality(msa, d["sigma"])
    counts = Q.pair_counts()
    max_len = int(np.diff(d["offsets"]).max())
    got = Q.metrics(counts, max_len=max_len, lev=lev)
    n = d["n"]
    ia, ib = np.triu_indices(n, 1)
    wlev = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
    assert np.array_equal(lev.cpu().numpy().astype(np.int64), wlev)
    want = orc.msa_quality(msa, d["sigma"], max_len, ia, ib, wlev)
    _check_metrics(got, want)
    assert (counts[0].cpu().numpy() >= wlev).all()
    assert got["distortion"] >= 1.0


def test_symbol_above_gap_reported():
    M = _msadp()
    msa = _random_msa(10, 40, 4, seed=1)
    msa[3, 7] = 9
    Q = M.Quality(msa, 4)
    counts = Q.pair_counts()
    with pytest.raises(RuntimeError, match="symbol"):
        Q.metrics(counts, max_len=40)


def test_pair_index_out_of_range_reported():
    M = _msadp()
    msa = _random_msa(10, 40, 4, seed=2)
    Q = M.Quality(msa, 4)
    counts = Q.pair_counts([0, 3, 10], [1, 2, 4])
    import torch
    torch.cuda.synchronize()
    with pytest.raises(RuntimeError, match="index"):
        Q.st.check("msa_pair_counts")
    del counts


def test_full_size_alignment_of_the_4096_set():
    # the configuration the bench times: the 4096-sequence set aligned on the
    # device, all 8,386,560 row pairs; counts checked on a seeded sample,
    # metrics against the oracle over every pair (same distances as input)
    import torch
    M = _msadp()
    d = synth.allpairs()
    n = d["n"]
    A = M.to_device(d["codes"], d["offsets"], d["sigma"])
    _, msa = M.align(A, use_graph=True)
    lev = M.lev_allpairs(A)
    Q = M.Quality(msa, d["sigma"])
    counts = Q.pair_counts()
    max_len = int(np.diff(d["offsets"]).max())
    got = Q.metrics(counts, max_len, lev=lev)
    host = [t.cpu().numpy() for t in counts]
    rng = np.random.default_rng(31)
    ia = rng.integers(0, n, size=20000)
    ib = rng.integers(0, n, size=20000)
    keep = ia != ib
    i, j = np.minimum(ia[keep], ib[keep]), np.maximum(ia[keep], ib[keep])
    c = i * n - i * (i + 1) // 2 + (j - i - 1)
    want = orc.msa_pair_counts(msa, d["sigma"], i, j)
    for g, w in zip(host, want):
        assert np.array_equal(g[c], w)
    ti, tj = np.triu_indices(n, 1)
    wq = orc.msa_quality(msa, d["sigma"], max_len, ti, tj, lev.cpu().numpy())
    _check_metrics(got, wq)
    assert (host[0] >= lev.cpu().numpy()).all()
    torch.cuda.synchronize()
