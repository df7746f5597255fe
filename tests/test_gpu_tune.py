"""Every tunable launch variant gives the oracle's exact results; the
autotuners pick one of them (GPU)."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


@pytest.fixture(autouse=True)
def _clean():
    M = _msadp()
    M.tune_clear()
    yield
    M.tune_clear()


def _long_set(seed, n, lo, hi):
    return synth.random_set(seed, n, lo, hi, 4)


def _condensed_oracle(codes, off):
    n = len(off) - 1
    i, j = np.triu_indices(n, 1)
    return orc.lev_pairs(codes, off, codes, off, i, j)


@pytest.mark.parametrize("wclass", [4, 8, 16, 20, 24, 28, 32])
def test_allpairs_every_class(wclass):
    """Patterns of up to 1700 rows (27 words): classes below that run as
    several passes through the carry buffer."""
    M = _msadp()
    codes, off = _long_set(600 + wclass, 36, 1, 1700)
    S = M.to_device(codes, off, 4)
    words = M.lev_words_bin(S)
    M.tune_set(M.MSA_TUNE_LEV, 4, words, wclass)
    print(f"[tune] allpairs class {wclass} words {words}", flush=True)
    got = M.lev_allpairs(S).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, _condensed_oracle(codes, off))


@pytest.mark.parametrize("wclass", [4, 20, 28])
def test_pair_list_every_class(wclass):
    M = _msadp()
    codes, off = _long_set(700 + wclass, 50, 0, 1500)
    S = M.to_device(codes, off, 4)
    M.tune_set(M.MSA_TUNE_LEV, 4, M.lev_words_bin(S), wclass)
    rng = np.random.default_rng(wclass)
    ia = rng.integers(0, 50, size=300)
    ib = rng.integers(0, 50, size=300)
    print(f"[tune] lev_batch class {wclass}", flush=True)
    got = M.lev_batch(S, S, ia, ib).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, orc.lev_pairs(codes, off, codes, off, ia, ib))


@pytest.mark.parametrize("R", [16, 32, 64])
def test_nw_every_round(R):
    M = _msadp()
    rng = np.random.default_rng(R)
    lens = [1, 33, 2047, 2049, 4100, 5000]
    A = [rng.integers(0, 4, size=L).astype(np.uint8) for L in lens]
    B = [synth.mutate(rng, a, 4, 0.1, 0.02, 0.02) for a in A]
    ca, oa = synth.to_csr(A)
    cb, ob = synth.to_csr(B)
    SA, SB = M.to_device(ca, oa, 4), M.to_device(cb, ob, 4)
    waves = -(-(-(-SA.max_len // 32)) // 64)
    M.tune_set(M.MSA_TUNE_NW, 4, waves, R)
    ia = np.arange(len(A))
    print(f"[tune] nw R={R} waves={waves}", flush=True)
    r = M.nw_batch(SA, SB, ia, ia)
    ops, ops_off, ops_len = M.nw_traceback(SA, SB, r)
    got = M.split_ops(ops, ops_off, ops_len)
    ws, wops = orc.nw_pairs(ca, oa, cb, ob, ia, ia)
    assert np.array_equal(r.score.cpu().numpy().astype(np.int64), ws)
    for p in range(len(A)):
        assert np.array_equal(got[p], wops[p]), p


def test_autotune_lev_and_cache_round_trip():
    M = _msadp()
    codes, off = _long_set(801, 300, 900, 1600)
    S = M.to_device(codes, off, 4)
    best, ms = M.autotune_lev(S, reps=1)
    print(f"[tune] autotune lev -> class {best}, {ms:.3f} ms", flush=True)
    assert best in M.tune_candidates(M.MSA_TUNE_LEV) and ms > 0
    assert M.tune_get(M.MSA_TUNE_LEV, 4, M.lev_words_bin(S)) == best
    text = M.tune_export()
    M.tune_clear()
    M.tune_import(text)
    assert M.tune_get(M.MSA_TUNE_LEV, 4, M.lev_words_bin(S)) == best
    got = M.lev_allpairs(S).cpu().numpy().astype(np.int64)
    i, j = np.triu_indices(300, 1)
    sel = np.random.default_rng(3).choice(len(i), 2000, replace=False)
    want = orc.lev_pairs(codes, off, codes, off, i[sel], j[sel])
    assert np.array_equal(got[sel], want)


def test_autotune_nw():
    M = _msadp()
    rng = np.random.default_rng(9)
    A = [rng.integers(0, 4, size=int(L)).astype(np.uint8) for L in rng.integers(2500, 4500, 24)]
    B = [synth.mutate(rng, a, 4, 0.1, 0.02, 0.02) for a in A]
    ca, oa = synth.to_csr(A)
    cb, ob = synth.to_csr(B)
    SA, SB = M.to_device(ca, oa, 4), M.to_device(cb, ob, 4)
    ia = np.arange(len(A))
    nb = M.NwBatch(SA, SB, ia, ia)
    best, ms = M.autotune_nw(nb, reps=1)
    print(f"[tune] autotune nw -> R {best}, {ms:.3f} ms", flush=True)
    assert best in (16, 32, 64) and ms > 0
    ws, _ = orc.nw_pairs(ca, oa, cb, ob, ia, ia)
    assert np.array_equal(nb.r.score.cpu().numpy().astype(np.int64), ws)


def _tree_matches_oracle(got, codes, off, want=None):
    want = orc.tree(codes, off) if want is None else want
    assert got["n_nodes"] == want["n_nodes"]
    for f in orc.TREE_FIELDS:
        assert np.array_equal(got[f].astype(np.int64), want[f].astype(np.int64)), f
    assert np.array_equal(got["perm"], want["perm"])


@pytest.mark.parametrize("wclass", [4, 8, 16, 20, 24, 32])
def test_tree_every_class(wclass):
    """Lengths 40-500 (8 words): every tree class is admissible; class 4
    runs two passes through the carry buffer."""
    M = _msadp()
    codes, off = _long_set(900 + wclass, 70, 40, 500)
    S = M.to_device(codes, off, 4)
    M.tune_set(M.MSA_TUNE_TREE, 4, M.lev_words_bin(S), wclass)
    print(f"[tune] tree class {wclass}", flush=True)
    got = M.tree_build(S, use_graph=(wclass % 16 == 0))
    _tree_matches_oracle(got, codes, off)


@pytest.mark.parametrize("wclass", [4, 16, 20, 24])
def test_tree_long_patterns_classes(wclass):
    """Lengths 40-1700 (27 words): 16 and 24 take two passes; 4 would take
    seven and is ignored (the default runs)."""
    M = _msadp()
    codes, off = _long_set(950 + wclass, 48, 40, 1700)
    S = M.to_device(codes, off, 4)
    M.tune_set(M.MSA_TUNE_TREE, 4, M.lev_words_bin(S), wclass)
    print(f"[tune] tree long class {wclass}", flush=True)
    _tree_matches_oracle(M.tree_build(S), codes, off)


def test_pruned_tree_tuned_class():
    M = _msadp()
    import torch
    codes, off = _long_set(990, 60, 40, 1700)
    n = len(off) - 1
    S = M.to_device(codes, off, 4)
    M.tune_set(M.MSA_TUNE_TREE, 4, M.lev_words_bin(S), 16)
    emb = np.random.default_rng(990).standard_normal((n, 128)).astype(np.float32)
    demb = torch.from_numpy(emb).to(S.codes.device)
    print("[tune] pruned tree, class 16", flush=True)
    got = M.tree_build(S, emb=demb, topk=4, exact_below=8, emb_offset=0.25)
    want = orc.tree_pruned(codes, off, emb, topk=4, exact_below=8,
                           emb_q0=M.emb_offset_q(0.25))
    _tree_matches_oracle(got, codes, off, want)


def test_autotune_tree():
    M = _msadp()
    codes, off = _long_set(995, 120, 40, 1700)
    S = M.to_device(codes, off, 4)
    best, ms = M.autotune_tree(S, reps=1)
    print(f"[tune] autotune tree -> class {best}, {ms:.3f} ms", flush=True)
    assert best in (16, 20, 24, 32) and ms > 0
    assert M.tune_get(M.MSA_TUNE_TREE, 4, M.lev_words_bin(S)) == best
    _tree_matches_oracle(M.tree_build(S, use_graph=True), codes, off)
