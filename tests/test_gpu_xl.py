"""Tree passes with a pair's pattern words spread across lanes (k_tree_xl).

Every variant of the across-lanes passes (words per lane, cluster-size caps,
group widths from 1 to 32 lanes, DNA and protein alphabets) builds the same
tree as the CPU oracle, node for node, in the exact, sampled and learned
(embedding-ranked) builds; the caps move work between the one-pattern-per-
wavefront kernel and the across-lanes one without changing any result."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth
from test_gpu_pruned import _emb, _equal_trees

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _words(off):
    return max(1, (int(np.diff(off).max()) + 63) // 64)


def _with_xl(sigma, off, value, fn):
    M = _msadp()
    M.tune_clear()
    try:
        M.tune_set(M.MSA_TUNE_TREE_XL, sigma, _words(off), value)
        return fn()
    finally:
        M.tune_clear()


VARIANTS = [  # (words per lane, sum cap, pole cap)
    (1, 0, 0), (1, 0, 16383), (1, 64, 16383), (2, 64, 16383), (1, 16383, 16383),
    (2, 16383, 16383), (1, 5, 3), (2, 40, 0),
]


def _exact(codes, off, sigma, v, use_graph=False):
    M = _msadp()
    print(f"[xl] exact n={len(off) - 1} sigma={sigma} variant={v} graph={use_graph}", flush=True)
    S = M.to_device(codes, off, sigma)
    got = _with_xl(sigma, off, M.xl_value(*v), lambda: M.tree_build(S, use_graph=use_graph))
    _equal_trees(got, orc.tree(codes, off))


@pytest.mark.parametrize("v", VARIANTS)
def test_exact_tree_dna_ragged(v):
    """Lengths 0-300 (up to 5 pattern words: groups of 8 or 4 lanes), an
    empty sequence, copies."""
    codes, off = synth.random_set(71, 160, 0, 300, 4)
    seqs = synth.from_csr(codes, off)
    seqs += [seqs[5].copy(), seqs[5].copy(), np.zeros(0, np.uint8), seqs[9][:64].copy()]
    c2, o2 = synth.to_csr(seqs)
    _exact(c2, o2, 4, v)


@pytest.mark.parametrize("v", [(1, 16383, 16383), (2, 64, 16383)])
def test_exact_tree_word_boundaries(v):
    """Lengths at and around multiples of 64 (the last row at bit 63 or 0 of
    its word; a pattern that fills its group exactly)."""
    rng = np.random.default_rng(72)
    lens = [1, 63, 64, 65, 127, 128, 129, 191, 192, 255, 256, 257] * 5
    seqs = [rng.integers(0, 4, size=L).astype(np.uint8) for L in lens]
    codes, off = synth.to_csr(seqs)
    _exact(codes, off, 4, v)


@pytest.mark.parametrize("v", [(1, 16383, 16383), (2, 16383, 16383), (1, 64, 16383)])
def test_exact_tree_protein_subset(v):
    """300 proteins of 50-2000 residues: 5 bit planes, groups of 32 (one
    word per lane) or 16 lanes (two)."""
    d = synth.protein_tree()
    rng = np.random.default_rng(73)
    sub = synth.subset(d, rng.choice(d["n"], size=300, replace=False))
    _exact(sub["codes"], sub["offsets"], 20, v)


def test_exact_tree_short_sequences_one_lane_groups():
    """Every sequence within one word: groups of one lane (no carries)."""
    codes, off = synth.random_set(74, 200, 0, 64, 4)
    _exact(codes, off, 4, (1, 16383, 16383))
    codes, off = synth.random_set(75, 120, 1, 128, 20)
    _exact(codes, off, 20, (2, 16383, 16383))    # two words in one lane


def test_exact_tree_graph_replay():
    d = synth.tiny()
    _exact(d["codes"], d["offsets"], d["sigma"], (1, 16383, 16383), use_graph=True)


@pytest.mark.parametrize("v", [(1, 16383, 16383), (2, 32, 16383), (1, 8, 0)])
def test_sampled_tree(v):
    M = _msadp()
    codes, off = synth.random_set(76, 400, 20, 260, 4)
    S = M.to_device(codes, off, 4)
    print(f"[xl] sampled variant={v}", flush=True)
    got = _with_xl(4, off, M.xl_value(*v),
                   lambda: M.tree_build(S, use_graph=True, pivots=8, topk=6))
    _equal_trees(got, orc.tree_sampled(codes, off, pivots=8, topk=6))


@pytest.mark.parametrize("v", [(1, 16383, 16383), (2, 64, 16383)])
def test_learned_tree(v):
    import torch
    M = _msadp()
    codes, off = synth.random_set(77, 300, 10, 200, 4)
    emb = _emb(78, 300)
    S = M.to_device(codes, off, 4)
    e = torch.from_numpy(emb).to(S.codes.device)
    print(f"[xl] learned variant={v}", flush=True)
    got = _with_xl(4, off, M.xl_value(*v), lambda: M.tree_build(S, emb=e, topk=5))
    _equal_trees(got, orc.tree_pruned(codes, off, emb, topk=5, emb_q0=M.emb_offset_q(0.0)))


def test_teacher_forced_centres_equal_across_variants():
    """tree_eval_centers replays the passes on a given tree: equal choices
    with the across-lanes passes on and off."""
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    t = M.tree_build(S)
    off = d["offsets"]
    a = _with_xl(4, off, M.xl_value(1, 0, 0),
                 lambda: M.tree_eval_centers(S, t, pivots=4, topk=3))
    b = _with_xl(4, off, M.xl_value(1, 16383, 16383),
                 lambda: M.tree_eval_centers(S, t, pivots=4, topk=3))
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_tune_value_validation():
    M = _msadp()
    M.tune_clear()
    try:
        for bad in (0, -1, 3 << 28, (3 << 28) | 5):
            with pytest.raises(M.MsaError):
                M.tune_set(M.MSA_TUNE_TREE_XL, 4, 2, bad)
        M.tune_set(M.MSA_TUNE_TREE_XL, 4, 2, M.xl_value(2, 16383, 0))
        assert M.tune_get(M.MSA_TUNE_TREE_XL, 4, 2) == M.xl_value(2, 16383, 0)
        assert len(M.tune_candidates(M.MSA_TUNE_TREE_XL)) >= 4
    finally:
        M.tune_clear()


def test_autotune_tree_xl_stores_a_candidate():
    """The tuner times every candidate on a sampled build, stores the fastest
    and a build under it equals the oracle's tree."""
    M = _msadp()
    codes, off = synth.random_set(79, 600, 50, 400, 4)
    S = M.to_device(codes, off, 4)
    M.tune_clear()
    try:
        best, ms = M.autotune_tree_xl(S, pivots=8, topk=8)
        print(f"[xl] tuned {M.xl_describe(best)} ({ms:.1f} ms)", flush=True)
        assert best in M.tune_candidates(M.MSA_TUNE_TREE_XL) and ms > 0
        assert M.tune_get(M.MSA_TUNE_TREE_XL, 4, _words(off)) == best
        got = M.tree_build(S, use_graph=True, pivots=8, topk=8)
    finally:
        M.tune_clear()
    _equal_trees(got, orc.tree_sampled(codes, off, pivots=8, topk=8))


@pytest.mark.parametrize("v", [(1, 0, 0), (2, 128, 16383), (2, 16383, 16383)])
def test_all_candidate_clusters_take_the_triangle(v):
    """Clusters of at most exact_below members take every member as a
    candidate; their candidate pass runs as the medoid triangle in both
    kernels (clusters of 129-300 members in the one-pattern-per-wavefront
    kernel under the default caps, every cluster in it with the across-lanes
    passes off, every cluster across lanes with caps for all)."""
    M = _msadp()
    codes, off = synth.random_set(80, 600, 20, 260, 4)
    S = M.to_device(codes, off, 4)
    print(f"[xl] all-candidate clusters variant={v}", flush=True)
    got = _with_xl(4, off, M.xl_value(*v),
                   lambda: M.tree_build(S, use_graph=True, pivots=8, topk=4, exact_below=300))
    _equal_trees(got, orc.tree_sampled(codes, off, pivots=8, topk=4, exact_below=300))
