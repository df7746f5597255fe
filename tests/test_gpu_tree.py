"""Alg. 1 guide tree on the GPU against the CPU oracle (node arrays equal)."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _compare(codes, off, sigma, use_graph=False):
    M = _msadp()
    n = len(off) - 1
    print(f"[tree] n={n} sigma={sigma} graph={use_graph}: device build", flush=True)
    S = M.to_device(codes, off, sigma)
    got = M.tree_build(S, use_graph=use_graph)
    print(f"[tree] device build done ({got['n_nodes']} nodes); oracle", flush=True)
    want = orc.tree(codes, off)
    assert got["n_nodes"] == want["n_nodes"]
    for f in orc.TREE_FIELDS:
        g = got[f].astype(np.int64)
        w = want[f].astype(np.int64)
        bad = np.flatnonzero(g != w)
        assert len(bad) == 0, (f, bad[:5], g[bad[:5]], w[bad[:5]])
    # members of a multi-member leaf (copies of one sequence) may come in
    # any order; everything else is fixed by the tree
    gp, wp = got["perm"].copy(), want["perm"].copy()
    for v in range(want["n_nodes"]):
        if want["left"][v] < 0 and want["mcount"][v] > 1:
            a, k = want["mstart"][v], want["mcount"][v]
            gp[a:a + k].sort()
            wp[a:a + k].sort()
    assert np.array_equal(gp, wp)
    return got


def test_hand_worked_inputs():
    for strs in (["A", "C", "G"], ["AAAA", "AAAC", "AACC", "CCCC"], ["AC", "ACG", "G"]):
        seqs = [np.array(["ACGT".index(c) for c in s], dtype=np.uint8) for s in strs]
        codes, off = synth.to_csr(seqs)
        _compare(codes, off, 4)


def test_tiny_workload_tree():
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"])


def test_tiny_workload_tree_graph_replay():
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], use_graph=True)


def test_protein_subset_tree():
    d = synth.protein_tree()
    rng = np.random.default_rng(33)
    sub = synth.subset(d, rng.choice(d["n"], size=300, replace=False))
    _compare(sub["codes"], sub["offsets"], 20, use_graph=True)


def test_random_ragged_and_single():
    codes, off = synth.random_set(41, 150, 1, 90, 4)
    _compare(codes, off, 4)
    codes, off = synth.to_csr([np.array([1, 2, 3], np.uint8)])
    got = _compare(codes, off, 4)
    assert got["n_nodes"] == 1


def test_duplicates_leaf():
    seqs = [np.array([0, 1, 2, 3], np.uint8)] * 3 + [np.array([3, 3], np.uint8)]
    codes, off = synth.to_csr(seqs)
    _compare(codes, off, 4)


def _check_msa(codes, off, sigma, use_graph=False):
    M = _msadp()
    n = len(off) - 1
    print(f"[merge] n={n} sigma={sigma}: device tree + merge", flush=True)
    S = M.to_device(codes, off, sigma)
    tree, msa = M.align(S, use_graph=use_graph)
    print(f"[merge] device done, width {msa.shape[1]}; oracle", flush=True)
    want_tree = orc.tree(codes, off)
    want = orc.merge(codes, off, sigma, want_tree)
    assert msa.shape == want.shape, (msa.shape, want.shape)
    bad = np.argwhere(msa != want)
    assert len(bad) == 0, bad[:5]


def test_tiny_workload_alignment_byte_equal():
    d = synth.tiny()
    _check_msa(d["codes"], d["offsets"], d["sigma"])


def test_hand_worked_alignment():
    seqs = [np.array(["ACGT".index(c) for c in s], dtype=np.uint8) for s in ["AC", "ACG", "G"]]
    codes, off = synth.to_csr(seqs)
    _check_msa(codes, off, 4)


def test_protein_subset_alignment():
    d = synth.protein_tree()
    rng = np.random.default_rng(34)
    sub = synth.subset(d, rng.choice(d["n"], size=150, replace=False))
    _check_msa(sub["codes"], sub["offsets"], 20, use_graph=True)
