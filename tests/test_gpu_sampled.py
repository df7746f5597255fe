"""Sampled-median Alg. 1 on the GPU (tree_build_sampled) against the oracle.

Pivots come from a hash of the input index and every estimate is a sum of
exact distances, so the device tree equals the oracle's node for node."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth
from test_gpu_pruned import _equal_trees

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _compare(codes, off, sigma, pivots, topk, exact_below=0, use_graph=False):
    M = _msadp()
    n = len(off) - 1
    print(f"[sampled] n={n} sigma={sigma} pivots={pivots} topk={topk} "
          f"exact_below={exact_below} graph={use_graph}", flush=True)
    S = M.to_device(codes, off, sigma)
    got = M.tree_build(S, use_graph=use_graph, pivots=pivots, topk=topk,
                       exact_below=exact_below)
    want = orc.tree_sampled(codes, off, pivots=pivots, topk=topk, exact_below=exact_below)
    _equal_trees(got, want)
    return got


@pytest.mark.parametrize("pivots,topk,exact_below", [(1, 1, 0), (4, 4, 0), (8, 16, 0),
                                                     (3, 2, 20), (64, 8, 0), (300, 4, 0)])
def test_tiny_workload(pivots, topk, exact_below):
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], pivots, topk, exact_below)


def test_tiny_workload_graph_replay():
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], 8, 4, use_graph=True)


def test_protein_subset():
    d = synth.protein_tree()
    rng = np.random.default_rng(51)
    sub = synth.subset(d, rng.choice(d["n"], size=600, replace=False))
    _compare(sub["codes"], sub["offsets"], 20, 8, 16)


def test_ragged_single_and_duplicates():
    rng = np.random.default_rng(52)
    seqs = [rng.integers(0, 4, size=int(rng.integers(0, 140))).astype(np.uint8)
            for _ in range(90)]
    seqs += [seqs[3].copy(), seqs[3].copy(), np.zeros(0, np.uint8)]
    codes, off = synth.to_csr(seqs)
    _compare(codes, off, 4, 5, 3)
    one_c, one_o = synth.to_csr(seqs[:1])
    _compare(one_c, one_o, 4, 5, 3)


def test_enough_pivots_equals_exact_device_tree():
    """Pivots covering every cluster make the estimate the exact row sum:
    the device's sampled tree is its exact tree."""
    M = _msadp()
    d = synth.protein_tree()
    rng = np.random.default_rng(53)
    sub = synth.subset(d, rng.choice(d["n"], size=400, replace=False))
    S = M.to_device(sub["codes"], sub["offsets"], 20)
    exact = M.tree_build(S)
    got = M.tree_build(S, pivots=400, topk=1)
    _equal_trees(got, exact)


def test_teacher_forced_sampled_matches_oracle():
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    t = M.tree_build(S)
    for pivots, topk, eb in ((2, 1, 0), (8, 4, 0), (4, 2, 12)):
        c, l, r = M.tree_eval_centers(S, t, pivots=pivots, topk=topk, exact_below=eb)
        for v in range(t["n_nodes"]):
            C = t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]]
            want = orc.select(d["codes"], d["offsets"], C, topk=topk, exact_below=eb,
                              pivots=pivots)
            assert (int(c[v]), int(l[v]), int(r[v])) == want, (pivots, topk, eb, v)


def test_bad_arguments():
    import ctypes as C
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    for pivots, topk, eb in ((2000, 4, 0), (4, 0, 0), (4, 2000, 0), (4, 4, -1)):
        with pytest.raises(M.MsaError) as ex:
            M.tree_build(S, pivots=pivots, topk=topk, exact_below=eb)
        assert ex.value.code == M.MSA_EINVAL
    # no pivots at all, straight through the C-ABI
    tb = M.TreeBuilder(S)
    nn = C.c_int32(0)
    rc = M.lib().tree_build_sampled(C.byref(tb.ss), 0, 4, 0, C.byref(tb.ts), C.byref(nn), 0,
                                    M._ptr(tb.ws), tb.wsb, M._ptr(tb.st.t), None)
    assert rc == M.MSA_EINVAL


def test_learned_workload_full_size_sampled_nodes():
    """The 100,000-sequence DNA set at full size with 8 pivots and 16
    candidates: the whole tree's shape; the root's poles and split from
    oracle distances to the chosen centre; sampled nodes of 20-200 members
    re-derived by the oracle's sampled Alg. 1 step on their member sets."""
    from test_gpu_tree import _check_structure, _dist_from
    M = _msadp()
    d = synth.learned()
    codes, off, n = d["codes"], d["offsets"], d["n"]
    S = M.to_device(codes, off, d["sigma"])
    print(f"[sampled] learned {n}: device build", flush=True)
    t = M.tree_build(S, use_graph=True, pivots=8, topk=16)
    print(f"[sampled] {t['n_nodes']} nodes; shape", flush=True)
    _check_structure(t, codes, off)
    allm = np.arange(n)
    c, l, r = int(t["center"][0]), int(t["lpole"][0]), int(t["rpole"][0])
    dc = _dist_from(codes, off, c, allm)
    assert l == int(np.argmax(dc))
    dl = _dist_from(codes, off, l, allm)
    assert r == int(np.argmax(dl))
    dr = _dist_from(codes, off, r, allm)
    lc = int(t["left"][0])
    in_left = np.zeros(n, bool)
    in_left[t["perm"][t["mstart"][lc]: t["mstart"][lc] + t["mcount"][lc]]] = True
    assert np.array_equal(in_left, dl <= dr)
    rng = np.random.default_rng(54)
    internal = np.flatnonzero((t["left"] >= 0) & (t["mcount"] >= 20) & (t["mcount"] <= 200))
    for v in rng.choice(internal, size=min(12, len(internal)), replace=False):
        mem = t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]]
        print(f"[sampled] node {v} ({len(mem)} members) against the oracle", flush=True)
        want = orc.select(codes, off, mem, topk=16, pivots=8)
        assert (int(t["center"][v]), int(t["lpole"][v]), int(t["rpole"][v])) == want, v
