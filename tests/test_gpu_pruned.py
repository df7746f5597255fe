"""Surrogate-pruned Alg. 1 on the GPU against the CPU oracle (node arrays equal).

The candidate ranking takes the same steps on both sides (int8 codes, exact
integer squared distances, one float32 square root and rounding), so the
pruned tree is reproduced exactly, not approximately."""
import numpy as np
import pytest

from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def _emb(seed, n, scale=0.1):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, 128)) * scale).astype(np.float32)


def _equal_trees(got, want):
    assert got["n_nodes"] == want["n_nodes"]
    for f in orc.TREE_FIELDS:
        g = got[f].astype(np.int64)
        w = want[f].astype(np.int64)
        bad = np.flatnonzero(g != w)
        assert len(bad) == 0, (f, bad[:5], g[bad[:5]], w[bad[:5]])
    gp, wp = got["perm"].copy(), want["perm"].copy()
    for v in range(want["n_nodes"]):
        if want["left"][v] < 0 and want["mcount"][v] > 1:
            a, k = want["mstart"][v], want["mcount"][v]
            gp[a:a + k].sort()
            wp[a:a + k].sort()
    assert np.array_equal(gp, wp)


def _compare(codes, off, sigma, emb, topk, use_graph=False, exact_below=0, emb_offset=0.0):
    import torch
    M = _msadp()
    n = len(off) - 1
    print(f"[pruned] n={n} sigma={sigma} topk={topk} exact_below={exact_below} "
          f"graph={use_graph}: device", flush=True)
    S = M.to_device(codes, off, sigma)
    e = torch.from_numpy(emb).to(S.codes.device)
    got = M.tree_build(S, use_graph=use_graph, emb=e, topk=topk, exact_below=exact_below,
                       emb_offset=emb_offset)
    print(f"[pruned] device done ({got['n_nodes']} nodes); oracle", flush=True)
    want = orc.tree_pruned(codes, off, emb, topk=topk, exact_below=exact_below,
                           emb_q0=M.emb_offset_q(emb_offset))
    _equal_trees(got, want)
    return got


@pytest.mark.parametrize("topk", [1, 4, 16])
def test_tiny_workload(topk):
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], _emb(20 + topk, d["n"]), topk)


@pytest.mark.parametrize("topk,exact_below", [(2, 12), (40, 0), (3, 70)])
def test_exact_below_and_large_topk(topk, exact_below):
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], _emb(40 + topk, d["n"]), topk,
             exact_below=exact_below)


@pytest.mark.parametrize("topk", [96, 256, 300])
def test_larger_candidate_lists(topk):
    """Candidate lists up to the thread count take the threshold selection,
    above it the round-by-round one; both give the oracle's candidates."""
    codes, off = synth.random_set(500 + topk, 900, 20, 120, 4)
    n = len(off) - 1
    _compare(codes, off, 4, _emb(44 + topk, n, 0.5), topk, emb_offset=0.75)


@pytest.mark.parametrize("offset", [0.3, 7.5])
def test_calibration_offset(offset):
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], _emb(50, d["n"]), 4, emb_offset=offset)
    codes, off = synth.random_set(51, 120, 1, 80, 4)
    _compare(codes, off, 4, _emb(52, 120, scale=0.3), 3, exact_below=9, emb_offset=offset)


def test_tiny_workload_graph_replay():
    d = synth.tiny()
    _compare(d["codes"], d["offsets"], d["sigma"], _emb(30, d["n"]), 8, use_graph=True)


def test_protein_subset():
    d = synth.protein_tree()
    rng = np.random.default_rng(35)
    sub = synth.subset(d, rng.choice(d["n"], size=300, replace=False))
    _compare(sub["codes"], sub["offsets"], 20, _emb(31, 300, scale=0.5), 16, use_graph=True)


def test_ragged_single_and_duplicates():
    codes, off = synth.random_set(42, 150, 1, 90, 4)
    _compare(codes, off, 4, _emb(32, 150), 2)
    codes, off = synth.to_csr([np.array([1, 2, 3], np.uint8)])
    assert _compare(codes, off, 4, _emb(33, 1), 16)["n_nodes"] == 1
    seqs = [np.array([0, 1, 2, 3], np.uint8)] * 3 + [np.array([3, 3], np.uint8)]
    codes, off = synth.to_csr(seqs)
    _compare(codes, off, 4, _emb(34, 4), 1)


def test_equal_estimates_and_ties():
    """All-equal embeddings (every estimate 0): lowest indices are the candidates."""
    codes, off = synth.random_set(43, 80, 10, 60, 4)
    _compare(codes, off, 4, np.zeros((80, 128), np.float32), 3)


def test_full_candidates_equal_exact_device_tree():
    """n <= topk: every cluster's candidates are all its members, so the
    pruned build is the exact one."""
    import torch
    M = _msadp()
    d = synth.tiny()
    sub = synth.subset(d, np.arange(32))
    S = M.to_device(sub["codes"], sub["offsets"], 4)
    exact = M.tree_build(S)
    pruned = M.tree_build(S, emb=torch.from_numpy(_emb(36, 32)).to(S.codes.device), topk=32)
    _equal_trees(pruned, exact)


def test_device_embeddings_pipeline():
    """Embeddings from the device CNN feed the pruned build; the oracle gets
    the same embeddings."""
    from oracle import cnn_ref as ref
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    E = M.Embedder()
    E.set_params(ref.init_params(5, sigma=4, width=128, layers=4))
    e = E.embed(S)
    got = M.tree_build(S, emb=e, topk=4)
    want = orc.tree_pruned(d["codes"], d["offsets"], e.cpu().numpy(), topk=4)
    _equal_trees(got, want)


@pytest.mark.parametrize("scale", [1e-20, 1e-3, 3.0, 1e6, 1e12])
def test_quantization_scales(scale):
    """Every regime of the quantization shift: tiny values (largest shift),
    ordinary ones, and large ones whose shift is limited (codes saturate)."""
    d = synth.tiny()
    emb = (_emb(40, d["n"], 1.0) * np.float32(scale)).astype(np.float32)
    emb[11] *= np.float32(50.0)                # one row far from the rest
    _compare(d["codes"], d["offsets"], d["sigma"], emb, 4)


def test_non_finite_embedding_reported():
    import torch
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    for bad in (np.nan, np.inf):
        emb = _emb(41, d["n"])
        emb[5, 3] = bad
        e = torch.from_numpy(emb).to(S.codes.device)
        with pytest.raises(RuntimeError, match="non-finite"):
            M.tree_build(S, emb=e, topk=4)


def test_bad_arguments():
    import torch
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    e = torch.zeros((d["n"], 128), dtype=torch.float32, device=S.codes.device)
    for k, eb in ((0, 0), (1025, 0), (4, -1)):
        with pytest.raises(M.MsaError) as ex:
            M.tree_build(S, emb=e, topk=k, exact_below=eb)
        assert ex.value.code == M.MSA_EINVAL
    with pytest.raises(ValueError):
        M.tree_build(S, emb=e[:10], topk=4)
    with pytest.raises(ValueError):
        M.tree_build(S, emb=e, topk=4, emb_offset=-1.0)


def test_teacher_forced_exact_reproduces_tree():
    """Evaluating the full median on the clusters of the exact tree gives
    back that tree's own (c, l, r)."""
    M = _msadp()
    d = synth.protein_tree()
    rng = np.random.default_rng(37)
    sub = synth.subset(d, rng.choice(d["n"], size=300, replace=False))
    S = M.to_device(sub["codes"], sub["offsets"], 20)
    t = M.tree_build(S)
    c, l, r = M.tree_eval_centers(S, t)
    assert np.array_equal(c, t["center"]) and np.array_equal(l, t["lpole"])
    assert np.array_equal(r, t["rpole"])


def test_teacher_forced_pruned_matches_oracle():
    """The pruned choice on every cluster of the exact tree, against the
    oracle's choice for the same member set."""
    import torch
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    t = M.tree_build(S)
    emb = _emb(38, d["n"])
    for topk, eb, offset in ((1, 0, 0.0), (5, 0, 0.0), (2, 10, 0.0), (3, 0, 2.25)):
        c, l, r = M.tree_eval_centers(S, t, emb=torch.from_numpy(emb).to(S.codes.device),
                                      topk=topk, exact_below=eb, emb_offset=offset)
        for v in range(t["n_nodes"]):
            C = t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]]
            want = orc.select(d["codes"], d["offsets"], C, emb, topk, eb,
                              emb_q0=M.emb_offset_q(offset))
            assert (int(c[v]), int(l[v]), int(r[v])) == want, (topk, eb, v)


def test_teacher_forced_rejects_bad_tree():
    M = _msadp()
    d = synth.tiny()
    S = M.to_device(d["codes"], d["offsets"], d["sigma"])
    t = M.tree_build(S)
    bad = dict(t)
    bad["mcount"] = t["mcount"].copy()
    bad["mcount"][1] += 1                     # overlaps its sibling
    with pytest.raises(M.MsaError) as ex:
        M.tree_eval_centers(S, bad)
    assert ex.value.code == M.MSA_EINVAL


def test_learned_workload_full_size_sampled():
    """The 100,000-sequence DNA set (1000 families) at full size with a fixed
    random embedding and a calibration offset: the whole tree's shape; the
    root's poles and split from oracle distances to the chosen centre; and
    sampled nodes of 20-200 members re-derived by the oracle's pruned Alg. 1
    step on their member sets (embedding quantized over the whole set)."""
    import torch
    from test_gpu_tree import _check_structure, _dist_from
    M = _msadp()
    d = synth.learned()
    codes, off, n = d["codes"], d["offsets"], d["n"]
    assert n == 100000
    S = M.to_device(codes, off, d["sigma"])
    emb = _emb(42, n, 0.3)
    e = torch.from_numpy(emb).to(S.codes.device)
    print(f"[pruned] learned {n}: device build", flush=True)
    t = M.tree_build(S, use_graph=True, emb=e, topk=16, emb_offset=0.5)
    print(f"[pruned] {t['n_nodes']} nodes; shape", flush=True)
    _check_structure(t, codes, off)
    allm = np.arange(n)
    c, l, r = int(t["center"][0]), int(t["lpole"][0]), int(t["rpole"][0])
    print("[pruned] root poles and split from oracle distances", flush=True)
    dc = _dist_from(codes, off, c, allm)
    assert l == int(np.argmax(dc))
    dl = _dist_from(codes, off, l, allm)
    assert r == int(np.argmax(dl))
    dr = _dist_from(codes, off, r, allm)
    lc = int(t["left"][0])
    in_left = np.zeros(n, bool)
    in_left[t["perm"][t["mstart"][lc]: t["mstart"][lc] + t["mcount"][lc]]] = True
    assert np.array_equal(in_left, dl <= dr)
    rng = np.random.default_rng(43)
    internal = np.flatnonzero((t["left"] >= 0) & (t["mcount"] >= 20) & (t["mcount"] <= 200))
    for v in rng.choice(internal, size=min(12, len(internal)), replace=False):
        mem = t["perm"][t["mstart"][v]: t["mstart"][v] + t["mcount"][v]]
        print(f"[pruned] node {v} ({len(mem)} members) against the oracle", flush=True)
        want = orc.select(codes, off, mem, emb, 16, 0, emb_q0=M.emb_offset_q(0.5))
        assert (int(t["center"][v]), int(t["lpole"][v]), int(t["rpole"][v])) == want, v


def test_every_member_a_candidate_on_a_large_cluster():
    """topk covering a 400-member root: the candidate pass then holds every
    member against every member (more work items than the medoid triangle),
    and the tree is the exact one."""
    import torch
    M = _msadp()
    d = synth.protein_tree()
    rng = np.random.default_rng(55)
    sub = synth.subset(d, rng.choice(d["n"], size=400, replace=False))
    S = M.to_device(sub["codes"], sub["offsets"], 20)
    exact = M.tree_build(S)
    e = torch.from_numpy(_emb(56, 400)).to(S.codes.device)
    _equal_trees(M.tree_build(S, emb=e, topk=1024), exact)
    _equal_trees(M.tree_build(S, emb=e, topk=4, exact_below=400), exact)
