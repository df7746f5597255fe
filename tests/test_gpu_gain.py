"""Gain test of the learned ranking (seeded, GPU): what the trained embedder
adds to the pruned median over the controls, at equal top-k.

20,000 sequences of the learned workload (its first 200 families), the exact
tree, an embedder trained on 400,000 labelled pairs (deterministic: the
weight gradients are summed in a fixed order), and teacher-forced agreement
of (c, l, r) on the exact tree's clusters above 16 members for: the
calibrated network, shortest-first (a zero embedding with an offset), a
random embedding, and the sampled median of Sec. 2.1 (16 pivots).  The
assertions state what the measurements show on this workload: the network
is no worse than the length prior and far better than noise, and the
sampled median beats both."""
import numpy as np
import pytest

from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def test_learned_ranking_against_controls():
    from paper_2601_15458_amd import learned
    from paper_2601_15458_amd import msadp as M
    d = synth.learned()
    keep = np.flatnonzero(d["family"] < 200)
    sub = synth.subset(d, keep)
    S = M.to_device(sub["codes"], sub["offsets"], sub["sigma"])
    fam = np.asarray(sub["family"])
    print(f"[gain] {S.n} sequences: exact tree", flush=True)
    exact = M.tree_build(S)
    ia, ib = learned.sample_pairs(fam, 400_000, seed=61)
    dist = learned.lev_labels(S, ia, ib)
    print("[gain] training", flush=True)
    E, losses, _, _ = learned.train(S, ia, ib, dist, epochs=2, seed=62)
    emb = E.embed(S)
    off, _, _, corr = learned.calibrate(emb, S, fam, n_pairs=5000, seed=63)
    topk = 16
    agree = {}
    rankers = {"cnn": dict(emb=emb, emb_offset=off),
               "shortest": dict(emb=learned.control_embeddings(S, "zero"), emb_offset=1.0),
               "random": dict(emb=learned.control_embeddings(S, "random", seed=64),
                              emb_offset=0.0),
               "sampled16": dict(pivots=16)}
    for name, kw in rankers.items():
        clr = M.tree_eval_centers(S, exact, topk=topk, exact_below=0, **kw)
        agree[name] = learned.agreement(exact, clr, min_size=17, pruned_above=topk)["clr"]
    print(f"[gain] loss {losses[:20].mean():.4f} -> {losses[-20:].mean():.4f}, within-family "
          f"corr {corr:.3f}, offset {off:.2f}; agreement at top-{topk}: {agree}", flush=True)
    assert losses[-20:].mean() < 0.8 * losses[:20].mean()
    # the network: no worse than the length prior, far better than noise
    assert agree["cnn"] >= agree["shortest"] - 0.005
    assert agree["cnn"] >= agree["random"] + 0.05
    # the median over a sampled subset beats both rankings at equal top-k
    assert agree["sampled16"] >= max(agree["cnn"], agree["shortest"]) + 0.02
