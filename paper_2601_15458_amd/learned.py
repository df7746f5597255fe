"""Training and evaluation of the learned surrogate that prunes the medoid.

The embedder (a 4-layer 1D CNN, include/msadp.h cnn_*) learns
||e_a - e_b|| ~ lev(a, b) / mean(|a|, |b|) from exact distances that the
library itself computes (lev_batch).  tree_build_pruned then ranks medoid
candidates by embedding distance and verifies the best topk exactly.

Everything that computes runs in the library's kernels; this module only
draws pairs, batches them and compares outcomes (agreement, error) on the
host.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import msadp as M

CNN_SIGMA = 4


def init_params(seed: int, sigma: int = CNN_SIGMA):
    """He-uniform weights and zero biases, W[l]: (K, cin, 128)."""
    rng = np.random.default_rng(seed)
    params = []
    cin = sigma
    for _ in range(M.CNN_LAYERS):
        bound = np.sqrt(6.0 / (cin * M.CNN_K))
        W = rng.uniform(-bound, bound, size=(M.CNN_K, cin, M.CNN_WIDTH)).astype(np.float32)
        params.append((W, np.zeros(M.CNN_WIDTH, np.float32)))
        cin = M.CNN_WIDTH
    return params


def sample_pairs(family, n_pairs: int, seed: int, within: float = 0.5):
    """`within` of the pairs from one family (distinct members), the rest
    uniform over all distinct pairs."""
    rng = np.random.default_rng(seed)
    family = np.asarray(family)
    n = len(family)
    order = np.argsort(family, kind="stable")
    fam_sorted = family[order]
    starts = np.searchsorted(fam_sorted, fam_sorted, side="left")
    ends = np.searchsorted(fam_sorted, fam_sorted, side="right")
    n_in = int(round(n_pairs * within))
    a_pos = rng.integers(0, n, size=n_in)
    size = ends[a_pos] - starts[a_pos]
    b_off = rng.integers(0, np.maximum(size - 1, 1))
    b_pos = starts[a_pos] + b_off
    b_pos = np.where(b_pos >= a_pos, b_pos + 1, b_pos)     # skip a itself
    ia_in, ib_in = order[a_pos], order[np.minimum(b_pos, ends[a_pos] - 1)]
    n_out = n_pairs - n_in
    ia_out = rng.integers(0, n, size=n_out)
    ib_out = (ia_out + rng.integers(1, n, size=n_out)) % n
    ia = np.concatenate([ia_in, ia_out]).astype(np.int32)
    ib = np.concatenate([ib_in, ib_out]).astype(np.int32)
    keep = ia != ib
    perm = rng.permutation(int(keep.sum()))
    return ia[keep][perm], ib[keep][perm]


def lev_labels(S, ia, ib):
    """Exact distances (device uint16) of the pairs, by lev_batch."""
    return M.lev_batch(S, S, ia, ib)


def train(S, ia, ib, dist, epochs: int = 1, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Adam on the pair loss; returns (embedder, per-step losses, seconds,
    sequence positions processed).  dist: device tensor of the pairs' exact
    distances."""
    E = M.Embedder()
    E.set_params(init_params(seed, S.sigma))
    rng = np.random.default_rng(seed + 1)
    losses = []
    positions = 0
    dist = dist.to(torch.int32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_pairs = len(ia)
    for ep in range(epochs):
        order = rng.permutation(n_pairs)
        for s in range(0, n_pairs - batch + 1, batch):
            sel = order[s:s + batch]
            a, b = ia[sel], ib[sel]
            idx, inv = np.unique(np.concatenate([a, b]), return_inverse=True)
            pa, pb = inv[: len(a)], inv[len(a):]
            positions += int(S.lengths[idx].sum())
            d = dist[torch.from_numpy(sel).to(dist.device)].to(torch.uint16)
            losses.append(E.train_step(S, idx, pa, pb, d, lr=lr))
            if log is not None and (len(losses) % 100 == 0):
                log(f"epoch {ep} step {len(losses)} loss {np.mean(losses[-100:]):.5f}")
    torch.cuda.synchronize()
    return E, np.asarray(losses), time.perf_counter() - t0, positions


# Multiply-adds of the embedder per sequence position (kernel width 5): the
# one-hot layer (sigma inputs) and three 128 x 128 layers.
def flops_per_position(sigma: int = CNN_SIGMA) -> int:
    return 2 * M.CNN_K * M.CNN_WIDTH * (sigma + 3 * M.CNN_WIDTH)


def pair_error(emb, S, ia, ib, dist):
    """Held-out error of the predicted distance ||e_a - e_b|| * mean length
    against the exact one: (MAE in edits, mean relative error)."""
    a = torch.from_numpy(np.asarray(ia, np.int64)).to(emb.device)
    b = torch.from_numpy(np.asarray(ib, np.int64)).to(emb.device)
    lens = torch.from_numpy(S.lengths.astype(np.float64)).to(emb.device)
    pred = (emb[a].double() - emb[b].double()).norm(dim=1) * (lens[a] + lens[b]) / 2
    d = dist.to(torch.float64)
    err = (pred - d).abs()
    return float(err.mean()), float((err / d.clamp(min=1)).mean())


def control_embeddings(S, kind: str, seed: int = 0):
    """Rankers without the network.  'zero': every embedding distance is 0,
    so with an offset the estimate is the length prior (shortest first);
    'length': |x| / mean length on one axis (the estimate grows with the
    length difference); 'random': Gaussian noise."""
    n = S.n
    e = np.zeros((n, M.CNN_WIDTH), np.float32)
    if kind == "length":
        e[:, 0] = S.lengths / max(float(S.lengths.mean()), 1.0)
    elif kind == "random":
        e = np.random.default_rng(seed).standard_normal((n, M.CNN_WIDTH)).astype(np.float32)
    elif kind != "zero":
        raise ValueError(kind)
    return torch.from_numpy(e).to(S.codes.device)


def calibrate(emb, S, family, n_pairs: int = 20000, seed: int = 21, cap: float = 1024.0):
    """Offset of the pruned ranking: fit the true normalized distance of
    held-out within-family pairs (the regime of most clusters) linearly on
    the predicted one, y ~ a + b * y_hat; the ranking only depends on
    y_hat + a / b.  A predictor with b <= 0 carries no ranking signal and
    gets the cap (the length prior).  Returns (offset, a, b, correlation)."""
    ia, ib = sample_pairs(family, n_pairs, seed=seed, within=1.0)
    d = lev_labels(S, ia, ib).to(torch.float64).cpu().numpy()
    L = S.lengths.astype(np.float64)
    y = d / ((L[ia] + L[ib]) / 2)
    a_t = torch.from_numpy(np.asarray(ia, np.int64)).to(emb.device)
    b_t = torch.from_numpy(np.asarray(ib, np.int64)).to(emb.device)
    yh = (emb[a_t].double() - emb[b_t].double()).norm(dim=1).cpu().numpy()
    return fit_offset(yh, y, cap)


def fit_offset(yh, y, cap: float = 1024.0):
    """Least-squares line y ~ a + b * yh through (predicted, true) normalized
    distances; the ranking offset is a / b clipped to [0, cap], and cap when
    b <= 0 (no ranking signal: the estimate falls back to the length prior).
    Returns (offset, a, b, correlation)."""
    yh = np.asarray(yh, np.float64)
    y = np.asarray(y, np.float64)
    if len(yh) < 2 or float(np.ptp(yh)) == 0.0:
        return cap, float(y.mean()) if len(y) else 0.0, 0.0, 0.0
    b, a = np.polyfit(yh, y, 1)
    corr = float(np.corrcoef(yh, y)[0, 1])
    off = cap if b <= 0 else float(min(max(a / b, 0.0), cap))
    return off, float(a), float(b), corr


def agreement(tree, clr, min_size: int = 17, pruned_above: int = 16):
    """Teacher-forced agreement of a choice (center, lpole, rpole per node of
    the exact tree) with the tree's own, as fractions of internal nodes:
    over those with at least min_size members ("clr", "c", "poles"), over
    all ("clr_all"), and over those above pruned_above members, the only
    ones whose choice was pruned ("clr_pruned")."""
    c, l, r = clr
    internal = tree["left"] >= 0
    big = internal & (tree["mcount"] >= min_size)
    pruned = internal & (tree["mcount"] > pruned_above)
    same_clr = (c == tree["center"]) & (l == tree["lpole"]) & (r == tree["rpole"])
    same_c = c == tree["center"]
    same_lr = (l == tree["lpole"]) & (r == tree["rpole"])

    def frac(mask, sel):
        return round(float(mask[sel].mean()), 4) if sel.any() else 1.0

    return {"clusters": int(big.sum()), "clr": frac(same_clr, big), "c": frac(same_c, big),
            "poles": frac(same_lr, big), "clr_all": frac(same_clr, internal),
            "internal": int(internal.sum()), "pruned_clusters": int(pruned.sum()),
            "clr_pruned": frac(same_clr, pruned)}


def reproduced_clusters(exact, other, seed: int = 0):
    """Fraction of the exact tree's internal clusters (member sets of two or
    more) that the other tree also holds, by 64-bit set hashes over each
    node's perm range."""
    n = len(exact["perm"])
    h = np.random.default_rng(seed).integers(0, 2 ** 63, size=n, dtype=np.uint64)

    def keys(t):
        pre = np.concatenate([[np.uint64(0)], np.cumsum(h[t["perm"]], dtype=np.uint64)])
        s = pre[t["mstart"] + t["mcount"]] - pre[t["mstart"]]
        big = t["mcount"] >= 2
        return set(zip(s[big].tolist(), t["mcount"][big].tolist()))

    ke, ko = keys(exact), keys(other)
    return len(ke & ko) / max(len(ke), 1)


def rowsum_excess(S, exact, clr, pruned_above: int):
    """How far a pruned center is from the full median where they differ:
    (sum f(c', x) - sum f(c, x)) / sum f(c, x) over the members x of each
    internal cluster above pruned_above members, exact sums by lev_batch.
    Returns (number of clusters that differ, mean and max relative excess)."""
    c2 = clr[0]
    sel = np.flatnonzero((exact["left"] >= 0) & (exact["mcount"] > pruned_above) &
                         (c2 != exact["center"]))
    if len(sel) == 0:
        return 0, 0.0, 0.0
    ia, ib, seg = [], [], []
    for j, v in enumerate(sel):
        mem = exact["perm"][exact["mstart"][v]: exact["mstart"][v] + exact["mcount"][v]]
        for t, c in enumerate((exact["center"][v], c2[v])):
            ia.append(np.full(len(mem), c, np.int32))
            ib.append(mem.astype(np.int32))
            seg.append(np.full(len(mem), 2 * j + t, np.int64))
    ia, ib = np.concatenate(ia), np.concatenate(ib)
    seg = np.concatenate(seg)
    d = M.lev_batch(S, S, ia, ib).to(torch.int64).cpu().numpy()
    sums = np.bincount(seg, weights=d, minlength=2 * len(sel)).reshape(len(sel), 2)
    rel = (sums[:, 1] - sums[:, 0]) / np.maximum(sums[:, 0], 1)
    return int(len(sel)), float(rel.mean()), float(rel.max())
