"""Seeded synthetic sequence sets shaped like the paper's workloads.

This module only draws random sequences; it computes no distance, alignment
or clustering.  Both the device path and the CPU checker read their inputs
from here, so it deliberately imports nothing else from the package.

The paper benchmarks on Greengenes 16S rRNA (DNA, lengths about 1.1k-2.4k,
Table 1), PDB and Pfam proteins (median length 224-255 with a long tail,
Table 1).  None of those datasets is available here, so the functions below
generate stand-ins with those length regimes from an explicit evolution
model:

* ``mutate``: every site independently undergoes at most one event:
  substitution (to a uniformly chosen *different* symbol), insertion of a
  Geometric(1/2) run of uniform symbols before the site, or deletion of a
  Geometric(1/2) run starting at the site.
* ``evolve_tree``: a random binary tree grown from a root by repeatedly
  picking a uniform current leaf and replacing it by two independently
  mutated copies of itself.

Sequences are returned as uint8 symbol codes (DNA A,C,G,T = 0..3; proteins
0..19) in CSR form: ``codes`` (all sequences concatenated) and ``offsets``
(int64, n+1 entries).  Duplicate sequences are re-mutated until every
sequence is distinct (the method assumes de-duplicated input, Sec. 2.1).
"""
from __future__ import annotations

import numpy as np

DNA = 4
PROTEIN = 20

# Seeds of the five named workloads.
SEEDS = {"tiny": 1, "allpairs": 2, "protein_tree": 3, "nw_long": 4, "learned": 5}


def mutate(rng, s, sigma, p_sub, p_ins, p_del):
    """One copy of ``s`` with per-site substitution/insertion/deletion events."""
    n = len(s)
    if n == 0:
        return s.copy()
    u = rng.random(n)
    sub = u < p_sub
    ins = (u >= p_sub) & (u < p_sub + p_ins)
    dele = (u >= p_sub + p_ins) & (u < p_sub + p_ins + p_del)
    base = s.astype(np.int64).copy()
    nsub = int(sub.sum())
    if nsub:
        base[sub] = (base[sub] + rng.integers(1, sigma, size=nsub)) % sigma
    keep = np.ones(n, dtype=bool)
    del_idx = np.flatnonzero(dele)
    if len(del_idx):
        runs = rng.geometric(0.5, size=len(del_idx))
        for st, ln in zip(del_idx, runs):
            keep[st:st + ln] = False
    ins_idx = np.flatnonzero(ins & keep)
    pieces = []
    prev = 0
    if len(ins_idx):
        runs = rng.geometric(0.5, size=len(ins_idx))
        for st, ln in zip(ins_idx, runs):
            seg = base[prev:st][keep[prev:st]]
            pieces.append(seg)
            pieces.append(rng.integers(0, sigma, size=int(ln)))
            prev = st
    pieces.append(base[prev:][keep[prev:]])
    return np.concatenate(pieces).astype(np.uint8)


def evolve_tree(rng, root, n_leaves, sigma, p_sub, p_ins, p_del):
    """Leaves of a random binary tree grown from ``root`` (Yule-style splits)."""
    leaves = [root]
    while len(leaves) < n_leaves:
        k = int(rng.integers(0, len(leaves)))
        parent = leaves[k]
        a = mutate(rng, parent, sigma, p_sub, p_ins, p_del)
        b = mutate(rng, parent, sigma, p_sub, p_ins, p_del)
        leaves[k] = a
        leaves.append(b)
    return leaves


def fit_length(rng, s, target, sigma):
    """Truncate ``s`` to ``target`` or pad it with uniform symbols."""
    if len(s) >= target:
        return s[:target].copy()
    pad = rng.integers(0, sigma, size=target - len(s)).astype(np.uint8)
    return np.concatenate([s, pad])


def clip_length(rng, s, lo, hi, sigma):
    if len(s) > hi:
        return s[:hi].copy()
    if len(s) < lo:
        return fit_length(rng, s, lo, sigma)
    return s


def dedupe(rng, seqs, sigma, p=0.02):
    """Re-mutate any sequence equal to an earlier one until all are distinct."""
    seen = set()
    out = []
    for s in seqs:
        key = s.tobytes()
        while key in seen:
            s = mutate(rng, s, sigma, p, 0.0, 0.0) if len(s) else \
                rng.integers(0, sigma, size=1).astype(np.uint8)
            key = s.tobytes()
        seen.add(key)
        out.append(s)
    return out


def to_csr(seqs):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    codes = np.concatenate(seqs).astype(np.uint8) if len(seqs) and offsets[-1] > 0 \
        else np.zeros(0, dtype=np.uint8)
    return codes, offsets


def from_csr(codes, offsets):
    return [codes[offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]


# ---------------------------------------------------------------- workloads

def tiny(seed=SEEDS["tiny"], n=64, root_len=200):
    """64 DNA leaves of a random tree from a 200-base root (5/1/1 % per edge)."""
    rng = np.random.default_rng(seed)
    root = rng.integers(0, DNA, size=root_len).astype(np.uint8)
    leaves = evolve_tree(rng, root, n, DNA, 0.05, 0.01, 0.01)
    leaves = dedupe(rng, leaves, DNA)
    codes, offsets = to_csr(leaves)
    return {"codes": codes, "offsets": offsets, "sigma": DNA, "n": n,
            "name": f"dna{n}_root{root_len}"}


def allpairs(seed=SEEDS["allpairs"], n=4096, lo=1000, hi=1600):
    """n DNA leaves from a ``hi``-base root, each fitted to a length U{lo..hi}."""
    rng = np.random.default_rng(seed)
    root = rng.integers(0, DNA, size=hi).astype(np.uint8)
    leaves = evolve_tree(rng, root, n, DNA, 0.05, 0.01, 0.01)
    lens = rng.integers(lo, hi + 1, size=n)
    leaves = [fit_length(rng, s, int(L), DNA) for s, L in zip(leaves, lens)]
    leaves = dedupe(rng, leaves, DNA)
    codes, offsets = to_csr(leaves)
    return {"codes": codes, "offsets": offsets, "sigma": DNA, "n": n,
            "name": f"dna{n}_len{lo}-{hi}"}


def families(rng, n_fam, per_fam, sigma, root_len_fn, d, lo, hi):
    seqs = []
    fam = []
    for f in range(n_fam):
        L = root_len_fn()
        root = rng.integers(0, sigma, size=L).astype(np.uint8)
        for _ in range(per_fam):
            s = mutate(rng, root, sigma, 0.8 * d, 0.1 * d, 0.1 * d)
            seqs.append(clip_length(rng, s, lo, hi, sigma))
            fam.append(f)
    return seqs, np.asarray(fam, dtype=np.int32)


def protein_tree(seed=SEEDS["protein_tree"], n_fam=200, per_fam=100):
    """Protein families: lognormal root lengths (median 350, sigma 0.6) in [50, 2000]."""
    rng = np.random.default_rng(seed)

    def root_len():
        return int(np.clip(round(rng.lognormal(np.log(350.0), 0.6)), 50, 2000))

    seqs, fam = families(rng, n_fam, per_fam, PROTEIN, root_len, 0.30, 50, 2000)
    seqs = dedupe(rng, seqs, PROTEIN)
    codes, offsets = to_csr(seqs)
    return {"codes": codes, "offsets": offsets, "sigma": PROTEIN, "n": len(seqs),
            "family": fam, "name": f"protein{len(seqs)}_fam{n_fam}"}


def nw_long(seed=SEEDS["nw_long"], n_pairs=512, lo=5000, hi=10000, d=0.10):
    """Pairs (a, b): a uniform DNA of length U{lo..hi}, b = mutate(a, d) in [lo, hi]."""
    rng = np.random.default_rng(seed)
    A, B = [], []
    for _ in range(n_pairs):
        L = int(rng.integers(lo, hi + 1))
        a = rng.integers(0, DNA, size=L).astype(np.uint8)
        b = mutate(rng, a, DNA, 0.8 * d, 0.1 * d, 0.1 * d)
        A.append(a)
        B.append(clip_length(rng, b, lo, hi, DNA))
    ca, oa = to_csr(A)
    cb, ob = to_csr(B)
    return {"a_codes": ca, "a_offsets": oa, "b_codes": cb, "b_offsets": ob,
            "sigma": DNA, "n_pairs": n_pairs, "name": f"nw{n_pairs}_len{lo}-{hi}"}


def learned(seed=SEEDS["learned"], n_fam=1000, per_fam=100, lo=100, hi=500):
    """DNA families: roots of length U{lo..hi}, members mutate(root, 0.30) in [lo, hi]."""
    rng = np.random.default_rng(seed)

    def root_len():
        return int(rng.integers(lo, hi + 1))

    seqs, fam = families(rng, n_fam, per_fam, DNA, root_len, 0.30, lo, hi)
    seqs = dedupe(rng, seqs, DNA)
    codes, offsets = to_csr(seqs)
    return {"codes": codes, "offsets": offsets, "sigma": DNA, "n": len(seqs),
            "family": fam, "name": f"dna{len(seqs)}_fam{n_fam}"}


def random_set(seed, n, lo, hi, sigma):
    """n uniform random sequences with lengths U{lo..hi} (edge-case tests)."""
    rng = np.random.default_rng(seed)
    seqs = [rng.integers(0, sigma, size=int(rng.integers(lo, hi + 1))).astype(np.uint8)
            for _ in range(n)]
    return to_csr(seqs)


def subset(data, idx):
    """Sub-collection of a CSR set, in the order given by ``idx``."""
    seqs = from_csr(data["codes"], data["offsets"])
    sel = [seqs[int(i)] for i in idx]
    codes, offsets = to_csr(sel)
    out = dict(data)
    out.update(codes=codes, offsets=offsets, n=len(sel))
    if "family" in data:
        out["family"] = np.asarray(data["family"])[np.asarray(idx)]
    return out
