"""CPU reference of the sequence embedder used to prune exact distance work.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline may use it; the device path never does).

The embedder is not part of the paper: it is this project's learned
surrogate for the distance f of Alg. 1.  Its definition, in float64:

  H0[t, c]   = [x_t == c]                       (one-hot, t < L, c < sigma)
  Z_l[t, o]  = b_l[o] + sum_{k<K} sum_i W_l[k, i, o] * H_{l-1}[t + k - K//2, i]
               (H = 0 outside 0 <= t < L: zero padding of each sequence)
  H_l        = relu(Z_l) for l = 1 .. n_layers-1;  H_last = Z_last
  e[o]       = (1/L) * sum_{t<L} H_last[t, o]   (mean over the sequence)

and for a pair (a, b) with label y = lev(a, b) / ((|a| + |b|) / 2):

  pred = ||e_a - e_b||_2,   loss = mean over pairs of (pred - y)^2.

Every function is a direct transcription with explicit shifts; gradients
are derived by hand (chain rule through the same steps, backwards).
"""
from __future__ import annotations

import numpy as np


def init_params(seed: int, sigma: int = 4, width: int = 128, layers: int = 4, K: int = 5):
    """He-uniform weights, zero biases (float64), shapes W[l]: (K, Cin, Cout)."""
    rng = np.random.default_rng(seed)
    params = []
    cin = sigma
    for _ in range(layers):
        bound = np.sqrt(6.0 / (cin * K))
        W = rng.uniform(-bound, bound, size=(K, cin, width))
        b = np.zeros(width)
        params.append((W, b))
        cin = width
    return params


def bf16(x):
    """Round to the nearest bfloat16 (8-bit significand, ties to even), as a
    float64 array: the storage format the device keeps activations and
    gradient rows in."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def one_hot(x, sigma):
    x = np.asarray(x, dtype=np.int64)
    H = np.zeros((len(x), sigma))
    H[np.arange(len(x)), x] = 1.0
    return H


def conv(H, W, b):
    """Z[t, o] = b[o] + sum_k sum_i W[k, i, o] H[t + k - K//2, i] with zero padding."""
    K = W.shape[0]
    L = H.shape[0]
    pad = K // 2
    Hp = np.zeros((L + 2 * pad, H.shape[1]))
    Hp[pad:pad + L] = H
    Z = np.tile(b, (L, 1))
    for k in range(K):
        Z = Z + Hp[k:k + L] @ W[k]
    return Z


def _same(x):
    return x


def forward(params, x, sigma, store=_same):
    """Embedding of one sequence and the per-layer cache for backward.

    store: applied to every hidden activation H_1 .. H_{n-1} as it is kept
    (identity: exact float64; a rounding function emulates a storage format)."""
    H = one_hot(x, sigma)
    cache = [H]
    n = len(params)
    for l, (W, b) in enumerate(params):
        Z = conv(H, W, b)
        H = store(np.maximum(Z, 0.0)) if l < n - 1 else Z
        cache.append((Z, H))
    e = H.mean(axis=0)
    return e, cache


def backward(params, cache, de, store=_same):
    """Gradients (dW, db per layer) given dL/de for one sequence.

    store: applied to every layer's output gradient dZ as it is kept."""
    n = len(params)
    L = cache[0].shape[0]
    dH = np.tile(de / L, (L, 1))              # mean pool
    grads = [None] * n
    for l in range(n - 1, -1, -1):
        W, b = params[l]
        Z, H = cache[l + 1]
        # the ReLU passes where the kept activation is positive
        dZ = store(dH * (H > 0) if l < n - 1 else dH)
        Hin = cache[0] if l == 0 else cache[l][1]
        K = W.shape[0]
        pad = K // 2
        Hp = np.zeros((L + 2 * pad, Hin.shape[1]))
        Hp[pad:pad + L] = Hin
        dW = np.zeros_like(W)
        for k in range(K):
            dW[k] = Hp[k:k + L].T @ dZ
        db = dZ.sum(axis=0)
        grads[l] = (dW, db)
        # dH_in[t] = sum_k dZ[t - k + pad] W[k]^T
        dZp = np.zeros((L + 2 * pad, dZ.shape[1]))
        dZp[pad:pad + L] = dZ
        dHin = np.zeros_like(Hin)
        for k in range(K):
            dHin += dZp[2 * pad - k: 2 * pad - k + L] @ W[k].T
        dH = dHin
    return grads


def embed(params, seqs, sigma):
    return np.stack([forward(params, s, sigma)[0] for s in seqs])


def pair_loss_and_grads(params, seqs, ia, ib, labels, sigma, store=_same):
    """Mean squared error of ||e_a - e_b|| against labels, and its gradients
    (store: see forward and backward)."""
    caches = {}
    embs = {}
    for i in set(np.asarray(ia).tolist()) | set(np.asarray(ib).tolist()):
        embs[i], caches[i] = forward(params, seqs[i], sigma, store)
    P = len(ia)
    loss = 0.0
    dE = {i: np.zeros_like(embs[i]) for i in embs}
    for a, b, y in zip(ia, ib, labels):
        diff = embs[a] - embs[b]
        pred = np.sqrt((diff * diff).sum())
        r = pred - y
        loss += r * r / P
        g = 2.0 * r / P * (diff / pred if pred > 0 else np.zeros_like(diff))
        dE[a] += g
        dE[b] -= g
    total = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    for i, de in dE.items():
        gi = backward(params, caches[i], de, store)
        total = [(tw + gw, tb + gb) for (tw, tb), (gw, gb) in zip(total, gi)]
    return loss, total


def pair_labels(dist, la, lb):
    """y = d / mean length of the pair."""
    return np.asarray(dist, dtype=np.float64) / ((np.asarray(la) + np.asarray(lb)) / 2.0)


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in float64; state = (t, m, v)."""
    t, m, v = state
    t += 1
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = b1 * mm + (1 - b1) * g
            vv = b2 * vv + (1 - b2) * g * g
            mh = mm / (1 - b1 ** t)
            vh = vv / (1 - b2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        (W2, mW2, vW2), (b2_, mb2, vb2) = out
        new_p.append((W2, b2_))
        new_m.append((mW2, mb2))
        new_v.append((vW2, vb2))
    return new_p, (t, new_m, new_v)


def adam_init(params):
    z = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    return (0, z, [(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
