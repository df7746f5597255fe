"""Pins of the CPU reference embedder (float64): library conv/autograd/Adam
and central finite differences (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import cnn_ref as ref


def _torch_forward(params, x, sigma):
    h = torch.tensor(ref.one_hot(x, sigma).T[None], dtype=torch.float64)
    n = len(params)
    tp = []
    for l, (W, b) in enumerate(params):
        w = torch.tensor(np.transpose(W, (2, 1, 0)).copy(), requires_grad=True)  # (Cout, Cin, K)
        bb = torch.tensor(b.copy(), requires_grad=True)
        tp.append((w, bb))
        h = torch.nn.functional.conv1d(h, w, bb, padding=W.shape[0] // 2)
        if l < n - 1:
            h = torch.relu(h)
    return h[0].mean(dim=1), tp


def test_conv_matches_library():
    rng = np.random.default_rng(1)
    H = rng.normal(size=(13, 6))
    W = rng.normal(size=(5, 6, 7))
    b = rng.normal(size=7)
    got = ref.conv(H, W, b)
    want = torch.nn.functional.conv1d(torch.tensor(H.T[None]), torch.tensor(np.transpose(W, (2, 1, 0)).copy()),
                                      torch.tensor(b), padding=2)[0].T.numpy()
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_forward_and_gradients_match_autograd():
    params = ref.init_params(3, sigma=4, width=16, layers=4)
    rng = np.random.default_rng(2)
    x = rng.integers(0, 4, size=23)
    e, cache = ref.forward(params, x, 4)
    te, tp = _torch_forward(params, x, 4)
    np.testing.assert_allclose(e, te.detach().numpy(), rtol=1e-10, atol=1e-12)
    de = rng.normal(size=e.shape)
    (te * torch.tensor(de)).sum().backward()
    grads = ref.backward(params, cache, de)
    for (gW, gb), (w, bb) in zip(grads, tp):
        np.testing.assert_allclose(gW, np.transpose(w.grad.numpy(), (2, 1, 0)), rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(gb, bb.grad.numpy(), rtol=1e-9, atol=1e-11)


def test_pair_loss_gradient_by_finite_differences():
    params = ref.init_params(4, sigma=4, width=6, layers=3)
    rng = np.random.default_rng(5)
    seqs = [rng.integers(0, 4, size=int(rng.integers(3, 8))) for _ in range(5)]
    ia, ib = np.array([0, 1, 2, 3]), np.array([1, 2, 4, 0])
    y = rng.uniform(0.2, 1.0, size=4)
    loss, grads = ref.pair_loss_and_grads(params, seqs, ia, ib, y, 4)
    h = 1e-6
    for l in range(len(params)):
        for which in (0, 1):
            arr = params[l][which]
            for _ in range(4):
                idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = ref.pair_loss_and_grads(params, seqs, ia, ib, y, 4)
                arr[idx] = old - h
                lm, _ = ref.pair_loss_and_grads(params, seqs, ia, ib, y, 4)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[l][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (l, which, idx, fd, an)


def test_adam_matches_library():
    params = ref.init_params(6, sigma=4, width=8, layers=2)
    rng = np.random.default_rng(7)
    tparams = [torch.tensor(p.copy(), requires_grad=True) for W, b in params for p in (W, b)]
    opt = torch.optim.Adam(tparams, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = ref.adam_init(params)
    for step in range(3):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
        flat = [g for gW, gb in grads for g in (gW, gb)]
        for t, g in zip(tparams, flat):
            t.grad = torch.tensor(g)
        opt.step()
        params, state = ref.adam_step(params, grads, state)
    mine = [p for W, b in params for p in (W, b)]
    for a, t in zip(mine, tparams):
        np.testing.assert_allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_mean_pool_ignores_padding_length():
    # the embedding of a sequence does not depend on anything outside it
    params = ref.init_params(8, sigma=4, width=8, layers=3)
    x = np.array([0, 1, 2, 3, 3, 1])
    e1, _ = ref.forward(params, x, 4)
    e2, _ = ref.forward(params, x.copy(), 4)
    np.testing.assert_array_equal(e1, e2)
    # identical sequences give a zero predicted distance
    assert np.linalg.norm(e1 - e2) == 0
