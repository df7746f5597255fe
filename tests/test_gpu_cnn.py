"""BF16 MFMA embedder on the GPU against the float64 CPU reference."""
import numpy as np
import pytest

from oracle import cnn_ref as ref
from oracle import pyoracle as orc
from paper_2601_15458_amd import synth

pytestmark = pytest.mark.gpu


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _bf16(x):
    """Round float64 to the nearest bfloat16 (ties to even), as the device does."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _setup(seed=1, n=48, lo=1, hi=90):
    M = _msadp()
    codes, off = synth.random_set(seed, n, lo, hi, 4)
    S = M.to_device(codes, off, 4)
    params = ref.init_params(seed, sigma=4, width=128, layers=4)
    # biases away from zero so that the bias paths are exercised
    rng = np.random.default_rng(seed)
    params = [(W, rng.normal(scale=0.05, size=b.shape)) for W, b in params]
    emb = M.Embedder()
    emb.set_params(params)
    seqs = synth.from_csr(codes, off)
    return M, S, emb, params, seqs


def test_forward_matches_reference():
    M, S, emb, params, seqs = _setup()
    got = emb.embed(S).cpu().numpy()
    # reference with the weights the device holds (bf16) and exact arithmetic
    pq = [(_bf16(W), b) for W, b in params]
    want = ref.embed(pq, seqs, 4)
    err = rel_l2(got, want)
    print("embedding rel L2", err)
    assert err < 2e-2, err
    # against the unrounded float64 model as well
    assert rel_l2(got, ref.embed(params, seqs, 4)) < 3e-2


def test_gradients_match_reference():
    M, S, emb, params, seqs = _setup(seed=2, n=40, lo=5, hi=70)
    rng = np.random.default_rng(3)
    P = 64
    pa = rng.integers(0, S.n, size=P)
    pb = rng.integers(0, S.n, size=P)
    d = orc.lev_pairs(*synth.to_csr(seqs), *synth.to_csr(seqs), pa, pb)
    idx = np.arange(S.n)
    emb.train_step(S, idx, pa, pb, d.astype(np.uint16), lr=0.0)
    _, grads = emb.get()
    y = ref.pair_labels(d, [len(seqs[i]) for i in pa], [len(seqs[i]) for i in pb])
    pq = [(_bf16(W), b) for W, b in params]
    _, want = ref.pair_loss_and_grads(pq, seqs, pa, pb, y, 4)
    for l in range(4):
        gW, gb = grads[l]
        wW, wb = want[l]
        if l == 0:
            gW = gW[:, :4, :]        # one-hot channels beyond sigma carry no gradient
        e1 = rel_l2(gW, wW)
        if l == 3:
            # the last bias gradient is exactly zero: the mean pool hands
            # dE to every row and each pair adds +g and -g to its two ends
            e2 = float(np.linalg.norm(gb - wb) / np.linalg.norm(wW))
        else:
            e2 = rel_l2(gb, wb)
        print(f"layer {l}: dW rel {e1:.4f}  db rel {e2:.4f}")
        # BF16 storage of activations and of each layer's gradient rows
        # (relative rounding 2^-9 per value, compounded over 4 layers each
        # way, with cancellation in the sums) allows a few percent.
        assert e1 < 5e-2 and e2 < 5e-2, (l, e1, e2)


def test_adam_update_matches_reference():
    M, S, emb, params, seqs = _setup(seed=4, n=24, lo=5, hi=40)
    rng = np.random.default_rng(5)
    pa = rng.integers(0, S.n, size=32)
    pb = rng.integers(0, S.n, size=32)
    d = orc.lev_pairs(*synth.to_csr(seqs), *synth.to_csr(seqs), pa, pb).astype(np.uint16)
    p0, _ = emb.get()
    emb.train_step(S, np.arange(S.n), pa, pb, d, lr=1e-3)
    p1, g = emb.get()
    # Adam from zero state: the first step moves every weight by lr * g / (|g| + eps)
    state = ref.adam_init([(W.astype(np.float64), b.astype(np.float64)) for W, b in p0])
    want, _ = ref.adam_step([(W.astype(np.float64), b.astype(np.float64)) for W, b in p0],
                            [(gW.astype(np.float64), gb.astype(np.float64)) for gW, gb in g], state)
    for (W1, b1), (Ww, bw) in zip(p1, want):
        np.testing.assert_allclose(W1, Ww, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(b1, bw, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    M, S, emb, params, seqs = _setup(seed=6, n=64, lo=20, hi=80)
    rng = np.random.default_rng(7)
    pa = rng.integers(0, S.n, size=256)
    pb = rng.integers(0, S.n, size=256)
    d = orc.lev_pairs(*synth.to_csr(seqs), *synth.to_csr(seqs), pa, pb).astype(np.uint16)
    losses = [emb.train_step(S, np.arange(S.n), pa, pb, d, lr=2e-3) for _ in range(30)]
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.5 * losses[0]
