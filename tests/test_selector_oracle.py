"""Pins of the selector's FP64 oracle (oracle/mlp.py) against facts fixed
outside it (CPU only): a hand-counted feature example, closed forms of small
ReLU networks, finite differences, PyTorch's CPU autograd, Adam's behaviour
under a constant gradient, and a brute-force argmin.
"""
import math

import numpy as np
import torch

from oracle import mlp


# --------------------------------------------------------------- features

def test_features_hand_example():
    # rows 0, 5, 7, 9, 11 hold 1, 2, 3, 4 and 8 entries: 18 entries in 5 rows,
    # in classes floor(log2 L) = 0, 1, 1, 2, 3 -> entry counts 1, 5, 4, 8.
    lens = {0: 1, 5: 2, 7: 3, 9: 4, 11: 8}
    rows, cols = [], []
    for r, L in lens.items():
        for j in range(L):
            rows.append(r)
            cols.append(100 + j)  # columns 100..107: 8 distinct
    f = mlp.features(rows, cols, kz=32, bf16=True)
    want = np.zeros(23)
    want[0:4] = [1 / 18, 5 / 18, 4 / 18, 8 / 18]
    want[16] = 3 / 16             # longest row 8
    want[17] = math.log2(5) / 16  # 5 rows
    want[18] = 3 / 16             # 8 columns
    want[19] = math.log2(18) / 24
    want[20] = math.log2(18 / 5) / 8
    want[21] = 5 / 8              # kz = 32
    want[22] = 1.0
    np.testing.assert_allclose(f, want, rtol=0, atol=1e-15)


def test_features_invariants():
    rng = np.random.default_rng(5)
    rows = rng.integers(0, 300, 5000)
    cols = rng.integers(0, 40, 5000)
    f = mlp.features(rows, cols, kz=16, bf16=False)
    assert abs(f[:16].sum() - 1.0) < 1e-12
    ft = mlp.features(cols, rows, kz=16, bf16=False, transpose=True)
    np.testing.assert_array_equal(f, ft)
    # a row longer than 2^16 lands in the last class; single-entry rows in the first
    rows = np.r_[np.zeros(70000, np.int64), np.arange(1, 11)]
    cols = np.r_[np.arange(70000), np.zeros(10, np.int64)]
    f = mlp.features(rows, cols, kz=8, bf16=False)
    assert f[15] == 70000 / 70010 and f[0] == 10 / 70010
    assert abs(f[16] - math.log2(70000) / 16) < 1e-15


# ------------------------------------------------------------ dense layers

def test_relu_network_closed_forms():
    # |x| = relu(x) + relu(-x);  max(a, b) = b + relu(a - b) - relu(-b) + relu(b)
    x = np.linspace(-3, 3, 13)[:, None]
    h = mlp.linear_fwd(x, np.array([[1.0], [-1.0]]), None, relu=True)
    y = mlp.linear_fwd(h, np.array([[1.0, 1.0]]), np.zeros(1))
    np.testing.assert_array_equal(y[:, 0], np.abs(x[:, 0]))
    ab = np.array([[1.0, 2.0], [5.0, -1.0], [-2.0, -3.0], [0.5, 0.5]])
    W1 = np.array([[1.0, -1.0], [0.0, 1.0], [0.0, -1.0]])
    h = mlp.linear_fwd(ab, W1, None, relu=True)
    y = mlp.linear_fwd(h, np.array([[1.0, 1.0, -1.0]]), None)
    np.testing.assert_array_equal(y[:, 0], ab.max(axis=1))


def _net(rng, sizes):
    return [(rng.standard_normal((o, i)) / math.sqrt(i), rng.standard_normal(o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(11)
    layers = _net(rng, [5, 7, 6, 3])
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 3))
    M = (rng.random((9, 3)) < 0.7).astype(np.float64)
    # keep every pre-activation away from the ReLU kink so the loss is smooth
    acts = mlp.mlp_forward(layers, X)
    for i in range(len(layers) - 1):
        W, b = layers[i]
        assert np.abs(acts[i] @ W.T + b).min() > 1e-4
    loss, grads = mlp.mlp_loss_grads(layers, X, T, M)
    h = 1e-6
    for li, (W, b) in enumerate(layers):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for k in range(flat.size):
                old = flat[k]
                flat[k] = old + h
                lp, _ = mlp.mlp_loss_grads(layers, X, T, M)
                flat[k] = old - h
                lm, _ = mlp.mlp_loss_grads(layers, X, T, M)
                flat[k] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[k]) <= 1e-6 * (1 + abs(fd)), (li, k, fd)


def test_gradients_match_torch_autograd():
    rng = np.random.default_rng(12)
    layers = _net(rng, [23, 16, 16, 10])
    X = rng.standard_normal((40, 23))
    T = rng.standard_normal((40, 10))
    M = (rng.random((40, 10)) < 0.5).astype(np.float64)
    loss, grads = mlp.mlp_loss_grads(layers, X, T, M)
    tl = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
          for W, b in layers]
    h = torch.tensor(X)
    for i, (W, b) in enumerate(tl):
        h = torch.nn.functional.linear(h, W, b)
        if i + 1 < len(tl):
            h = torch.relu(h)
    Mt = torch.tensor(M)
    tloss = (Mt * (h - torch.tensor(T)) ** 2).sum() / Mt.sum()
    tloss.backward()
    assert abs(tloss.item() - loss) <= 1e-12 * abs(loss)
    for (W, b), (dW, db) in zip(tl, grads):
        np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_mse_closed_form_and_mask():
    T = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    M = np.array([[1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    P = T + 0.5 * M + 100.0 * (1 - M)   # masked-out entries are far off
    loss, dP = mlp.mse(P, T, M)
    assert loss == 0.25
    np.testing.assert_array_equal(dP, 2 * 0.5 * M / 4)
    loss0, dP0 = mlp.mse(P, T, np.zeros_like(M))
    assert loss0 == 0.0 and not dP0.any()


# ------------------------------------------------------------------ Adam

def test_adam_constant_gradient_moves_by_lr():
    # Under a constant gradient g the bias-corrected moments equal g and g^2
    # exactly at every step, so each step moves w by lr * g / (|g| + eps).
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    w = np.array([1.0, -1.0, 0.5, 0.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        w, m, v = mlp.adam(w, g, m, v, lr, 0.9, 0.999, eps, t)
        want = np.array([1.0, -1.0, 0.5, 0.0]) - t * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(w, want, rtol=0, atol=1e-14)


def test_adam_first_moments():
    m = np.zeros(2)
    v = np.zeros(2)
    w, m, v = mlp.adam(np.zeros(2), np.array([1.0, -2.0]), m, v, 0.1, 0.9, 0.99, 1e-8, 1)
    np.testing.assert_allclose(m, [0.1, -0.2], rtol=1e-15)
    np.testing.assert_allclose(v, [0.01, 0.04], rtol=1e-15)


# ---------------------------------------------------------------- argmin

def test_masked_argmin_brute_force():
    rng = np.random.default_rng(3)
    P = rng.integers(0, 4, (200, 9)).astype(np.float64)   # many ties
    M = (rng.random((200, 9)) < 0.6).astype(np.float64)
    M[7] = 0
    got = mlp.masked_argmin(P, M)
    masked = np.where(M != 0, P, np.inf)
    want = np.where(M.any(axis=1), np.argmin(masked, axis=1), -1)  # argmin: first minimum
    np.testing.assert_array_equal(got, want)
    assert got[7] == -1


def test_masked_argmin_preferred_column():
    """The preferred column is kept while within margin of the least allowed
    value, and only then; hand cases, then brute force."""
    P = np.array([[1.0, 0.5, 0.49], [1.0, 0.5, 0.4], [1.0, 0.5, 0.4], [2.0, 0.5, 9.0]],
                 np.float32)
    M = np.array([[1, 1, 1], [1, 1, 1], [0, 1, 1], [1, 1, 1]], np.float32)
    # pref 1: within 0.05 of 0.49 -> 1; 0.1 above 0.4 -> 2; pref 0 masked off
    np.testing.assert_array_equal(mlp.masked_argmin(P[:2], M[:2], pref=1, margin=0.05), [1, 2])
    np.testing.assert_array_equal(mlp.masked_argmin(P[2:3], M[2:3], pref=0, margin=5.0), [2])
    np.testing.assert_array_equal(mlp.masked_argmin(P[3:], M[3:], pref=0, margin=1.5), [0])
    np.testing.assert_array_equal(mlp.masked_argmin(P[3:], M[3:], pref=0, margin=1.4), [1])
    rng = np.random.default_rng(5)
    P = rng.integers(0, 8, (300, 7)).astype(np.float32) / 4
    M = (rng.random((300, 7)) < 0.7).astype(np.float32)
    for pref, margin in ((0, 0.0), (3, 0.25), (6, 1.0)):
        got = mlp.masked_argmin(P, M, pref=pref, margin=margin)
        base = mlp.masked_argmin(P, M)
        for r in range(300):
            if base[r] < 0:
                assert got[r] == -1
            elif M[r, pref] and P[r, pref] <= P[r, base[r]] + margin:
                assert got[r] == pref
            else:
                assert got[r] == base[r]
