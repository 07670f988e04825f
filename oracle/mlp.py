"""FP64 oracle of the learned variant selector (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product path never does.  Plain
NumPy float64, written from the definitions below and sharing nothing with
the HIP library.  The selector is an extension of this project: the paper
(which times fixed kernels) has no counterpart, so the citations are to the
standard definitions each step follows.

  features      per-block sparsity statistics from the COO pattern itself
                (distinct rows and columns, entries per row)
  linear_*      a dense layer y = x W^T + b and its chain-rule gradients
  relu          max(0, x), derivative 0 at x <= 0
  mse           masked mean squared error and its gradient
  adam          one step of Adam (Kingma and Ba, 2015, Algorithm 1)
  masked_argmin the least entry among the allowed ones, first on ties
"""
from __future__ import annotations

import numpy as np

NFEAT = 23
NBINS = 16


def _log2_floor_at_1(x: float) -> float:
    return float(np.log2(x)) if x > 1.0 else 0.0


def features(rows, cols, kz: int, bf16: bool, transpose: bool = False) -> np.ndarray:
    """Feature vector of one orientation of a block given by its COO entries.

    Entry lengths come from counting the entries of every distinct row
    (columns when transpose): entries of a row of length L fall in class
    floor(log2 L), the last class taking every longer row.  Layout:
    [0,16) class fractions of nnz, 16 log2(longest)/16, 17 log2(rows)/16,
    18 log2(cols)/16, 19 log2(nnz)/24, 20 log2(nnz/rows)/8, 21 log2(kz)/8,
    22 BF16 flag.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if transpose:
        rows, cols = cols, rows
    nnz = rows.shape[0]
    _, lens = np.unique(rows, return_counts=True)
    nrows = lens.shape[0]
    ncols = np.unique(cols).shape[0]
    f = np.zeros(NFEAT)
    for L in lens:
        b = min(int(L).bit_length() - 1, NBINS - 1)
        f[b] += L
    if nnz:
        f[:NBINS] /= nnz
    f[16] = _log2_floor_at_1(float(lens.max()) if nrows else 0.0) / 16
    f[17] = _log2_floor_at_1(float(nrows)) / 16
    f[18] = _log2_floor_at_1(float(ncols)) / 16
    f[19] = _log2_floor_at_1(float(nnz)) / 24
    f[20] = _log2_floor_at_1(nnz / nrows) / 8 if nrows else 0.0
    f[21] = _log2_floor_at_1(float(kz)) / 8
    f[22] = 1.0 if bf16 else 0.0
    return f


def linear_fwd(X, W, b=None, relu: bool = False):
    """Y = act(X W^T + b) for X [n x fin], W [fout x fin]."""
    Z = np.asarray(X, np.float64) @ np.asarray(W, np.float64).T
    if b is not None:
        Z = Z + np.asarray(b, np.float64)[None, :]
    return np.where(Z > 0, Z, 0.0) if relu else Z


def linear_bwd(X, W, Y, dY, relu: bool = False):
    """Gradients of linear_fwd: returns (dX, dW, db)."""
    X = np.asarray(X, np.float64)
    W = np.asarray(W, np.float64)
    G = np.asarray(dY, np.float64)
    if relu:
        G = np.where(np.asarray(Y) > 0, G, 0.0)
    return G @ W, G.T @ X, G.sum(axis=0)


def mse(P, T, M):
    """Masked mean squared error: (loss, dP) with c = sum M (1 when 0)."""
    P = np.asarray(P, np.float64)
    T = np.asarray(T, np.float64)
    M = np.asarray(M, np.float64)
    c = M.sum()
    c = c if c > 0 else 1.0
    D = P - T
    return float((M * D * D).sum() / c), 2.0 * M * D / c


def adam(w, g, m, v, lr, b1, b2, eps, t):
    """One Adam step at step count t >= 1: returns new (w, m, v)."""
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * np.asarray(g, np.float64)
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * np.asarray(g, np.float64) ** 2
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return np.asarray(w, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def masked_argmin(P, M, pref: int = -1, margin: float = 0.0) -> np.ndarray:
    """Per row, the index of the least P among entries with M != 0 (first on
    ties), -1 for a row with none.  With pref >= 0: pref instead when M allows
    it and P[pref] <= least + margin, the sum taken in FP32 as the device
    takes it (a preference kept unless beaten by more than margin)."""
    P = np.asarray(P)
    M = np.asarray(M)
    out = np.full(P.shape[0], -1, dtype=np.int64)
    for r in range(P.shape[0]):
        best = -1
        for o in range(P.shape[1]):
            if M[r, o] != 0 and (best < 0 or P[r, o] < P[r, best]):
                best = o
        if best >= 0 and pref >= 0 and M[r, pref] != 0:
            bound = np.float32(np.float32(P[r, best]) + np.float32(margin))
            if np.float32(P[r, pref]) <= bound:
                best = pref
        out[r] = best
    return out


def mlp_forward(layers, X):
    """layers: list of (W, b); ReLU after every layer but the last.  Returns
    the list of activations [X, h1, ..., out]."""
    acts = [np.asarray(X, np.float64)]
    for i, (W, b) in enumerate(layers):
        acts.append(linear_fwd(acts[-1], W, b, relu=i + 1 < len(layers)))
    return acts


def mlp_loss_grads(layers, X, T, M):
    """Masked MSE of the network output and its gradients [(dW, db), ...]."""
    acts = mlp_forward(layers, X)
    loss, d = mse(acts[-1], T, M)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        dX, dW, db = linear_bwd(acts[i], W, acts[i + 1], d, relu=i + 1 < len(layers))
        grads[i] = (dW, db)
        d = dX
    return loss, grads
