"""fp64 reference for the strategy-selector network -- TEST INFRASTRUCTURE ONLY.

The selector is a fully connected network 6 -> 64 -> 64 -> k with ReLU after
the two hidden layers and a linear output: one predicted log-time per scan
strategy.  Training minimises the masked mean squared error
    loss = sum_{i,j} m_ij (out_ij - y_ij)^2 / sum_{i,j} m_ij
(m_ij = 1 where strategy j was timed on row i) with Adam (Kingma and Ba,
"Adam: A Method for Stochastic Optimization", 2015, Algorithm 1).

Parameter layout shared with the GPU kernels through plain arrays (not code):
W1 [64, 6], b1 [64], W2 [64, 64], b2 [64], W3 [k, 64], b3 [k], row-major,
flattened in that order.  Every function is plain numpy in float64.
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 6, 64


def n_params(k: int) -> int:
    return D_H * D_IN + D_H + D_H * D_H + D_H + k * D_H + k


def unflatten(theta: np.ndarray, k: int):
    theta = np.asarray(theta, dtype=np.float64)
    shapes = [(D_H, D_IN), (D_H,), (D_H, D_H), (D_H,), (k, D_H), (k,)]
    out, off = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(theta[off:off + size].reshape(s))
        off += size
    if off != len(theta):
        raise ValueError("parameter vector has the wrong length")
    return out


def flatten(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, x, k: int):
    """Returns (out, cache): out[i, j] = predicted log-time of strategy j for row i."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, k)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3.T + b3
    return out, (x, z1, h1, z2, h2)


def loss(theta, x, y, mask, k: int) -> float:
    out, _ = forward(theta, x, k)
    m = np.asarray(mask, dtype=np.float64)
    return float(np.sum(m * (out - y) ** 2) / np.sum(m))


def backward(theta, x, y, mask, k: int):
    """(loss, gradient of the loss w.r.t. the flattened parameters) by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, k)
    out, (x, z1, h1, z2, h2) = forward(theta, x, k)
    m = np.asarray(mask, dtype=np.float64)
    denom = np.sum(m)
    diff = out - np.asarray(y, dtype=np.float64)
    L = float(np.sum(m * diff * diff) / denom)
    dout = 2.0 * m * diff / denom
    gW3 = dout.T @ h2
    gb3 = dout.sum(axis=0)
    dz2 = (dout @ W3) * (z2 > 0.0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0.0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return L, flatten([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta', m', v')."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def argmin_strategy(pred, valid=None) -> np.ndarray:
    """Index of the smallest predicted time per row, ties to the lowest index;
    strategies with valid == False are never chosen."""
    p = np.array(pred, dtype=np.float64, copy=True)
    if valid is not None:
        p[~np.asarray(valid, dtype=bool)] = np.inf
    return np.argmin(p, axis=1)


def choose_with_margin(pred, valid, heuristic, margin: float) -> np.ndarray:
    """The selector's choice per row with a fallback margin: the heuristic's
    class h unless pred[h] exceeds the smallest valid prediction by at least
    `margin` (then the argmin over the valid classes, ties to the lowest
    index).  margin = 0 is the plain argmin."""
    p = np.array(pred, dtype=np.float64, copy=True)
    valid = np.asarray(valid, dtype=bool)
    h = np.asarray(heuristic, dtype=np.int64)
    best = argmin_strategy(p, valid)
    rows = np.arange(p.shape[0])
    pm = np.where(valid, p, np.inf)
    keep = valid[rows, h] & (p[rows, h] - pm[rows, best] < margin)
    return np.where(keep, h, best)


# ------------------------------------------------------------- features
def features(b: int, n: int, enc: int, zmin, zmax, lo, hi, counts=None) -> np.ndarray:
    """Selector features of one column, from its zone maps only.

    zmin/zmax are the per-block min/max in the domain the predicate is tested
    in (values for frame-of-reference and delta, codes for dictionary, with
    [lo, hi) already mapped to codes); counts are the valid values per block
    (1024 except a short tail).
      f0 = b / 32
      f1 = log2(n) / 24
      f2 = log10(max(s, 1e-6)) / 6, where s = sum_k c_k * overlap_k / n is the
           selectivity estimated by assuming values spread evenly over each
           block's [min, max]: overlap_k = |[lo,hi) & [min_k, max_k+1)| / (max_k - min_k + 1)
      f3 = fraction of blocks whose [min, max] meets [lo, hi)
      f4 = 1 - mean_k(max_k - min_k) / (max_k(max) - min_k(min) + 1)   (clustering)
      f5 = encoding / 2   (0 frame of reference, 0.5 delta, 1 dictionary)
    """
    zmin = np.asarray(zmin, dtype=np.float64)
    zmax = np.asarray(zmax, dtype=np.float64)
    nb = len(zmin)
    if counts is None:
        counts = np.full(nb, 1024.0)
        counts[-1] = n - 1024 * (nb - 1)
    counts = np.asarray(counts, dtype=np.float64)
    lo, hi = float(lo), float(hi)
    if lo < hi:
        width = zmax - zmin + 1.0
        ov = np.clip(np.minimum(hi, zmax + 1.0) - np.maximum(lo, zmin), 0.0, None) / width
        s = float(np.sum(counts * ov) / n)
        frac = float(np.mean(~((zmax < lo) | (zmin >= hi))))
    else:
        s, frac = 0.0, 0.0
    spread = float(np.max(zmax) - np.min(zmin) + 1.0)
    clust = 1.0 - float(np.mean(zmax - zmin)) / spread
    return np.array([b / 32.0, np.log2(n) / 24.0, np.log10(max(s, 1e-6)) / 6.0, frac, clust,
                     enc / 2.0])
