"""Reference k-nearest-neighbour roadmap (PRM) construction.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU leg, never by the
library.

A PRM roadmap connects every sample to its k nearest samples in configuration space and
validates those connections as motions (the PRM of Sec. III-E, measured in Sec. IV, Table II;
the planner itself is outside this repository).  Nearest neighbours use the Euclidean norm of
the configuration difference (Sec. III-E).

Two references live here.

* `knn_exact` is the definition: squared Euclidean distances of the FP32 samples evaluated in
  FP64 (exact up to FP64 rounding, about 1e-15 relative), neighbours in ascending distance with
  equal distances going to the lower sample index.  A sample with a non-finite coordinate is
  nobody's neighbour.  This is the parity reference of the GPU lists.
* `knn` takes the same decision in FP32 arithmetic written out step by step: d_j = x_j - y_j
  rounded to FP32, then s = s + d_j * d_j accumulated in joint order with the product and the
  sum each rounded to FP32 (no fused multiply-add).  It is a second, determinism reference: it
  says which of two candidates whose exact distances lie within FP32 rounding of each other a
  fixed-order FP32 evaluation picks.

`fp32_rel_bound(dim)` bounds how far any FP32 evaluation of the squared distance in that order
can be from the exact value, relative to it: each difference and each square is one rounding,
and the dim - 1 additions of positive terms add at most one rounding each, so the relative
error is at most (1 + u)^(dim + 2) - 1 with u = 2^-24.  Two candidates whose exact squared
distances a < b satisfy b - a > bound * (a + b) are ordered the same way by every such
evaluation; closer pairs are "near ties".
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def fp32_rel_bound(dim: int) -> float:
    """Relative error bound of an FP32 squared distance over `dim` coordinates (see above)."""
    return (1.0 + U32) ** (dim + 2) - 1.0


def dist2_exact(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances between rows of x [n][d] and rows of y [m][d], in FP64."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    s = np.zeros((x.shape[0], y.shape[0]), np.float64)
    for j in range(x.shape[1]):
        d = x[:, j][:, None] - y[:, j][None, :]
        s += d * d
    return s


def knn_exact(x: np.ndarray, k: int, rows=None):
    """The k nearest other samples of each row of x [n][d] (FP32 values, distances in FP64).

    Returns idx [r][k] (int32, -1 where a row has fewer than k neighbours), d2 [r][k] (FP64
    squared distances, +inf for missing entries) and d2_next [r] (the (k+1)-th smallest squared
    distance, +inf if there is none), for r = n rows or the rows listed in `rows`.  Order:
    ascending distance, equal distances to the lower index."""
    x = np.asarray(x, np.float32)
    n = x.shape[0]
    if k < 1:
        raise ValueError("need k >= 1")
    q = np.arange(n) if rows is None else np.asarray(rows)
    finite = np.all(np.isfinite(x), axis=1)
    idx = np.full((len(q), k), -1, np.int32)
    d2 = np.full((len(q), k), np.inf, np.float64)
    d2_next = np.full(len(q), np.inf, np.float64)
    for r, i in enumerate(q):
        if not finite[i]:
            continue
        s = dist2_exact(x[i:i + 1], x)[0]
        s[~finite] = np.inf
        s[i] = np.inf                               # a sample is not its own neighbour
        order = np.lexsort((np.arange(n), s))       # by distance, then by index
        take = [int(j) for j in order[:k + 1] if np.isfinite(s[j])]
        for m, j in enumerate(take[:k]):
            idx[r, m] = j
            d2[r, m] = s[j]
        if len(take) > k:
            d2_next[r] = s[take[k]]
    return idx, d2, d2_next


def dist2_f32(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Squared distances between rows of x [n][d] and rows of y [m][d], FP32, joint order."""
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    s = np.zeros((x.shape[0], y.shape[0]), np.float32)
    for j in range(x.shape[1]):
        d = (x[:, j][:, None] - y[:, j][None, :]).astype(np.float32)
        s = (s + (d * d).astype(np.float32)).astype(np.float32)
    return s


def knn(x: np.ndarray, k: int, rows=None):
    """Indices [n][k] and FP32 squared distances of the k nearest other samples of each row
    (ascending distance, ties by index).  Samples at a non-finite distance are not neighbours;
    slots left without one hold index -1 and distance +inf.  `rows` restricts the queries to a
    subset."""
    x = np.asarray(x, np.float32)
    n = x.shape[0]
    if k < 1:
        raise ValueError("need k >= 1")
    q = np.arange(n) if rows is None else np.asarray(rows)
    idx = np.full((len(q), k), -1, np.int32)
    d2 = np.full((len(q), k), np.inf, np.float32)
    kk = min(k, n)
    with np.errstate(invalid="ignore", over="ignore"):
        for b0 in range(0, len(q), 256):
            qb = q[b0:b0 + 256]
            s = dist2_f32(x[qb], x)
            s[~np.isfinite(s)] = np.inf
            s[np.arange(len(qb)), qb] = np.inf        # a sample is not its own neighbour
            order = np.lexsort((np.broadcast_to(np.arange(n), s.shape), s), axis=1)[:, :kk]
            dd = np.take_along_axis(s, order, axis=1)
            order = np.where(np.isfinite(dd), order, -1)
            idx[b0:b0 + 256, :kk] = order
            d2[b0:b0 + 256, :kk] = dd
    return idx, d2


def knn_pairs(idx: np.ndarray) -> np.ndarray:
    """Undirected roadmap edges from kNN lists, one slot per (i, m): slot i*k+m holds (i, j) for
    j = idx[i][m] when i < j or when i is not among j's neighbours, else (-1, -1), so every
    undirected edge is listed exactly once, in a fixed order.  Entries outside [0, n) or equal
    to i leave their slot empty."""
    idx = np.asarray(idx)
    n, k = idx.shape
    out = np.full((n * k, 2), -1, np.int32)
    for i in range(n):
        for m in range(k):
            j = int(idx[i, m])
            if j < 0 or j >= n or j == i:
                continue
            if i < j or i not in idx[j]:
                out[i * k + m] = (i, j)
    return out
