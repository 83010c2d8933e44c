"""Reference k-nearest-neighbour roadmap (PRM) construction.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU leg, never by the
library.

A PRM roadmap connects every sample to its k nearest samples in configuration space and
validates those connections as motions (the PRM of Sec. III-E, measured in Sec. IV, Table II;
the planner itself is outside this repository).  Nearest neighbours use the Euclidean norm of
the configuration difference (Sec. III-E).

Precision reading: a neighbour list is an integer decision taken on floating-point distances,
so the reference takes it in the same FP32 arithmetic the GPU kernel uses, written out
step by step: d_j = x_j - y_j rounded to FP32, then s = s + d_j * d_j accumulated in joint
order with the product and the sum each rounded to FP32 (no fused multiply-add).  Ties in
distance go to the lower sample index.  Independent FP64 checks live in the tests.
"""
from __future__ import annotations

import numpy as np


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
