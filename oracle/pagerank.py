"""Oracle PageRank by the power method (paper, Section "PageRank", Eq. (1)).

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

Eq. (1): p_t = a p_0 + (1 - a) p_{t-1} M with M = D^{-1} A the random-walk
matrix and a the teleport probability.  Readings taken here:
  - `beta` is the link-following weight 1 - a (beta = 0.85 means a = 0.15);
  - the teleport vector v and the start vector are separate (the paper uses
    p_0 for both; its runs start from the uniform vector);
  - M is undefined on rows with d_u = 0 (dangling nodes); their mass
    delta = sum of p_u over dangling u is sent to v, which keeps sum(p) = 1;
  - the left product p M is taken as a right product with the transposed
    matrix, as the paper does: the input holds in-link lists, row v listing
    every u with an edge u -> v, and d_u is the number of rows u appears in;
  - iteration stops at the first t with ||p_t - p_{t-1}||_1 < tol.
"""
from __future__ import annotations

import numpy as np

from .product import matvec


def out_degrees(rowptr, col):
    """d_u = number of in-link rows that list u (column counts)."""
    n = len(rowptr) - 1
    return np.bincount(np.asarray(col, dtype=np.int64), minlength=n).astype(np.int64)


def pagerank(rowptr, col, beta=0.85, tol=1e-6, max_iter=1000, teleport=None, start=None,
             iters=None):
    """Power method in float64 on in-link lists.

    Returns (p, t, resid, converged).  With `iters` given, runs exactly that
    many iterations (no stopping test)."""
    n = len(rowptr) - 1
    d = out_degrees(rowptr, col)
    v = np.full(n, 1.0 / n) if teleport is None else np.asarray(teleport, dtype=np.float64)
    p = v.copy() if start is None else np.asarray(start, dtype=np.float64).copy()
    dangling = d == 0
    inv = np.zeros(n)
    inv[~dangling] = 1.0 / d[~dangling]
    resid = np.inf
    t = 0
    limit = iters if iters is not None else max_iter
    for t in range(1, limit + 1):
        delta = float(np.sum(p[dangling]))
        z = p * inv
        y = matvec(rowptr, col, z)                      # (p M)_v = sum_{u -> v} p_u / d_u
        p_new = (1.0 - beta) * v + beta * (y + delta * v)
        resid = float(np.sum(np.abs(p_new - p)))
        p = p_new
        if iters is None and resid < tol:
            return p, t, resid, True
    return p, t, resid, iters is not None


def pagerank_dense(out_lists_dense, beta=0.85, teleport=None):
    """Exact fixed point by a dense linear solve (tiny n; textbook form).

    out_lists_dense: n x n 0/1 matrix A with A[u, v] = 1 iff u -> v.
    S = D^{-1} A with each dangling row replaced by v^T; the fixed point of
    p = (1 - beta) v + beta p S solves (I - beta S^T) p^T = (1 - beta) v^T."""
    A = np.asarray(out_lists_dense, dtype=np.float64)
    n = A.shape[0]
    v = np.full(n, 1.0 / n) if teleport is None else np.asarray(teleport, dtype=np.float64)
    d = A.sum(axis=1)
    S = np.zeros_like(A)
    for u in range(n):
        S[u] = A[u] / d[u] if d[u] > 0 else v
    return np.linalg.solve(np.eye(n) - beta * S.T, (1.0 - beta) * v)
