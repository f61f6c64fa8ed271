"""Oracle for the product y = A x^T on the biclique format.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

The format (paper, Section "Final Remarks", after Hernandez and Navarro's
biclique extraction): the edges of G are decomposed into bicliques (S_r, C_r),
every node of S_r pointing to every node of C_r, plus a residual set of
edges; a biclique's |S_r| |C_r| edges are stored as the |S_r| + |C_r| ids of
its two sets.

`lists` writes out the adjacency lists the decomposition stands for (its
definition), so the reference product is the plain per-row sum of
``product.matvec`` over them.  `paper_product` is the paper's own algorithm:
first c_r = sum_{j in C_r} x_j for every biclique, then counters y = 0 to
which c_r is added for each i in S_r, then x_j for each residual edge
(i, j).  The two agree exactly for integer-valued x and within rounding
otherwise; the second route pins the first.
"""
from __future__ import annotations

import numpy as np


def lists(b):
    """Adjacency lists (CSR rowptr uint64, col uint32, rows ascending) of
    the graph the decomposition represents: row i holds C_r for every
    biclique r with i in S_r, and the residual targets of i.  An edge listed
    twice stays twice (the format requires a partition; tests check that no
    row repeats an id)."""
    n = int(b.n)
    rows = [[] for _ in range(n)]
    for r in range(len(b.sptr) - 1):
        S = b.sidx[int(b.sptr[r]):int(b.sptr[r + 1])]
        C = b.cidx[int(b.cptr[r]):int(b.cptr[r + 1])].tolist()
        for i in S.tolist():
            rows[i].extend(C)
    for i in range(n):
        rows[i].extend(b.rcol[int(b.rptr[i]):int(b.rptr[i + 1])].tolist())
    rp = np.zeros(n + 1, dtype=np.uint64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.asarray([j for r in rows for j in sorted(r)], dtype=np.uint32)
    return rp, col


def paper_product(b, x):
    """The paper's algorithm, in float64: c_r over each C_r, then y_i += c_r
    for i in S_r (bicliques in order), then y_i += x_j per residual edge."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(b.sptr) - 1
    c = np.zeros(nb, dtype=np.float64)
    for r in range(nb):
        C = b.cidx[int(b.cptr[r]):int(b.cptr[r + 1])].astype(np.int64)
        c[r] = np.sum(x[C]) if C.size else 0.0
    y = np.zeros(int(b.n), dtype=np.float64)
    for r in range(nb):
        S = b.sidx[int(b.sptr[r]):int(b.sptr[r + 1])].astype(np.int64)
        y[S] += c[r]
    for i in range(int(b.n)):
        R = b.rcol[int(b.rptr[i]):int(b.rptr[i + 1])].astype(np.int64)
        if R.size:
            y[i] += np.sum(x[R])
    return y


def dense(b):
    """Brute force: the dense n x n matrix, built by adding 1 on S_r x C_r for
    every biclique and on every residual edge (tiny n only).  A partition
    gives a 0/1 matrix."""
    n = int(b.n)
    A = np.zeros((n, n), dtype=np.float64)
    for r in range(len(b.sptr) - 1):
        S = b.sidx[int(b.sptr[r]):int(b.sptr[r + 1])].astype(np.int64)
        C = b.cidx[int(b.cptr[r]):int(b.cptr[r + 1])].astype(np.int64)
        A[np.ix_(S, C)] += 1.0
    for i in range(n):
        A[i, b.rcol[int(b.rptr[i]):int(b.rptr[i + 1])].astype(np.int64)] += 1.0
    return A
