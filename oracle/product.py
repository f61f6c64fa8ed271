"""Oracle for the product y = A x^T on a binary adjacency matrix.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

What is computed (paper, Section "Introduction" and Section "PageRank"):
A is the n x n binary adjacency matrix, A_ij = 1 iff j is in row i's list,
and y_i = sum over j in row i of x_j.  The method reaches exactly this
result in exact arithmetic (the Proposition of Section "Our Approach"), so
the oracle is the definition itself, in float64.

`reuse_product` is the paper's own sequential algorithm on the difference
form (A', r) (Section "Our Approach", the three-step algorithm after the
Proposition, with the fallback rule of Section "Experimental Evaluation"
that keeps v_i whenever |v_i - v_{r_i}| >= |v_i|).  It serves as a second,
independent route that pins the Proposition, not as the reference result.

`left_matvec` is the left product y = x A of PageRank's p M (Section
"PageRank"), by its definition; `left_reuse_product` reaches it through the
same difference form, x A = x (I - R)^{-1} A'.
"""
from __future__ import annotations

import math

import numpy as np


def matvec_exact(rowptr, col, x):
    """y_i = sum_{j in L_i} x_j, each row correctly rounded (math.fsum)."""
    n = len(rowptr) - 1
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        if b > a:
            y[i] = math.fsum(x[col[a:b]].tolist())
    return y


def matvec_rows(rowptr, col, x, rows):
    """Correctly rounded y_i for the given rows only (sampled checks at full size)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(len(rows), dtype=np.float64)
    for k, i in enumerate(rows):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        out[k] = math.fsum(x[col[a:b]].tolist()) if b > a else 0.0
    return out


def matvec(rowptr, col, x):
    """y = A x in float64 with numpy: gather, then one sequential sum per row."""
    n = len(rowptr) - 1
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    deg = np.diff(np.asarray(rowptr, dtype=np.int64))
    nz = np.flatnonzero(deg > 0)
    if nz.size:
        vals = x[np.asarray(col, dtype=np.int64)]
        y[nz] = np.add.reduceat(vals, np.asarray(rowptr, dtype=np.int64)[nz])
    return y


def matvec_dense(rowptr, col, x):
    """Brute force: build the dense 0/1 matrix and multiply (tiny n only)."""
    n = len(rowptr) - 1
    A = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        A[i, col[int(rowptr[i]):int(rowptr[i + 1])]] = 1.0
    return A @ np.asarray(x, dtype=np.float64)


def difference_form(rowptr, col, refs):
    """The difference matrix A' and referencing vector r of the paper.

    Row i of A' is v_i - v_{r_i}: +1 on entries of v_i missing from the
    reference row, -1 on entries of the reference row that v_i lacks.  When
    |v_i - v_{r_i}| >= |v_i| the row keeps v_i itself (no reference), as in
    the paper's experiments.  Returns (r, plus, minus, m_prime) with r[i] = -1
    for "no reference" (the paper's v_0 = 0)."""
    n = len(rowptr) - 1
    r = np.full(n, -1, dtype=np.int64)
    plus, minus = [], []
    m_prime = 0
    for i in range(n):
        vi = set(col[int(rowptr[i]):int(rowptr[i + 1])].tolist())
        g = int(refs[i])
        if g > 0:
            ri = i - g
            vr = set(col[int(rowptr[ri]):int(rowptr[ri + 1])].tolist())
            add, sub = sorted(vi - vr), sorted(vr - vi)
            if len(add) + len(sub) < len(vi):
                r[i] = ri
                plus.append(add)
                minus.append(sub)
                m_prime += len(add) + len(sub)
                continue
        plus.append(sorted(vi))
        minus.append([])
        m_prime += len(vi)
    return r, plus, minus, m_prime


def reuse_product(r, plus, minus, x):
    """The paper's algorithm: y = 0, y_0 = 0; for i in order,
    y_i = y_{r_i} + sum_j A'_ij x_j (r_i < i, so y_{r_i} is already known)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(r)
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        base = y[r[i]] if r[i] >= 0 else 0.0
        y[i] = base + math.fsum(x[plus[i]].tolist()) - math.fsum(x[minus[i]].tolist())
    return y


# ------------------------------------------------------------ left products
# PageRank multiplies a row vector by the matrix (Section "PageRank", p M):
# the left product y = x A, y_j = sum over the rows i that list j of x_i.

def left_matvec(rowptr, col, x):
    """y = x A in float64: each column's terms summed in ascending row order."""
    n = len(rowptr) - 1
    x = np.asarray(x, dtype=np.float64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(rowptr, dtype=np.int64)))
    return np.bincount(np.asarray(col, dtype=np.int64), weights=x[rows], minlength=n).astype(np.float64)


def left_matvec_exact(rowptr, col, x):
    """y = x A, each column correctly rounded (math.fsum over its rows)."""
    n = len(rowptr) - 1
    x = np.asarray(x, dtype=np.float64)
    terms = [[] for _ in range(n)]
    for i in range(n):
        for j in col[int(rowptr[i]):int(rowptr[i + 1])].tolist():
            terms[j].append(x[i])
    return np.array([math.fsum(t) for t in terms], dtype=np.float64)


def left_reuse_product(r, plus, minus, x):
    """x A through the difference form (A', r): row i of A is row i of A' plus
    row r_i of A, so A = (I - R)^{-1} A' with R_ik = [r_i = k], and
    x A = c A' with c = x (I - R)^{-1}, i.e. c_k = x_k + the sum of c_i over
    the rows i that reference k; since r_i < i, c is final once taken from
    the last row down.  Then y_j = sum_i c_i A'_ij: +c_i on the entries row i
    adds, -c_i on the reference entries it drops."""
    x = np.asarray(x, dtype=np.float64)
    n = len(r)
    c = x.copy()
    for i in range(n - 1, -1, -1):
        if r[i] >= 0:
            c[r[i]] += c[i]
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        for j in plus[i]:
            y[j] += c[i]
        for j in minus[i]:
            y[j] -= c[i]
    return y
