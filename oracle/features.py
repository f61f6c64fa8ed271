"""Oracle for the inputs, target and restart vector of the learned PageRank
warm restart.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

The graph is held as the loaded rows B: row v lists the in-neighbours of v
(the transposed matrix that PageRank multiplies by, Section "Experimental
Evaluation"), so indeg_v = |B_v| and the out-degree d_u is the number of
rows listing u.  `stats` is how each row is coded in the compressed stream
(reference-chain depth, reference entries skipped, intervals, their total
length, residuals; Section "Our Approach"), as read by the oracle decoder.

The network sees 12 inputs per node v, all float64 here:
  structural (fixed per graph)
   0  log1p(indeg_v)                      1  log1p(d_v)
   2  depth_v / R                          3  1 if d_v = 0 else 0
   4  log1p(intervals_v)                   5  log1p(residuals_v)
   6  log1p((B d)_v / max(indeg_v, 1))     mean out-degree of v's in-neighbours
   7  log1p((B indeg)_v / max(indeg_v, 1)) mean in-degree of v's in-neighbours
  trajectory (from the last four iterates p_K, p_{K-1}, p_{K-2}, p_{K-3} of
  the power method, Eq. (1), and delta = ||p_K - p_{K-1}||_1)
   8  log(n p_K(v))
   9  n (p_K - p_{K-1})_v / delta
  10  n (p_{K-1} - p_{K-2})_v / delta
  11  n (p_{K-2} - p_{K-3})_v / delta
The network's output s_v estimates the remaining correction in the same
units, t_v = n (p*_v - p_K(v)) / delta, p* the fixed point; the restart
vector is p'_v = max(p_K(v) + s_v delta / n, p_K(v) / 1000), divided by its
sum.  The floor keeps p' positive, so every later iterate stays positive.
The two products B x use the oracle's plain definition of the product.
"""
from __future__ import annotations

import numpy as np

from . import pagerank as _pr
from . import product as _product

NFEAT = 12
NSTRUCT = 8
FLOOR = 1e-3


def structural(rowptr, col, stats, R):
    """(n, 8) float64: inputs 0..7 (see the module docstring)."""
    rowptr = np.asarray(rowptr, dtype=np.uint64)
    col = np.asarray(col)
    stats = np.asarray(stats, dtype=np.int64)
    n = len(rowptr) - 1
    indeg = np.diff(rowptr.astype(np.int64)).astype(np.float64)
    d = _pr.out_degrees(rowptr, col).astype(np.float64)
    den = np.maximum(indeg, 1.0)
    F = np.zeros((n, NSTRUCT))
    F[:, 0] = np.log1p(indeg)
    F[:, 1] = np.log1p(d)
    F[:, 2] = stats[:, 0] / float(max(R, 1))
    F[:, 3] = (d == 0).astype(np.float64)
    F[:, 4] = np.log1p(stats[:, 2])
    F[:, 5] = np.log1p(stats[:, 4])
    F[:, 6] = np.log1p(_product.matvec(rowptr, col, d) / den)
    F[:, 7] = np.log1p(_product.matvec(rowptr, col, indeg) / den)
    return F


def trajectory(pK, pK1, pK2, pK3):
    """(n, 4) float64: inputs 8..11 and delta, from the last four iterates."""
    pK, pK1, pK2, pK3 = (np.asarray(a, dtype=np.float64) for a in (pK, pK1, pK2, pK3))
    n = pK.size
    delta = float(np.sum(np.abs(pK - pK1)))
    T = np.zeros((n, 4))
    T[:, 0] = np.log(n * pK)
    T[:, 1] = n * (pK - pK1) / delta
    T[:, 2] = n * (pK1 - pK2) / delta
    T[:, 3] = n * (pK2 - pK3) / delta
    return T, delta


def target(p_star, pK, delta):
    """t_v = n (p*_v - p_K(v)) / delta."""
    p_star, pK = np.asarray(p_star, dtype=np.float64), np.asarray(pK, dtype=np.float64)
    return pK.size * (p_star - pK) / delta


def restart_vector(pK, s, delta):
    """p' = max(p_K + s delta / n, p_K / 1000), normalised to sum 1."""
    pK, s = np.asarray(pK, dtype=np.float64), np.asarray(s, dtype=np.float64)
    q = np.maximum(pK + s * delta / pK.size, FLOOR * pK)
    return q / np.sum(q)


def row_stats_from_lists(rowptr, col, refs, Lmin):
    """The coding statistics a row must have, derived from the lists alone:
    skipped = |L_r \\ L_v|; the added entries L_v \\ L_r (all of L_v without a
    reference) split into maximal runs of consecutive ids, runs of length >=
    Lmin being intervals and the rest residuals.  Depth from the references.
    Used to pin the decoder's statistics."""
    n = len(rowptr) - 1
    out = np.zeros((n, 5), dtype=np.int64)
    depth = np.zeros(n, dtype=np.int64)
    for v in range(n):
        Lv = set(int(c) for c in col[int(rowptr[v]):int(rowptr[v + 1])])
        g = int(refs[v])
        if g:
            r = v - g
            Lr = set(int(c) for c in col[int(rowptr[r]):int(rowptr[r + 1])])
            depth[v] = depth[r] + 1
            out[v, 1] = len(Lr - Lv)
            added = sorted(Lv - Lr)
        else:
            added = sorted(Lv)
        out[v, 0] = depth[v]
        nint = intlen = 0
        k = 0
        while k < len(added):
            e = k + 1
            while e < len(added) and added[e] == added[e - 1] + 1:
                e += 1
            if e - k >= Lmin:
                nint += 1
                intlen += e - k
            k = e
        out[v, 2] = nint
        out[v, 3] = intlen
        out[v, 4] = len(added) - intlen
    return out
