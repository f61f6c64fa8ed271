"""Oracle for the per-node structural features of the learned PageRank warm start.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

The graph is held as the loaded rows B: row v lists the in-neighbours of v
(the transposed matrix that PageRank multiplies by, Section "Experimental
Evaluation"), so indeg_v = |B_v| and the out-degree d_u is the number of
rows listing u.  `stats` is how each row is coded in the compressed stream
(reference-chain depth, reference entries skipped, intervals, their total
length, residuals; Section "Our Approach"), as read by the oracle decoder.

Features of node v, all float64:
   0  log1p(indeg_v)                      1  log1p(d_v)
   2  depth_v / R                          3  1 if d_v = 0 else 0
   4  log1p(skipped_v)                     5  log1p(intervals_v)
   6  log1p(interval length_v)             7  log1p(residuals_v)
   8  log1p((B d)_v / max(indeg_v, 1))     the mean out-degree of v's in-neighbours
   9  log1p((B indeg)_v / max(indeg_v, 1)) the mean in-degree of v's in-neighbours
  10  log1p(n (B invd)_v), invd_u = 1/d_u (0 if d_u = 0): n times one
      link-following step from the uniform vector (Eq. (1) without teleport)
  11  log(n)
The three products B x use the oracle's plain definition of the product.
"""
from __future__ import annotations

import numpy as np

from . import pagerank as _pr
from . import product as _product

NFEAT = 12


def features(rowptr, col, stats, R):
    """(n, 12) float64 feature matrix (see the module docstring)."""
    rowptr = np.asarray(rowptr, dtype=np.uint64)
    col = np.asarray(col)
    stats = np.asarray(stats, dtype=np.int64)
    n = len(rowptr) - 1
    indeg = np.diff(rowptr.astype(np.int64)).astype(np.float64)
    d = _pr.out_degrees(rowptr, col).astype(np.float64)
    invd = np.zeros(n)
    invd[d > 0] = 1.0 / d[d > 0]
    den = np.maximum(indeg, 1.0)
    F = np.zeros((n, NFEAT))
    F[:, 0] = np.log1p(indeg)
    F[:, 1] = np.log1p(d)
    F[:, 2] = stats[:, 0] / float(max(R, 1))
    F[:, 3] = (d == 0).astype(np.float64)
    F[:, 4] = np.log1p(stats[:, 1])
    F[:, 5] = np.log1p(stats[:, 2])
    F[:, 6] = np.log1p(stats[:, 3])
    F[:, 7] = np.log1p(stats[:, 4])
    F[:, 8] = np.log1p(_product.matvec(rowptr, col, d) / den)
    F[:, 9] = np.log1p(_product.matvec(rowptr, col, indeg) / den)
    F[:, 10] = np.log1p(n * _product.matvec(rowptr, col, invd))
    F[:, 11] = np.log(float(n))
    return F


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
