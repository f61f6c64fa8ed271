"""Oracle for PageRank with learned warm restarts.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

The power method of Eq. (1) (oracle.pagerank, same readings) from the
uniform vector, interrupted every K iterations (counted from the last
restart) by a warm restart predicted per node by a network: the inputs of
oracle.features from the last four iterates, the network's estimate s of the
remaining correction, and the restart vector p'.  The plain method
decides: one iteration from p' gives q = G p' and the residual r' =
||q - p'||_1, and p' is kept only if r' < beta * delta, delta = ||p_K -
p_{K-1}||_1.  Since G is a beta-contraction in the L1 norm, the plain
method's next residual ||G p_K - p_K||_1 is at most beta * delta, so a kept
restart is never behind the bound the plain method guarantees.  A rejected
restart costs that one product, the run goes on from p_K, and no further
restart is tried.  The stopping test, ||p_t - p_{t-1}||_1 < tol, is the plain
method's, so the result has the plain method's error bound
||p_t - p*||_1 <= resid * beta / (1 - beta).
"""
from __future__ import annotations

import numpy as np

from . import features as _feat
from .pagerank import out_degrees
from .product import matvec


def pagerank_restarted(rowptr, col, predict, F_struct, beta=0.85, tol=1e-6, max_iter=1000, K=10,
                       max_restarts=2):
    """Returns (p, iters, resid, converged, info): iters counts the kept
    iterations (an accepted probe is one), info = dict(products, accepted,
    rejected) with products = iters + rejected probes.

    predict: callable mapping the (n, 12) inputs to s (n,)."""
    n = len(rowptr) - 1
    d = out_degrees(rowptr, col)
    dangling = d == 0
    inv = np.zeros(n)
    inv[~dangling] = 1.0 / d[~dangling]
    v = np.full(n, 1.0 / n)

    def step(p):
        y = matvec(rowptr, col, p * inv)
        q = (1.0 - beta) * v + beta * (y + float(np.sum(p[dangling])) * v)
        return q, float(np.sum(np.abs(q - p)))

    p = v.copy()
    hist = [p]        # the last four iterates, the newest last
    since = 0         # iterations since the start or the last kept restart
    t, rejected, accepted = 0, 0, 0
    enabled = max_restarts > 0 and K >= 3
    resid = np.inf
    while t < max_iter:
        p, resid = step(p)
        t += 1
        since += 1
        if resid < tol:
            break
        hist = (hist + [p])[-4:]
        if not (enabled and since == K and t < max_iter):
            continue
        # warm restart after K iterations since the last one
        pK, pK1, pK2, pK3 = hist[-1], hist[-2], hist[-3], hist[-4]
        Tr, delta = _feat.trajectory(pK, pK1, pK2, pK3)
        s = np.asarray(predict(np.concatenate([F_struct, Tr], axis=1)), dtype=np.float64)
        p_new = _feat.restart_vector(pK, s, delta)
        q, r = step(p_new)
        if r < beta * delta:
            accepted += 1
            p, resid = q, r
            t += 1
            if resid < tol:
                break
            hist = [p_new, q]
            since = 1
            if accepted + rejected >= max_restarts:
                enabled = False
        else:
            rejected += 1
            enabled = False
    return p, t, resid, bool(resid < tol), dict(products=t + rejected, accepted=accepted, rejected=rejected)
