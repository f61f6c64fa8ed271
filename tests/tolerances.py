"""Parity tolerances of the device paths against the CPU oracle, in one
place (relative, per entry: |y - y*| <= tol |y*|, and exactly 0 where the
oracle gives 0).

F64       1e-12   double vectors and double accumulation
F32C      1e-5    float vectors; row partials in double, reuse chains as
                  TwoSum-compensated float pairs
F32_NAIVE 1e-3    float vectors and float accumulation along reuse chains,
                  interval sums from float prefix sums: an uncompensated
                  comparison mode that does NOT meet the 1e-5 FP32 bar (its
                  error grows with chain depth and with the prefix sums'
                  magnitude; about 2e-5 on the social-like workload)

Vectors of wide dynamic range (personalized PageRank, whose entries span
dozens of orders of magnitude away from the seed nodes) take a floor on top:
the method subtracts -- a reference row's sum less its skipped entries, an
interval as P[s+len] - P[s] of the tile's window prefix -- so a row's
rounding error scales with the magnitudes its tile subtracts, not with its
own sum.  A tiny entry next to large ones therefore carries an absolute
error of a few roundings of its neighbours, and an entry the oracle gives as
exactly 0 (a node not yet reached) may hold such a residue.  The floor is a
few units in the last place of the vector's largest entry:
    |p - p*| <= tol |p*| + FLOOR[prec] * max|p*|.
"""
import numpy as np

F64 = 1e-12
F32C = 1e-5
F32_NAIVE = 1e-3

# units of max|p*|: 2^-48 is 16 double roundings of the largest entry (the
# window prefixes and reference sums a row subtracts are sums of at most a
# few hundred entries, all <= max|p*|); the two-sum mode carries reuse chains
# as TwoSum pairs of ~48 significant bits and rounds the result to float;
# the uncompensated float mode subtracts in float: 16 float roundings
FLOOR = {"f64": 2.0 ** -48, "f32c": 2.0 ** -40, "f32": 2.0 ** -20}


def within(p, p_ref, tol, floor):
    """Largest ratio |p - p*| / (tol |p*| + floor max|p*|) over all entries
    (must be <= 1), and, for the record, the largest plain relative error
    among entries the floor does not cover (p* >= floor max|p*| / tol)."""
    p = np.asarray(p, dtype=np.float64)
    p_ref = np.asarray(p_ref, dtype=np.float64)
    scale = float(np.max(np.abs(p_ref)))
    d = np.abs(p - p_ref)
    ratio = float(np.max(d / (tol * np.abs(p_ref) + floor * scale)))
    big = np.abs(p_ref) >= floor * scale / tol
    rel_big = float(np.max(d[big] / np.abs(p_ref[big]))) if np.any(big) else 0.0
    return ratio, rel_big
