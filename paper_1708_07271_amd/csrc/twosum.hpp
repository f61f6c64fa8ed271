// Compensated float pairs for the reuse chains of the FP32 two-sum mode.
//
// A value is carried as an unevaluated sum hi + lo of two floats.  two_sum is
// Knuth's TwoSum (The Art of Computer Programming, vol. 2, 4.2.2): with
// round-to-nearest float addition, s = fl(a + b) and e = (a + b) - s exactly,
// with no condition on the magnitudes of a and b.  pair_add adds two pairs:
// the TwoSum of the high parts, the low parts folded into the error term, and
// a renormalisation so that |lo| <= ulp(hi) / 2 (the fast two-sum step, valid
// because |s| >= |e| after the first step).
//
// The same steps in double (DPair, dpair_add) carry the left product's
// running window prefix, whose terms cancel (an interval adds at its start
// and subtracts at its end).
//
// Used by device code (the tile kernel's reuse levels) and compiled as host
// code by the exactness tests.
#pragma once

namespace bvmv {

struct Pair {
  float hi, lo;
};

template <class T>
__host__ __device__ __forceinline__ void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  const T bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

__host__ __device__ __forceinline__ Pair pair_add(Pair a, Pair b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  const float hi = s + e;
  return Pair{hi, e - (hi - s)};
}

struct DPair {
  double hi, lo;
};

__host__ __device__ __forceinline__ DPair dpair_add(DPair a, DPair b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  const double hi = s + e;
  return DPair{hi, e - (hi - s)};
}

}  // namespace bvmv
