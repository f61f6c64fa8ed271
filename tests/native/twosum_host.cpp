// Host build of the device's compensated pair arithmetic (twosum.hpp) for the
// exactness tests: the device qualifiers are dropped, the arithmetic is the
// header's own.  Built with g++ by tests/test_host.py, without contraction or
// excess precision (SSE float arithmetic, round to nearest).
#define __host__
#define __device__
#define __forceinline__ inline
#include "twosum.hpp"

extern "C" {
void host_two_sum(const float* a, const float* b, float* s, float* e, int n) {
  for (int i = 0; i < n; ++i) bvmv::two_sum(a[i], b[i], s[i], e[i]);
}
void host_pair_add(const float* ah, const float* al, const float* bh, const float* bl, float* h, float* l, int n) {
  for (int i = 0; i < n; ++i) {
    const bvmv::Pair r = bvmv::pair_add(bvmv::Pair{ah[i], al[i]}, bvmv::Pair{bh[i], bl[i]});
    h[i] = r.hi;
    l[i] = r.lo;
  }
}
}
