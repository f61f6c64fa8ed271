// HIP kernels for the reuse product on the tiled layout, the plain CSR
// baseline, and the fused PageRank iteration.  gfx950, wave64, 256 threads.
//
// One block per tile.  A tile's rows are either direct or reuse the sum of a
// reference row inside the same tile (y_i = y_{r_i} + sum_j A'_ij x_j, the
// algorithm after the Proposition of Section "Our Approach"), so no data
// crosses tiles and the kernel needs no grid-wide synchronisation:
//   1. row info -> LDS, block scan of row lengths -> per-row word offsets,
//      list of long rows, deepest level;
//   2. the tile's 16-bit words and its x window -> LDS (coalesced), and with
//      prefix mode the exclusive prefix P of the window in double (block
//      scan), so an interval [s, s+len) costs P[s+len] - P[s];
//   3. one thread per short row walks its words, a whole block sums each
//      long row (fixed-shape tree: deterministic);
//   4. levels 1..max: y_i = y_{i-g_i} + partial_i in LDS;
//   5. epilogue: store y, or the PageRank update.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bvmv {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// ------------------------------------------------------------ precision modes
struct Pair {
  float hi, lo;
};

// Knuth's TwoSum: s + e == a + b exactly; the error is folded into lo.
__device__ __forceinline__ void two_sum_into(Pair& a, float v) {
  const float s = a.hi + v;
  const float bp = s - a.hi;
  const float e = (a.hi - (s - bp)) + (v - bp);
  a.hi = s;
  a.lo += e;
}
__device__ __forceinline__ Pair pair_add(Pair a, Pair b) {
  const float s = a.hi + b.hi;
  const float bp = s - a.hi;
  float e = (a.hi - (s - bp)) + (b.hi - bp);
  e += a.lo + b.lo;
  const float hi = s + e;
  return Pair{hi, e - (hi - s)};
}

struct MF64 {
  using X = double;
  using Acc = double;
  static constexpr bool kInt = false;
  __device__ static Acc zero() { return 0.0; }
  __device__ static void add(Acc& a, X v) { a += v; }
  __device__ static void add_d(Acc& a, double v) { a += v; }
  __device__ static Acc comb(Acc a, Acc b) { return a + b; }
  __device__ static X out(Acc a) { return a; }
  __device__ static double to_d(Acc a) { return a; }
  __device__ static Acc shfl_down(Acc a, int d) { return __shfl_down(a, d, 64); }
};
struct MF32 {
  using X = float;
  using Acc = float;
  static constexpr bool kInt = false;
  __device__ static Acc zero() { return 0.0f; }
  __device__ static void add(Acc& a, X v) { a += v; }
  __device__ static void add_d(Acc& a, double v) { a += float(v); }
  __device__ static Acc comb(Acc a, Acc b) { return a + b; }
  __device__ static X out(Acc a) { return a; }
  __device__ static double to_d(Acc a) { return a; }
  __device__ static Acc shfl_down(Acc a, int d) { return __shfl_down(a, d, 64); }
};
struct MF32C {
  using X = float;
  using Acc = Pair;
  static constexpr bool kInt = false;
  __device__ static Acc zero() { return Pair{0.0f, 0.0f}; }
  __device__ static void add(Acc& a, X v) { two_sum_into(a, v); }
  __device__ static void add_d(Acc& a, double v) {
    const float h = float(v);
    two_sum_into(a, h);
    a.lo += float(v - double(h));
  }
  __device__ static Acc comb(Acc a, Acc b) { return pair_add(a, b); }
  __device__ static X out(Acc a) { return a.hi + a.lo; }
  __device__ static double to_d(Acc a) { return double(a.hi) + double(a.lo); }
  __device__ static Acc shfl_down(Acc a, int d) {
    return Pair{__shfl_down(a.hi, d, 64), __shfl_down(a.lo, d, 64)};
  }
};
// integer counting (x = 1): degrees by reuse
struct MINT {
  using X = int32_t;
  using Acc = int32_t;
  static constexpr bool kInt = true;
  __device__ static Acc zero() { return 0; }
  __device__ static void add(Acc& a, X v) { a += v; }
  __device__ static void add_d(Acc& a, double v) { a += int32_t(v); }
  __device__ static Acc comb(Acc a, Acc b) { return a + b; }
  __device__ static X out(Acc a) { return a; }
  __device__ static double to_d(Acc a) { return a; }
  __device__ static Acc shfl_down(Acc a, int d) { return __shfl_down(a, d, 64); }
};

// ------------------------------------------------------------- block helpers
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* s_tmp, uint64_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) s_tmp[wid] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint64_t s = s_tmp[w];
    if (w < wid) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

__device__ __forceinline__ double block_excl_scan_f64(double v, double* s_tmp, double& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) s_tmp[wid] = inc;
  __syncthreads();
  double base = 0.0, tot = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const double s = s_tmp[w];
    if (w < wid) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + (inc - v);
}

// Deterministic block reduction (fixed shuffle tree, waves combined in order).
template <class M>
__device__ __forceinline__ typename M::Acc block_reduce(typename M::Acc a, typename M::Acc* s_red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) a = M::comb(a, M::shfl_down(a, d));
  if (lane == 0) s_red[wid] = a;
  __syncthreads();
  typename M::Acc r = s_red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) r = M::comb(r, s_red[w]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum_f64(double a, double* s_red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) a += __shfl_down(a, d, 64);
  if (lane == 0) s_red[wid] = a;
  __syncthreads();
  double r = s_red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) r += s_red[w];
  __syncthreads();
  return r;
}

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// LDS carve of the tile kernel
template <class M, bool PREFIX>
struct Carve {
  using X = typename M::X;
  using Acc = typename M::Acc;
  __host__ __device__ static size_t info(uint32_t) { return 0; }
  __host__ __device__ static size_t off(uint32_t t) { return align16(size_t(t) * 4); }
  __host__ __device__ static size_t list(uint32_t t) { return off(t) + align16(size_t(t) * 4); }
  __host__ __device__ static size_t part(uint32_t t) { return list(t) + align16(size_t(t) * 4); }
  __host__ __device__ static size_t y(uint32_t t) { return part(t) + align16(size_t(t) * sizeof(Acc)); }
  __host__ __device__ static size_t x(uint32_t t) { return y(t) + align16(size_t(t) * sizeof(Acc)); }
  __host__ __device__ static size_t P(uint32_t t, uint32_t w) {
    return x(t) + (M::kInt ? 0 : align16(size_t(w) * sizeof(X)));
  }
  __host__ __device__ static size_t words(uint32_t t, uint32_t w) {
    return P(t, w) + (PREFIX ? align16((size_t(w) + 1) * 8) : 0);
  }
  __host__ __device__ static size_t red(uint32_t t, uint32_t w, uint32_t e) {
    return words(t, w) + align16((size_t(e) + 16) * 2);
  }
  __host__ __device__ static size_t total(uint32_t t, uint32_t w, uint32_t e) { return red(t, w, e) + 256; }
};

struct TileCtx {
  uint32_t row0, nrows, graph, tile;
};

// ---------------------------------------------------------------- epilogues
template <class M>
struct EpiStore {
  typename M::X* y;
  __device__ void operator()(const TileCtx& tc, const typename M::Acc* s_y, unsigned char*) const {
    for (uint32_t r = threadIdx.x; r < tc.nrows; r += kThreads) y[tc.row0 + r] = M::out(s_y[r]);
  }
};

// PageRank update of Eq. (1) with dangling mass sent to the teleport vector,
// then residual and dangling partials, then the member's last block folds
// the per-tile partials (fixed order) into the member state.
template <class M>
struct EpiPR {
  PRArgs a;
  __device__ void operator()(const TileCtx& tc, const typename M::Acc* s_y, unsigned char* scratch) const {
    using X = typename M::X;
    const X* p = static_cast<const X*>(a.p_cur);
    X* pn = static_cast<X*>(a.p_new);
    X* zn = static_cast<X*>(a.z_new);
    const X* tele = static_cast<const X*>(a.tele);
    PRState* st = a.st + tc.graph;
    const double delta = st->delta, inv_n = st->inv_n, beta = a.beta;
    double rs = 0.0, dg = 0.0;
    for (uint32_t r = threadIdx.x; r < tc.nrows; r += kThreads) {
      const uint32_t v = tc.row0 + r;
      const double y = M::to_d(s_y[r]);
      const double t = tele ? double(tele[v]) : inv_n;
      const X pnew = X((1.0 - beta) * t + beta * (y + delta * t));
      pn[v] = pnew;
      const int32_t d = a.outdeg[v];
      zn[v] = d > 0 ? pnew / X(d) : X(0);
      rs += fabs(double(pnew) - double(p[v]));
      if (d == 0) dg += double(pnew);
    }
    double* s_red = reinterpret_cast<double*>(scratch);
    rs = block_sum_f64(rs, s_red);
    dg = block_sum_f64(dg, s_red);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
      a.slots[2 * size_t(tc.tile)] = rs;
      a.slots[2 * size_t(tc.tile) + 1] = dg;
      __threadfence();
      const uint32_t prev = atomicAdd(&st->ticket, 1u);
      s_last = prev + 1 == st->tile_hi - st->tile_lo;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double R = 0.0, D = 0.0;
    for (uint32_t t = st->tile_lo + threadIdx.x; t < st->tile_hi; t += kThreads) {
      R += __builtin_nontemporal_load(&a.slots[2 * size_t(t)]);
      D += __builtin_nontemporal_load(&a.slots[2 * size_t(t) + 1]);
    }
    R = block_sum_f64(R, s_red);
    D = block_sum_f64(D, s_red);
    if (threadIdx.x == 0) {
      st->resid = R;
      st->delta = D;
      st->iter += 1;
      st->ticket = 0;
      if (R < a.tol) {
        st->done = 1;
        st->converged = 1;
        st->final_buf = a.buf;
      } else if (st->iter >= a.max_iter) {
        st->done = 1;
        st->final_buf = a.buf;
      }
      __threadfence();
    }
  }
};

// --------------------------------------------------------------- tile kernel
template <class M, bool PREFIX>
__device__ __forceinline__ typename M::Acc short_row(const uint16_t* w, uint32_t len, const typename M::X* sx,
                                                     const double* sP, const typename M::X* __restrict__ x,
                                                     int64_t win0) {
  using X = typename M::X;
  typename M::Acc a = M::zero();
  uint32_t k = 0;
  while (k < len) {
    const uint32_t wd = w[k++];
    const bool neg = wd & 0x8000u;
    const uint32_t off = wd & 0x3FFFu;
    if (wd & 0x4000u) {
      const uint32_t ln = w[k++];
      if constexpr (M::kInt) {
        M::add(a, neg ? -int32_t(ln) : int32_t(ln));
      } else if constexpr (PREFIX) {
        const double d = sP[off + ln] - sP[off];
        M::add_d(a, neg ? -d : d);
      } else {
        for (uint32_t t = 0; t < ln; ++t) {
          const X v = sx[off + t];
          M::add(a, neg ? -v : v);
        }
      }
    } else {
      X v;
      if constexpr (M::kInt) {
        if (off == kEscape) k += 2;
        v = 1;
      } else if (off == kEscape) {
        const int32_t rel = int32_t((uint32_t(w[k]) << 16) | uint32_t(w[k + 1]));
        k += 2;
        v = x[win0 + rel];
      } else {
        v = sx[off];
      }
      M::add(a, neg ? -v : v);
    }
  }
  return a;
}

// Steps 1-2 shared by the single- and multi-vector kernels: row info ->
// LDS, per-row offsets (short rows: word offset; long rows: entry offset),
// the list of long rows, the deepest level, and the tile's words -> LDS.
struct RowsStaged {
  uint32_t nlong, maxlvl;
};
__device__ __forceinline__ RowsStaged stage_rows(const DevLayout& L, const TileDesc& td, uint32_t* s_info,
                                                 uint32_t* s_off, uint32_t* s_list, uint16_t* s_w,
                                                 unsigned char* s_red) {
  __shared__ uint32_t s_nlong, s_maxlvl;
  const uint32_t tid = threadIdx.x;
  const uint32_t nrows = td.nrows;
  // packed per-thread sums: short words | long count << 24 | long entries << 34
  const uint32_t per = (L.tcap + kThreads - 1) / kThreads;
  const uint32_t r_begin = tid * per;
  uint64_t local = 0;
  uint32_t lvl_max = 0;
  for (uint32_t q = 0; q < per; ++q) {
    const uint32_t r = r_begin + q;
    if (r < nrows) {
      const uint32_t inf = L.info[td.row0 + r];
      s_info[r] = inf;
      const uint64_t len = inf >> 9;
      local += (inf & kInfoLong) ? ((uint64_t(1) << 24) | (len << 34)) : len;
      lvl_max = max(lvl_max, (inf >> 4) & 15u);
    }
  }
  if (tid == 0) s_maxlvl = 0;
  __syncthreads();
  if (lvl_max) atomicMax(&s_maxlvl, lvl_max);
  uint64_t total;
  uint64_t run = block_excl_scan_u64(local, reinterpret_cast<uint64_t*>(s_red), total);
  for (uint32_t q = 0; q < per; ++q) {
    const uint32_t r = r_begin + q;
    if (r < nrows) {
      const uint32_t inf = s_info[r];
      const uint64_t len = inf >> 9;
      if (inf & kInfoLong) {
        s_off[r] = uint32_t(run >> 34);
        s_list[(run >> 24) & 1023u] = r;
        run += (uint64_t(1) << 24) | (len << 34);
      } else {
        s_off[r] = uint32_t(run & 0xFFFFFFu);
        run += len;
      }
    }
  }
  if (tid == 0) s_nlong = uint32_t((total >> 24) & 1023u);
  {
    const uint4* src = reinterpret_cast<const uint4*>(L.words + td.word0);
    uint4* dst = reinterpret_cast<uint4*>(s_w);
    const uint32_t nv = (td.nwords + 7) / 8;
    for (uint32_t k = tid; k < nv; k += kThreads) dst[k] = src[k];
  }
  __syncthreads();
  return RowsStaged{s_nlong, s_maxlvl};
}

template <class M, bool PREFIX, class Epi>
__global__ void __launch_bounds__(kThreads) bv_tile_kernel(DevLayout L, const typename M::X* __restrict__ x,
                                                           Epi epi, const PRState* __restrict__ skip_done) {
  using X = typename M::X;
  using Acc = typename M::Acc;
  using C = Carve<M, PREFIX>;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t tile = blockIdx.x;
  const TileDesc td = L.tiles[tile];
  if (skip_done && skip_done[td.graph].done) return;
  const uint32_t T = L.tcap, WC = L.wcap;
  uint32_t* s_info = reinterpret_cast<uint32_t*>(smem + C::info(T));
  uint32_t* s_off = reinterpret_cast<uint32_t*>(smem + C::off(T));
  uint32_t* s_list = reinterpret_cast<uint32_t*>(smem + C::list(T));
  Acc* s_part = reinterpret_cast<Acc*>(smem + C::part(T));
  Acc* s_y = reinterpret_cast<Acc*>(smem + C::y(T));
  X* s_x = reinterpret_cast<X*>(smem + C::x(T));
  double* s_P = reinterpret_cast<double*>(smem + C::P(T, WC));
  uint16_t* s_w = reinterpret_cast<uint16_t*>(smem + C::words(T, WC));
  unsigned char* s_red = smem + C::red(T, WC, L.ecap);
  const uint32_t tid = threadIdx.x;
  const uint32_t nrows = td.nrows;
  // 1-2. rows and words
  const RowsStaged rs = stage_rows(L, td, s_info, s_off, s_list, s_w, s_red);
  // 2b. the x window, and with prefix mode its exclusive prefix in double
  const int64_t win0 = td.win0;
  const uint32_t winlen = td.winlen;
  if constexpr (!M::kInt) {
    for (uint32_t k = tid; k < winlen; k += kThreads) s_x[k] = x[win0 + k];
  }
  if constexpr (PREFIX && !M::kInt) {
    __syncthreads();
    const uint32_t chunk = (winlen + kThreads - 1) / kThreads;
    const uint32_t b0 = min(winlen, tid * chunk), b1 = min(winlen, b0 + chunk);
    double acc = 0.0;
    for (uint32_t k = b0; k < b1; ++k) acc += double(s_x[k]);
    double tot;
    double base = block_excl_scan_f64(acc, reinterpret_cast<double*>(s_red), tot);
    for (uint32_t k = b0; k < b1; ++k) {
      s_P[k] = base;
      base += double(s_x[k]);
    }
    if (tid == 0) s_P[winlen] = tot;
  }
  __syncthreads();
  // 3a. short rows, one thread each
  for (uint32_t r = tid; r < nrows; r += kThreads) {
    const uint32_t inf = s_info[r];
    if (!(inf & kInfoLong)) s_part[r] = short_row<M, PREFIX>(s_w + s_off[r], inf >> 9, s_x, s_P, x, win0);
  }
  // 3b. long rows, the whole block each
  const uint32_t nlong = rs.nlong;
  for (uint32_t l = 0; l < nlong; ++l) {
    const uint32_t r = s_list[l];
    const uint32_t len = s_info[r] >> 9;
    const uint32_t* e = L.longs + td.long0 + s_off[r];
    Acc a = M::zero();
    for (uint32_t k = tid; k < len; k += kThreads) {
      const uint32_t v = e[k];
      X xv;
      if constexpr (M::kInt) {
        xv = 1;
      } else {
        const int64_t c = int64_t(v & 0x7FFFFFFFu) - int64_t(kLongBias);
        xv = uint64_t(c) < winlen ? s_x[c] : x[win0 + c];
      }
      M::add(a, (v & 0x80000000u) ? -xv : xv);
    }
    a = block_reduce<M>(a, reinterpret_cast<Acc*>(s_red));
    if (tid == 0) s_part[r] = a;
  }
  __syncthreads();
  // 4. reuse levels: y_i = y_{i-g} + partial_i
  for (uint32_t r = tid; r < nrows; r += kThreads)
    if (((s_info[r] >> 4) & 15u) == 0) s_y[r] = s_part[r];
  const uint32_t maxlvl = rs.maxlvl;
  for (uint32_t lv = 1; lv <= maxlvl; ++lv) {
    __syncthreads();
    for (uint32_t r = tid; r < nrows; r += kThreads) {
      const uint32_t inf = s_info[r];
      if (((inf >> 4) & 15u) == lv) s_y[r] = M::comb(s_y[r - (inf & 15u)], s_part[r]);
    }
  }
  __syncthreads();
  // 5. epilogue
  epi(TileCtx{td.row0, nrows, td.graph, tile}, s_y, s_red);
}

// PageRank start: p0 = start (or teleport, or uniform), z0 = p0 / d, dangling mass
template <class M>
__global__ void __launch_bounds__(kThreads) pr_init_kernel(const uint32_t* __restrict__ row0s, uint32_t row_stride,
                                                           const uint32_t* __restrict__ graphs, const void* start_,
                                                           const void* tele_, void* p0_, void* z0_,
                                                           const int32_t* __restrict__ outdeg, PRState* st_all,
                                                           double* slots) {
  using X = typename M::X;
  // row0s: per tile first row, stride between entries `row_stride` uint32s; nrows at +1
  const uint32_t tile = blockIdx.x;
  const uint32_t row0 = row0s[size_t(tile) * row_stride];
  const uint32_t nrows = row0s[size_t(tile) * row_stride + 1] & 0x7FFFFFFFu;
  const uint32_t graph = graphs ? graphs[size_t(tile) * row_stride] : 0u;
  PRState* st = st_all + graph;
  const X* start = static_cast<const X*>(start_);
  const X* tele = static_cast<const X*>(tele_);
  X* p0 = static_cast<X*>(p0_);
  X* z0 = static_cast<X*>(z0_);
  const double inv_n = st->inv_n;
  double dg = 0.0;
  for (uint32_t r = threadIdx.x; r < nrows; r += kThreads) {
    const uint32_t v = row0 + r;
    const X pv = start ? start[v] : (tele ? tele[v] : X(inv_n));
    p0[v] = pv;
    const int32_t d = outdeg[v];
    z0[v] = d > 0 ? pv / X(d) : X(0);
    if (d == 0) dg += double(pv);
  }
  __shared__ double s_red[kWaves];
  __shared__ int s_last;
  dg = block_sum_f64(dg, s_red);
  if (threadIdx.x == 0) {
    slots[2 * size_t(tile) + 1] = dg;
    __threadfence();
    const uint32_t prev = atomicAdd(&st->ticket, 1u);
    s_last = prev + 1 == st->tile_hi - st->tile_lo;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double D = 0.0;
  for (uint32_t t = st->tile_lo + threadIdx.x; t < st->tile_hi; t += kThreads)
    D += __builtin_nontemporal_load(&slots[2 * size_t(t) + 1]);
  D = block_sum_f64(D, s_red);
  if (threadIdx.x == 0) {
    st->delta = D;
    st->resid = 0.0;
    st->iter = 0;
    st->done = 0;
    st->converged = 0;
    st->final_buf = 0;
    st->ticket = 0;
    __threadfence();
  }
}

// ---------------------------------------------------------------- CSR kernel
// A tile is a run of short rows whose columns are staged in LDS, or one long
// row (bit 31 of nrows) summed by the whole block.
template <class M, class Epi>
__global__ void __launch_bounds__(kThreads) csr_tile_kernel(DevCsr C, const typename M::X* __restrict__ x, Epi epi,
                                                            const PRState* __restrict__ skip_done) {
  using X = typename M::X;
  using Acc = typename M::Acc;
  extern __shared__ __align__(16) unsigned char smem[];
  if (skip_done && skip_done[0].done) return;
  const uint32_t tile = blockIdx.x;
  const CsrTile td = C.tiles[tile];
  const bool is_long = td.nrows & 0x80000000u;
  const uint32_t nrows = td.nrows & 0x7FFFFFFFu;
  const uint32_t RC = C.rcap;
  uint32_t* s_rp = reinterpret_cast<uint32_t*>(smem);                          // RC + 1
  Acc* s_y = reinterpret_cast<Acc*>(smem + align16((size_t(RC) + 1) * 4));     // RC
  uint32_t* s_col = reinterpret_cast<uint32_t*>(smem + align16((size_t(RC) + 1) * 4) + align16(size_t(RC) * sizeof(Acc)));
  unsigned char* s_red = reinterpret_cast<unsigned char*>(s_col + C.ccap);
  const uint32_t tid = threadIdx.x;
  if (is_long) {
    Acc a = M::zero();
    for (uint32_t k = tid; k < td.ncols; k += kThreads) M::add(a, x[C.col[size_t(td.c0) + k]]);
    a = block_reduce<M>(a, reinterpret_cast<Acc*>(s_red));
    if (tid == 0) s_y[0] = a;
  } else {
    for (uint32_t r = tid; r <= nrows; r += kThreads) s_rp[r] = C.rowptr[td.row0 + r] - td.c0;
    for (uint32_t k = tid; k < td.ncols; k += kThreads) s_col[k] = C.col[size_t(td.c0) + k];
    __syncthreads();
    for (uint32_t r = tid; r < nrows; r += kThreads) {
      Acc a = M::zero();
      const uint32_t e = s_rp[r + 1];
      for (uint32_t k = s_rp[r]; k < e; ++k) M::add(a, x[s_col[k]]);
      s_y[r] = a;
    }
  }
  __syncthreads();
  epi(TileCtx{td.row0, nrows, 0u, tile}, s_y, s_red);
}

// ------------------------------------------------------------- dispatching
template <class M, bool PREFIX, class Epi>
hipError_t launch_tile(const DevLayout& L, const void* x, const Epi& epi, const PRState* skip, hipStream_t s) {
  using C = Carve<M, PREFIX>;
  const size_t smem = C::total(L.tcap, L.wcap, L.ecap);
  auto k = bv_tile_kernel<M, PREFIX, Epi>;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(smem));
    if (e != hipSuccess) return e;
  }
  if (L.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(L.ntiles), dim3(kThreads), smem, s, L, static_cast<const typename M::X*>(x), epi,
                     skip);
  return hipGetLastError();
}

template <class M, class Epi>
hipError_t launch_csr(const DevCsr& Cs, const void* x, const Epi& epi, const PRState* skip, hipStream_t s) {
  using Acc = typename M::Acc;
  const size_t smem = align16((size_t(Cs.rcap) + 1) * 4) + align16(size_t(Cs.rcap) * sizeof(Acc)) +
                      size_t(Cs.ccap) * 4 + 256;
  auto k = csr_tile_kernel<M, Epi>;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(smem));
    if (e != hipSuccess) return e;
  }
  if (Cs.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(Cs.ntiles), dim3(kThreads), smem, s, Cs, static_cast<const typename M::X*>(x), epi,
                     skip);
  return hipGetLastError();
}

// -------------------------------------------------------- multi-vector kernel
// Y = A X for k right-hand sides, node-major (element (v, c) at v * ld + c).
// Lanes map to right-hand sides: a team of G lanes handles one row, walking
// the row's words (broadcast LDS reads) while each lane gathers its column
// of X, so one pass over the layout serves all k products.  X is not staged
// (a window would hold G values per column); intervals are summed directly.
// Partials live in LDS as T x G accumulators and the reuse levels are
// resolved in place; right-hand sides beyond G are done in further passes
// over the staged words.
template <class M, int G>
__global__ void __launch_bounds__(kThreads) bv_batch_kernel(DevLayout L, const typename M::X* __restrict__ X,
                                                            typename M::X* __restrict__ Y, int k, int64_t ld) {
  using Xt = typename M::X;
  using Acc = typename M::Acc;
  constexpr uint32_t kTeams = kThreads / G;
  extern __shared__ __align__(16) unsigned char smem[];
  const TileDesc td = L.tiles[blockIdx.x];
  const uint32_t T = L.tcap;
  uint32_t* s_info = reinterpret_cast<uint32_t*>(smem);
  uint32_t* s_off = reinterpret_cast<uint32_t*>(smem + align16(size_t(T) * 4));
  uint32_t* s_list = reinterpret_cast<uint32_t*>(smem + 2 * align16(size_t(T) * 4));
  Acc* s_acc = reinterpret_cast<Acc*>(smem + 3 * align16(size_t(T) * 4));
  Acc* s_tmp = reinterpret_cast<Acc*>(smem + 3 * align16(size_t(T) * 4) + align16(size_t(T) * G * sizeof(Acc)));
  uint16_t* s_w = reinterpret_cast<uint16_t*>(reinterpret_cast<unsigned char*>(s_tmp) +
                                              align16(size_t(kThreads) * sizeof(Acc)));
  unsigned char* s_red = reinterpret_cast<unsigned char*>(s_w) + align16((size_t(L.ecap) + 16) * 2);
  const RowsStaged rs = stage_rows(L, td, s_info, s_off, s_list, s_w, s_red);
  const uint32_t tid = threadIdx.x, team = tid / G, lane = tid % G;
  const uint32_t nrows = td.nrows;
  const int64_t win0 = td.win0;
  for (int c0 = 0; c0 < k; c0 += G) {
    const int c = c0 + int(lane);
    const bool act = c < k;
    const Xt* Xc = X + c;
    for (uint32_t r = team; r < nrows; r += kTeams) {
      const uint32_t inf = s_info[r];
      if (inf & kInfoLong) continue;
      Acc a = M::zero();
      const uint16_t* w = s_w + s_off[r];
      const uint32_t len = inf >> 9;
      uint32_t q = 0;
      while (q < len) {
        const uint32_t wd = w[q++];
        const bool neg = wd & 0x8000u;
        const uint32_t off = wd & 0x3FFFu;
        if (wd & 0x4000u) {
          const uint32_t ln = w[q++];
          if (act)
            for (uint32_t t = 0; t < ln; ++t) {
              const Xt v = Xc[(win0 + int64_t(off + t)) * ld];
              M::add(a, neg ? -v : v);
            }
        } else {
          int64_t col = win0 + int64_t(off);
          if (off == kEscape) {
            col = win0 + int64_t(int32_t((uint32_t(w[q]) << 16) | uint32_t(w[q + 1])));
            q += 2;
          }
          if (act) {
            const Xt v = Xc[col * ld];
            M::add(a, neg ? -v : v);
          }
        }
      }
      s_acc[r * G + lane] = a;
    }
    for (uint32_t l = 0; l < rs.nlong; ++l) {
      const uint32_t r = s_list[l];
      const uint32_t len = s_info[r] >> 9;
      const uint32_t* e = L.longs + td.long0 + s_off[r];
      Acc a = M::zero();
      for (uint32_t q = team; q < len; q += kTeams) {
        const uint32_t v = e[q];
        const int64_t col = win0 + int64_t(v & 0x7FFFFFFFu) - int64_t(kLongBias);
        if (act) {
          const Xt xv = Xc[col * ld];
          M::add(a, (v & 0x80000000u) ? -xv : xv);
        }
      }
      s_tmp[team * G + lane] = a;
      __syncthreads();
      if (team == 0) {
        Acc sum = s_tmp[lane];
        for (uint32_t t = 1; t < kTeams; ++t) sum = M::comb(sum, s_tmp[t * G + lane]);
        s_acc[r * G + lane] = sum;
      }
      __syncthreads();
    }
    __syncthreads();
    for (uint32_t lv = 1; lv <= rs.maxlvl; ++lv) {
      for (uint32_t idx = tid; idx < nrows * G; idx += kThreads) {
        const uint32_t r = idx / G;
        const uint32_t inf = s_info[r];
        if (((inf >> 4) & 15u) == lv) s_acc[idx] = M::comb(s_acc[idx - (inf & 15u) * G], s_acc[idx]);
      }
      __syncthreads();
    }
    for (uint32_t idx = tid; idx < nrows * G; idx += kThreads) {
      const int cc = c0 + int(idx % G);
      if (cc < k) Y[int64_t(td.row0 + idx / G) * ld + cc] = M::out(s_acc[idx]);
    }
    __syncthreads();
  }
}

template <class M, int G>
size_t batch_smem(const DevLayout& L) {
  using Acc = typename M::Acc;
  return 3 * align16(size_t(L.tcap) * 4) + align16(size_t(L.tcap) * G * sizeof(Acc)) +
         align16(size_t(kThreads) * sizeof(Acc)) + align16((size_t(L.ecap) + 16) * 2) + 256;
}

template <class M, int G>
hipError_t launch_batch_g(const DevLayout& L, const void* X, void* Y, int k, int64_t ld, hipStream_t s) {
  const size_t smem = batch_smem<M, G>(L);
  auto kern = bv_batch_kernel<M, G>;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(smem));
    if (e != hipSuccess) return e;
  }
  if (L.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(L.ntiles), dim3(kThreads), smem, s, L, static_cast<const typename M::X*>(X),
                     static_cast<typename M::X*>(Y), k, ld);
  return hipGetLastError();
}

// Team width: the smallest power of two >= k (at least 4), shrunk until the
// T x G accumulators fit the LDS budget.
template <class M>
hipError_t launch_batch(const DevLayout& L, const void* X, void* Y, int k, int64_t ld, hipStream_t s) {
  constexpr size_t kBudget = 96 * 1024;
  int G = 4;
  while (G < k && G < 64) G *= 2;
  auto fits = [&](int g) {
    switch (g) {
      case 64: return batch_smem<M, 64>(L) <= kBudget;
      case 32: return batch_smem<M, 32>(L) <= kBudget;
      case 16: return batch_smem<M, 16>(L) <= kBudget;
      case 8: return batch_smem<M, 8>(L) <= kBudget;
      default: return true;
    }
  };
  while (G > 4 && !fits(G)) G /= 2;
  switch (G) {
    case 64: return launch_batch_g<M, 64>(L, X, Y, k, ld, s);
    case 32: return launch_batch_g<M, 32>(L, X, Y, k, ld, s);
    case 16: return launch_batch_g<M, 16>(L, X, Y, k, ld, s);
    case 8: return launch_batch_g<M, 8>(L, X, Y, k, ld, s);
    default: return launch_batch_g<M, 4>(L, X, Y, k, ld, s);
  }
}

}  // namespace

hipError_t launch_bv_multiply(const DevLayout& L, int prec, int interval_mode, const void* x, void* y,
                              hipStream_t s) {
  const bool prefix = interval_mode == 0;
  switch (prec) {
    case 0:
      return launch_tile<MF64, false>(L, x, EpiStore<MF64>{static_cast<double*>(y)}, nullptr, s);
    case 1:
      return prefix ? launch_tile<MF32, true>(L, x, EpiStore<MF32>{static_cast<float*>(y)}, nullptr, s)
                    : launch_tile<MF32, false>(L, x, EpiStore<MF32>{static_cast<float*>(y)}, nullptr, s);
    case 2:
      return prefix ? launch_tile<MF32C, true>(L, x, EpiStore<MF32C>{static_cast<float*>(y)}, nullptr, s)
                    : launch_tile<MF32C, false>(L, x, EpiStore<MF32C>{static_cast<float*>(y)}, nullptr, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_bv_degrees(const DevLayout& L, int32_t* deg, hipStream_t s) {
  return launch_tile<MINT, false>(L, nullptr, EpiStore<MINT>{deg}, nullptr, s);
}

hipError_t launch_bv_pagerank_iter(const DevLayout& L, int prec, int interval_mode, const PRArgs& a,
                                   hipStream_t s) {
  const bool prefix = interval_mode == 0;
  switch (prec) {
    case 0:
      return launch_tile<MF64, false>(L, a.z_cur, EpiPR<MF64>{a}, a.st, s);
    case 1:
      return prefix ? launch_tile<MF32, true>(L, a.z_cur, EpiPR<MF32>{a}, a.st, s)
                    : launch_tile<MF32, false>(L, a.z_cur, EpiPR<MF32>{a}, a.st, s);
    case 2:
      return prefix ? launch_tile<MF32C, true>(L, a.z_cur, EpiPR<MF32C>{a}, a.st, s)
                    : launch_tile<MF32C, false>(L, a.z_cur, EpiPR<MF32C>{a}, a.st, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_pr_init(const DevLayout& L, int prec, const void* start, const void* tele, void* p0, void* z0,
                          const int32_t* outdeg, PRState* st, double* slots, hipStream_t s) {
  if (L.ntiles == 0) return hipSuccess;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(L.tiles);
  const uint32_t stride = sizeof(TileDesc) / 4;
  const uint32_t* graphs = base + offsetof(TileDesc, graph) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(pr_init_kernel<MF64>, dim3(L.ntiles), dim3(kThreads), 0, s, base, stride, graphs, start,
                       tele, p0, z0, outdeg, st, slots);
  else
    hipLaunchKernelGGL(pr_init_kernel<MF32>, dim3(L.ntiles), dim3(kThreads), 0, s, base, stride, graphs, start,
                       tele, p0, z0, outdeg, st, slots);
  return hipGetLastError();
}

hipError_t launch_csr_multiply(const DevCsr& C, int prec, const void* x, void* y, hipStream_t s) {
  switch (prec) {
    case 0:
      return launch_csr<MF64>(C, x, EpiStore<MF64>{static_cast<double*>(y)}, nullptr, s);
    case 1:
      return launch_csr<MF32>(C, x, EpiStore<MF32>{static_cast<float*>(y)}, nullptr, s);
    case 2:
      return launch_csr<MF32C>(C, x, EpiStore<MF32C>{static_cast<float*>(y)}, nullptr, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_csr_pagerank_iter(const DevCsr& C, int prec, const PRArgs& a, hipStream_t s) {
  switch (prec) {
    case 0:
      return launch_csr<MF64>(C, a.z_cur, EpiPR<MF64>{a}, a.st, s);
    case 1:
      return launch_csr<MF32>(C, a.z_cur, EpiPR<MF32>{a}, a.st, s);
    case 2:
      return launch_csr<MF32C>(C, a.z_cur, EpiPR<MF32C>{a}, a.st, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_csr_pr_init(const DevCsr& C, int prec, const void* start, const void* tele, void* p0, void* z0,
                              const int32_t* outdeg, PRState* st, double* slots, hipStream_t s) {
  if (C.ntiles == 0) return hipSuccess;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(C.tiles);
  const uint32_t stride = sizeof(CsrTile) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(pr_init_kernel<MF64>, dim3(C.ntiles), dim3(kThreads), 0, s, base, stride, nullptr, start,
                       tele, p0, z0, outdeg, st, slots);
  else
    hipLaunchKernelGGL(pr_init_kernel<MF32>, dim3(C.ntiles), dim3(kThreads), 0, s, base, stride, nullptr, start,
                       tele, p0, z0, outdeg, st, slots);
  return hipGetLastError();
}

hipError_t launch_bv_multiply_batch(const DevLayout& L, int prec, const void* X, void* Y, int k, int64_t ld,
                                    hipStream_t s) {
  switch (prec) {
    case 0:
      return launch_batch<MF64>(L, X, Y, k, ld, s);
    case 1:
      return launch_batch<MF32>(L, X, Y, k, ld, s);
    case 2:
      return launch_batch<MF32C>(L, X, Y, k, ld, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bvmv
