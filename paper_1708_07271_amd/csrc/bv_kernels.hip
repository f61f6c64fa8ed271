// HIP kernels for the reuse product on the tiled layout, the plain CSR
// baseline, the fused PageRank iteration and the multi-vector product.
// gfx950, wave64.
//
// Single-vector kernels: a tile of up to 128 rows is processed by one
// wavefront, one or two rows per lane, with no block-wide barrier; a
// 256-thread block holds 4 consecutive tiles.  A tile's rows are direct or reuse the
// sum of a reference row inside the same tile (y_i = y_{r_i} +
// sum_j A'_ij x_j, the algorithm after the Proposition of Section "Our
// Approach"), so tiles are independent:
//   1. every global load of the tile is issued at once: the lane's row info,
//      the three entry streams (16-byte vectors), the x window;
//   2. a wave scan of the per-row counts gives the stream offsets; with
//      prefix mode an exclusive prefix P of the window (double) turns an
//      interval [s, s+len) into P[s+len] - P[s];
//   3. singles and wide entries are summed by tagged flat passes: each lane
//      takes an equal contiguous chunk of entries whatever the row lengths,
//      reads it 16 bytes at a time and cuts it at row ends, which the row
//      owners mark beforehand with a one-byte tag per entry; a row split over
//      several lanes is completed by its owner, which adds the pieces in lane
//      order (deterministic);
//   4. each lane adds its row's intervals; long rows are summed by the whole
//      wave (fixed reduction tree);
//   5. reuse levels 1..max: y_i = y_{i-g_i} + partial_i in LDS;
//   6. epilogue: store y, or the PageRank update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "kernels.hpp"
#include "twosum.hpp"

namespace bvmv {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
static_assert(kWaves == kTilesPerBlock, "one tile per wavefront");

// ------------------------------------------------------------ precision modes
// (Pair and pair_add, the TwoSum-compensated chain sums, are in twosum.hpp)

// PAcc accumulates a row's partial sum; CAcc carries sums along reuse chains.
struct MF64 {
  using X = double;
  using PAcc = double;
  using CAcc = double;
  static constexpr bool kInt = false;
  __device__ static PAcc pzero() { return 0.0; }
  __device__ static void padd(PAcc& a, X v) { a += v; }
  __device__ static void padd_d(PAcc& a, double v) { a += v; }
  __device__ static PAcc pcomb(PAcc a, PAcc b) { return a + b; }
  __device__ static PAcc pshfl_down(PAcc a, int d) { return __shfl_down(a, d, 64); }
  __device__ static PAcc pbcast(PAcc a, int l) { return __shfl(a, l, 64); }
  __device__ static CAcc chain(PAcc a) { return a; }
  __device__ static CAcc comb(CAcc a, CAcc b) { return a + b; }
  __device__ static X out(CAcc a) { return a; }
  __device__ static X add_out(X y, CAcc a) { return y + a; }
  __device__ static double to_d(CAcc a) { return a; }
};
// float everywhere: the naive mode (window values and prefix sums are read
// from the staged doubles and rounded to float)
struct MF32 {
  using X = float;
  using PAcc = float;
  using CAcc = float;
  static constexpr bool kInt = false;
  __device__ static PAcc pzero() { return 0.0f; }
  __device__ static void padd(PAcc& a, X v) { a += v; }
  __device__ static void padd_d(PAcc& a, double v) { a += float(v); }
  __device__ static PAcc pcomb(PAcc a, PAcc b) { return a + b; }
  __device__ static PAcc pshfl_down(PAcc a, int d) { return __shfl_down(a, d, 64); }
  __device__ static PAcc pbcast(PAcc a, int l) { return __shfl(a, l, 64); }
  __device__ static CAcc chain(PAcc a) { return a; }
  __device__ static CAcc comb(CAcc a, CAcc b) { return a + b; }
  __device__ static X out(CAcc a) { return a; }
  __device__ static X add_out(X y, CAcc a) { return y + a; }
  __device__ static double to_d(CAcc a) { return a; }
};
// float vectors; a row's partial in double (one add per entry), reuse chains
// as (hi, lo) float pairs with TwoSum compensation
struct MF32C {
  using X = float;
  using PAcc = double;
  using CAcc = Pair;
  static constexpr bool kInt = false;
  __device__ static PAcc pzero() { return 0.0; }
  __device__ static void padd(PAcc& a, X v) { a += double(v); }
  __device__ static void padd_d(PAcc& a, double v) { a += v; }
  __device__ static PAcc pcomb(PAcc a, PAcc b) { return a + b; }
  __device__ static PAcc pshfl_down(PAcc a, int d) { return __shfl_down(a, d, 64); }
  __device__ static PAcc pbcast(PAcc a, int l) { return __shfl(a, l, 64); }
  __device__ static CAcc chain(PAcc a) {
    const float h = float(a);
    return Pair{h, float(a - double(h))};
  }
  __device__ static CAcc comb(CAcc a, CAcc b) { return pair_add(a, b); }
  __device__ static X out(CAcc a) { return a.hi + a.lo; }
  __device__ static X add_out(X y, CAcc a) { return float((double(y) + double(a.hi)) + double(a.lo)); }
  __device__ static double to_d(CAcc a) { return double(a.hi) + double(a.lo); }
};
// integer counting with x = 1: degrees by reuse
struct MINT {
  using X = int32_t;
  using PAcc = int32_t;
  using CAcc = int32_t;
  static constexpr bool kInt = true;
  __device__ static PAcc pzero() { return 0; }
  __device__ static void padd(PAcc& a, X v) { a += v; }
  __device__ static void padd_d(PAcc& a, double v) { a += int32_t(v); }
  __device__ static PAcc pcomb(PAcc a, PAcc b) { return a + b; }
  __device__ static PAcc pshfl_down(PAcc a, int d) { return __shfl_down(a, d, 64); }
  __device__ static PAcc pbcast(PAcc a, int l) { return __shfl(a, l, 64); }
  __device__ static CAcc chain(PAcc a) { return a; }
  __device__ static CAcc comb(CAcc a, CAcc b) { return a + b; }
  __device__ static X out(CAcc a) { return a; }
  __device__ static X add_out(X y, CAcc a) { return y + a; }
  __device__ static double to_d(CAcc a) { return a; }
};

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }
__device__ __forceinline__ uint32_t dalign16u(uint32_t b) { return (b + 15u) & ~15u; }

// ------------------------------------------------------------- wave helpers
// LDS written by some lanes of a wave and read by others: keep the order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t wave_excl_scan_u64(uint64_t v, uint64_t& total) {
  const uint32_t lane = lane_id();
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t t = __shfl_up(inc, d, 64);
    if (lane >= uint32_t(d)) inc += t;
  }
  total = __shfl(inc, 63, 64);
  return inc - v;
}

// fixed shuffle tree, result broadcast to all lanes
template <class M>
__device__ __forceinline__ typename M::PAcc wave_reduce(typename M::PAcc a) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) a = M::pcomb(a, M::pshfl_down(a, d));
  return M::pbcast(a, 0);
}

__device__ __forceinline__ double wave_sum_f64(double a) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) a += __shfl_down(a, d, 64);
  return __shfl(a, 0, 64);
}

// One wave copies nbytes (a multiple of 16) from global to LDS with 16-byte
// vector loads; each lane issues kBatch loads before its first LDS write, so
// a tile pays one memory round trip, not one per loop turn.  src and dst are
// 16-byte aligned.
template <int kBatch>
__device__ __forceinline__ void wave_copy16(const void* __restrict__ src, void* dst, uint32_t nbytes) {
  const uint32_t lane = lane_id();
  const uint32_t nv = nbytes / 16;
  const uint4* s = static_cast<const uint4*>(src);
  uint4* d = static_cast<uint4*>(dst);
  // Loads are unconditional (lanes past the end re-read the last vector) so
  // that the batch stays in registers.
  for (uint32_t base = 0; base < nv; base += 64 * kBatch) {
    uint4 r[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) r[j] = s[min(base + lane + 64u * j, nv - 1)];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint32_t k = base + lane + 64u * j;
      if (k < nv) d[k] = r[j];
    }
  }
}

// Stage elements [first, first + count) of a global array of `len` elements
// into the LDS buffer `buf` (room for count + 16 bytes); returns the LDS
// address of element `first`.  Whole 16-byte vectors when the array is
// aligned and they stay inside it, else batched element loads.
template <class T>
__device__ __forceinline__ T* stage_range(const T* __restrict__ arr, uint64_t len, int64_t first, uint32_t count,
                                          T* buf) {
  constexpr uint32_t V = 16 / sizeof(T);
  const int64_t a0 = first & ~int64_t(V - 1);
  const uint32_t shift = uint32_t(first - a0);
  const uint32_t total = shift + count;
  const uint32_t vec_elems = (total + V - 1) / V * V;
  if ((reinterpret_cast<uintptr_t>(arr) & 15u) == 0 && uint64_t(a0) + vec_elems <= len) {
    wave_copy16<4>(arr + a0, buf, vec_elems * uint32_t(sizeof(T)));
  } else {
    const uint32_t lane = lane_id();
    for (uint32_t base = 0; base < total; base += 64 * 8) {
      T r[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t k = base + lane + 64u * j;
        if (k < total) r[j] = arr[a0 + k];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t k = base + lane + 64u * j;
        if (k < total) buf[k] = r[j];
      }
    }
  }
  return buf + shift;
}

// q = floor(a / C) for an entry offset a of a flat pass (a < 64 C) and its
// chunk length C < 2^14, from invC within 1 ulp of 1 / C: (a + 1/2) / C lies
// at least 1 / (2C) > 3e-5 from every integer, while one fused multiply-add
// of a value below 65 errs by less than 2e-5.
__device__ __forceinline__ uint32_t div_small(uint32_t a, uint32_t /*C*/, float invC) {
  return uint32_t(fmaf(float(a), invC, 0.5f * invC));
}

// Inclusive wave scan of a u32 by DPP row shifts and row broadcasts (no LDS).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  int x = int(v);
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false); // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false); // row_bcast:31 into rows 2, 3
  return uint32_t(x);
}

// One DPP step of a double scan: the value of the lane `ctrl` selects
// (0 outside the row or in rows the row mask leaves out) is added.
template <int kCtrl, int kRowMask, bool kBound>
__device__ __forceinline__ double dpp_add_f64(double v) {
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), kCtrl, kRowMask, 0xf, kBound));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), kCtrl, kRowMask, 0xf, kBound));
  return v + __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// Inclusive wave scan of a double (same DPP pattern as the u32 scan).
__device__ __forceinline__ double wave_incl_scan_f64(double v) {
  v = dpp_add_f64<0x111, 0xf, true>(v);
  v = dpp_add_f64<0x112, 0xf, true>(v);
  v = dpp_add_f64<0x114, 0xf, true>(v);
  v = dpp_add_f64<0x118, 0xf, true>(v);
  v = dpp_add_f64<0x142, 0xa, false>(v);
  v = dpp_add_f64<0x143, 0xc, false>(v);
  return v;
}

// set bits of m in the lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

// Chunk length of a flat pass over E entries: ceil(E / 64) rounded up to a
// multiple of `Q` (so that a lane's chunk starts on a 4-byte boundary of a
// u16 stream, Q = 2, or on a 4-entry boundary of the CSR tags, Q = 4).
template <uint32_t Q>
__device__ __forceinline__ uint32_t flat_chunk(uint32_t E) { return ((E + 63) / 64 + Q - 1) / Q * Q; }

constexpr int kRound = 8;  // stream dwords a lane has in flight per round of a flat pass
static_assert(kDataPadBytes >= 4 * kRound, "a round may read kRound dwords past a stream's last dword");

// Load dwords first .. first + kRound - 1 of a stream, clamped to its last
// dword: every word is an entry of the stream (end_pass decodes whole rounds,
// gathers included, before it stops at the lane's chunk end).
__device__ __forceinline__ void load_round(const uint32_t* __restrict__ g, uint32_t first, uint32_t last,
                                           uint32_t (&d)[kRound]) {
#pragma unroll
  for (int k = 0; k < kRound; ++k) d[k] = g[min(first + uint32_t(k), last)];
}

// Load dwords f .. f + kRound - 1, f = min(first, last), with one address and
// immediate offsets.  Dwords past `last` belong to the next stream or to the
// zero padding of at least kRound dwords that ends the device data array, so
// the loads stay in bounds; only for passes that zero every word past the
// lane's chunk before decoding it (the running-sum singles pass).
__device__ __forceinline__ void load_round_raw(const uint32_t* __restrict__ g, uint32_t first, uint32_t last,
                                               uint32_t (&d)[kRound]) {
  const uint32_t* q = g + min(first, last);
#pragma unroll
  for (int k = 0; k < kRound; ++k) d[k] = q[k];
}

// Geometry of a lane's chunk of a flat pass: P entries per dword, the chunk
// [b, b + C) clipped to the E entries, nd dwords from dword d0 on, and the
// stream's last dword.
template <uint32_t P>
struct Chunk {
  uint32_t b, nd, d0, last;
  __device__ Chunk(uint32_t E, uint32_t C) {
    b = lane_id() * C;
    const uint32_t cnt = b < E ? min(E, b + C) - b : 0u;
    nd = (cnt + P - 1) / P;
    d0 = b / P;
    last = E ? (E + P - 1) / P - 1 : 0u;
  }
};

// Flat pass of one wave over a stream of E entries (P per dword) whose last
// entry in every row carries the row-end bit kEnd.  Lane l sums its chunk
// [l*C, min(E, (l+1)*C)) in order, kRound dwords per round (the first round,
// `pre`, loaded by the caller ahead of other work): every value of the round
// is read first, then the running sum takes them in order.  At a row end the
// running sum -- that row's piece in this chunk -- goes to seg[slot] and
// restarts, slot counting the rows that end in the stream from `slot0` on
// (the lane's exclusive count of row ends); the sum left at the chunk end
// goes to carry[l].  A row that starts in an earlier chunk is completed by
// its owner (flat_row_sum): no lane waits on another inside the loop, and the
// summation order is fixed.  Dwords past the chunk are clamped copies of
// stream words (their values are read but not added); with u16 words the
// chunk's last dword may hold the zero padding word after the stream's end,
// which `val` maps to 0.
template <class M, uint32_t P, uint32_t kEnd, class ValFn, class AddFn>
__device__ __forceinline__ void end_pass(uint32_t E, uint32_t C, const uint32_t* __restrict__ g,
                                         const uint32_t (&pre)[kRound], uint32_t slot0, typename M::PAcc* seg,
                                         typename M::PAcc* carry, ValFn val, AddFn add) {
  using PAcc = typename M::PAcc;
  const Chunk<P> ch(E, C);
  if (ch.nd == 0) return;
  PAcc a = M::pzero();
  uint32_t slot = slot0;
  auto round = [&](const uint32_t (&d)[kRound], uint32_t r) {
    decltype(val(0u)) v[kRound * P];
#pragma unroll
    for (int k = 0; k < kRound; ++k)
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) v[k * P + h] = val(P == 2 ? (h ? d[k] >> 16 : d[k] & 0xFFFFu) : d[k]);
#pragma unroll
    for (int k = 0; k < kRound; ++k) {
      if (r + uint32_t(k) >= ch.nd) break;
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        add(a, v[k * P + h]);
        if ((P == 2 ? (h ? d[k] >> 16 : d[k]) : d[k]) & kEnd) {
          seg[slot++] = a;
          a = M::pzero();
        }
      }
    }
  };
  round(pre, 0);
  for (uint32_t r = kRound; r < ch.nd; r += kRound) {
    uint32_t q[kRound];
    load_round(g, ch.d0 + r, ch.last, q);
    round(q, r);
  }
  carry[lane_id()] = a;
}

// Row ends inside the lane's chunk of an end-bit stream (see end_pass);
// kZeroed: the words of `pre` past the chunk are already 0.
template <uint32_t P, uint32_t m, bool kZeroed = false>
__device__ __forceinline__ uint32_t chunk_ends(uint32_t E, uint32_t C, const uint32_t* __restrict__ g,
                                               const uint32_t (&pre)[kRound]) {
  const Chunk<P> ch(E, C);
  uint32_t n = 0;
#pragma unroll
  for (int k = 0; k < kRound; ++k) n += __popc(kZeroed || uint32_t(k) < ch.nd ? pre[k] & m : 0u);
  for (uint32_t r = kRound; r < ch.nd; ++r) n += __popc(g[ch.d0 + r] & m);
  return n;
}

// Bit-field extract and the sign word of an entry as single VALU operations
// (the compiler otherwise rewrites them into shift-and-mask pairs).
template <int O, int W>
__device__ __forceinline__ uint32_t vbfe(uint32_t d) {
  uint32_t r;
  asm("v_bfe_u32 %0, %1, %2, %3" : "=v"(r) : "v"(d), "i"(O), "i"(W));
  return r;
}
// high word of +-1.0: 0x3FF00000 with the sign bit of d's bit 15 (h = 0) or 31 (h = 1)
template <int H>
__device__ __forceinline__ uint32_t sign_word(uint32_t d, uint32_t one_hi, uint32_t sign_mask) {
  uint32_t r;
  if constexpr (H == 0) {
    const uint32_t b = vbfe<15, 1>(d);
    asm("v_lshl_or_b32 %0, %1, 31, %2" : "=v"(r) : "v"(b), "v"(one_hi));
  } else {
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(sign_mask), "v"(d), "v"(one_hi));
  }
  return r;
}

// Load dwords first .. first + kRound - 1 of a stream (first <= last: the
// words past it are in bounds as for load_round); those at or past `end` (the
// end of the lane's chunk) read as 0: an entry that adds Z[0] = 0 and ends no
// row.
__device__ __forceinline__ void load_round_z(const uint32_t* __restrict__ g, uint32_t first, uint32_t end,
                                             uint32_t last, uint32_t (&d)[kRound]) {
  const uint32_t* q = g + min(first, last);
#pragma unroll
  for (int k = 0; k < kRound; ++k) {
    const uint32_t w = q[k];
    d[k] = first + uint32_t(k) < end ? w : 0u;
  }
}

// Singles pass of the two-sum mode by running sums.  Lane l adds its chunk's
// entries in order into one double that is never reset, and stores the
// running value after every entry at *p.  p starts at seg + slot0, slot0 =
// (row ends in earlier chunks) + l, and steps past every row end, so each of
// the lane's slots ends up holding the running sum at one row end, and the
// slot after its last row end the running sum at the chunk's end (each lane
// has one slot more than its row ends).  Rows are read back as differences
// (run_row_sum); the running sums stay within a few rows' sums, far inside
// the mode's tolerance.  An entry's sign enters as a factor +-1 built from
// its sign bit.  Rounds of kRound dwords are taken two dwords at a time while
// some lane of the wave has them (`pre` and later rounds load the dwords past
// the lane's chunk as 0).
__device__ __forceinline__ void run_pass(uint32_t ndmax, const Chunk<2>& ch, const uint32_t* __restrict__ g,
                                         const uint32_t (&pre)[kRound], uint32_t slot0, double* seg,
                                         const double* Z) {
  double acc = 0.0;
  double* p = seg + slot0;
  const uint32_t one_hi = 0x3FF00000u, sign_mask = 0x80000000u;
  // entry H (0: bits 0..15, 1: bits 16..31) of dword d: 14 bits of f, the
  // row-end bit, the sign bit
  auto entry = [&](auto hc, uint32_t d, double v) {
    constexpr int H = decltype(hc)::value;
    const double sg = __hiloint2double(int(sign_word<H>(d, one_hi, sign_mask)), 0);
    acc = fma(sg, v, acc);
    *p = acc;
    p += vbfe<16 * H + 14, 1>(d);
  };
  using H0 = std::integral_constant<int, 0>;
  using H1 = std::integral_constant<int, 1>;
  auto round = [&](const uint32_t (&d)[kRound], uint32_t r) {
#pragma unroll
    for (int k = 0; k < kRound; k += 2) {
      if (r + uint32_t(k) >= ndmax) break;
      const double v0 = Z[d[k] & kS16Off], v1 = Z[vbfe<16, 14>(d[k])];
      const double v2 = Z[d[k + 1] & kS16Off], v3 = Z[vbfe<16, 14>(d[k + 1])];
      entry(H0{}, d[k], v0);
      entry(H1{}, d[k], v1);
      entry(H0{}, d[k + 1], v2);
      entry(H1{}, d[k + 1], v3);
    }
  };
  round(pre, 0);
  for (uint32_t r = kRound; r < ndmax; r += kRound) {
    uint32_t q[kRound];
    load_round_z(g, ch.d0 + r, ch.d0 + ch.nd, ch.last, q);
    round(q, r);
  }
}

// Owner side of run_pass: the sum of the owner's row, entries [ob, oe) with
// oe > ob, whose end is row end number gi of the stream (its rank among the
// rows that have entries).  In every chunk l from L0 to L1 the row's running
// sum sits in slot gi + l (the row's end in chunk L1, the chunk's end in the
// others), less the running sum at the previous row's end when that lies in
// chunk L0 (the row does not start the chunk).
__device__ __forceinline__ double run_row_sum(uint32_t ob, uint32_t oe, uint32_t C, float invC, uint32_t gi,
                                              const double* seg) {
  const uint32_t L0 = div_small(ob, C, invC), L1 = div_small(oe - 1, C, invC);
  double s = seg[gi + L0];
  for (uint32_t l = L0 + 1; l <= L1; ++l) s += seg[gi + l];
  if (ob != L0 * C) s -= seg[gi - 1 + L0];
  return s;
}

// Owner side of a flat pass: the sum of the owner's row occupying entries
// [ob, oe) (oe > ob) of a pass with chunk length C: the pieces of the earlier
// chunks it spans (carry, in lane order), then its final piece.
template <class M>
__device__ __forceinline__ typename M::PAcc flat_row_sum(uint32_t ob, uint32_t oe, uint32_t C, float invC,
                                                         typename M::PAcc last, const typename M::PAcc* carry) {
  const uint32_t L0 = div_small(ob, C, invC), L1 = div_small(oe - 1, C, invC);
  if (L1 == L0) return last;
  typename M::PAcc s = carry[L0];
  for (uint32_t l = L0 + 1; l < L1; ++l) s = M::pcomb(s, carry[l]);
  return M::pcomb(s, last);
}

// Fill n bytes (n a multiple of 16) of LDS with 0xFF.
__device__ __forceinline__ void wave_fill_ff(uint8_t* dst, uint32_t n) {
  uint4* d = reinterpret_cast<uint4*>(dst);
  const uint4 ff = make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint32_t k = lane_id(); k < n / 16; k += 64) d[k] = ff;
}

// per-wave LDS carve of the tile kernel (bytes from the wave's base); a
// wave holds up to 64 * RPL rows, RPL consecutive rows per lane
template <class M, int RPL>
struct WaveCarve {
  using X = typename M::X;
  using PAcc = typename M::PAcc;
  using CAcc = typename M::CAcc;
  static constexpr uint32_t kRows = 64 * RPL;
  uint32_t WC;
  // y shares the pieces' slots: they are read by their owners before the
  // reuse levels write y
  static constexpr size_t kSlot = sizeof(PAcc) > sizeof(CAcc) ? sizeof(PAcc) : sizeof(CAcc);
  __host__ __device__ static constexpr size_t seg() { return 0; }
  __host__ __device__ static constexpr size_t y() { return 0; }
  // kRows + 64 slots: the running-sum pass keeps one more slot per lane.  A
  // pass cut at row-end bits has at most one piece per row, so its 64 lane
  // carries take the slots past the rows (the wide pass starts after the
  // running sums are read).
  __host__ __device__ static constexpr size_t carry() { return kRows * sizeof(PAcc); }
  static_assert(kRows * sizeof(PAcc) + 64 * sizeof(PAcc) <= (kRows + 64) * kSlot, "carries inside the slots");
  // the window array Z, placed 8 bytes past a 16-byte boundary so that Z + 1
  // is 16-byte aligned
  __host__ __device__ static constexpr size_t Z() { return align16((kRows + 64) * kSlot) + 8; }
  __host__ __device__ size_t wave_bytes() const { return align16(Z() + (M::kInt ? 0 : (2 * size_t(WC) + 2) * 8)); }
  // the waves' regions, then the block's PageRank partials (two doubles a wave)
  __host__ __device__ size_t block_bytes() const { return kWaves * wave_bytes() + kWaves * 16; }
};

struct TileCtx {
  uint32_t row0, nrows, graph;
  uint32_t slot;  // the block partial's slot (PageRank epilogue)
};

// ---------------------------------------------------------------- epilogues
// Every wave of the block calls them (a wave may have no rows).  In the tile
// kernel: block_start(block, member, s_blk) runs first, with every thread of
// the block (the fused PageRank's fold); prepare(tc) runs once per wave before the tile is decoded and
// returns per-lane state; fetch(tc, c) issues vector c's global loads ahead
// of their use (vector 0 with the tile's own loads, vector c + 1 while c is
// summed); skip(st, c) passes over vector c and all_done(st) over the whole
// tile (both block-uniform); col(...) takes vector c's sums; finish(...) runs
// once per block after the last vector, with every wave present.  operator()
// is the CSR kernel's one-call form.
constexpr int kEpiRows = kTileRowsMax / 64;  // rows of a tile per lane

// y = the rows' sums, or with kAdd y += them (one product of a sum of
// column blocks, taken in block order)
template <class M, bool kAdd = false>
struct EpiStore {
  typename M::X* y;
  __device__ void block_start(uint32_t, uint32_t, unsigned char*) const {}
  struct State {};
  struct Fetch {};
  __device__ State prepare(const TileCtx&) const { return {}; }
  __device__ Fetch fetch(const TileCtx&, int) const { return {}; }
  __device__ bool skip(const State&, int) const { return false; }
  __device__ bool all_done(const State&) const { return false; }
  __device__ void store(const TileCtx& tc, const typename M::CAcc* s_y) const {
    for (uint32_t r = lane_id(); r < tc.nrows; r += 64) {
      if constexpr (kAdd)
        y[tc.row0 + r] = M::add_out(y[tc.row0 + r], s_y[r]);
      else
        y[tc.row0 + r] = M::out(s_y[r]);
    }
  }
  __device__ void col(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char*, int, State&,
                      const Fetch&) const {
    store(tc, s_y);
  }
  __device__ void finish(const State&, unsigned char*, size_t, uint32_t) const {}
  __device__ void operator()(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char*, int) const {
    store(tc, s_y);
  }
};

// The block's residual and dangling partials go to its slot with plain
// stores; pr_finish_kernel folds a member's slots, in a fixed order, after the
// launch (the kernel boundary makes them visible: no device-scope fence,
// which on a multi-XCD part would write back the L2 once per block).
__device__ __forceinline__ void pr_block_partial(double rs, double dg, double* slots, unsigned char* s_blk,
                                                 uint32_t slot) {
  double* blk = reinterpret_cast<double*>(s_blk);
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  if (lane == 0) {
    blk[2 * wave] = rs;
    blk[2 * wave + 1] = dg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double R = blk[0], D = blk[1];
    for (int w = 1; w < kWaves; ++w) {
      R += blk[2 * w];
      D += blk[2 * w + 1];
    }
    slots[2 * size_t(slot)] = R;
    slots[2 * size_t(slot) + 1] = D;
  }
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), l), hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), l);
  return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// The fold of one member's block partials (residual and dangling sums) in
// one fixed order: 256 threads, thread t adding slots blk_lo + t, + 256, ...
// in sequence, each wave's sums by the shuffle reduction, then the four
// waves in order.  Every fold below gives the same two doubles bit for bit:
// fold_block with a whole block, fold_wave with one wave taking the four
// waves' threads in turn.
struct Fold {
  double R, D;
};

// (every thread of the block calls it; s_red: 4 double2 of LDS, free again
// after the caller's next __syncthreads; kU loads in flight per thread, which
// does not change the order of the sums)
template <int kU = 16>
__device__ __forceinline__ Fold fold_block(const PRState& st, const double* __restrict__ slots, double2* s_red) {
  // each thread's slots t, t + 256, ... in batches of kU loads in flight
  const double2* sl = reinterpret_cast<const double2*>(slots) + st.slot0;
  const uint32_t hi = st.blk_hi;
  double R = 0.0, D = 0.0;
  for (uint32_t b = st.blk_lo + threadIdx.x; b < hi; b += kThreads * kU) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t t = b + uint32_t(u) * kThreads;
      v[u] = t < hi ? sl[t] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      R += v[u].x;
      D += v[u].y;
    }
  }
  R = wave_sum_f64(R);
  D = wave_sum_f64(D);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = make_double2(R, D);
  __syncthreads();
  Fold f{s_red[0].x, s_red[0].y};
  for (int w = 1; w < kWaves; ++w) {
    f.R += s_red[w].x;
    f.D += s_red[w].y;
  }
  return f;
}

// (the same sums from one wave; the zero terms fold_block adds past the
// last slot leave its non-negative sums unchanged)
__device__ __forceinline__ Fold fold_wave(const PRState& st, const double* __restrict__ slots) {
  const double2* sl = reinterpret_cast<const double2*>(slots) + st.slot0;
  const uint32_t hi = st.blk_hi;
  Fold f{0.0, 0.0};
  for (int w = 0; w < kWaves; ++w) {
    double R = 0.0, D = 0.0;
    for (uint32_t b = st.blk_lo + uint32_t(w) * 64u + lane_id(); b < hi; b += kThreads) {
      const double2 v = sl[b];
      R += v.x;
      D += v.y;
    }
    R = wave_sum_f64(R);
    D = wave_sum_f64(D);
    if (w == 0) {
      f = Fold{R, D};
    } else {
      f.R += R;
      f.D += D;
    }
  }
  return f;
}

// A member's state after a fold: after an iteration (with_resid = 1; the
// folded iterate is in buffer buf) the stopping test, else the start state,
// whose iteration count is iter0 (nonzero when a run resumes from a restart
// vector).
__device__ __forceinline__ void pr_apply(PRState& st, const Fold& f, int with_resid, double tol, int32_t max_iter,
                                         int32_t buf, int32_t iter0) {
  st.delta = f.D;
  if (with_resid) {
    st.resid_prev = st.resid;
    st.resid = f.R;
    st.iter += 1;
    if (f.R < tol) {
      st.done = 1;
      st.converged = 1;
      st.final_buf = buf;
    } else if (st.iter >= max_iter) {
      st.done = 1;
      st.final_buf = buf;
    }
  } else {
    st.resid = 0.0;
    st.resid_prev = 0.0;
    st.iter = iter0;
    st.done = 0;
    st.converged = 0;
    st.final_buf = 0;
    st.pending = 0;
  }
}

// One block per member: the member's residual and dangling mass from its
// blocks' slots, then the stopping test (with_resid = 1, after an iteration;
// members already done were skipped by the iteration and are left alone) or
// the start state (with_resid = 0, after pr_init_kernel).
__global__ void __launch_bounds__(kThreads) pr_finish_kernel(PRState* st_all, const double* __restrict__ slots,
                                                             int with_resid, double tol, int32_t max_iter,
                                                             int32_t buf, int32_t iter0) {
  __shared__ double2 s_red[kWaves];
  PRState* st = st_all + blockIdx.x;
  if (with_resid && st->done) return;
  PRState F = *st;
  const Fold f = fold_block(F, slots, s_red);
  if (threadIdx.x == 0) {
    pr_apply(F, f, with_resid, tol, max_iter, buf, iter0);
    *st = F;
  }
}

// The published value of a fused iteration (below): the dangling mass of
// the iterate being multiplied, kPubDone once the member has converged, or
// the not-yet-published pattern (a NaN).
constexpr double kPubDone = -1.0;
__device__ __forceinline__ double pub_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pub_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double pub_unset() { return __longlong_as_double(int64_t(-1)); }

// After a run of fused iterations the last iterate's partials are still
// unfolded (pending): one block per member folds them into the member's state
// (the run has even length, so that iterate is in buffer 0 and its partials
// in the slots of parity 0), and both published values are cleared for the
// next run.  A member without blocks (no rows) folds zeros.
__global__ void __launch_bounds__(kThreads) pr_flush_kernel(PRState* st_all, const double* __restrict__ slots,
                                                            double tol, int32_t max_iter, double* pub) {
  __shared__ double2 s_red[kWaves];
  PRState* st = st_all + blockIdx.x;
  PRState F = *st;
  if (!F.done && (F.pending || F.blk_lo == F.blk_hi)) {
    const Fold f = fold_block(F, slots, s_red);
    if (threadIdx.x == 0) pr_apply(F, f, 1, tol, max_iter, 0, 0);
  }
  if (threadIdx.x == 0) {
    F.pending = 0;
    *st = F;
    pub[2 * size_t(blockIdx.x)] = pub_unset();
    pub[2 * size_t(blockIdx.x) + 1] = pub_unset();
  }
}

// PageRank update of Eq. (1), dangling mass sent to the teleport vector.
// With a.fused the dangling mass of the iterate being multiplied comes from
// the member's published value (block_start), not from its state.
template <class M>
struct EpiPR {
  PRArgs a;
  // parity of the iterate being multiplied
  __device__ int32_t cur() const { return 1 - a.buf; }

  // Fused iterations: the first block of each member folds the partials of
  // the iterate being multiplied (if not folded yet), writes the member's
  // next state and publishes the dangling mass, or kPubDone; every thread of
  // every block calls it first (s_blk: 64 bytes of LDS).
  __device__ void block_start(uint32_t block, uint32_t graph, unsigned char* s_blk) const {
    if (!a.fused) return;
    const PRState* st = a.st + graph;
    if (block != st->blk_lo) return;  // (block-uniform)
    PRState F = *st;
    if (!F.done && F.pending) {
      // (8 loads in flight per thread: the fold's registers stay below the tile's)
      const Fold f = fold_block<8>(F, a.slots_prev, reinterpret_cast<double2*>(s_blk));
      pr_apply(F, f, 1, a.tol, a.max_iter, cur(), 0);
    }
    if (threadIdx.x == 0) {
      F.pending = F.done ? 0 : 1;
      a.st_next[graph] = F;
      pub_store(a.pub + 2 * size_t(graph) + (1 - cur()), pub_unset());
      pub_store(a.pub + 2 * size_t(graph) + cur(), F.done ? kPubDone : F.delta);
    }
    __syncthreads();
  }

  // The dangling mass for this iteration (fused): the published value (a
  // first read `early` taken with the tile's loads), or, when it is still
  // unset after a.pub_polls reads, the same fold done by this wave from the
  // same state and partials.  kPubDone: the member has converged.
  __device__ double resolve(uint32_t graph, double early) const {
    const double* pp = a.pub + 2 * size_t(graph) + cur();
    double v = a.pub_polls < 0 ? pub_unset() : readlane_f64(early, 0);
    for (int k = 0; k < a.pub_polls && __builtin_isnan(v); ++k) {
      if (k) __builtin_amdgcn_s_sleep(8);
      v = readlane_f64(pub_load(pp), 0);
    }
    if (__builtin_isnan(v)) {
      PRState F = a.st[graph];
      if (!F.done && F.pending) pr_apply(F, fold_wave(F, a.slots_prev), 1, a.tol, a.max_iter, cur(), 0);
      v = F.done ? kPubDone : F.delta;
    }
    return v;
  }

  __device__ void operator()(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char* s_blk, int) const {
    using X = typename M::X;
    const X* p = static_cast<const X*>(a.p_cur);
    X* pn = static_cast<X*>(a.p_new);
    X* zn = static_cast<X*>(a.z_new);
    const X* tele = static_cast<const X*>(a.tele);
    PRState* st = a.st + tc.graph;
    double delta = st->delta;
    if (a.fused) {
      delta = resolve(tc.graph, pub_load(a.pub + 2 * size_t(tc.graph) + cur()));
      if (delta < 0.0) return;  // converged: every wave of the block returns
    }
    const double inv_n = st->inv_n, beta = a.beta;
    double rs = 0.0, dg = 0.0;
    for (uint32_t r = lane_id(); r < tc.nrows; r += 64) {
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
    rs = wave_sum_f64(rs);
    dg = wave_sum_f64(dg);
    pr_block_partial(rs, dg, a.slots, s_blk, tc.slot);
  }
  // the tile kernel's form: out-degrees, p and the teleport values are loaded
  // with the tile's own loads (rows past the tile read element 0), and with
  // fused iterations a first read of the published dangling mass
  using X = typename M::X;
  struct State {
    int32_t d[kEpiRows];
    double delta, inv_n;  // the member's dangling mass and 1/n
    double pub0;
  };
  struct Fetch {
    X p[kEpiRows], t[kEpiRows];
  };
  __device__ State prepare(const TileCtx& tc) const {
    State S;
    const PRState* st = a.st + tc.graph;
    S.delta = st->delta;
    S.inv_n = st->inv_n;
    S.pub0 = a.fused ? pub_load(a.pub + 2 * size_t(tc.graph) + cur()) : 0.0;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane_id() + 64u * q;
      S.d[q] = a.outdeg[r < tc.nrows ? tc.row0 + r : 0u];
    }
    return S;
  }
  __device__ Fetch fetch(const TileCtx& tc, int) const {
    const X* p = static_cast<const X*>(a.p_cur);
    const X* tele = static_cast<const X*>(a.tele);
    Fetch f;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane_id() + 64u * q;
      const uint32_t v = r < tc.nrows ? tc.row0 + r : 0u;
      f.p[q] = p[v];
      f.t[q] = tele ? tele[v] : X(0);
    }
    return f;
  }
  __device__ bool skip(const State&, int) const { return false; }
  __device__ bool all_done(const State&) const { return false; }
  __device__ void col(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char* s_blk, int, State& S,
                      const Fetch& f) const {
    X* pn = static_cast<X*>(a.p_new) + tc.row0;
    X* zn = static_cast<X*>(a.z_new) + tc.row0;
    double delta = S.delta;
    if (a.fused) {
      delta = resolve(tc.graph, S.pub0);
      if (delta < 0.0) return;  // converged: every wave of the block returns
    }
    const double inv_n = S.inv_n, beta = a.beta;
    double rs = 0.0, dg = 0.0;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane_id() + 64u * q;
      if (r < tc.nrows) {
        const double y = M::to_d(s_y[r]);
        const double t = a.tele ? double(f.t[q]) : inv_n;
        const X pnew = X((1.0 - beta) * t + beta * (y + delta * t));
        pn[r] = pnew;
        const int32_t d = S.d[q];
        zn[r] = d > 0 ? pnew / X(d) : X(0);
        rs += fabs(double(pnew) - double(f.p[q]));
        if (d == 0) dg += double(pnew);
      }
    }
    rs = wave_sum_f64(rs);
    dg = wave_sum_f64(dg);
    pr_block_partial(rs, dg, a.slots, s_blk, tc.slot);
  }
  __device__ void finish(const State&, unsigned char*, size_t, uint32_t) const {}
};

// Multi-vector epilogues (the same interface).

// Column c of a column-major block (leading dimension ld) for the tile's rows.
template <class M>
struct EpiStoreCols {
  typename M::X* y;
  int64_t ld;
  __device__ void block_start(uint32_t, uint32_t, unsigned char*) const {}
  struct State {};
  struct Fetch {};
  __device__ State prepare(const TileCtx&) const { return {}; }
  __device__ Fetch fetch(const TileCtx&, int) const { return {}; }
  __device__ bool skip(const State&, int) const { return false; }
  __device__ bool all_done(const State&) const { return false; }
  __device__ void col(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char*, int c, State&,
                      const Fetch&) const {
    typename M::X* yc = y + int64_t(c) * ld + tc.row0;
    for (uint32_t r = lane_id(); r < tc.nrows; r += 64) yc[r] = M::out(s_y[r]);
  }
  __device__ void finish(const State&, unsigned char*, size_t, uint32_t) const {}
};

// Personalized PageRank update of Eq. (1) for right-hand sides c = 0 .. k-1
// (k <= 64): each its own teleport column, dangling mass and stopping state
// st[c]; p, z and the teleport vectors are column-major with leading
// dimension n.  Lane c of every wave holds column c's state (read once) and
// the wave's residual and dangling partial sums of column c; finish() adds
// the block's waves and stores column c's pair to slot c * blocks + block.
// Columns that are done are passed over and their slots left alone.
template <class M>
struct EpiPRCols {
  using X = typename M::X;
  PRArgs a;
  int64_t n;
  __device__ void block_start(uint32_t, uint32_t, unsigned char*) const {}
  struct State {
    uint64_t done;  // bit c: column c is done
    double delta, inv_n, rs, dg;
    int32_t d[kEpiRows];  // out-degrees of the lane's rows lane + 64 q
  };
  struct Fetch {
    X p[kEpiRows], t[kEpiRows];  // p and the teleport value of the lane's rows
  };
  __device__ State prepare(const TileCtx& tc) const {
    const uint32_t lane = lane_id();
    const bool has = lane < uint32_t(a.k);
    const PRState* st = a.st + (has ? lane : 0u);
    State S;
    S.delta = st->delta;
    S.inv_n = st->inv_n;
    S.done = __ballot(has && st->done != 0);
    S.rs = 0.0;
    S.dg = 0.0;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane + 64u * q;
      S.d[q] = a.outdeg[r < tc.nrows ? tc.row0 + r : 0u];
    }
    return S;
  }
  // (rows past the tile read element 0: every address is in bounds)
  __device__ Fetch fetch(const TileCtx& tc, int c) const {
    const X* p = static_cast<const X*>(a.p_cur);
    const X* tele = static_cast<const X*>(a.tele);
    Fetch f;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane_id() + 64u * q;
      const int64_t e = r < tc.nrows ? int64_t(c) * n + tc.row0 + r : 0;
      f.p[q] = p[e];
      f.t[q] = tele ? tele[e] : X(0);
    }
    return f;
  }
  __device__ bool skip(const State& S, int c) const { return (S.done >> c) & 1u; }
  __device__ bool all_done(const State& S) const {
    return S.done == (a.k >= 64 ? ~uint64_t(0) : (uint64_t(1) << a.k) - 1);
  }
  __device__ void col(const TileCtx& tc, const typename M::CAcc* s_y, unsigned char*, int c, State& S,
                      const Fetch& f) const {
    const int64_t base = int64_t(c) * n + tc.row0;
    X* pn = static_cast<X*>(a.p_new) + base;
    X* zn = static_cast<X*>(a.z_new) + base;
    const double delta = readlane_f64(S.delta, c), inv_n = readlane_f64(S.inv_n, c), beta = a.beta;
    double rs = 0.0, dg = 0.0;
#pragma unroll
    for (int q = 0; q < kEpiRows; ++q) {
      const uint32_t r = lane_id() + 64u * q;
      if (r < tc.nrows) {
        const double y = M::to_d(s_y[r]);
        const double t = a.tele ? double(f.t[q]) : inv_n;
        const X pnew = X((1.0 - beta) * t + beta * (y + delta * t));
        pn[r] = pnew;
        const int32_t d = S.d[q];
        zn[r] = d > 0 ? pnew / X(d) : X(0);
        rs += fabs(double(pnew) - double(f.p[q]));
        if (d == 0) dg += double(pnew);
      }
    }
    rs = wave_sum_f64(rs);
    dg = wave_sum_f64(dg);
    if (lane_id() == uint32_t(c)) {
      S.rs = rs;
      S.dg = dg;
    }
  }
  // smem: the block's LDS, wave w's region at w * wbytes (>= 1 KiB each, free
  // once the wave's last vector is done)
  __device__ void finish(const State& S, unsigned char* smem, size_t wbytes, uint32_t slot) const {
    const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
    reinterpret_cast<double2*>(smem + wave * wbytes)[lane] = make_double2(S.rs, S.dg);
    __syncthreads();
    if (wave == 0 && lane < uint32_t(a.k) && !((S.done >> lane) & 1u)) {
      double R = 0.0, D = 0.0;
      for (int w = 0; w < kWaves; ++w) {
        const double2 v = reinterpret_cast<const double2*>(smem + w * wbytes)[lane];
        R += v.x;
        D += v.y;
      }
      const size_t q = size_t(lane) * gridDim.x + slot;
      a.slots[2 * q] = R;
      a.slots[2 * q + 1] = D;
    }
  }
};

// --------------------------------------------------------------- tile kernel
// The vectors a tile kernel multiplies (col(c) = the first element of vector
// c).  OneCol: one vector x, whose window values come with the tile's other
// loads.  Cols: columns 0 .. k-1 of a column-major block (element (v, c) at
// c * ld + v), taken one after another by the same decoded tile.
template <class X>
struct OneCol {
  const X* x;
  static constexpr bool kMulti = false;
  __device__ int count() const { return 1; }
  __device__ const X* col(int) const { return x; }
};
template <class X>
struct Cols {
  const X* x;
  int k;
  int64_t ld;
  static constexpr bool kMulti = true;
  __device__ int count() const { return k; }
  __device__ const X* col(int c) const { return x + int64_t(c) * ld; }
};

// The lane's first SV values of column c's x window (addresses clamped to
// the window; the slots past the lane's chunk hold values it never uses).
template <class X, int SV, class Src>
__device__ __forceinline__ void load_window(const Src& src, int64_t win0, uint32_t n, int c, X (&xs)[SV]) {
  const uint32_t lane = lane_id();
  const uint32_t w = (n + 63) / 64, b = min(n, lane * w);
  const X* xc = src.col(c) + win0;
  // values past the lane's chunk are read (in the window) but never used
#pragma unroll
  for (int j = 0; j < SV; ++j) xs[j] = xc[min(b + uint32_t(j), n - 1)];
}

// Global data of one tile, loaded before any of it is used: the first round
// of the lane's singles chunk, its rows' info, and its first SV values of
// the x window.
template <class M, int RPL, int SV>
struct TileLoads {
  uint32_t pre[kRound];
  uint32_t inf[RPL], ns[RPL];
  typename M::X xs[M::kInt ? 1 : SV];  // (the integer mode stages no window)
};

// Issue a tile's loads into `ld` from in-bounds addresses only (clamped, or
// within the zero padding after the last stream); the values are masked
// where process_tile uses them, so all the loads are in flight together
// before the first is waited for.
template <class M, int RPL, int SV, class Src>
__device__ __forceinline__ void issue_loads(const DevLayout& L, const TileDesc& td, const Src& src,
                                            TileLoads<M, RPL, SV>& ld) {
  const uint32_t lane = lane_id(), r0 = lane * RPL;
  const uint32_t n16 = td.n16;
  // Every load is unconditional (a tile without singles reads its stream's
  // first words, one without a window the value at win0, which is below n),
  // so that no branch join waits for a load before the tile's data is used.
  {
    const uint32_t* g16 = reinterpret_cast<const uint32_t*>(L.data + td.data16);
    const Chunk<2> ch(n16, flat_chunk<2>(n16));
    // the running-sum mode zeros the words past the lane's chunk before use;
    // the other modes decode whole rounds (clamped copies)
    if constexpr (std::is_same<M, MF32C>::value)
      load_round_raw(g16, ch.d0, ch.last, ld.pre);
    else
      load_round(g16, ch.d0, ch.last, ld.pre);
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const uint32_t r = r0 + q < td.nrows ? td.row0 + r0 + q : 0u;
    ld.inf[q] = L.info[r];
    ld.ns[q] = uint32_t(L.ns[r]);
  }
  if constexpr (!M::kInt && !Src::kMulti) load_window(src, td.win0, max(td.winlen, 1u), 0, ld.xs);
}

// Stage a tile's x window of n values into the LDS array Z (doubles): Z[0] =
// 0, Z[2j+2] = x[win0+j] for j < n, and, with `prefix`, Z[2p+1] = P[p] =
// x[win0] + ... + x[win0+p-1] for p <= n (odd entries are left undefined
// otherwise; no entry reads them then).  Lane l takes the ceil(n/64)
// consecutive values from l*ceil(n/64) on: the first SV are in xs, a longer
// chunk reads the rest here through xw(j), the window's j-th value.  A wave
// scan of the lanes' sums gives each lane's first prefix.  Z + 1 is 16-byte
// aligned, so every (P[j], x[j]) pair is one 16-byte LDS write.
template <class X, int SV, class XA>
__device__ __forceinline__ void stage_regs(const X (&xs)[SV], XA xw, uint32_t n, bool prefix, double* Z) {
  const uint32_t lane = lane_id();
  const uint32_t ch = (n + 63) / 64;
  const uint32_t b = min(n, lane * ch), e = min(n, b + ch);
  if (ch <= uint32_t(SV)) {
    // the lane's chunk is in registers: the values past it count as zeros,
    // so the sums are those of the general form below, term for term
    const uint32_t cnt = e - b;
    double xv[SV];
#pragma unroll
    for (int j = 0; j < SV; ++j) xv[j] = uint32_t(j) < cnt ? double(xs[j]) : 0.0;
    double run = 0.0;
    if (prefix) {
      double t = xv[0];
#pragma unroll
      for (int j = 1; j < SV; ++j) t += xv[j];
      const double inc = wave_incl_scan_f64(t);
      run = inc - t;
      if (lane == 63) Z[2 * size_t(n) + 1] = inc;
    }
    if (lane == 0) Z[0] = 0.0;
    double2* Zp = reinterpret_cast<double2*>(Z + 1);
#pragma unroll
    for (int j = 0; j < SV; ++j) {
      if (uint32_t(j) < cnt) Zp[b + j] = make_double2(run, xv[j]);
      run += xv[j];
    }
    return;
  }
  double t = 0.0;
  if (prefix) {
#pragma unroll
    for (int j = 0; j < SV; ++j)
      if (b + uint32_t(j) < e) t += double(xs[j]);
    for (uint32_t k = b + SV; k < e; ++k) t += double(xw(k));
  }
  double run = 0.0;
  if (prefix) {
    const double inc = wave_incl_scan_f64(t);
    run = inc - t;
    if (lane == 63) Z[2 * size_t(n) + 1] = inc;
  }
  if (lane == 0) Z[0] = 0.0;
  double2* Zp = reinterpret_cast<double2*>(Z + 1);  // Zp[j] = (P[j], x[win0+j])
#pragma unroll
  for (int j = 0; j < SV; ++j)
    if (b + uint32_t(j) < e) {
      const double xv = double(xs[j]);
      Zp[b + j] = make_double2(run, xv);
      run += xv;
    }
  for (uint32_t k = b + SV; k < e; ++k) {
    const double xv = double(xw(k));
    Zp[k] = make_double2(run, xv);
    run += xv;
  }
}

// One tile by one wavefront, its global data already in `ld`: tile rows
// [row0, row0 + nrows), lane l owns rows [l * RPL, (l + 1) * RPL).  The
// decode (offsets, row ranks, chunk row ends) is done once; then for each
// vector of the source its window is staged and steps 3 to 6 run.
template <class M, int RPL, int SV, class Src, class Epi>
__device__ __forceinline__ void process_tile(const DevLayout& L, const TileDesc& td, const TileLoads<M, RPL, SV>& ld,
                                             const Src& src, const Epi& epi, uint32_t slot, unsigned char* ws,
                                             unsigned char* s_blk) {
  using X = typename M::X;
  using PAcc = typename M::PAcc;
  using CAcc = typename M::CAcc;
  using Cv = WaveCarve<M, RPL>;
  constexpr bool kRun = std::is_same<M, MF32C>::value;  // running-sum singles pass
  PAcc* s_seg = reinterpret_cast<PAcc*>(ws + Cv::seg());
  CAcc* s_y = reinterpret_cast<CAcc*>(ws + Cv::y());
  PAcc* s_carry = reinterpret_cast<PAcc*>(ws + Cv::carry());
  double* Z = reinterpret_cast<double*>(ws + Cv::Z());
  static_assert(!(Src::kMulti && M::kInt), "the integer mode multiplies one vector");
  // the multi-vector epilogue's per-lane state, read before the decode
  const TileCtx tc{td.row0, td.nrows, td.graph, slot};
  auto S = epi.prepare(tc);
  if (epi.all_done(S)) return;  // every vector is done: the whole block returns
  // the first vector's epilogue loads: with one vector they go out with the
  // tile's own loads (with several, after the decode, to spare registers)
  decltype(epi.fetch(tc, 0)) f_next;
  if constexpr (!Src::kMulti) f_next = epi.fetch(tc, 0);
  const uint32_t lane = lane_id();
  const uint32_t nrows = td.nrows;
  const int64_t win0 = td.win0;
  const uint32_t winlen = td.winlen;
  const uint32_t r0 = lane * RPL;
  const uint32_t n16 = td.n16, nwide = td.nwide;
  const uint32_t* g16 = reinterpret_cast<const uint32_t*>(L.data + td.data16);  // singles stream
  const uint32_t* gw = g16 + dalign16u(n16 * 2u) / 4;                          // wide entries
  const uint32_t C16 = flat_chunk<2>(n16);
  const Chunk<2> ch16(n16, C16);
  // the loaded words, masked: stream dwords past the lane's chunk are 0
  // in the running-sum mode (clamped copies otherwise), rows past the tile 0
  uint32_t pre[kRound];
#pragma unroll
  for (int k = 0; k < kRound; ++k) {
    if constexpr (kRun)
      pre[k] = n16 && uint32_t(k) < ch16.nd ? ld.pre[k] : 0u;
    else
      pre[k] = n16 ? ld.pre[k] : 0u;
  }
  uint32_t inf[RPL], ns[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const bool has = r0 + q < nrows;
    inf[q] = has ? ld.inf[q] : 0u;
    ns[q] = has ? ld.ns[q] : 0u;
  }
  // 2. offsets of the lanes' rows in the streams, and of their row ends
  uint32_t c16[RPL], cw[RPL], s16 = 0, sw = 0;
  uint64_t m16[RPL], mw[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const bool lng = inf[q] & kInfoLong;
    c16[q] = lng ? 0u : ns[q];
    cw[q] = lng ? 0u : (inf[q] >> 13);
    s16 += c16[q];
    sw += cw[q];
    m16[q] = __ballot(c16[q] != 0);
    mw[q] = __ballot(cw[q] != 0);
  }
  // the lanes' singles (bits 0..15) and the row ends in the lane's chunk (16..31)
  const uint32_t sc16 = s16 | ((n16 ? chunk_ends<2, kS16End | (kS16End << 16), kRun>(n16, C16, g16, pre) : 0u) << 16);
  const uint32_t ex16 = wave_incl_scan_u32(sc16) - sc16;
  uint32_t o16[RPL], k16[RPL], kw[RPL];
  {
    uint32_t a16 = ex16 & 0xFFFFu, b16 = 0, bw = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      b16 += lanes_below(m16[q]);
      bw += lanes_below(mw[q]);
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      o16[q] = a16;
      k16[q] = b16;
      kw[q] = bw;
      a16 += c16[q];
      b16 += c16[q] != 0;
      bw += cw[q] != 0;
    }
  }
  wave_sync();

  X xs_next[SV];
  if constexpr (Src::kMulti) {
    f_next = epi.fetch(tc, 0);
    load_window(src, win0, max(winlen, 1u), 0, xs_next);
  }
  for (int col = 0; col < src.count(); ++col) {
  const auto f_cur = f_next;
  const X* xcol = src.col(col);
  // 1. the x window of this vector (with its prefix sums when the tile has
  //    intervals) into Z; the next vector's window values are loaded meanwhile
  //    (also when this vector is passed over, so that they stay in step)
  if constexpr (!M::kInt) {
    if constexpr (Src::kMulti) {
      X xs[SV];
#pragma unroll
      for (int j = 0; j < SV; ++j) xs[j] = xs_next[j];
      if (col + 1 < src.count()) {
        f_next = epi.fetch(tc, col + 1);
        load_window(src, win0, max(winlen, 1u), col + 1, xs_next);
      }
      if (epi.skip(S, col)) continue;
      stage_regs<X, SV>(xs, [&](uint32_t j) { return xcol[win0 + j]; }, winlen, td.nint != 0, Z);
    } else {
      stage_regs<X, SV>(ld.xs, [&](uint32_t j) { return xcol[win0 + j]; }, winlen, td.nint != 0, Z);
    }
  }
  wave_sync();
  // 3. singles (with the intervals' prefix pairs), then wide entries: flat
  //    passes cut at the row-end bits; the owner adds its rows' pieces in
  //    registers
  PAcc a[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) a[q] = M::pzero();
  if (n16) {
    const float invC = __builtin_amdgcn_rcpf(float(C16));
    if constexpr (kRun) {
      run_pass((min(C16, n16) + 1) / 2, ch16, g16, pre, (ex16 >> 16) + lane, s_seg, Z);
      wave_sync();
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (c16[q]) a[q] = run_row_sum(o16[q], o16[q] + c16[q], C16, invC, k16[q], s_seg);
    } else if constexpr (M::kInt) {
      // degrees: a column counts 1, a prefix entry P[p] counts p
      end_pass<M, 2, kS16End>(n16, C16, g16, pre, ex16 >> 16, s_seg, s_carry, [&](uint32_t w) -> X {
        const int32_t f = int32_t(w & kS16Off);
        const int32_t v = (f & 1) ? (f >> 1) : (f ? 1 : 0);
        return (w & kS16Neg) ? -v : v;
      }, [](PAcc& acc, X v) { M::padd(acc, v); });
    } else {
      end_pass<M, 2, kS16End>(n16, C16, g16, pre, ex16 >> 16, s_seg, s_carry, [&](uint32_t w) -> double {
        const double v = Z[w & kS16Off];
        return (w & kS16Neg) ? -v : v;
      }, [](PAcc& acc, double v) { M::padd_d(acc, v); });
    }
    if constexpr (!kRun) {
      wave_sync();
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (c16[q]) a[q] = flat_row_sum<M>(o16[q], o16[q] + c16[q], C16, invC, s_seg[k16[q]], s_carry);
    }
  }
  // window value of column win0 + c, else the global one (read through a
  // global address-space pointer, so that the two loads stay apart: merged
  // into one flat load, the double-precision instances do not compile)
  auto xval = [&](int64_t c) -> X {
    if constexpr (M::kInt) {
      return 1;
    } else {
      using GX = const __attribute__((address_space(1))) X;
      return uint64_t(c) < winlen ? X(Z[2 * c + 2]) : ((GX*)xcol)[win0 + c];
    }
  };
  if (nwide) {
    const uint32_t Cw = flat_chunk<1>(nwide);
    const float invC = __builtin_amdgcn_rcpf(float(Cw));
    uint32_t prew[kRound];
    {
      const Chunk<1> ch(nwide, Cw);
      load_round(gw, ch.d0, ch.last, prew);
    }
    const uint32_t scw = sw | (chunk_ends<1, kWideEnd>(nwide, Cw, gw, prew) << 16);
    const uint32_t exw = wave_incl_scan_u32(scw) - scw;
    wave_sync();  // the singles' pieces are read
    end_pass<M, 1, kWideEnd>(nwide, Cw, gw, prew, exw >> 16, s_seg, s_carry, [&](uint32_t w) -> X {
      const X v = xval(int64_t(w & kWideOff) - int64_t(kWideBias));
      return (w & kWideNeg) ? -v : v;
    }, [](PAcc& acc, X v) { M::padd(acc, v); });
    wave_sync();
    uint32_t aw = exw & 0xFFFFu;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      if (cw[q]) a[q] = M::pcomb(a[q], flat_row_sum<M>(aw, aw + cw[q], Cw, invC, s_seg[kw[q]], s_carry));
      aw += cw[q];
    }
  }

  // 4. long rows, the whole wave each
  bool any_long = false;
#pragma unroll
  for (int q = 0; q < RPL; ++q) any_long |= (inf[q] & kInfoLong) != 0;
  if (__ballot(any_long)) {
    uint64_t cnt[RPL], csum = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      cnt[q] = (inf[q] & kInfoLong) ? (uint64_t(inf[q] >> 13) | (uint64_t(ns[q]) << 19)) : 0;
      csum += cnt[q];
    }
    uint64_t totL;
    uint64_t exL = wave_excl_scan_u64(csum, totL);
    uint64_t offq[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      offq[q] = exL;
      exL += cnt[q];
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      uint64_t lmask = __ballot((inf[q] & kInfoLong) != 0);
      while (lmask) {
        const int l = __ffsll(static_cast<unsigned long long>(lmask)) - 1;
        lmask &= lmask - 1;
        const uint64_t len = __shfl(cnt[q], l, 64);
        const uint64_t off = __shfl(offq[q], l, 64);
        const uint32_t* e = L.longs + size_t(td.long0) + off;
        PAcc s = M::pzero();
        // batches of 8 entries per lane: all loads, then all gathers, then adds
        for (uint64_t base = 0; base < len; base += 64 * 8) {
          uint32_t w[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const uint64_t k = base + lane + 64u * j;
            w[j] = k < len ? e[k] : 0u;
          }
          X v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            v[j] = base + lane + 64u * j >= len ? X(0)
                                               : xval(int64_t(w[j] & 0x7FFFFFFFu) - int64_t(kLongBias));
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (base + lane + 64u * j < len) M::padd(s, (w[j] & 0x80000000u) ? -v[j] : v[j]);
        }
        s = wave_reduce<M>(s);
        if (lane == uint32_t(l)) a[q] = s;
      }
    }
  }

  // 5. reuse levels: y_i = y_{i-g} + partial_i, while some row is at the level
  wave_sync();  // every piece is read before y overwrites the slots
  CAcc ca[RPL];
  uint32_t lvmax = 0;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    ca[q] = M::chain(a[q]);
    const uint32_t lv = (inf[q] >> 4) & 15u;
    lvmax = max(lvmax, lv);
    if (lv == 0) s_y[r0 + q] = ca[q];
  }
  for (uint32_t lv = 1; __ballot(lvmax >= lv); ++lv) {
    wave_sync();
#pragma unroll
    for (int q = 0; q < RPL; ++q)
      if (((inf[q] >> 4) & 15u) == lv) s_y[r0 + q] = M::comb(s_y[r0 + q - (inf[q] & 15u)], ca[q]);
  }
  wave_sync();
  // 6. epilogue
  epi.col(tc, s_y, s_blk, col, S, f_cur);
  wave_sync();  // y is read before the next vector's pieces overwrite it
  }
  const size_t wb = Cv{L.wcap}.wave_bytes();
  epi.finish(S, s_blk - kWaves * wb, wb, slot);
}

// Tile kernel: block b takes the group of kWaves consecutive tiles from
// kWaves * b on, wave w the w-th, and multiplies the source's vectors.  A
// block of a member that is done (skip_done) returns at once.
template <class M, int RPL, int SV, class Src, class Epi>
__global__ void __launch_bounds__(kThreads) bv_wave_kernel(DevLayout L, Src src, Epi epi,
                                                           const PRState* __restrict__ skip_done) {
  using Cv = WaveCarve<M, RPL>;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Cv cv{L.wcap};
  unsigned char* ws = smem + size_t(wave) * cv.wave_bytes();
  unsigned char* s_blk = smem + size_t(kWaves) * cv.wave_bytes();
  const TileDesc td = L.tiles[blockIdx.x * kWaves + wave];
  epi.block_start(blockIdx.x, td.graph, s_blk);        // (a block holds one member's tiles)
  if (skip_done && skip_done[td.graph].done) return;
  TileLoads<M, RPL, SV> ld;
  issue_loads<M, RPL, SV>(L, td, src, ld);
  process_tile<M, RPL, SV>(L, td, ld, src, epi, blockIdx.x, ws, s_blk);
}

// PageRank start: p0 = start (or teleport, or uniform), z0 = p0 / d, dangling mass.
// With `normalize`, p0 = start / (the member's delta field), which then holds
// the start's sum (restart_vector_kernel and an init-mode finish put it there).
// Tiles are read through (row0, nrows) at a stride; the member through `graphs`.
template <class M>
__global__ void __launch_bounds__(kThreads) pr_init_kernel(const uint32_t* __restrict__ row0s, uint32_t row_stride,
                                                           const uint32_t* __restrict__ graphs, const void* start_,
                                                           const void* tele_, void* p0_, void* z0_,
                                                           const int32_t* __restrict__ outdeg, PRState* st_all,
                                                           double* slots, int normalize) {
  using X = typename M::X;
  __shared__ __align__(16) unsigned char s_blk[256];
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const size_t tile = size_t(blockIdx.x) * kWaves + wave;
  const uint32_t row0 = row0s[tile * row_stride];
  const uint32_t nrows = row0s[tile * row_stride + 1] & 0x7FFFFFFFu;
  const uint32_t graph = graphs ? graphs[size_t(blockIdx.x) * kWaves * row_stride] : 0u;
  PRState* st = st_all + graph;
  const X* start = static_cast<const X*>(start_);
  const X* tele = static_cast<const X*>(tele_);
  X* p0 = static_cast<X*>(p0_);
  X* z0 = static_cast<X*>(z0_);
  const double inv_sum = normalize ? 1.0 / st->delta : 1.0;
  double dg = 0.0;
  for (uint32_t r = lane; r < nrows; r += 64) {
    const uint32_t v = row0 + r;
    const X pv = start ? (normalize ? X(double(start[v]) * inv_sum) : start[v]) : (tele ? tele[v] : X(st->inv_n));
    p0[v] = pv;
    const int32_t d = outdeg[v];
    z0[v] = d > 0 ? pv / X(d) : X(0);
    if (d == 0) dg += double(pv);
  }
  dg = wave_sum_f64(dg);
  pr_block_partial(0.0, dg, slots, s_blk, blockIdx.x);
}

// Personalized PageRank start for k right-hand sides on the tile kernel's
// grid: p0 = start (or the teleport columns, or uniform), z0 = p0 / d, and
// each column's dangling mass per block (slot c * blocks + block).  Every
// n x k block is column-major with leading dimension n.
template <class M>
__global__ void __launch_bounds__(kThreads) pr_init_cols_kernel(DevLayout L, int k, const void* start_,
                                                                const void* tele_, void* p0_, void* z0_,
                                                                const int32_t* __restrict__ outdeg,
                                                                const PRState* st_all, double* slots) {
  using X = typename M::X;
  __shared__ __align__(16) unsigned char s_blk[256];
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const TileDesc td = L.tiles[blockIdx.x * kWaves + wave];
  const X* start = static_cast<const X*>(start_);
  const X* tele = static_cast<const X*>(tele_);
  X* p0 = static_cast<X*>(p0_);
  X* z0 = static_cast<X*>(z0_);
  for (int c = 0; c < k; ++c) {
    double dg = 0.0;
    for (uint32_t r = lane; r < td.nrows; r += 64) {
      const uint32_t v = td.row0 + r;
      const int64_t e = int64_t(c) * L.n + v;
      const X pv = start ? start[e] : (tele ? tele[e] : X(st_all[c].inv_n));
      p0[e] = pv;
      const int32_t d = outdeg[v];
      z0[e] = d > 0 ? pv / X(d) : X(0);
      if (d == 0) dg += double(pv);
    }
    dg = wave_sum_f64(dg);
    pr_block_partial(0.0, dg, slots, s_blk, uint32_t(c) * gridDim.x + blockIdx.x);
    __syncthreads();  // s_blk is read before the next column writes it
  }
}

// ----------------------------------------------------------- warm restarts
// Inputs 8..11 of the restart network for every row v of a tile, from the
// last four iterates p_K, p_{K-1}, p_{K-2}, p_{K-3} of the member, whose
// delta = ||p_K - p_{K-1}||_1 is its state's residual and whose node count is
// 1 / inv_n: log(n p_K), then n (p_j - p_{j-1}) / delta for the last three
// steps, newest first.  With p_star given, also the training target
// T_v = n (p*_v - p_K(v)) / delta.  The four inputs of v are one 16-byte
// store at Ft + v * ft_stride.
template <class M>
__global__ void __launch_bounds__(kThreads) restart_inputs_kernel(
    const uint32_t* __restrict__ row0s, uint32_t row_stride, const uint32_t* __restrict__ graphs, const void* pK_,
    const void* pK1_, const void* pK2_, const void* pK3_, const void* p_star_, const PRState* __restrict__ st_all,
    float* __restrict__ Ft, int64_t ft_stride, float* __restrict__ T) {
  using X = typename M::X;
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const size_t tile = size_t(blockIdx.x) * kWaves + wave;
  const uint32_t row0 = row0s[tile * row_stride];
  const uint32_t nrows = row0s[tile * row_stride + 1] & 0x7FFFFFFFu;
  const uint32_t graph = graphs ? graphs[size_t(blockIdx.x) * kWaves * row_stride] : 0u;
  const PRState* st = st_all + graph;
  const double n = 1.0 / st->inv_n, scale = n / st->resid;
  const X* pK = static_cast<const X*>(pK_);
  const X* pK1 = static_cast<const X*>(pK1_);
  const X* pK2 = static_cast<const X*>(pK2_);
  const X* pK3 = static_cast<const X*>(pK3_);
  const X* p_star = static_cast<const X*>(p_star_);
  for (uint32_t r = lane; r < nrows; r += 64) {
    const uint32_t v = row0 + r;
    const double a = double(pK[v]), b = double(pK1[v]), c = double(pK2[v]), d = double(pK3[v]);
    *reinterpret_cast<float4*>(Ft + int64_t(v) * ft_stride) =
        make_float4(float(log(n * a)), float(scale * (a - b)), float(scale * (b - c)), float(scale * (c - d)));
    if (p_star) T[v] = float(scale * (double(p_star[v]) - a));
  }
}

// Unnormalised restart vector q_v = max(p_K(v) + s_v delta / n, p_K(v) / 1000)
// (delta and n as above), stored in the iterate's type; the block sums of the
// stored values go to the dangling half of the block's slot, so that an
// init-mode pr_finish_kernel leaves each member's sum of q in its delta field.
template <class M>
__global__ void __launch_bounds__(kThreads) restart_vector_kernel(
    const uint32_t* __restrict__ row0s, uint32_t row_stride, const uint32_t* __restrict__ graphs, const void* pK_,
    const float* __restrict__ s, const PRState* __restrict__ st_all, void* q_, double* slots) {
  using X = typename M::X;
  __shared__ __align__(16) unsigned char s_blk[256];
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const size_t tile = size_t(blockIdx.x) * kWaves + wave;
  const uint32_t row0 = row0s[tile * row_stride];
  const uint32_t nrows = row0s[tile * row_stride + 1] & 0x7FFFFFFFu;
  const uint32_t graph = graphs ? graphs[size_t(blockIdx.x) * kWaves * row_stride] : 0u;
  const PRState* st = st_all + graph;
  const double step = st->resid * st->inv_n;
  const X* pK = static_cast<const X*>(pK_);
  X* q = static_cast<X*>(q_);
  double sum = 0.0;
  for (uint32_t r = lane; r < nrows; r += 64) {
    const uint32_t v = row0 + r;
    const double a = double(pK[v]);
    const X qv = X(fmax(a + double(s[v]) * step, 1e-3 * a));
    q[v] = qv;
    sum += double(qv);
  }
  sum = wave_sum_f64(sum);
  pr_block_partial(0.0, sum, slots, s_blk, blockIdx.x);
}

// ---------------------------------------------------------------- CSR kernel
// Same structure on plain CSR: a wave takes a run of up to 64 rows whose
// column ids are staged in LDS with an x window (columns inside it read from
// LDS), summed by the same flat pass; or one long row (bit 31 of nrows)
// summed by the whole wave.
template <class M>
struct CsrCarve {
  using X = typename M::X;
  using PAcc = typename M::PAcc;
  using CAcc = typename M::CAcc;
  uint32_t WC, CC;
  static constexpr size_t kSlot = sizeof(PAcc) > sizeof(CAcc) ? sizeof(PAcc) : sizeof(CAcc);
  __host__ __device__ static constexpr size_t seg() { return 0; }  // y shares the pieces' slots
  __host__ __device__ static constexpr size_t y() { return 0; }
  __host__ __device__ static constexpr size_t carry() { return align16(64 * kSlot); }
  __host__ __device__ static constexpr size_t x() { return carry() + align16(64 * sizeof(PAcc)); }
  __host__ __device__ size_t tags() const { return x() + align16(size_t(WC) * sizeof(X) + 16); }
  __host__ __device__ size_t wave_bytes() const { return tags() + align16(size_t(CC) + 64); }
  __host__ __device__ size_t block_bytes() const { return kWaves * wave_bytes() + 256; }
};

constexpr int kCsrPre = 4;  // 16-byte batches of the lane's column ids loaded up front (16 ids)

// Tagged flat pass of the CSR tile: as end_pass, but over 16-byte batches of
// column ids (4 per batch; the first kCsrPre batches loaded by the caller) in
// entries counted from the 16-byte aligned id at or before the tile's first
// (entries before `lo` belong to no row of the tile).  Entry e's row end is
// read from tags[e] (the tile row whose last entry it is, or 0xFF), written
// beforehand by the row owners, and the piece goes to seg[row].
template <class M, class ValFn>
__device__ __forceinline__ void csr_pass(uint32_t lo, uint32_t E, uint32_t C, const uint4* __restrict__ g,
                                         const uint4 (&pre)[kCsrPre], const uint8_t* tags, typename M::PAcc* seg,
                                         typename M::PAcc* carry, ValFn val) {
  using PAcc = typename M::PAcc;
  using X = typename M::X;
  const uint32_t lane = lane_id();
  const uint32_t b = lane * C;
  if (b >= E) return;
  const uint32_t end = min(E, b + C);
  PAcc a = M::pzero();
  auto batch = [&](const uint4& q, uint32_t e) {
    const uint32_t tg = *reinterpret_cast<const uint32_t*>(tags + e);
    const uint32_t c[4] = {q.x, q.y, q.z, q.w};
    X v[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) v[j] = val(c[j], e + j >= lo && e + j < end);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      M::padd(a, v[j]);
      const uint32_t t = (tg >> (8 * j)) & 0xFFu;
      if (t != 0xFFu && e + j < end) {
        seg[t] = a;
        a = M::pzero();
      }
    }
  };
#pragma unroll
  for (int k = 0; k < kCsrPre; ++k)
    if (b + uint32_t(k) * 4 < end) batch(pre[k], b + uint32_t(k) * 4);
  for (uint32_t k = kCsrPre; b + k * 4 < end; ++k) batch(g[b / 4 + k], b + k * 4);
  carry[lane] = a;
}

template <class M, class Epi>
__global__ void __launch_bounds__(kThreads) csr_wave_kernel(DevCsr C, const typename M::X* __restrict__ x, Epi epi,
                                                            const PRState* __restrict__ skip_done) {
  using X = typename M::X;
  using PAcc = typename M::PAcc;
  using CAcc = typename M::CAcc;
  extern __shared__ __align__(16) unsigned char smem[];
  const CsrCarve<M> cv0{C.wcap, C.ccap};
  epi.block_start(blockIdx.x, 0u, smem + size_t(kWaves) * cv0.wave_bytes());
  if (skip_done && skip_done[0].done) return;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t tile = blockIdx.x * kWaves + wave;
  const CsrTile td = C.tiles[tile];
  // an id's value: x below nx, the second source at and above it
  const X* __restrict__ aux = static_cast<const X*>(C.aux);
  const uint32_t nx = C.nx;
  auto gval = [&](uint32_t c) -> X { return c < nx ? x[c] : aux[c - nx]; };
  const bool is_long = td.nrows & 0x80000000u;
  const uint32_t nrows = td.nrows & 0x7FFFFFFFu;
  const CsrCarve<M> cv{C.wcap, C.ccap};
  unsigned char* ws = smem + size_t(wave) * cv.wave_bytes();
  unsigned char* s_blk = smem + size_t(kWaves) * cv.wave_bytes();
  PAcc* s_seg = reinterpret_cast<PAcc*>(ws + cv.seg());
  CAcc* s_y = reinterpret_cast<CAcc*>(ws + cv.y());
  PAcc* s_carry = reinterpret_cast<PAcc*>(ws + cv.carry());
  X* s_xbuf = reinterpret_cast<X*>(ws + cv.x());
  uint8_t* s_tags = reinterpret_cast<uint8_t*>(ws + cv.tags());
  if (is_long) {
    PAcc s = M::pzero();
    const uint32_t* cl = C.col + size_t(td.c0);
    for (uint32_t base = 0; base < td.ncols; base += 64 * 8) {  // 8 loads in flight per lane
      uint32_t c[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t k = base + lane + 64u * j;
        c[j] = k < td.ncols ? cl[k] : 0u;
      }
      X v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = base + lane + 64u * j < td.ncols ? gval(c[j]) : X(0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (base + lane + 64u * j < td.ncols) M::padd(s, v[j]);
    }
    s = wave_reduce<M>(s);
    if (lane == 0) s_y[0] = M::chain(s);
  } else {
    const int64_t win0 = td.win0;
    const uint32_t winlen = td.winlen;
    // entries are counted from the 16-byte aligned column id at or before
    // c0; the lane's chunk of ids is read straight from global memory
    const uint32_t shift = td.c0 & 3u;
    const uint32_t E = td.ncols + shift;
    const uint4* g = reinterpret_cast<const uint4*>(C.col + (size_t(td.c0) - shift));
    const uint32_t Cc = flat_chunk<4>(E);
    uint4 pre[kCsrPre];
    if (td.ncols) {
      const uint32_t nb = (E + 3) / 4;
#pragma unroll
      for (int k = 0; k < kCsrPre; ++k) pre[k] = g[min(lane * Cc / 4 + uint32_t(k), nb - 1)];
    }
    uint32_t ob = 0, oe = 0;
    if (lane < nrows) {
      ob = uint32_t(C.rowptr[td.row0 + lane] - td.c0) + shift;
      oe = uint32_t(C.rowptr[td.row0 + lane + 1] - td.c0) + shift;
    }
    const X* s_x = stage_range<X>(x, C.n, win0, winlen, s_xbuf);
    wave_fill_ff(s_tags, dalign16u(E + 16));
    wave_sync();
    if (oe > ob) s_tags[oe - 1] = uint8_t(lane);
    wave_sync();
    PAcc a = M::pzero();
    if (td.ncols) {
      const float invC = 1.0f / float(Cc);
      // ids past the chunk are the next rows' or the array's zero padding,
      // so every gather stays in bounds; only the source depends on `ok`
      csr_pass<M>(shift, E, Cc, g, pre, s_tags, s_seg, s_carry, [&](uint32_t c, bool ok) -> X {
        const int64_t d = int64_t(c) - win0;
        const bool inwin = uint64_t(d) < winlen;
        X v = s_x[inwin ? uint32_t(d) : 0u];
        if (ok && !inwin) v = gval(c);
        return ok ? v : X(0);
      });
      wave_sync();
      if (oe > ob) a = flat_row_sum<M>(ob, oe, Cc, invC, s_seg[lane], s_carry);
      wave_sync();  // pieces read before y overwrites the slots
    }
    s_y[lane] = M::chain(a);
  }
  wave_sync();
  epi(TileCtx{td.row0, nrows, 0u, blockIdx.x}, s_y, s_blk, 0);
}

// Rows [r0, r1) of p and z from src: p = src and z = src / d (0 where d = 0),
// as the PageRank epilogue writes them.
template <class X>
__global__ void __launch_bounds__(kThreads) pr_restore_kernel(const X* __restrict__ src, X* __restrict__ p,
                                                              X* __restrict__ z, const int32_t* __restrict__ outdeg,
                                                              int64_t r0, int64_t r1) {
  for (int64_t v = r0 + int64_t(blockIdx.x) * kThreads + threadIdx.x; v < r1; v += int64_t(gridDim.x) * kThreads) {
    const X pv = src[v];
    p[v] = pv;
    const int32_t d = outdeg[v];
    z[v] = d > 0 ? pv / X(d) : X(0);
  }
}

// p_out column c (column-major, leading dimension n; column c = blockIdx.y)
// = the buffer holding column c's final iterate.
template <class X>
__global__ void __launch_bounds__(kThreads) pr_select_kernel(const PRState* __restrict__ st, const X* __restrict__ p0,
                                                             const X* __restrict__ p1, X* __restrict__ out,
                                                             int64_t n) {
  const int64_t base = int64_t(blockIdx.y) * n;
  const X* src = (st[blockIdx.y].final_buf ? p1 : p0) + base;
  for (int64_t v = int64_t(blockIdx.x) * kThreads + threadIdx.x; v < n; v += int64_t(gridDim.x) * kThreads)
    out[base + v] = src[v];
}

// ------------------------------------------------------------- dispatching
hipError_t set_lds(const void* k, size_t smem) {
  if (smem <= 65536) return hipSuccess;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(smem));
}

// rows per lane of the kernel instance that covers the layout's tiles
inline int rows_per_lane(const DevLayout& L) { return L.tcap <= 64 ? 1 : 2; }
static_assert(kTileRowsMax <= 128, "row tags are bytes below 0xFF");

template <class M>
size_t tile_lds(const DevLayout& L) {
  switch (rows_per_lane(L)) {
    case 1: return WaveCarve<M, 1>{L.wcap}.block_bytes();
    default: return WaveCarve<M, 2>{L.wcap}.block_bytes();
  }
}

template <class M, int RPL, int SV, class Src, class Epi>
hipError_t launch_tile_sv(const DevLayout& L, const Src& src, const Epi& epi, const PRState* skip, hipStream_t s) {
  const size_t smem = WaveCarve<M, RPL>{L.wcap}.block_bytes();
  // a multi-vector epilogue combines 64 pairs of doubles per wave region
  if (Src::kMulti && WaveCarve<M, RPL>{L.wcap}.wave_bytes() < 64 * sizeof(double2)) return hipErrorInvalidValue;
  auto k = bv_wave_kernel<M, RPL, SV, Src, Epi>;
  if (hipError_t e = set_lds(reinterpret_cast<const void*>(k), smem)) return e;
  if (L.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(L.ntiles / kWaves), dim3(kThreads), smem, s, L, src, epi, skip);
  return hipGetLastError();
}

// window values a lane loads up front: 4 up to 256 columns, 8 up to 512, else
// 16 (a longer lane chunk loads the rest while it stages); no more than the
// widest chunk, since every slot costs loads and staging work
template <class M, int RPL, class Src, class Epi>
hipError_t launch_tile_rpl(const DevLayout& L, const Src& src, const Epi& epi, const PRState* skip, hipStream_t s) {
  if (L.wcap <= 256) return launch_tile_sv<M, RPL, 4>(L, src, epi, skip, s);
  if (L.wcap <= 512) return launch_tile_sv<M, RPL, 8>(L, src, epi, skip, s);
  return launch_tile_sv<M, RPL, 16>(L, src, epi, skip, s);
}

template <class M, class Src, class Epi>
hipError_t launch_tile_src(const DevLayout& L, const Src& src, const Epi& epi, const PRState* skip, hipStream_t s) {
  switch (rows_per_lane(L)) {
    case 1: return launch_tile_rpl<M, 1>(L, src, epi, skip, s);
    default: return launch_tile_rpl<M, 2>(L, src, epi, skip, s);
  }
}

template <class M, class Epi>
hipError_t launch_tile(const DevLayout& L, const void* x, const Epi& epi, const PRState* skip, hipStream_t s) {
  return launch_tile_src<M>(L, OneCol<typename M::X>{static_cast<const typename M::X*>(x)}, epi, skip, s);
}

// k columns of a column-major block, each multiplied by the tile kernel's shared decode
template <class M, class Epi>
hipError_t launch_tile_cols(const DevLayout& L, const void* X, int k, int64_t ld, const Epi& epi, hipStream_t s) {
  return launch_tile_src<M>(L, Cols<typename M::X>{static_cast<const typename M::X*>(X), k, ld}, epi, nullptr, s);
}

template <class M>
size_t csr_lds(const DevCsr& C) {
  return CsrCarve<M>{C.wcap, C.ccap}.block_bytes();
}

template <class M, class Epi>
hipError_t launch_csr(const DevCsr& Cs, const void* x, const Epi& epi, const PRState* skip, hipStream_t s) {
  const size_t smem = csr_lds<M>(Cs);
  auto k = csr_wave_kernel<M, Epi>;
  if (hipError_t e = set_lds(reinterpret_cast<const void*>(k), smem)) return e;
  if (Cs.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(Cs.ntiles / kWaves), dim3(kThreads), smem, s, Cs,
                     static_cast<const typename M::X*>(x), epi, skip);
  return hipGetLastError();
}

}  // namespace

size_t bv_kernel_lds_bytes(const DevLayout& L, int prec) {
  switch (prec) {
    case 0: return tile_lds<MF64>(L);
    case 1: return tile_lds<MF32>(L);
    case 2: return tile_lds<MF32C>(L);
    default: return 0;
  }
}

size_t csr_kernel_lds_bytes(const DevCsr& C, int prec) {
  switch (prec) {
    case 0: return csr_lds<MF64>(C);
    case 1: return csr_lds<MF32>(C);
    case 2: return csr_lds<MF32C>(C);
    default: return 0;
  }
}

hipError_t launch_bv_multiply(const DevLayout& L, int prec, const void* x, void* y, hipStream_t s) {
  switch (prec) {
    case 0: return launch_tile<MF64>(L, x, EpiStore<MF64>{static_cast<double*>(y)}, nullptr, s);
    case 1: return launch_tile<MF32>(L, x, EpiStore<MF32>{static_cast<float*>(y)}, nullptr, s);
    case 2: return launch_tile<MF32C>(L, x, EpiStore<MF32C>{static_cast<float*>(y)}, nullptr, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bv_multiply_add(const DevLayout& L, int prec, const void* x, void* y, hipStream_t s) {
  switch (prec) {
    case 0: return launch_tile<MF64>(L, x, EpiStore<MF64, true>{static_cast<double*>(y)}, nullptr, s);
    case 1: return launch_tile<MF32>(L, x, EpiStore<MF32, true>{static_cast<float*>(y)}, nullptr, s);
    case 2: return launch_tile<MF32C>(L, x, EpiStore<MF32C, true>{static_cast<float*>(y)}, nullptr, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bv_degrees(const DevLayout& L, int32_t* deg, hipStream_t s) {
  return launch_tile<MINT>(L, nullptr, EpiStore<MINT>{deg}, nullptr, s);
}

hipError_t launch_pr_finish(const PRArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(pr_finish_kernel, dim3(a.members), dim3(kThreads), 0, s, a.st, a.slots, 1, a.tol, a.max_iter,
                     a.buf, 0);
  return hipGetLastError();
}

hipError_t launch_bv_pagerank_iter(const DevLayout& L, int prec, const PRArgs& a, hipStream_t s) {
  hipError_t e;
  switch (prec) {
    case 0: e = launch_tile<MF64>(L, a.z_cur, EpiPR<MF64>{a}, a.st, s); break;
    case 1: e = launch_tile<MF32>(L, a.z_cur, EpiPR<MF32>{a}, a.st, s); break;
    case 2: e = launch_tile<MF32C>(L, a.z_cur, EpiPR<MF32C>{a}, a.st, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || a.fused) return e;
  return launch_pr_finish(a, s);
}

hipError_t launch_pr_flush(PRState* st, const double* slots, double tol, int32_t max_iter, double* pub, int members,
                           hipStream_t s) {
  if (members <= 0) return hipSuccess;
  hipLaunchKernelGGL(pr_flush_kernel, dim3(members), dim3(kThreads), 0, s, st, slots, tol, max_iter, pub);
  return hipGetLastError();
}

hipError_t launch_pr_init(const DevLayout& L, int prec, const void* start, const void* tele, void* p0, void* z0,
                          const int32_t* outdeg, PRState* st, double* slots, int members, hipStream_t s,
                          int normalize, int32_t iter0) {
  if (L.ntiles == 0) return hipSuccess;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(L.tiles);
  const uint32_t stride = sizeof(TileDesc) / 4;
  const uint32_t* graphs = base + offsetof(TileDesc, graph) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(pr_init_kernel<MF64>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride, graphs,
                       start, tele, p0, z0, outdeg, st, slots, normalize);
  else
    hipLaunchKernelGGL(pr_init_kernel<MF32>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride, graphs,
                       start, tele, p0, z0, outdeg, st, slots, normalize);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(pr_finish_kernel, dim3(members), dim3(kThreads), 0, s, st, slots, 0, 0.0, 0, 0, iter0);
  return hipGetLastError();
}

hipError_t launch_bv_multiply_cols(const DevLayout& L, int prec, const void* X, void* Y, int k, int64_t ld,
                                   hipStream_t s) {
  switch (prec) {
    case 0: return launch_tile_cols<MF64>(L, X, k, ld, EpiStoreCols<MF64>{static_cast<double*>(Y), ld}, s);
    case 1: return launch_tile_cols<MF32>(L, X, k, ld, EpiStoreCols<MF32>{static_cast<float*>(Y), ld}, s);
    case 2: return launch_tile_cols<MF32C>(L, X, k, ld, EpiStoreCols<MF32C>{static_cast<float*>(Y), ld}, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bv_cols_pagerank_iter(const DevLayout& L, int prec, const PRArgs& a, hipStream_t s) {
  if (a.k < 1 || a.k > 64) return hipErrorInvalidValue;  // lane c of a wave holds column c
  hipError_t e;
  switch (prec) {
    case 0: e = launch_tile_cols<MF64>(L, a.z_cur, a.k, L.n, EpiPRCols<MF64>{a, L.n}, s); break;
    case 1: e = launch_tile_cols<MF32>(L, a.z_cur, a.k, L.n, EpiPRCols<MF32>{a, L.n}, s); break;
    case 2: e = launch_tile_cols<MF32C>(L, a.z_cur, a.k, L.n, EpiPRCols<MF32C>{a, L.n}, s); break;
    default: return hipErrorInvalidValue;
  }
  return e != hipSuccess ? e : launch_pr_finish(a, s);
}

hipError_t launch_cols_pr_init(const DevLayout& L, int prec, int k, const void* start, const void* tele, void* p0,
                               void* z0, const int32_t* outdeg, PRState* st, double* slots, hipStream_t s) {
  if (L.ntiles == 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(pr_init_cols_kernel<MF64>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, L, k, start, tele,
                       p0, z0, outdeg, st, slots);
  else
    hipLaunchKernelGGL(pr_init_cols_kernel<MF32>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, L, k, start, tele,
                       p0, z0, outdeg, st, slots);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(pr_finish_kernel, dim3(k), dim3(kThreads), 0, s, st, slots, 0, 0.0, 0, 0, 0);
  return hipGetLastError();
}

hipError_t launch_restart_inputs(const DevLayout& L, int prec, const void* pK, const void* pK1, const void* pK2,
                                 const void* pK3, const void* p_star, const PRState* st, float* Ft,
                                 int64_t ft_stride, float* T, hipStream_t s) {
  if (L.ntiles == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(Ft) | uintptr_t(ft_stride) * 4) & 15) return hipErrorInvalidValue;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(L.tiles);
  const uint32_t stride = sizeof(TileDesc) / 4;
  const uint32_t* graphs = base + offsetof(TileDesc, graph) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(restart_inputs_kernel<MF64>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride,
                       graphs, pK, pK1, pK2, pK3, p_star, st, Ft, ft_stride, T);
  else
    hipLaunchKernelGGL(restart_inputs_kernel<MF32>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride,
                       graphs, pK, pK1, pK2, pK3, p_star, st, Ft, ft_stride, T);
  return hipGetLastError();
}

hipError_t launch_restart_vector(const DevLayout& L, int prec, const void* pK, const float* svec, PRState* st,
                                 void* q, double* slots, int members, hipStream_t s) {
  if (L.ntiles == 0) return hipSuccess;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(L.tiles);
  const uint32_t stride = sizeof(TileDesc) / 4;
  const uint32_t* graphs = base + offsetof(TileDesc, graph) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(restart_vector_kernel<MF64>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride,
                       graphs, pK, svec, st, q, slots);
  else
    hipLaunchKernelGGL(restart_vector_kernel<MF32>, dim3(L.ntiles / kWaves), dim3(kThreads), 0, s, base, stride,
                       graphs, pK, svec, st, q, slots);
  if (hipError_t e = hipGetLastError()) return e;
  // each member's sum of q into its delta field
  hipLaunchKernelGGL(pr_finish_kernel, dim3(members), dim3(kThreads), 0, s, st, slots, 0, 0.0, 0, 0, 0);
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
  hipError_t e;
  switch (prec) {
    case 0: e = launch_csr<MF64>(C, a.z_cur, EpiPR<MF64>{a}, a.st, s); break;
    case 1: e = launch_csr<MF32>(C, a.z_cur, EpiPR<MF32>{a}, a.st, s); break;
    case 2: e = launch_csr<MF32C>(C, a.z_cur, EpiPR<MF32C>{a}, a.st, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || a.fused) return e;
  return launch_pr_finish(a, s);
}

hipError_t launch_csr_pr_init(const DevCsr& C, int prec, const void* start, const void* tele, void* p0, void* z0,
                              const int32_t* outdeg, PRState* st, double* slots, hipStream_t s) {
  if (C.ntiles == 0) return hipSuccess;
  const uint32_t* base = reinterpret_cast<const uint32_t*>(C.tiles);
  const uint32_t stride = sizeof(CsrTile) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(pr_init_kernel<MF64>, dim3(C.ntiles / kWaves), dim3(kThreads), 0, s, base, stride, nullptr,
                       start, tele, p0, z0, outdeg, st, slots, 0);
  else
    hipLaunchKernelGGL(pr_init_kernel<MF32>, dim3(C.ntiles / kWaves), dim3(kThreads), 0, s, base, stride, nullptr,
                       start, tele, p0, z0, outdeg, st, slots, 0);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(pr_finish_kernel, dim3(1), dim3(kThreads), 0, s, st, slots, 0, 0.0, 0, 0, 0);
  return hipGetLastError();
}

hipError_t launch_pr_restore(int prec, const void* src, void* p, void* z, const int32_t* outdeg, int64_t r0,
                             int64_t r1, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  const uint32_t blocks = uint32_t(std::min<int64_t>((r1 - r0 + kThreads - 1) / kThreads, 4096));
  if (prec == 0)
    hipLaunchKernelGGL(pr_restore_kernel<double>, dim3(blocks), dim3(kThreads), 0, s, static_cast<const double*>(src),
                       static_cast<double*>(p), static_cast<double*>(z), outdeg, r0, r1);
  else
    hipLaunchKernelGGL(pr_restore_kernel<float>, dim3(blocks), dim3(kThreads), 0, s, static_cast<const float*>(src),
                       static_cast<float*>(p), static_cast<float*>(z), outdeg, r0, r1);
  return hipGetLastError();
}

hipError_t launch_pr_select(int prec, const PRState* st, const void* p0, const void* p1, void* out, int64_t n, int k,
                            hipStream_t s) {
  if (n == 0 || k == 0) return hipSuccess;
  const dim3 grid(uint32_t(std::min<int64_t>((n + kThreads - 1) / kThreads, 4096)), uint32_t(k));
  if (prec == 0)
    hipLaunchKernelGGL(pr_select_kernel<double>, grid, dim3(kThreads), 0, s, st, static_cast<const double*>(p0),
                       static_cast<const double*>(p1), static_cast<double*>(out), n);
  else
    hipLaunchKernelGGL(pr_select_kernel<float>, grid, dim3(kThreads), 0, s, st, static_cast<const float*>(p0),
                       static_cast<const float*>(p1), static_cast<float*>(out), n);
  return hipGetLastError();
}

// ------------------------------------------------------------ left product
namespace {
// LDS of one wave of the left tile kernel: c of up to 128 rows, their
// reference gaps, and the group sums T over the window's Z indices
template <class M>
struct LeftCarve {
  using PAcc = typename M::PAcc;
  uint32_t WC;
  __host__ __device__ static constexpr size_t c() { return 0; }
  __host__ __device__ static constexpr size_t gap() { return 128 * sizeof(PAcc); }
  __host__ __device__ static constexpr size_t T() { return align16(gap() + 128); }
  __host__ __device__ size_t wave_bytes() const { return align16(T() + (2 * size_t(WC) + 2) * sizeof(PAcc)); }
  __host__ __device__ size_t block_bytes() const { return kWaves * wave_bytes(); }
};

// One tile per wave: c = x (I - R)^{-1} on the tile's rows, the group sums
// T[f] of its A' entries read column-wise, and its window contribution
// out[j] = T[2j+2] + sum_{p <= j} T[2p+1], written to the tile's part slots.
template <class M>
__global__ void __launch_bounds__(kThreads) bv_left_tile_kernel(DevLayout L, DevLeft D,
                                                                const typename M::X* __restrict__ x) {
  using PAcc = typename M::PAcc;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t t = blockIdx.x * kWaves + wave;
  const TileDesc td = L.tiles[t];
  const LeftTile lt = D.lt[t];
  const LeftCarve<M> cv{L.wcap};
  unsigned char* ws = smem + size_t(wave) * cv.wave_bytes();
  PAcc* s_c = reinterpret_cast<PAcc*>(ws + cv.c());
  uint8_t* s_g = reinterpret_cast<uint8_t*>(ws + cv.gap());
  PAcc* T = reinterpret_cast<PAcc*>(ws + cv.T());
  const uint32_t nrows = td.nrows;
  // 1. c = x, then each row at level l - 1 adds its children (rows at level
  //    l that reference it: row r + g with gap g), from the deepest level up
  uint32_t lv[2];
  uint32_t lvmax = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t r = lane + 64u * q;
    lv[q] = 0;
    if (r < nrows) {
      const uint32_t inf = L.info[td.row0 + r];
      s_c[r] = PAcc(x[td.row0 + r]);
      s_g[r] = uint8_t(inf & 15u);
      lv[q] = (inf >> 4) & 15u;
      lvmax = max(lvmax, lv[q]);
    } else {
      s_g[r] = 0;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) lvmax = max(lvmax, uint32_t(__shfl_xor(int(lvmax), d, 64)));
  const uint32_t Tlen = 2 * td.winlen + 2;
  for (uint32_t k = lane; k < Tlen; k += 64) T[k] = PAcc(0);
  wave_sync();
  for (uint32_t l = lvmax; l >= 1; --l) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t r = lane + 64u * q;
      if (r < nrows && lv[q] == l - 1) {
        PAcc a = s_c[r];
        for (uint32_t g = 1; g <= 15 && r + g < nrows; ++g)
          if (s_g[r + g] == g) a += s_c[r + g];
        s_c[r] = a;
      }
    }
    wave_sync();
  }
  // 2. group sums: lane l takes whole groups [gs, ge) with entries [es, ee)
  {
    const uint32_t a = D.lanes[lt.lane0 + lane], b = D.lanes[lt.lane0 + lane + 1];
    uint32_t g = a >> 16;
    const uint32_t es = a & 0xFFFFu, ee = b & 0xFFFFu;
    const uint16_t* ent = D.ent + lt.e0;
    const uint16_t* grp = D.grp + lt.g0;
    PAcc acc = PAcc(0);
    for (uint32_t e = es; e < ee; e += 8) {
      uint32_t w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = e + k < ee ? uint32_t(ent[e + k]) : 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (e + k >= ee) break;
        const PAcc v = s_c[w[k] & 127u];
        acc += (w[k] & 0x8000u) ? -v : v;
        if (w[k] & 0x4000u) {
          T[grp[g]] = acc;
          acc = PAcc(0);
          ++g;
        }
      }
    }
  }
  wave_sync();
  // 3. out[j] = T[2j+2] + sum_{p <= j} T[2p+1]: lane chunks, a wave scan of
  //    the chunks' sums of the prefix entries
  {
    // the prefix of the difference array as a double pair: its terms cancel
    // (an interval adds at its start and subtracts at its end), so a plain
    // running sum would leave absolute errors of the window's mass on small
    // columns
    const uint32_t n = td.winlen;
    const uint32_t ch = (n + 63) / 64;
    const uint32_t b = min(n, lane * ch), e = min(n, b + ch);
    DPair tot{0.0, 0.0};
    for (uint32_t j = b; j < e; ++j) tot = dpair_add(tot, DPair{double(T[2 * j + 1]), 0.0});
    DPair inc = tot;
    for (int d = 1; d < 64; d <<= 1) {
      const DPair o{__shfl_up(inc.hi, d, 64), __shfl_up(inc.lo, d, 64)};
      if (lane >= uint32_t(d)) inc = dpair_add(o, inc);
    }
    DPair run{__shfl_up(inc.hi, 1, 64), __shfl_up(inc.lo, 1, 64)};
    if (lane == 0) run = DPair{0.0, 0.0};
    PAcc* part = static_cast<PAcc*>(D.part) + lt.part0;
    for (uint32_t j = b; j < e; ++j) {
      run = dpair_add(run, DPair{double(T[2 * j + 1]), 0.0});
      part[j] = PAcc((double(T[2 * j + 2]) + run.hi) + run.lo);
    }
  }
  // 4. the rows' c for the escapes' gather
  if (lt.esc) {
    PAcc* cb = static_cast<PAcc*>(D.cbuf);
    for (uint32_t r = lane; r < nrows; r += 64) cb[td.row0 + r] = s_c[r];
  }
}

// y_j = the contributions of the tiles whose window covers j (in tile order)
// + the escapes of column j (in row order); one wave per 64 columns.
template <class M>
__global__ void __launch_bounds__(kThreads) bv_left_gather_kernel(DevLayout L, DevLeft D, typename M::X* __restrict__ y) {
  using PAcc = typename M::PAcc;
  using X = typename M::X;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t g = blockIdx.x * kWaves + wave;
  if (uint64_t(g) * 64 >= D.n) return;
  const uint32_t j = g * 64 + lane_id();
  const PAcc* part = static_cast<const PAcc*>(D.part);
  double acc = 0.0;
  for (uint32_t k = D.cov_off[g]; k < D.cov_off[g + 1]; ++k) {
    const uint32_t t = D.cov[k];
    const uint32_t w0 = L.tiles[t].win0, wl = L.tiles[t].winlen, p0 = D.lt[t].part0;
    const uint32_t d = j - w0;
    if (j >= w0 && d < wl) acc += double(part[p0 + d]);
  }
  const PAcc* cb = static_cast<const PAcc*>(D.cbuf);
  for (uint32_t k = D.esc_off[g]; k < D.esc_off[g + 1]; ++k) {
    const LeftEscape e = D.esc[k];
    if (e.col == j) {
      const double v = double(cb[e.row & 0x7FFFFFFFu]);
      acc += (e.row & 0x80000000u) ? -v : v;
    }
  }
  if (j < D.n) y[j] = X(acc);
}

template <class M>
hipError_t launch_left(const DevLayout& L, const DevLeft& D, const void* x, void* y, hipStream_t s) {
  const size_t smem = LeftCarve<M>{L.wcap}.block_bytes();
  auto k1 = bv_left_tile_kernel<M>;
  if (hipError_t e = set_lds(reinterpret_cast<const void*>(k1), smem)) return e;
  if (L.ntiles)
    hipLaunchKernelGGL(k1, dim3(L.ntiles / kWaves), dim3(kThreads), smem, s, L, D,
                       static_cast<const typename M::X*>(x));
  if (hipError_t e = hipGetLastError()) return e;
  const uint32_t groups = (D.n + 63) / 64;
  hipLaunchKernelGGL(bv_left_gather_kernel<M>, dim3((groups + kWaves - 1) / kWaves), dim3(kThreads), 0, s, L, D,
                     static_cast<typename M::X*>(y));
  return hipGetLastError();
}
}  // namespace

size_t bv_left_lds_bytes(const DevLayout& L, int prec) {
  return prec == 1 ? LeftCarve<MF32>{L.wcap}.block_bytes() : LeftCarve<MF64>{L.wcap}.block_bytes();
}

hipError_t launch_bv_left(const DevLayout& L, const DevLeft& D, int prec, const void* x, void* y, hipStream_t s) {
  switch (prec) {
    case 0: return launch_left<MF64>(L, D, x, y, s);
    case 1: return launch_left<MF32>(L, D, x, y, s);
    case 2: return launch_left<MF32C>(L, D, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------- allocation-free working set
// The working set of the allocation-free PageRank: a fixed device array, one
// copy on every device the library's code is loaded on, held until the process
// ends.  In host code the name `scratch` stands for a host-side shadow, not a
// device address: host code only ever uses the address hipGetSymbolAddress
// returns for it, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
__global__ void pr_state_set_kernel(PRState* st, PRState v) {
  if (threadIdx.x == 0) *st = v;
}
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    if (hipError_t e = hipGetDevice(&cur)) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_pr_state_set(PRState* st, const PRState& v, hipStream_t s) {
  hipLaunchKernelGGL(pr_state_set_kernel, dim3(1), dim3(64), 0, s, st, v);
  return hipGetLastError();
}

}  // namespace bvmv
