// Host interpretation of the tiled device layout, in double precision.
// A test aid for the layout builder: it reads tiles, row info, the three
// entry streams and the long rows exactly as the kernels do and resolves the
// reuse levels, so layout mistakes show up without a device.  No product
// entry point calls it.
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bvmv.h"
#include "bv_decode.hpp"
#include "bv_layout.hpp"
// the compensated pair arithmetic of twosum.hpp in this host-only file (no
// HIP headers here): the device qualifiers are dropped
#define __host__
#define __device__
#define __forceinline__ inline
#include "twosum.hpp"

using namespace bvmv;

namespace bvmv {
int set_error(int code, const std::string& msg);
}

extern "C" int bvmv_layout_selfcheck(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts,
                                     const double* x, double* y, int64_t* stats) {
  if (!bitstream || !x || !y) return set_error(BVMV_EINVAL, "null argument");
  DecodedGraph dg;
  std::string err;
  if (decode_stream(static_cast<const uint8_t*>(bitstream), nbytes, 4, dg, err)) return set_error(BVMV_EFORMAT, err);
  LayoutParams prm;
  if (opts) {
    if (opts->tile_rows) prm.tile_rows = opts->tile_rows;
    if (opts->window_cap) prm.window_cap = opts->window_cap;
    if (opts->stage_bytes) prm.stage_bytes = opts->stage_bytes;
    prm.long_row_bytes = opts->long_row_bytes ? opts->long_row_bytes : prm.stage_bytes / 2;
    if (opts->interval_mode == 1) prm.min_interval = INT_MAX;
  }
  HostLayout hl;
  if (build_layout(dg, prm, 4, hl, err)) return set_error(BVMV_EINVAL, err);
  std::vector<double> part, yy;
  for (const TileDesc& td : hl.tiles) {
    if (tile_stage_bytes(td) > uint32_t(prm.stage_bytes)) return set_error(BVMV_EINVAL, "tile over the staging budget");
    const uint8_t* base = hl.data.data() + size_t(td.data16) * 16;
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(base);
    const uint32_t* w32 = reinterpret_cast<const uint32_t*>(base + align16u(td.n16 * 2u));
    const int64_t win0 = td.win0;
    // Z[0] = 0, Z[2p+1] = P[p] (prefix sums of the window), Z[2j+2] = x[win0+j]
    std::vector<double> Z(2 * size_t(td.winlen) + 2, 0.0);
    {
      double run = 0.0;
      for (uint32_t j = 0; j < td.winlen; ++j) {
        Z[2 * size_t(j) + 1] = run;
        Z[2 * size_t(j) + 2] = x[win0 + j];
        run += x[win0 + j];
      }
      Z[2 * size_t(td.winlen) + 1] = run;
    }
    uint32_t pairs = 0;
    part.assign(td.nrows, 0.0);
    yy.assign(td.nrows, 0.0);
    uint64_t o16 = 0, ow = 0, ol = 0;
    auto lng = [&](uint32_t w) {
      const int64_t c = win0 + int64_t(w & 0x7FFFFFFFu) - int64_t(kLongBias);
      return (w & 0x80000000u) ? -x[c] : x[c];
    };
    for (uint32_t r = 0; r < td.nrows; ++r) {
      const uint32_t inf = hl.info[td.row0 + r];
      const uint32_t ns = hl.ns[td.row0 + r];
      double a = 0.0;
      if (inf & kInfoLong) {
        const uint64_t len = uint64_t(info_nwide(inf)) | (uint64_t(ns) << 19);
        for (uint64_t k = 0; k < len; ++k) a += lng(hl.longs[td.long0 + ol + k]);
        ol += len;
      } else {
        for (uint32_t k = 0; k < ns; ++k) {
          const uint32_t w = s16[o16 + k];
          const uint32_t f = w & kS16Off;
          if (f == 0 || f > 2 * td.winlen + 1) return set_error(BVMV_EINVAL, "single outside the window");
          if (((w & kS16End) != 0) != (k + 1 == ns)) return set_error(BVMV_EINVAL, "single row-end bit misplaced");
          if (f & 1) {  // an interval: +P[b] then -P[a], a < b, opposite signs
            if (k + 1 >= ns) return set_error(BVMV_EINVAL, "unpaired prefix entry");
            const uint32_t w2 = s16[o16 + k + 1], f2 = w2 & kS16Off;
            if (!(f2 & 1) || f2 >= f || ((w ^ w2) & kS16Neg) == 0 || (w & kS16End))
              return set_error(BVMV_EINVAL, "malformed interval pair");
            const double v = Z[f] - Z[f2];
            a += (w & kS16Neg) ? -v : v;
            ++k;
            ++pairs;
            if (((w2 & kS16End) != 0) != (k + 1 == ns)) return set_error(BVMV_EINVAL, "single row-end bit misplaced");
            continue;
          }
          a += (w & kS16Neg) ? -Z[f] : Z[f];
        }
        o16 += ns;
        for (uint32_t k = 0; k < info_nwide(inf); ++k) {
          const uint32_t w = w32[ow + k];
          if (((w & kWideEnd) != 0) != (k + 1 == info_nwide(inf)))
            return set_error(BVMV_EINVAL, "wide row-end bit misplaced");
          const int64_t c = win0 + int64_t(w & kWideOff) - int64_t(kWideBias);
          if (c < 0 || c >= int64_t(hl.n)) return set_error(BVMV_EINVAL, "wide column out of range");
          a += (w & kWideNeg) ? -x[c] : x[c];
        }
        ow += info_nwide(inf);
        if ((inf >> 9) & 15u) return set_error(BVMV_EINVAL, "row info bits 9..12 set");
      }
      part[r] = a;
    }
    if (o16 != td.n16 || ow != td.nwide || pairs != td.nint)
      return set_error(BVMV_EINVAL, "tile stream count mismatch");
    // padding words up to 16 bytes are zero (no row-end bit)
    for (uint32_t k = td.n16; k < align16u(td.n16 * 2u) / 2; ++k)
      if (s16[k]) return set_error(BVMV_EINVAL, "nonzero singles padding");
    for (uint32_t k = td.nwide; k < align16u(td.nwide * 4u) / 4; ++k)
      if (w32[k]) return set_error(BVMV_EINVAL, "nonzero wide padding");
    for (uint32_t lv = 0; lv <= 15; ++lv)
      for (uint32_t r = 0; r < td.nrows; ++r) {
        const uint32_t inf = hl.info[td.row0 + r];
        if (info_level(inf) != lv) continue;
        const uint32_t g = info_g(inf);
        if (lv == 0) { yy[r] = part[r]; continue; }
        if (g == 0 || g > r) return set_error(BVMV_EINVAL, "reference outside the tile");
        yy[r] = yy[r - g] + part[r];
      }
    for (uint32_t r = 0; r < td.nrows; ++r) y[td.row0 + r] = yy[r];
  }
  if (stats) {
    stats[0] = int64_t(hl.tiles.size());
    stats[1] = hl.units;
    stats[2] = hl.diff_rows;
    stats[3] = hl.direct_rows;
    stats[4] = hl.long_rows;
    stats[5] = hl.escapes;
    stats[6] = hl.bytes();
    stats[7] = hl.m_prime;
    stats[8] = hl.max_level;
  }
  return BVMV_OK;
}

// Host interpretation of the left product's layout, in double precision, as
// the two device passes read it: c = x (I - R)^{-1} per tile from the deepest
// level up, the column-wise group sums T[f], the window contributions
// out[j] = T[2j+2] + sum_{p <= j} T[2p+1], then per column the covering
// tiles' contributions and the escapes.  x and y are HOST arrays of n doubles.
extern "C" int bvmv_left_selfcheck(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts,
                                   const double* x, double* y) {
  if (!bitstream || !x || !y) return set_error(BVMV_EINVAL, "null argument");
  DecodedGraph dg;
  std::string err;
  if (decode_stream(static_cast<const uint8_t*>(bitstream), nbytes, 4, dg, err)) return set_error(BVMV_EFORMAT, err);
  LayoutParams prm;
  if (opts) {
    if (opts->tile_rows) prm.tile_rows = opts->tile_rows;
    if (opts->window_cap) prm.window_cap = opts->window_cap;
    if (opts->stage_bytes) prm.stage_bytes = opts->stage_bytes;
    prm.long_row_bytes = opts->long_row_bytes ? opts->long_row_bytes : prm.stage_bytes / 2;
    if (opts->interval_mode == 1) prm.min_interval = INT_MAX;
  }
  HostLayout hl;
  if (build_layout(dg, prm, 4, hl, err)) return set_error(BVMV_EINVAL, err);
  LeftLayout ll;
  if (build_left_layout(hl, ll, err)) return set_error(BVMV_EINVAL, err);
  const int64_t n = hl.n;
  std::vector<double> part(ll.part_len, 0.0), cb(size_t(n), 0.0);
  for (size_t t = 0; t < hl.tiles.size(); ++t) {
    const TileDesc& td = hl.tiles[t];
    const LeftTile& lt = ll.tiles[t];
    std::vector<double> c(td.nrows), T(2 * size_t(td.winlen) + 2, 0.0);
    int lvmax = 0;
    for (uint32_t r = 0; r < td.nrows; ++r) {
      c[r] = x[td.row0 + r];
      lvmax = std::max<int>(lvmax, int(info_level(hl.info[td.row0 + r])));
    }
    for (int l = lvmax; l >= 1; --l)
      for (uint32_t r = 0; r < td.nrows; ++r) {
        if (int(info_level(hl.info[td.row0 + r])) != l - 1) continue;
        for (uint32_t g = 1; g <= 15 && r + g < td.nrows; ++g)
          if (info_g(hl.info[td.row0 + r + g]) == g) c[r] += c[r + g];
      }
    for (uint32_t l = 0; l < 64; ++l) {
      const uint32_t a = ll.lanes[lt.lane0 + l], b = ll.lanes[lt.lane0 + l + 1];
      uint32_t g = a >> 16;
      double acc = 0.0;
      for (uint32_t e = a & 0xFFFFu; e < (b & 0xFFFFu); ++e) {
        const uint32_t w = ll.entries[lt.e0 + e];
        if ((w & 127u) >= td.nrows) return set_error(BVMV_EINVAL, "left entry row outside the tile");
        acc += (w & 0x8000u) ? -c[w & 127u] : c[w & 127u];
        if (w & 0x4000u) {
          const uint32_t f = ll.groups[lt.g0 + g];
          if (f >= T.size()) return set_error(BVMV_EINVAL, "left group outside the window");
          T[f] = acc;
          acc = 0.0;
          ++g;
        }
      }
      if (acc != 0.0) return set_error(BVMV_EINVAL, "lane run ends inside a group");
    }
    DPair run{0.0, 0.0};
    for (uint32_t j = 0; j < td.winlen; ++j) {
      run = dpair_add(run, DPair{T[2 * size_t(j) + 1], 0.0});
      part[lt.part0 + j] = (T[2 * size_t(j) + 2] + run.hi) + run.lo;
    }
    if (lt.esc)
      for (uint32_t r = 0; r < td.nrows; ++r) cb[td.row0 + r] = c[r];
  }
  for (int64_t j = 0; j < n; ++j) {
    const size_t g = size_t(j / 64);
    double acc = 0.0;
    for (uint32_t k = ll.cov_off[g]; k < ll.cov_off[g + 1]; ++k) {
      const uint32_t t = ll.cov[k];
      const TileDesc& td = hl.tiles[t];
      if (j >= int64_t(td.win0) && j < int64_t(td.win0) + int64_t(td.winlen))
        acc += part[ll.tiles[t].part0 + uint64_t(j - td.win0)];
    }
    for (uint32_t k = ll.esc_off[g]; k < ll.esc_off[g + 1]; ++k) {
      const LeftEscape& e = ll.esc[k];
      if (int64_t(e.col) == j) acc += (e.row & 0x80000000u) ? -cb[e.row & 0x7FFFFFFFu] : cb[e.row & 0x7FFFFFFFu];
    }
    y[j] = acc;
  }
  return BVMV_OK;
}
