// Host interpretation of the tiled device layout, in double precision.
// A test aid for the layout builder: it reads tiles, row info, the three
// entry streams and the long rows exactly as the kernels do and resolves the
// reuse levels, so layout mistakes show up without a device.  No product
// entry point calls it.
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bvmv.h"
#include "bv_decode.hpp"
#include "bv_layout.hpp"

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
  }
  HostLayout hl;
  if (build_layout(dg, prm, 4, hl, err)) return set_error(BVMV_EINVAL, err);
  std::vector<double> part, yy;
  for (const TileDesc& td : hl.tiles) {
    if (tile_stage_bytes(td) > uint32_t(prm.stage_bytes)) return set_error(BVMV_EINVAL, "tile over the staging budget");
    const uint8_t* base = hl.data.data() + size_t(td.data16) * 16;
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(base);
    const uint32_t* w32 = reinterpret_cast<const uint32_t*>(base + align16u(td.n16 * 2u));
    const uint32_t* i32 = reinterpret_cast<const uint32_t*>(base + align16u(td.n16 * 2u) + align16u(td.nwide * 4u));
    const int64_t win0 = td.win0;
    part.assign(td.nrows, 0.0);
    yy.assign(td.nrows, 0.0);
    uint64_t o16 = 0, ow = 0, oi = 0, ol = 0;
    auto wide = [&](uint32_t w) {
      const int64_t c = win0 + int64_t(w & 0x7FFFFFFFu) - int64_t(kLongBias);
      return (w & 0x80000000u) ? -x[c] : x[c];
    };
    for (uint32_t r = 0; r < td.nrows; ++r) {
      const uint32_t inf = hl.info[td.row0 + r];
      const uint32_t ns = hl.ns[td.row0 + r];
      double a = 0.0;
      if (inf & kInfoLong) {
        const uint64_t len = uint64_t(info_nwide(inf)) | (uint64_t(ns) << 19);
        for (uint64_t k = 0; k < len; ++k) a += wide(hl.longs[td.long0 + ol + k]);
        ol += len;
      } else {
        for (uint32_t k = 0; k < ns; ++k) {
          const uint32_t w = s16[o16 + k];
          if ((w & 0x7FFFu) >= td.winlen) return set_error(BVMV_EINVAL, "single outside the window");
          a += (w & 0x8000u) ? -x[win0 + (w & 0x7FFFu)] : x[win0 + (w & 0x7FFFu)];
        }
        o16 += ns;
        for (uint32_t k = 0; k < info_nwide(inf); ++k) a += wide(w32[ow + k]);
        ow += info_nwide(inf);
        for (uint32_t k = 0; k < info_nint(inf); ++k) {
          const uint32_t w = i32[oi + k];
          const uint32_t s = (w >> 16) & 0x7FFFu, ln = w & 0xFFFFu;
          if (s + ln > td.winlen) return set_error(BVMV_EINVAL, "interval outside the window");
          double v = 0.0;
          for (uint32_t t = 0; t < ln; ++t) v += x[win0 + s + t];
          a += (w & 0x80000000u) ? -v : v;
        }
        oi += info_nint(inf);
      }
      part[r] = a;
    }
    if (o16 != td.n16 || ow != td.nwide || oi != td.nint) return set_error(BVMV_EINVAL, "tile stream count mismatch");
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
