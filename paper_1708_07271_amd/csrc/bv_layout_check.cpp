// Host interpretation of the tiled device layout, in double precision.
// A test aid for the layout builder: it reads tiles, row info, 16-bit words,
// escapes and long-row entries exactly as the kernels do and resolves the
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
    if (opts->long_row_words) prm.long_row_words = opts->long_row_words;
  }
  HostLayout hl;
  if (build_layout(dg, prm, 4, hl, err)) return set_error(BVMV_EINVAL, err);
  std::vector<double> part, yy;
  for (const TileDesc& td : hl.tiles) {
    part.assign(td.nrows, 0.0);
    yy.assign(td.nrows, 0.0);
    uint32_t woff = 0, loff = 0;
    for (uint32_t r = 0; r < td.nrows; ++r) {
      const uint32_t inf = hl.info[td.row0 + r];
      const uint32_t len = inf >> 9;
      double a = 0.0;
      if (inf & kInfoLong) {
        for (uint32_t k = 0; k < len; ++k) {
          const uint32_t v = hl.longs[td.long0 + loff + k];
          const int64_t c = int64_t(td.win0) + int64_t(v & 0x7FFFFFFFu) - int64_t(kLongBias);
          a += (v & 0x80000000u) ? -x[c] : x[c];
        }
        loff += len;
      } else {
        const uint16_t* w = hl.words.data() + td.word0 + woff;
        uint32_t k = 0;
        while (k < len) {
          const uint32_t wd = w[k++];
          const bool neg = wd & 0x8000u;
          const uint32_t off = wd & 0x3FFFu;
          double v = 0.0;
          if (wd & 0x4000u) {
            const uint32_t ln = w[k++];
            if (off + ln > td.winlen) return set_error(BVMV_EINVAL, "interval outside the window");
            for (uint32_t t = 0; t < ln; ++t) v += x[td.win0 + off + t];
          } else if (off == kEscape) {
            const int32_t rel = int32_t((uint32_t(w[k]) << 16) | uint32_t(w[k + 1]));
            k += 2;
            v = x[int64_t(td.win0) + rel];
          } else {
            if (off >= td.winlen) return set_error(BVMV_EINVAL, "offset outside the window");
            v = x[td.win0 + off];
          }
          a += neg ? -v : v;
        }
        woff += len;
      }
      part[r] = a;
    }
    if (woff != td.nwords) return set_error(BVMV_EINVAL, "tile word count mismatch");
    for (uint32_t lv = 0; lv <= 15; ++lv)
      for (uint32_t r = 0; r < td.nrows; ++r) {
        const uint32_t inf = hl.info[td.row0 + r];
        if (((inf >> 4) & 15u) != lv) continue;
        const uint32_t g = inf & 15u;
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
