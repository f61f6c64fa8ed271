// Replays, on the host, the global-memory index arithmetic of the tile
// kernel (bv_kernels.hip) over every tile of a layout built from each given
// bitstream, for every lane and every round the kernel issues:
//   - the first stream round of the running-sum mode (one address, 8 dwords
//     from min(d0, last)) and its later rounds (8 dwords from min(d0 + r,
//     last) while r < the wave's largest dword count);
//   - the clamped rounds and row-end counts of the other passes and of the
//     wide entries;
//   - row info / count loads, x-window loads (every tile loads its first
//     stream round and window values, also without singles or a window),
//     Z indices of the singles, and the columns the wide and long entries
//     gather.
// Every stream dword index must lie below the device data array's size plus
// its zero padding (kDataPadBytes), every gathered column below n, every Z
// index inside the staged window.  Exit status 0 when all hold; built with g++
// by tests/test_host.py.  The formulas are written out here from the kernel
// source (flat_chunk, Chunk, load_round_raw / load_round_z / load_round).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "bv_decode.hpp"
#include "bv_layout.hpp"
#include "kernels.hpp"

namespace bvmv {
int set_error(int code, const std::string& msg) {
  std::fprintf(stderr, "library error %d: %s\n", code, msg.c_str());
  return code;
}
}  // namespace bvmv

using namespace bvmv;

static const uint32_t kRoundW = 8;
static uint32_t flat_chunk(uint32_t E, uint32_t Q) { return ((E + 63) / 64 + Q - 1) / Q * Q; }

struct ChunkH {
  uint32_t b, nd, d0, last;
  ChunkH(uint32_t lane, uint32_t E, uint32_t C, uint32_t P) {
    b = lane * C;
    const uint32_t cnt = b < E ? std::min(E, b + C) - b : 0u;
    nd = (cnt + P - 1) / P;
    d0 = b / P;
    last = E ? (E + P - 1) / P - 1 : 0u;
  }
};

static int fails = 0;
static void bad(const char* what, size_t t, uint64_t v, uint64_t lim) {
  if (fails++ < 20) std::fprintf(stderr, "tile %zu: %s %llu >= %llu\n", t, what, (unsigned long long)v,
                                 (unsigned long long)lim);
}

static void replay(const HostLayout& hl, int64_t n) {
  const uint64_t data_dw = (hl.data.size() + kDataPadBytes) / 4;
  const uint32_t* data = reinterpret_cast<const uint32_t*>(hl.data.data());
  for (size_t t = 0; t < hl.tiles.size(); ++t) {
    const TileDesc& td = hl.tiles[t];
    const uint64_t base = uint64_t(td.data16) * 4;   // dword index of the singles stream
    if (td.nrows && uint64_t(td.row0) + td.nrows > uint64_t(n)) bad("row", t, td.row0 + td.nrows, n);
    if (td.winlen && uint64_t(td.win0) + td.winlen > uint64_t(n)) bad("window end", t, td.win0 + td.winlen, n);
    const uint32_t n16 = td.n16, nwide = td.nwide;
    // the tile's first loads are unconditional: the first stream round (also
    // for a tile without singles) and the lanes' first window values, at
    // win0 + min(b + j, max(winlen, 1) - 1) (also for a tile without a window)
    {
      const uint32_t C = flat_chunk(n16, 2);
      for (uint32_t lane = 0; lane < 64; ++lane) {
        const ChunkH ch(lane, n16, C, 2);
        const uint64_t hi0 = base + std::min(ch.d0, ch.last) + kRoundW - 1;
        if (hi0 >= data_dw) bad("unconditional first-round dword", t, hi0, data_dw);
        const uint32_t wl = std::max(td.winlen, 1u), w = (wl + 63) / 64, b = std::min(wl, lane * w);
        for (uint32_t j = 0; j < 16; ++j) {
          const uint64_t col = uint64_t(td.win0) + std::min(b + j, wl - 1);
          if (col >= uint64_t(n)) bad("window value column", t, col, n);
        }
      }
    }
    if (n16) {
      const uint32_t C = flat_chunk(n16, 2);
      uint32_t ndmax = (std::min(C, n16) + 1) / 2;
      for (uint32_t lane = 0; lane < 64; ++lane) {
        const ChunkH ch(lane, n16, C, 2);
        // first round, one address (running-sum mode) or clamped words
        const uint64_t hi0 = base + std::min(ch.d0, ch.last) + kRoundW - 1;
        if (hi0 >= data_dw) bad("first-round dword", t, hi0, data_dw);
        for (uint32_t r = kRoundW; r < ndmax; r += kRoundW) {
          const uint64_t hi = base + std::min(ch.d0 + r, ch.last) + kRoundW - 1;
          if (hi >= data_dw) bad("later-round dword", t, hi, data_dw);
        }
        for (uint32_t r = kRoundW; r < ch.nd; ++r)   // row-end counts past the first round
          if (base + ch.d0 + r > base + ch.last) bad("row-end dword", t, ch.d0 + r, ch.last + 1);
      }
      // every singles entry indexes the staged window Z[0 .. 2 winlen + 1]
      const uint16_t* s16 = reinterpret_cast<const uint16_t*>(data + base);
      for (uint32_t e = 0; e < n16; ++e) {
        const uint32_t f = s16[e] & kS16Off;
        if (f > 2 * td.winlen + 1) bad("Z index", t, f, 2 * td.winlen + 2);
      }
    }
    if (nwide) {
      const uint64_t wbase = base + align16u(n16 * 2u) / 4;
      const uint32_t C = flat_chunk(nwide, 1);
      for (uint32_t lane = 0; lane < 64; ++lane) {
        const ChunkH ch(lane, nwide, C, 1);
        for (uint32_t r = 0; r < std::max(ch.nd, kRoundW); ++r) {
          const uint64_t idx = wbase + std::min(ch.d0 + r, ch.last);
          if (idx >= data_dw) bad("wide dword", t, idx, data_dw);
        }
      }
      for (uint32_t e = 0; e < nwide; ++e) {
        const int64_t col = int64_t(data[wbase + e] & kWideOff) - int64_t(kWideBias) + int64_t(td.win0);
        if (col < 0 || col >= n) bad("wide column", t, uint64_t(col), uint64_t(n));
      }
    }
  }
  // long rows: every entry's column
  for (size_t t = 0; t < hl.tiles.size(); ++t) {
    const TileDesc& td = hl.tiles[t];
    uint64_t off = td.long0;
    for (uint32_t r = 0; r < td.nrows; ++r) {
      const uint32_t inf = hl.info[td.row0 + r];
      if (!(inf & kInfoLong)) continue;
      const uint64_t len = uint64_t(inf >> 13) | (uint64_t(hl.ns[td.row0 + r]) << 19);
      for (uint64_t k = 0; k < len; ++k) {
        if (off + k >= hl.longs.size()) { bad("long entry", t, off + k, hl.longs.size()); break; }
        const int64_t col = int64_t(hl.longs[off + k] & 0x7FFFFFFFu) - int64_t(kLongBias) + int64_t(td.win0);
        if (col < 0 || col >= n) bad("long column", t, uint64_t(col), uint64_t(n));
      }
      off += len;
    }
  }
}

int main(int argc, char** argv) {
  const int shapes[][4] = {{64, 256, 4096, 2048}, {16, 64, 512, 16}, {32, 256, 1024, 40},
                           {128, 768, 6144, 3072}, {64, 2048, 8192, 4096}, {8, 64, 512, 16}};
  size_t layouts = 0, tiles = 0;
  for (int i = 1; i < argc; ++i) {
    std::ifstream f(argv[i], std::ios::binary);
    std::vector<uint8_t> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    DecodedGraph g;
    std::string err;
    if (decode_stream(bytes.data(), bytes.size(), 4, g, err)) {
      std::fprintf(stderr, "%s: %s\n", argv[i], err.c_str());
      return 1;
    }
    for (const auto& sh : shapes) {
      LayoutParams prm;
      prm.tile_rows = sh[0];
      prm.window_cap = sh[1];
      prm.stage_bytes = sh[2];
      prm.long_row_bytes = sh[3];
      HostLayout hl;
      if (build_layout(g, prm, 4, hl, err)) {
        std::fprintf(stderr, "%s: layout: %s\n", argv[i], err.c_str());
        return 1;
      }
      replay(hl, g.n);
      ++layouts;
      tiles += hl.tiles.size();
    }
  }
  if (fails) return 1;
  std::printf("ok %zu layouts %zu tiles\n", layouts, tiles);
  return 0;
}
