// Device layout of a compressed graph for the reuse product.
//
// The product y_i = y_{r_i} + sum_j A'_ij x_j (Section "Our Approach") is
// organised in tiles of consecutive rows.  A row is either
//   differential: y_i = y_{r_i} - sum over its skipped entries + sum over the
//     entries it adds (the row v_i - v_{r_i} of A'), or
//   direct: y_i = sum over its own list,
// and a row is differential only when that costs fewer entries than direct
// (the paper keeps v_i when |v_i - v_{r_i}| >= |v_i|) AND its reference lies
// in the same tile.  Reference chains therefore never leave a tile, so tiles
// are independent and a tile resolves its chains level by level in LDS
// (level = 0 for direct rows, level(r_i) + 1 otherwise, at most R).
//
// Entries are single ids or intervals [s, s+len) of consecutive ids, each
// with a sign.  Per tile, an x window [win0, win0+winlen) is staged in LDS;
// short rows are coded in 16-bit words relative to it:
//   bit 15 = subtract, bit 14 = interval;
//   single:   bits 0..13 = column - win0 (0x3FFF = escape: the next two words
//             hold the 32-bit two's-complement column - win0, high word first);
//   interval: bits 0..13 = start - win0, next word = length (both inside the
//             window).
// Rows coded in more than `long_row_words` words are long rows: their entries
// are 32-bit (bit 31 = subtract, bits 0..30 = column - win0 + 2^30, intervals
// expanded) and a whole block sums them.
//
// Row info (u32): bits 0..3 reference gap g (0 for direct), 4..7 level,
// bit 8 long, bits 9..31 length (words for short rows, entries for long).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "bv_decode.hpp"

namespace bvmv {

struct TileDesc {
  uint32_t row0;    // first row (global)
  uint32_t nrows;   // rows in the tile
  uint32_t word0;   // first 16-bit word of the short rows (multiple of 8)
  uint32_t nwords;  // words of the short rows
  uint32_t win0;    // first column of the x window
  uint32_t winlen;  // window length
  uint32_t long0;   // first 32-bit entry of the long rows
  uint32_t graph;   // member index inside a group (0 for a single graph)
};

struct LayoutParams {
  int tile_rows = 256;
  int window_cap = 2048;
  int word_cap = 4096;       // max short-row words per tile (LDS staging)
  int long_row_words = 192;
  int min_interval = 3;      // runs of at least this many ids become intervals
};

struct HostLayout {
  LayoutParams prm;
  std::vector<TileDesc> tiles;
  std::vector<uint32_t> info;
  std::vector<uint16_t> words;
  std::vector<uint32_t> longs;
  int64_t n = 0;
  int64_t units = 0, diff_rows = 0, direct_rows = 0, long_rows = 0, escapes = 0, m_prime = 0;
  int max_level = 0;
  int64_t bytes() const {
    return int64_t(tiles.size() * sizeof(TileDesc) + info.size() * 4 + words.size() * 2 + longs.size() * 4);
  }
};

constexpr uint32_t kInfoLong = 1u << 8;
constexpr uint32_t kEscape = 0x3FFF;
constexpr uint32_t kLongBias = 1u << 30;

int build_layout(const DecodedGraph& g, const LayoutParams& prm, int nthreads, HostLayout& out, std::string& err);

// Plain CSR tiles for the baseline: a tile is either a run of rows whose
// columns fit `word_cap` entries (staged in LDS) or a single long row.
struct CsrTile {
  uint32_t row0, nrows, c0, ncols;  // columns [c0, c0+ncols) of rowptr-relative storage
};
void build_csr_tiles(const uint64_t* rowptr, int64_t n, int rows_cap, int col_cap, std::vector<CsrTile>& tiles);

}  // namespace bvmv
