// Device layout of a compressed graph for the reuse product.
//
// The product y_i = y_{r_i} + sum_j A'_ij x_j (Section "Our Approach") is
// organised in tiles of consecutive rows.  A row is either
//   differential: y_i = y_{r_i} - sum over the reference entries it skips +
//     sum over the entries it adds (the row v_i - v_{r_i} of A'), or
//   direct: y_i = sum over its own list,
// and a row is differential only when that costs less than direct (the paper
// keeps v_i when |v_i - v_{r_i}| >= |v_i|) AND its reference lies in the same
// tile.  Reference chains therefore never leave a tile: tiles are independent
// and each resolves its chains level by level in LDS (level 0 for direct
// rows, level(r_i) + 1 otherwise, at most R).
//
// A row's entries are signed single ids or signed intervals [s, s+len).  Per
// tile an x window [win0, win0+winlen) is staged in LDS together with its
// prefix sums P[p] = x[win0] + ... + x[win0+p-1] (p = 0..winlen), both as
// doubles in one array Z: Z[0] = 0, Z[2p+1] = P[p], Z[2j+2] = x[win0+j].  An
// interval inside the window is the pair +P[s+len] - P[s] (the O(1) interval
// sum of Section "Our Approach"), so the tile's entries form two fixed-width
// streams, each in row order:
//   singles (u16):   bit 15 = subtract, bit 14 = last entry of its row,
//                    bits 0..13 = f, the Z index: 2j+2 for column win0+j,
//                    2p+1 for P[p] (an interval's pair, upper end first);
//                    f = 0 is the zero padding word, which adds nothing;
//   wide (u32):      bit 31 = subtract, bit 30 = last wide entry of its row,
//                    bits 0..29 = column - win0 + 2^29 (columns outside the
//                    window; intervals that leave the window are expanded
//                    into these).
// The row-end bits let a wave cut an equal share of a stream into row pieces
// without reading the row offsets.  The two streams of a tile are contiguous,
// each padded with zero words to 16 bytes, at data16 * 16 bytes.  Rows whose
// staged bytes exceed `long_row_bytes` (or with a column too far from the
// window for the wide code) are long rows: all their entries go to a
// per-graph long stream (u32: bit 31 = subtract, bits 0..30 = column - win0 +
// 2^30, intervals expanded) that the tile's whole wavefront sums.
//
// Row info (u32): bits 0..3 reference gap g (0 = direct), 4..7 level, bit 8
// long, bits 9..12 zero, bits 13..31 wide count (long rows: low 19 bits of
// the long-entry count).  Row `ns` (u16): singles-stream count (long rows:
// high bits of the long-entry count).  TileDesc.nint counts the tile's
// interval pairs (0: the tile needs no prefix sums).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "bv_decode.hpp"

namespace bvmv {

struct TileDesc {
  uint32_t row0;    // first row (global)
  uint32_t nrows;   // rows in the tile
  uint32_t data16;  // tile streams at data16 * 16 bytes
  uint32_t n16;     // singles-stream entries
  uint32_t nwide;   // wide entries
  uint32_t nint;    // interval pairs among the singles
  uint32_t win0;    // first column of the x window
  uint32_t winlen;  // window length
  uint32_t long0;   // first long entry of the tile's long rows
  uint32_t graph;   // member index inside a group (0 for a single graph)
  uint32_t pad0, pad1;
};

inline uint32_t align16u(uint32_t b) { return (b + 15u) & ~15u; }
// byte size of a tile's streams
inline uint32_t tile_stage_bytes(const TileDesc& t) { return align16u(t.n16 * 2u) + align16u(t.nwide * 4u); }

// A tile is processed by one 64-lane wavefront (up to 2 consecutive rows per
// lane); a block holds kTilesPerBlock consecutive tiles, and tile lists are
// padded with empty tiles to a multiple of it, so a block never spans two
// graphs of a group.
constexpr int kTileRowsMax = 128;
constexpr int kTilesPerBlock = 4;

struct LayoutParams {
  int tile_rows = 64;
  int window_cap = 256;
  int stage_bytes = 4096;      // max staged stream bytes per tile (LDS)
  int long_row_bytes = 2048;   // rows staging more than this are summed by the whole wave
  int min_interval = 3;        // runs of at least this many ids become intervals (a huge value: none)
};

struct HostLayout {
  LayoutParams prm;
  std::vector<TileDesc> tiles;
  std::vector<uint32_t> info;
  std::vector<uint16_t> ns;
  std::vector<uint8_t> data;    // staged streams of all tiles (16-byte aligned blocks)
  std::vector<uint32_t> longs;
  int64_t n = 0;
  int64_t units = 0, diff_rows = 0, direct_rows = 0, long_rows = 0, escapes = 0, m_prime = 0;
  int64_t n_singles = 0, n_wide = 0, n_intervals = 0;
  int max_level = 0;
  int64_t bytes() const {
    return int64_t(tiles.size() * sizeof(TileDesc) + info.size() * 4 + ns.size() * 2 + data.size() +
                   longs.size() * 4);
  }
};

constexpr uint32_t kInfoLong = 1u << 8;
constexpr uint32_t kLongBias = 1u << 30;    // long stream: column - win0 + 2^30
constexpr uint32_t kS16Neg = 0x8000u, kS16End = 0x4000u, kS16Off = 0x3FFFu;  // kS16Off masks f
constexpr uint32_t kWideNeg = 0x80000000u, kWideEnd = 0x40000000u, kWideOff = 0x3FFFFFFFu;
constexpr uint32_t kWideBias = 1u << 29;    // wide stream: column - win0 + 2^29

inline uint32_t info_g(uint32_t inf) { return inf & 15u; }
inline uint32_t info_level(uint32_t inf) { return (inf >> 4) & 15u; }
inline uint32_t info_nwide(uint32_t inf) { return inf >> 13; }

int build_layout(const DecodedGraph& g, const LayoutParams& prm, int nthreads, HostLayout& out, std::string& err);

// ------------------------------------------------------------ left product
// Layout of the left product y = x A on the same tiles (PageRank's p M,
// Section "PageRank"), without the transposed graph: with R the tile's
// references (R_ik = [r_i = k]), A = (I - R)^{-1} A', so x A = c A' with
// c = x (I - R)^{-1}, c_k = x_k + the sum of c_i over the rows i that
// reference k.  Per tile, A' is read column-wise: the tile's singles entries
// sorted by their Z index f (then by row) form groups, one per distinct f;
// a group's sum T[f] = sum of s * c_row over its entries, with s the entry's
// sign for a column (f = 2j+2) and the opposite sign for a prefix entry
// (f = 2p+1: an interval [a, b) of row i puts +c_i at P[a] and -c_i at P[b]
// of a difference array).  The tile's window contribution is then
// out[j] = T[2j+2] + sum_{p <= j} T[2p+1].  Entries outside the window (wide
// entries, long rows) are escapes, summed per column from a global list.
//   entries (u16): bits 0..6 tile row, bit 14 last entry of its group,
//                  bit 15 subtract;
//   groups  (u16): f of each group, ascending;
//   lanes   (u32 x 65 per tile): (group start << 16) | entry start of lane l's
//                  contiguous run of whole groups, balanced on entries.
struct LeftTile {
  uint32_t e0;      // first entry (u16 index into entries)
  uint32_t g0;      // first group (index into groups)
  uint32_t lane0;   // lane table at lanes[lane0 .. lane0 + 64]
  uint32_t part0;   // the tile's window contribution at part[part0 .. part0 + winlen)
  uint32_t esc;     // 1 if the tile has escapes (its rows' c go to the global c)
  uint32_t pad0, pad1, pad2;
};
struct LeftEscape {
  uint32_t col;     // target column
  uint32_t row;     // bit 31 subtract, bits 0..30 global row
};
struct LeftLayout {
  std::vector<LeftTile> tiles;     // one per layout tile
  std::vector<uint16_t> entries;   // padded to 8 entries per tile
  std::vector<uint16_t> groups;
  std::vector<uint32_t> lanes;
  std::vector<LeftEscape> esc;     // sorted by (col, row)
  std::vector<uint32_t> esc_off;   // per 64-column group: escapes [esc_off[g], esc_off[g+1])
  std::vector<uint32_t> cov_off;   // per 64-column group: covering tiles cov[cov_off[g] .. cov_off[g+1])
  std::vector<uint32_t> cov;       // tile ids, ascending within a group
  uint64_t part_len = 0;           // elements of the window contributions
  int64_t bytes() const {
    return int64_t(tiles.size() * sizeof(LeftTile) + entries.size() * 2 + groups.size() * 2 + lanes.size() * 4 +
                   esc.size() * sizeof(LeftEscape) + esc_off.size() * 4 + cov_off.size() * 4 + cov.size() * 4);
  }
};
int build_left_layout(const HostLayout& hl, LeftLayout& out, std::string& err);

// Plain CSR tiles for the baseline: runs of rows whose column ids fit the
// staging budget (with an x window chosen like the compressed tiles'), or a
// single long row summed block-wide (bit 31 of nrows).
struct CsrTile {
  uint32_t row0, nrows, c0, ncols, win0, winlen, pad0, pad1;
};
// Row tiles of a CSR matrix with n rows for the CSR tile kernel.  Windows
// cover ids below xlen only (ids at or above it are not columns of x), and
// every window lies inside [0, xlen).
void build_csr_tiles(const uint64_t* rowptr, const uint32_t* col, int64_t n, int rows_cap, int col_cap,
                     int long_cols, int window_cap, std::vector<CsrTile>& tiles, uint64_t xlen);

}  // namespace bvmv
