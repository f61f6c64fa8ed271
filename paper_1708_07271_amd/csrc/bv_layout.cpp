// Host construction of the tiled device layout (see bv_layout.hpp).
#include "bv_layout.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>

namespace bvmv {
namespace {

struct Entry {
  uint32_t col;
  uint32_t len;  // 0 = single id, else interval length
  bool neg;
};

// Split a sorted id list into intervals (runs >= min_len) and singles.
void to_entries(const uint32_t* a, size_t na, bool neg, int min_len, std::vector<Entry>& out) {
  for (size_t k = 0; k < na;) {
    size_t e = k + 1;
    while (e < na && a[e] == a[e - 1] + 1) ++e;
    if (int64_t(e - k) >= min_len) {
      size_t s = k;
      while (s < e) {  // lengths fit 16 bits
        size_t l = std::min<size_t>(e - s, 65535);
        out.push_back({a[s], uint32_t(l), neg});
        s += l;
      }
    } else {
      for (size_t t = k; t < e; ++t) out.push_back({a[t], 0, neg});
    }
    k = e;
  }
}

// staged bytes if every entry falls inside the window
int64_t entry_bytes(const std::vector<Entry>& es) {
  int64_t b = 0;
  for (auto& e : es) b += e.len ? 4 : 2;
  return b;
}

struct RowPlan {
  std::vector<Entry> ent;
  int g = 0;                // 0 = direct
  int64_t est = 0;          // staged bytes if every entry falls in the window
  bool force_long = false;  // its coded streams alone overflow a tile
};

struct ChunkOut {
  std::vector<TileDesc> tiles;
  std::vector<uint32_t> info;
  std::vector<uint16_t> ns;
  std::vector<uint8_t> data;
  std::vector<uint32_t> longs;
  int64_t units = 0, diff_rows = 0, direct_rows = 0, long_rows = 0, escapes = 0, m_prime = 0;
  int64_t n_singles = 0, n_wide = 0, n_intervals = 0;
  int max_level = 0;
  std::string err;
};

inline uint32_t long_code(int64_t col, int64_t win0, bool neg) {
  return (neg ? 0x80000000u : 0u) | uint32_t(col - win0 + int64_t(kLongBias));
}
inline bool wide_fits(int64_t col, int64_t win0) {
  return col - win0 >= -int64_t(kWideBias) && col - win0 < int64_t(kWideBias);
}
inline uint32_t wide_code(int64_t col, int64_t win0, bool neg) {
  return (neg ? kWideNeg : 0u) | uint32_t(col - win0 + int64_t(kWideBias));
}

// window of at most `cap` columns covering the most points (sorted in place)
void best_window(std::vector<uint32_t>& pts, int cap, uint32_t def, uint32_t& win0, uint32_t& winlen) {
  std::sort(pts.begin(), pts.end());
  win0 = def;
  winlen = 0;
  if (pts.empty()) return;
  size_t best_a = 0, best_b = 0, b = 0;
  for (size_t a = 0; a < pts.size(); ++a) {
    if (b < a) b = a;
    while (b + 1 < pts.size() && int64_t(pts[b + 1]) - int64_t(pts[a]) < cap) ++b;
    if (b - a > best_b - best_a) { best_a = a; best_b = b; }
  }
  win0 = pts[best_a];
  winlen = pts[best_b] - pts[best_a] + 1;
}

class Builder {
 public:
  Builder(const DecodedGraph& g, const LayoutParams& p) : g_(g), p_(p) {}

  void plan_row(int64_t i, int64_t i0, RowPlan& rp, std::vector<uint32_t>& K, std::vector<uint32_t>& E,
                std::vector<Entry>& tmp) {
    const uint32_t* Li = g_.col.data() + g_.rowptr[i];
    const size_t di = size_t(g_.rowptr[i + 1] - g_.rowptr[i]);
    rp.ent.clear();
    rp.force_long = false;
    to_entries(Li, di, false, p_.min_interval, rp.ent);
    rp.g = 0;
    rp.est = entry_bytes(rp.ent);
    const int gi = g_.refs[size_t(i)];
    if (gi == 0 || i - gi < i0 || di == 0) return;
    const int64_t r = i - gi;
    const uint32_t* Lr = g_.col.data() + g_.rowptr[r];
    const size_t dr = size_t(g_.rowptr[r + 1] - g_.rowptr[r]);
    K.clear();
    E.clear();
    std::set_difference(Lr, Lr + dr, Li, Li + di, std::back_inserter(K));
    std::set_difference(Li, Li + di, Lr, Lr + dr, std::back_inserter(E));
    tmp.clear();
    to_entries(K.data(), K.size(), true, p_.min_interval, tmp);
    to_entries(E.data(), E.size(), false, p_.min_interval, tmp);
    const int64_t b = entry_bytes(tmp);
    if (b < rp.est) {
      rp.ent.swap(tmp);
      rp.g = gi;
      rp.est = b;
    }
  }

  // the paper's nonzeros of A' for row i: |v_i - v_r| if smaller than |v_i|, else |v_i|
  int64_t mprime_row(int64_t i) {
    const int64_t di = int64_t(g_.rowptr[i + 1] - g_.rowptr[i]);
    const int gi = g_.refs[size_t(i)];
    if (gi == 0) return di;
    const int64_t r = i - gi;
    const uint32_t* Li = g_.col.data() + g_.rowptr[i];
    const uint32_t* Lr = g_.col.data() + g_.rowptr[r];
    const int64_t dr = int64_t(g_.rowptr[r + 1] - g_.rowptr[r]);
    int64_t a = 0, b = 0, common = 0;
    while (a < di && b < dr) {
      if (Li[a] == Lr[b]) { ++common; ++a; ++b; }
      else if (Li[a] < Lr[b]) ++a;
      else ++b;
    }
    const int64_t diff = (di - common) + (dr - common);
    return diff < di ? diff : di;
  }

  bool is_long_row(const RowPlan& rp) const { return rp.force_long || rp.est > p_.long_row_bytes; }

  void run_chunk(int64_t lo, int64_t hi, ChunkOut& co) {
    std::vector<RowPlan> plans;
    std::vector<uint32_t> K, E;
    std::vector<Entry> tmp;
    std::vector<uint8_t> level(size_t(hi - lo), 0);
    for (int64_t i = lo; i < hi; ++i) co.m_prime += mprime_row(i);
    int64_t i = lo;
    while (i < hi) {
      const int64_t i0 = i;
      plans.clear();
      int64_t bytes = 0;
      while (i < hi && i - i0 < p_.tile_rows) {
        plans.emplace_back();
        RowPlan& rp = plans.back();
        plan_row(i, i0, rp, K, E, tmp);
        const bool lng = is_long_row(rp);
        if (!lng && bytes + rp.est + 48 > p_.stage_bytes && i > i0) {
          plans.pop_back();
          break;
        }
        if (!lng) bytes += rp.est;
        ++i;
      }
      // emit; shrink the tile while escapes push it past the staging budget
      for (;;) {
        const int rc = emit_tile(i0, plans, level.data() - lo, co);
        if (rc == kEmitted) break;
        if (rc == kRetry) continue;  // a row was made long
        if (plans.size() == 1) {
          if (plans[0].force_long) { co.err = "row does not fit a tile"; return; }
          plans[0].force_long = true;  // sum it block-wide instead
          continue;
        }
        plans.pop_back();
        --i;
      }
      if (!co.err.empty()) return;
    }
  }

  // kEmitted, or (emitting nothing) kOverflow if the staged streams exceed
  // the budget, or kRetry after marking long a row whose column is out of
  // the wide code's reach.
  static constexpr int kEmitted = 0, kOverflow = 1, kRetry = 2;
  int emit_tile(int64_t i0, std::vector<RowPlan>& plans, uint8_t* level, ChunkOut& co) {
    const int64_t nr = int64_t(plans.size());
    std::vector<uint32_t> pts;
    for (auto& rp : plans) {
      if (is_long_row(rp)) continue;
      for (auto& e : rp.ent) {
        pts.push_back(e.col);
        if (e.len) pts.push_back(e.col + e.len - 1);
      }
    }
    uint32_t win0, winlen;
    best_window(pts, p_.window_cap, uint32_t(i0), win0, winlen);
    auto in_win = [&](int64_t c) { return c >= int64_t(win0) && c < int64_t(win0) + int64_t(winlen); };
    std::vector<uint16_t> s16;
    std::vector<uint32_t> w32;
    uint32_t npairs = 0;
    std::vector<uint32_t> info(static_cast<size_t>(nr), 0u);
    std::vector<uint16_t> nsv(static_cast<size_t>(nr), 0);
    const size_t lbase = co.longs.size();
    int64_t esc = 0;
    for (int64_t k = 0; k < nr; ++k) {
      RowPlan& rp = plans[size_t(k)];
      if (!is_long_row(rp))
        for (auto& e : rp.ent) {
          const uint32_t cnt = e.len ? e.len : 1;
          if (!wide_fits(e.col, win0) || !wide_fits(int64_t(e.col) + cnt - 1, win0)) {
            rp.force_long = true;
            return kRetry;
          }
        }
    }
    for (int64_t k = 0; k < nr; ++k) {
      const RowPlan& rp = plans[size_t(k)];
      const int64_t i = i0 + k;
      const bool lng = is_long_row(rp);
      const int lvl = rp.g ? level[i - rp.g] + 1 : 0;
      level[i] = uint8_t(lvl);
      uint64_t c16 = 0, cw = 0;
      if (!lng) {
        const size_t b16 = s16.size(), bw = w32.size();
        auto single = [&](uint32_t c, bool neg) {
          if (in_win(c)) {
            s16.push_back(uint16_t((neg ? kS16Neg : 0u) | (2u * (c - win0) + 2u)));
          } else {
            w32.push_back(wide_code(c, win0, neg));
            ++esc;
          }
        };
        for (auto& e : rp.ent) {
          if (e.len == 0) {
            single(e.col, e.neg);
          } else if (in_win(e.col) && in_win(int64_t(e.col) + e.len - 1)) {
            // +P[s+len] - P[s] (signs swapped for a subtracted interval)
            const uint32_t sw0 = e.col - win0;
            s16.push_back(uint16_t((e.neg ? kS16Neg : 0u) | (2u * (sw0 + e.len) + 1u)));
            s16.push_back(uint16_t((e.neg ? 0u : kS16Neg) | (2u * sw0 + 1u)));
            ++npairs;
          } else {
            for (uint32_t t = 0; t < e.len; ++t) single(e.col + t, e.neg);
          }
        }
        c16 = s16.size() - b16;
        cw = w32.size() - bw;
        if (c16) s16.back() = uint16_t(s16.back() | kS16End);
        if (cw) w32.back() |= kWideEnd;
        if (c16 > 0xFFFF || cw >= (1u << 19)) {
          co.longs.resize(lbase);
          return kOverflow;
        }
      } else {
        for (auto& e : rp.ent) {
          const uint32_t cnt = e.len ? e.len : 1;
          for (uint32_t t = 0; t < cnt; ++t) co.longs.push_back(long_code(int64_t(e.col) + t, win0, e.neg));
          cw += cnt;
        }
        if (cw >= (uint64_t(1) << 35)) {
          co.err = "row too long for the layout";
          return kEmitted;
        }
        c16 = cw >> 19;
        cw &= (1u << 19) - 1;
      }
      info[size_t(k)] = uint32_t(rp.g) | (uint32_t(lvl) << 4) | (lng ? kInfoLong : 0u) | (uint32_t(cw) << 13);
      nsv[size_t(k)] = uint16_t(c16);
    }
    TileDesc td{};
    td.row0 = uint32_t(i0);
    td.nrows = uint32_t(nr);
    td.n16 = uint32_t(s16.size());
    td.nwide = uint32_t(w32.size());
    td.nint = npairs;
    if (tile_stage_bytes(td) > uint32_t(p_.stage_bytes)) {
      co.longs.resize(lbase);
      return kOverflow;
    }
    // append the two streams, each padded to 16 bytes
    const size_t base = co.data.size();
    td.data16 = uint32_t(base / 16);
    co.data.resize(base + tile_stage_bytes(td), 0);
    uint8_t* dst = co.data.data() + base;
    if (!s16.empty()) std::memcpy(dst, s16.data(), s16.size() * 2);
    dst += align16u(td.n16 * 2u);
    if (!w32.empty()) std::memcpy(dst, w32.data(), w32.size() * 4);

    td.win0 = win0;
    td.winlen = winlen;
    td.long0 = uint32_t(lbase);
    td.graph = 0;
    co.tiles.push_back(td);
    co.info.insert(co.info.end(), info.begin(), info.end());
    co.ns.insert(co.ns.end(), nsv.begin(), nsv.end());
    co.escapes += esc;
    co.n_singles += td.n16;
    co.n_wide += td.nwide;
    co.n_intervals += td.nint;
    for (int64_t k = 0; k < nr; ++k) {
      const RowPlan& rp = plans[size_t(k)];
      co.units += int64_t(rp.ent.size()) + (rp.g ? 1 : 0);
      if (rp.g) ++co.diff_rows; else ++co.direct_rows;
      if (is_long_row(rp)) ++co.long_rows;
      co.max_level = std::max<int>(co.max_level, level[i0 + k]);
    }
    return kEmitted;
  }

 private:
  const DecodedGraph& g_;
  const LayoutParams& p_;
};

}  // namespace

int build_layout(const DecodedGraph& g, const LayoutParams& prm, int nthreads, HostLayout& out, std::string& err) {
  if (prm.tile_rows < 1 || prm.tile_rows > kTileRowsMax || prm.window_cap < 1 || 2 * prm.window_cap + 1 > int(kS16Off) ||
      prm.stage_bytes < 256 || prm.stage_bytes > 65536 || prm.long_row_bytes < 16 ||
      prm.long_row_bytes > prm.stage_bytes || prm.min_interval < 2) {
    err = "layout parameter out of range";
    return -1;
  }
  if (g.n >= int64_t(kLongBias)) {
    err = "graph too large for 31-bit relative entries";
    return -1;
  }
  const int64_t n = g.n;
  const int64_t chunk_rows = std::max<int64_t>(prm.tile_rows, 1 << 16);
  const int64_t nchunks = (n + chunk_rows - 1) / chunk_rows;
  std::vector<ChunkOut> outs(static_cast<size_t>(nchunks), ChunkOut());
  Builder b(g, prm);
  const int nt = std::max(1, std::min<int>(nthreads, 64));
  std::atomic<int64_t> next{0};
  auto worker = [&] {
    for (int64_t c = next.fetch_add(1); c < nchunks; c = next.fetch_add(1))
      b.run_chunk(c * chunk_rows, std::min(n, (c + 1) * chunk_rows), outs[size_t(c)]);
  };
  if (nt == 1 || nchunks == 1) {
    worker();
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
  }
  out = HostLayout();
  out.prm = prm;
  out.n = n;
  out.info.reserve(size_t(n));
  out.ns.reserve(size_t(n));
  for (auto& co : outs) {
    if (!co.err.empty()) { err = co.err; return -1; }
    const uint64_t db = out.data.size(), lb = out.longs.size();
    if ((db + co.data.size()) / 16 >= (uint64_t(1) << 32) || lb + co.longs.size() >= (uint64_t(1) << 32)) {
      err = "layout exceeds 32-bit offsets";
      return -1;
    }
    for (auto td : co.tiles) {
      td.data16 += uint32_t(db / 16);
      td.long0 += uint32_t(lb);
      out.tiles.push_back(td);
    }
    out.info.insert(out.info.end(), co.info.begin(), co.info.end());
    out.ns.insert(out.ns.end(), co.ns.begin(), co.ns.end());
    out.data.insert(out.data.end(), co.data.begin(), co.data.end());
    out.longs.insert(out.longs.end(), co.longs.begin(), co.longs.end());
    out.units += co.units;
    out.diff_rows += co.diff_rows;
    out.direct_rows += co.direct_rows;
    out.long_rows += co.long_rows;
    out.escapes += co.escapes;
    out.m_prime += co.m_prime;
    out.n_singles += co.n_singles;
    out.n_wide += co.n_wide;
    out.n_intervals += co.n_intervals;
    out.max_level = std::max(out.max_level, co.max_level);
  }
  out.data.resize(out.data.size() + 16, 0);  // one spare block for vector loads
  if (out.longs.empty()) out.longs.push_back(0);
  // empty tiles up to a whole block of tiles
  while (out.tiles.size() % kTilesPerBlock) {
    TileDesc td{};
    td.row0 = uint32_t(n);
    out.tiles.push_back(td);
  }
  return 0;
}

void build_csr_tiles(const uint64_t* rowptr, const uint32_t* col, int64_t n, int rows_cap, int col_cap,
                     int long_cols, int window_cap, std::vector<CsrTile>& tiles, uint64_t xlen) {
  tiles.clear();
  std::vector<uint32_t> pts;
  const uint32_t wmax = uint32_t(std::min<uint64_t>(xlen, 0xFFFFFFFFull));
  const uint32_t wpad = uint32_t(std::min<uint64_t>(uint64_t(n), wmax));  // window start of an empty tile
  int64_t i = 0;
  while (i < n) {
    const uint64_t d = rowptr[i + 1] - rowptr[i];
    if (d > uint64_t(long_cols)) {
      tiles.push_back({uint32_t(i), 1u | 0x80000000u, uint32_t(rowptr[i]), uint32_t(d), 0, 0, 0, 0});
      ++i;
      continue;
    }
    const int64_t i0 = i;
    while (i < n && i - i0 < rows_cap && rowptr[i + 1] - rowptr[i] <= uint64_t(long_cols) &&
           rowptr[i + 1] - rowptr[i0] <= uint64_t(col_cap))
      ++i;
    CsrTile t{uint32_t(i0), uint32_t(i - i0), uint32_t(rowptr[i0]), uint32_t(rowptr[i] - rowptr[i0]), 0, 0, 0, 0};
    pts.clear();
    for (uint64_t k = rowptr[i0]; k < rowptr[i]; ++k)
      if (col[k] < wmax) pts.push_back(col[k]);
    best_window(pts, window_cap, std::min(uint32_t(i0), wmax), t.win0, t.winlen);
    tiles.push_back(t);
  }
  while (tiles.size() % kTilesPerBlock) tiles.push_back({uint32_t(n), 0, 0, 0, wpad, 0, 0, 0});
}

int build_left_layout(const HostLayout& hl, LeftLayout& out, std::string& err) {
  out = LeftLayout();
  const int64_t n = hl.n;
  const size_t ng = size_t((n + 63) / 64);
  struct Ent {
    uint16_t f, row;
    uint16_t neg;
  };
  std::vector<Ent> ents;
  std::vector<std::vector<uint32_t>> cover(ng);
  uint64_t part = 0;
  for (size_t t = 0; t < hl.tiles.size(); ++t) {
    const TileDesc& td = hl.tiles[t];
    LeftTile lt{};
    lt.e0 = uint32_t(out.entries.size());
    lt.g0 = uint32_t(out.groups.size());
    lt.lane0 = uint32_t(out.lanes.size());
    lt.part0 = uint32_t(part);
    if (td.nrows > 128) {
      err = "left product: tile of more than 128 rows";
      return -1;
    }
    const uint8_t* base = hl.data.data() + size_t(td.data16) * 16;
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(base);
    const uint32_t* w32 = reinterpret_cast<const uint32_t*>(base + align16u(td.n16 * 2u));
    ents.clear();
    uint64_t o16 = 0, ow = 0, ol = 0;
    for (uint32_t r = 0; r < td.nrows; ++r) {
      const uint32_t inf = hl.info[td.row0 + r];
      const uint32_t ns = hl.ns[td.row0 + r];
      const uint32_t grow = td.row0 + r;
      if (inf & kInfoLong) {
        const uint64_t len = uint64_t(info_nwide(inf)) | (uint64_t(ns) << 19);
        for (uint64_t k = 0; k < len; ++k) {
          const uint32_t w = hl.longs[td.long0 + ol + k];
          const int64_t c = int64_t(td.win0) + int64_t(w & 0x7FFFFFFFu) - int64_t(kLongBias);
          out.esc.push_back({uint32_t(c), grow | (w & 0x80000000u)});
        }
        ol += len;
        lt.esc = 1;
        continue;
      }
      for (uint32_t k = 0; k < ns; ++k) {
        const uint32_t w = s16[o16 + k];
        const uint16_t f = uint16_t(w & kS16Off);
        // a column adds with its sign; a prefix entry with the opposite one
        const bool neg = (f & 1) ? !(w & kS16Neg) : (w & kS16Neg) != 0;
        ents.push_back({f, uint16_t(r), uint16_t(neg)});
      }
      o16 += ns;
      for (uint32_t k = 0; k < info_nwide(inf); ++k) {
        const uint32_t w = w32[ow + k];
        const int64_t c = int64_t(td.win0) + int64_t(w & kWideOff) - int64_t(kWideBias);
        out.esc.push_back({uint32_t(c), grow | ((w & kWideNeg) ? 0x80000000u : 0u)});
        lt.esc = 1;
      }
      ow += info_nwide(inf);
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
      return a.f != b.f ? a.f < b.f : a.row < b.row;
    });
    // groups, and the lanes' runs of whole groups balanced on entries
    const uint32_t E = uint32_t(ents.size());
    std::vector<uint32_t> gstart;  // entry index of each group's first entry
    for (uint32_t k = 0; k < E; ++k) {
      const bool last = k + 1 == E || ents[k + 1].f != ents[k].f;
      if (k == 0 || ents[k - 1].f != ents[k].f) {
        gstart.push_back(k);
        out.groups.push_back(ents[k].f);
      }
      out.entries.push_back(uint16_t(ents[k].row | (last ? 0x4000u : 0u) | (ents[k].neg ? 0x8000u : 0u)));
    }
    const uint32_t G = uint32_t(gstart.size());
    if (G > 0xFFFF || E > 0xFFFF) {
      err = "left product: tile stream too long";
      return -1;
    }
    uint32_t gi = 0;
    for (uint32_t l = 0; l <= 64; ++l) {
      const uint64_t target = (uint64_t(E) * l + 63) / 64;
      while (gi < G && gstart[gi] < target) ++gi;
      const uint32_t es = gi < G ? gstart[gi] : E;
      out.lanes.push_back((gi << 16) | es);
    }
    while (out.entries.size() % 8) out.entries.push_back(0);
    while (out.groups.size() % 8) out.groups.push_back(0);
    if (td.winlen) {
      for (uint64_t g = td.win0 / 64; g <= (uint64_t(td.win0) + td.winlen - 1) / 64 && g < ng; ++g)
        cover[g].push_back(uint32_t(t));
      part += (td.winlen + 3u) & ~3u;
    }
    out.tiles.push_back(lt);
  }
  if (part >= (uint64_t(1) << 32) || out.entries.size() >= (uint64_t(1) << 32)) {
    err = "left product layout exceeds 32-bit offsets";
    return -1;
  }
  out.part_len = part;
  std::sort(out.esc.begin(), out.esc.end(), [](const LeftEscape& a, const LeftEscape& b) {
    return a.col != b.col ? a.col < b.col : (a.row & 0x7FFFFFFFu) < (b.row & 0x7FFFFFFFu);
  });
  out.esc_off.assign(ng + 1, 0);
  for (const auto& e : out.esc) {
    if (int64_t(e.col) >= n) {
      err = "left product: escape column out of range";
      return -1;
    }
    ++out.esc_off[e.col / 64 + 1];
  }
  for (size_t g = 0; g < ng; ++g) out.esc_off[g + 1] += out.esc_off[g];
  out.cov_off.assign(ng + 1, 0);
  for (size_t g = 0; g < ng; ++g) {
    out.cov_off[g + 1] = out.cov_off[g] + uint32_t(cover[g].size());
    out.cov.insert(out.cov.end(), cover[g].begin(), cover[g].end());
  }
  if (out.esc.empty()) out.esc.push_back({0, 0});
  if (out.cov.empty()) out.cov.push_back(0);
  if (out.groups.empty()) out.groups.push_back(0);
  if (out.entries.empty()) out.entries.push_back(0);
  return 0;
}

}  // namespace bvmv
