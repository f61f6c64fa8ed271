// Host construction of the tiled device layout (see bv_layout.hpp).
#include "bv_layout.hpp"

#include <algorithm>
#include <atomic>
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
      while (s < e) {  // lengths fit the 16-bit length word
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

int64_t entry_words(const std::vector<Entry>& es) {
  int64_t w = 0;
  for (auto& e : es) w += e.len ? 2 : 1;
  return w;
}

struct RowPlan {
  std::vector<Entry> ent;
  int g = 0;        // 0 = direct
  int64_t est = 0;  // words if every entry falls in the window
  bool force_long = false;  // its coded words alone overflow a tile
};

struct ChunkOut {
  std::vector<TileDesc> tiles;
  std::vector<uint32_t> info;
  std::vector<uint16_t> words;
  std::vector<uint32_t> longs;
  int64_t units = 0, diff_rows = 0, direct_rows = 0, long_rows = 0, escapes = 0, m_prime = 0;
  int max_level = 0;
  std::string err;
};

class Builder {
 public:
  Builder(const DecodedGraph& g, const LayoutParams& p) : g_(g), p_(p) {}

  void plan_row(int64_t i, int64_t i0, RowPlan& rp, std::vector<uint32_t>& K, std::vector<uint32_t>& E,
                std::vector<Entry>& tmp) {
    const uint32_t* Li = g_.col.data() + g_.rowptr[i];
    const size_t di = size_t(g_.rowptr[i + 1] - g_.rowptr[i]);
    rp.ent.clear();
    to_entries(Li, di, false, p_.min_interval, rp.ent);
    rp.g = 0;
    rp.est = entry_words(rp.ent);
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
    const int64_t w = entry_words(tmp);
    if (w < rp.est) {
      rp.ent.swap(tmp);
      rp.g = gi;
      rp.est = w;
    }
  }

  // paper's nonzeros of A' for row i: |v_i - v_r| if smaller than |v_i|, else |v_i|
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
      int64_t words = 0;
      while (i < hi && i - i0 < p_.tile_rows) {
        plans.emplace_back();
        RowPlan& rp = plans.back();
        plan_row(i, i0, rp, K, E, tmp);
        const bool is_long = rp.est > p_.long_row_words;
        if (!is_long && words + rp.est > p_.word_cap && i > i0) {
          plans.pop_back();
          break;
        }
        if (!is_long) words += rp.est;
        ++i;
      }
      // emit; shrink the tile while escapes push it past the word cap
      for (;;) {
        if (emit_tile(i0, plans, level.data() - lo, co)) break;
        if (plans.size() == 1) {
          if (plans[0].force_long) { co.err = "row does not fit a tile"; return; }
          plans[0].force_long = true;  // escapes overflow the staging: sum it block-wide
          continue;
        }
        plans.pop_back();
        --i;
      }
      if (!co.err.empty()) return;
    }
  }

  bool is_long_row(const RowPlan& rp) const { return rp.force_long || rp.est > p_.long_row_words; }

  // Returns false (and emits nothing) if the coded short rows exceed word_cap.
  bool emit_tile(int64_t i0, const std::vector<RowPlan>& plans, uint8_t* level, ChunkOut& co) {
    const int64_t nr = int64_t(plans.size());
    // window: the span of at most window_cap columns covering most points
    std::vector<uint32_t> pts;
    for (auto& rp : plans) {
      if (is_long_row(rp)) continue;
      for (auto& e : rp.ent) {
        pts.push_back(e.col);
        if (e.len) pts.push_back(e.col + e.len - 1);
      }
    }
    std::sort(pts.begin(), pts.end());
    uint32_t win0 = uint32_t(i0), winlen = 0;
    if (!pts.empty()) {
      size_t best_a = 0, best_b = 0, b = 0;
      for (size_t a = 0; a < pts.size(); ++a) {
        if (b < a) b = a;
        while (b + 1 < pts.size() && int64_t(pts[b + 1]) - int64_t(pts[a]) < p_.window_cap) ++b;
        if (b - a > best_b - best_a) { best_a = a; best_b = b; }
      }
      win0 = pts[best_a];
      winlen = pts[best_b] - pts[best_a] + 1;
    }
    auto in_win = [&](int64_t c) { return c >= int64_t(win0) && c < int64_t(win0) + int64_t(winlen); };
    // code short rows
    const size_t wbase = co.words.size();
    std::vector<uint16_t>& W = co.words;
    std::vector<uint32_t> info(static_cast<size_t>(nr), 0u);
    int64_t esc = 0;
    const size_t lbase = co.longs.size();
    for (int64_t k = 0; k < nr; ++k) {
      const RowPlan& rp = plans[size_t(k)];
      const int64_t i = i0 + k;
      const bool is_long = is_long_row(rp);
      const int lvl = rp.g ? level[i - rp.g] + 1 : 0;
      level[i] = uint8_t(lvl);
      uint64_t len = 0;
      if (!is_long) {
        const size_t before = W.size();
        auto single = [&](uint32_t c, bool neg) {
          const uint16_t sg = neg ? 0x8000 : 0;
          if (in_win(c)) {
            W.push_back(uint16_t(sg | (c - win0)));
          } else {
            const uint32_t rel = uint32_t(int64_t(c) - int64_t(win0));
            W.push_back(uint16_t(sg | kEscape));
            W.push_back(uint16_t(rel >> 16));
            W.push_back(uint16_t(rel & 0xFFFF));
            ++esc;
          }
        };
        for (auto& e : rp.ent) {
          if (e.len == 0) {
            single(e.col, e.neg);
          } else if (in_win(e.col) && in_win(int64_t(e.col) + e.len - 1)) {
            W.push_back(uint16_t((e.neg ? 0x8000 : 0) | 0x4000 | (e.col - win0)));
            W.push_back(uint16_t(e.len));
          } else {
            for (uint32_t t = 0; t < e.len; ++t) single(e.col + t, e.neg);
          }
        }
        len = W.size() - before;
      } else {
        for (auto& e : rp.ent) {
          const uint32_t cnt = e.len ? e.len : 1;
          for (uint32_t t = 0; t < cnt; ++t) {
            const int64_t rel = int64_t(e.col + t) - int64_t(win0) + int64_t(kLongBias);
            co.longs.push_back((e.neg ? 0x80000000u : 0u) | uint32_t(rel));
          }
          len += cnt;
        }
      }
      if (len >= (1u << 23)) {
        co.err = "row too long for the layout";
        return true;
      }
      info[size_t(k)] = uint32_t(rp.g) | (uint32_t(lvl) << 4) | (is_long ? kInfoLong : 0u) | (uint32_t(len) << 9);
    }
    const int64_t nwords = int64_t(W.size() - wbase);
    if (nwords > p_.word_cap) {
      W.resize(wbase);
      co.longs.resize(lbase);
      return false;
    }
    // pad to a multiple of 8 words so the next tile starts 16-byte aligned
    while (W.size() % 8) W.push_back(0);
    TileDesc td;
    td.row0 = uint32_t(i0);
    td.nrows = uint32_t(nr);
    td.word0 = uint32_t(wbase);
    td.nwords = uint32_t(nwords);
    td.win0 = win0;
    td.winlen = winlen;
    td.long0 = uint32_t(lbase);
    td.graph = 0;
    co.tiles.push_back(td);
    co.info.insert(co.info.end(), info.begin(), info.end());
    co.escapes += esc;
    for (int64_t k = 0; k < nr; ++k) {
      const RowPlan& rp = plans[size_t(k)];
      co.units += int64_t(rp.ent.size()) + (rp.g ? 1 : 0);
      if (rp.g) ++co.diff_rows; else ++co.direct_rows;
      if (is_long_row(rp)) ++co.long_rows;
      co.max_level = std::max<int>(co.max_level, level[i0 + k]);
    }
    return true;
  }

 private:
  const DecodedGraph& g_;
  const LayoutParams& p_;
};

}  // namespace

int build_layout(const DecodedGraph& g, const LayoutParams& prm, int nthreads, HostLayout& out, std::string& err) {
  if (prm.tile_rows < 1 || prm.tile_rows > 1024 || prm.window_cap < 1 || prm.window_cap > 16383 ||
      prm.word_cap < 64 || prm.word_cap > 65536 || prm.long_row_words < 1 || prm.min_interval < 2) {
    err = "layout parameter out of range";
    return -1;
  }
  if (g.n >= int64_t(kLongBias)) {
    err = "graph too large for 32-bit relative long entries";
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
  for (auto& co : outs) {
    if (!co.err.empty()) { err = co.err; return -1; }
    const uint64_t wb = out.words.size(), lb = out.longs.size();
    if (wb + co.words.size() >= (uint64_t(1) << 32) || lb + co.longs.size() >= (uint64_t(1) << 32)) {
      err = "layout exceeds 32-bit offsets";
      return -1;
    }
    for (auto td : co.tiles) {
      td.word0 += uint32_t(wb);
      td.long0 += uint32_t(lb);
      out.tiles.push_back(td);
    }
    out.info.insert(out.info.end(), co.info.begin(), co.info.end());
    out.words.insert(out.words.end(), co.words.begin(), co.words.end());
    out.longs.insert(out.longs.end(), co.longs.begin(), co.longs.end());
    out.units += co.units;
    out.diff_rows += co.diff_rows;
    out.direct_rows += co.direct_rows;
    out.long_rows += co.long_rows;
    out.escapes += co.escapes;
    out.m_prime += co.m_prime;
    out.max_level = std::max(out.max_level, co.max_level);
  }
  // slack so 16-byte vector loads of the last tile stay in bounds
  out.words.resize(out.words.size() + 16, 0);
  if (out.longs.empty()) out.longs.push_back(0);
  return 0;
}

void build_csr_tiles(const uint64_t* rowptr, int64_t n, int rows_cap, int col_cap, std::vector<CsrTile>& tiles) {
  tiles.clear();
  int64_t i = 0;
  while (i < n) {
    const int64_t d = int64_t(rowptr[i + 1] - rowptr[i]);
    if (d > col_cap) {
      tiles.push_back({uint32_t(i), 1, uint32_t(rowptr[i]), uint32_t(d)});
      ++i;
      continue;
    }
    const int64_t i0 = i;
    while (i < n && i - i0 < rows_cap && int64_t(rowptr[i + 1] - rowptr[i0]) <= col_cap) ++i;
    tiles.push_back({uint32_t(i0), uint32_t(i - i0), uint32_t(rowptr[i0]), uint32_t(rowptr[i] - rowptr[i0])});
  }
}

}  // namespace bvmv
