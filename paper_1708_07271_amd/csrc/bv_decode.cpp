// Host decoder of the BV-style bitstream (see bv_decode.hpp).
//
// Codes: unary (x zeros then a one), Elias gamma on x+1, Boldi-Vigna zeta_k
// on x+1 (minimal binary code inside each bucket [2^(hk), 2^((h+1)k))), and
// the signed map nu(z) = 2z / 2|z|-1.  The body is MSB-first.
//
// Parallel decode: the stream carries the bit offset of every node k*S,
// and no reference crosses a multiple of S, so each segment of S nodes
// decodes independently; consecutive segments are handed to threads.
#include "bv_decode.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>

namespace bvmv {
namespace {

inline uint64_t be64(const uint8_t* q) {
  uint64_t v;
  std::memcpy(&v, q, 8);
  return __builtin_bswap64(v);
}

class BitIn {
 public:
  BitIn(const uint8_t* padded, uint64_t nbits, uint64_t pos) : p_(padded), nbits_(nbits), pos_(pos) {}
  bool ok() const { return !bad_; }
  uint64_t pos() const { return pos_; }

  // 64 bits starting at pos_, MSB-aligned (the buffer is zero padded by 16 bytes)
  uint64_t window() const {
    const uint64_t byte = pos_ >> 3;
    const unsigned sh = unsigned(pos_ & 7);
    uint64_t w = be64(p_ + byte);
    if (sh) w = (w << sh) | (uint64_t(p_[byte + 8]) >> (8 - sh));
    return w;
  }
  uint64_t bits(unsigned k) {  // k <= 64
    if (k == 0) return 0;
    if (pos_ + k > nbits_) { bad_ = true; return 0; }
    uint64_t v = window() >> (64 - k);
    pos_ += k;
    return v;
  }
  uint64_t unary() {
    uint64_t z = 0;
    for (;;) {
      if (pos_ >= nbits_) { bad_ = true; return 0; }
      const uint64_t w = window();
      if (w) {
        const unsigned lz = unsigned(__builtin_clzll(w));
        if (pos_ + lz + 1 > nbits_) { bad_ = true; return 0; }
        pos_ += lz + 1;
        return z + lz;
      }
      z += 64;
      pos_ += 64;
    }
  }
  uint64_t gamma() {
    const uint64_t b = unary();
    if (b > 63) { bad_ = true; return 0; }
    return ((uint64_t(1) << b) | bits(unsigned(b))) - 1;
  }
  uint64_t zeta(unsigned k) {
    const uint64_t h = unary();
    if ((h + 1) * k > 63) { bad_ = true; return 0; }
    const uint64_t left = uint64_t(1) << (h * k);
    const uint64_t zmax = (uint64_t(1) << ((h + 1) * k)) - left;
    const unsigned s = zmax <= 1 ? 0 : unsigned(64 - __builtin_clzll(zmax - 1));
    if (s == 0) return left - 1;
    const uint64_t thr = (uint64_t(1) << s) - zmax;
    uint64_t z = bits(s - 1);
    if (z >= thr) z = ((z << 1) | bits(1)) - thr;
    return left + z - 1;
  }

 private:
  const uint8_t* p_;
  uint64_t nbits_, pos_;
  bool bad_ = false;
};

inline int64_t nu_inv(uint64_t u) { return (u & 1) ? -int64_t((u + 1) >> 1) : int64_t(u >> 1); }

struct SegOut {
  std::vector<uint32_t> col;      // lists of rows [lo, hi)
  std::vector<uint64_t> len;      // per row
  std::vector<uint8_t> refs;
  std::vector<RowStats> stats;
  uint64_t end_pos = 0;
  std::string err;
};

// Decode rows [lo, hi) starting at bit offset `pos`.  References must stay
// inside [seg_lo(i), i) where seg_lo is the start of row i's segment.
void decode_range(const StreamHeader& h, const uint8_t* padded, uint64_t lo, uint64_t hi, uint64_t pos,
                  uint64_t stride, SegOut& out) {
  BitIn in(padded, h.body_bits, pos);
  const uint64_t nrow = hi - lo;
  std::vector<uint64_t> start(nrow), len(nrow, 0);
  std::vector<uint8_t> depth(nrow, 0), refs(nrow, 0);
  std::vector<RowStats> stats(nrow, RowStats{0, 0, 0, 0, 0});
  std::vector<uint32_t> col;
  col.reserve(size_t(nrow * 24));
  std::vector<uint32_t> copied, extras;
  auto fail = [&](const char* what, uint64_t i) {
    out.err = std::string(what) + " at node " + std::to_string(i);
  };
  for (uint64_t i = lo; i < hi; ++i) {
    if (h.nseg && i % stride == 0 && in.pos() != h.seg_offsets[i / stride]) {
      fail("segment offset mismatch", i);
      return;
    }
    const uint64_t li = i - lo;
    start[li] = col.size();
    const uint64_t d = in.gamma();
    if (!in.ok()) { fail("truncated stream", i); return; }
    if (d == 0) continue;
    if (d > h.n) { fail("degree larger than n", i); return; }
    uint64_t g = h.W ? in.unary() : 0;
    if (!in.ok() || g > h.W || g > i) { fail("reference outside the window", i); return; }
    copied.clear();
    if (g) {
      const uint64_t r = i - g;
      if (r < lo || (h.nseg && r / stride != i / stride)) { fail("reference crosses a segment boundary", i); return; }
      if (depth[r - lo] + 1u > h.R) { fail("reference chain deeper than R", i); return; }
      depth[li] = uint8_t(depth[r - lo] + 1);
      const uint64_t rlen = len[r - lo];
      const uint32_t* rl = col.data() + start[r - lo];
      const uint64_t nb = in.gamma();
      uint64_t p = 0;
      bool keep = true;
      for (uint64_t b = 0; b < nb; ++b) {
        // a block's length is gamma (first block) or gamma + 1: bounded by
        // what is left of the reference list before any arithmetic on it
        const uint64_t code = in.gamma();
        if (!in.ok() || code > rlen - p || (b > 0 && code == rlen - p)) {
          fail("copy blocks exceed the reference list", i);
          return;
        }
        const uint64_t ln = b == 0 ? code : code + 1;
        if (keep) copied.insert(copied.end(), rl + p, rl + p + ln);
        p += ln;
        keep = !keep;
      }
      if (!in.ok()) { fail("truncated stream", i); return; }
      if (keep) copied.insert(copied.end(), rl + p, rl + rlen);
      refs[li] = uint8_t(g);
      stats[li].depth = depth[li];
      stats[li].skipped = uint32_t(rlen - copied.size());
    }
    if (copied.size() > d) { fail("more copied entries than the degree", i); return; }
    const uint64_t ne = d - copied.size();
    extras.clear();
    if (ne) {
      const uint64_t nint = ne >= h.Lmin ? in.gamma() : 0;
      int64_t prev_last = 0;
      for (uint64_t k = 0; k < nint; ++k) {
        // every decoded value is checked against n (or the entries left)
        // before it enters any sum, so no arithmetic below can wrap
        const uint64_t cs = in.gamma();
        const uint64_t cl = in.gamma();
        const uint64_t left = ne - extras.size();
        if (!in.ok() || cs >= 2 * h.n || left < h.Lmin || cl > left - h.Lmin) {
          fail("bad interval", i);
          return;
        }
        const int64_t s = k == 0 ? int64_t(i) + nu_inv(cs) : prev_last + 2 + int64_t(cs);
        const uint64_t ln = cl + h.Lmin;
        if (s < 0 || uint64_t(s) + ln > h.n) {
          fail("bad interval", i);
          return;
        }
        for (uint64_t t = 0; t < ln; ++t) extras.push_back(uint32_t(uint64_t(s) + t));
        prev_last = s + int64_t(ln) - 1;
      }
      const uint64_t nres = ne - extras.size();
      const size_t int_end = extras.size();
      stats[li].nint = uint32_t(nint);
      stats[li].intlen = uint32_t(int_end);
      stats[li].nres = uint32_t(nres);
      int64_t prev = 0;
      for (uint64_t k = 0; k < nres; ++k) {
        const uint64_t cz = in.zeta(h.zeta_k);
        if (!in.ok() || cz >= 2 * h.n) { fail("bad residual", i); return; }
        const int64_t j = k == 0 ? int64_t(i) + nu_inv(cz) : prev + 1 + int64_t(cz);
        if (j < 0 || uint64_t(j) >= h.n) { fail("bad residual", i); return; }
        extras.push_back(uint32_t(j));
        prev = j;
      }
      std::inplace_merge(extras.begin(), extras.begin() + int64_t(int_end), extras.end());
    }
    // merge copied (sorted) and extras (sorted) into the row; reject duplicates
    const size_t base = col.size();
    col.resize(base + d);
    std::merge(copied.begin(), copied.end(), extras.begin(), extras.end(), col.begin() + int64_t(base));
    for (size_t t = base + 1; t < base + d; ++t)
      if (col[t] <= col[t - 1]) { fail("duplicate or unsorted id", i); return; }
    len[li] = d;
  }
  out.end_pos = in.pos();
  out.col.swap(col);
  out.len.swap(len);
  out.refs.swap(refs);
  out.stats.swap(stats);
}

}  // namespace

int parse_header(const uint8_t* data, size_t nbytes, StreamHeader& h, std::string& err) {
  if (!data || nbytes < 64 || std::memcmp(data, "BVMV", 4) != 0) { err = "bad magic"; return -2; }
  uint32_t version;
  std::memcpy(&version, data + 4, 4);
  if (version != 1) { err = "unsupported version"; return -2; }
  std::memcpy(&h.n, data + 8, 8);
  std::memcpy(&h.m, data + 16, 8);
  std::memcpy(&h.W, data + 24, 4);
  std::memcpy(&h.R, data + 28, 4);
  std::memcpy(&h.Lmin, data + 32, 4);
  std::memcpy(&h.zeta_k, data + 36, 4);
  std::memcpy(&h.stride, data + 40, 4);
  std::memcpy(&h.body_bits, data + 48, 8);
  std::memcpy(&h.nseg, data + 56, 8);
  if (h.n == 0 || h.n >= 0xFFFFFFFFull || h.W > 15 || h.R > 15 || h.Lmin < 1 || h.zeta_k < 1 || h.zeta_k > 8) {
    err = "header field out of range";
    return -2;
  }
  if (h.nseg > (nbytes - 64) / 8) { err = "truncated stream"; return -2; }
  const size_t off = 64 + size_t(h.nseg) * 8;
  if (h.body_bits / 8 + off > nbytes || off + (h.body_bits + 7) / 8 > nbytes) { err = "truncated stream"; return -2; }
  h.seg_offsets.resize(h.nseg);
  if (h.nseg) std::memcpy(h.seg_offsets.data(), data + 64, h.nseg * 8);
  if (h.nseg) {
    if (h.stride == 0 || (h.n + h.stride - 1) / h.stride != h.nseg) {
      err = "bad segment table";
      return -2;
    }
    for (uint64_t k = 0; k < h.nseg; ++k)
      if (h.seg_offsets[k] > h.body_bits || (k && h.seg_offsets[k] < h.seg_offsets[k - 1])) {
        err = "bad segment table";
        return -2;
      }
    if (h.seg_offsets[0] != 0) { err = "bad segment table"; return -2; }
  }
  h.body = data + off;
  h.body_bytes = size_t((h.body_bits + 7) / 8);
  return 0;
}

int decode_stream(const uint8_t* data, size_t nbytes, int nthreads, DecodedGraph& out, std::string& err) {
  StreamHeader h;
  if (int rc = parse_header(data, nbytes, h, err)) return rc;
  std::vector<uint8_t> padded(h.body_bytes + 16, 0);
  std::memcpy(padded.data(), h.body, h.body_bytes);
  const uint64_t n = h.n;
  // work items: contiguous runs of segments
  uint64_t nseg = h.nseg ? h.nseg : 1;
  const uint64_t stride = h.nseg ? h.stride : n;
  int nt = std::max(1, std::min<int>(nthreads, 64));
  if (!h.nseg) nt = 1;
  uint64_t nchunks = std::min<uint64_t>(nseg, uint64_t(nt) * 4);
  std::vector<SegOut> outs(nchunks);
  auto work = [&](uint64_t c) {
    const uint64_t s0 = nseg * c / nchunks, s1 = nseg * (c + 1) / nchunks;
    const uint64_t lo = s0 * stride, hi = std::min<uint64_t>(n, s1 * stride);
    const uint64_t pos = h.nseg ? h.seg_offsets[s0] : 0;
    decode_range(h, padded.data(), lo, hi, pos, stride, outs[c]);
    // the chunk must end where the next one starts
    if (outs[c].err.empty() && h.nseg && s1 < nseg && outs[c].end_pos != h.seg_offsets[s1])
      outs[c].err = "segment offset mismatch at node " + std::to_string(hi);
  };
  if (nt == 1 || nchunks == 1) {
    for (uint64_t c = 0; c < nchunks; ++c) work(c);
  } else {
    std::vector<std::thread> th;
    std::atomic<uint64_t> next{0};
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&] {
        for (uint64_t c = next.fetch_add(1); c < nchunks; c = next.fetch_add(1)) work(c);
      });
    for (auto& t : th) t.join();
  }
  for (auto& o : outs)
    if (!o.err.empty()) { err = o.err; return -2; }
  if (outs.back().end_pos != h.body_bits) { err = "trailing bits after the last node"; return -2; }
  out.n = int64_t(n);
  out.rowptr.assign(n + 1, 0);
  out.refs.resize(n);
  out.stats.resize(n);
  uint64_t m = 0, row = 0;
  for (auto& o : outs) m += o.col.size();
  if (m != h.m) { err = "edge count differs from the header"; return -2; }
  out.col.resize(m);
  uint64_t pos = 0;
  for (auto& o : outs) {
    if (!o.col.empty()) std::memcpy(out.col.data() + pos, o.col.data(), o.col.size() * 4);
    for (size_t k = 0; k < o.len.size(); ++k) {
      out.refs[row] = o.refs[k];
      out.stats[row] = o.stats[k];
      out.rowptr[row + 1] = out.rowptr[row] + o.len[k];
      ++row;
    }
    pos += o.col.size();
  }
  if (row != n) { err = "row count mismatch"; return -2; }
  out.m = int64_t(m);
  out.hdr = h;
  out.hdr.body = nullptr;
  return 0;
}

}  // namespace bvmv
