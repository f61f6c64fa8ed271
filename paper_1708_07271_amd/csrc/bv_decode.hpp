// Host decoder of the BV-style bitstream into adjacency lists (CSR) and the
// reference gaps g_i = i - r_i.  Row i is coded against a reference row
// r_i within a window W, by copy/skip blocks over the reference's list, then
// intervals and gap-coded residuals for the entries it adds (list
// referencing, Section "Our Approach" of the paper).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace bvmv {

struct StreamHeader {
  uint64_t n = 0, m = 0;
  uint32_t W = 0, R = 0, Lmin = 0, zeta_k = 0, stride = 0;
  uint64_t body_bits = 0, nseg = 0;
  std::vector<uint64_t> seg_offsets;
  const uint8_t* body = nullptr;
  size_t body_bytes = 0;
};

// How a row is coded in the stream (counts read while decoding it): the depth
// of its reference chain, the reference entries it skips, its intervals and
// their total length, and its residuals.
struct RowStats {
  uint32_t depth, skipped, nint, intlen, nres;
};

struct DecodedGraph {
  int64_t n = 0, m = 0;
  std::vector<uint64_t> rowptr;  // n+1
  std::vector<uint32_t> col;     // m
  std::vector<uint8_t> refs;     // n, g_i (0 = none)
  std::vector<RowStats> stats;   // n
  StreamHeader hdr;
};

// Returns 0 on success; -2 (format) with a message in err otherwise.
int parse_header(const uint8_t* data, size_t nbytes, StreamHeader& h, std::string& err);
int decode_stream(const uint8_t* data, size_t nbytes, int nthreads, DecodedGraph& out, std::string& err);

}  // namespace bvmv
