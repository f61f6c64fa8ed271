// Test driver for the host decoder and layout builder under AddressSanitizer
// and UndefinedBehaviorSanitizer (built with g++ by tests/test_host.py; no
// device code).  For each bitstream file given:
//   - decode it (1 and 4 threads) and check the two decodes agree;
//   - build the device layout under several tile / window / stage shapes and
//     run the host layout interpreter on x = 1, 2, 3, ... (exact in double),
//     comparing with the plain row sums of the decoded lists;
//   - decode truncated copies and copies with one flipped bit: each must
//     either decode or fail with a message, never touch memory out of bounds.
// A path given as reject:<file> is a hand-built hostile stream (decoded
// values near 2^64): its decode must fail with a message.
// Exit status 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "../../include/bvmv.h"
#include "bv_decode.hpp"
#include "bv_layout.hpp"

namespace bvmv {
int set_error(int code, const std::string& msg) {
  std::fprintf(stderr, "library error %d: %s\n", code, msg.c_str());
  return code;
}
}  // namespace bvmv

using namespace bvmv;

static int check_file(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  std::vector<uint8_t> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  DecodedGraph g1, g4;
  std::string err;
  if (decode_stream(bytes.data(), bytes.size(), 1, g1, err)) {
    std::fprintf(stderr, "%s: decode failed: %s\n", path.c_str(), err.c_str());
    return 1;
  }
  if (decode_stream(bytes.data(), bytes.size(), 4, g4, err) || g1.rowptr != g4.rowptr || g1.col != g4.col) {
    std::fprintf(stderr, "%s: 1- and 4-thread decodes differ\n", path.c_str());
    return 1;
  }
  const int64_t n = g1.n;
  std::vector<double> x(static_cast<size_t>(n)), want(static_cast<size_t>(n), 0.0), y(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) x[size_t(i)] = double(i % 97 + 1);
  for (int64_t i = 0; i < n; ++i)
    for (uint64_t k = g1.rowptr[size_t(i)]; k < g1.rowptr[size_t(i) + 1]; ++k) want[size_t(i)] += x[g1.col[k]];
  const int shapes[][4] = {{64, 256, 4096, 2048}, {16, 64, 512, 16}, {32, 256, 1024, 40}, {128, 768, 6144, 3072}};
  for (const auto& sh : shapes) {
    bvmv_load_opts o;
    std::memset(&o, 0, sizeof(o));
    o.tile_rows = sh[0];
    o.window_cap = sh[1];
    o.stage_bytes = sh[2];
    o.long_row_bytes = sh[3];
    int64_t stats[16] = {0};
    if (bvmv_layout_selfcheck(bytes.data(), bytes.size(), &o, x.data(), y.data(), stats)) {
      std::fprintf(stderr, "%s: layout %d/%d/%d failed\n", path.c_str(), sh[0], sh[1], sh[2]);
      return 1;
    }
    if (y != want) {
      std::fprintf(stderr, "%s: layout %d/%d/%d gives wrong sums\n", path.c_str(), sh[0], sh[1], sh[2]);
      return 1;
    }
  }
  // damaged copies: no crash, no out-of-bounds access
  const size_t step = bytes.size() / 61 + 1;
  for (size_t cut = 0; cut < bytes.size(); cut += step) {
    DecodedGraph d;
    (void)decode_stream(bytes.data(), cut, 2, d, err);
  }
  for (size_t pos = 64; pos < bytes.size(); pos += step) {
    std::vector<uint8_t> b = bytes;
    b[pos] ^= uint8_t(1u << (pos % 8));
    DecodedGraph d;
    if (decode_stream(b.data(), b.size(), 2, d, err) == 0) {
      LayoutParams prm;
      HostLayout hl;
      (void)build_layout(d, prm, 2, hl, err);
    }
  }
  return 0;
}

static int check_rejected(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  std::vector<uint8_t> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  for (int threads : {1, 2}) {
    DecodedGraph d;
    std::string err;
    if (decode_stream(bytes.data(), bytes.size(), threads, d, err) == 0 || err.empty()) {
      std::fprintf(stderr, "%s: hostile stream was not rejected\n", path.c_str());
      return 1;
    }
  }
  return 0;
}

int main(int argc, char** argv) {
  int bad = 0;
  for (int i = 1; i < argc; ++i) {
    const std::string a = argv[i];
    bad |= a.rfind("reject:", 0) == 0 ? check_rejected(a.substr(7)) : check_file(a);
  }
  if (!bad) std::printf("ok %d streams\n", argc - 1);
  return bad;
}
