// C ABI of the library (declared in include/bvmv.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bvmv.h"
#include "bv_decode.hpp"
#include "bv_layout.hpp"
#include "kernels.hpp"

using namespace bvmv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(BVMV_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int default_threads(int req) {
  if (req > 0) return std::min(req, 64);
  unsigned hc = std::thread::hardware_concurrency();
  return int(std::max(1u, std::min(hc ? hc : 4u, 16u)));
}

// Device copy of count elements, followed by `pad` zeroed elements (so that
// 16-byte vector loads may run past the last element).
template <class T>
int dev_upload(T** dst, const T* src, size_t count, size_t pad = 0) {
  *dst = nullptr;
  const size_t alloc = std::max<size_t>(count + pad, 1);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), alloc * sizeof(T));
  if (e != hipSuccess) { *dst = nullptr; return fail(BVMV_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); }
  if (src && count) {
    e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(BVMV_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  if (alloc > count) {
    e = hipMemset(*dst + count, 0, (alloc - count) * sizeof(T));
    if (e != hipSuccess) return fail(BVMV_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
  }
  return BVMV_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

size_t elem_size(int prec) { return prec == BVMV_F64 ? 8 : 4; }

// PageRank working set kept with a handle between calls.
struct PRWork {
  int prec = -1;
  int64_t n = 0;
  void* p[2] = {nullptr, nullptr};
  void* z[2] = {nullptr, nullptr};
  PRState* st = nullptr;     // 2 x members: the states of parity 0 (read back by the host) and 1
  double* slots = nullptr;   // 2 x nslots block slots of 2 doubles: parity 0, then 1
  double* pub = nullptr;     // 2 doubles per member: the fused iterations' published values
  PRState* h_st = nullptr;  // pinned
  int nst = 0;
  int64_t nslots = 0;
  // captured runs of iterations, by length: the chunk and its halvings down to 2
  static constexpr int kGraphs = 12;
  hipGraphExec_t exec[kGraphs] = {};
  hipGraph_t graph[kGraphs] = {};
  int glen[kGraphs] = {};
  // key of the captured graphs
  const void* key_tele = nullptr;
  double key_beta = -1, key_tol = -1;
  int key_max_iter = -1, key_chunk = -1, key_fused = -1, key_polls = -2;

  void drop_graph() {
    for (int i = 0; i < kGraphs; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
      exec[i] = nullptr;
      graph[i] = nullptr;
      glen[i] = 0;
    }
    key_chunk = -1;
  }
  void release() {
    drop_graph();
    for (int b = 0; b < 2; ++b) { dev_free(p[b]); dev_free(z[b]); p[b] = z[b] = nullptr; }
    dev_free(st);
    dev_free(slots);
    dev_free(pub);
    if (h_st) (void)hipHostFree(h_st);
    st = nullptr;
    slots = nullptr;
    pub = nullptr;
    h_st = nullptr;
    prec = -1;
  }
  int ensure(int pr, int64_t nn, int members, int64_t nsl) {
    nsl = std::max<int64_t>(nsl, 1);
    if (prec == pr && n == nn && nst == members && nslots == nsl && slots) return BVMV_OK;
    release();
    const size_t es = elem_size(pr);
    for (int b = 0; b < 2; ++b) {
      HIP_TRY(hipMalloc(&p[b], size_t(nn) * es));
      HIP_TRY(hipMalloc(&z[b], size_t(nn) * es));
    }
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&st), sizeof(PRState) * 2 * size_t(members)));
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&slots), sizeof(double) * 4 * size_t(nsl)));
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&pub), sizeof(double) * 2 * size_t(members)));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h_st), sizeof(PRState) * size_t(members), hipHostMallocDefault));
    prec = pr;
    n = nn;
    nst = members;
    nslots = nsl;
    return BVMV_OK;
  }
};

// Buffers of the learned warm restarts kept with a graph: the network inputs
// per node (the 8 structural ones, n x 8, filled once; the 4 of the current
// restart, n x 4), the network output, and two iterate snapshots of the
// iterate type.
struct LearnWork {
  int64_t n = 0;
  int prec = -1;
  float* Fs = nullptr;
  float* Ft = nullptr;
  float* s = nullptr;
  void* t[2] = {nullptr, nullptr};
  bool struct_ready = false;

  void release() {
    dev_free(Fs);
    dev_free(Ft);
    dev_free(s);
    dev_free(t[0]);
    dev_free(t[1]);
    Fs = Ft = s = nullptr;
    t[0] = t[1] = nullptr;
    n = 0;
    prec = -1;
    struct_ready = false;
  }
  int ensure(int pr, int64_t nn) {
    if (n != nn) {
      release();
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&Fs), size_t(std::max<int64_t>(nn, 1)) * 8 * sizeof(float)));
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&Ft), size_t(std::max<int64_t>(nn, 1)) * 4 * sizeof(float)));
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&s), size_t(std::max<int64_t>(nn, 1)) * sizeof(float)));
      n = nn;
    }
    if (prec != pr) {
      dev_free(t[0]);
      dev_free(t[1]);
      t[0] = t[1] = nullptr;
      prec = -1;
      for (int b = 0; b < 2; ++b)
        HIP_TRY(hipMalloc(&t[b], size_t(std::max<int64_t>(nn, 1)) * elem_size(pr)));
      prec = pr;
    }
    return BVMV_OK;
  }
};

struct PROptsResolved {
  double beta, tol;
  int max_iter, prec, chunk, fallback;
  const bvmv_mlp* mlp;
  int restart_every, max_restarts;
};

int resolve_pr_opts(const bvmv_pr_opts* o, PROptsResolved& r) {
  r.beta = 0.85;
  r.tol = 1e-6;
  r.max_iter = 1000;
  r.prec = BVMV_F32_COMP;
  r.chunk = 16;
  r.fallback = 0;
  r.mlp = nullptr;
  r.restart_every = 10;
  r.max_restarts = 2;
  if (o) {
    r.fallback = o->fallback_check;
    r.mlp = o->mlp;
    if (o->restart_every) r.restart_every = o->restart_every;
    if (o->max_restarts) r.max_restarts = o->max_restarts;
    if (o->damping != 0.0 || o->exact_zero_damping) r.beta = o->damping;
    if (o->tol != 0.0) r.tol = o->tol;
    if (o->max_iter) r.max_iter = o->max_iter;
    r.prec = o->prec;
    if (o->chunk) r.chunk = o->chunk;
  }
  if (!(r.beta >= 0.0 && r.beta < 1.0) || !(r.tol > 0.0) || r.max_iter < 1 || r.prec < 0 || r.prec > 2 ||
      r.chunk < 1 || r.chunk > 1024 || r.restart_every < 3 || r.restart_every > 100000 || r.max_restarts < 0 ||
      r.max_restarts > 100000)
    return fail(BVMV_EINVAL, "PageRank option out of range");
  if (r.chunk % 2) ++r.chunk;  // even, so every replay starts from buffer 0
  return BVMV_OK;
}

}  // namespace

namespace bvmv {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace bvmv

struct bvmv_graph {
  int device = 0;
  bvmv_load_opts opts{};
  int interval_mode = 0;
  DecodedGraph dec;          // lists kept only with keep_lists
  bool lists_kept = false;
  HostLayout hl;             // host copy (groups are built from it)
  std::vector<int32_t> h_outdeg;
  int64_t n = 0, m = 0, m_prime = 0, stream_bytes = 0;
  int W = 0, R = 0, Lmin = 0, zk = 0;
  // device
  TileDesc* d_tiles = nullptr;
  uint32_t* d_info = nullptr;
  uint16_t* d_ns = nullptr;
  uint8_t* d_data = nullptr;
  uint32_t* d_longs = nullptr;
  int32_t* d_outdeg = nullptr;
  uint32_t* d_stats = nullptr;  // per-row coding statistics (5 u32), uploaded by bvmv_features
  DevLayout L;
  // group
  int ngraphs = 1;
  int autotuned = 0;                   // 1: layout chosen by timing, 2: from the autotuner's cache
  std::vector<int64_t> offsets;        // ngraphs + 1
  std::vector<uint32_t> tile_offsets;  // ngraphs + 1
  PRWork pr;   // one right-hand side per member
  PRWork prb;  // k right-hand sides
  LearnWork lw;
  hipStream_t cap = nullptr;
  // left product (built on first use)
  bool left_ready = false;
  int64_t left_bytes = 0;
  DevLeft left{};
  std::vector<void*> left_bufs;

  void release_left() {
    for (void* p : left_bufs) dev_free(p);
    left_bufs.clear();
    left = DevLeft{};
    left_ready = false;
  }
  void release_device() {
    release_left();
    pr.release();
    prb.release();
    lw.release();
    dev_free(d_tiles);
    dev_free(d_info);
    dev_free(d_ns);
    dev_free(d_data);
    dev_free(d_longs);
    dev_free(d_outdeg);
    dev_free(d_stats);
    d_stats = nullptr;
    d_tiles = nullptr;
    d_info = nullptr;
    d_ns = nullptr;
    d_data = nullptr;
    d_longs = nullptr;
    d_outdeg = nullptr;
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
};

struct bvmv_csr {
  int device = 0;
  int64_t n = 0, m = 0;
  std::vector<CsrTile> tiles;
  CsrTile* d_tiles = nullptr;
  uint32_t* d_rowptr = nullptr;
  uint32_t* d_col = nullptr;
  int32_t* d_outdeg = nullptr;
  DevCsr C;
  PRWork pr;
  hipStream_t cap = nullptr;
};

namespace {

// A launch must fit the device's LDS per block.
int check_lds(int device, size_t bytes) {
  int lim = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || lim <= 0)
    lim = 65536;
  if (bytes > size_t(lim))
    return fail(BVMV_EINVAL, "layout needs " + std::to_string(bytes) + " bytes of LDS per block, the device allows " +
                                 std::to_string(lim) + ": lower window_cap or stage_bytes");
  return BVMV_OK;
}

int upload_layout(bvmv_graph* g) {
  const HostLayout& hl = g->hl;
  if (int rc = dev_upload(&g->d_tiles, hl.tiles.data(), hl.tiles.size())) return rc;
  if (int rc = dev_upload(&g->d_info, hl.info.data(), hl.info.size())) return rc;
  if (int rc = dev_upload(&g->d_ns, hl.ns.data(), hl.ns.size())) return rc;
  // zero padding after the last stream: a lane's round of stream words may
  // run up to kRound dwords past its stream's last dword
  if (int rc = dev_upload(&g->d_data, hl.data.data(), hl.data.size(), kDataPadBytes)) return rc;
  if (int rc = dev_upload(&g->d_longs, hl.longs.data(), hl.longs.size())) return rc;
  if (int rc = dev_upload(&g->d_outdeg, g->h_outdeg.data(), g->h_outdeg.size())) return rc;
  g->L.tiles = g->d_tiles;
  g->L.info = g->d_info;
  g->L.ns = g->d_ns;
  g->L.data = reinterpret_cast<const uint4*>(g->d_data);
  g->L.longs = g->d_longs;
  g->L.ntiles = uint32_t(hl.tiles.size());
  g->L.n = uint32_t(g->n);
  // LDS carve sizes: the largest use of any tile, rounded up
  uint32_t tcap = 0, wcap = 0, sb = 0;
  for (const auto& t : hl.tiles) {
    tcap = std::max(tcap, t.nrows);
    wcap = std::max(wcap, t.winlen);
    sb = std::max(sb, tile_stage_bytes(t));
  }
  g->L.tcap = std::max<uint32_t>(64, (tcap + 63) / 64 * 64);
  g->L.wcap = std::max<uint32_t>(64, (wcap + 3) / 4 * 4);
  g->L.sbytes = std::max<uint32_t>(256, (sb + 255) / 256 * 256);
  size_t need = 0;
  for (int prec = 0; prec <= 2; ++prec) need = std::max(need, bv_kernel_lds_bytes(g->L, prec));
  if (int rc = check_lds(g->device, need)) return rc;
  HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
  return BVMV_OK;
}

// Reads of an unset published value before a wave of a fused PageRank
// iteration folds the partials itself: kPubPolls, or BVMV_FOLD_POLLS from the
// environment (-1: every wave folds itself; a test of that path).
int32_t fold_polls() {
  const char* e = std::getenv("BVMV_FOLD_POLLS");
  if (!e || !*e) return kPubPolls;
  const long v = std::strtol(e, nullptr, 10);
  return int32_t(std::max<long>(-1, std::min<long>(v, 1 << 20)));
}

// Whether PageRank iterations fold the previous partials inside the product
// launch (fused) or in a finish kernel between launches.  Fused only for one
// graph and one right-hand side, and up to kFusedMaxBlocks blocks: the fold
// in the member's first block reads every block's partials, and past about
// 12k blocks it outlasts the first round of tiles, so the other waves wait
// on it.  Measured on web-like graphs, median of 40 runs: fused 4% faster at
// 8k blocks and 2% at 11.7k, equal at 17.6k, 3% slower at 31k; the CSR
// baseline's iteration 1% faster at 10.5k blocks, 2% slower at 15k and 52%
// slower at 50k.  A group keeps its finish kernel: with many members the
// waves of each wait on that member's first block (a 48-graph group ran
// about 5% slower fused).
constexpr int64_t kFusedMaxBlocks = 12288;
// BVMV_PR_FUSED from the environment: "0" never fuses, "1" fuses every run
// with one right-hand side (groups and graphs past kFusedMaxBlocks too);
// unset or anything else follows the rule above.  A knob for measuring and
// testing both forms; the fold order, and so every result, is the same.
int fused_mode() {
  const char* e = std::getenv("BVMV_PR_FUSED");
  if (e && e[0] == '0' && !e[1]) return 0;
  if (e && e[0] == '1' && !e[1]) return 1;
  return -1;
}
bool use_fused(int members, int k, int64_t blocks) {
  const int m = fused_mode();
  if (k != 1 || m == 0) return false;
  return m == 1 || (members == 1 && blocks <= kFusedMaxBlocks);
}

// Arguments of the iteration that reads buffer c % 2 and writes the other;
// fused: without a finish kernel, states and slots taken by parity (PRArgs).
PRArgs pr_args(const PRWork& w, const PROptsResolved& o, const void* tele, const int32_t* outdeg, int members, int k,
               int c, bool fused) {
  PRArgs a{};
  a.p_cur = w.p[c % 2];
  a.p_new = w.p[(c + 1) % 2];
  a.z_cur = w.z[c % 2];
  a.z_new = w.z[(c + 1) % 2];
  a.tele = tele;
  a.outdeg = outdeg;
  a.fused = fused ? 1 : 0;
  a.pub = w.pub;
  a.pub_polls = fold_polls();
  if (fused) {
    a.st = w.st + size_t(c % 2) * size_t(members);
    a.st_next = w.st + size_t((c + 1) % 2) * size_t(members);
    a.slots = w.slots + size_t((c + 1) % 2) * 2 * size_t(w.nslots);
    a.slots_prev = w.slots + size_t(c % 2) * 2 * size_t(w.nslots);
  } else {
    a.st = w.st;
    a.slots = w.slots;
  }
  a.beta = o.beta;
  a.tol = o.tol;
  a.max_iter = o.max_iter;
  a.buf = (c + 1) % 2;
  a.members = members;
  a.k = k;
  return a;
}

// Fold a run of fused iterations' last partials into the states of parity 0
// (no-op after iterations with a finish kernel) and clear the published values.
int flush_states(PRWork& w, const PROptsResolved& o, int members, hipStream_t s) {
  HIP_TRY(launch_pr_flush(w.st, w.slots, o.tol, o.max_iter, w.pub, members, s));
  return BVMV_OK;
}

// Host copy of the members' states (synchronises s).
int read_states(PRWork& w, int members, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(w.h_st, w.st, sizeof(PRState) * size_t(members), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return BVMV_OK;
}

// Iterations still to run after a replay: for each member not done, the
// count at which its residual, contracting by the ratio of its last two
// residuals, falls below tol (one more, and a whole chunk when the ratio is
// not yet known or not below 1), at most its iterations left; the largest
// over the members, rounded up to even.  A ratio below the damping factor
// is taken halfway to it: the power method's contraction tends to the
// damping factor from below on these graphs, and one more host round trip
// costs about as much as eight iterations whose blocks all return at once.
int planned_iterations(const PRState* sts, const PROptsResolved& o, int members) {
  int plan = 0;
  for (int gI = 0; gI < members; ++gI) {
    const PRState& st = sts[gI];
    if (st.done) continue;
    int need = o.chunk;
    if (st.resid > 0.0 && st.resid_prev > st.resid && st.resid >= o.tol) {
      double rate = st.resid / st.resid_prev;
      if (rate < o.beta) rate = 0.5 * (rate + o.beta);
      const double it = std::ceil(std::log(o.tol / st.resid) / std::log(rate));
      if (it >= 0.0 && it < 4.0 * o.chunk) need = int(it) + 1;
    }
    need = std::max(1, std::min(need, o.max_iter - st.iter));
    plan = std::max(plan, need);
  }
  return std::max(2, (plan + 1) / 2 * 2);
}

// Run PageRank iterations as replays of captured runs of iterations, each
// starting from buffer 0 (an even length) until every member is done: first
// one chunk, then as many iterations as the members' residuals predict
// (planned_iterations), as runs of the chunk's length and its halvings,
// launched back to back before the states are read.  The runs are captured
// once and kept with the working set while its key holds.
template <class IterFn>
int replay_until_done(PRWork& w, hipStream_t cap, const PROptsResolved& o, const void* tele, const int32_t* outdeg,
                      int members, int k, hipStream_t s, IterFn iter, bool fused) {
  const bool same = w.exec[0] && w.key_tele == tele && w.key_beta == o.beta && w.key_tol == o.tol &&
                    w.key_max_iter == o.max_iter && w.key_chunk == o.chunk && w.key_fused == int(fused) &&
                    w.key_polls == fold_polls();
  if (!same) {
    w.drop_graph();
    w.key_tele = tele;
    w.key_beta = o.beta;
    w.key_tol = o.tol;
    w.key_max_iter = o.max_iter;
    w.key_chunk = o.chunk;
    w.key_fused = int(fused);
    w.key_polls = fold_polls();
  }
  // the captured run of `len` iterations (captured on first use)
  auto run_of = [&](int len, hipGraphExec_t* out) -> int {
    int slot = -1;
    for (int i = 0; i < PRWork::kGraphs; ++i) {
      if (w.glen[i] == len && w.exec[i]) {
        *out = w.exec[i];
        return BVMV_OK;
      }
      if (slot < 0 && !w.exec[i]) slot = i;
    }
    if (slot < 0) return fail(BVMV_EDEVICE, "PageRank: no free graph slot");
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int c = 0; c < len && ce == hipSuccess; ++c)
      ce = iter(pr_args(w, o, tele, outdeg, members, k, c, fused), cap);
    hipGraph_t gr = nullptr;
    hipError_t ee = hipStreamEndCapture(cap, &gr);
    if (ce != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return fail(BVMV_EDEVICE, std::string("PageRank launch: ") + hipGetErrorString(ce));
    }
    if (ee != hipSuccess) return fail(BVMV_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    w.graph[slot] = gr;
    HIP_TRY(hipGraphInstantiate(&w.exec[slot], gr, nullptr, nullptr, 0));
    w.glen[slot] = len;
    *out = w.exec[slot];
    return BVMV_OK;
  };
  // the chunk first: it also occupies slot 0, whose presence marks the key as captured
  hipGraphExec_t first = nullptr;
  if (int rc = run_of(o.chunk, &first)) return rc;
  int plan = o.chunk;
  for (int done_iters = 0; done_iters <= o.max_iter + o.chunk;) {
    // plan as runs of the chunk's length and its even halvings
    for (int left = plan; left > 0;) {
      int len = o.chunk;
      while (len > left && len > 2) len = std::max(2, (len / 2 + 1) / 2 * 2);
      hipGraphExec_t ex = nullptr;
      if (int rc = run_of(len, &ex)) return rc;
      HIP_TRY(hipGraphLaunch(ex, s));
      left -= len;
      done_iters += len;
    }
    if (int rc = flush_states(w, o, members, s)) return rc;
    if (int rc = read_states(w, members, s)) return rc;
    bool all = true;
    for (int gI = 0; gI < members; ++gI) all = all && w.h_st[gI].done;
    if (all) break;
    plan = planned_iterations(w.h_st, o, members);
  }
  return BVMV_OK;
}

// Results from the host copy of the states; BVMV_NOT_CONVERGED if a member
// did not converge.
// rejected / accepted: per-member restart counts, or null (none).
int fill_results(const PRWork& w, int members, int used, const int* rejected, const int* accepted,
                 bvmv_pr_result* res) {
  int status = BVMV_OK;
  for (int gI = 0; gI < members; ++gI) {
    const PRState& st = w.h_st[gI];
    if (res) {
      const int rj = rejected ? rejected[gI] : 0, ac = accepted ? accepted[gI] : 0;
      res[gI].iters = st.iter;
      res[gI].converged = st.converged;
      res[gI].residual = st.resid;
      res[gI].used_start = used;
      res[gI].products = st.iter + rj;
      res[gI].restarts_accepted = ac;
      res[gI].restarts_rejected = rj;
    }
    if (!st.converged) status = BVMV_NOT_CONVERGED;
  }
  return status;
}

// Launch chunked PageRank on a tile layout, a group or a CSR, for one or k
// right-hand sides.  `states` holds the members' start states (1/n, slot
// ranges); p and z hold n_elems elements; `iter` launches one iteration on a
// stream, `init` the start kernels, `out` writes p_out from the final
// buffers once every member is done.
template <class IterFn, class InitFn, class OutFn>
int run_pagerank(PRWork& w, hipStream_t cap, const PROptsResolved& o, int64_t n_elems, int k,
                 const std::vector<PRState>& states, int64_t nslots, const void* tele, const void* start,
                 bvmv_pr_result* res, hipStream_t s, const int32_t* outdeg, IterFn iter, InitFn init, OutFn out) {
  const int members = int(states.size());
  if (int rc = w.ensure(o.prec, n_elems, members, nslots)) return rc;
  if (!outdeg || !w.p[0] || !w.p[1] || !w.z[0] || !w.z[1] || !w.st || !w.slots || !w.h_st)
    return fail(BVMV_EINVAL, "PageRank working set is incomplete");
  auto reset = [&](const void* st0) -> int {
    std::memcpy(w.h_st, states.data(), sizeof(PRState) * size_t(members));
    HIP_TRY(hipMemcpyAsync(w.st, w.h_st, sizeof(PRState) * size_t(members), hipMemcpyHostToDevice, s));
    HIP_TRY(init(st0, tele, w.p[0], w.z[0], s));
    // (clears the published values of fused iterations; nothing is pending)
    return flush_states(w, o, members, s);
  };
  int used = start ? 1 : 0;
  if (o.fallback && start && members == 1 && k == 1) {
    // one eager iteration from each candidate start; keep `start` only if
    // its first residual is the smaller
    double r[2] = {0.0, 0.0};
    for (int cand = 0; cand < 2; ++cand) {
      if (int rc = reset(cand == 0 ? start : nullptr)) return rc;
      HIP_TRY(iter(pr_args(w, o, tele, outdeg, members, k, 0, false), s));
      if (int rc = read_states(w, 1, s)) return rc;
      r[cand] = w.h_st[0].resid;
    }
    if (!(r[0] < r[1])) {
      start = nullptr;
      used = 0;
    }
  }
  if (int rc = reset(start)) return rc;
  // (the slots are the blocks' partials plus one)
  const bool fused = use_fused(members, k, nslots - 1);
  if (int rc = replay_until_done(w, cap, o, tele, outdeg, members, k, s, iter, fused)) return rc;
  HIP_TRY(out(w, s));
  return fill_results(w, members, used, 0, 0, res);
}

}  // namespace

namespace {
template <class T>
struct DevBuf {  // device scratch freed on scope exit
  T* p = nullptr;
  hipError_t alloc(size_t count) { return hipMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T)); }
  ~DevBuf() { dev_free(p); }
};
}  // namespace

// ------------------------------------------------------------ learned warm start
namespace {
std::vector<PRState> member_states(const std::vector<int64_t>& offsets, const std::vector<uint32_t>& tile_offsets) {
  std::vector<PRState> v(offsets.size() - 1);
  for (size_t gI = 0; gI < v.size(); ++gI) {
    std::memset(&v[gI], 0, sizeof(PRState));
    v[gI].inv_n = 1.0 / double(offsets[gI + 1] - offsets[gI]);
    v[gI].blk_lo = tile_offsets[gI] / kTilesPerBlock;
    v[gI].blk_hi = tile_offsets[gI + 1] / kTilesPerBlock;
  }
  return v;
}

// p_out rows of each member from the buffer holding its final iterate
hipError_t copy_member_outputs(const PRWork& w, const std::vector<int64_t>& offsets, int prec, void* p_out,
                               hipStream_t s) {
  const size_t es = elem_size(prec);
  for (size_t gI = 0; gI + 1 < offsets.size(); ++gI) {
    const PRState& st = w.h_st[gI];
    const size_t off = size_t(offsets[gI]) * es;
    const size_t bytes = size_t(offsets[gI + 1] - offsets[gI]) * es;
    const int fb = st.done ? st.final_buf : 0;
    if (hipError_t e = hipMemcpyAsync(static_cast<char*>(p_out) + off, static_cast<const char*>(w.p[fb]) + off,
                                      bytes, hipMemcpyDeviceToDevice, s))
      return e;
  }
  return hipSuccess;
}
}  // namespace

struct bvmv_mlp {
  int device = 0;
  float* theta = nullptr;   // FP32 master parameters
  uint16_t* wq = nullptr;   // BF16 weight copies
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* grad = nullptr;    // gradient + loss
  float* part = nullptr;    // per-tile gradient partials
  int64_t part_rows = 0;
  int step = 0;
};


namespace {

// Structural inputs 0..7 of every node into columns 0..7 of F (synchronous:
// the scratch is freed on return).
int compute_structural(bvmv_graph* g, float* F, int64_t stride, hipStream_t s) {
  if (g->dec.stats.size() != size_t(g->n)) return fail(BVMV_EINVAL, "row statistics missing");
  const int64_t n = g->n;
  if (!g->d_stats) {
    static_assert(sizeof(RowStats) == 5 * sizeof(uint32_t), "row statistics layout");
    if (int rc = dev_upload(&g->d_stats, reinterpret_cast<const uint32_t*>(g->dec.stats.data()), size_t(n) * 5))
      return rc;
  }
  DevBuf<int32_t> indeg;
  DevBuf<float> xb, yb;
  if (indeg.alloc(size_t(n)) || xb.alloc(2 * size_t(n)) || yb.alloc(2 * size_t(n)))
    return fail(BVMV_ENOMEM, "feature scratch");
  float* xd = xb.p;
  float* xi = xb.p + n;
  float* yd = yb.p;
  float* yi = yb.p + n;
  HIP_TRY(launch_bv_degrees(g->L, indeg.p, s));
  HIP_TRY(launch_feature_inputs(n, indeg.p, g->d_outdeg, xd, xi, s));
  HIP_TRY(launch_bv_multiply(g->L, BVMV_F32_COMP, xd, yd, s));
  HIP_TRY(launch_bv_multiply(g->L, BVMV_F32_COMP, xi, yi, s));
  HIP_TRY(launch_features(n, indeg.p, g->d_outdeg, g->d_stats, yd, yi, 1.0f / float(std::max(g->R, 1)), F, stride,
                          s));
  HIP_TRY(hipStreamSynchronize(s));
  return BVMV_OK;
}

// Plain PageRank from the uniform vector (or a restart) on a single graph,
// driven eagerly.  `c` is the buffer index of the current iterate and `since`
// the number of iterations since the start or the last kept restart; the
// phase runs until since = K, copying the iterate K - 3 into lw.t[0] and the
// iterate K - 2 into lw.t[1] just before the buffers they occupy are
// overwritten, so that at the end p_K, p_{K-1}, p_{K-2}, p_{K-3} are in
// w.p[c % 2], w.p[(c + 1) % 2], lw.t[1], lw.t[0].  Iterations of a member
// already done are skipped by the kernels.  The states start and end folded
// in w.st (parity 0).  Where run_pagerank would fuse (use_fused) and the
// phase ends on an even c, its iterations are fused (no finish kernel
// between products; the states
// enter at parity c % 2 and the last partials are folded by the flush), else
// each has its finish kernel, as run_pagerank does.
int run_phase(bvmv_graph* g, const PROptsResolved& o, int K, int& c, int& since, hipStream_t s) {
  PRWork& w = g->pr;
  LearnWork& lw = g->lw;
  const int M = g->ngraphs;
  const size_t bytes = size_t(g->n) * elem_size(o.prec);
  const bool fused =
      use_fused(M, 1, int64_t(g->L.ntiles) / kTilesPerBlock) && since < K && (c + K - since) % 2 == 0;
  if (fused && c % 2)
    HIP_TRY(hipMemcpyAsync(w.st + M, w.st, sizeof(PRState) * size_t(M), hipMemcpyDeviceToDevice, s));
  for (; since < K; ++since, ++c) {
    if (since == K - 2) HIP_TRY(hipMemcpyAsync(lw.t[0], w.p[(c + 1) % 2], bytes, hipMemcpyDeviceToDevice, s));
    if (since == K - 1) HIP_TRY(hipMemcpyAsync(lw.t[1], w.p[(c + 1) % 2], bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_bv_pagerank_iter(g->L, o.prec, pr_args(w, o, nullptr, g->d_outdeg, M, 1, c, fused), s));
  }
  if (fused) return flush_states(w, o, M, s);
  return BVMV_OK;
}

// Working sets and the uniform start state for run_phase.
int start_learned(bvmv_graph* g, const PROptsResolved& o, hipStream_t s) {
  PRWork& w = g->pr;
  const std::vector<PRState> states = member_states(g->offsets, g->tile_offsets);
  const int M = g->ngraphs;
  if (int rc = w.ensure(o.prec, g->n, M, int64_t(g->L.ntiles) / kTilesPerBlock + 1)) return rc;
  if (int rc = g->lw.ensure(o.prec, g->n)) return rc;
  std::memcpy(w.h_st, states.data(), sizeof(PRState) * size_t(M));
  HIP_TRY(hipMemcpyAsync(w.st, w.h_st, sizeof(PRState) * size_t(M), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_pr_init(g->L, o.prec, nullptr, nullptr, w.p[0], w.z[0], g->d_outdeg, w.st, w.slots, M, s));
  // (clears the published values of fused iterations; nothing is pending)
  return flush_states(w, o, M, s);
}

// PageRank with learned warm restarts (a single graph or a group, uniform
// teleport).  After each phase of K iterations: the inputs, the network, the
// restart vector q and its sum, p' = q / sum as every member's new iterate
// with the iteration count kept, and one probe iteration.  Each member keeps
// its restart if its probe residual r' < beta * delta, else it resumes from
// p_K (saved in lw.t[1]) with the state it had at the phase's end.  A restart
// is tried only while every member is active, and not after a rejection.
// The rest runs as captured chunks.
int run_learned(bvmv_graph* g, const PROptsResolved& o, const bvmv_mlp* m, void* p_out, bvmv_pr_result* res,
                hipStream_t s) {
  PRWork& w = g->pr;
  LearnWork& lw = g->lw;
  const int M = g->ngraphs;
  if (int rc = start_learned(g, o, s)) return rc;
  if (!lw.struct_ready) {
    if (int rc = compute_structural(g, lw.Fs, 8, s)) return rc;
    lw.struct_ready = true;
  }
  const DevLayout& L = g->L;
  const size_t bytes = size_t(g->n) * elem_size(o.prec);
  std::vector<int> accepted(size_t(M), 0), rejected(size_t(M), 0);
  std::vector<PRState> at_k(static_cast<size_t>(M));
  int c = 0, since = 0;
  bool done = false;
  auto all_done = [&] {
    for (int i = 0; i < M; ++i)
      if (!w.h_st[i].done) return false;
    return true;
  };
  for (int tried = 0; tried < o.max_restarts; ++tried) {
    if (int rc = run_phase(g, o, o.restart_every, c, since, s)) return rc;
    if (int rc = read_states(w, M, s)) return rc;
    if (all_done()) {
      done = true;
      break;
    }
    bool any_done = false;
    for (int i = 0; i < M; ++i) any_done = any_done || w.h_st[i].done;
    if (any_done) break;
    std::copy(w.h_st, w.h_st + M, at_k.begin());  // every member at iteration at_k[0].iter
    HIP_TRY(launch_restart_inputs(L, o.prec, w.p[c % 2], w.p[(c + 1) % 2], lw.t[1], lw.t[0], nullptr, w.st, lw.Ft,
                                  4, nullptr, s));
    HIP_TRY(launch_mlp_forward(m->theta, m->wq, FeatIn{lw.Fs, lw.Ft, 8, 4}, g->n, lw.s, s));
    HIP_TRY(launch_restart_vector(L, o.prec, w.p[c % 2], lw.s, w.st, lw.t[0], w.slots, M, s));
    HIP_TRY(hipMemcpyAsync(lw.t[1], w.p[c % 2], bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_pr_init(L, o.prec, lw.t[0], nullptr, w.p[0], w.z[0], g->d_outdeg, w.st, w.slots, M, s, 1,
                           at_k[0].iter));
    HIP_TRY(launch_bv_pagerank_iter(L, o.prec, pr_args(w, o, nullptr, g->d_outdeg, M, 1, 0, false), s));
    c = 1;
    if (int rc = read_states(w, M, s)) return rc;
    bool any_rejected = false;
    for (int i = 0; i < M; ++i) {
      if (w.h_st[i].resid < o.beta * at_k[size_t(i)].resid) {
        ++accepted[size_t(i)];
        continue;
      }
      // back to p_K and the phase-end state (the probe still counts as a product)
      ++rejected[size_t(i)];
      any_rejected = true;
      HIP_TRY(launch_pr_restore(o.prec, lw.t[1], w.p[1], w.z[1], g->d_outdeg, g->offsets[size_t(i)],
                                g->offsets[size_t(i) + 1], s));
      w.h_st[i] = at_k[size_t(i)];
    }
    if (any_rejected) {
      HIP_TRY(hipMemcpyAsync(w.st, w.h_st, sizeof(PRState) * size_t(M), hipMemcpyHostToDevice, s));
      break;
    }
    since = 1;
    if (all_done()) {
      done = true;
      break;
    }
  }
  if (!done && c % 2) {
    // the captured chunk starts from buffer 0
    HIP_TRY(launch_bv_pagerank_iter(L, o.prec, pr_args(w, o, nullptr, g->d_outdeg, M, 1, c, false), s));
    if (int rc = read_states(w, M, s)) return rc;
    done = all_done();
  }
  if (!done) {
    // (fused where run_pagerank would fuse; the published values were
    // cleared by the last flush, and the iterations since then had finish
    // kernels and left them alone)
    auto iter = [&](const PRArgs& a, hipStream_t cs) { return launch_bv_pagerank_iter(L, o.prec, a, cs); };
    const bool fused = use_fused(M, 1, int64_t(L.ntiles) / kTilesPerBlock);
    if (int rc = replay_until_done(w, g->cap, o, nullptr, g->d_outdeg, M, 1, s, iter, fused)) return rc;
  }
  HIP_TRY(copy_member_outputs(w, g->offsets, o.prec, p_out, s));
  return fill_results(w, M, 0, rejected.data(), accepted.data(), res);
}

}  // namespace


namespace {

// Candidate layouts of the load-time autotuner: (tile rows, x-window columns,
// staged entry bytes).  The stage grows with the tile so that rows of the
// same length stay off the long-row path.
constexpr int kTuneCands[][3] = {{32, 256, 2048}, {64, 256, 4096}, {64, 384, 3072},
                                 {64, 512, 4096}, {64, 768, 6144}, {128, 768, 6144}};
constexpr int kTuneCount = int(sizeof(kTuneCands) / sizeof(kTuneCands[0]));

// The winner per size bucket (floor(log2 n), rounded 2 log2(mean degree + 1)),
// kept for the life of the process.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune_cache;

std::pair<int, int> tune_key(int64_t n, int64_t m) {
  int ln = 0;
  while ((int64_t(1) << (ln + 1)) <= n) ++ln;
  const double deg = n > 0 ? double(m) / double(n) : 0.0;
  return {ln, int(std::lround(2.0 * std::log2(deg + 1.0)))};
}

// Average time of one FP32 two-sum product on the uploaded layout: two
// warm-up launches, then `reps` back-to-back launches between HIP events.
int time_product(bvmv_graph* g, const float* x, float* y, int reps, float* us) {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  auto cleanup = [&] {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
  };
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch_bv_multiply(g->L, BVMV_F32_COMP, x, y, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_bv_multiply(g->L, BVMV_F32_COMP, x, y, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  cleanup();
  if (e != hipSuccess) return fail(BVMV_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
  *us = 1000.0f * ms / float(reps);
  return BVMV_OK;
}

}  // namespace

extern "C" {

const char* bvmv_last_error(void) { return g_err.c_str(); }
const char* bvmv_version(void) { return "bvmv 0.1 (gfx950)"; }

int bvmv_decode(const void* bitstream, size_t nbytes, int nthreads, uint64_t* rowptr, uint32_t* col, uint8_t* refs,
                int64_t* n, int64_t* m) {
  if (!bitstream || !n || !m) return fail(BVMV_EINVAL, "null argument");
  DecodedGraph dg;
  std::string err;
  if (decode_stream(static_cast<const uint8_t*>(bitstream), nbytes, default_threads(nthreads), dg, err))
    return fail(BVMV_EFORMAT, err);
  *n = dg.n;
  *m = dg.m;
  if (rowptr) std::memcpy(rowptr, dg.rowptr.data(), dg.rowptr.size() * 8);
  if (col && dg.m) std::memcpy(col, dg.col.data(), dg.col.size() * 4);
  if (refs) std::memcpy(refs, dg.refs.data(), dg.refs.size());
  return BVMV_OK;
}

int bvmv_load(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts, bvmv_graph** out) {
  if (!bitstream || !out) return fail(BVMV_EINVAL, "null argument");
  *out = nullptr;
  bvmv_load_opts o{};
  if (opts) o = *opts;
  if (o.tile_rows == 0) o.tile_rows = 64;
  if (o.window_cap == 0) o.window_cap = 256;
  if (o.stage_bytes == 0) o.stage_bytes = 4096;
  if (o.long_row_bytes == 0) o.long_row_bytes = o.stage_bytes / 2;
  if (o.tile_rows < 8 || o.tile_rows > kTileRowsMax || o.window_cap < 64 || o.window_cap > 8191 ||
      o.stage_bytes < 512 || o.stage_bytes > 16384 || o.long_row_bytes < 16 || o.long_row_bytes > o.stage_bytes ||
      o.interval_mode < 0 || o.interval_mode > 1 || o.device < 0)
    return fail(BVMV_EINVAL, "load option out of range");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) return fail(BVMV_EINVAL, "no such device");
  std::unique_ptr<bvmv_graph> g(new bvmv_graph());
  g->device = o.device;
  g->opts = o;
  g->interval_mode = o.interval_mode;
  std::string err;
  const int nt = default_threads(o.nthreads);
  if (decode_stream(static_cast<const uint8_t*>(bitstream), nbytes, nt, g->dec, err)) return fail(BVMV_EFORMAT, err);
  g->n = g->dec.n;
  g->m = g->dec.m;
  g->stream_bytes = int64_t(nbytes);
  g->W = int(g->dec.hdr.W);
  g->R = int(g->dec.hdr.R);
  g->Lmin = int(g->dec.hdr.Lmin);
  g->zk = int(g->dec.hdr.zeta_k);
  g->h_outdeg.assign(size_t(g->n), 0);
  for (uint32_t c : g->dec.col) ++g->h_outdeg[c];
  LayoutParams prm;
  prm.tile_rows = o.tile_rows;
  prm.window_cap = o.window_cap;
  prm.long_row_bytes = o.long_row_bytes;
  prm.stage_bytes = o.stage_bytes;
  if (o.interval_mode == 1) prm.min_interval = INT_MAX;  // runs stay single entries
  DeviceGuard dg(o.device);
  if (dg.err != hipSuccess) return fail(BVMV_EDEVICE, "hipSetDevice failed");
  if (o.autotune) {
    // candidate layouts, each built, uploaded and timed in turn; the fastest
    // (or the cached winner of this size bucket) is rebuilt below
    const std::pair<int, int> key = tune_key(g->n, g->m);
    int best = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) best = it->second;
    }
    g->autotuned = best >= 0 ? 2 : 1;
    if (best < 0) {
      DevBuf<float> xb, yb;
      if (xb.alloc(size_t(g->n)) || yb.alloc(size_t(g->n))) return fail(BVMV_ENOMEM, "autotune vectors");
      HIP_TRY(hipMemset(xb.p, 0, size_t(std::max<int64_t>(g->n, 1)) * sizeof(float)));
      float best_us = 0.0f;
      for (int c = 0; c < kTuneCount; ++c) {
        LayoutParams cp = prm;
        cp.tile_rows = kTuneCands[c][0];
        cp.window_cap = kTuneCands[c][1];
        cp.stage_bytes = kTuneCands[c][2];
        cp.long_row_bytes = cp.stage_bytes / 2;
        g->hl = HostLayout();
        if (build_layout(g->dec, cp, nt, g->hl, err)) continue;
        if (upload_layout(g.get()) != BVMV_OK) {  // e.g. more LDS than a block may use
          g->release_device();
          continue;
        }
        float us = 0.0f;
        const int rc = time_product(g.get(), xb.p, yb.p, 20, &us);
        g->release_device();
        if (rc) return rc;
        if (best < 0 || us < best_us) {
          best = c;
          best_us = us;
        }
      }
      if (best < 0) return fail(BVMV_EINVAL, "no autotune candidate fits the device");
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = best;
    }
    prm.tile_rows = kTuneCands[best][0];
    prm.window_cap = kTuneCands[best][1];
    prm.stage_bytes = kTuneCands[best][2];
    prm.long_row_bytes = prm.stage_bytes / 2;
    g->hl = HostLayout();
  }
  if (build_layout(g->dec, prm, nt, g->hl, err)) return fail(BVMV_EINVAL, err);
  g->m_prime = g->hl.m_prime;
  if (o.device_mem_budget && uint64_t(g->hl.bytes()) + uint64_t(g->n) * 4 > o.device_mem_budget)
    return fail(BVMV_ENOMEM, "layout exceeds the device memory budget");
  g->offsets = {0, g->n};
  g->tile_offsets = {0, uint32_t(g->hl.tiles.size())};
  if (int rc = upload_layout(g.get())) {
    g->release_device();
    return rc;
  }
  if (o.keep_lists) {
    g->lists_kept = true;
  } else if (!o.autotune) {
    // (an autotuned graph keeps its lists, so that a group of graphs tuned to
    // different layouts can lay them all out with one layout)
    std::vector<uint32_t>().swap(g->dec.col);
    std::vector<uint64_t>().swap(g->dec.rowptr);
    std::vector<uint8_t>().swap(g->dec.refs);
  }
  *out = g.release();
  return BVMV_OK;
}

namespace {
// [a, a + na) and [b, b + nb) share a byte
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}
}  // namespace

void bvmv_free(bvmv_graph* g) {
  if (!g) return;
  {
    DeviceGuard dg(g->device);
    g->release_device();
  }
  delete g;
}

int bvmv_multiply(bvmv_graph* g, const void* x, void* y, int prec, void* stream) {
  if (!g || !x || !y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return fail(BVMV_EINVAL, "bad precision");
  const size_t vbytes = size_t(g->n) * elem_size(prec);
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(BVMV_EINVAL, "x and y must not overlap");
  DeviceGuard dg(g->device);
  HIP_TRY(launch_bv_multiply(g->L, prec, x, y, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

// y = x A on the tiles of the layout (built once per graph, on first use).
int bvmv_multiply_left(bvmv_graph* g, const void* x, void* y, int prec, void* stream) {
  if (!g || !x || !y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return fail(BVMV_EINVAL, "bad precision");
  if (g->ngraphs != 1) return fail(BVMV_EINVAL, "the left product takes a single graph, not a group");
  const size_t vbytes = size_t(g->n) * elem_size(prec);
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(BVMV_EINVAL, "x and y must not overlap");
  DeviceGuard dg(g->device);
  if (!g->left_ready) {
    LeftLayout ll;
    std::string err;
    if (build_left_layout(g->hl, ll, err)) return fail(BVMV_EINVAL, err);
    if (int rc = check_lds(g->device, std::max(bv_left_lds_bytes(g->L, 0), bv_left_lds_bytes(g->L, 1)))) return rc;
    DevLeft D;
    auto up = [&](auto** dst, const auto& v) -> int {
      if (int rc = dev_upload(dst, v.data(), v.size())) return rc;
      g->left_bufs.push_back(*dst);
      return BVMV_OK;
    };
    LeftTile* lt = nullptr;
    uint16_t *ent = nullptr, *grp = nullptr;
    uint32_t *lanes = nullptr, *eo = nullptr, *co = nullptr, *cov = nullptr;
    LeftEscape* esc = nullptr;
    if (up(&lt, ll.tiles) || up(&ent, ll.entries) || up(&grp, ll.groups) || up(&lanes, ll.lanes) ||
        up(&esc, ll.esc) || up(&eo, ll.esc_off) || up(&co, ll.cov_off) || up(&cov, ll.cov)) {
      g->release_left();
      return BVMV_ENOMEM;
    }
    void *part = nullptr, *cb = nullptr;
    if (hipMalloc(&part, std::max<uint64_t>(ll.part_len, 1) * 8) != hipSuccess) part = nullptr;
    if (part) g->left_bufs.push_back(part);
    if (hipMalloc(&cb, size_t(std::max<int64_t>(g->n, 1)) * 8) != hipSuccess) cb = nullptr;
    if (cb) g->left_bufs.push_back(cb);
    if (!part || !cb) {
      g->release_left();
      return fail(BVMV_ENOMEM, "hipMalloc of the left product's buffers failed");
    }
    D.lt = lt;
    D.ent = ent;
    D.grp = grp;
    D.lanes = lanes;
    D.part = part;
    D.cbuf = cb;
    D.esc = esc;
    D.esc_off = eo;
    D.cov_off = co;
    D.cov = cov;
    D.n = uint32_t(g->n);
    g->left = D;
    g->left_bytes = ll.bytes();
    g->left_ready = true;
  }
  HIP_TRY(launch_bv_left(g->L, g->left, prec, x, y, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_multiply_batch(bvmv_graph* g, const void* X, void* Y, int k, int64_t ld, int prec, void* stream) {
  if (!g || !X || !Y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2 || k < 1 || k > 64 || ld < g->n) return fail(BVMV_EINVAL, "bad batch arguments");
  const size_t bbytes = (size_t(k - 1) * size_t(ld) + size_t(g->n)) * elem_size(prec);
  if (ranges_overlap(X, bbytes, Y, bbytes)) return fail(BVMV_EINVAL, "X and Y must not overlap");
  DeviceGuard dg(g->device);
  HIP_TRY(launch_bv_multiply_cols(g->L, prec, X, Y, k, ld, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_degrees(bvmv_graph* g, int32_t* deg, void* stream) {
  if (!g || !deg) return fail(BVMV_EINVAL, "null argument");
  DeviceGuard dg(g->device);
  HIP_TRY(launch_bv_degrees(g->L, deg, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_pagerank(bvmv_graph* g, const bvmv_pr_opts* opts, const void* teleport, const void* start, void* p_out,
                  int k, bvmv_pr_result* res, void* stream) {
  if (!g || !p_out) return fail(BVMV_EINVAL, "null argument");
  PROptsResolved o;
  if (int rc = resolve_pr_opts(opts, o)) return rc;
  if (k < 1 || k > 64) return fail(BVMV_EINVAL, "k must be in 1..64");
  if (k > 1 && g->ngraphs != 1) return fail(BVMV_EINVAL, "k > 1 needs a single graph, not a group");
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevLayout L = g->L;
  const int prec = o.prec;
  if (o.mlp) {
    if (k != 1 || teleport || start)
      return fail(BVMV_EINVAL, "learned restarts need k = 1, uniform teleport and no start vector");
    if (o.mlp->device != g->device) return fail(BVMV_EINVAL, "graph and network on different devices");
    return run_learned(g, o, o.mlp, p_out, res, s);
  }
  if (k == 1) {
    auto iter = [&](const PRArgs& a, hipStream_t cs) { return launch_bv_pagerank_iter(L, prec, a, cs); };
    auto init = [&](const void* st, const void* te, void* p0, void* z0, hipStream_t ss) {
      return launch_pr_init(L, prec, st, te, p0, z0, g->d_outdeg, g->pr.st, g->pr.slots,
                            int(g->offsets.size()) - 1, ss);
    };
    auto out = [&](const PRWork& w, hipStream_t ss) { return copy_member_outputs(w, g->offsets, prec, p_out, ss); };
    return run_pagerank(g->pr, g->cap, o, g->n, 1, member_states(g->offsets, g->tile_offsets),
                        int64_t(L.ntiles) / kTilesPerBlock + 1, teleport, start, res, s, g->d_outdeg, iter, init,
                        out);
  }
  // k right-hand sides: one state per column, each column's block partials at
  // slots c * groups .. (c + 1) * groups - 1 (one block per group of tiles)
  const uint32_t groups = L.ntiles / kTilesPerBlock;
  if (int64_t(groups) * k >= (int64_t(1) << 32)) return fail(BVMV_EINVAL, "too many tiles for k right-hand sides");
  std::vector<PRState> states(static_cast<size_t>(k));
  for (int c = 0; c < k; ++c) {
    std::memset(&states[size_t(c)], 0, sizeof(PRState));
    states[size_t(c)].inv_n = 1.0 / double(g->n);
    states[size_t(c)].blk_lo = 0;
    states[size_t(c)].blk_hi = groups;
    states[size_t(c)].slot0 = uint32_t(c) * groups;
  }
  PRWork& w = g->prb;
  auto iter = [&](const PRArgs& a, hipStream_t cs) { return launch_bv_cols_pagerank_iter(L, prec, a, cs); };
  auto init = [&](const void* st, const void* te, void* p0, void* z0, hipStream_t ss) {
    return launch_cols_pr_init(L, prec, k, st, te, p0, z0, g->d_outdeg, w.st, w.slots, ss);
  };
  auto out = [&](const PRWork& ww, hipStream_t ss) {
    return launch_pr_select(prec, ww.st, ww.p[0], ww.p[1], p_out, g->n, k, ss);
  };
  return run_pagerank(w, g->cap, o, g->n * k, k, states, int64_t(groups) * k + 1, teleport, start, res, s,
                      g->d_outdeg, iter, init, out);
}

// PageRank of one graph, k = 1, with its working set in the library's fixed
// device array instead of allocated buffers: no allocation, no graph capture,
// no pinned host memory.  Iterations are launched eagerly, `chunk` at a time,
// and the state is read back after each chunk by a synchronising copy into a
// host stack variable.  The iterations are always fused (bvmv_pagerank fuses
// them up to kFusedMaxBlocks blocks, and the array's limit keeps 64-row
// layouts below that); the fold order is the same in both forms, so the
// results are bit-identical to bvmv_pagerank's.
static_assert(BVMV_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "the header states the array's size");

int bvmv_pagerank_noalloc(bvmv_graph* g, const bvmv_pr_opts* opts, const void* teleport, const void* start,
                          void* p_out, bvmv_pr_result* res, void* stream) {
  if (!g || !p_out) return fail(BVMV_EINVAL, "null argument");
  PROptsResolved o;
  if (int rc = resolve_pr_opts(opts, o)) return rc;
  if (o.mlp || o.fallback)
    return fail(BVMV_EINVAL, "the allocation-free PageRank takes no network and no fallback check");
  if (g->ngraphs != 1) return fail(BVMV_EINVAL, "the allocation-free PageRank takes a single graph, not a group");
  DeviceGuard dg(g->device);
  if (dg.err != hipSuccess) return fail(BVMV_EDEVICE, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLayout& L = g->L;
  const int prec = o.prec;
  // carve: p0, p1, z0, z1 (n elements each), the block partials of both
  // parities, the states of both parities, the two published values
  auto up256 = [](uint64_t v) { return (v + 255) / 256 * 256; };
  const uint64_t vec = up256(uint64_t(g->n) * elem_size(prec));
  const uint64_t nslots = uint64_t(L.ntiles) / kTilesPerBlock + 1;
  const uint64_t slot_bytes = up256(16 * nslots);
  const uint64_t st_bytes = up256(2 * sizeof(PRState));
  const uint64_t need = 4 * vec + 2 * slot_bytes + st_bytes + 256;
  if (need > kNoAllocScratchBytes)
    return fail(BVMV_EINVAL, "graph too large for the allocation-free PageRank: its working set needs " +
                                 std::to_string(need) + " bytes, the fixed array holds " +
                                 std::to_string(kNoAllocScratchBytes));
  void* base = nullptr;
  HIP_TRY(noalloc_scratch(g->device, &base));
  unsigned char* b = static_cast<unsigned char*>(base);
  void* p[2] = {b, b + vec};
  void* z[2] = {b + 2 * vec, b + 3 * vec};
  double* slots = reinterpret_cast<double*>(b + 4 * vec);  // parity 0, then parity 1 at slot_bytes
  PRState* st = reinterpret_cast<PRState*>(b + 4 * vec + 2 * slot_bytes);  // parity 0, then 1
  double* pub = reinterpret_cast<double*>(b + 4 * vec + 2 * slot_bytes + st_bytes);
  PRState st0;
  std::memset(&st0, 0, sizeof(st0));
  st0.inv_n = 1.0 / double(g->n);
  st0.blk_lo = 0;
  st0.blk_hi = L.ntiles / kTilesPerBlock;
  HIP_TRY(launch_pr_state_set(st, st0, s));
  HIP_TRY(launch_pr_init(L, prec, start, teleport, p[0], z[0], g->d_outdeg, st, slots, 1, s));
  // (clears the published values; the start state has nothing pending)
  HIP_TRY(launch_pr_flush(st, slots, o.tol, o.max_iter, pub, 1, s));
  PRArgs a{};
  a.tele = teleport;
  a.outdeg = g->d_outdeg;
  a.fused = 1;
  a.pub = pub;
  a.pub_polls = fold_polls();
  a.beta = o.beta;
  a.tol = o.tol;
  a.max_iter = o.max_iter;
  a.members = 1;
  a.k = 1;
  PRState h;
  std::memset(&h, 0, sizeof(h));
  // a chunk, then as many iterations as the residuals predict (an even
  // count, so every run starts from buffer 0)
  int plan = o.chunk;
  for (int done_iters = 0; done_iters <= o.max_iter + o.chunk; done_iters += plan) {
    for (int c = 0; c < plan; ++c) {
      a.p_cur = p[c % 2];
      a.p_new = p[(c + 1) % 2];
      a.z_cur = z[c % 2];
      a.z_new = z[(c + 1) % 2];
      a.buf = (c + 1) % 2;
      a.st = st + c % 2;
      a.st_next = st + (c + 1) % 2;
      a.slots = slots + size_t((c + 1) % 2) * (slot_bytes / 8);
      a.slots_prev = slots + size_t(c % 2) * (slot_bytes / 8);
      HIP_TRY(launch_bv_pagerank_iter(L, prec, a, s));
    }
    HIP_TRY(launch_pr_flush(st, slots, o.tol, o.max_iter, pub, 1, s));
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(PRState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h.done) break;
    plan = planned_iterations(&h, o, 1);
  }
  HIP_TRY(launch_pr_select(prec, st, p[0], p[1], p_out, g->n, 1, s));
  if (res) {
    res->iters = h.iter;
    res->converged = h.converged;
    res->residual = h.resid;
    res->used_start = start ? 1 : 0;
    res->products = h.iter;
    res->restarts_accepted = 0;
    res->restarts_rejected = 0;
  }
  return h.converged ? BVMV_OK : BVMV_NOT_CONVERGED;
}

namespace {
bool same_layout(const LayoutParams& a, const LayoutParams& b) {
  return a.tile_rows == b.tile_rows && a.window_cap == b.window_cap && a.stage_bytes == b.stage_bytes &&
         a.long_row_bytes == b.long_row_bytes && a.min_interval == b.min_interval;
}

// The members' layouts (`lay[i]` for member i) one after another as the
// group's layout, with the members' rows, tiles and row statistics.
int concat_group(bvmv_graph* g, bvmv_graph* const* graphs, int count, const HostLayout* const* lay) {
  g->device = graphs[0]->device;
  g->opts = graphs[0]->opts;
  g->interval_mode = graphs[0]->interval_mode;
  g->ngraphs = count;
  g->n = g->m = g->m_prime = g->stream_bytes = 0;
  g->offsets.assign(1, 0);
  g->tile_offsets.assign(1, 0);
  g->h_outdeg.clear();
  g->dec.stats.clear();
  HostLayout& hl = g->hl;
  hl = HostLayout();
  hl.prm = lay[0]->prm;
  for (int i = 0; i < count; ++i) {
    const bvmv_graph* m = graphs[i];
    const HostLayout& ml = *lay[i];
    const uint64_t rb = uint64_t(g->n), db = hl.data.size(), lb = hl.longs.size();
    if (rb + uint64_t(m->n) >= (uint64_t(1) << 30) || (db + ml.data.size()) / 16 >= (uint64_t(1) << 32) ||
        lb + ml.longs.size() >= (uint64_t(1) << 32))
      return fail(BVMV_EINVAL, "group too large");
    for (TileDesc td : ml.tiles) {
      td.row0 += uint32_t(rb);
      td.win0 += uint32_t(rb);
      td.data16 += uint32_t(db / 16);
      td.long0 += uint32_t(lb);
      td.graph = uint32_t(i);
      hl.tiles.push_back(td);
    }
    hl.info.insert(hl.info.end(), ml.info.begin(), ml.info.end());
    hl.ns.insert(hl.ns.end(), ml.ns.begin(), ml.ns.end());
    hl.data.insert(hl.data.end(), ml.data.begin(), ml.data.end());
    hl.longs.insert(hl.longs.end(), ml.longs.begin(), ml.longs.end());
    hl.n_singles += ml.n_singles;
    hl.n_wide += ml.n_wide;
    hl.n_intervals += ml.n_intervals;
    g->h_outdeg.insert(g->h_outdeg.end(), m->h_outdeg.begin(), m->h_outdeg.end());
    hl.units += ml.units;
    hl.diff_rows += ml.diff_rows;
    hl.direct_rows += ml.direct_rows;
    hl.long_rows += ml.long_rows;
    hl.escapes += ml.escapes;
    hl.m_prime += ml.m_prime;
    hl.max_level = std::max(hl.max_level, ml.max_level);
    g->n += m->n;
    g->m += m->m;
    g->m_prime += ml.m_prime;
    g->stream_bytes += m->stream_bytes;
    g->offsets.push_back(g->n);
    g->tile_offsets.push_back(uint32_t(hl.tiles.size()));
  }
  hl.n = g->n;
  // row statistics for the learned restarts' inputs: kept when every member
  // has them and the members share R (the depth input is depth / R)
  bool stats = true;
  for (int i = 0; i < count; ++i)
    stats = stats && graphs[i]->dec.stats.size() == size_t(graphs[i]->n) && graphs[i]->R == graphs[0]->R;
  if (stats)
    for (int i = 0; i < count; ++i)
      g->dec.stats.insert(g->dec.stats.end(), graphs[i]->dec.stats.begin(), graphs[i]->dec.stats.end());
  g->W = graphs[0]->W;
  g->R = graphs[0]->R;
  g->Lmin = graphs[0]->Lmin;
  g->zk = graphs[0]->zk;
  return BVMV_OK;
}
}  // namespace

int bvmv_group(bvmv_graph* const* graphs, int count, bvmv_graph** out) {
  if (!graphs || count < 1 || !out) return fail(BVMV_EINVAL, "bad group arguments");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    const bvmv_graph* m = graphs[i];
    if (!m || m->ngraphs != 1) return fail(BVMV_EINVAL, "group members must be loaded graphs");
    if (m->device != graphs[0]->device) return fail(BVMV_EINVAL, "group members must share the device");
  }
  std::unique_ptr<bvmv_graph> g(new bvmv_graph());
  DeviceGuard dg(graphs[0]->device);
  std::vector<const HostLayout*> lay(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) lay[size_t(i)] = &graphs[i]->hl;
  // Members laid out with different layouts (each tuned alone) would force
  // the widest LDS carve and the two-rows-per-lane kernel on every block of
  // the group.  When every member still has its lists (autotuned loads keep
  // them), each of the members' layouts is timed over the whole group and
  // the fastest is used for all of them.
  std::vector<LayoutParams> classes;
  bool relayable = true;
  for (int i = 0; i < count; ++i) {
    const bvmv_graph* m = graphs[i];
    relayable = relayable && m->dec.col.size() == size_t(m->m) && m->dec.rowptr.size() == size_t(m->n) + 1;
    bool seen = false;
    for (const auto& c : classes) seen = seen || same_layout(c, m->hl.prm);
    if (!seen) classes.push_back(m->hl.prm);
  }
  std::vector<HostLayout> own_lay;
  if (classes.size() > 1 && relayable) {
    const int nt = default_threads(0);
    std::string err;
    DevBuf<float> xb, yb;
    int64_t ntot = 0;
    for (int i = 0; i < count; ++i) ntot += graphs[i]->n;
    if (xb.alloc(size_t(ntot)) || yb.alloc(size_t(ntot))) return fail(BVMV_ENOMEM, "group autotune vectors");
    HIP_TRY(hipMemset(xb.p, 0, size_t(std::max<int64_t>(ntot, 1)) * sizeof(float)));
    int best = -1;
    float best_us = 0.0f;
    for (size_t c = 0; c < classes.size(); ++c) {
      std::vector<HostLayout> tl(static_cast<size_t>(count));
      std::vector<const HostLayout*> tp(static_cast<size_t>(count));
      bool ok = true;
      for (int i = 0; i < count && ok; ++i) {
        if (same_layout(graphs[i]->hl.prm, classes[c])) {
          tp[size_t(i)] = &graphs[i]->hl;
        } else {
          ok = build_layout(graphs[i]->dec, classes[c], nt, tl[size_t(i)], err) == 0;
          tp[size_t(i)] = &tl[size_t(i)];
        }
      }
      if (!ok) continue;
      bvmv_graph trial;
      if (int rc = concat_group(&trial, graphs, count, tp.data())) return rc;
      if (upload_layout(&trial) != BVMV_OK) {
        trial.release_device();
        continue;
      }
      float us = 0.0f;
      const int rc = time_product(&trial, xb.p, yb.p, 10, &us);
      trial.release_device();
      if (rc) return rc;
      if (best < 0 || us < best_us) {
        best = int(c);
        best_us = us;
      }
    }
    if (best < 0) return fail(BVMV_EINVAL, "no member layout fits the group on the device");
    own_lay.resize(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) {
      if (same_layout(graphs[i]->hl.prm, classes[size_t(best)])) continue;
      if (build_layout(graphs[i]->dec, classes[size_t(best)], nt, own_lay[size_t(i)], err))
        return fail(BVMV_EINVAL, err);
      lay[size_t(i)] = &own_lay[size_t(i)];
    }
    g->autotuned = 1;
  }
  if (int rc = concat_group(g.get(), graphs, count, lay.data())) return rc;
  if (int rc = upload_layout(g.get())) {
    g->release_device();
    return rc;
  }
  *out = g.release();
  return BVMV_OK;
}

int bvmv_group_offsets(const bvmv_graph* g, int64_t* offsets, int* count) {
  if (!g) return fail(BVMV_EINVAL, "null argument");
  if (count) *count = g->ngraphs;
  if (offsets) std::copy(g->offsets.begin(), g->offsets.end(), offsets);
  return BVMV_OK;
}

int bvmv_get_info(const bvmv_graph* g, bvmv_info* out) {
  if (!g || !out) return fail(BVMV_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->n = g->n;
  out->m = g->m;
  out->m_prime = g->m_prime;
  out->units = g->hl.units;
  out->diff_rows = g->hl.diff_rows;
  out->direct_rows = g->hl.direct_rows;
  out->long_rows = g->hl.long_rows;
  out->escapes = g->hl.escapes;
  out->ntiles = int64_t(g->hl.tiles.size());
  out->layout_bytes = g->hl.bytes();
  out->stream_bytes = g->stream_bytes;
  out->W = g->W;
  out->R = g->R;
  out->Lmin = g->Lmin;
  out->zeta_k = g->zk;
  out->tile_rows = g->hl.prm.tile_rows;
  out->window_cap = g->hl.prm.window_cap;
  out->long_row_bytes = g->hl.prm.long_row_bytes;
  out->stage_bytes = g->hl.prm.stage_bytes;
  out->n_singles = g->hl.n_singles;
  out->n_wide = g->hl.n_wide;
  out->n_intervals = g->hl.n_intervals;
  out->interval_mode = g->interval_mode;
  out->max_level = g->hl.max_level;
  out->ngraphs = g->ngraphs;
  out->autotuned = g->autotuned;
  return BVMV_OK;
}

int bvmv_export_csr(const bvmv_graph* g, uint64_t* rowptr, uint32_t* col) {
  if (!g || !rowptr || !col) return fail(BVMV_EINVAL, "null argument");
  if (!g->lists_kept) return fail(BVMV_EINVAL, "graph was loaded without keep_lists");
  std::memcpy(rowptr, g->dec.rowptr.data(), g->dec.rowptr.size() * 8);
  if (g->m) std::memcpy(col, g->dec.col.data(), g->dec.col.size() * 4);
  return BVMV_OK;
}

// ------------------------------------------------------------------ CSR
int bvmv_csr_create_host(int64_t n, const uint64_t* rowptr, const uint32_t* col, int device, bvmv_csr** out) {
  if (n < 1 || !rowptr || !out) return fail(BVMV_EINVAL, "bad CSR arguments");
  *out = nullptr;
  if (uint64_t(n) >= 0xFFFFFFFFull) return fail(BVMV_EINVAL, "n too large for 32-bit row ids");
  // a decreasing offset would make a row length wrap around and send the
  // tiles' column reads past the array
  if (rowptr[0] != 0) return fail(BVMV_EINVAL, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(BVMV_EINVAL, "rowptr must be nondecreasing");
  const uint64_t m = rowptr[n];
  if (m >= (uint64_t(1) << 32) - 1) return fail(BVMV_EINVAL, "CSR too large for 32-bit row pointers");
  static const uint32_t kNoColumns = 0;
  if (!col) {
    if (m) return fail(BVMV_EINVAL, "bad CSR arguments");
    col = &kNoColumns;  // an edgeless graph: never read
  }
  std::unique_ptr<bvmv_csr> c(new bvmv_csr());
  c->device = device;
  c->n = n;
  c->m = int64_t(m);
  std::vector<uint32_t> rp32(size_t(n) + 1);
  for (int64_t i = 0; i <= n; ++i) rp32[size_t(i)] = uint32_t(rowptr[i]);
  std::vector<int32_t> outdeg(size_t(n), 0);
  for (uint64_t k = 0; k < m; ++k) {
    if (col[k] >= uint64_t(n)) return fail(BVMV_EINVAL, "column out of range");
    ++outdeg[col[k]];
  }
  // the compressed layout's defaults: 64 rows per wave, 4 KB of staged ids,
  // rows over 2 KB summed by the whole wave, x windows up to 512 columns
  const int rcap = 64, ccap = 1024, long_cols = 512, wcap_max = 512;
  build_csr_tiles(rowptr, col, n, rcap, ccap, long_cols, wcap_max, c->tiles, uint64_t(n));
  uint32_t wcap = 0;
  for (const auto& t : c->tiles) wcap = std::max(wcap, t.winlen);
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(BVMV_EDEVICE, "hipSetDevice failed");
  auto cleanup = [&] {
    dev_free(c->d_tiles);
    dev_free(c->d_rowptr);
    dev_free(c->d_col);
    dev_free(c->d_outdeg);
  };
  if (dev_upload(&c->d_tiles, c->tiles.data(), c->tiles.size()) ||
      dev_upload(&c->d_rowptr, rp32.data(), rp32.size()) || dev_upload(&c->d_col, col, size_t(m), 4) ||
      dev_upload(&c->d_outdeg, outdeg.data(), outdeg.size())) {
    cleanup();
    return BVMV_ENOMEM;
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    cleanup();
    return fail(BVMV_EDEVICE, "hipStreamCreate failed");
  }
  c->C.tiles = c->d_tiles;
  c->C.rowptr = c->d_rowptr;
  c->C.col = c->d_col;
  c->C.ntiles = uint32_t(c->tiles.size());
  c->C.n = uint32_t(n);
  c->C.col_len = m + 4;
  uint32_t cmax = 0;
  for (const auto& t : c->tiles)
    if (!(t.nrows & 0x80000000u)) cmax = std::max(cmax, t.ncols);
  c->C.ccap = std::max<uint32_t>(64, (cmax + 63) / 64 * 64);
  c->C.wcap = std::max<uint32_t>(64, (wcap + 63) / 64 * 64);
  if (int rc = check_lds(device, std::max(csr_kernel_lds_bytes(c->C, BVMV_F64), csr_kernel_lds_bytes(c->C, BVMV_F32_COMP)))) {
    cleanup();
    (void)hipStreamDestroy(c->cap);
    return rc;
  }
  *out = c.release();
  return BVMV_OK;
}

int bvmv_csr_create(const bvmv_graph* g, bvmv_csr** out) {
  if (!g || !out) return fail(BVMV_EINVAL, "null argument");
  if (!g->lists_kept || g->ngraphs != 1) return fail(BVMV_EINVAL, "graph was loaded without keep_lists");
  return bvmv_csr_create_host(g->n, g->dec.rowptr.data(), g->dec.col.empty() ? nullptr : g->dec.col.data(),
                              g->device, out);
}

int bvmv_csr_multiply(bvmv_csr* c, const void* x, void* y, int prec, void* stream) {
  if (!c || !x || !y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return fail(BVMV_EINVAL, "bad precision");
  const size_t vbytes = size_t(c->n) * elem_size(prec);
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(BVMV_EINVAL, "x and y must not overlap");
  DeviceGuard dg(c->device);
  HIP_TRY(launch_csr_multiply(c->C, prec, x, y, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_csr_pagerank(bvmv_csr* c, const bvmv_pr_opts* opts, const void* teleport, const void* start, void* p_out,
                      bvmv_pr_result* res, void* stream) {
  if (!c || !p_out) return fail(BVMV_EINVAL, "null argument");
  PROptsResolved o;
  if (int rc = resolve_pr_opts(opts, o)) return rc;
  DeviceGuard dg(c->device);
  DevCsr C = c->C;
  const int prec = o.prec;
  std::vector<int64_t> offsets{0, c->n};
  std::vector<PRState> states(1);
  std::memset(&states[0], 0, sizeof(PRState));
  states[0].inv_n = 1.0 / double(c->n);
  states[0].blk_hi = C.ntiles / kTilesPerBlock;
  auto iter = [&](const PRArgs& a, hipStream_t cs) { return launch_csr_pagerank_iter(C, prec, a, cs); };
  auto init = [&](const void* st, const void* te, void* p0, void* z0, hipStream_t ss) {
    return launch_csr_pr_init(C, prec, st, te, p0, z0, c->d_outdeg, c->pr.st, c->pr.slots, ss);
  };
  auto out = [&](const PRWork& w, hipStream_t ss) { return copy_member_outputs(w, offsets, prec, p_out, ss); };
  return run_pagerank(c->pr, c->cap, o, c->n, 1, states, int64_t(C.ntiles) / kTilesPerBlock + 1, teleport, start,
                      res, static_cast<hipStream_t>(stream), c->d_outdeg, iter, init, out);
}

int64_t bvmv_csr_bytes(const bvmv_csr* c) {
  if (!c) return 0;
  return int64_t(c->n + 1) * 4 + c->m * 4;
}

void bvmv_csr_free(bvmv_csr* c) {
  if (!c) return;
  {
    DeviceGuard dg(c->device);
    c->pr.release();
    dev_free(c->d_tiles);
    dev_free(c->d_rowptr);
    dev_free(c->d_col);
    dev_free(c->d_outdeg);
    if (c->cap) (void)hipStreamDestroy(c->cap);
  }
  delete c;
}



// --------------------------------------------------------- column blocks
// A matrix split into submatrices of consecutive columns, each loaded as a
// graph of its own (same n; its own references, so a row may match different
// reference rows in different blocks): y = A_1 x + A_2 x + ..., the first
// block storing y and the others adding to it, in block order.
struct bvmv_colblocks {
  int device = 0;
  int64_t n = 0;
  std::vector<bvmv_graph*> blocks;  // owned by the caller
};

int bvmv_colblocks_create(bvmv_graph* const* blocks, int count, bvmv_colblocks** out) {
  if (!blocks || count < 1 || !out) return fail(BVMV_EINVAL, "bad column-block arguments");
  *out = nullptr;
  std::unique_ptr<bvmv_colblocks> c(new bvmv_colblocks());
  c->device = blocks[0] ? blocks[0]->device : 0;
  c->n = blocks[0] ? blocks[0]->n : 0;
  for (int b = 0; b < count; ++b) {
    const bvmv_graph* g = blocks[b];
    if (!g || g->ngraphs != 1) return fail(BVMV_EINVAL, "column blocks must be loaded graphs");
    if (g->n != c->n || g->device != c->device)
      return fail(BVMV_EINVAL, "column blocks must share n and the device");
    c->blocks.push_back(blocks[b]);
  }
  *out = c.release();
  return BVMV_OK;
}

int bvmv_colblocks_multiply(bvmv_colblocks* c, const void* x, void* y, int prec, void* stream) {
  if (!c || !x || !y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return fail(BVMV_EINVAL, "bad precision");
  const size_t vbytes = size_t(c->n) * elem_size(prec);
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(BVMV_EINVAL, "x and y must not overlap");
  DeviceGuard dg(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (size_t b = 0; b < c->blocks.size(); ++b) {
    if (b == 0)
      HIP_TRY(launch_bv_multiply(c->blocks[b]->L, prec, x, y, s));
    else
      HIP_TRY(launch_bv_multiply_add(c->blocks[b]->L, prec, x, y, s));
  }
  return BVMV_OK;
}

void bvmv_colblocks_free(bvmv_colblocks* c) { delete c; }

// ------------------------------------------------------------ bicliques
// The biclique format (Section "Final Remarks"): c_r = sum_{j in C_r} x_j for
// every biclique, then y_i = sum_{r : i in S_r} c_r + sum_{j in Res_i} x_j.
// Both passes run the CSR tile kernel: the first over the C lists (rows =
// bicliques, ids = columns of x), the second over each node's residual
// columns followed by its bicliques' ids n + r, which read the sums c.
struct bvmv_biclique {
  int device = 0;
  int64_t n = 0, m = 0, nbic = 0, s_ids = 0, c_ids = 0, res = 0;
  std::vector<CsrTile> t_sum, t_row;
  CsrTile *d_tsum = nullptr, *d_trow = nullptr;
  uint32_t *d_cptr = nullptr, *d_cidx = nullptr, *d_rptr = nullptr, *d_ridx = nullptr;
  void* d_c = nullptr;  // the biclique sums, nbic elements of the precision's type
  DevCsr Csum, Crow;
  int64_t layout_bytes = 0;
  void release() {
    dev_free(d_tsum);
    dev_free(d_trow);
    dev_free(d_cptr);
    dev_free(d_cidx);
    dev_free(d_rptr);
    dev_free(d_ridx);
    dev_free(d_c);
    d_tsum = d_trow = nullptr;
    d_cptr = d_cidx = d_rptr = d_ridx = nullptr;
    d_c = nullptr;
  }
};

namespace {
// offsets p[0..cnt] start at 0 and do not decrease
bool offsets_ok(const uint64_t* p, int64_t cnt) {
  if (p[0] != 0) return false;
  for (int64_t i = 0; i < cnt; ++i)
    if (p[i + 1] < p[i]) return false;
  return true;
}
// ids a[0..len) strictly increasing and below n
bool ids_ok(const uint32_t* a, uint64_t len, int64_t n) {
  for (uint64_t k = 0; k < len; ++k)
    if (int64_t(a[k]) >= n || (k && a[k] <= a[k - 1])) return false;
  return true;
}
}  // namespace

int bvmv_biclique_load(int64_t n, int64_t nbic, const uint64_t* sptr, const uint32_t* sidx, const uint64_t* cptr,
                       const uint32_t* cidx, const uint64_t* rptr, const uint32_t* rcol, int device,
                       bvmv_biclique** out) {
  if (!out) return fail(BVMV_EINVAL, "null argument");
  *out = nullptr;
  if (n < 1 || nbic < 0 || !rptr || (nbic > 0 && (!sptr || !cptr)))
    return fail(BVMV_EINVAL, "bad biclique arguments");
  if (uint64_t(n) + uint64_t(nbic) >= 0xFFFFFFFFull) return fail(BVMV_EINVAL, "n + bicliques must be below 2^32 - 1");
  static const uint64_t kZero = 0;
  if (nbic == 0) sptr = cptr = &kZero;
  if (!offsets_ok(sptr, nbic) || !offsets_ok(cptr, nbic) || !offsets_ok(rptr, n))
    return fail(BVMV_EFORMAT, "offsets must start at 0 and not decrease");
  const uint64_t ns = sptr[nbic], nc = cptr[nbic], nr = rptr[n];
  if ((ns && !sidx) || (nc && !cidx) || (nr && !rcol)) return fail(BVMV_EINVAL, "bad biclique arguments");
  for (int64_t r = 0; r < nbic; ++r)
    if (!ids_ok(sidx + sptr[r], sptr[r + 1] - sptr[r], n) || !ids_ok(cidx + cptr[r], cptr[r + 1] - cptr[r], n))
      return fail(BVMV_EFORMAT, "biclique " + std::to_string(r) + ": ids must be strictly increasing and below n");
  for (int64_t i = 0; i < n; ++i)
    if (!ids_ok(rcol + rptr[i], rptr[i + 1] - rptr[i], n))
      return fail(BVMV_EFORMAT, "residual row " + std::to_string(i) + ": ids must be strictly increasing and below n");
  // each node's bicliques (ascending r), by counting
  std::vector<uint64_t> mp(size_t(n) + 1, 0);
  for (uint64_t k = 0; k < ns; ++k) ++mp[size_t(sidx[k]) + 1];
  for (int64_t i = 0; i < n; ++i) mp[size_t(i) + 1] += mp[size_t(i)];
  std::vector<uint32_t> memb(ns ? ns : 1);
  {
    std::vector<uint64_t> pos(mp.begin(), mp.end() - 1);
    for (int64_t r = 0; r < nbic; ++r)
      for (uint64_t k = sptr[r]; k < sptr[r + 1]; ++k) memb[pos[sidx[k]]++] = uint32_t(r);
  }
  // the edges must be a partition: no (i, j) in two bicliques or in a biclique
  // and the residual (rows checked in parallel blocks)
  std::atomic<int64_t> dup_row{-1};
  uint64_t m = nr;
  for (int64_t r = 0; r < nbic; ++r) m += (sptr[r + 1] - sptr[r]) * (cptr[r + 1] - cptr[r]);
  {
    const int nt = default_threads(0);
    std::atomic<int64_t> next{0};
    const int64_t blk = 4096;
    auto worker = [&] {
      std::vector<uint32_t> row;
      for (int64_t b = next.fetch_add(blk); b < n && dup_row.load() < 0; b = next.fetch_add(blk))
        for (int64_t i = b; i < std::min(n, b + blk); ++i) {
          row.assign(rcol + rptr[i], rcol + rptr[i + 1]);
          for (uint64_t k = mp[size_t(i)]; k < mp[size_t(i) + 1]; ++k) {
            const uint32_t r = memb[k];
            row.insert(row.end(), cidx + cptr[r], cidx + cptr[r + 1]);
          }
          std::sort(row.begin(), row.end());
          if (std::adjacent_find(row.begin(), row.end()) != row.end()) {
            int64_t none = -1;
            dup_row.compare_exchange_strong(none, i);
            return;
          }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
  }
  if (dup_row.load() >= 0)
    return fail(BVMV_EFORMAT, "row " + std::to_string(dup_row.load()) +
                                  " lists an edge twice (the bicliques and residual must partition the edges)");
  if (m >= (uint64_t(1) << 32) || ns + nr >= (uint64_t(1) << 32) || nc >= (uint64_t(1) << 32))
    return fail(BVMV_EINVAL, "biclique format too large for 32-bit offsets");
  std::unique_ptr<bvmv_biclique> b(new bvmv_biclique());
  b->device = device;
  b->n = n;
  b->m = int64_t(m);
  b->nbic = nbic;
  b->s_ids = int64_t(ns);
  b->c_ids = int64_t(nc);
  b->res = int64_t(nr);
  // second pass rows: residual columns, then n + r for the node's bicliques
  std::vector<uint64_t> rp2(size_t(n) + 1, 0);
  std::vector<uint32_t> ids2(ns + nr ? ns + nr : 1);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t o = rp2[size_t(i)];
    for (uint64_t k = rptr[i]; k < rptr[i + 1]; ++k) ids2[o++] = rcol[k];
    for (uint64_t k = mp[size_t(i)]; k < mp[size_t(i) + 1]; ++k) ids2[o++] = uint32_t(n) + memb[k];
    rp2[size_t(i) + 1] = o;
  }
  // the CSR baseline's tile shape: 64 rows, 1024 staged ids, rows over 512 ids
  // summed by the whole wave, windows up to 512 columns
  const int rcap = 64, ccap = 1024, long_cols = 512, wcap_max = 512;
  if (nbic) build_csr_tiles(cptr, cidx, nbic, rcap, ccap, long_cols, wcap_max, b->t_sum, uint64_t(n));
  build_csr_tiles(rp2.data(), ids2.data(), n, rcap, ccap, long_cols, wcap_max, b->t_row, uint64_t(n));
  std::vector<uint32_t> cp32(size_t(nbic) + 1), rp32(size_t(n) + 1);
  for (int64_t r = 0; r <= nbic; ++r) cp32[size_t(r)] = uint32_t(cptr[r]);
  for (int64_t i = 0; i <= n; ++i) rp32[size_t(i)] = uint32_t(rp2[size_t(i)]);
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(BVMV_EDEVICE, "hipSetDevice failed");
  static const uint32_t kNoIds = 0;
  if (dev_upload(&b->d_tsum, b->t_sum.data(), b->t_sum.size()) ||
      dev_upload(&b->d_trow, b->t_row.data(), b->t_row.size()) ||
      dev_upload(&b->d_cptr, cp32.data(), cp32.size()) ||
      dev_upload(&b->d_cidx, nc ? cidx : &kNoIds, nc ? size_t(nc) : 1, 4) ||
      dev_upload(&b->d_rptr, rp32.data(), rp32.size()) ||
      dev_upload(&b->d_ridx, ids2.data(), size_t(ns + nr ? ns + nr : 1), 4)) {
    b->release();
    return BVMV_ENOMEM;
  }
  if (hipMalloc(&b->d_c, size_t(std::max<int64_t>(nbic, 1)) * 8) != hipSuccess) {
    b->d_c = nullptr;
    b->release();
    return fail(BVMV_ENOMEM, "hipMalloc of the biclique sums failed");
  }
  auto setup = [&](DevCsr& C, const std::vector<CsrTile>& tiles, const CsrTile* dt, const uint32_t* drp,
                   const uint32_t* dcol, uint64_t len) {
    C.tiles = dt;
    C.rowptr = drp;
    C.col = dcol;
    C.ntiles = uint32_t(tiles.size());
    C.n = uint32_t(n);
    C.col_len = len + 4;
    uint32_t cmax = 0, wcap = 0;
    for (const auto& t : tiles) {
      if (!(t.nrows & 0x80000000u)) cmax = std::max(cmax, t.ncols);
      wcap = std::max(wcap, t.winlen);
    }
    C.ccap = std::max<uint32_t>(64, (cmax + 63) / 64 * 64);
    C.wcap = std::max<uint32_t>(64, (wcap + 63) / 64 * 64);
  };
  setup(b->Csum, b->t_sum, b->d_tsum, b->d_cptr, b->d_cidx, nc);
  setup(b->Crow, b->t_row, b->d_trow, b->d_rptr, b->d_ridx, ns + nr);
  b->Crow.nx = uint32_t(n);
  size_t lds = 0;
  for (int prec = 0; prec <= 2; ++prec)
    lds = std::max({lds, csr_kernel_lds_bytes(b->Csum, prec), csr_kernel_lds_bytes(b->Crow, prec)});
  if (int rc = check_lds(device, lds)) {
    b->release();
    return rc;
  }
  b->layout_bytes = int64_t((cp32.size() + rp32.size() + nc + ns + nr) * 4 +
                            (b->t_sum.size() + b->t_row.size()) * sizeof(CsrTile));
  *out = b.release();
  return BVMV_OK;
}

int bvmv_biclique_multiply(bvmv_biclique* b, const void* x, void* y, int prec, void* stream) {
  if (!b || !x || !y) return fail(BVMV_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return fail(BVMV_EINVAL, "bad precision");
  const size_t vbytes = size_t(b->n) * elem_size(prec);
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(BVMV_EINVAL, "x and y must not overlap");
  DeviceGuard dg(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->nbic) HIP_TRY(launch_csr_multiply(b->Csum, prec, x, b->d_c, s));
  DevCsr C = b->Crow;
  C.aux = b->d_c;
  HIP_TRY(launch_csr_multiply(C, prec, x, y, s));
  return BVMV_OK;
}

int bvmv_biclique_get_info(const bvmv_biclique* b, bvmv_biclique_info* out) {
  if (!b || !out) return fail(BVMV_EINVAL, "null argument");
  out->n = b->n;
  out->m = b->m;
  out->nbic = b->nbic;
  out->s_ids = b->s_ids;
  out->c_ids = b->c_ids;
  out->residual = b->res;
  out->words = b->s_ids + b->c_ids + b->res;
  out->layout_bytes = b->layout_bytes;
  return BVMV_OK;
}

void bvmv_biclique_free(bvmv_biclique* b) {
  if (!b) return;
  {
    DeviceGuard dg(b->device);
    b->release();
  }
  delete b;
}

int bvmv_features(bvmv_graph* g, float* F, void* stream) {
  if (!g || !F) return fail(BVMV_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(F) & 15) return fail(BVMV_EINVAL, "F must be 16-byte aligned");
  if (g->ngraphs != 1) return fail(BVMV_EINVAL, "features need a single graph");
  DeviceGuard dg(g->device);
  return compute_structural(g, F, kMlpIn, static_cast<hipStream_t>(stream));
}

int bvmv_restart_sample(bvmv_graph* g, int K, int prec, const void* p_star, float* F, float* T, double* delta,
                        void* stream) {
  if (!g || !F || (p_star && !T)) return fail(BVMV_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(F) & 15) return fail(BVMV_EINVAL, "F must be 16-byte aligned");
  if (g->ngraphs != 1) return fail(BVMV_EINVAL, "restart samples need a single graph");
  if (K < 3 || prec < 0 || prec > 2) return fail(BVMV_EINVAL, "K must be >= 3 and prec valid");
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bvmv_pr_opts po{};
  po.prec = prec;
  po.max_iter = K + 1;
  PROptsResolved o;
  if (int rc = resolve_pr_opts(&po, o)) return rc;
  if (int rc = compute_structural(g, F, kMlpIn, s)) return rc;
  if (int rc = start_learned(g, o, s)) return rc;
  int c = 0, since = 0;
  if (int rc = run_phase(g, o, K, c, since, s)) return rc;
  if (int rc = read_states(g->pr, 1, s)) return rc;
  if (g->pr.h_st[0].done) return fail(BVMV_EINVAL, "PageRank converged within K iterations");
  PRWork& w = g->pr;
  HIP_TRY(launch_restart_inputs(g->L, prec, w.p[c % 2], w.p[(c + 1) % 2], g->lw.t[1], g->lw.t[0], p_star, w.st, F + 8, kMlpIn, T,
                                s));
  HIP_TRY(hipStreamSynchronize(s));
  if (delta) *delta = w.h_st[0].resid;
  return BVMV_OK;
}

int bvmv_mlp_create(int device, const float* params, bvmv_mlp** out) {
  if (!params || !out) return fail(BVMV_EINVAL, "null argument");
  *out = nullptr;
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(BVMV_EDEVICE, "hipSetDevice failed");
  std::unique_ptr<bvmv_mlp> m(new bvmv_mlp());
  m->device = device;
  auto cleanup = [&] {
    dev_free(m->theta);
    dev_free(m->wq);
    dev_free(m->m);
    dev_free(m->v);
    dev_free(m->grad);
  };
  if (dev_upload(&m->theta, params, kMlpParams) ||
      hipMalloc(reinterpret_cast<void**>(&m->wq), kMlpWeights * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&m->m), kMlpParams * sizeof(float)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&m->v), kMlpParams * sizeof(float)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&m->grad), (kMlpParams + 1) * sizeof(float)) != hipSuccess) {
    cleanup();
    return fail(BVMV_ENOMEM, "network allocation");
  }
  if (hipMemset(m->m, 0, kMlpParams * sizeof(float)) != hipSuccess ||
      hipMemset(m->v, 0, kMlpParams * sizeof(float)) != hipSuccess ||
      launch_mlp_quantize(m->theta, m->wq, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    cleanup();
    return fail(BVMV_EDEVICE, "network initialisation");
  }
  *out = m.release();
  return BVMV_OK;
}

int bvmv_mlp_params(const bvmv_mlp* m, float* params) {
  if (!m || !params) return fail(BVMV_EINVAL, "null argument");
  DeviceGuard dg(m->device);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(params, m->theta, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
  return BVMV_OK;
}

int bvmv_mlp_forward(bvmv_mlp* m, const float* F, int64_t n, float* s, void* stream) {
  if (!m || !F || !s || n < 0) return fail(BVMV_EINVAL, "bad network arguments");
  if (reinterpret_cast<uintptr_t>(F) & 15) return fail(BVMV_EINVAL, "F must be 16-byte aligned");
  DeviceGuard dg(m->device);
  HIP_TRY(launch_mlp_forward(m->theta, m->wq, feat_rows12(F), n, s, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_mlp_gradient(bvmv_mlp* m, const float* F, const float* target, int64_t n, float* grad, void* stream) {
  if (!m || !F || !target || !grad || n < 1 || n > kMlpMaxBatch) return fail(BVMV_EINVAL, "bad network arguments");
  if (reinterpret_cast<uintptr_t>(F) & 15) return fail(BVMV_EINVAL, "F must be 16-byte aligned");
  DeviceGuard dg(m->device);
  const int64_t rows = (n + 31) / 32;
  if (rows > m->part_rows) {
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    dev_free(m->part);
    m->part = nullptr;
    m->part_rows = 0;
    if (hipMalloc(reinterpret_cast<void**>(&m->part), size_t(rows) * (kMlpParams + 1) * sizeof(float)) != hipSuccess)
      return fail(BVMV_ENOMEM, "gradient partials");
    m->part_rows = rows;
  }
  HIP_TRY(launch_mlp_gradient(m->theta, m->wq, F, target, n, m->part, grad, static_cast<hipStream_t>(stream)));
  return BVMV_OK;
}

int bvmv_mlp_train_step(bvmv_mlp* m, const float* F, const float* target, int64_t n, float lr, float* loss,
                        void* stream) {
  if (!m || !(lr > 0.0f)) return fail(BVMV_EINVAL, "bad network arguments");
  if (int rc = bvmv_mlp_gradient(m, F, target, n, m->grad, stream)) return rc;
  DeviceGuard dg(m->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_mlp_adam(m->theta, m->wq, m->m, m->v, m->grad, lr, 0.9f, 0.999f, 1e-8f, ++m->step, s));
  if (loss) HIP_TRY(hipMemcpyAsync(loss, m->grad + kMlpParams, sizeof(float), hipMemcpyDeviceToDevice, s));
  return BVMV_OK;
}

void bvmv_mlp_free(bvmv_mlp* m) {
  if (!m) return;
  {
    DeviceGuard dg(m->device);
    (void)hipDeviceSynchronize();
    dev_free(m->theta);
    dev_free(m->wq);
    dev_free(m->m);
    dev_free(m->v);
    dev_free(m->grad);
    dev_free(m->part);
  }
  delete m;
}

}  // extern "C"
