// Host-side launchers of the HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bv_layout.hpp"

namespace bvmv {

// Zero bytes after the last stream of the device data array (the tile kernel
// reads whole rounds of stream words without clamping them to the stream).
constexpr size_t kDataPadBytes = 64;

struct DevLayout {
  const TileDesc* tiles = nullptr;
  const uint32_t* info = nullptr;
  const uint16_t* ns = nullptr;
  const uint4* data = nullptr;
  const uint32_t* longs = nullptr;
  uint32_t ntiles = 0;                              // a multiple of kTilesPerBlock
  uint32_t tcap = 64, wcap = 512, sbytes = 4096;    // LDS carve sizes (>= every tile's use)
  uint32_t n = 0;                                   // rows = columns (length of x)
};

struct DevCsr {
  const CsrTile* tiles = nullptr;
  const uint32_t* rowptr = nullptr;  // n+1, 32-bit
  const uint32_t* col = nullptr;
  uint32_t ntiles = 0;               // a multiple of kTilesPerBlock
  uint32_t ccap = 1024, wcap = 512;
  uint32_t n = 0;                    // length of x (= rows, except for the biclique sums)
  uint64_t col_len = 0;              // readable elements of col (m plus padding to a 16-byte boundary)
  // ids at or above nx read aux[id - nx] instead of x[id] (the biclique
  // product's second pass: a row's bicliques are ids n + r of their sums);
  // nx = 2^32 - 1 leaves every id to x
  uint32_t nx = 0xFFFFFFFFu;
  const void* aux = nullptr;         // the second source (X*), or nullptr
};

// LDS bytes per block of the single-vector kernels (0 if the mode is unknown);
// the loader checks them against the device limit.
size_t bv_kernel_lds_bytes(const DevLayout& L, int prec);
size_t csr_kernel_lds_bytes(const DevCsr& C, int prec);

// Per-member PageRank state, updated by the last block of every iteration.
struct PRState {
  double delta;      // dangling mass of the current iterate
  double resid;      // ||p_t - p_{t-1}||_1 of the last iteration
  double inv_n;      // 1/n of the member (uniform teleport)
  int32_t iter;      // iterations done
  int32_t done;      // 1 once converged or out of iterations
  int32_t converged;
  int32_t final_buf; // buffer (0/1) holding the final iterate once done
  uint32_t blk_lo, blk_hi;    // block range of the member's partial slots
  uint32_t slot0;             // the member's first slot (slots slot0 + blk_lo .. slot0 + blk_hi - 1)
  int32_t pending;            // fused iterations: the iterate's partials are not folded in yet
  double resid_prev;          // the residual of the iteration before the last (0 before two iterations)
};

struct PRArgs {
  const void* p_cur;     // current iterate (X*)
  void* p_new;           // next iterate (X*)
  const void* z_cur;     // p_cur / d (X*), gathered by the product
  void* z_new;           // p_new / d (X*)
  const void* tele;      // teleport (X*), nullptr = uniform per member
  const int32_t* outdeg; // d_u
  PRState* st;           // per member
  double* slots;         // 2 doubles per tile
  double beta, tol;
  int32_t max_iter;
  int32_t buf;           // index of p_new's buffer (0/1)
  int32_t members;       // PRState entries (member graphs, or right-hand sides)
  int32_t k;             // right-hand sides (column-major p, z, teleport with leading dimension n)
  // Fused iterations (one right-hand side): no finish kernel between
  // products.  The iteration reading buffer c = 1 - buf reads the states st
  // and the partials slots_prev of parity c (left by the iteration before),
  // writes its partials to slots and, from the first block of each member,
  // the member's next state to st_next; that block folds the pending partials
  // and publishes the dangling mass in pub[2 member + c] for the member's
  // other blocks.
  int32_t fused;
  PRState* st_next;
  const double* slots_prev;
  double* pub;           // 2 doubles per member
  // reads of an unset published value before a wave folds the partials
  // itself; -1: every wave folds itself (a test of that path)
  int32_t pub_polls;
};
constexpr int32_t kPubPolls = 48;

hipError_t launch_bv_multiply(const DevLayout& L, int prec, const void* x, void* y, hipStream_t s);
// y += A x (column blocks after the first)
hipError_t launch_bv_multiply_add(const DevLayout& L, int prec, const void* x, void* y, hipStream_t s);
hipError_t launch_bv_degrees(const DevLayout& L, int32_t* deg, hipStream_t s);
hipError_t launch_bv_pagerank_iter(const DevLayout& L, int prec, const PRArgs& a, hipStream_t s);
// fold the last fused iteration's partials into the states (see PRArgs)
hipError_t launch_pr_flush(PRState* st, const double* slots, double tol, int32_t max_iter, double* pub, int members,
                           hipStream_t s);
// z = p / d, dangling mass and state reset for the start vector (tile grid)
// (normalize: p0 = start / the member's delta field; iter0: the states' iteration count)
hipError_t launch_pr_init(const DevLayout& L, int prec, const void* start, const void* tele, void* p0, void* z0,
                          const int32_t* outdeg, PRState* st, double* slots, int members, hipStream_t s,
                          int normalize = 0, int32_t iter0 = 0);
// k columns of a column-major block (leading dimension ld) through the tile
// kernel: the tile is decoded once and each column staged and summed in turn
hipError_t launch_bv_multiply_cols(const DevLayout& L, int prec, const void* X, void* Y, int k, int64_t ld,
                                   hipStream_t s);
// one personalized PageRank iteration for a.k <= 64 columns (p, z column-major,
// ld = n; column c's state a.st[c], its block partials at slots c * groups + group)
hipError_t launch_bv_cols_pagerank_iter(const DevLayout& L, int prec, const PRArgs& a, hipStream_t s);
hipError_t launch_cols_pr_init(const DevLayout& L, int prec, int k, const void* start, const void* tele, void* p0,
                               void* z0, const int32_t* outdeg, PRState* st, double* slots, hipStream_t s);
// Warm restart: inputs 8..11 of every node v into Ft + v * ft_stride (four
// floats, 16-byte aligned) and, with p_star, the target into T, from the last
// four iterates and the states' residuals.
hipError_t launch_restart_inputs(const DevLayout& L, int prec, const void* pK, const void* pK1, const void* pK2,
                                 const void* pK3, const void* p_star, const PRState* st, float* Ft,
                                 int64_t ft_stride, float* T, hipStream_t s);
// Unnormalised restart vector q from p_K and the network output s; each
// member's sum of q ends in its state's delta field.
hipError_t launch_restart_vector(const DevLayout& L, int prec, const void* pK, const float* svec, PRState* st,
                                 void* q, double* slots, int members, hipStream_t s);

// ------------------------------------------------------------ left product
struct DevLeft {
  const LeftTile* lt = nullptr;
  const uint16_t* ent = nullptr;
  const uint16_t* grp = nullptr;
  const uint32_t* lanes = nullptr;
  void* part = nullptr;              // window contributions (row-sum type: double, or float for BVMV_F32)
  void* cbuf = nullptr;              // c of the rows of tiles with escapes (same type)
  const LeftEscape* esc = nullptr;
  const uint32_t* esc_off = nullptr;
  const uint32_t* cov_off = nullptr;
  const uint32_t* cov = nullptr;
  uint32_t n = 0;
};
// y = x A: the tiles' window contributions, then one gather per column
hipError_t launch_bv_left(const DevLayout& L, const DevLeft& D, int prec, const void* x, void* y, hipStream_t s);
size_t bv_left_lds_bytes(const DevLayout& L, int prec);

// ---------------------------------------------- allocation-free working set
// Bytes of the fixed device array that holds the working set of the
// allocation-free PageRank entry point (one copy per device, kept until the
// process ends): four iterate-sized vectors of up to 2^21 floats (2^20
// doubles) plus the block partials and the state.
constexpr size_t kNoAllocScratchBytes = (size_t(32) << 20) + (size_t(1) << 20);
// Device address of that array on `device`, which must be the current device;
// looked up once per device (hipGetSymbolAddress) and kept.
hipError_t noalloc_scratch(int device, void** ptr);
// *st = v by a one-thread kernel (no host-to-device copy)
hipError_t launch_pr_state_set(PRState* st, const PRState& v, hipStream_t s);

hipError_t launch_csr_multiply(const DevCsr& C, int prec, const void* x, void* y, hipStream_t s);
hipError_t launch_csr_pagerank_iter(const DevCsr& C, int prec, const PRArgs& a, hipStream_t s);
hipError_t launch_csr_pr_init(const DevCsr& C, int prec, const void* start, const void* tele, void* p0, void* z0,
                              const int32_t* outdeg, PRState* st, double* slots, hipStream_t s);

// rows [r0, r1) of p and z restored from the iterate src (z = src / d)
hipError_t launch_pr_restore(int prec, const void* src, void* p, void* z, const int32_t* outdeg, int64_t r0,
                             int64_t r1, hipStream_t s);
// out column c (column-major, ld = n) = the buffer (p0 or p1) holding column
// c's final iterate
hipError_t launch_pr_select(int prec, const PRState* st, const void* p0, const void* p1, void* out, int64_t n, int k,
                            hipStream_t s);


// ------------------------------------------------------------ learned warm start
constexpr int kMlpIn = 12, kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
constexpr int kMlpWeights = kMlpHidden * kMlpIn + kMlpHidden * kMlpHidden + kMlpHidden;  // BF16 copies
constexpr int64_t kMlpMaxBatch = 1 << 20; // feature rows per gradient call
// The network's inputs of node v: inputs 0..7 at s + v * ss, inputs 8..11 at
// t + v * ts (16-byte aligned rows).  The public n x 12 rows are {F, F + 8,
// 12, 12}; the learned restarts keep the two parts apart ({Fs, Ft, 8, 4}) so
// that each restart writes its four inputs as whole rows.
struct FeatIn {
  const float* s;
  const float* t;
  int64_t ss, ts;
};
__host__ __device__ inline FeatIn feat_rows12(const float* F) { return FeatIn{F, F + 8, 12, 12}; }
// s = MLP(inputs) for n nodes
hipError_t launch_mlp_forward(const float* theta, const uint16_t* wq, const FeatIn& in, int64_t n, float* s,
                              hipStream_t st);
// grad[0..kMlpParams) = gradient of the mean squared error, grad[kMlpParams] = the loss;
// part: one row of kMlpParams + 1 floats per 32 feature rows (ceil(n / 32) rows)
int mlp_grad_blocks(int64_t n);
hipError_t launch_mlp_gradient(const float* theta, const uint16_t* wq, const float* F, const float* target, int64_t n,
                               float* part, float* grad, hipStream_t st);
hipError_t launch_mlp_adam(float* theta, uint16_t* wq, float* m, float* v, const float* grad, float lr, float b1,
                           float b2, float eps, int step, hipStream_t st);
hipError_t launch_mlp_quantize(const float* theta, uint16_t* wq, hipStream_t st);
// product inputs of the structural features: d and indeg as floats
hipError_t launch_feature_inputs(int64_t n, const int32_t* indeg, const int32_t* outdeg, float* xd, float* xi,
                                 hipStream_t st);
// structural inputs 0..7 into F + v * stride (stride 12: columns 0..7 of the
// n x 12 rows; stride 8: rows of their own); yd = B d, yi = B indeg
hipError_t launch_features(int64_t n, const int32_t* indeg, const int32_t* outdeg, const uint32_t* stats,
                           const float* yd, const float* yi, float inv_r, float* F, int64_t stride, hipStream_t st);

}  // namespace bvmv
