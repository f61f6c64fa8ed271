// Kernels of the learned PageRank warm start, gfx950:
//   - per-node structural features (12 per node) from degrees, the stream's
//     row statistics and three products with the compressed graph;
//   - the MLP 12 -> 64 -> 64 -> 1 with GELU: forward and backward of both
//     hidden layers on MFMA (v_mfma_f32_32x32x16_bf16: BF16 operands, FP32
//     accumulation), biases, GELU and the output layer in FP32;
//   - deterministic reduction of per-wave gradient partials and Adam on FP32
//     master parameters with BF16 weight copies.
// The restart vector built from the network's output is written by
// restart_vector_kernel in bv_kernels.hip.
// The network's arithmetic is defined operand by operand in the CPU oracle
// (BF16 rounding, round to nearest even, of every operand that enters a
// matrix product; the output layer takes h2 unrounded).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace bvmv {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kNin = kMlpIn, kNh = kMlpHidden;
constexpr int oW1 = 0, oB1 = oW1 + kNh * kNin, oW2 = oB1 + kNh, oB2 = oW2 + kNh * kNh, oW3 = oB2 + kNh,
              oB3 = oW3 + kNh;
static_assert(oB3 + 1 == kMlpParams, "parameter layout");
// BF16 weight copies: W1, W2, w3 (the master layout without the biases)
constexpr int qW1 = 0, qW2 = qW1 + kNh * kNin, qW3 = qW2 + kNh * kNh;

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// gelu(z) = z s(1.702 z) with s the logistic function (the sigmoid form of
// GELU), and its derivative s + 1.702 z s (1 - s); one exponential and one
// reciprocal each (exp(-u) overflowing to +inf gives s = 0)
__device__ __forceinline__ float gelu_s(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-1.702f * z)); }
__device__ __forceinline__ float gelu(float z) { return z * gelu_s(z); }
__device__ __forceinline__ float gelu_grad(float z) {
  const float s = gelu_s(z);
  return s + 1.702f * z * s * (1.0f - s);
}

// One 32x32x16 product over two 8-wide K steps: D += A0 B0 + A1 B1.  A lane
// holds 8 K positions of its A row and the same 8 of its B column, so pairing
// the steps' operands the same way in A and B gives this sum whatever the
// hardware's order of K within the instruction.
__device__ __forceinline__ f16v mfma2(s4 a0, s4 a1, s4 b0, s4 b1, f16v c) {
  const s8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
  const s8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}

// four values rounded to BF16 (to nearest, ties to even: the same rounding
// as bf16_bits for finite values), two per conversion instruction
__device__ __forceinline__ s4 pack4(float a, float b, float c, float d) {
  const bf2v lo = __builtin_convertvector((f2v){a, b}, bf2v), hi = __builtin_convertvector((f2v){c, d}, bf2v);
  return __builtin_bit_cast(s4, (u2v){__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi)});
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Operands are built in 8-wide K steps (64 lanes, h = lane / 32):
//   A (32 x 8):  lane holds A[lane % 32][4h + e], e = 0..3;
//   B (8 x 32):  lane holds B[4h + e][lane % 32];
//   D (32 x 32): register v of a lane holds D[8 (v / 4) + 4h + v % 4][lane % 32],
// and two steps go to one 32x32x16 instruction (mfma2).  So the D registers
// 4s .. 4s+3 of a lane are, for its column, the rows 8s + 4h + e: exactly an
// A operand of a step whose K runs over those rows (used for the weight
// gradients, K = nodes).
__device__ __forceinline__ uint32_t drow(uint32_t v, uint32_t h) { return 8 * (v / 4) + 4 * h + (v % 4); }

constexpr int kSStride = 68;   // bf16 per row of the per-wave transpose buffer (8-byte aligned rows)
constexpr int kTStride = 33;   // floats per row of the output-layer buffer

struct alignas(16) WaveLds {
  uint16_t S[32 * kSStride];   // node x hidden, BF16
  float T[32 * kTStride];      // node x hidden slot, FP32
  float G[32];                 // per-node output gradient
};

// Forward of one 32-node tile by one wave, node-major (rows of each product
// are the tile's nodes), keeping what the backward pass needs.
struct Fwd {
  f16v z1[2], z2[2];   // pre-activations, D layout (rows = nodes, column = hidden % 32 of block b)
  s4 h1q[2][4];        // bf16(h1) as A/B operands over 8-node steps (D registers 4s..4s+3)
  float s;             // output of node lane % 32 (both halves)
};

// Inputs 4h .. 4h+3 and 8 + 4h .. 8 + 4h + 3 (zero past 11) of node
// node0 + lane % 32 (zero past n).
__device__ __forceinline__ void load_x_tile(const FeatIn& in, int64_t n, int64_t node0, s4 (&a1)[2]) {
  const uint32_t lane = lane_id(), h = lane >> 5;
  const int64_t node = node0 + (lane & 31);
  float x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (node < n) {
    const float4 lo = *reinterpret_cast<const float4*>(in.s + node * in.ss + 4 * h);
    x[0] = lo.x; x[1] = lo.y; x[2] = lo.z; x[3] = lo.w;
    if (h == 0) {
      const float4 hi = *reinterpret_cast<const float4*>(in.t + node * in.ts);
      x[4] = hi.x; x[5] = hi.y; x[6] = hi.z; x[7] = hi.w;
    }
  }
  a1[0] = pack4(x[0], x[1], x[2], x[3]);   // k = 4h + e
  a1[1] = pack4(x[4], x[5], x[6], x[7]);   // k = 8 + 4h + e (zero for h = 1: k >= 12)
}

// Weight operands of one wave: B[k][j] = W1[j][k] over 8-wide k steps (W2's
// are read from the block's LDS copy, row j = output unit, when needed).
struct FwdWeights {
  s4 b1[2][2];
  float bias1[2], bias2[2], w3[2], b3;
};

// W2 (bf16) into LDS, row j (output unit) at j * kSStride
__device__ __forceinline__ void stage_w2(const uint16_t* __restrict__ wq, uint16_t* s_w2) {
  for (uint32_t q = threadIdx.x; q < uint32_t(kNh * kNh); q += kThreads) s_w2[(q / kNh) * kSStride + q % kNh] = wq[qW2 + q];
  __syncthreads();
}

__device__ __forceinline__ void load_weights(const float* __restrict__ theta, const uint16_t* __restrict__ wq,
                                             FwdWeights& W) {
  const uint32_t lane = lane_id(), h = lane >> 5, c = lane & 31;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const uint32_t j = 32 * b + c;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t k = 8 * s + 4 * h + e;
        W.b1[b][s][e] = short(k < uint32_t(kNin) ? wq[qW1 + j * kNin + k] : 0);
      }
    W.bias1[b] = theta[oB1 + j];
    W.bias2[b] = theta[oB2 + j];
    W.w3[b] = bf16_float(wq[qW3 + j]);
  }
  W.b3 = theta[oB3];
}

__device__ __forceinline__ void forward_tile(const FeatIn& in, int64_t n, int64_t node0, const FwdWeights& W,
                                             const uint16_t* s_w2, WaveLds& L, Fwd& o) {
  const uint32_t lane = lane_id(), h = lane >> 5, c = lane & 31;
  s4 a1[2];
  load_x_tile(in, n, node0, a1);
  const f16v zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // layer 1: z1 = W1 bf(x) + b1, h1 = gelu(z1)
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    f16v d = mfma2(a1[0], a1[1], W.b1[b][0], W.b1[b][1], zero);
#pragma unroll
    for (int v = 0; v < 16; ++v) d[v] += W.bias1[b];
    o.z1[b] = d;
    float hv[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) hv[v] = gelu(d[v]);
#pragma unroll
    for (int s = 0; s < 4; ++s) o.h1q[b][s] = pack4(hv[4 * s], hv[4 * s + 1], hv[4 * s + 2], hv[4 * s + 3]);
    // transpose to the A layout of layer 2 (node x hidden)
#pragma unroll
    for (int v = 0; v < 16; ++v) L.S[drow(v, h) * kSStride + 32 * b + c] = uint16_t(o.h1q[b][v / 4][v % 4]);
  }
  wave_sync();
  s4 a2[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) a2[s] = *reinterpret_cast<const s4*>(&L.S[c * kSStride + 8 * s + 4 * h]);
  // layer 2: z2 = W2 bf(h1) + b2, h2 = gelu(z2)
  float part[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) part[v] = 0.0f;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    f16v d = zero;
#pragma unroll
    for (int s = 0; s < 8; s += 2)  // B[k][j] = W2[j][k], k = 8s + 4h + e, j = 32b + lane % 32
      d = mfma2(a2[s], a2[s + 1], *reinterpret_cast<const s4*>(&s_w2[(32 * b + c) * kSStride + 8 * s + 4 * h]),
                *reinterpret_cast<const s4*>(&s_w2[(32 * b + c) * kSStride + 8 * s + 8 + 4 * h]), d);
#pragma unroll
    for (int v = 0; v < 16; ++v) d[v] += W.bias2[b];
    o.z2[b] = d;
#pragma unroll
    for (int v = 0; v < 16; ++v) part[v] += gelu(d[v]) * W.w3[b];
  }
  // output layer: s = w3 . h2 + b3, the hidden sum over the 32 lanes of a half
#pragma unroll
  for (int v = 0; v < 16; ++v) L.T[drow(v, h) * kTStride + c] = part[v];
  wave_sync();
  float acc = 0.0f;
#pragma unroll
  for (int t = 0; t < 16; ++t) acc += L.T[c * kTStride + 16 * h + t];
  acc += __shfl_xor(acc, 32, 64);
  o.s = acc + W.b3;
  wave_sync();  // L is reused by the next tile
}

// ------------------------------------------------------------------ forward
// Inference, one 32-node tile per wave and turn, in the transposed form: the
// hidden units are the rows of each product and the tile's nodes its columns,
//   layer 1: z1' (64 x 32) = W1 x',        A = rows of W1, B = x' (inputs x nodes)
//   layer 2: z2' (64 x 32) = W2 bf(h1)',   A = rows of W2, B = bf(h1)'
// so that the D registers 4s .. 4s+3 of layer 1's block s / 4 are, for the
// lane's node, hidden units 8s + 4h + e: layer 2's B operand of step s, with
// no transpose through LDS.  Register v of block b holds unit 32b + drow(v, h);
// the output layer sums the lane's 32 units and the other half's.  The
// arithmetic is the node-major form's (the same operands and roundings).
// The pass is bound by the GELUs' VALU issue, so it asks for at least five
// waves per SIMD (the accumulators then stay in VGPRs: 77 registers, six
// waves, no spills).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) mlp_forward_kernel(const float* __restrict__ theta,
                                                               const uint16_t* __restrict__ wq, FeatIn in, int64_t n,
                                                               float* __restrict__ out) {
  __shared__ __align__(16) uint16_t s_w2[kNh * kSStride];
  __shared__ __align__(16) float s_c[3 * kNh];  // b1, b2, and w3 as its BF16 value
  for (uint32_t q = threadIdx.x; q < uint32_t(kNh); q += kThreads) {
    s_c[q] = theta[oB1 + q];
    s_c[kNh + q] = theta[oB2 + q];
    s_c[2 * kNh + q] = bf16_float(wq[qW3 + q]);
  }
  stage_w2(wq, s_w2);  // (ends with a block barrier)
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id(), h = lane >> 5, c = lane & 31;
  FwdWeights W;
  load_weights(theta, wq, W);
  const f16v zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t ntiles = (n + 31) / 32;
  const int64_t stride = int64_t(gridDim.x) * (kThreads / 64);
  for (int64_t t = int64_t(blockIdx.x) * (kThreads / 64) + wave; t < ntiles; t += stride) {
    // zero (t < 2^40), but not known to the compiler: the LDS operands below
    // are read once per tile instead of being held in registers for the loop
    const uint32_t z = uint32_t(t >> 40);
    s4 a1[2];
    load_x_tile(in, n, t * 32, a1);
    // layer 1: h1 = gelu(W1 x + b1), rounded to BF16
    s4 h1q[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      f16v d = mfma2(W.b1[b][0], W.b1[b][1], a1[0], a1[1], zero);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 bb = *reinterpret_cast<const float4*>(&s_c[z + 32 * b + 8 * q + 4 * h]);
        h1q[b][q] = pack4(gelu(d[4 * q] + bb.x), gelu(d[4 * q + 1] + bb.y), gelu(d[4 * q + 2] + bb.z),
                          gelu(d[4 * q + 3] + bb.w));
      }
    }
    // layer 2 and the output layer: s = w3 . gelu(W2 bf(h1) + b2) + b3
    float part = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      f16v d = zero;
#pragma unroll
      for (int s = 0; s < 8; s += 2)  // A[j][k] = W2[j][k], j = 32b + lane % 32, k = 8s + 4h + e
        d = mfma2(*reinterpret_cast<const s4*>(&s_w2[z + (32 * b + c) * kSStride + 8 * s + 4 * h]),
                  *reinterpret_cast<const s4*>(&s_w2[z + (32 * b + c) * kSStride + 8 * s + 8 + 4 * h]),
                  h1q[s / 4][s % 4], h1q[s / 4][s % 4 + 1], d);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 bb = *reinterpret_cast<const float4*>(&s_c[z + kNh + 32 * b + 8 * q + 4 * h]);
        const float4 ww = *reinterpret_cast<const float4*>(&s_c[z + 2 * kNh + 32 * b + 8 * q + 4 * h]);
        part += gelu(d[4 * q] + bb.x) * ww.x;
        part += gelu(d[4 * q + 1] + bb.y) * ww.y;
        part += gelu(d[4 * q + 2] + bb.z) * ww.z;
        part += gelu(d[4 * q + 3] + bb.w) * ww.w;
      }
    }
    part += __shfl_xor(part, 32, 64);
    const int64_t node = t * 32 + c;
    if (lane < 32 && node < n) out[node] = part + W.b3;
  }
}

// ----------------------------------------------------------------- backward
// One wave per 32-node tile t: the tile's contribution to the gradient of
// sum_i (s_i - t_i)^2 / n, into row t of `part` (kMlpParams + 1 floats: the
// gradient, then the tile's share of the loss).  Each weight-gradient block
// is stored as soon as its products are done, so no accumulator outlives it.
__global__ void __launch_bounds__(kThreads) mlp_backward_kernel(const float* __restrict__ theta,
                                                                const uint16_t* __restrict__ wq,
                                                                const float* __restrict__ F,
                                                                const float* __restrict__ target, int64_t n,
                                                                float* __restrict__ part) {
  __shared__ WaveLds lds[kThreads / 64];
  __shared__ __align__(16) uint16_t s_w2[kNh * kSStride];  // W2 (bf16), row j = output unit
  stage_w2(wq, s_w2);
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id(), h = lane >> 5, c = lane & 31;
  const int64_t ntiles = (n + 31) / 32;
  const int64_t t = int64_t(blockIdx.x) * (kThreads / 64) + wave;
  if (t >= ntiles) return;
  WaveLds& L = lds[wave];
  FwdWeights W;
  load_weights(theta, wq, W);
  const f16v zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  float* out = part + size_t(t) * (kMlpParams + 1);
  const float inv_n = 1.0f / float(n);
  const int64_t node0 = t * 32;
  Fwd o;
  forward_tile(feat_rows12(F), n, node0, W, s_w2, L, o);
  // output gradient g_i = 2 (s_i - t_i) / n of node i = lane % 32
  const int64_t node = node0 + c;
  float gi = 0.0f, lsum = 0.0f;
  if (node < n) {
    const float r = o.s - target[node];
    gi = 2.0f * r * inv_n;
    lsum = h == 0 ? r * r : 0.0f;
  }
  if (h == 0) L.G[c] = gi;
  wave_sync();
  float gv[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) gv[v] = L.G[drow(v, h)];
  // layer 2: dz2 = g w3 gelu'(z2); dw3 = sum g h2 (h2 recomputed); db2 = sum dz2.
  // bf(dz2) is the A operand of dW2 = bf(dz2)^T bf(h1) (K = the tile's nodes,
  // D registers as operands), and goes transposed to node x hidden in S for dh1.
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    s4 dq[4];
    float gw3 = 0.0f, gb2 = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float z = o.z2[bj][v];
      gw3 += gv[v] * gelu(z);
      const float d = gv[v] * W.w3[bj] * gelu_grad(z);
      gb2 += d;
      dq[v / 4][v % 4] = short(bf16_bits(d));
    }
    gw3 += __shfl_xor(gw3, 32, 64);
    gb2 += __shfl_xor(gb2, 32, 64);
    if (h == 0) {
      out[oW3 + 32 * bj + c] = gw3;
      out[oB2 + 32 * bj + c] = gb2;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) L.S[drow(v, h) * kSStride + 32 * bj + c] = uint16_t(dq[v / 4][v % 4]);
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) {
      f16v gw = zero;
#pragma unroll
      for (int s = 0; s < 4; s += 2) gw = mfma2(dq[s], dq[s + 1], o.h1q[bk][s], o.h1q[bk][s + 1], gw);
#pragma unroll
      for (int v = 0; v < 16; ++v) out[oW2 + (32 * bj + drow(v, h)) * kNh + 32 * bk + c] = gw[v];
    }
  }
  wave_sync();
  // dh1 = bf(dz2) W2, dz1 = dh1 gelu'(z1), db1 = sum dz1, dW1 = bf(dz1)^T bf(x)
  s4 a2[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) a2[s] = *reinterpret_cast<const s4*>(&L.S[c * kSStride + 8 * s + 4 * h]);
  s4 bx[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    float xv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t nd = node0 + 8 * s + 4 * h + e;
      xv[e] = (nd < n && c < uint32_t(kNin)) ? F[nd * kNin + c] : 0.0f;
    }
    bx[s] = pack4(xv[0], xv[1], xv[2], xv[3]);
  }
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    f16v d = zero;
#pragma unroll
    for (int s = 0; s < 8; s += 2) {
      s4 bw[2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) bw[u][e] = short(s_w2[(8 * (s + u) + 4 * h + e) * kSStride + 32 * bk + c]);
      d = mfma2(a2[s], a2[s + 1], bw[0], bw[1], d);
    }
    s4 dq[4];
    float gb1 = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float dz = d[v] * gelu_grad(o.z1[bk][v]);
      gb1 += dz;
      dq[v / 4][v % 4] = short(bf16_bits(dz));
    }
    gb1 += __shfl_xor(gb1, 32, 64);
    if (h == 0) out[oB1 + 32 * bk + c] = gb1;
    f16v gw = zero;
#pragma unroll
    for (int s = 0; s < 4; s += 2) gw = mfma2(dq[s], dq[s + 1], bx[s], bx[s + 1], gw);
    if (c < uint32_t(kNin))
#pragma unroll
      for (int v = 0; v < 16; ++v) out[oW1 + (32 * bk + drow(v, h)) * kNin + c] = gw[v];
  }
  // b3 and the loss: sums over the 32 nodes (first half of the lanes)
  float gb3 = h == 0 ? gi : 0.0f;
#pragma unroll
  for (int d = 16; d >= 1; d >>= 1) {
    gb3 += __shfl_xor(gb3, d, 64);
    lsum += __shfl_xor(lsum, d, 64);
  }
  if (lane == 0) {
    out[oB3] = gb3;
    out[kMlpParams] = lsum * inv_n;
  }
}

// grad[p] = sum over the tiles' partials in tile order (deterministic)
__global__ void __launch_bounds__(kThreads) mlp_reduce_kernel(const float* __restrict__ part, int nparts,
                                                              float* __restrict__ grad) {
  const int p = int(blockIdx.x) * kThreads + int(threadIdx.x);
  if (p > kMlpParams) return;
  float s = 0.0f;
  for (int w = 0; w < nparts; ++w) s += part[size_t(w) * (kMlpParams + 1) + p];
  grad[p] = s;
}

// Adam on the FP32 master parameters; the BF16 copies of the weights follow.
__global__ void __launch_bounds__(kThreads) mlp_adam_kernel(float* __restrict__ theta, uint16_t* __restrict__ wq,
                                                            float* __restrict__ m, float* __restrict__ v,
                                                            const float* __restrict__ grad, float lr, float b1,
                                                            float b2, float eps, float c1, float c2) {
  const int p = int(blockIdx.x) * kThreads + int(threadIdx.x);
  if (p >= kMlpParams) return;
  const float g = grad[p];
  const float mp = b1 * m[p] + (1.0f - b1) * g;
  const float vp = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mp;
  v[p] = vp;
  const float th = theta[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
  theta[p] = th;
  int q = -1;
  if (p < oB1) q = qW1 + p;
  else if (p >= oW2 && p < oB2) q = qW2 + (p - oW2);
  else if (p >= oW3 && p < oB3) q = qW3 + (p - oW3);
  if (q >= 0) wq[q] = bf16_bits(th);
}

__global__ void __launch_bounds__(kThreads) mlp_quantize_kernel(const float* __restrict__ theta,
                                                                uint16_t* __restrict__ wq) {
  const int p = int(blockIdx.x) * kThreads + int(threadIdx.x);
  if (p < oB1) wq[qW1 + p] = bf16_bits(theta[p]);
  else if (p >= oW2 && p < oB2) wq[qW2 + (p - oW2)] = bf16_bits(theta[p]);
  else if (p >= oW3 && p < oB3) wq[qW3 + (p - oW3)] = bf16_bits(theta[p]);
}

// ------------------------------------------------------- structural inputs
// Columns 0..7 of node v's input row: log1p(indeg), log1p(d), depth / R,
// [d = 0], log1p(intervals), log1p(residuals), log1p(B d / max(indeg, 1)),
// log1p(B indeg / max(indeg, 1)).  stats holds 5 u32 per row: depth, skipped
// reference entries, intervals, interval length, residuals.
__global__ void __launch_bounds__(kThreads) features_kernel(int64_t n, const int32_t* __restrict__ indeg,
                                                            const int32_t* __restrict__ outdeg,
                                                            const uint32_t* __restrict__ stats,
                                                            const float* __restrict__ yd,
                                                            const float* __restrict__ yi, float inv_r,
                                                            float* __restrict__ F, int64_t stride) {
  for (int64_t v = int64_t(blockIdx.x) * kThreads + threadIdx.x; v < n; v += int64_t(gridDim.x) * kThreads) {
    const float ind = float(indeg[v]), d = float(outdeg[v]);
    const float den = fmaxf(ind, 1.0f);
    const uint32_t* st = stats + 5 * v;
    float* f = F + v * stride;
    f[0] = log1pf(ind);
    f[1] = log1pf(d);
    f[2] = float(st[0]) * inv_r;
    f[3] = d == 0.0f ? 1.0f : 0.0f;
    f[4] = log1pf(float(st[2]));
    f[5] = log1pf(float(st[4]));
    f[6] = log1pf(yd[v] / den);
    f[7] = log1pf(yi[v] / den);
  }
}

// product inputs of the structural features: d and indeg as floats
__global__ void __launch_bounds__(kThreads) feature_inputs_kernel(int64_t n, const int32_t* __restrict__ indeg,
                                                                  const int32_t* __restrict__ outdeg,
                                                                  float* __restrict__ xd, float* __restrict__ xi) {
  for (int64_t v = int64_t(blockIdx.x) * kThreads + threadIdx.x; v < n; v += int64_t(gridDim.x) * kThreads) {
    xd[v] = float(outdeg[v]);
    xi[v] = float(indeg[v]);
  }
}

int grid_for(int64_t items, int cap) { return int(std::max<int64_t>(1, std::min<int64_t>((items + kThreads - 1) / kThreads, cap))); }

}  // namespace

hipError_t launch_mlp_forward(const float* theta, const uint16_t* wq, const FeatIn& in, int64_t n, float* s,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (((reinterpret_cast<uintptr_t>(in.s) | reinterpret_cast<uintptr_t>(in.t) | uintptr_t(in.ss) * 4 |
        uintptr_t(in.ts) * 4) & 15) || in.ss < 8 || in.ts < 4)
    return hipErrorInvalidValue;
  const int64_t tiles = (n + 31) / 32;
  const int blocks = int(std::min<int64_t>((tiles + 3) / 4, 4096));
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(kThreads), 0, st, theta, wq, in, n, s);
  return hipGetLastError();
}

int mlp_grad_blocks(int64_t n) { return int(((n + 31) / 32 + 3) / 4); }

hipError_t launch_mlp_gradient(const float* theta, const uint16_t* wq, const float* F, const float* target, int64_t n,
                               float* part, float* grad, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  const int blocks = mlp_grad_blocks(n);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(blocks), dim3(kThreads), 0, st, theta, wq, F, target, n, part);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     part, int((n + 31) / 32), grad);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* theta, uint16_t* wq, float* m, float* v, const float* grad, float lr, float b1,
                           float b2, float eps, int step, hipStream_t st) {
  const float c1 = 1.0f - std::pow(b1, float(step)), c2 = 1.0f - std::pow(b2, float(step));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + kThreads - 1) / kThreads), dim3(kThreads), 0, st, theta,
                     wq, m, v, grad, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_quantize(const float* theta, uint16_t* wq, hipStream_t st) {
  hipLaunchKernelGGL(mlp_quantize_kernel, dim3((kMlpParams + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     theta, wq);
  return hipGetLastError();
}

hipError_t launch_feature_inputs(int64_t n, const int32_t* indeg, const int32_t* outdeg, float* xd, float* xi,
                                 hipStream_t st) {
  hipLaunchKernelGGL(feature_inputs_kernel, dim3(grid_for(n, 4096)), dim3(kThreads), 0, st, n, indeg, outdeg, xd,
                     xi);
  return hipGetLastError();
}

hipError_t launch_features(int64_t n, const int32_t* indeg, const int32_t* outdeg, const uint32_t* stats,
                           const float* yd, const float* yi, float inv_r, float* F, int64_t stride, hipStream_t st) {
  hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, 4096)), dim3(kThreads), 0, st, n, indeg, outdeg, stats, yd,
                     yi, inv_r, F, stride);
  return hipGetLastError();
}

}  // namespace bvmv
