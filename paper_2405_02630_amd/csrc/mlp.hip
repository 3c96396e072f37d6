// Kernels of the learned surrogate: an MLP embedding f (BF16 weights and
// activations, FP32 accumulation on the matrix cores) whose inner products
// stand in for kernel entries, either in the log domain through the squared
// distance of the embeddings [x, f(x)], ln K_hat = -c (1 - exp(-s d2)), or as
// K_hat(x, y) = sigmoid(alpha <f(x), f(y)> + beta).
//
// * bf16_gemm_dl<MT, WN, BK, EPI>: the same product for k-contiguous
//   operands on 256 x 256 (8 waves, 64-deep K steps), 256 x 128 or 128 x 128
//   tiles, operands moved global -> LDS by the DMA loads
//   (global_load_lds_dwordx4), double-buffered; used whenever M and N are
//   multiples of 128 (the forward layers and the activation gradients).
// * bf16_gemm<TA, TB, EPI>: C = op(A) op(B) on v_mfma_f32_32x32x16_bf16.
//   A 64 x 64 output tile per block of 4 waves (each wave one 32 x 32
//   accumulator), K in steps of 64 staged through LDS with both operands
//   stored k-contiguous so every lane reads its 8 k-values as one 16-byte
//   LDS load.  Dimensions are multiples of the tile (the host pads), so no
//   bounds checks are needed.  Fused epilogues: FP32 store; bias + GELU
//   (keeps the pre-activation for the backward pass); bias + FP32/BF16 store;
//   multiply by GELU'(pre-activation) (backward through the activation).
// * sigmoid_gram_kernel: K_hat of all pairs, FP64, with per-tile maxima of
//   the off-diagonal entries (write-bound; 128 x 64 blocks, non-temporal
//   stores).
// * gather_features: FP64 feature rows -> zero-padded BF16 rows.
// * transpose_bf16: the forward pass's k-contiguous copy of each weight.
// * transpose64_bf16, sum_slabs: the weight gradients' operands
//   copied k-contiguous (the activations with a row of ones appended, whose
//   product row is the bias gradient) and the fixed-order reduction of their
//   split-K partial products.
// * pair_head: per pair, K_hat, the loss (squared error or soft-target
//   cross-entropy) and its gradient w.r.t. both embeddings, alpha and beta;
//   per-pair partial sums reduced in a fixed order.
// * pair_head_log, sat_log_gram_kernel: the log-domain head
//   ln K_hat = -c (1 - exp(-s d2)) on the squared distance of the embeddings
//   [x, f(x)] (loss and gradients per pair; the whole Gram with per-tile
//   maxima of ln K_hat).
// * adamw: decoupled-weight-decay Adam on FP32 master weights, BF16 copy.
// * flag_pairs_kernel: lists the pairs of flagged tiles whose K_hat reaches
//   the fallback threshold (tiles with many go to a dense tile list).
// * flag_tiles: compacts the tiles whose largest off-diagonal K_hat reaches
//   the fallback threshold.
//
// GELU is the exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2, with Phi
// evaluated to a relative error near 1e-7 (normal_cdf).

#include <hip/hip_runtime.h>

#include <atomic>
#include <math.h>
#include <stdint.h>

#include "mlp.h"

namespace qsvm {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDS_STRIDE = BK + 8;  // bf16 elements per LDS row (16-byte pad)
constexpr int GBK = 64;                   // K step of bf16_gemm
constexpr int GEMM_LDS_STRIDE = GBK + 8;  // its LDS row, 16-byte pad

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// Round to nearest even through the hardware conversion (v_cvt_pk_bf16_f32,
// two values per instruction in bf16_pair).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// Standard normal CDF Phi(x) without branches, through the complementary
// error function of Numerical Recipes (Press et al., "erfcc": a Chebyshev
// fit with fractional error below 1.2e-7 for every z >= 0):
// Phi(x) = 1 - erfc(z)/2 for x >= 0 and erfc(z)/2 for x < 0, z = |x|/sqrt 2.
// Every lane takes the same instructions, so a GEMM epilogue over mixed-sign
// pre-activations does not run both sides of a branch.
__device__ __forceinline__ float normal_cdf(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));  // 1 ulp
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  const float h = 0.5f * t * __expf(fmaf(-z, z, p));  // erfc(z) / 2
  return (x >= 0.0f) ? 1.0f - h : h;
}

// GELU x Phi(x) written as max(x, 0) - |x| Q(|x|) with the normal tail
// Q(u) = Phi(-u) = exp2(R(min(u, 6)) - k u): R(v) = log2 Q(v) + k v is a
// degree-8 polynomial (Chebyshev least-squares fit on [0, 6], refitted to the
// power basis) and k = 8.884812 is the slope of -log2 Q at u = 6, so the tail
// beyond 6 continues as the tangent of log2 Q there.  Once the argument of
// exp2 is rounded to FP32 the result's relative error stays below 5e-6
// wherever |GELU| > 1e-8, and below that its absolute error below 5e-11.
// One transcendental and no reciprocal or select: the forward epilogues are
// bound by these instructions.
__device__ __forceinline__ float gelu(float x) {
  const float u = fabsf(x), v = fminf(u, 6.0f);
  float p = -7.983291e-09f;
  p = fmaf(p, v, -1.6980216e-06f);
  p = fmaf(p, v, 6.081319e-05f);
  p = fmaf(p, v, -0.00092938275f);
  p = fmaf(p, v, 0.008512783f);
  p = fmaf(p, v, -0.053979937f);
  p = fmaf(p, v, -0.45844033f);
  p = fmaf(p, v, 7.733552f);
  p = fmaf(p, v, -0.99999475f);
  const float q = __builtin_amdgcn_exp2f(fmaf(u, -8.884812f, p));
  return fmaf(-u, q, fmaxf(x, 0.0f));
}

__device__ __forceinline__ float gelu_grad(float x) {
  const float pdf = 0.39894228040143268f * __expf(-0.5f * x * x);
  return normal_cdf(x) + x * pdf;
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Piece p (0..511) of a 64 x 64 step tile of an operand whose rows r0.. pair
// with K values k0..: 8 consecutive bf16, 8 pieces per row.  KMAJ = 0: the
// source is k-contiguous (M[r * ld + k]), piece p = row p / 8, k (p % 8) * 8;
// KMAJ = 1: the source is r-contiguous (M[k * ld + r]), piece p = k p / 8,
// rows (p % 8) * 8.  The LDS tile is [row][k] with row stride GEMM_LDS_STRIDE.
template <int KMAJ>
__device__ __forceinline__ uint4 load_piece(const uint16_t* __restrict__ M, int64_t ld, int64_t r0, int64_t k0, int p) {
  if (KMAJ == 0) return *reinterpret_cast<const uint4*>(M + (r0 + (p >> 3)) * ld + k0 + (p & 7) * 8);
  return *reinterpret_cast<const uint4*>(M + (k0 + (p >> 3)) * ld + r0 + (p & 7) * 8);
}

template <int KMAJ>
__device__ __forceinline__ void stash_piece(uint16_t* S, uint4 v, int p) {
  const int a = p >> 3, b = (p & 7) * 8;
  if (KMAJ == 0) {
    *reinterpret_cast<uint4*>(&S[a * GEMM_LDS_STRIDE + b]) = v;
  } else {  // a = k, b = first row: transpose into [row][k]
    S[(b + 0) * GEMM_LDS_STRIDE + a] = uint16_t(v.x);
    S[(b + 1) * GEMM_LDS_STRIDE + a] = uint16_t(v.x >> 16);
    S[(b + 2) * GEMM_LDS_STRIDE + a] = uint16_t(v.y);
    S[(b + 3) * GEMM_LDS_STRIDE + a] = uint16_t(v.y >> 16);
    S[(b + 4) * GEMM_LDS_STRIDE + a] = uint16_t(v.z);
    S[(b + 5) * GEMM_LDS_STRIDE + a] = uint16_t(v.z >> 16);
    S[(b + 6) * GEMM_LDS_STRIDE + a] = uint16_t(v.w);
    S[(b + 7) * GEMM_LDS_STRIDE + a] = uint16_t(v.w >> 16);
  }
}

// op(A)[m][k]: TA = 0 -> A[m*lda + k]; TA = 1 -> A[k*lda + m].
// op(B)[k][n]: TB = 0 -> B[k*ldb + n]; TB = 1 -> B[n*ldb + k].
// The K loop moves GBK = 64 values per step; the next step's operands are
// loaded into registers while the current step's MFMAs run, so each block
// keeps a step of loads in flight (the blocks are otherwise latency-bound:
// 8 per compute unit, a few MFMAs per step).
template <int TA, int TB, int EPI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) bf16_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * GEMM_LDS_STRIDE];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * GEMM_LDS_STRIDE];  // [n][k]
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // XCD-aware tile order: blocks are dealt to the 8 XCDs round-robin, so when
  // the tile count allows, XCD x takes the x-th contiguous range of tiles and
  // the column tiles of one row tile share that XCD's L2 copy of the A rows.
  const uint32_t nx = gridDim.x, tiles = gridDim.x * gridDim.y;
  uint32_t u = blockIdx.y * nx + blockIdx.x;
  if ((tiles & 7u) == 0) u = (u & 7u) * (tiles >> 3) + (u >> 3);
  const int64_t m0 = int64_t(u / nx) * BM;
  const int64_t n0 = int64_t(u % nx) * BN;
  const uint16_t* __restrict__ A = static_cast<const uint16_t*>(g.A);
  const uint16_t* __restrict__ B = static_cast<const uint16_t*>(g.B);

  f32x16_t acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;

  // Each thread moves two 16-byte pieces of each operand per step (pieces
  // t and t + 256 of the 64 x 64 step tile; see load_piece / stash_piece).
  uint4 ra0, ra1, rb0, rb1;
  // split-K: block z covers K range [z K / splits, (z + 1) K / splits)
  const int64_t kspan = g.K / g.splits;
  const int64_t kbeg = int64_t(blockIdx.z) * kspan;
  const int64_t kend = kbeg + kspan;
  ra0 = load_piece<TA>(A, g.lda, m0, kbeg, t);
  ra1 = load_piece<TA>(A, g.lda, m0, kbeg, t + 256);
  rb0 = load_piece<1 - TB>(B, g.ldb, n0, kbeg, t);
  rb1 = load_piece<1 - TB>(B, g.ldb, n0, kbeg, t + 256);
  for (int64_t k0 = kbeg; k0 < kend; k0 += GBK) {
    stash_piece<TA>(As, ra0, t);
    stash_piece<TA>(As, ra1, t + 256);
    stash_piece<1 - TB>(Bs, rb0, t);
    stash_piece<1 - TB>(Bs, rb1, t + 256);
    __syncthreads();
    if (k0 + GBK < kend) {  // the next step's operands, in flight during this step's MFMAs
      ra0 = load_piece<TA>(A, g.lda, m0, k0 + GBK, t);
      ra1 = load_piece<TA>(A, g.lda, m0, k0 + GBK, t + 256);
      rb0 = load_piece<1 - TB>(B, g.ldb, n0, k0 + GBK, t);
      rb1 = load_piece<1 - TB>(B, g.ldb, n0, k0 + GBK, t + 256);
    }
    const int i = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 16) {
      const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&As[(wm * 32 + i) * GEMM_LDS_STRIDE + ks + kh * 8]);
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(&Bs[(wn * 32 + i) * GEMM_LDS_STRIDE + ks + kh * 8]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- epilogue: element v of the accumulator is row i, column j ----
  const int j = lane & 31;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
    const int64_t r = m0 + wm * 32 + i;
    const int64_t c = n0 + wn * 32 + j;
    const float x = acc[v];
    if (EPI == EPI_F32) {
      static_cast<float*>(g.C)[int64_t(blockIdx.z) * g.M * g.ldc + r * g.ldc + c] = x;
    } else if (EPI == EPI_BIAS_GELU) {
      const float h = x + g.bias[c];
      static_cast<float*>(g.C)[r * g.ldc + c] = h;
      static_cast<uint16_t*>(g.C2)[r * g.ldc + c] = f32_to_bf16(gelu(h));
    } else if (EPI == EPI_BIAS) {
      const float h = x + g.bias[c];
      static_cast<float*>(g.C)[r * g.ldc + c] = h;
      static_cast<uint16_t*>(g.C2)[r * g.ldc + c] = f32_to_bf16(h);
    } else if (EPI == EPI_GELU_BWD) {
      const float d = x * gelu_grad(g.aux[r * g.ldc + c]);
      static_cast<uint16_t*>(g.C2)[r * g.ldc + c] = f32_to_bf16(d);
    } else if (EPI == EPI_BIAS_GELU_BF16) {
      static_cast<uint16_t*>(g.C2)[r * g.ldc + c] = f32_to_bf16(gelu(x + g.bias[c]));
    } else if (EPI == EPI_BIAS_BF16) {
      static_cast<uint16_t*>(g.C2)[r * g.ldc + c] = f32_to_bf16(x + g.bias[c]);
    }
  }
}

// C = A B^T-style GEMM with both operands k-contiguous (A[m*lda + k],
// op(B)[k][n] = B[n*ldb + k]) on (64 MT) x (64 WN) output tiles: 2 WN waves
// in a 2 x WN grid, each wave (32 MT) x 64 = MT x 2 accumulators of
// v_mfma_f32_32x32x16_bf16.  Three shapes are launched: MT = 2, WN = 2
// (128 x 128, 4 waves; 64-deep K steps in 64 KB of LDS when the grid puts at
// most two blocks on a compute unit), MT = 4, WN = 2 (256 x 128: half the
// LDS bytes per MFMA) and MT = 4, WN = 4 (256 x 256, 8 waves, one block per
// compute unit, 64-deep K steps in 128 KB of LDS: a third less DMA into LDS
// per MFMA and half the barriers).  The operands reach LDS without passing through
// registers: each wave issues global_load_lds_dwordx4 for 1 KB chunks of the
// next BK-deep K step while the current step's MFMAs run (two LDS buffers,
// one barrier per step).  A DMA chunk is 64 consecutive 16-byte LDS slots;
// slot s of a tile holds row s / PR, 16-byte piece (s % PR) ^ sw(row) of that
// row's BK k-values (PR = BK / 8), the XOR swizzle keeping every 16-lane
// group of a fragment read on distinct LDS banks: for PR = 4
// sw(row) = ((row >> 1) ^ (row >> 3)) & 1 | (row >> 1) & 2, for PR = 8
// sw(row) = (row ^ (row >> 3)) & 7.  Waits are explicit (vmcnt for this
// wave's DMA, then a plain barrier): a fenced barrier would also wait for
// the step being prefetched.  M must be a multiple of 64 MT, N of 64 WN,
// K / splits of BK, lda and ldb of 8; the epilogues are those of bf16_gemm.
constexpr int DL_BK = 32;      // K step
constexpr int DL_PR = DL_BK / 8;  // 16-byte pieces per tile row and step

__device__ __forceinline__ int dl_swizzle(int row) { return (((row >> 1) ^ (row >> 3)) & 1) | ((row >> 1) & 2); }

template <int PR>
__device__ __forceinline__ int dl_swz(int row) {
  static_assert(PR == 4 || PR == 8, "16-byte pieces per row: 4 or 8");
  if constexpr (PR == 4) return dl_swizzle(row);
  else return (row ^ (row >> 3)) & 7;
}

// Epilogue of one 32 x 32 accumulator whose top-left output is (r0, c0):
// element v is row r0 + (v/4)*8 + (lane/32)*4 + v%4, column c0 + lane%32.
// Elements v and v + 1 (rows r and r + 1) share one BF16 conversion.
template <int EPI>
__device__ __forceinline__ void gemm_store32(const GemmArgs& g, const f32x16_t& acc, int64_t r0, int64_t c0, int lane) {
  const int64_t c = c0 + (lane & 31);
  float* const Cf = static_cast<float*>(g.C);
  uint16_t* const C2 = static_cast<uint16_t*>(g.C2);
  const bool has_bias = EPI == EPI_BIAS_GELU || EPI == EPI_BIAS || EPI == EPI_BIAS_GELU_BF16 || EPI == EPI_BIAS_BF16;
  const float bc = has_bias ? g.bias[c] : 0.0f;
#pragma unroll
  for (int v = 0; v < 16; v += 2) {
    const int64_t r = r0 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
    const int64_t o0 = r * g.ldc + c, o1 = o0 + g.ldc;
    const float x0 = acc[v], x1 = acc[v + 1];
    uint32_t q = 0;
    if (EPI == EPI_F32) {
      const int64_t z = int64_t(blockIdx.z) * g.M * g.ldc;
      Cf[z + o0] = x0;
      Cf[z + o1] = x1;
      continue;
    } else if (EPI == EPI_BIAS) {
      const float h0 = x0 + bc, h1 = x1 + bc;
      Cf[o0] = h0;
      C2[o0] = f32_to_bf16(h0);
      Cf[o1] = h1;
      C2[o1] = f32_to_bf16(h1);
      continue;
    } else if (EPI == EPI_BIAS_GELU) {
      const float h0 = x0 + bc, h1 = x1 + bc;
      q = bf16_pair(gelu(h0), gelu(h1));
      Cf[o0] = h0;
      Cf[o1] = h1;
    } else if (EPI == EPI_GELU_BWD) {
      q = bf16_pair(x0 * gelu_grad(g.aux[o0]), x1 * gelu_grad(g.aux[o1]));
    } else if (EPI == EPI_BIAS_GELU_BF16) {
      q = bf16_pair(gelu(x0 + bc), gelu(x1 + bc));
    } else if (EPI == EPI_BIAS_BF16) {
      q = bf16_pair(x0 + bc, x1 + bc);
    }
    C2[o0] = uint16_t(q);
    C2[o1] = uint16_t(q >> 16);
  }
}

template <int MT, int WN, int BK, int EPI>
__global__ void __launch_bounds__(128 * WN) __attribute__((amdgpu_waves_per_eu(2, 8))) bf16_gemm_dl(GemmArgs g) {
  constexpr int NT = 2, NW = 2 * WN, PR = BK / 8;
  constexpr int TM = 64 * MT, TN = 32 * NT * WN;   // output tile
  constexpr int SA = TM * PR, SB = TN * PR;        // 16-byte LDS slots per buffer and operand
  constexpr int CA = SA / (64 * NW), CB = SB / (64 * NW);  // 64-slot DMA chunks per wave and step
  static_assert(CA * 64 * NW == SA && CB * 64 * NW == SB, "whole DMA chunks per wave");
  extern __shared__ uint4 lds[];                   // 2 buffers x (SA + SB) slots, sized at launch
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const uint32_t nx = gridDim.x, tiles = gridDim.x * gridDim.y;
  uint32_t u = blockIdx.y * nx + blockIdx.x;
  if ((tiles & 7u) == 0) u = (u & 7u) * (tiles >> 3) + (u >> 3);  // XCD-aware order, as in bf16_gemm
  const int64_t m0 = int64_t(u / nx) * TM;
  const int64_t n0 = int64_t(u % nx) * TN;
  const int64_t kspan = g.K / g.splits;
  const int64_t kbeg = int64_t(blockIdx.z) * kspan;
  const int nsteps = int(kspan / BK);

  // source of the 16 bytes this lane moves in each of its chunks
  const uint16_t* ga[CA];
  const uint16_t* gb[CB];
#pragma unroll
  for (int c = 0; c < CA; ++c) {
    const int s = (wave + NW * c) * 64 + lane, row = s / PR;
    ga[c] = static_cast<const uint16_t*>(g.A) + (m0 + row) * g.lda + kbeg + ((s % PR) ^ dl_swz<PR>(row)) * 8;
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int s = (wave + NW * c) * 64 + lane, row = s / PR;
    gb[c] = static_cast<const uint16_t*>(g.B) + (n0 + row) * g.ldb + kbeg + ((s % PR) ^ dl_swz<PR>(row)) * 8;
  }
  // The builtin's operands are taken through plain pointers and the shared
  // array itself (operands of template-dependent type drop the kernel's host
  // stub).
#define QSVM_DL_ISSUE(buf, koff)                                                                      \
  do {                                                                                               \
    _Pragma("unroll") for (int c = 0; c < CA; ++c) {                                                 \
      const uint16_t* src_ = ga[c];                                                                  \
      __builtin_amdgcn_global_load_lds(src_ + (koff), lds + (buf) * (SA + SB) + (wave + NW * c) * 64, 16, 0, 0); \
    }                                                                                                \
    _Pragma("unroll") for (int c = 0; c < CB; ++c) {                                                 \
      const uint16_t* src_ = gb[c];                                                                  \
      __builtin_amdgcn_global_load_lds(src_ + (koff), lds + (buf) * (SA + SB) + SA + (wave + NW * c) * 64, 16, 0, 0); \
    }                                                                                                \
  } while (0)

  // LDS slots of this lane's fragments: row i = lane % 32 of each 32-row
  // block, 8 k-values at piece 2 * slice + lane / 32
  const int i = lane & 31, kh = lane >> 5;
  constexpr int NS = BK / 16;  // 16-deep MFMA slices per K step
  int oa[MT][NS], ob[NT][NS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int row = wm * MT * 32 + mt * 32 + i;
      oa[mt][sl] = row * PR + ((sl * 2 + kh) ^ dl_swz<PR>(row));
    }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int row = wn * NT * 32 + nt * 32 + i;
      ob[nt][sl] = SA + row * PR + ((sl * 2 + kh) ^ dl_swz<PR>(row));
    }

  f32x16_t acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mt][nt][v] = 0.0f;

  QSVM_DL_ISSUE(0, 0);
  for (int kk = 0; kk < nsteps; ++kk) {
    // this wave's DMA of step kk has landed (vmcnt(0)) and its LDS reads of
    // step kk - 1 are done (lgkmcnt(0)); the barrier makes both block-wide
    __builtin_amdgcn_s_waitcnt(0x0070);
    __builtin_amdgcn_s_barrier();
    if (kk + 1 < nsteps) QSVM_DL_ISSUE((kk + 1) & 1, int64_t(kk + 1) * BK);
    const uint4* base = lds + (kk & 1) * (SA + SB);
    bf16x8_t fa[NS][MT], fb[NS][NT];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) fa[sl][mt] = *reinterpret_cast<const bf16x8_t*>(base + oa[mt][sl]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) fb[sl][nt] = *reinterpret_cast<const bf16x8_t*>(base + ob[nt][sl]);
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[sl][mt], fb[sl][nt], acc[mt][nt], 0, 0, 0);
  }
#undef QSVM_DL_ISSUE

#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      gemm_store32<EPI>(g, acc[mt][nt], m0 + wm * MT * 32 + mt * 32, n0 + wn * NT * 32 + nt * 32, lane);
}

// Sigmoid-scaled Gram of the embeddings, K = sigmoid(ab[0] E E^T + ab[1])
// with K[i][i] = 1, on 128 x 64 output blocks (two 64 x 64 tiles of
// tile_max), the inner dimension staged through LDS 32 at a time as in
// bf16_gemm.  The kernel is bound by writing K (8 B per entry, the whole
// square: recomputing the lower triangle keeps every store stream
// row-sequential, which measured faster than mirroring the upper one); the
// 128-row blocks halve the operand traffic per output byte of a 64 x 64
// block, and the stores are non-temporal (K is not read back here).  Rows
// past N_pad (an odd tile count) are clamped on load and never stored.
__global__ void __launch_bounds__(256)
sigmoid_gram_kernel(const uint16_t* __restrict__ E, int64_t N_pad, int32_t d, const float* __restrict__ ab,
                    double* __restrict__ K, int64_t ldk, int64_t valid, float* __restrict__ tile_max) {
  constexpr int GM = 128, GN = 64;
  __shared__ __attribute__((aligned(16))) uint16_t As[GM * LDS_STRIDE];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GN * LDS_STRIDE];  // [n][k]
  __shared__ float red[2][4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t T = N_pad / 64;
  const int64_t m0 = int64_t(blockIdx.y) * GM, n0 = int64_t(blockIdx.x) * GN;

  f32x16_t acc[2];
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[w][v] = 0.0f;
  for (int k0 = 0; k0 < d; k0 += BK) {
    const int kk = (t & 3) * 8;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int m = w * 64 + (t >> 2);
      const int64_t row = (m0 + m < N_pad) ? m0 + m : N_pad - 1;
      *reinterpret_cast<uint4*>(&As[m * LDS_STRIDE + kk]) = *reinterpret_cast<const uint4*>(E + row * d + k0 + kk);
    }
    {
      const int n = t >> 2;
      *reinterpret_cast<uint4*>(&Bs[n * LDS_STRIDE + kk]) = *reinterpret_cast<const uint4*>(E + (n0 + n) * d + k0 + kk);
    }
    __syncthreads();
    const int i = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(&Bs[(wn * 32 + i) * LDS_STRIDE + ks + kh * 8]);
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&As[(w * 64 + wm * 32 + i) * LDS_STRIDE + ks + kh * 8]);
        acc[w] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[w], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // element v of an accumulator is row (v / 4) * 8 + (lane / 32) * 4 + v % 4, column lane % 32
  const float alpha = ab[0], beta = ab[1];
  const int64_t c = n0 + wn * 32 + (lane & 31);
  float tmax[2] = {-INFINITY, -INFINITY};
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = m0 + w * 64 + wm * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (r < valid && c < valid) {
        const float sg = sigmoidf(alpha * acc[w][v] + beta);
        __builtin_nontemporal_store((r == c) ? 1.0 : double(sg), &K[r * ldk + c]);
        if (r != c) tmax[w] = fmaxf(tmax[w], sg);
      }
    }
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    for (int off = 32; off > 0; off >>= 1) tmax[w] = fmaxf(tmax[w], __shfl_xor(tmax[w], off, 64));
    if (lane == 0) red[w][wave] = tmax[w];
  }
  __syncthreads();
  if (t < 2) {
    const int64_t ti = 2 * int64_t(blockIdx.y) + t;
    if (ti < T)
      tile_max[ti * T + blockIdx.x] = fmaxf(fmaxf(red[t][0], red[t][1]), fmaxf(red[t][2], red[t][3]));
  }
}

// Squared norms of the rows of z = [X16 row, E row] (FP32 sums of the squares
// of the BF16 values), one wave per row, stored as -s log2(e) |z|^2
// (s = exp(head[1])): the Gram's exponent then adds a row's and a column's
// value, which is symmetric in the two.
__global__ void __launch_bounds__(256) sat_row_norms(const uint16_t* __restrict__ X16, int32_t d_in,
                                                     const uint16_t* __restrict__ E, int32_t d, int64_t N_pad,
                                                     const float* __restrict__ head, float* __restrict__ norms) {
  const int lane = threadIdx.x & 63;
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= N_pad) return;
  float acc = 0.0f;
  for (int p = lane; p < (d_in + d) / 8; p += 64) {
    const bool x = p * 8 < d_in;
    const uint4 q = x ? *reinterpret_cast<const uint4*>(X16 + row * d_in + p * 8)
                      : *reinterpret_cast<const uint4*>(E + row * d + (p * 8 - d_in));
    const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const float lo = bf16_to_f32(uint16_t(u[h])), hi = bf16_to_f32(uint16_t(u[h] >> 16));
      acc = fmaf(lo, lo, acc);
      acc = fmaf(hi, hi, acc);
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) norms[row] = -(__expf(head[1]) * 1.44269504f) * acc;
}

// expm1(t ln 2) for t <= 0 in FP32 (t = x log2 e): the Taylor polynomial of
// expm1(x) to degree 6, written in t, above x = -1/4 (truncation below 6e-8
// relative), 2^t - 1 below (|expm1| >= 0.22 there, so the rounding of
// v_exp_f32 and of the subtraction stays below 4e-7 relative).
__device__ __forceinline__ float expm1_neg_base2(float t) {
  // ln2^k / k!, k = 6 .. 1
  float p = fmaf(t, 1.5403530e-4f, 1.3333558e-3f);
  p = fmaf(t, p, 9.6181291e-3f);
  p = fmaf(t, p, 5.5504109e-2f);
  p = fmaf(t, p, 2.4022651e-1f);
  p = fmaf(t, p, 6.9314718e-1f);
  p *= t;
  return t > -0.36067376f ? p : __builtin_amdgcn_exp2f(t) - 1.0f;
}

// Upper-triangular super-tile `st` (row-major over Is <= Js < S) -> (Is, Js).
__device__ __forceinline__ void upper_index(int64_t st, int64_t S, int64_t* is, int64_t* js) {
  const double b = double(2 * S + 1);
  int64_t i = int64_t((b - sqrt(b * b - 8.0 * double(st))) * 0.5);
  auto first = [S](int64_t r) { return r * S - r * (r - 1) / 2; };  // index of (r, r)
  if (i < 0) i = 0;
  if (i > S - 1) i = S - 1;
  while (i > 0 && first(i) > st) --i;
  while (i + 1 < S && first(i + 1) <= st) ++i;
  *is = i;
  *js = i + (st - first(i));
}

// Log-domain surrogate Gram on the embedding z = [x, f(x)] (two BF16
// segments: the gathered inputs X16, d_in wide, and the MLP output E, d wide):
//   d2 = ||z_i - z_j||^2 = |z_i|^2 + |z_j|^2 - 2 <z_i, z_j>,
//   ln K_hat = -c (1 - exp(-s d2)) = c expm1(-s d2),  c = exp(head[0]), s = exp(head[1]),
// K[i][j] = exp(ln K_hat) (FP64 store of the FP32 value), K[i][i] = 1, and
// per 64 x 64 tile the largest off-diagonal ln K_hat.
//
// Only blocks on or above the diagonal run: 128 x 128 outputs per block, the
// inner products on the direct-to-LDS pipeline of bf16_gemm_dl (both segments
// in turn, double-buffered, SG_KS 32-deep slices per step).  Alone, this loop
// runs at 0.37 of the BF16 peak with 32-deep steps and 0.48 with 64-deep ones,
// but the 64 KB of LDS the latter takes leaves two blocks per compute unit
// instead of four, too few to overlap one block's stores with another's
// inner products: the whole kernel measured 5 % slower.  Each value is formed once;
// a block off the diagonal stores its entries row by row and also their
// mirror image, each wave passing its 32 x 32 accumulators through LDS so the
// mirror rows leave as contiguous 256-byte row pieces too.  Blocks are
// grouped in 8 x 8 super-tiles that each run on one XCD (the 16 operand
// panels of a super-tile are read from its L2 once instead of once per
// block).  The row norms come precomputed (sat_row_norms).  Rows past N_pad
// (an odd tile count) are clamped on load and never stored.
constexpr int SG_G = 8;  // super-tile side, in 128-row blocks (4 and 16 measured the same)
constexpr int SG_P = 34;      // doubles per row of a wave's transpose tile (16-byte aligned rows)
constexpr int SG_KS = 1;  // 32-deep slices per K step
constexpr int SG_OPER = 2 * SG_KS * 2 * 128 * DL_PR * 16;  // two buffers of both operands, bytes
constexpr int SG_TRAN = 4 * 32 * SG_P * 8;  // the four waves' transpose tiles, bytes (reusing the operand buffers)
constexpr int SG_LDS = SG_OPER > SG_TRAN ? SG_OPER : SG_TRAN;

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
sat_log_gram_kernel(const uint16_t* __restrict__ X16, int32_t d_in, const uint16_t* __restrict__ E, int32_t d,
                    int64_t N_pad, const float* __restrict__ norms, const float* __restrict__ head,
                    double* __restrict__ K, int64_t ldk, int64_t valid, float* __restrict__ tile_max) {
  constexpr int MT = 2, NT = 2;
  constexpr int SL = 128 * DL_PR;      // 16-byte LDS slots of one operand's 32-deep slice
  constexpr int SA = SG_KS * SL;       // of one operand in a buffer
  constexpr int CA = SA / 256;         // 64-slot DMA chunks per wave and step, per operand (chunk c: slice c / 2)
  static_assert(CA == 2 * SG_KS, "chunk c of a wave holds slice c / 2");  // (wave + 4 c) / 8 = c / 2
  extern __shared__ uint4 lds[];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t T2 = (N_pad + 127) / 128, S = (T2 + SG_G - 1) / SG_G;
  // consecutive blocks of one XCD (hardware ids b, b + 8, ...) take consecutive u
  const uint32_t nb = gridDim.x;  // SG_G^2 per super-tile, a multiple of 8
  const uint32_t u = (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3);
  int64_t is, js;
  upper_index(int64_t(u / (SG_G * SG_G)), S, &is, &js);
  const int64_t I = is * SG_G + (u % (SG_G * SG_G)) / SG_G, J = js * SG_G + u % SG_G;
  if (I > J || J >= T2) return;  // the lower half of a diagonal super-tile, or past the last block
  const int64_t m0 = I * 128, n0 = J * 128;
  const int dtot = d_in + d;

  // source of the 16 bytes this lane moves in each chunk, per segment (the
  // chunk's slice offset is added at issue)
  const uint16_t* ax[CA];
  const uint16_t* ae[CA];
  const uint16_t* bx[CA];
  const uint16_t* be[CA];
#pragma unroll
  for (int c = 0; c < CA; ++c) {
    const int r = ((wave + 4 * c) * 64 + lane) % SL, row = r / DL_PR;
    const int piece = ((r % DL_PR) ^ dl_swizzle(row)) * 8;
    const int64_t ra = (m0 + row < N_pad) ? m0 + row : N_pad - 1;
    const int64_t rb = (n0 + row < N_pad) ? n0 + row : N_pad - 1;
    ax[c] = d_in ? X16 + ra * d_in + piece : E;
    bx[c] = d_in ? X16 + rb * d_in + piece : E;
    ae[c] = E + ra * d + piece;
    be[c] = E + rb * d + piece;
  }
  // step `st` (inner values 64 st ..) into buffer `buf`; each slice from the
  // segment holding it (d_in % 32 == 0), a slice past the end not at all
#define QSVM_SAT_ISSUE(buf, st)                                                                          \
  do {                                                                                                  \
    _Pragma("unroll") for (int c = 0; c < CA; ++c) {                                                    \
      const int k_ = (st) * (SG_KS * DL_BK) + (c >> 1) * DL_BK;                                         \
      if (k_ < dtot) {                                                                                  \
        const bool x_ = k_ < d_in;                                                                      \
        const int ko_ = x_ ? k_ : k_ - d_in;                                                            \
        const uint16_t* sa_ = (x_ ? ax[c] : ae[c]) + ko_;                                               \
        __builtin_amdgcn_global_load_lds(sa_, lds + (buf) * (2 * SA) + (wave + 4 * c) * 64, 16, 0, 0);   \
        const uint16_t* sb_ = (x_ ? bx[c] : be[c]) + ko_;                                               \
        __builtin_amdgcn_global_load_lds(sb_, lds + (buf) * (2 * SA) + SA + (wave + 4 * c) * 64, 16, 0, 0); \
      }                                                                                                 \
    }                                                                                                   \
  } while (0)

  const int i = lane & 31, kh = lane >> 5;
  int oa[MT][2], ob[NT][2];  // within a slice
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int row = wm * MT * 32 + mt * 32 + i;
      oa[mt][sl] = row * DL_PR + ((sl * 2 + kh) ^ dl_swizzle(row));
    }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int row = wn * NT * 32 + nt * 32 + i;
      ob[nt][sl] = SA + row * DL_PR + ((sl * 2 + kh) ^ dl_swizzle(row));
    }

  f32x16_t acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mt][nt][v] = 0.0f;

  const int nsteps = (dtot + SG_KS * DL_BK - 1) / (SG_KS * DL_BK);
  QSVM_SAT_ISSUE(0, 0);
  for (int kk = 0; kk < nsteps; ++kk) {
    __builtin_amdgcn_s_waitcnt(0x0070);  // as in bf16_gemm_dl
    __builtin_amdgcn_s_barrier();
    if (kk + 1 < nsteps) QSVM_SAT_ISSUE((kk + 1) & 1, kk + 1);
    const uint4* base = lds + (kk & 1) * (2 * SA);
#pragma unroll
    for (int ks = 0; ks < SG_KS; ++ks) {
      if (kk * (SG_KS * DL_BK) + ks * DL_BK >= dtot) break;  // uniform: the last step's missing slice
      bf16x8_t fa[2][MT], fb[2][NT];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) fa[sl][mt] = *reinterpret_cast<const bf16x8_t*>(base + ks * SL + oa[mt][sl]);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) fb[sl][nt] = *reinterpret_cast<const bf16x8_t*>(base + ks * SL + ob[nt][sl]);
      }
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[sl][mt], fb[sl][nt], acc[mt][nt], 0, 0, 0);
    }
  }
#undef QSVM_SAT_ISSUE
  __syncthreads();  // every wave is past its last operand read: the LDS becomes the transpose tiles

  // in base 2: t = -s d2 log2(e) = fma(2 s log2(e), acc, n_r + n_c) with the
  // scaled norms n = -s log2(e) |z|^2, log2 K_hat = c log2(e) expm1(t ln 2)
  const float c = __expf(head[0]), s = __expf(head[1]);
  const float sl = s * 1.44269504f, cl = c * 1.44269504f, a2 = 2.0f * sl;
  const bool mirror = I != J;
  double* tw = reinterpret_cast<double*>(lds) + wave * 32 * SG_P;  // this wave's [column][row] tile
  const int h = lane >> 5;
  float tmax = -INFINITY;  // largest off-diagonal log2 K_hat of this wave's 64 x 64 tile
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      // element v: row r0 + (v / 4) * 8 + h * 4 + v % 4, column c0 + i
      const int64_t r0 = m0 + wm * 64 + mt * 32, c0 = n0 + wn * 64 + nt * 32;
      if (r0 >= valid || c0 >= valid) continue;  // wave-uniform; r0, c0 < valid <= N_pad keep the norm reads in range
      const bool whole = r0 + 32 <= valid && c0 + 32 <= valid;  // no entry past N (wave-uniform)
      const bool diag = r0 == c0;  // the accumulator holds (r, r) at v with (v / 4) * 8 + h * 4 + v % 4 == i
      const int64_t col = c0 + i;
      const float bn = norms[col];
      float kf[16], l2[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 na = *reinterpret_cast<const float4*>(norms + r0 + q * 8 + h * 4);
        const float nav[4] = {na.x, na.y, na.z, na.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int v = q * 4 + e;
          const float t = fminf(fmaf(a2, acc[mt][nt][v], nav[e] + bn), 0.0f);
          l2[v] = cl * expm1_neg_base2(t);
          kf[v] = __builtin_amdgcn_exp2f(l2[v]);
        }
      }
      // rows r0 + h * 4 + e + 8 q, column col
      double* row = K + (r0 + h * 4) * ldk + col;
      const int64_t ld8 = 8 * ldk;
      if (whole && !diag) {
#pragma unroll
        for (int v = 0; v < 16; ++v) tmax = fmaxf(tmax, l2[v]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) __builtin_nontemporal_store(double(kf[q * 4 + e]), row + q * ld8 + e * ldk);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int v = q * 4 + e, rl = q * 8 + h * 4 + e;
            const bool self = diag && rl == i;
            if (self) kf[v] = 1.0f;
            if (r0 + rl < valid && col < valid) {
              if (!self) tmax = fmaxf(tmax, l2[v]);
              __builtin_nontemporal_store(double(kf[v]), row + q * ld8 + e * ldk);
            }
          }
      }
      if (mirror) {
        // tw[column - c0][row - r0], then rows c0 + j of K from row j of tw
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; e += 2) {
            double2 pr;
            pr.x = double(kf[q * 4 + e]);
            pr.y = double(kf[q * 4 + e + 1]);
            *reinterpret_cast<double2*>(&tw[i * SG_P + q * 8 + h * 4 + e]) = pr;
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // row c0 + 2 q + h, column r0 + i
        double* mrow = K + (c0 + h) * ldk + r0 + i;
        const int64_t ld2 = 2 * ldk;
        if (whole) {
#pragma unroll
          for (int q = 0; q < 16; ++q) __builtin_nontemporal_store(tw[(q * 2 + h) * SG_P + i], mrow + q * ld2);
        } else {
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (c0 + q * 2 + h < valid && r0 + i < valid)
              __builtin_nontemporal_store(tw[(q * 2 + h) * SG_P + i], mrow + q * ld2);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  for (int off = 32; off > 0; off >>= 1) tmax = fmaxf(tmax, __shfl_xor(tmax, off, 64));
  tmax *= 0.693147181f;  // natural log
  const int64_t T = N_pad / 64, ti = 2 * I + wm, tj = 2 * J + wn;
  if (lane == 0 && ti < T && tj < T) {
    tile_max[ti * T + tj] = tmax;
    if (mirror) tile_max[tj * T + ti] = tmax;
  }
}

// out (Cp x R, row stride R) = in (R x C, row stride C)^T for two large bf16
// matrices with the same R (R, C multiples of 8; C and Cp multiples of 64):
// output rows C .. Cp - 1 hold a row of ones, then zeros.  Block row
// blockIdx.y < y0 belongs to job 0, the others to job 1.  64 x 64 tiles,
// 16-byte loads and stores (each thread two pieces of 8 values each way)
// through a padded LDS tile.
__global__ void __launch_bounds__(256) transpose64_bf16(T64Job j0, T64Job j1, int64_t R, int32_t y0) {
  constexpr int TP = 64 + 8;  // LDS row (bf16): 144 bytes, 16-byte aligned
  __shared__ __attribute__((aligned(16))) uint16_t tile[64 * TP];
  const int t = threadIdx.x;
  const bool second = int32_t(blockIdx.y) >= y0;
  const T64Job& j = second ? j1 : j0;
  const int64_t r0 = int64_t(blockIdx.x) * 64, c0 = int64_t(second ? blockIdx.y - y0 : blockIdx.y) * 64;
  if (c0 >= j.C) {  // padding rows of the output (uniform per block)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = t + 256 * h, oc = p >> 3, pr = (p & 7) * 8;
      const uint32_t w = (c0 + oc == j.C) ? 0x3F803F80u : 0u;  // bf16 1.0 twice
      if (c0 + oc < j.Cp && r0 + pr < R)
        *reinterpret_cast<uint4*>(j.out + (c0 + oc) * R + r0 + pr) = make_uint4(w, w, w, w);
    }
    return;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p = t + 256 * h, row = p >> 3, pc = (p & 7) * 8;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (r0 + row < R && c0 + pc < j.C) v = *reinterpret_cast<const uint4*>(j.in + (r0 + row) * j.C + c0 + pc);
    *reinterpret_cast<uint4*>(&tile[row * TP + pc]) = v;
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p = t + 256 * h, oc = p >> 3, pr = (p & 7) * 8;  // output row c0 + oc, its values r0 + pr ..
    if (c0 + oc < j.C && r0 + pr < R) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w[e] = uint32_t(tile[(pr + 2 * e) * TP + oc]) | (uint32_t(tile[(pr + 2 * e + 1) * TP + oc]) << 16);
      *reinterpret_cast<uint4*>(j.out + (c0 + oc) * R + r0 + pr) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

// out_q (C_q x R_q) = in_q (R_q x C_q)^T for up to three bf16 matrices in one
// launch: block b works on matrix q with first_block[q] <= b < first_block[q + 1],
// one 32 x 32 tile through LDS (padded rows: the column reads hit distinct banks).
__global__ void __launch_bounds__(256) transpose_bf16(TransposeJobs j) {
  __shared__ uint16_t tile[32][34];
  const int b = int(blockIdx.x);
  const int q = (b >= j.first_block[2]) ? 2 : (b >= j.first_block[1]) ? 1 : 0;
  const int64_t R = j.R[q], C = j.C[q];
  const int64_t tiles_c = (C + 31) / 32;
  const int64_t u = b - j.first_block[q];
  const int64_t r0 = (u / tiles_c) * 32, c0 = (u % tiles_c) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32
  const uint16_t* __restrict__ in = j.in[q];
  uint16_t* __restrict__ out = j.out[q];
#pragma unroll
  for (int i = ty; i < 32; i += 8)
    if (r0 + i < R && c0 + tx < C) tile[i][tx] = in[(r0 + i) * C + c0 + tx];
  __syncthreads();
#pragma unroll
  for (int i = ty; i < 32; i += 8)
    if (c0 + i < C && r0 + tx < R) out[(c0 + i) * R + r0 + tx] = tile[tx][i];
}

// Indices outside [0, N) (padding rows) give zero rows.  Consecutive threads
// take consecutive feature pairs of a row (vec = 1: n and d_pad even, X
// 16-byte and out 4-byte aligned; one 16-byte load and one 4-byte store per
// thread, so a wave reads 1 KB of FP64 and writes 256 B of BF16, both
// contiguous) or consecutive single features (vec = 0).
__global__ void __launch_bounds__(256) gather_features(const double* __restrict__ X, int64_t N, int32_t n,
                                                       const int32_t* __restrict__ idx, int64_t rows, int32_t d_pad,
                                                       uint16_t* __restrict__ out, int32_t vec) {
  const int32_t per_row = vec ? d_pad / 2 : d_pad;  // work items per row
  const int64_t total = rows * per_row;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t r = (total <= int64_t(0xffffffffu)) ? int64_t(uint32_t(q) / uint32_t(per_row)) : q / per_row;
    const int32_t w = int32_t(q - r * per_row);
    const int32_t p = idx[r];
    const int32_t m = (p >= 0 && p < N) ? n : 0;  // features copied (0: padding row)
    const double* __restrict__ xr = X + int64_t(m ? p : 0) * n;
    if (vec) {
      const int32_t c = 2 * w;  // c < m implies c + 1 < m (m even)
      uint32_t h = 0u;
      if (c < m) {
        const double2 v = *reinterpret_cast<const double2*>(xr + c);
        h = uint32_t(f32_to_bf16(float(v.x))) | (uint32_t(f32_to_bf16(float(v.y))) << 16);
      }
      *reinterpret_cast<uint32_t*>(out + r * d_pad + c) = h;
    } else {
      out[r * d_pad + w] = (w < m) ? f32_to_bf16(float(xr[w])) : uint16_t(0);
    }
  }
}

// sum over z (in order) of slabs[z stride + t], t < count, into out[t] for
// t < split and out2[t - split] above.
__global__ void sum_slabs(const float* __restrict__ slabs, int32_t n_slabs, int64_t count, int64_t stride,
                          float* __restrict__ out, int64_t split, float* __restrict__ out2) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  float s = 0.0f;
  for (int32_t z = 0; z < n_slabs; ++z) s += slabs[int64_t(z) * stride + t];
  if (t < split)
    out[t] = s;
  else
    out2[t - split] = s;
}

__device__ __forceinline__ float softplusf(float z) {  // log(1 + e^z), no overflow
  return fmaxf(z, 0.0f) + log1pf(__expf(-fabsf(z)));
}

// One wave per pair p: rows p (point i) and P + p (point j) of E.  loss_kind
// 0: squared error (K_hat - t)^2; 1: cross-entropy with the soft target t,
// -t log K_hat - (1 - t) log(1 - K_hat), whose gradient in the logit s is
// K_hat - t (it does not vanish as K_hat -> 0).
__global__ void __launch_bounds__(256) pair_head(const float* __restrict__ E, int64_t P, int32_t d,
                                                 const float* __restrict__ target, const float* __restrict__ ab,
                                                 int32_t loss_kind, uint16_t* __restrict__ dE16,
                                                 float* __restrict__ partial) {
  const int64_t p = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (p >= P) return;
  const float* ei = E + p * d;
  const float* ej = E + (P + p) * d;
  float dot = 0.0f;
  for (int c = lane; c < d; c += 64) dot = fmaf(ei[c], ej[c], dot);
  for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
  const float alpha = ab[0], beta = ab[1];
  const float z = alpha * dot + beta;
  const float kh = sigmoidf(z);
  const float t = target[p];
  float lp, ds;
  if (loss_kind == 1) {
    lp = t * softplusf(-z) + (1.0f - t) * softplusf(z);
    ds = (kh - t) / float(P);
  } else {
    const float err = kh - t;
    lp = err * err;
    ds = (2.0f * err / float(P)) * kh * (1.0f - kh);
  }
  for (int c = lane; c < d; c += 64) {
    dE16[p * d + c] = f32_to_bf16(ds * alpha * ej[c]);
    dE16[(P + p) * d + c] = f32_to_bf16(ds * alpha * ei[c]);
  }
  if (lane == 0) {
    partial[3 * p + 0] = lp;
    partial[3 * p + 1] = ds * dot;
    partial[3 * p + 2] = ds;
  }
}

// Log-domain pair head, one wave per pair p: rows p (point i) and P + p
// (point j) of the gathered inputs X16 (d_in wide, BF16) and of the MLP
// output E (d wide, FP32).  d2 = ||x_i - x_j||^2 + ||e_i - e_j||^2,
// ln K_hat = c expm1(-s d2) with c = exp(head[0]), s = exp(head[1]),
// loss_p = ((ln K_hat - t) / scale)^2 with t the exact ln K.  Writes the BF16
// gradient of the mean loss w.r.t. both rows of E (the input part has no
// parameters) and the per-pair partials (loss, d/d log c, d/d log s);
// pred (optional) receives (ln K_hat, d2) per pair.
__global__ void __launch_bounds__(256) pair_head_log(const uint16_t* __restrict__ X16, int32_t d_in,
                                                     const float* __restrict__ E, int32_t d, int64_t P,
                                                     const float* __restrict__ target, const float* __restrict__ head,
                                                     float scale, uint16_t* __restrict__ dE16,
                                                     float* __restrict__ partial, float* __restrict__ pred) {
  const int64_t p = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (p >= P) return;
  const uint16_t* xi = X16 + p * d_in;
  const uint16_t* xj = X16 + (P + p) * d_in;
  const float* ei = E + p * d;
  const float* ej = E + (P + p) * d;
  float d2 = 0.0f;
  for (int c = lane; c < d_in; c += 64) {
    const float q = bf16_to_f32(xi[c]) - bf16_to_f32(xj[c]);
    d2 = fmaf(q, q, d2);
  }
  for (int c = lane; c < d; c += 64) {
    const float q = ei[c] - ej[c];
    d2 = fmaf(q, q, d2);
  }
  for (int off = 32; off > 0; off >>= 1) d2 += __shfl_xor(d2, off, 64);
  const float cc = __expf(head[0]), s = __expf(head[1]);
  const float ex = __expf(-s * d2);
  const float lk = cc * expm1f(-s * d2);
  const float r = (lk - target[p]) / scale;
  const float dl = 2.0f * r / (scale * float(P));  // d loss / d ln K_hat
  const float g = dl * (-cc * s * ex);              // d loss / d d2
  for (int c = lane; c < d; c += 64) {
    const float q = 2.0f * g * (ei[c] - ej[c]);
    dE16[p * d + c] = f32_to_bf16(q);
    dE16[(P + p) * d + c] = f32_to_bf16(-q);
  }
  if (lane == 0) {
    partial[3 * p + 0] = r * r;
    partial[3 * p + 1] = dl * lk;
    partial[3 * p + 2] = dl * (-cc * s * d2 * ex);
    if (pred) {
      pred[2 * p] = lk;
      pred[2 * p + 1] = d2;
    }
  }
}

// out[0] = mean per-pair loss, out[1] = d loss / d alpha, out[2] = d loss / d beta.
__global__ void __launch_bounds__(1024) reduce_partials(const float* __restrict__ partial, int64_t P,
                                                        float* __restrict__ out) {
  __shared__ double s[3][1024];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
    a0 += partial[3 * p];
    a1 += partial[3 * p + 1];
    a2 += partial[3 * p + 2];
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  s[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = float(s[0][0] / double(P));
    out[1] = float(s[1][0]);
    out[2] = float(s[2][0]);
  }
}

__global__ void adamw(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ m,
                      float* __restrict__ v, uint16_t* __restrict__ w16, int64_t count, AdamArgs o) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const float gr = grad[t];
  const float mt = o.beta1 * m[t] + (1.0f - o.beta1) * gr;
  const float vt = o.beta2 * v[t] + (1.0f - o.beta2) * gr * gr;
  m[t] = mt;
  v[t] = vt;
  const float mhat = mt / o.bc1;
  const float vhat = vt / o.bc2;
  float wt = w[t] * (1.0f - o.lr * o.weight_decay);
  wt -= o.lr * mhat / (sqrtf(vhat) + o.eps);
  w[t] = wt;
  if (w16) w16[t] = f32_to_bf16(wt);
}

__global__ void flag_tiles(const float* __restrict__ tile_max, int32_t T, float tau, int32_t* __restrict__ list,
                           int32_t* __restrict__ count) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(T) * T) return;
  const int32_t ti = int32_t(t / T), tj = int32_t(t % T);
  if (ti > tj) return;
  if (tile_max[t] >= tau) {
    const int32_t slot = atomicAdd(count, 1);
    list[2 * slot] = ti;
    list[2 * slot + 1] = tj;
  }
}

// Pairs of the listed tiles (a symmetric Gram's upper triangle: i < j) whose
// K_hat reaches `cut`.  One block per listed tile (grid-stride over the
// device count): a tile with at most `cap` such pairs appends them to the
// pair list (one reservation per tile), a tile with more goes to the dense
// tile list.  A tile whose reservation would pass max_pairs goes dense too,
// and fills the slots it reserved below max_pairs with (-1, -1), which the
// consumer skips.  Both counts must be zero before the launch.
__global__ void __launch_bounds__(256)
flag_pairs_kernel(const double* __restrict__ K, int64_t N, int64_t ldk, const int32_t* __restrict__ tiles,
                  const int32_t* __restrict__ tile_count, int64_t max_tiles, double cut, int32_t cap,
                  int32_t* __restrict__ pairs, int32_t* __restrict__ pair_count, int64_t max_pairs,
                  int32_t* __restrict__ dense, int32_t* __restrict__ dense_count) {
  __shared__ int32_t pre[256];
  __shared__ int64_t base_s;
  const int t = threadIdx.x;
  int64_t nt = *tile_count;
  nt = nt < 0 ? 0 : (nt < max_tiles ? nt : max_tiles);
  for (int64_t u = blockIdx.x; u < nt; u += gridDim.x) {  // block-uniform
    const int32_t ti = tiles[2 * u], tj = tiles[2 * u + 1];
    // this thread's 16 entries: e = t + 256 q, row e / 64, column e % 64
    uint32_t hits = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + 256 * q, r = e >> 6, c = e & 63;
      const int64_t i = int64_t(ti) * 64 + r, j = int64_t(tj) * 64 + c;
      const bool ok = ti >= 0 && tj >= ti && i < N && j < N && (ti < tj || c > r) && K[i * ldk + j] >= cut;
      hits |= uint32_t(ok) << q;
    }
    // block prefix sum of the hit counts (Hillis-Steele in LDS)
    pre[t] = __builtin_popcount(hits);
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int32_t v = (t >= off) ? pre[t - off] : 0;
      __syncthreads();
      pre[t] += v;
      __syncthreads();
    }
    const int32_t total = pre[255];
    const int32_t mine = pre[t] - __builtin_popcount(hits);  // exclusive prefix
    if (t == 0) base_s = (total > 0 && total <= cap) ? int64_t(atomicAdd(pair_count, total)) : -1;
    __syncthreads();
    const int64_t base = base_s;
    const bool listed = base >= 0 && base + total <= max_pairs;
    if (t == 0 && total > 0 && !listed) {
      const int32_t slot = atomicAdd(dense_count, 1);
      dense[2 * slot] = ti;
      dense[2 * slot + 1] = tj;
    }
    int64_t w = base + mine;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (!((hits >> q) & 1u)) continue;
      if (base >= 0 && w < max_pairs) {
        const int e = t + 256 * q;
        pairs[2 * w] = listed ? ti * 64 + (e >> 6) : -1;
        pairs[2 * w + 1] = listed ? tj * 64 + (e & 63) : -1;
      }
      ++w;
    }
    __syncthreads();  // pre[] and base_s are rewritten for the next tile
  }
}

__global__ void zero_two(int32_t* a, int32_t* b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *a = 0;
    *b = 0;
  }
}

__global__ void zero_int(int32_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

template <int TA, int TB, int EPI>
hipError_t launch_gemm_t(const GemmArgs& g, hipStream_t s) {
  // both operands k-contiguous, 16-byte rows: the direct-to-LDS kernel, on
  // 256 x 256 tiles with 64-deep K steps when they fill every compute unit
  // (one 8-wave block each, 128 KB of LDS), else on 256 x 128 tiles when
  // there are at least 512 of them (two per compute unit), else 128 x 128,
  // with 64-deep steps when at most two blocks share a compute unit
  const bool dl = TA == 0 && TB == 1 && g.M % 128 == 0 && g.N % 128 == 0 && g.lda % 8 == 0 && g.ldb % 8 == 0 &&
                  g.K % g.splits == 0;
  if (dl && g.M % 256 == 0 && g.N % 256 == 0 && (g.K / g.splits) % 64 == 0 &&
      (g.M / 256) * (g.N / 256) * g.splits >= 256) {
    constexpr int lds = 2 * (256 + 256) * 8 * 16;
    // more than the default 64 KB of dynamic LDS: raised once per device
    static std::atomic<uint64_t> lds_raised{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? uint64_t(1) << dev : 0;
    if (!(lds_raised.load() & bit)) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bf16_gemm_dl<4, 4, 64, EPI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      lds_raised.fetch_or(bit);
    }
    const dim3 grid(unsigned(g.N / 256), unsigned(g.M / 256), unsigned(g.splits));
    hipLaunchKernelGGL((bf16_gemm_dl<4, 4, 64, EPI>), grid, dim3(512), lds, s, g);
    return hipGetLastError();
  }
  if (dl && (g.K / g.splits) % DL_BK == 0) {
    if (g.M % 256 == 0 && (g.M / 256) * (g.N / 128) >= 512) {
      const dim3 grid(unsigned(g.N / 128), unsigned(g.M / 256), unsigned(g.splits));
      const size_t lds = 2 * (256 + 128) * DL_PR * 16;
      hipLaunchKernelGGL((bf16_gemm_dl<4, 2, DL_BK, EPI>), grid, dim3(256), lds, s, g);
    } else if ((g.K / g.splits) % 64 == 0 && (g.M / 128) * (g.N / 128) * g.splits <= 512) {
      // at most two blocks per compute unit: 64-deep steps in 64 KB of LDS
      const dim3 grid(unsigned(g.N / 128), unsigned(g.M / 128), unsigned(g.splits));
      const size_t lds = 2 * (128 + 128) * 8 * 16;
      hipLaunchKernelGGL((bf16_gemm_dl<2, 2, 64, EPI>), grid, dim3(256), lds, s, g);
    } else {
      const dim3 grid(unsigned(g.N / 128), unsigned(g.M / 128), unsigned(g.splits));
      const size_t lds = 2 * (128 + 128) * DL_PR * 16;
      hipLaunchKernelGGL((bf16_gemm_dl<2, 2, DL_BK, EPI>), grid, dim3(256), lds, s, g);
    }
    return hipGetLastError();
  }
  const dim3 grid(unsigned(g.N / BN), unsigned(g.M / BM), unsigned(g.splits));
  hipLaunchKernelGGL((bf16_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(int ta, int tb, int epi, const GemmArgs& g, hipStream_t s) {
  switch (ta * 100 + tb * 10 + epi) {
    case 0 * 100 + 0 * 10 + EPI_BIAS_GELU: return launch_gemm_t<0, 0, EPI_BIAS_GELU>(g, s);
    case 0 * 100 + 0 * 10 + EPI_BIAS: return launch_gemm_t<0, 0, EPI_BIAS>(g, s);
    case 0 * 100 + 0 * 10 + EPI_F32: return launch_gemm_t<0, 0, EPI_F32>(g, s);
    case 1 * 100 + 0 * 10 + EPI_F32: return launch_gemm_t<1, 0, EPI_F32>(g, s);
    case 0 * 100 + 1 * 10 + EPI_BIAS_GELU: return launch_gemm_t<0, 1, EPI_BIAS_GELU>(g, s);
    case 0 * 100 + 1 * 10 + EPI_BIAS: return launch_gemm_t<0, 1, EPI_BIAS>(g, s);
    case 0 * 100 + 1 * 10 + EPI_GELU_BWD: return launch_gemm_t<0, 1, EPI_GELU_BWD>(g, s);
    case 0 * 100 + 1 * 10 + EPI_F32: return launch_gemm_t<0, 1, EPI_F32>(g, s);
    case 0 * 100 + 1 * 10 + EPI_BIAS_GELU_BF16: return launch_gemm_t<0, 1, EPI_BIAS_GELU_BF16>(g, s);
    case 0 * 100 + 1 * 10 + EPI_BIAS_BF16: return launch_gemm_t<0, 1, EPI_BIAS_BF16>(g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sigmoid_gram(const uint16_t* E, int64_t N_pad, int32_t d, const float* ab, double* K, int64_t ldk,
                               int64_t valid, float* tile_max, hipStream_t s) {
  const int64_t T = N_pad / 64;
  const dim3 grid(unsigned(T), unsigned((T + 1) / 2));
  hipLaunchKernelGGL(sigmoid_gram_kernel, grid, dim3(256), 0, s, E, N_pad, d, ab, K, ldk, valid, tile_max);
  return hipGetLastError();
}

hipError_t launch_transpose64_bf16(T64Job j0, T64Job j1, int64_t R, hipStream_t s) {
  auto bad = [](const T64Job& j) { return j.C < 64 || j.C % 64 || j.Cp < j.C || j.Cp % 64; };
  if (R < 1 || R % 8 || bad(j0) || bad(j1) || (R + 63) / 64 > INT32_MAX || (j0.Cp + j1.Cp) / 64 > 65535)
    return hipErrorInvalidValue;
  const int32_t y0 = int32_t(j0.Cp / 64);
  hipLaunchKernelGGL(transpose64_bf16, dim3(unsigned((R + 63) / 64), unsigned(y0 + j1.Cp / 64)), dim3(256), 0, s, j0,
                     j1, R, y0);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(TransposeJobs j, int32_t count, hipStream_t s) {
  if (count < 1 || count > 3) return hipErrorInvalidValue;
  int32_t blocks = 0;
  for (int q = 0; q < 3; ++q) {
    j.first_block[q] = blocks;
    if (q < count) blocks += int32_t(((j.R[q] + 31) / 32) * ((j.C[q] + 31) / 32));
  }
  j.first_block[3] = blocks;
  for (int q = count; q < 3; ++q) j.first_block[q] = blocks;  // unused slots own no block
  hipLaunchKernelGGL(transpose_bf16, dim3(unsigned(blocks)), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_gather(const double* X, int64_t N, int32_t n, const int32_t* idx, int64_t rows, int32_t d_pad,
                         uint16_t* out, hipStream_t s) {
  const int32_t vec = (n % 2 == 0 && d_pad % 2 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
                       (reinterpret_cast<uintptr_t>(out) & 3) == 0) ? 1 : 0;
  const int64_t work = (rows * (vec ? d_pad / 2 : d_pad) + 255) / 256;
  const int64_t blocks = work < 1 ? 1 : (work < 65536 ? work : 65536);  // grid-stride beyond
  hipLaunchKernelGGL(gather_features, dim3(unsigned(blocks)), dim3(256), 0, s, X, N, n, idx, rows, d_pad, out, vec);
  return hipGetLastError();
}

hipError_t launch_sum_slabs(const float* slabs, int32_t n_slabs, int64_t count, int64_t stride, float* out,
                            int64_t split, float* out2, hipStream_t s) {
  hipLaunchKernelGGL(sum_slabs, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, slabs, n_slabs, count, stride,
                     out, split, out2);
  return hipGetLastError();
}

hipError_t launch_pair_head(const float* E, int64_t P, int32_t d, const float* target, const float* ab,
                            int32_t loss_kind, uint16_t* dE16, float* partial, float* out3, hipStream_t s) {
  const int64_t threads = P * 64;
  hipLaunchKernelGGL(pair_head, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, E, P, d, target, ab,
                     loss_kind, dE16, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(1024), 0, s, partial, P, out3);
  return hipGetLastError();
}

hipError_t launch_pair_head_log(const uint16_t* X16, int32_t d_in, const float* E, int32_t d, int64_t P,
                                const float* target, const float* head, float scale, uint16_t* dE16, float* partial,
                                float* out3, float* pred, hipStream_t s) {
  const int64_t threads = P * 64;
  hipLaunchKernelGGL(pair_head_log, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, X16, d_in, E, d, P,
                     target, head, scale, dE16, partial, pred);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(1024), 0, s, partial, P, out3);
  return hipGetLastError();
}

hipError_t launch_sat_log_gram(const uint16_t* X16, int32_t d_in, const uint16_t* E, int32_t d, int64_t N_pad,
                               const float* head, double* K, int64_t ldk, int64_t valid, float* tile_max,
                               float* norms, hipStream_t s) {
  const int64_t T2 = (N_pad + 127) / 128, S = (T2 + SG_G - 1) / SG_G;
  const int64_t blocks = S * (S + 1) / 2 * SG_G * SG_G;
  if (blocks * 256 >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sat_row_norms, dim3(unsigned((N_pad + 3) / 4)), dim3(256), 0, s, X16, d_in, E, d, N_pad, head,
                     norms);
  hipLaunchKernelGGL(sat_log_gram_kernel, dim3(unsigned(blocks)), dim3(256), SG_LDS, s, X16, d_in, E, d, N_pad, norms,
                     head, K, ldk, valid, tile_max);
  return hipGetLastError();
}

hipError_t launch_adamw(float* w, const float* grad, float* m, float* v, uint16_t* w16, int64_t count,
                        const AdamArgs& o, hipStream_t s) {
  hipLaunchKernelGGL(adamw, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, w, grad, m, v, w16, count, o);
  return hipGetLastError();
}

hipError_t launch_flag_pairs(const double* K, int64_t N, int64_t ldk, const int32_t* tiles, const int32_t* tile_count,
                             int64_t max_tiles, double cut, int32_t cap, int32_t* pairs, int32_t* pair_count,
                             int64_t max_pairs, int32_t* dense, int32_t* dense_count, hipStream_t s) {
  hipLaunchKernelGGL(zero_two, dim3(1), dim3(64), 0, s, pair_count, dense_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || max_tiles <= 0) return e;
  const int64_t blocks = max_tiles < 8192 ? max_tiles : 8192;  // grid-stride over the listed tiles
  hipLaunchKernelGGL(flag_pairs_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, K, N, ldk, tiles, tile_count,
                     max_tiles, cut, cap, pairs, pair_count, max_pairs, dense, dense_count);
  return hipGetLastError();
}

hipError_t launch_flag_tiles(const float* tile_max, int32_t T, float tau, int32_t* list, int32_t* count,
                             hipStream_t s) {
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(64), 0, s, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = int64_t(T) * T;
  hipLaunchKernelGGL(flag_tiles, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, tile_max, T, tau, list, count);
  return hipGetLastError();
}

}  // namespace qsvm
