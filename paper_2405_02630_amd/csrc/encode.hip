// MPS encode kernel: writes the exact closed-form MPS of every data point.
//
// The paper converts each pair's circuit into an einsum expression plus
// operands and updates the operands in place for the next pair (§3.4.2,
// §4.1).  Here the operands are built once per point.  For the ZZ feature
// map every repetition is H^n followed by a diagonal phase
// exp(i[sum_k 2 x_k b_k + sum_k theta_k (b_k XOR b_{k+1})]); inserting the
// computational basis between repetitions gives each qubit an r-bit "column"
// c = (value after rep 1, ..., value after rep r) and
//     psi(s) = sum_{c : c_{k,r} = s_k} prod_k w_k(c_k) prod_k J_k(c_k, c_{k+1}),
//     w_k(c) = 2^{-r/2} (-1)^{sum_l c_l c_{l-1}} exp(2 i x_k |c|),
//     J_k(c, c') = exp(i theta_k |c XOR c'|),
// i.e. an MPS with bond dimension exactly 2^r and site tensor
// A_k[alpha][beta] = J_{k-1}(alpha, beta) w_k(beta) (the dense tensors);
// Section G stores the generators (a_k, b_k, g_{n-1}) of the same
// MPS in the diagonal gauge D_k = diag(1, g_k) per bond bit, where
// J_{k-1} w_k factorises into 2x2 blocks [[1, a_k], [1, b_k]], and Section L
// the FP32 residuals of those generators (FP32 value + residual = the FP64
// value to ~2^-48), read only by the FP64 refinement (layout and formulas in
// include/qsvm.h).  The MPS buffer holds Sections G and L; the dense tensors
// A_k are written on request into a buffer of their own (only the dense
// sweep reads them).
//
// One thread per (site k, point i) in both kernels.  All phases are formed in
// FP64 (the largest angle is below 4 * (2 pi + 2 pi^2) ~ 104 rad) and each
// value is rounded to FP32 once.

#include "qsvm_internal.h"

namespace qsvm {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double zz_theta(double a, double b) {
  return 2.0 * (kPi - a) * (kPi - b);
}

// Dense site tensors (the opt-in buffer of qsvm_encode_dense): one thread per
// (site k, point i) computes the point's chi x chi tensor; the tensors go out
// through LDS so that consecutive lanes store consecutive addresses.
template <int R>
__global__ void __launch_bounds__(256)
encode_dense_kernel(const double* __restrict__ X, int64_t N, int32_t n, float2* __restrict__ dense) {
  constexpr int CHI = 1 << R;
  constexpr int E = CHI * CHI;             // entries per site tensor
  constexpr int CH = (E < 16) ? E : 16;    // entries staged per round
  __shared__ float2 stage[256 * CH];
  const int64_t i0 = int64_t(blockIdx.x) * blockDim.x;
  const int64_t i = i0 + threadIdx.x;
  const int32_t k = blockIdx.y;
  const bool valid = i < N;
  const double* x = X + (valid ? i : N - 1) * n;  // idle threads compute a valid point, store nothing

  const double xk = x[k];
  const double th_prev = (k >= 1) ? zz_theta(x[k - 1], xk) : 0.0;  // theta_{k-1}
  // powers p^m = exp(2 i x_k m) and t^m = exp(i theta_{k-1} m), m = 0..R, in FP64
  double pr[R + 1], pi_[R + 1], tr[R + 1], ti[R + 1];
  double sp, cp, st, ct;
  sincos(2.0 * xk, &sp, &cp);
  sincos(th_prev, &st, &ct);
  pr[0] = 1.0; pi_[0] = 0.0; tr[0] = 1.0; ti[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    pr[m] = pr[m - 1] * cp - pi_[m - 1] * sp;
    pi_[m] = pr[m - 1] * sp + pi_[m - 1] * cp;
    tr[m] = tr[m - 1] * ct - ti[m - 1] * st;
    ti[m] = tr[m - 1] * st + ti[m - 1] * ct;
  }
  // 2^{-R/2}
  const double scale = (R == 1)   ? 0.70710678118654752440
                       : (R == 2) ? 0.5
                       : (R == 3) ? 0.35355339059327376220
                                  : 0.25;
  const int64_t base = (int64_t(k) * N + i0) * E;  // the block's points are contiguous
  const int64_t npts = (N - i0 < 256) ? N - i0 : 256;
#pragma unroll
  for (int c = 0; c < E / CH; ++c) {
#pragma unroll
    for (int e = 0; e < CH; ++e) {
      const int ab = c * CH + e;
      const int a = ab / CHI, b = ab % CHI;
      const int pb = __builtin_popcount(b);
      const int pab = __builtin_popcount(a ^ b);
      const int sgn_bits = __builtin_popcount(b & (b >> 1)) & 1;  // sum_l b_l b_{l-1} mod 2
      const double re = pr[pb] * tr[pab] - pi_[pb] * ti[pab];
      const double im = pr[pb] * ti[pab] + pi_[pb] * tr[pab];
      const double sg = sgn_bits ? -scale : scale;
      stage[threadIdx.x * CH + e] = make_float2(float(re * sg), float(im * sg));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 256 * CH; t += 256) {
      const int p = t / CH, e = t % CH;
      if (p < npts) dense[base + int64_t(p) * E + c * CH + e] = stage[t];
    }
    __syncthreads();
  }
}

// Sections G and L (the MPS buffer): one thread per (site k, point i) forms
// the generator phases in FP64, rounds each component to FP32 once and keeps
// the residual; consecutive threads write consecutive 16-byte entries.
__global__ void __launch_bounds__(256)
encode_gen_kernel(const double* __restrict__ X, int64_t N, int32_t n, float4* __restrict__ gen,
                  float4* __restrict__ gen_lo) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int32_t k = blockIdx.y;
  if (i >= N) return;
  const double* x = X + i * n;
  double g0, g1, g2, g3;
  if (k >= 1) {
    // G_{k-1} = 2 x_{k-1} + theta_{k-2};  a_k = e^{i(theta_{k-1} + G_{k-1})},
    // b_k = e^{i(G_{k-1} - theta_{k-1})}
    const double xm = x[k - 1];
    const double th_prev = zz_theta(xm, x[k]);
    const double th_pp = (k >= 2) ? zz_theta(x[k - 2], xm) : 0.0;
    const double G = 2.0 * xm + th_pp;
    sincos(G + th_prev, &g1, &g0);
    sincos(G - th_prev, &g3, &g2);
  } else {
    // closure phase g_{n-1} = e^{i(2 x_{n-1} + theta_{n-2})}
    const double xl = x[n - 1];
    const double th_l = (n >= 2) ? zz_theta(x[n - 2], xl) : 0.0;
    sincos(2.0 * xl + th_l, &g1, &g0);
    g2 = g3 = 0.0;
  }
  const float4 hi = make_float4(float(g0), float(g1), float(g2), float(g3));
  gen[int64_t(k) * N + i] = hi;
  gen_lo[int64_t(k) * N + i] = make_float4(float(g0 - double(hi.x)), float(g1 - double(hi.y)), float(g2 - double(hi.z)),
                                           float(g3 - double(hi.w)));
}

}  // namespace

hipError_t launch_encode(const double* X, int64_t N, int32_t n, int32_t reps, void* mps,
                         hipStream_t stream) {
  if (reps < 1 || reps > kMaxReps) return hipErrorInvalidValue;
  float4* gen = static_cast<float4*>(mps);
  float4* gen_lo = gen + int64_t(n) * N;  // Section L follows Section G
  hipLaunchKernelGGL(encode_gen_kernel, dim3(unsigned((N + 255) / 256), unsigned(n)), dim3(256), 0, stream, X, N, n,
                     gen, gen_lo);
  return hipGetLastError();
}

hipError_t launch_encode_dense(const double* X, int64_t N, int32_t n, int32_t reps, void* dense,
                               hipStream_t stream) {
  const dim3 block(256);
  const dim3 grid(unsigned((N + 255) / 256), unsigned(n));
  float2* d = static_cast<float2*>(dense);
  switch (reps) {
    case 1: hipLaunchKernelGGL(encode_dense_kernel<1>, grid, block, 0, stream, X, N, n, d); break;
    case 2: hipLaunchKernelGGL(encode_dense_kernel<2>, grid, block, 0, stream, X, N, n, d); break;
    case 3: hipLaunchKernelGGL(encode_dense_kernel<3>, grid, block, 0, stream, X, N, n, d); break;
    case 4: hipLaunchKernelGGL(encode_dense_kernel<4>, grid, block, 0, stream, X, N, n, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qsvm
