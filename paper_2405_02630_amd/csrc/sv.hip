// State-vector engine: the full 2^n-amplitude state of every point and the
// Gram as one dense complex product of the state matrices.
//
// This is the paper's first simulation method (state-vector simulation of
// the kernel circuit, §3.4.1 and Alg. 1) rebuilt for a whole Gram: instead
// of simulating QC(x_i) followed by QC(x_j)^dagger once per pair, each
// point's state psi(x) = U(x)|0^n> is built once, and
//     K_ij = |<psi(x_j)|psi(x_i)>|^2 = |(Psi_a Psi_b^H)_ij|^2,
// a complex GEMM with inner dimension 2^n.  Everything is FP64.
//
// State: one repetition of the ZZ feature map is H on every qubit followed
// by the diagonal phase exp(i Phi(b)),
//     Phi(b) = sum_k 2 x_k b_k + sum_{k<n-1} theta_k (b_k XOR b_{k+1}),
// theta_k = 2 (pi - x_k)(pi - x_{k+1}), bit k of b being qubit k.  So
// psi = (D H)^r |0>: the first H gives the uniform state, each later H is an
// unnormalised Walsh-Hadamard transform (register-radix passes of up to 4
// bits), and the phase pass applies 2^(-n/2) exp(i Phi(b)) (the H
// normalisation folded in).
//
// Gram: v_mfma_f64_16x16x4_f64 on 64 x 64 output tiles (4 waves of 32 x 32),
// inner dimension staged through LDS 16 complex values at a time, complex
// product as two real accumulators (re: ar br + ai bi, im: ai br - ar bi,
// the conjugate on the bra side), and |G|^2 written by the same finalize
// (mirror, diagonal rule, optional log K) as the MPS sweeps.

#include "../../include/qsvm.h"
#include "sweep_common.h"

namespace qsvm {
namespace {

constexpr double kPiD = 3.14159265358979323846;

// psi(b) <- 2^(-n/2) exp(i Phi_x(b)) * (FIRST ? 1 : psi(b)); each thread
// handles 4 consecutive entries of one point (chunks = ceil(D / 4) per point).
template <bool FIRST>
__global__ void __launch_bounds__(256)
sv_phase_kernel(const double* __restrict__ X, int64_t N, int32_t n, int64_t D, double2* __restrict__ sv) {
  const int64_t chunks = (D + 3) / 4;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= N * chunks) return;
  const int64_t p = t / chunks;
  const int64_t b0 = (t - p * chunks) * 4;
  const double* x = X + p * n;
  double ph[4] = {0.0, 0.0, 0.0, 0.0};
  double xk = x[0];
  for (int k = 0; k < n; ++k) {
    const double xn = (k + 1 < n) ? x[k + 1] : 0.0;
    const double al = 2.0 * xk;
    const double th = 2.0 * (kPiD - xk) * (kPiD - xn);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t b = b0 + e;
      const int bk = int((b >> k) & 1);
      if (bk) ph[e] += al;
      if (k + 1 < n && (bk ^ int((b >> (k + 1)) & 1))) ph[e] += th;
    }
    xk = xn;
  }
  const double scale = exp2(-0.5 * double(n));
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t b = b0 + e;
    if (b >= D) break;
    double s, c;
    sincos(ph[e], &s, &c);
    c *= scale;
    s *= scale;
    double2* q = sv + p * D + b;
    if (FIRST) {
      *q = make_double2(c, s);
    } else {
      const double2 v = *q;
      *q = make_double2(fma(c, v.x, -(s * v.y)), fma(c, v.y, s * v.x));
    }
  }
}

// Unnormalised Walsh-Hadamard transform on bits [s, s + G) of every state:
// each thread loads the 2^G entries that differ only in those bits.
template <int G>
__global__ void __launch_bounds__(256)
sv_wht_kernel(int64_t N, int32_t n, int32_t s, double2* __restrict__ sv) {
  constexpr int P = 1 << G;
  const int64_t per_point = int64_t(1) << (n - G);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= N * per_point) return;
  const int64_t p = t / per_point;
  const int64_t r = t - p * per_point;
  const int64_t low = r & ((int64_t(1) << s) - 1);
  const int64_t high = r >> s;
  double2* base = sv + (p << n) + (high << (s + G)) + low;
  const int64_t stride = int64_t(1) << s;
  double2 v[P];
#pragma unroll
  for (int u = 0; u < P; ++u) v[u] = base[u * stride];
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (u & (1 << g)) continue;
      const double2 a = v[u], c = v[u | (1 << g)];
      v[u] = make_double2(a.x + c.x, a.y + c.y);
      v[u | (1 << g)] = make_double2(a.x - c.x, a.y - c.y);
    }
  }
#pragma unroll
  for (int u = 0; u < P; ++u) base[u * stride] = v[u];
}

typedef double dvec4 __attribute__((ext_vector_type(4)));

constexpr int kKB = 16;  // complex inner-dimension values per LDS stage

// One 64 x 64 tile of K = |Psi_a Psi_b^H|^2.  Wave w owns rows (w / 2) * 32 and
// columns (w % 2) * 32 of the tile as 2 x 2 MFMA blocks of 16 x 16.
// MFMA f64 16x16x4 operand layout (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result element v of lane l is
// D[4 v + l / 16][l % 16].
// With splits > 1 the inner dimension is cut into `splits` chunks of kchunk
// values; block (tile, split) writes its partial product to W and
// sv_reduce_kernel adds the partials in split order.
__global__ void __launch_bounds__(256)
sv_gram_kernel(SweepArgs a, const double2* __restrict__ A, const double2* __restrict__ B, int64_t D,
               int32_t splits, int64_t kchunk, double2* __restrict__ W) {
  __shared__ double2 sA[kKB][64];
  __shared__ double2 sB[kKB][64];
  const uint32_t L = xcd_logical_block();
  if (L >= a.num_blocks) return;
  const uint32_t tile = L / uint32_t(splits);
  const int32_t split = int32_t(L % uint32_t(splits));
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;
  const int64_t i0 = int64_t(ti) * kTile, j0 = int64_t(tj) * kTile;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  dvec4 accr[2][2], acci[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) {
      accr[mi][nj] = dvec4{0.0, 0.0, 0.0, 0.0};
      acci[mi][nj] = dvec4{0.0, 0.0, 0.0, 0.0};
    }

  // loader: thread t stages row t / 4, inner values (t % 4) * 4 .. + 3
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const int64_t ga = i0 + lrow, gb = j0 + lrow;
  const bool va = ga < a.Na, vb = gb < a.Nb;
  const double2* pa = A + (va ? ga : 0) * D;
  const double2* pb = B + (vb ? gb : 0) * D;

  const int64_t kbeg = int64_t(split) * kchunk;
  const int64_t kend = (kbeg + kchunk < D) ? kbeg + kchunk : D;
  // the next stage's values are loaded into registers while the current
  // stage's MFMAs run
  double2 na[4], nb[4];
  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t k = k0 + lk + e;
      const bool kin = k < kend;
      na[e] = (va && kin) ? pa[k] : make_double2(0.0, 0.0);
      nb[e] = (vb && kin) ? pb[k] : make_double2(0.0, 0.0);
    }
  };
  load_stage(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kKB) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sA[lk + e][lrow] = na[e];
      sB[lk + e][lrow] = nb[e];
    }
    __syncthreads();
    if (k0 + kKB < kend) load_stage(k0 + kKB);
#pragma unroll
    for (int ks = 0; ks < kKB; ks += 4) {
      const int kk = ks + (lane >> 4);
      double2 fa[2], fb[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) fa[mi] = sA[kk][wr + mi * 16 + (lane & 15)];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) fb[nj] = sB[kk][wc + nj * 16 + (lane & 15)];
      const double nar[2] = {-fa[0].x, -fa[1].x};
      // re += ar br + ai bi ; im += ai br - ar bi.  The eight accumulators are
      // visited in turn, so no MFMA waits on the one just issued.
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
          accr[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi].x, fb[nj].x, accr[mi][nj], 0, 0, 0);
          acci[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi].y, fb[nj].x, acci[mi][nj], 0, 0, 0);
        }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
          accr[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi].y, fb[nj].y, accr[mi][nj], 0, 0, 0);
          acci[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(nar[mi], fb[nj].y, acci[mi][nj], 0, 0, 0);
        }
    }
    __syncthreads();
  }

#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr + mi * 16 + 4 * v + (lane >> 4);
        const int c = wc + nj * 16 + (lane & 15);
        const double gr = accr[mi][nj][v], gi = acci[mi][nj][v];
        if (splits > 1) {
          W[(int64_t(tile) * splits + split) * (kTile * kTile) + r * kTile + c] = make_double2(gr, gi);
          continue;
        }
        const int64_t i = i0 + r, j = j0 + c;
        if (!pair_active(a, i, j)) continue;
        store_entry(a, i, j, fma(gr, gr, gi * gi), 0);
      }
}

// Sum the split partials of every tile entry in split order, then finalize.
__global__ void __launch_bounds__(256)
sv_reduce_kernel(SweepArgs a, int32_t splits, const double2* __restrict__ W) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // (tile, entry)
  const uint32_t tile = uint32_t(t / (kTile * kTile));
  if (tile >= a.num_blocks) return;
  const int e = int(t % (kTile * kTile));
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;
  const int64_t i = int64_t(ti) * kTile + e / kTile, j = int64_t(tj) * kTile + e % kTile;
  if (!pair_active(a, i, j)) return;
  double gr = 0.0, gi = 0.0;
  const double2* w = W + int64_t(tile) * splits * (kTile * kTile) + e;
  for (int s = 0; s < splits; ++s) {
    const double2 g = w[int64_t(s) * (kTile * kTile)];
    gr += g.x;
    gi += g.y;
  }
  store_entry(a, i, j, fma(gr, gr, gi * gi), 0);
}

}  // namespace

hipError_t launch_encode_sv(const double* X, int64_t N, int32_t n, int32_t reps, void* sv, hipStream_t stream) {
  const int64_t D = int64_t(1) << n;
  double2* s = static_cast<double2*>(sv);
  const dim3 pgrid(unsigned((N * ((D + 3) / 4) + 255) / 256));
  for (int l = 0; l < reps; ++l) {
    if (l > 0) {
      // unnormalised H on every qubit, up to 4 bits per pass
      for (int s0 = 0; s0 < n; s0 += 4) {
        const int g = (n - s0 < 4) ? n - s0 : 4;
        const int64_t threads = N * (D >> g);
        const dim3 grid(unsigned((threads + 255) / 256));
        switch (g) {
          case 1: hipLaunchKernelGGL(sv_wht_kernel<1>, grid, dim3(256), 0, stream, N, n, s0, s); break;
          case 2: hipLaunchKernelGGL(sv_wht_kernel<2>, grid, dim3(256), 0, stream, N, n, s0, s); break;
          case 3: hipLaunchKernelGGL(sv_wht_kernel<3>, grid, dim3(256), 0, stream, N, n, s0, s); break;
          default: hipLaunchKernelGGL(sv_wht_kernel<4>, grid, dim3(256), 0, stream, N, n, s0, s); break;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(sv_phase_kernel<false>, pgrid, dim3(256), 0, stream, X, N, n, D, s);
    } else {
      hipLaunchKernelGGL(sv_phase_kernel<true>, pgrid, dim3(256), 0, stream, X, N, n, D, s);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sv_gram(const SweepArgs& a0, const void* sv_a, const void* sv_b, int32_t n, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = 1;
  const int64_t tiles = launch_tiles(a);
  if (tiles <= 0) return hipSuccess;
  const int64_t D = int64_t(1) << n;
  // split the inner dimension until about 1024 blocks are in flight, keeping
  // at least 256 values (16 LDS stages) per split
  int64_t splits = (1024 + tiles - 1) / tiles;
  if (splits > D / 256) splits = D / 256;
  if (splits < 1) splits = 1;
  const int64_t kchunk = ((D + splits - 1) / splits + kKB - 1) / kKB * kKB;
  splits = (D + kchunk - 1) / kchunk;
  const int64_t blocks = tiles * splits;
  if (blocks > (int64_t(1) << 31) - 8) return hipErrorInvalidValue;
  a.num_blocks = uint32_t(blocks);
  double2* W = nullptr;
  if (splits > 1) {
    const hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&W), size_t(blocks) * kTile * kTile * sizeof(double2),
                                        stream);
    if (e != hipSuccess) return e;
  }
  const uint32_t padded = uint32_t((blocks + 7) / 8 * 8);
  hipLaunchKernelGGL(sv_gram_kernel, dim3(padded), dim3(256), 0, stream, a, static_cast<const double2*>(sv_a),
                     static_cast<const double2*>(sv_b), D, int32_t(splits), kchunk, W);
  hipError_t e = hipGetLastError();
  if (splits > 1) {
    if (e == hipSuccess) {
      SweepArgs r = a;
      r.num_blocks = uint32_t(tiles);
      const int64_t threads = tiles * kTile * kTile;
      hipLaunchKernelGGL(sv_reduce_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, stream, r,
                         int32_t(splits), static_cast<const double2*>(W));
      e = hipGetLastError();
    }
    const hipError_t f = hipFreeAsync(W, stream);
    if (e == hipSuccess) e = f;
  }
  return e;
}

}  // namespace qsvm
