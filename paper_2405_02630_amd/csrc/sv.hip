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
// unnormalised Walsh-Hadamard transform (passes over LDS tiles), and each
// repetition ends by multiplying with 2^(-n/2) exp(i Phi(b)) (the H
// normalisation folded in), read from two small per-point tables.
//
// Gram: v_mfma_f64_16x16x4_f64 on 64 x 64 output tiles (4 waves of 32 x 32),
// inner dimension staged through LDS 16 complex values at a time, complex
// product as two real accumulators (re: ar br + ai bi, im: ai br - ar bi,
// the conjugate on the bra side), and |G|^2 written by the same finalize
// (mirror, diagonal rule, optional log K) as the MPS sweeps.

#include <atomic>

#include "../../include/qsvm.h"
#include "sweep_common.h"

namespace qsvm {
namespace {

constexpr double kPiD = 3.14159265358979323846;

constexpr int kLogTileAmps = 11;
constexpr int kTileAmps = 1 << kLogTileAmps;  // amplitudes per LDS tile (32 KB)

// The phase splits over the low L = min(n, 11) bits and the rest:
//     Phi(b) = Phi_lo(b mod 2^L) + Phi_hi(b >> L) + theta_{L-1} (b_{L-1} XOR b_L),
// Phi_lo holding the terms of qubits below L (and the pairs inside them),
// Phi_hi those of qubits L and up.  Per point two tables hold
//     lo[l]        = 2^(-n/2) exp(i Phi_lo(l)),                      l < 2^L,
//     hi[2 h + t]  = exp(i (Phi_hi(h) + theta_{L-1} (t XOR h_0))),  h < 2^(n-L),
// so that 2^(-n/2) exp(i Phi(b)) = lo[b mod 2^L] hi[b >> (L-1)]  (for n = L
// the boundary term is absent and hi = {1, 1}).  Each entry is one FP64
// angle sum and one sincos.
__host__ __device__ inline int32_t low_bits(int32_t n) { return n < kLogTileAmps ? n : kLogTileAmps; }
__host__ __device__ inline int64_t table_size(int32_t n) {
  return (int64_t(1) << low_bits(n)) + (int64_t(2) << (n - low_bits(n)));
}

__device__ __forceinline__ double zz_theta(const double* __restrict__ x, int k) {
  return 2.0 * (kPiD - x[k]) * (kPiD - x[k + 1]);
}

__global__ void __launch_bounds__(256)
sv_table_kernel(const double* __restrict__ X, int64_t N, int32_t n, double2* __restrict__ tab) {
  const int32_t L = low_bits(n);
  const int64_t TS = table_size(n), lo_size = int64_t(1) << L;
  const double scale = exp2(-0.5 * double(n));
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < N * TS; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t p = t / TS, e = t - p * TS;
    const double* x = X + p * n;
    double ph = 0.0, amp = 1.0;
    if (e < lo_size) {
      for (int k = 0; k < L; ++k) {
        const int bk = int((e >> k) & 1);
        if (bk) ph += 2.0 * x[k];
        if (k + 1 < L && (bk ^ int((e >> (k + 1)) & 1))) ph += zz_theta(x, k);
      }
      amp = scale;
    } else if (n > L) {
      const int64_t u = e - lo_size, h = u >> 1;
      const int tb = int(u & 1);  // bit L-1 of b
      if (tb ^ int(h & 1)) ph += zz_theta(x, L - 1);
      for (int k = L; k < n; ++k) {
        const int bk = int((h >> (k - L)) & 1);
        if (bk) ph += 2.0 * x[k];
        if (k + 1 < n && (bk ^ int((h >> (k + 1 - L)) & 1))) ph += zz_theta(x, k);
      }
    }
    double sn, cs;
    sincos(ph, &sn, &cs);
    tab[t] = make_double2(cs * amp, sn * amp);
  }
}

// 2^(-n/2) exp(i Phi(b)) from the point's tables.
__device__ __forceinline__ double2 phase_of(const double2* __restrict__ tab, int32_t L, int64_t b) {
  const double2 l = tab[b & ((int64_t(1) << L) - 1)];
  const double2 h = tab[(int64_t(1) << L) + (b >> (L - 1))];
  return make_double2(fma(l.x, h.x, -(l.y * h.y)), fma(l.x, h.y, l.y * h.x));
}

// One pass over every state, in LDS tiles: the unnormalised Walsh-Hadamard
// transform on bits [s, s + G), optionally preceded by GEN (the tile is the
// first repetition's state 2^(-n/2) exp(i Phi(b)), computed instead of read)
// and followed by FUSE (each amplitude multiplied by 2^(-n/2) exp(i Phi(b))).
// `stages` is G, or 0 for a pass that only generates the first state.
// A tile is 2^G rows (the bits of the pass) x 2^LC consecutive columns (the
// indices below bit s, LC <= s), row u / column c at
// b = h 2^(s+G) + u 2^s + cg 2^LC + c, so global accesses run over 2^LC
// contiguous amplitudes.  Blocks stride over the N 2^n / 2^(G+LC) tiles.
template <bool GEN, bool FUSE>
__global__ void __launch_bounds__(256)
sv_pass_kernel(const double2* __restrict__ tab, int64_t N, int32_t n, int32_t s, int32_t G, int32_t LC,
               int32_t stages, double2* __restrict__ sv) {
  __shared__ double2 t_[kTileAmps];
  const int T = 1 << (G + LC);                       // amplitudes per tile (<= kTileAmps)
  const int cmask = (1 << LC) - 1;
  const int32_t log_tpp = n - G - LC;                // log2 tiles per point
  const int32_t log_groups = s - LC;                 // log2 column groups below bit s
  const int64_t total = N << log_tpp;
  const int32_t L = low_bits(n);
  const int64_t TS = table_size(n);
  for (int64_t tl = blockIdx.x; tl < total; tl += gridDim.x) {  // block-uniform
    const int64_t p = tl >> log_tpp;
    const int64_t tile = tl & ((int64_t(1) << log_tpp) - 1);
    const int64_t cg = tile & ((int64_t(1) << log_groups) - 1), h = tile >> log_groups;
    const int64_t base = (h << (s + G)) + (cg << LC);
    const double2* tp = tab + p * TS;
    double2* psi = sv + (p << n);
    auto amp_index = [&](int idx) { return base + (int64_t(idx >> LC) << s) + (idx & cmask); };

    for (int idx = threadIdx.x; idx < T; idx += 256) {
      const int64_t bi = amp_index(idx);
      t_[idx] = GEN ? phase_of(tp, L, bi) : psi[bi];
    }
    for (int g = 0; g < stages; ++g) {
      __syncthreads();
      for (int q = threadIdx.x; q < T / 2; q += 256) {
        const int c = q & cmask, ur = q >> LC;
        const int u0 = ((ur >> g) << (g + 1)) | (ur & ((1 << g) - 1));
        const int i0 = (u0 << LC) + c, i1 = ((u0 | (1 << g)) << LC) + c;
        const double2 a = t_[i0], d = t_[i1];
        t_[i0] = make_double2(a.x + d.x, a.y + d.y);
        t_[i1] = make_double2(a.x - d.x, a.y - d.y);
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < T; idx += 256) {
      const int64_t bi = amp_index(idx);
      double2 v = t_[idx];
      if (FUSE) {
        const double2 f = phase_of(tp, L, bi);
        v = make_double2(fma(f.x, v.x, -(f.y * v.y)), fma(f.x, v.y, f.y * v.x));
      }
      psi[bi] = v;
    }
    __syncthreads();  // the tile buffer is reused by the next tile
  }
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
// Two waves per SIMD: with the 3M product's three accumulator sets (170
// VGPRs) this measured faster than three waves, where 2 registers spill
// (at 20 qubits, 512 points: 20.4 vs 21.1 ms; the four-product form at three
// waves, 130 VGPRs: 23.1 ms).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
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

  // 3M form of the complex product A conj(B): P1 = Ar Br, P2 = Ai Bi and
  // P3 = (Ar + Ai)(Br - Bi) give re = P1 + P2 and im = P3 - P1 + P2, three
  // real MFMA products instead of four.
  dvec4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) {
      p1[mi][nj] = dvec4{0.0, 0.0, 0.0, 0.0};
      p2[mi][nj] = dvec4{0.0, 0.0, 0.0, 0.0};
      p3[mi][nj] = dvec4{0.0, 0.0, 0.0, 0.0};
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
      const double sa[2] = {fa[0].x + fa[0].y, fa[1].x + fa[1].y};
      const double db[2] = {fb[0].x - fb[0].y, fb[1].x - fb[1].y};
      // the twelve accumulators are visited in turn, so no MFMA waits on the
      // one just issued
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
          p1[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi].x, fb[nj].x, p1[mi][nj], 0, 0, 0);
          p2[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi].y, fb[nj].y, p2[mi][nj], 0, 0, 0);
          p3[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[mi], db[nj], p3[mi][nj], 0, 0, 0);
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
        const double q1 = p1[mi][nj][v], q2 = p2[mi][nj][v];
        const double gr = q1 + q2, gi = (p3[mi][nj][v] - q1) + q2;
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
  double2* st = static_cast<double2*>(sv);
  // passes of one full transform: the low bits as whole contiguous tiles,
  // then the remaining bits in the fewest groups of at most 9 bits, balanced
  // in size, each over tiles of 2^11 amplitudes (2^(11-G) contiguous columns)
  struct Pass { int s, G, LC; };
  Pass passes[8];
  int np = 0;
  {
    const int g0 = low_bits(n);
    passes[np++] = {0, g0, 0};
    const int rest = n - g0;
    const int groups = (rest + 8) / 9;
    for (int q = 0, s = g0; q < groups; ++q) {
      const int g = (n - s + (groups - q) - 1) / (groups - q);
      passes[np++] = {s, g, kLogTileAmps - g};  // kLogTileAmps - g <= s since s >= 11
      s += g;
    }
  }
  // the phase tables live in a stream-ordered temporary
  const int64_t tab_entries = N * table_size(n);
  double2* tab = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&tab), size_t(tab_entries) * sizeof(double2), stream);
  if (e != hipSuccess) return e;
  {
    const int64_t blocks = (tab_entries + 255) / 256;
    hipLaunchKernelGGL(sv_table_kernel, dim3(unsigned(blocks < kMaxGridBlocks ? blocks : kMaxGridBlocks / 8 * 8)),
                       dim3(256), 0, stream, X, N, n, tab);
    e = hipGetLastError();
  }
  auto launch = [&](const Pass& pa, bool gen, bool fuse, int stages) {
    const int64_t tiles = N << (n - pa.G - pa.LC);
    const int64_t blocks = tiles < kMaxGridBlocks ? tiles : kMaxGridBlocks / 8 * 8;
    const dim3 grid{unsigned(blocks)};
    if (gen && fuse)
      hipLaunchKernelGGL((sv_pass_kernel<true, true>), grid, dim3(256), 0, stream, tab, N, n, pa.s, pa.G, pa.LC,
                         stages, st);
    else if (gen)
      hipLaunchKernelGGL((sv_pass_kernel<true, false>), grid, dim3(256), 0, stream, tab, N, n, pa.s, pa.G, pa.LC,
                         stages, st);
    else if (fuse)
      hipLaunchKernelGGL((sv_pass_kernel<false, true>), grid, dim3(256), 0, stream, tab, N, n, pa.s, pa.G, pa.LC,
                         stages, st);
    else
      hipLaunchKernelGGL((sv_pass_kernel<false, false>), grid, dim3(256), 0, stream, tab, N, n, pa.s, pa.G, pa.LC,
                         stages, st);
    return hipGetLastError();
  };
  if (e == hipSuccess) {
    if (reps == 1) {
      // the first repetition alone: write the phase state (no transform)
      e = launch(passes[0], true, false, 0);
    } else {
      // repetitions 2..reps: transform then phase; the first repetition's
      // state is generated inside the first pass instead of being written and
      // read back
      for (int l = 2; l <= reps && e == hipSuccess; ++l)
        for (int q = 0; q < np && e == hipSuccess; ++q)
          e = launch(passes[q], l == 2 && q == 0, q == np - 1, passes[q].G);
    }
  }
  const hipError_t f = hipFreeAsync(tab, stream);
  return e != hipSuccess ? e : f;
}

namespace {

// Blocks of sv_gram_kernel resident on the current device at once (compute
// units x blocks per unit), cached per device.
hipError_t resident_gram_blocks(int64_t* out) {
  static std::atomic<int64_t> cache[64];  // zero-initialised (static storage)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < 64) {
    const int64_t c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) {
      *out = c;
      return hipSuccess;
    }
  }
  int cus = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sv_gram_kernel, 256, 0);
  if (e != hipSuccess) return e;
  const int64_t r = int64_t(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  if (dev >= 0 && dev < 64) cache[dev].store(r, std::memory_order_relaxed);  // the same value from any thread
  *out = r;
  return hipSuccess;
}

// Split count for `tiles` output tiles over an inner dimension of D values:
// the count s that minimises the run time in units of one unsplit tile,
// ceil(tiles s / resident) / s, i.e. that fills the rounds of resident blocks
// best; a larger count must gain 3 %.  At least 256 values (16 LDS stages)
// per split, and at most kMaxPartialTiles partial tiles (256 MB of workspace).
constexpr int64_t kMaxPartialTiles = 4096;
int64_t choose_splits(int64_t tiles, int64_t D, int64_t resident) {
  const int64_t smax = D / 256 < 1 ? 1 : D / 256;
  int64_t best = 1;
  double best_t = double((tiles + resident - 1) / resident);
  for (int64_t s = 2; s <= smax && tiles * s <= kMaxPartialTiles; ++s) {
    const double t = double((tiles * s + resident - 1) / resident) / double(s);
    if (t < best_t * 0.97) {
      best_t = t;
      best = s;
    }
  }
  return best;
}

// One launch (plus its split-K reduction) over the tiles of `a`.
hipError_t sv_gram_chunk(SweepArgs a, const void* sv_a, const void* sv_b, int32_t n, hipStream_t stream) {
  const int64_t tiles = launch_tiles(a);
  if (tiles <= 0) return hipSuccess;
  const int64_t D = int64_t(1) << n;
  int64_t resident = 0;
  hipError_t e0 = resident_gram_blocks(&resident);
  if (e0 != hipSuccess) return e0;
  int64_t splits = choose_splits(tiles, D, resident);
  const int64_t kchunk = ((D + splits - 1) / splits + kKB - 1) / kKB * kKB;
  splits = (D + kchunk - 1) / kchunk;
  const int64_t blocks = tiles * splits;  // <= kMaxPartialTiles when split
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

}  // namespace

hipError_t launch_sv_gram(const SweepArgs& a0, const void* sv_a, const void* sv_b, int32_t n, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = 1;
  return launch_chunked(a, 1, [&](const SweepArgs& c) { return sv_gram_chunk(c, sv_a, sv_b, n, stream); });
}

}  // namespace qsvm
