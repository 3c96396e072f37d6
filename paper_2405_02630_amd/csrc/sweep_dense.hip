// Dense sweep: <psi(y)|psi(x)> from the dense site tensors of Section D.
//
// Generic MPS overlap in the fixed left-to-right order (the single
// contraction path Alg. 2 reuses for every pair): starting from E = e_0 e_0^T,
// for every site
//     E'[b'][b] = [top(b') = top(b)] sum_a' conj(B[a'][b']) sum_{a: top(a) = top(a')} E[a'][a] A[a][b],
// i.e. E <- sum_s B_s^dagger E A_s with the physical index s = top bit of the
// bond index, and the amplitude is the sum of all entries of the final E (the
// all-ones right boundary).  E keeps only its chi^2/2 entries with equal top
// bits; one site costs chi^3 complex multiply-adds.  Unlike the butterfly
// sweep, nothing here assumes the closed-form structure of the tensors.
//
// Work layout: one pair per lane; a wave owns one ket point (wave-uniform:
// its tensor arrives by scalar/broadcast loads) and 64 bra points.  Each
// lane reads its bra tensor once per site, column by column:
//     V[a] = sum_a' conj(B[a'][b']) E[a'][a]      (chi^2/2 multiply-adds)
//     E'[b'][b] = sum_a V[a] A[a][b]               (chi^2/2 multiply-adds)
// E is renormalised by powers of two every `renorm_every` sites as in the
// butterfly sweep; the final |amp|^2 is formed in FP64.

#include "sweep_common.h"

namespace qsvm {
namespace {

__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {  // acc + a b
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}

__device__ __forceinline__ float2 cmac_conj(float2 acc, float2 a, float2 b) {  // acc + conj(a) b
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
  return acc;
}

template <int R>
__global__ void __launch_bounds__(256)
sweep_dense_kernel(SweepArgs a) {
  constexpr int CHI = 1 << R;
  constexpr int H = CHI / 2;  // entries per top-bit block
  const uint32_t L = xcd_logical_block();
  if (L >= a.num_blocks) return;
  const uint32_t tile = L / uint32_t(a.blocks_per_tile);
  const uint32_t sub = L % uint32_t(a.blocks_per_tile);
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t j = int64_t(tj) * kTile + lane;
  const int64_t i = int64_t(ti) * kTile + int64_t(sub) * 4 + wave;  // wave-uniform

  const bool active = pair_active(a, i, j);
  const bool comp = pair_computed(a, i, j);
  if (!__builtin_amdgcn_ballot_w64(active)) return;
  const int64_t jc = (j < a.Nb) ? j : a.Nb - 1;
  const int64_t ic = (i < a.Na) ? i : a.Na - 1;

  // E[a'][a] for top(a') == top(a): block t, e[t][a'_low][a_low]
  float2 e[2][H][H];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int p = 0; p < H; ++p)
#pragma unroll
      for (int q = 0; q < H; ++q) e[t][p][q] = make_float2(0.0f, 0.0f);
  e[0][0][0] = make_float2(1.0f, 0.0f);
  int32_t acc = 0;

  if (__builtin_amdgcn_ballot_w64(comp)) {
    int countdown = a.renorm_every;
    for (int k = 0; k < a.n; ++k) {
      const float2* __restrict__ A = a.dense_a + (int64_t(k) * a.Na + ic) * (CHI * CHI);
      const float2* __restrict__ B = a.dense_b + (int64_t(k) * a.Nb + jc) * (CHI * CHI);
      float2 en[2][H][H];
#pragma unroll
      for (int bp = 0; bp < CHI; ++bp) {  // column b' of B
        float2 bcol[CHI];
#pragma unroll
        for (int ap = 0; ap < CHI; ++ap) bcol[ap] = B[ap * CHI + bp];
        // V[a] = sum_{a'} conj(B[a'][b']) E[a'][a], top(a') = top(a)
        float2 vv[CHI];
#pragma unroll
        for (int aa = 0; aa < CHI; ++aa) {
          const int t = aa / H, aq = aa % H;
          float2 s = make_float2(0.0f, 0.0f);
#pragma unroll
          for (int ap = 0; ap < H; ++ap) s = cmac_conj(s, bcol[t * H + ap], e[t][ap][aq]);
          vv[aa] = s;
        }
        // E'[b'][b] = sum_a V[a] A[a][b] for top(b) = top(b')
        const int tb = bp / H, bq = bp % H;
#pragma unroll
        for (int bl = 0; bl < H; ++bl) {
          const int b = tb * H + bl;
          float2 s = make_float2(0.0f, 0.0f);
#pragma unroll
          for (int aa = 0; aa < CHI; ++aa) s = cmac(s, vv[aa], A[aa * CHI + b]);
          en[tb][bq][bl] = s;
        }
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int p = 0; p < H; ++p)
#pragma unroll
          for (int q = 0; q < H; ++q) e[t][p][q] = en[t][p][q];
      if (--countdown == 0) {
        float m = 0.0f;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int p = 0; p < H; ++p)
#pragma unroll
            for (int q = 0; q < H; ++q) m = fmaxf(m, fmaxf(fabsf(e[t][p][q].x), fabsf(e[t][p][q].y)));
        const int ex = __builtin_amdgcn_frexp_expf(m);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int p = 0; p < H; ++p)
#pragma unroll
            for (int q = 0; q < H; ++q) {
              e[t][p][q].x = __builtin_amdgcn_ldexpf(e[t][p][q].x, -ex);
              e[t][p][q].y = __builtin_amdgcn_ldexpf(e[t][p][q].y, -ex);
            }
        acc += ex;
        countdown = a.renorm_every;
      }
    }
  }

  if (!active) return;
  double s2 = 1.0;
  if (comp) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int p = 0; p < H; ++p)
#pragma unroll
        for (int q = 0; q < H; ++q) {
          sr += double(e[t][p][q].x);
          si += double(e[t][p][q].y);
        }
    s2 = fma(sr, sr, si * si);
  }
  store_entry(a, i, j, s2, 2 * acc);
}

template <int R>
hipError_t launch_r(const SweepArgs& a0, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = kTile / 4;
  return launch_chunked(a, a.blocks_per_tile, [&](SweepArgs c) {
    const int64_t blocks = launch_tiles(c) * c.blocks_per_tile;
    if (blocks <= 0) return hipSuccess;
    c.num_blocks = uint32_t(blocks);
    const uint32_t padded = uint32_t((blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((sweep_dense_kernel<R>), dim3(padded), dim3(256), 0, stream, c);
    return hipGetLastError();
  });
}

}  // namespace

hipError_t launch_sweep_dense_args(const SweepArgs& a, int32_t reps, hipStream_t stream) {
  switch (reps) {
    case 1: return launch_r<1>(a, stream);
    case 2: return launch_r<2>(a, stream);
    case 3: return launch_r<3>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qsvm
