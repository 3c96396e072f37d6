// Butterfly sweep: <psi(y)|psi(x)> for every pair of a tile, from the
// gauge generators of Section G (layout in include/qsvm.h).
//
// The overlap of two MPS is the left-to-right environment recursion
// E <- sum_s B_s^dagger E A_s (the contraction Alg. 2 repeats per pair, in
// the one fixed order that is optimal for a chain).  E is indexed by the
// bond states (c, c') of ket and bra; the physical index forces the top bit
// of c and c' to agree, so E has 2^(2r-1) entries.  In the diagonal gauge of
// Section G each site tensor is sgn(new) * prod_l C[new_l][old_l] with
// C = [[1, a], [1, b]] (times 2^(-r/2), kept in the exponent), so one site
// step is a sequence of 2x2 butterflies, one per bit axis:
//   ket bit axes l < r : (u0, u1) -> (u0 + a_x u1, u0 + b_x u1)
//   bra bit axes l < r : (u0, u1) -> (u0 + conj(a_y) u1, u0 + conj(b_y) u1)
//   shared top bit     : (u0, u1) -> (u0 + a_x conj(a_y) u1, u0 + b_x conj(b_y) u1)
// followed by the sign pattern (-1)^(sum_l c_l c_{l-1} + same for c'), folded
// into the second output of each butterfly.  That is (2r-1) 2^(2r-2) * 2
// complex multiply-adds per site instead of the chi^3 of the dense update.
//
// Work layout: a tile is 64 ket points x 64 bra points.  A wave owns PI ket
// points (wave-uniform, their generators come through scalar loads) and 64
// bra points (one per lane), and keeps the PI environments of its lane in
// VGPRs for the whole chain.  A block is 4 waves on consecutive ket groups of
// one tile.  Every `renorm_every` sites the environment is divided by the
// power of two nearest its largest component (exact) and the exponent added
// to an integer log2 accumulator.  The final closure with the right boundary
// g^|c| conj(g')^|c'| and |amp|^2 are formed in FP64.

#pragma once

#include "sweep_common.h"

namespace qsvm {
namespace {

// t0 = u0 + (ar + i ai) u1 ; t1 = u0 + (br + i bi) u1 ; u1 <- NEG ? -t1 : t1
template <bool NEG>
__device__ __forceinline__ void bfly(float2& u0, float2& u1, float ar, float ai, float br, float bi) {
  const float x0 = u0.x, y0 = u0.y, x1 = u1.x, y1 = u1.y;
  float t0r = fmaf(ar, x1, x0);
  t0r = fmaf(-ai, y1, t0r);
  float t0i = fmaf(ar, y1, y0);
  t0i = fmaf(ai, x1, t0i);
  float t1r, t1i;
  if (NEG) {
    t1r = fmaf(-br, x1, -x0);
    t1r = fmaf(bi, y1, t1r);
    t1i = fmaf(-br, y1, -y0);
    t1i = fmaf(-bi, x1, t1i);
  } else {
    t1r = fmaf(br, x1, x0);
    t1r = fmaf(-bi, y1, t1r);
    t1i = fmaf(br, y1, y0);
    t1i = fmaf(bi, x1, t1i);
  }
  u0 = make_float2(t0r, t0i);
  u1 = make_float2(t1r, t1i);
}

template <int R>
struct Layout {
  static constexpr int NB = 2 * R - 1;      // index bits of the environment
  static constexpr int M = 1 << NB;         // environment entries
  static constexpr int S = NB - 1;          // shared top (physical) bit
  __host__ __device__ static constexpr int ket_bit(int l) { return l - 1; }          // l = 1..R-1
  __host__ __device__ static constexpr int bra_bit(int l) { return R - 1 + l - 1; }  // l = 1..R-1
};

// One bit axis over an environment (or a lane's part of one) of M entries.
template <int AXBIT, int SIGNBIT, int SIGNBIT2, int M>
__device__ __forceinline__ void axis(float2 (&v)[M], float ar, float ai, float br, float bi) {
#pragma unroll
  for (int i0 = 0; i0 < M; ++i0) {
    if (i0 & (1 << AXBIT)) continue;
    const int i1 = i0 | (1 << AXBIT);
    bool neg = false;
    if constexpr (SIGNBIT >= 0) neg ^= ((i0 >> SIGNBIT) & 1) != 0;
    if constexpr (SIGNBIT2 >= 0) neg ^= ((i0 >> SIGNBIT2) & 1) != 0;
    if (neg)
      bfly<true>(v[i0], v[i1], ar, ai, br, bi);
    else
      bfly<false>(v[i0], v[i1], ar, ai, br, bi);
  }
}

// Ket axes and bra axes for l = 1..R-1 (compile-time recursion).  They act
// on index bits below the shared bit only, so the same code serves the whole
// environment (M = 2^(2R-1)) and a lane's half of it split on the shared bit.
template <int R, int L>
struct Axes {
  template <int M>
  __device__ __forceinline__ static void ket(float2 (&v)[M], const float4& c) {
    if constexpr (L <= R - 1) {
      axis<Layout<R>::ket_bit(L), (L >= 2 ? Layout<R>::ket_bit(L - 1) : -1), -1>(v, c.x, c.y, c.z, c.w);
      Axes<R, L + 1>::ket(v, c);
    }
  }
  template <int M>
  __device__ __forceinline__ static void bra(float2 (&v)[M], const float4& c) {
    if constexpr (L <= R - 1) {
      axis<Layout<R>::bra_bit(L), (L >= 2 ? Layout<R>::bra_bit(L - 1) : -1), -1>(v, c.x, -c.y, c.z, -c.w);
      Axes<R, L + 1>::bra(v, c);
    }
  }
};

template <int R>
__device__ __forceinline__ void site_step(float2 (&v)[Layout<R>::M], const float4& cx, const float4& cy) {
  Axes<R, 1>::ket(v, cx);
  Axes<R, 1>::bra(v, cy);
  // shared top bit: coefficients a_x conj(a_y), b_x conj(b_y)
  const float asr = fmaf(cx.x, cy.x, cx.y * cy.y);
  const float asi = fmaf(cx.y, cy.x, -(cx.x * cy.y));
  const float bsr = fmaf(cx.z, cy.z, cx.w * cy.w);
  const float bsi = fmaf(cx.w, cy.z, -(cx.z * cy.w));
  constexpr int SB1 = (R >= 2) ? Layout<R>::ket_bit(R - 1) : -1;
  constexpr int SB2 = (R >= 2) ? Layout<R>::bra_bit(R - 1) : -1;
  axis<Layout<R>::S, SB1, SB2>(v, asr, asi, bsr, bsi);
}

// max(|a|, |b|, |c|) in one instruction (source modifiers take the absolute
// values; the inputs are finite, so no NaN handling is needed).
__device__ __forceinline__ float absmax3(float a, float b, float c) {
  float r;
  asm("v_max3_f32 %0, |%1|, |%2|, |%3|" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Largest |component| of the M entries (a tree of three-input maxima).
template <int M>
__device__ __forceinline__ float absmax(const float2 (&v)[M]) {
  constexpr int F = 2 * M;  // real components
  float f[F];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    f[2 * q] = v[q].x;
    f[2 * q + 1] = v[q].y;
  }
  // largest |component|: a tree of three-input maxima
  constexpr int P = (F + 2) / 3;
  float part[P];
#pragma unroll
  for (int t = 0; t < P; ++t)
    part[t] = absmax3(f[3 * t], f[3 * t + 1 < F ? 3 * t + 1 : F - 1], f[3 * t + 2 < F ? 3 * t + 2 : F - 1]);
  float m = part[0];
#pragma unroll
  for (int t = 1; t < P; t += 2) m = absmax3(m, part[t], part[t + 1 < P ? t + 1 : P - 1]);
  return m;
}

// Divide the entries by 2^e, e the exponent of m (m = f 2^e, f in [0.5, 1);
// e = 0 for m = 0); returns e.
template <int M>
__device__ __forceinline__ int rescale(float2 (&v)[M], float m) {
  const int e = __builtin_amdgcn_frexp_expf(m);
  // v * 2^-e, exact; ldexp per component stays correct even where 2^-e alone
  // would not be representable
#pragma unroll
  for (int q = 0; q < M; ++q) {
    v[q].x = __builtin_amdgcn_ldexpf(v[q].x, -e);
    v[q].y = __builtin_amdgcn_ldexpf(v[q].y, -e);
  }
  return e;
}

template <int R>
__device__ __forceinline__ int renorm(float2 (&v)[Layout<R>::M]) {
  return rescale(v, absmax(v));
}

// Sign of a bond column: (-1)^(sum_{l=1}^{r-1} c_l c_{l-1}) over the bits
// (c_0 .. c_{r-2} from `low`, c_{r-1} = s).
template <int R>
__device__ __forceinline__ constexpr int col_sign_parity(int low, int s) {
  const int c = low | (s << (R - 1));
  return __builtin_popcount(c & (c >> 1)) & 1;
}

template <int R>
__device__ __forceinline__ void init_env(float2 (&v)[Layout<R>::M]) {
  constexpr int M = Layout<R>::M;
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int ket = q & LOWMASK;
    const int bra = (q >> (R - 1)) & LOWMASK;
    const int s = (q >> Layout<R>::S) & 1;
    const int par = col_sign_parity<R>(ket, s) ^ col_sign_parity<R>(bra, s);
    v[q] = make_float2(par ? -1.0f : 1.0f, 0.0f);
  }
}

// |sum_q g_x^|c| conj(g_y)^|c'| v[q]|^2 in FP64 (every product-sum written as
// an explicit fma, so the result is the same in every kernel variant).
template <int R>
__device__ __forceinline__ double closure(const float2 (&v)[Layout<R>::M], float4 gx4, float4 gy4) {
  constexpr int M = Layout<R>::M;
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
  double pxr[R + 1], pxi[R + 1], pyr[R + 1], pyi[R + 1];
  pxr[0] = 1.0; pxi[0] = 0.0; pyr[0] = 1.0; pyi[0] = 0.0;
  const double gxr = gx4.x, gxi = gx4.y, gyr = gy4.x, gyi = -double(gy4.y);  // conj(g_y)
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    pxr[m] = fma(pxr[m - 1], gxr, -(pxi[m - 1] * gxi));
    pxi[m] = fma(pxr[m - 1], gxi, pxi[m - 1] * gxr);
    pyr[m] = fma(pyr[m - 1], gyr, -(pyi[m - 1] * gyi));
    pyi[m] = fma(pyr[m - 1], gyi, pyi[m - 1] * gyr);
  }
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int s = (q >> Layout<R>::S) & 1;
    const int hk = __builtin_popcount(q & LOWMASK) + s;
    const int hb = __builtin_popcount((q >> (R - 1)) & LOWMASK) + s;
    const double wr = fma(pxr[hk], pyr[hb], -(pxi[hk] * pyi[hb]));
    const double wi = fma(pxr[hk], pyi[hb], pxi[hk] * pyr[hb]);
    const double vx = v[q].x, vy = v[q].y;
    sr = fma(wr, vx, fma(-wi, vy, sr));
    si = fma(wr, vy, fma(wi, vx, si));
  }
  return fma(sr, sr, si * si);
}

// One work item: the PI wave-uniform ket points i0 .. i0+PI-1 against the 64
// bra points j0 + lane, over all sites; writes their entries.
template <int R, int PI>
__device__ __forceinline__ void butterfly_item(const SweepArgs& a, int64_t i0, int64_t j0) {
  constexpr int M = Layout<R>::M;
  const int lane = threadIdx.x & 63;
  const int64_t j = j0 + lane;

  bool comp[PI];
  bool any_comp = false, any_active = false;
#pragma unroll
  for (int p = 0; p < PI; ++p) {
    comp[p] = pair_computed(a, i0 + p, j);
    any_comp |= comp[p];
    any_active |= pair_active(a, i0 + p, j);
  }
  if (!__builtin_amdgcn_ballot_w64(any_active)) return;  // wave has nothing to write

  const int64_t jc = (j < a.Nb) ? j : a.Nb - 1;  // clamp loads of idle lanes in bounds
  int64_t ic[PI];
#pragma unroll
  for (int p = 0; p < PI; ++p) ic[p] = (i0 + p < a.Na) ? i0 + p : a.Na - 1;

  float2 v[PI][M];
  int32_t acc[PI];
#pragma unroll
  for (int p = 0; p < PI; ++p) {
    init_env<R>(v[p]);
    acc[p] = 0;
  }

  const float4* __restrict__ gA = a.gen_a;
  const float4* __restrict__ gB = a.gen_b;
  // sites 1 .. n-1 (none for one qubit: the generator plane then holds only
  // site 0, so nothing is loaded beyond it)
  if (a.n > 1 && __builtin_amdgcn_ballot_w64(any_comp)) {
    int countdown = a.renorm_every;
    // one site: apply it to every environment, renormalise on schedule
    auto step = [&](const float4 (&cx)[PI], const float4& cy) {
#pragma unroll
      for (int p = 0; p < PI; ++p) site_step<R>(v[p], cx[p], cy);
      if (--countdown == 0) {
#pragma unroll
        for (int p = 0; p < PI; ++p) acc[p] += renorm<R>(v[p]);
        countdown = a.renorm_every;
      }
    };
    // generators of one site (clamped to the last site)
    auto load = [&](int k, float4 (&cx)[PI], float4& cy) {
      const int kc = (k < a.n) ? k : a.n - 1;
      cy = gB[int64_t(kc) * a.Nb + jc];
#pragma unroll
      for (int p = 0; p < PI; ++p) cx[p] = gA[int64_t(kc) * a.Na + ic[p]];
    };
    // two sites per iteration with ping-pong registers, so the prefetched
    // generators never have to be copied into the registers of the current site
    float4 cxA[PI], cxB[PI], cyA, cyB;
    load(1, cxA, cyA);
    int k = 1;
    for (; k + 1 < a.n; k += 2) {
      load(k + 1, cxB, cyB);
      step(cxA, cyA);
      load(k + 2, cxA, cyA);
      step(cxB, cyB);
    }
    if (k < a.n) step(cxA, cyA);  // last site when n - 1 is odd
  }

  // Epilogue one pair at a time (rolled loop over the ket points, rotating
  // the per-pair registers) so the FP64 closures do not all stay live at once.
  const float4 gy = gB[jc];
#pragma unroll 1
  for (int p = 0; p < PI; ++p) {
    const int64_t i = i0 + p;
    if (pair_active(a, i, j)) {
      const double s2 = comp[0] ? closure<R>(v[0], gA[ic[0]], gy) : 1.0;
      // amp = closure * 2^(acc - R n)  =>  K = s2 * 2^(2 (acc - R n))
      store_entry(a, i, j, s2, 2 * (acc[0] - R * a.n));
    }
#pragma unroll
    for (int q = 0; q + 1 < PI; ++q) {
#pragma unroll
      for (int e = 0; e < M; ++e) v[q][e] = v[q + 1][e];
      acc[q] = acc[q + 1];
      comp[q] = comp[q + 1];
      ic[q] = ic[q + 1];
    }
  }
}

}  // namespace
}  // namespace qsvm
