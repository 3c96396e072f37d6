// Butterfly sweep with each pair's environment split across L = 2^(2r-7)
// lanes, for bond dimensions whose environment does not fit one lane's
// registers: reps = 4 (chi = 16, 128 entries, 2 lanes), reps = 5 (chi = 32,
// 512 entries, 8 lanes) and reps = 6 (chi = 64, 2048 entries, 32 lanes).
// Every lane holds 64 entries.
//
// The recursion, gauge and butterflies are those of the one-lane sweep
// (sweep_butterfly_item.h).  The environment index has 2r-1 bits: ket bits
// for l = 1..r-1, bra bits for l = 1..r-1 and the shared (physical) bit.
// The entries of the ket and bra bits l = 1..3 are a lane's own (in-lane
// index q: ket bits 0..2, bra bits 3..5), so those six axes run inside each
// lane with the unchanged code.  The other 2r-7 bits select the lane within
// its group: lane bit 0 is the shared bit, bits 1..r-4 the ket bits
// l = 4..r-1, bits r-3..2r-8 the bra bits l = 4..r-1.  An axis on a lane bit
// pairs lane g (bit clear, holding u0) with lane g' = g ^ bit (holding u1):
//     (u0, u1) -> (u0 + alpha u1, sg (u0 + beta u1)),
// with (alpha, beta) = (a_x, b_x) for a ket axis, (conj a_y, conj b_y) for a
// bra axis and (a_x conj a_y, b_x conj b_y) for the shared one, and sg the
// sign pattern.  To give both lanes one instruction stream, a lane whose bit
// b is set stores its entries divided by a per-bit phase Phi_b (all lanes of
// a group divide by the product of the phases of their set bits).  With
// Phi_b' = beta Phi_b,
//     lane without the bit:  u0 <- u0 + (alpha Phi_b) p       (p = partner)
//     lane with the bit:     u~1 <- sg (u~1 + (1 / Phi_b') p),
// after which Phi_b <- Phi_b'.  Both lanes compute "own + c * partner" with
// their own coefficient c; the phases are carried in FP64 and multiply each
// lane's part of the closure at the end.  The partner's values come through
// the LDS crossbar (ds_swizzle, bit-mask mode with the xor mask of the lane
// bit), four or eight entries per wait, or by DPP moves: at reps 4 (two
// waves per SIMD, VALU-bound) the swizzles keep the exchange off the VALU,
// where DPP moves measured about 8 extra issue cycles each; at reps 5 and 6
// (one wave per SIMD, the exchange latency exposed) xor 1, 2 and 8 go by DPP
// (7-8 % faster; xor 4 as two row rotations and a select measured slower).  Renormalisation takes
// the largest of the group's maxima, so the group shares one power-of-two
// scale.  The closure reduces the group's FP64 partial sums over the lane
// bits in a fixed order, identical in every lane.
//
// Work layout: a tile is 64 ket x 64 bra points; a wave owns one ket point
// (wave-uniform, scalar loads) and P = 64 / L bra points (L lanes each); a
// block of 4 waves covers KPB ket points x 4 / KPB chunks of P bra points.

#include "../../include/qsvm.h"
#include "sweep_butterfly_item.h"

namespace qsvm {
namespace {

template <int R>
struct Split {
  static constexpr int C = 2 * R - 7;    // lane bits of a pair's group
  static constexpr int L = 1 << C;       // lanes per pair
  static constexpr int P = 64 / L;       // pairs per wave
  static constexpr int CH = kTile / P;   // bra chunks per tile row
  static constexpr int ML = 64;          // entries per lane
  static constexpr int kbit(int l) { return 1 + (l - 4); }      // lane bit of ket axis l >= 4
  static constexpr int bbit(int l) { return R - 3 + (l - 4); }  // lane bit of bra axis l >= 4
};

// ds_swizzle in bit-mask mode (and 0x1f, or 0, xor XM) for four complex
// entries, one wait for all eight values.  One asm block, so that the
// compiler cannot hoist the swizzles of a whole site ahead of their use (it
// does with the builtin, and the results then spill); the wait also covers
// any scalar loads still in flight.
#define QSVM_SWZ4(OFF)                                                                          \
  asm volatile("ds_swizzle_b32 %0, %8 offset:" OFF "\n"                                         \
               "ds_swizzle_b32 %1, %9 offset:" OFF "\n"                                         \
               "ds_swizzle_b32 %2, %10 offset:" OFF "\n"                                        \
               "ds_swizzle_b32 %3, %11 offset:" OFF "\n"                                        \
               "ds_swizzle_b32 %4, %12 offset:" OFF "\n"                                        \
               "ds_swizzle_b32 %5, %13 offset:" OFF "\n"                                        \
               "ds_swizzle_b32 %6, %14 offset:" OFF "\n"                                        \
               "ds_swizzle_b32 %7, %15 offset:" OFF "\n"                                        \
               "s_waitcnt lgkmcnt(0)"                                                           \
               : "=&v"(p[0]), "=&v"(p[1]), "=&v"(p[2]), "=&v"(p[3]), "=&v"(p[4]), "=&v"(p[5]), \
                 "=&v"(p[6]), "=&v"(p[7])                                                       \
               : "v"(v0.x), "v"(v0.y), "v"(v1.x), "v"(v1.y), "v"(v2.x), "v"(v2.y), "v"(v3.x), "v"(v3.y))

// Offsets: 0x1f | XM << 10 for XM = 1, 2, 4, 8, 16.
template <int XM>
__device__ __forceinline__ void swizzle4(const float2& v0, const float2& v1, const float2& v2, const float2& v3,
                                         float (&p)[8]) {
  if constexpr (XM == 1) QSVM_SWZ4("1055");
  else if constexpr (XM == 2) QSVM_SWZ4("2079");
  else if constexpr (XM == 4) QSVM_SWZ4("4127");
  else if constexpr (XM == 8) QSVM_SWZ4("8223");
  else QSVM_SWZ4("16415");
}
#undef QSVM_SWZ4

// The same for eight complex entries (sixteen swizzles, one wait).
#define QSVM_SWZ8(OFF)                                                                               \
  asm volatile("ds_swizzle_b32 %0, %16 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %1, %17 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %2, %18 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %3, %19 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %4, %20 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %5, %21 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %6, %22 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %7, %23 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %8, %24 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %9, %25 offset:" OFF "\n"                                            \
               "ds_swizzle_b32 %10, %26 offset:" OFF "\n"                                           \
               "ds_swizzle_b32 %11, %27 offset:" OFF "\n"                                           \
               "ds_swizzle_b32 %12, %28 offset:" OFF "\n"                                           \
               "ds_swizzle_b32 %13, %29 offset:" OFF "\n"                                           \
               "ds_swizzle_b32 %14, %30 offset:" OFF "\n"                                           \
               "ds_swizzle_b32 %15, %31 offset:" OFF "\n"                                           \
               "s_waitcnt lgkmcnt(0)"                                                                \
               : "=&v"(p[0]), "=&v"(p[1]), "=&v"(p[2]), "=&v"(p[3]), "=&v"(p[4]), "=&v"(p[5]),      \
                 "=&v"(p[6]), "=&v"(p[7]), "=&v"(p[8]), "=&v"(p[9]), "=&v"(p[10]), "=&v"(p[11]),    \
                 "=&v"(p[12]), "=&v"(p[13]), "=&v"(p[14]), "=&v"(p[15])                            \
               : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y),      \
                 "v"(v[3].x), "v"(v[3].y), "v"(v[4].x), "v"(v[4].y), "v"(v[5].x), "v"(v[5].y),      \
                 "v"(v[6].x), "v"(v[6].y), "v"(v[7].x), "v"(v[7].y))

template <int XM>
__device__ __forceinline__ void swizzle8(const float2* v, float (&p)[16]) {
  if constexpr (XM == 1) QSVM_SWZ8("1055");
  else if constexpr (XM == 2) QSVM_SWZ8("2079");
  else if constexpr (XM == 4) QSVM_SWZ8("4127");
  else if constexpr (XM == 8) QSVM_SWZ8("8223");
  else QSVM_SWZ8("16415");
}
#undef QSVM_SWZ8

// The value of x in lane ^ XM (a few values per site or per pair: the
// renormalisation maximum and the closure's partial sums).
template <int XM>
__device__ __forceinline__ float swz_xor(float x) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x1f | (XM << 10)));
}

template <int XM>
__device__ __forceinline__ double swz_xor(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_swizzle(int(uint32_t(b)), 0x1f | (XM << 10));
  const int hi = __builtin_amdgcn_ds_swizzle(int(uint32_t(uint64_t(b) >> 32)), 0x1f | (XM << 10));
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// Axis on lane bit b (xor mask XM = 2^b): v <- f(q) (v + c * partner(v)),
// with f(q) = f1 for the entries whose in-lane sign bits (IB1, IB2; -1 =
// none) have odd parity and f0 for the others.  The lane without the bit
// passes f0 = f1 = 1; the lane with it passes its sign pattern (f0 = the
// lane-bit part of the sign, f1 = -f0).  LANE_SIGN = false: f0 is 1 in every
// lane, so the even entries are not multiplied.
// x of lane l ^ XM for XM = 1, 2 (quad permutations) and 8 (rotation of a
// row of 16 by 8), a VALU move.
template <int XM>
__device__ __forceinline__ float dpp_xor(float x) {
  static_assert(XM == 1 || XM == 2 || XM == 8, "DPP covers xor 1, 2 and 8");
  constexpr int ctrl = XM == 1 ? 0xB1 : XM == 2 ? 0x4E : 0x128;  // quad_perm [1,0,3,2], [2,3,0,1]; row_ror:8
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, false));
}

// DP: the partner values of xor 1, 2 and 8 come by DPP (reps >= 5, one wave
// per SIMD: the exchange latency is exposed and the VALU has room), the
// others through ds_swizzle.
template <int XM, int IB1, int IB2, bool LANE_SIGN, int ML, int B = 4, bool DP = false>
__device__ __forceinline__ void cross_axis(float2 (&v)[ML], float cr, float ci, float f0, float f1) {
  constexpr bool dpp = DP && (XM == 1 || XM == 2 || XM == 8);
#pragma unroll
  for (int c = 0; c < ML / B; ++c) {
    float p[2 * B];
    if constexpr (dpp) {
#pragma unroll
      for (int e = 0; e < B; ++e) {
        p[2 * e] = dpp_xor<dpp ? XM : 1>(v[B * c + e].x);
        p[2 * e + 1] = dpp_xor<dpp ? XM : 1>(v[B * c + e].y);
      }
    } else if constexpr (B == 8) {
      swizzle8<XM>(&v[8 * c], p);
    } else {
      swizzle4<XM>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3], p);
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = B * c + e;
      const float pr = p[2 * e], pim = p[2 * e + 1];
      float tr = fmaf(cr, pr, v[q].x);
      tr = fmaf(-ci, pim, tr);
      float ti = fmaf(cr, pim, v[q].y);
      ti = fmaf(ci, pr, ti);
      int par = 0;
      if constexpr (IB1 >= 0) par ^= (q >> (IB1 < 0 ? 0 : IB1)) & 1;
      if constexpr (IB2 >= 0) par ^= (q >> (IB2 < 0 ? 0 : IB2)) & 1;
      if (par) {
        tr *= f1;
        ti *= f1;
      } else if constexpr (LANE_SIGN) {
        tr *= f0;
        ti *= f0;
      }
      v[q] = make_float2(tr, ti);
    }
  }
}

// FP64 coefficient of a cross axis for this lane, and the phase update:
// lane without the bit: alpha Phi; with it: 1 / (beta Phi); Phi <- beta Phi.
__device__ __forceinline__ void axis_coeff(bool upper, double ar, double ai, double br, double bi, double& phr,
                                           double& phi, float& cr, float& ci) {
  const double nr = fma(br, phr, -(bi * phi));
  const double ni = fma(br, phi, bi * phr);
  if (upper) {
    const double inv = 1.0 / fma(nr, nr, ni * ni);
    cr = float(nr * inv);
    ci = float(-ni * inv);
  } else {
    cr = float(fma(ar, phr, -(ai * phi)));
    ci = float(fma(ar, phi, ai * phr));
  }
  phr = nr;
  phi = ni;
}

// Closure of one lane: sum_q g_x^|c| conj(g_y)^|c'| v[q] over the in-lane
// bits (|c|, |c'| counted over ket and bra bits l = 1..3), in FP64.  The
// weight depends only on (|c|, |c'|), so the entries of each of the 4 x 4
// weight classes are summed first (in a fixed order) and each class sum is
// multiplied by its weight once.
template <int ML>
__device__ __forceinline__ void closure_lane(const float2 (&v)[ML], double gxr, double gxi, double gyr, double gyi,
                                             double& sr, double& si) {
  double pxr[4], pxi[4], pyr[4], pyi[4];
  pxr[0] = 1.0; pxi[0] = 0.0; pyr[0] = 1.0; pyi[0] = 0.0;
#pragma unroll
  for (int m = 1; m < 4; ++m) {
    pxr[m] = fma(pxr[m - 1], gxr, -(pxi[m - 1] * gxi));
    pxi[m] = fma(pxr[m - 1], gxi, pxi[m - 1] * gxr);
    pyr[m] = fma(pyr[m - 1], gyr, -(pyi[m - 1] * gyi));
    pyi[m] = fma(pyr[m - 1], gyi, pyi[m - 1] * gyr);
  }
  sr = 0.0;
  si = 0.0;
#pragma unroll
  for (int hk = 0; hk < 4; ++hk) {
#pragma unroll
    for (int hb = 0; hb < 4; ++hb) {
      double cr = 0.0, ci = 0.0;
#pragma unroll
      for (int q = 0; q < ML; ++q) {
        if (__builtin_popcount(q & 7) != hk || __builtin_popcount((q >> 3) & 7) != hb) continue;
        cr += double(v[q].x);
        ci += double(v[q].y);
      }
      const double wr = fma(pxr[hk], pyr[hb], -(pxi[hk] * pyi[hb]));
      const double wi = fma(pxr[hk], pyi[hb], pxi[hk] * pyr[hb]);
      sr = fma(wr, cr, fma(-wi, ci, sr));
      si = fma(wr, ci, fma(wi, cr, si));
    }
  }
}

// Group-wide maximum and sum over the lane bits b < NB (fixed order: the
// lane without the bit's value first, so every lane adds identically).
template <int NB>
__device__ __forceinline__ float group_max(float m) {
  if constexpr (NB >= 1) m = fmaxf(m, swz_xor<1>(m));
  if constexpr (NB >= 2) m = fmaxf(m, swz_xor<2>(m));
  if constexpr (NB >= 3) m = fmaxf(m, swz_xor<4>(m));
  if constexpr (NB >= 4) m = fmaxf(m, swz_xor<8>(m));
  if constexpr (NB >= 5) m = fmaxf(m, swz_xor<16>(m));
  return m;
}

template <int XM>
__device__ __forceinline__ void group_add_bit(double& sr, double& si, int g) {
  const double or_ = swz_xor<XM>(sr), oi = swz_xor<XM>(si);
  const bool hi = (g & XM) != 0;
  sr = hi ? or_ + sr : sr + or_;
  si = hi ? oi + si : si + oi;
}

template <int NB>
__device__ __forceinline__ void group_sum(double& sr, double& si, int g) {
  if constexpr (NB >= 1) group_add_bit<1>(sr, si, g);
  if constexpr (NB >= 2) group_add_bit<2>(sr, si, g);
  if constexpr (NB >= 3) group_add_bit<4>(sr, si, g);
  if constexpr (NB >= 4) group_add_bit<8>(sr, si, g);
  if constexpr (NB >= 5) group_add_bit<16>(sr, si, g);
}

// Cross ket axes l = L0..R-1 (compile-time recursion); the sign bit of axis
// l is ket bit l-1: in-lane bit 2 for l = 4, lane bit kbit(l-1) above.
template <int R, int L0>
struct CrossKet {
  __device__ __forceinline__ static void run(float2 (&v)[64], int g, const double (&a)[4], double (&phr)[8],
                                             double (&phi)[8]) {
    if constexpr (L0 <= R - 1) {
      constexpr int B = Split<R>::kbit(L0);
      const bool upper = (g >> B) & 1;
      float cr, ci;
      axis_coeff(upper, a[0], a[1], a[2], a[3], phr[B], phi[B], cr, ci);
      if constexpr (L0 == 4) {
        cross_axis<1 << B, 2, -1, false, 64, 8, true>(v, cr, ci, 1.0f, upper ? -1.0f : 1.0f);
      } else {
        const float f0 = (upper && ((g >> Split<R>::kbit(L0 - 1)) & 1)) ? -1.0f : 1.0f;
        cross_axis<1 << B, -1, -1, true, 64, 8, true>(v, cr, ci, f0, f0);
      }
      CrossKet<R, L0 + 1>::run(v, g, a, phr, phi);
    }
  }
};

template <int R, int L0>
struct CrossBra {
  __device__ __forceinline__ static void run(float2 (&v)[64], int g, const double (&a)[4], double (&phr)[8],
                                             double (&phi)[8]) {
    if constexpr (L0 <= R - 1) {
      constexpr int B = Split<R>::bbit(L0);
      const bool upper = (g >> B) & 1;
      float cr, ci;
      axis_coeff(upper, a[0], a[1], a[2], a[3], phr[B], phi[B], cr, ci);
      if constexpr (L0 == 4) {
        cross_axis<1 << B, 5, -1, false, 64, 8, true>(v, cr, ci, 1.0f, upper ? -1.0f : 1.0f);
      } else {
        const float f0 = (upper && ((g >> Split<R>::bbit(L0 - 1)) & 1)) ? -1.0f : 1.0f;
        cross_axis<1 << B, -1, -1, true, 64, 8, true>(v, cr, ci, f0, f0);
      }
      CrossBra<R, L0 + 1>::run(v, g, a, phr, phi);
    }
  }
};

// Initial environment of lane g: the sign pattern of its 64 entries.
template <int R>
__device__ __forceinline__ void init_split(float2 (&v)[64], int g) {
  int kl = 0, bl = 0;  // the lane's ket and bra bits l = 4..R-1 (as bond bits 3..R-2)
#pragma unroll
  for (int l = 4; l <= R - 1; ++l) {
    kl |= ((g >> Split<R>::kbit(l)) & 1) << (l - 1);
    bl |= ((g >> Split<R>::bbit(l)) & 1) << (l - 1);
  }
  const int s = g & 1;
#pragma unroll
  for (int q = 0; q < 64; ++q) {
    const int ket = (q & 7) | kl, bra = ((q >> 3) & 7) | bl;
    const int par = col_sign_parity<R>(ket, s) ^ col_sign_parity<R>(bra, s);
    v[q] = make_float2(par ? -1.0f : 1.0f, 0.0f);
  }
}

// One work item: ket point i against bra points j0 .. j0+P-1 (L lanes each).
template <int R>
__device__ __forceinline__ void split_item(const SweepArgs& a, int64_t i, int64_t j0) {
  using S = Split<R>;
  constexpr int C = S::C;
  const int lane = threadIdx.x & 63;
  const int g = lane & (S::L - 1);  // lane within the pair's group
  const int64_t j = j0 + (lane >> C);

  const bool comp = pair_computed(a, i, j);
  const bool active = pair_active(a, i, j);
  if (!__builtin_amdgcn_ballot_w64(active)) return;

  const int64_t jc = (j < a.Nb) ? j : a.Nb - 1;  // clamp loads of idle lanes in bounds
  const int64_t ic = (i < a.Na) ? i : a.Na - 1;

  float2 v[64];
  init_split<R>(v, g);
  int32_t acc = 0;
  double phr[8], phi[8];  // Phi_b of lane bit b (carried by every lane of the group)
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    phr[b] = 1.0;
    phi[b] = 0.0;
  }
  const bool up_s = g & 1;
  // sign of the shared axis in the lane with the bit: in-lane bits 2 and 5
  // (reps 4), else the lane's ket and bra bits l = R-1
  float fs = 1.0f;
  if constexpr (R >= 5)
    fs = (up_s && (((g >> S::kbit(R - 1)) ^ (g >> S::bbit(R - 1))) & 1)) ? -1.0f : 1.0f;

  const float4* __restrict__ gA = a.gen_a;
  const float4* __restrict__ gB = a.gen_b;
  // sites 1 .. n-1 (none for one qubit: the generator plane then holds only
  // site 0, so nothing is loaded beyond it)
  if (a.n > 1 && __builtin_amdgcn_ballot_w64(comp)) {
    int countdown = a.renorm_every;
    float4 cy = gB[a.Nb + jc];  // site 1
    float4 cx = gA[a.Na + ic];
    for (int k = 1; k < a.n; ++k) {
      const int kn = (k + 1 < a.n) ? k + 1 : k;
      const float4 cy_next = gB[int64_t(kn) * a.Nb + jc];
      const float4 cx_next = gA[int64_t(kn) * a.Na + ic];
      // coefficients in FP64 (products of FP32 values are exact there)
      const double xar = cx.x, xai = cx.y, xbr = cx.z, xbi = cx.w;
      const double yar = cy.x, yai = -double(cy.y), ybr = cy.z, ybi = -double(cy.w);  // conj(a_y), conj(b_y)
      Axes<4, 1>::ket(v, cx);
      if constexpr (R >= 5) {
        const double ka[4] = {xar, xai, xbr, xbi};
        CrossKet<R, 4>::run(v, g, ka, phr, phi);
      }
      Axes<4, 1>::bra(v, cy);
      if constexpr (R >= 5) {
        const double ba[4] = {yar, yai, ybr, ybi};
        CrossBra<R, 4>::run(v, g, ba, phr, phi);
      }
      // shared bit: a_x conj(a_y), b_x conj(b_y)
      {
        const double asr = fma(xar, yar, -(xai * yai)), asi = fma(xar, yai, xai * yar);
        const double bsr = fma(xbr, ybr, -(xbi * ybi)), bsi = fma(xbr, ybi, xbi * ybr);
        float cr, ci;
        axis_coeff(up_s, asr, asi, bsr, bsi, phr[0], phi[0], cr, ci);
        if constexpr (R == 4)
          cross_axis<1, 2, 5, false>(v, cr, ci, 1.0f, up_s ? -1.0f : 1.0f);
        else
          cross_axis<1, -1, -1, true, 64, 8, true>(v, cr, ci, fs, fs);
      }
      if (--countdown == 0) {
        acc += rescale(v, group_max<C>(absmax(v)));
        countdown = a.renorm_every;
      }
      cy = cy_next;
      cx = cx_next;
    }
  }

  // closure: the lane's in-lane sum, times g_x^h conj(g_y)^h' for its lane
  // bits (h, h' = ket, bra bits set among l >= 4, plus the shared bit) and
  // the phases of its set bits; then the group's sum
  const float4 gx4 = gA[ic];
  const float4 gy4 = gB[jc];
  const double gxr = gx4.x, gxi = gx4.y, gyr = gy4.x, gyi = -double(gy4.y);
  double sr, si;
  closure_lane<64>(v, gxr, gxi, gyr, gyi, sr, si);
  int hk = g & 1, hb = g & 1;
#pragma unroll
  for (int l = 4; l <= R - 1; ++l) {
    hk += (g >> S::kbit(l)) & 1;
    hb += (g >> S::bbit(l)) & 1;
  }
  double wr = 1.0, wi = 0.0;
#pragma unroll
  for (int m = 0; m < R - 2; ++m) {  // hk, hb <= R - 3
    if (m < hk) {
      const double t = fma(wr, gxr, -(wi * gxi));
      wi = fma(wr, gxi, wi * gxr);
      wr = t;
    }
    if (m < hb) {
      const double t = fma(wr, gyr, -(wi * gyi));
      wi = fma(wr, gyi, wi * gyr);
      wr = t;
    }
  }
#pragma unroll
  for (int b = 0; b < C; ++b)
    if ((g >> b) & 1) {
      const double t = fma(wr, phr[b], -(wi * phi[b]));
      wi = fma(wr, phi[b], wi * phr[b]);
      wr = t;
    }
  {
    const double tr = fma(sr, wr, -(si * wi));
    si = fma(sr, wi, si * wr);
    sr = tr;
  }
  group_sum<C>(sr, si, g);
  if (g == 0 && active) {
    const double s2 = comp ? fma(sr, sr, si * si) : 1.0;
    // amp = closure * 2^(acc - R n)  =>  K = s2 * 2^(2 (acc - R n))
    store_entry(a, i, j, s2, 2 * (acc - R * a.n));
  }
}

// KPB = ket points per block: a block's 4 waves cover KPB ket points x
// 4 / KPB chunks of P bra points (16 CH blocks per tile).  W = target waves
// per SIMD.
template <int R, int W, int KPB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8)))
sweep_split_kernel(SweepArgs a) {
  using S = Split<R>;
  const uint32_t Lb = xcd_logical_block();
  if (Lb >= a.num_blocks) return;
  const uint32_t tile = Lb / uint32_t(a.blocks_per_tile);
  const uint32_t sub = Lb % uint32_t(a.blocks_per_tile);
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int CPB = 4 / KPB;           // chunks per block
  constexpr int BPR = S::CH / CPB;       // blocks per ket group of the tile
  const int64_t ket = int64_t(sub / BPR) * KPB + wave / CPB;
  const int64_t chunk = int64_t(sub % BPR) * CPB + wave % CPB;
  split_item<R>(a, int64_t(ti) * kTile + ket, int64_t(tj) * kTile + chunk * S::P);
}

template <int R, int W, int KPB>
hipError_t launch_split(const SweepArgs& a0, hipStream_t stream) {
  static_assert(Split<R>::CH * KPB >= 4, "a block needs 4 / KPB chunks");
  SweepArgs a = a0;
  a.blocks_per_tile = split_blocks_per_tile(R);
  return launch_chunked(a, a.blocks_per_tile, [&](SweepArgs c) {
    const int64_t blocks = launch_tiles(c) * c.blocks_per_tile;
    if (blocks <= 0) return hipSuccess;
    c.num_blocks = uint32_t(blocks);
    const uint32_t padded = uint32_t((blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((sweep_split_kernel<R, W, KPB>), dim3(padded), dim3(256), 0, stream, c);
    return hipGetLastError();
  });
}

}  // namespace

// 16 L blocks per tile (64 ket points x L chunks of 64 / L bra points, 4 per block).
int32_t split_blocks_per_tile(int32_t reps) { return 16 << (2 * reps - 7); }

// Variants of the split sweep (target waves per SIMD W, ket points per block
// KPB); all compute bitwise identical results.  Variant 0 is the default of
// each reps.  At reps 5 and 6 a two-wave register budget (variant 3) spills
// about 300 bytes per lane, so the defaults run one wave per SIMD.
hipError_t launch_sweep_split_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream) {
  switch (reps * 16 + variant) {
    case 64 + 0: return launch_split<4, 2, 2>(a, stream);
    case 64 + 1: return launch_split<4, 2, 4>(a, stream);
    case 64 + 2: return launch_split<4, 1, 2>(a, stream);
    case 64 + 3: return launch_split<4, 1, 4>(a, stream);
    case 80 + 0: return launch_split<5, 1, 1>(a, stream);
    case 80 + 1: return launch_split<5, 1, 2>(a, stream);
    case 80 + 2: return launch_split<5, 1, 4>(a, stream);
    case 80 + 3: return launch_split<5, 2, 1>(a, stream);
    case 96 + 0: return launch_split<6, 1, 1>(a, stream);
    case 96 + 1: return launch_split<6, 1, 2>(a, stream);
    case 96 + 2: return launch_split<6, 1, 4>(a, stream);
    case 96 + 3: return launch_split<6, 2, 1>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qsvm
