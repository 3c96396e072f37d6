// FP64 refinement of the tiles whose largest entry is large.
//
// The sweep carries the environment in FP32.  Its rounding error in K is
// biased (an FP32 emulation of 784-qubit self-overlaps gives K = 1 - 1.0e-5
// ... 1.5e-5 from the arithmetic and < 3e-6 from the FP32 generators), so at
// 784 qubits an entry close to 1 can miss an absolute bar of 1e-5 while small
// entries stay far inside it (the threshold rule is auto_refine_threshold in
// refine.h).  After a sweep launch, refine_scan_kernel reads the K tiles the
// launch wrote and lists those whose largest computed entry exceeds a
// threshold, and
// refine_kernel recomputes the pairs of the listed tiles whose entry exceeds
// the threshold with an FP64 environment from FP64 generators (Section G
// value + Section L residual), overwriting K and log K; a wave whose pairs
// are all below it skips its item (a tile listed for one near-duplicate
// pair costs one wave, not 64).  The list length stays on the device: the
// refinement kernel is launched with a fixed grid whose waves take (tile,
// ket point) items until the list is exhausted (none when nothing was
// listed), so no host synchronisation is needed and the three launches can
// be captured in a graph.
//
// The FP64 sweep is the one-lane butterfly sweep of sweep_butterfly_item.h
// (same recursion, gauge, sign pattern, renormalisation and closure) with
// doubles: one pair per lane and one ket point per wave for reps <= 3; at
// reps >= 4 (128 to 2048 environment entries) one pair per wave.  A pair
// list (pairs_fp64_group_kernel, reps <= 3) takes one pair per group of 2
// or 4 lanes and writes bitwise the one-lane values.

#include "../../include/qsvm.h"
#include "refine.h"
#include "sweep_common.h"

namespace qsvm {
namespace {

constexpr int64_t kScanBlocksDeviceCount = 4096;  // scan grid when the list length is on the device

template <int R>
struct DLayout {
  static constexpr int NB = 2 * R - 1;
  static constexpr int M = 1 << NB;
  static constexpr int S = NB - 1;
  __host__ __device__ static constexpr int ket_bit(int l) { return l - 1; }
  __host__ __device__ static constexpr int bra_bit(int l) { return R - 1 + l - 1; }
};

struct Gen64 {
  double ar, ai, br, bi;
};

__device__ __forceinline__ Gen64 gen64(const float4* __restrict__ hi, const float4* __restrict__ lo, int64_t idx) {
  const float4 h = hi[idx], l = lo[idx];
  return {double(h.x) + double(l.x), double(h.y) + double(l.y), double(h.z) + double(l.z), double(h.w) + double(l.w)};
}

// (u0, u1) -> (u0 + (ar + i ai) u1, +-(u0 + (br + i bi) u1))
template <bool NEG>
__device__ __forceinline__ void dbfly(double2& u0, double2& u1, double ar, double ai, double br, double bi) {
  const double x0 = u0.x, y0 = u0.y, x1 = u1.x, y1 = u1.y;
  double t0r = fma(ar, x1, x0);
  t0r = fma(-ai, y1, t0r);
  double t0i = fma(ar, y1, y0);
  t0i = fma(ai, x1, t0i);
  double t1r = fma(br, x1, x0);
  t1r = fma(-bi, y1, t1r);
  double t1i = fma(br, y1, y0);
  t1i = fma(bi, x1, t1i);
  u0 = make_double2(t0r, t0i);
  u1 = NEG ? make_double2(-t1r, -t1i) : make_double2(t1r, t1i);
}

template <int AXBIT, int SIGNBIT, int SIGNBIT2, int M>
__device__ __forceinline__ void daxis(double2 (&v)[M], double ar, double ai, double br, double bi) {
#pragma unroll
  for (int i0 = 0; i0 < M; ++i0) {
    if (i0 & (1 << AXBIT)) continue;
    const int i1 = i0 | (1 << AXBIT);
    bool neg = false;
    if constexpr (SIGNBIT >= 0) neg ^= ((i0 >> SIGNBIT) & 1) != 0;
    if constexpr (SIGNBIT2 >= 0) neg ^= ((i0 >> SIGNBIT2) & 1) != 0;
    if (neg)
      dbfly<true>(v[i0], v[i1], ar, ai, br, bi);
    else
      dbfly<false>(v[i0], v[i1], ar, ai, br, bi);
  }
}

template <int R, int L>
struct DAxes {
  template <int M>
  __device__ __forceinline__ static void ket(double2 (&v)[M], const Gen64& c) {
    if constexpr (L <= R - 1) {
      daxis<DLayout<R>::ket_bit(L), (L >= 2 ? DLayout<R>::ket_bit(L - 1) : -1), -1>(v, c.ar, c.ai, c.br, c.bi);
      DAxes<R, L + 1>::ket(v, c);
    }
  }
  template <int M>
  __device__ __forceinline__ static void bra(double2 (&v)[M], const Gen64& c) {
    if constexpr (L <= R - 1) {
      daxis<DLayout<R>::bra_bit(L), (L >= 2 ? DLayout<R>::bra_bit(L - 1) : -1), -1>(v, c.ar, -c.ai, c.br, -c.bi);
      DAxes<R, L + 1>::bra(v, c);
    }
  }
};

template <int R>
__device__ __forceinline__ void dsite_step(double2 (&v)[DLayout<R>::M], const Gen64& cx, const Gen64& cy) {
  DAxes<R, 1>::ket(v, cx);
  DAxes<R, 1>::bra(v, cy);
  // shared top bit: a_x conj(a_y), b_x conj(b_y)
  const double asr = fma(cx.ar, cy.ar, cx.ai * cy.ai);
  const double asi = fma(cx.ai, cy.ar, -(cx.ar * cy.ai));
  const double bsr = fma(cx.br, cy.br, cx.bi * cy.bi);
  const double bsi = fma(cx.bi, cy.br, -(cx.br * cy.bi));
  constexpr int SB1 = (R >= 2) ? DLayout<R>::ket_bit(R - 1) : -1;
  constexpr int SB2 = (R >= 2) ? DLayout<R>::bra_bit(R - 1) : -1;
  daxis<DLayout<R>::S, SB1, SB2>(v, asr, asi, bsr, bsi);
}

// Divide by the power of two of the largest |component| (exact); returns it.
template <int M>
__device__ __forceinline__ int drenorm(double2 (&v)[M]) {
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < M; ++q) m = fmax(m, fmax(fabs(v[q].x), fabs(v[q].y)));
  int e = 0;
  (void)frexp(m, &e);
#pragma unroll
  for (int q = 0; q < M; ++q) v[q] = make_double2(ldexp(v[q].x, -e), ldexp(v[q].y, -e));
  return e;
}

template <int R>
__device__ __forceinline__ constexpr int dcol_sign_parity(int low, int s) {
  const int c = low | (s << (R - 1));
  return __builtin_popcount(c & (c >> 1)) & 1;
}

template <int R>
__device__ __forceinline__ void dinit_env(double2 (&v)[DLayout<R>::M]) {
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
#pragma unroll
  for (int q = 0; q < DLayout<R>::M; ++q) {
    const int s = (q >> DLayout<R>::S) & 1;
    const int par = dcol_sign_parity<R>(q & LOWMASK, s) ^ dcol_sign_parity<R>((q >> (R - 1)) & LOWMASK, s);
    v[q] = make_double2(par ? -1.0 : 1.0, 0.0);
  }
}

// |sum_q g_x^|c| conj(g_y)^|c'| v[q]|^2 (right boundary of the gauge form).
template <int R>
__device__ __forceinline__ double dclosure(const double2 (&v)[DLayout<R>::M], double gxr, double gxi, double gyr,
                                           double gyi) {
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
  double pxr[R + 1], pxi[R + 1], pyr[R + 1], pyi[R + 1];
  pxr[0] = 1.0; pxi[0] = 0.0; pyr[0] = 1.0; pyi[0] = 0.0;
  gyi = -gyi;  // conj(g_y)
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    pxr[m] = fma(pxr[m - 1], gxr, -(pxi[m - 1] * gxi));
    pxi[m] = fma(pxr[m - 1], gxi, pxi[m - 1] * gxr);
    pyr[m] = fma(pyr[m - 1], gyr, -(pyi[m - 1] * gyi));
    pyi[m] = fma(pyr[m - 1], gyi, pyi[m - 1] * gyr);
  }
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int q = 0; q < DLayout<R>::M; ++q) {
    const int s = (q >> DLayout<R>::S) & 1;
    const int hk = __builtin_popcount(q & LOWMASK) + s;
    const int hb = __builtin_popcount((q >> (R - 1)) & LOWMASK) + s;
    const double wr = fma(pxr[hk], pyr[hb], -(pxi[hk] * pyi[hb]));
    const double wi = fma(pxr[hk], pyi[hb], pxi[hk] * pyr[hb]);
    sr = fma(wr, v[q].x, fma(-wi, v[q].y, sr));
    si = fma(wr, v[q].y, fma(wi, v[q].x, si));
  }
  return fma(sr, sr, si * si);
}

__global__ void refine_reset(uint32_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0u;
}

// One block per tile of the launch: the largest computed entry of the tile
// (the assigned symmetric diagonal excluded); tiles above `thresh` are
// appended to the list.
__global__ void __launch_bounds__(256)
refine_scan_kernel(SweepArgs a, double thresh, uint32_t* __restrict__ list, uint32_t* __restrict__ count) {
  __shared__ double red[4];
  const uint32_t tiles = uint32_t(device_tiles(a));
  for (uint32_t u = blockIdx.x; u < tiles; u += gridDim.x) {  // block-uniform
    int32_t ti, tj;
    const bool valid = decode_tile(a, u, ti, tj);
    double m = 0.0;
    if (valid) {
      for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int64_t i = int64_t(ti) * kTile + e / kTile, j = int64_t(tj) * kTile + e % kTile;
        if (pair_computed(a, i, j)) m = fmax(m, a.K[i * a.ldk + j]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
      if (mx > thresh) list[atomicAdd(count, 1u)] = u;
    }
    __syncthreads();  // red is reused by the next tile
  }
}

// FP64 sweep of one pair per lane, (i, j) per lane; every lane of the wave
// takes part (lanes with comp = false compute a clamped pair and store
// nothing), so the caller keeps the whole wave in the call.  PF sites per
// load group (below).
template <int R, int PF>
__device__ __forceinline__ void fp64_pair_lanes(const SweepArgs& a, int64_t i, int64_t j, bool comp) {
  constexpr int M = DLayout<R>::M;
  const float4* __restrict__ gA = a.gen_a;
  const float4* __restrict__ gB = a.gen_b;
  const float4* __restrict__ lA = a.gen_a + int64_t(a.n) * a.Na;  // Section L follows Section G
  const float4* __restrict__ lB = a.gen_b + int64_t(a.n) * a.Nb;
  const int64_t ic = (i >= 0 && i < a.Na) ? i : a.Na - 1;  // loads of idle lanes stay in bounds
  const int64_t jc = (j >= 0 && j < a.Nb) ? j : a.Nb - 1;
  double2 v[M];
  dinit_env<R>(v);
  int32_t acc = 0;
  int countdown = a.renorm_every;
  auto step = [&](const Gen64& cx, const Gen64& cy) {
    dsite_step<R>(v, cx, cy);
    if (--countdown == 0) {
      acc += drenorm(v);
      countdown = a.renorm_every;
    }
  };
  // generators of sites k .. k + PF - 1 as loaded (clamped to the last
  // site, so a prefetch past the end stays in bounds); two groups of PF sites
  // alternate, the loads of one group in flight while the other's sites are
  // swept.  Scattered points (a pair list) miss the caches at every site and
  // take PF = 4; the bra points of a tile are consecutive and PF = 1 keeps
  // the registers (and occupancy) of the refinement kernel.
  struct Raw {
    float4 xh, xl, yh, yl;
  };
  Raw buf[2][PF];
  auto load = [&](int k0, Raw(&g)[PF]) {
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      const int64_t kc = (k0 + d < a.n) ? k0 + d : a.n - 1;
      g[d].xh = gA[kc * a.Na + ic];
      g[d].xl = lA[kc * a.Na + ic];
      g[d].yh = gB[kc * a.Nb + jc];
      g[d].yl = lB[kc * a.Nb + jc];
    }
  };
  auto sweep = [&](int k0, const Raw(&g)[PF]) {
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      if (k0 + d >= a.n) break;  // uniform
      const Gen64 cx = {double(g[d].xh.x) + double(g[d].xl.x), double(g[d].xh.y) + double(g[d].xl.y),
                        double(g[d].xh.z) + double(g[d].xl.z), double(g[d].xh.w) + double(g[d].xl.w)};
      const Gen64 cy = {double(g[d].yh.x) + double(g[d].yl.x), double(g[d].yh.y) + double(g[d].yl.y),
                        double(g[d].yh.z) + double(g[d].yl.z), double(g[d].yh.w) + double(g[d].yl.w)};
      step(cx, cy);
    }
  };
  if (a.n > 1) {
    load(1, buf[0]);
    for (int k = 1; k < a.n; k += 2 * PF) {
      load(k + PF, buf[1]);
      sweep(k, buf[0]);
      if (k + PF >= a.n) break;
      load(k + 2 * PF, buf[0]);
      sweep(k + PF, buf[1]);
    }
  }
  if (comp) {
    const Gen64 gx = gen64(gA, lA, ic), gy = gen64(gB, lB, jc);
    const double s2 = dclosure<R>(v, gx.ar, gx.ai, gy.ar, gy.ai);
    store_entry(a, i, j, s2, 2 * (acc - R * a.n));
  }
}

// Each wave takes items (listed tile, ket point of the tile) and recomputes
// that ket point against the tile's 64 bra points in FP64.
template <int R>
__global__ void __launch_bounds__(256)
refine_kernel(SweepArgs a, double thresh, const uint32_t* __restrict__ list, const uint32_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t items = uint64_t(*count) * kTile;
  for (uint64_t it = uint64_t(blockIdx.x) * 4 + wave; it < items; it += uint64_t(gridDim.x) * 4) {  // wave-uniform
    int32_t ti, tj;
    if (!decode_tile(a, list[it / kTile], ti, tj)) continue;
    const int64_t i = int64_t(ti) * kTile + int64_t(it % kTile);
    const int64_t j = int64_t(tj) * kTile + lane;
    // only the pairs whose FP32 entry exceeds the threshold (entries at or
    // below it are within the FP32 sweep's error budget); a wave with none
    // of them skips the item
    const bool comp = pair_computed(a, i, j) && a.K[i * a.ldk + j] > thresh;
    if (!__builtin_amdgcn_ballot_w64(comp)) continue;
    fp64_pair_lanes<R, 1>(a, i, j, comp);
  }
}

// Pair i <= j of list entry p (a symmetric Gram's upper triangle; the pair
// is swapped if given the other way round); false for entries past the
// count, invalid indices (e.g. -1 placeholders) and pairs the Gram does not
// compute (the assigned diagonal).
__device__ __forceinline__ bool listed_pair(const SweepArgs& a, const int32_t* __restrict__ pairs, int64_t count,
                                            int64_t p, int64_t& i, int64_t& j) {
  i = 0;
  j = 0;
  if (p >= count) return false;
  int64_t x = pairs[2 * p], y = pairs[2 * p + 1];
  if (x < 0 || y < 0 || x >= a.Na || y >= a.Nb) return false;
  if (x > y) {
    const int64_t t = x;
    x = y;
    y = t;
  }
  i = x;
  j = y;
  return pair_computed(a, i, j);
}

__device__ __forceinline__ int64_t listed_count(const int32_t* __restrict__ count, int64_t max_pairs) {
  const int64_t c = *count;
  return c < 0 ? 0 : (c < max_pairs ? c : max_pairs);
}

// reps >= 4: one pair per wave.  The 2^(2r-1) environment entries q sit
// E = 2^(2r-7) per lane: lane = bits 0..5 of q, register e = the bits above
// (ket bits 0..r-2, bra bits r-1..2r-3, shared bit 2r-2, as in the one-lane
// sweep).  An axis on a register bit runs as register butterflies; an axis
// on bit B < 6 pairs lane l with lane l ^ 2^B: the lane without the bit
// computes u0 + a u1, the lane with it +-(u0 + b u1), each from its own value
// and its partner's (__shfl_xor).  Sign rule, renormalisation and closure as
// in the one-lane sweep, with wave-wide reductions.
template <int R>
struct WLayout {
  static constexpr int E = 1 << (2 * R - 7);  // entries per lane
  static constexpr int ket_bit(int l) { return l - 1; }
  static constexpr int bra_bit(int l) { return R + l - 2; }
  static constexpr int S = 2 * R - 2;
};

// Axis on entry bit B of an environment whose entries q sit E per lane:
// lane bits 0 .. LB - 1 of q are bits of the lane, the bits above index the
// registers (q = lane % 2^LB + e 2^LB).  A register bit runs as register
// butterflies; a lane bit B pairs lane l with lane l ^ 2^B: the lane without
// the bit computes u0 + a u1, the lane with it +-(u0 + b u1), each from its
// own value and its partner's (xor_lane), the same operations as dbfly.
// x of the lane of l's pair (l, l ^ 2^B) without bit B (HI = false) or with
// it (HI = true), B = 0, 1: a DPP quad permutation that hands both lanes the
// same value, so neither has to select between its own and its partner's.
template <int B, bool HI>
__device__ __forceinline__ double pair_lane(double x) {
  static_assert(B <= 1, "quad permutations cover lane bits 0 and 1");
  // quad_perm [0,0,2,2] / [1,1,3,3] (bit 0), [0,1,0,1] / [2,3,2,3] (bit 1)
  constexpr int ctrl = (B == 0) ? (HI ? 0xF5 : 0xA0) : (HI ? 0xEE : 0x44);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// x of lane l ^ 2^B: a DPP quad permutation for B = 0, 1 (no trip through
// the LDS crossbar), __shfl_xor above.
template <int B>
__device__ __forceinline__ double xor_lane(double x) {
  if constexpr (B <= 1) {
    constexpr int ctrl = (B == 0) ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
  } else {
    return __shfl_xor(x, 1 << B, 64);
  }
}

template <int E, int LB, int B, int SB1, int SB2>
__device__ __forceinline__ void group_axis(double2 (&v)[E], int lane, double ar, double ai, double br, double bi) {
  constexpr int LM = (1 << LB) - 1;
  if constexpr (B >= LB) {  // register bit
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
      if (e0 & (1 << (B - LB))) continue;
      const int e1 = e0 | (1 << (B - LB));
      const int i0 = (lane & LM) | (e0 << LB);
      bool neg = false;
      if constexpr (SB1 >= 0) neg ^= ((i0 >> SB1) & 1) != 0;
      if constexpr (SB2 >= 0) neg ^= ((i0 >> SB2) & 1) != 0;
      dbfly<false>(v[e0], v[e1], ar, ai, br, bi);
      if (neg) v[e1] = make_double2(-v[e1].x, -v[e1].y);
    }
  } else {  // lane bit
    const bool upper = (lane >> B) & 1;
    const double cr = upper ? br : ar, ci = upper ? bi : ai;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double2 u0, u1;  // the entries of the lanes without and with bit B
      if constexpr (B <= 1) {
        u0 = make_double2(pair_lane<B, false>(v[e].x), pair_lane<B, false>(v[e].y));
        u1 = make_double2(pair_lane<B, true>(v[e].x), pair_lane<B, true>(v[e].y));
      } else {
        const double pr = xor_lane<B>(v[e].x), pim = xor_lane<B>(v[e].y);
        u0 = upper ? make_double2(pr, pim) : v[e];
        u1 = upper ? v[e] : make_double2(pr, pim);
      }
      double tr = fma(cr, u1.x, u0.x);
      tr = fma(-ci, u1.y, tr);
      double ti = fma(cr, u1.y, u0.y);
      ti = fma(ci, u1.x, ti);
      const int i0 = ((lane & LM) | (e << LB)) & ~(1 << B);
      bool neg = false;
      if constexpr (SB1 >= 0) neg ^= ((i0 >> SB1) & 1) != 0;
      if constexpr (SB2 >= 0) neg ^= ((i0 >> SB2) & 1) != 0;
      v[e] = (upper && neg) ? make_double2(-tr, -ti) : make_double2(tr, ti);
    }
  }
}

template <int R, int B, int SB1, int SB2>
__device__ __forceinline__ void wave_axis(double2 (&v)[WLayout<R>::E], int lane, double ar, double ai, double br,
                                          double bi) {
  group_axis<WLayout<R>::E, 6, B, SB1, SB2>(v, lane, ar, ai, br, bi);
}

template <int R, int L>
struct WAxes {
  __device__ __forceinline__ static void ket(double2 (&v)[WLayout<R>::E], int lane, const Gen64& c) {
    if constexpr (L <= R - 1) {
      wave_axis<R, WLayout<R>::ket_bit(L), (L >= 2 ? WLayout<R>::ket_bit(L - 1) : -1), -1>(v, lane, c.ar, c.ai, c.br,
                                                                                             c.bi);
      WAxes<R, L + 1>::ket(v, lane, c);
    }
  }
  __device__ __forceinline__ static void bra(double2 (&v)[WLayout<R>::E], int lane, const Gen64& c) {
    if constexpr (L <= R - 1) {
      wave_axis<R, WLayout<R>::bra_bit(L), (L >= 2 ? WLayout<R>::bra_bit(L - 1) : -1), -1>(v, lane, c.ar, -c.ai,
                                                                                             c.br, -c.bi);
      WAxes<R, L + 1>::bra(v, lane, c);
    }
  }
};

template <int R, int LB, int E, int L>
struct GAxes {
  __device__ __forceinline__ static void ket(double2 (&v)[E], int lane, const Gen64& c) {
    if constexpr (L <= R - 1) {
      group_axis<E, LB, DLayout<R>::ket_bit(L), (L >= 2 ? DLayout<R>::ket_bit(L - 1) : -1), -1>(v, lane, c.ar, c.ai,
                                                                                                c.br, c.bi);
      GAxes<R, LB, E, L + 1>::ket(v, lane, c);
    }
  }
  __device__ __forceinline__ static void bra(double2 (&v)[E], int lane, const Gen64& c) {
    if constexpr (L <= R - 1) {
      group_axis<E, LB, DLayout<R>::bra_bit(L), (L >= 2 ? DLayout<R>::bra_bit(L - 1) : -1), -1>(v, lane, c.ar, -c.ai,
                                                                                                c.br, -c.bi);
      GAxes<R, LB, E, L + 1>::bra(v, lane, c);
    }
  }
};

// FP64 sweep of one pair per wave (reps >= 4), the pair wave-uniform.
template <int R>
__device__ __forceinline__ void fp64_pair_wave(const SweepArgs& a, int64_t i, int64_t j) {
  using W = WLayout<R>;
  constexpr int E = W::E;
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
  const int lane = threadIdx.x & 63;
  const float4* __restrict__ gA = a.gen_a;
  const float4* __restrict__ gB = a.gen_b;
  const float4* __restrict__ lA = a.gen_a + int64_t(a.n) * a.Na;  // Section L follows Section G
  const float4* __restrict__ lB = a.gen_b + int64_t(a.n) * a.Nb;
  double2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = lane | (e << 6);
    const int s = (q >> W::S) & 1;
    const int par = dcol_sign_parity<R>(q & LOWMASK, s) ^ dcol_sign_parity<R>((q >> (R - 1)) & LOWMASK, s);
    v[e] = make_double2(par ? -1.0 : 1.0, 0.0);
  }
  int32_t acc = 0;
  int countdown = a.renorm_every;
  for (int k = 1; k < a.n; ++k) {
    const Gen64 cx = gen64(gA, lA, int64_t(k) * a.Na + i);
    const Gen64 cy = gen64(gB, lB, int64_t(k) * a.Nb + j);
    WAxes<R, 1>::ket(v, lane, cx);
    WAxes<R, 1>::bra(v, lane, cy);
    // shared bit: a_x conj(a_y), b_x conj(b_y); sign bits ket and bra l = R-1
    const double asr = fma(cx.ar, cy.ar, cx.ai * cy.ai);
    const double asi = fma(cx.ai, cy.ar, -(cx.ar * cy.ai));
    const double bsr = fma(cx.br, cy.br, cx.bi * cy.bi);
    const double bsi = fma(cx.bi, cy.br, -(cx.br * cy.bi));
    wave_axis<R, W::S, W::ket_bit(R - 1), W::bra_bit(R - 1)>(v, lane, asr, asi, bsr, bsi);
    if (--countdown == 0) {
      double m = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) m = fmax(m, fmax(fabs(v[e].x), fabs(v[e].y)));
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
      int ex = 0;
      (void)frexp(m, &ex);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = make_double2(ldexp(v[e].x, -ex), ldexp(v[e].y, -ex));
      acc += ex;
      countdown = a.renorm_every;
    }
  }
  // closure: sum over the wave of g_x^|c| conj(g_y)^|c'| v[q]
  const Gen64 gx = gen64(gA, lA, i), gy = gen64(gB, lB, j);
  double pxr[R + 1], pxi[R + 1], pyr[R + 1], pyi[R + 1];
  pxr[0] = 1.0; pxi[0] = 0.0; pyr[0] = 1.0; pyi[0] = 0.0;
  const double gyi = -gy.ai;  // conj(g_y)
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    pxr[m] = fma(pxr[m - 1], gx.ar, -(pxi[m - 1] * gx.ai));
    pxi[m] = fma(pxr[m - 1], gx.ai, pxi[m - 1] * gx.ar);
    pyr[m] = fma(pyr[m - 1], gy.ar, -(pyi[m - 1] * gyi));
    pyi[m] = fma(pyr[m - 1], gyi, pyi[m - 1] * gy.ar);
  }
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = lane | (e << 6);
    const int s = (q >> W::S) & 1;
    const int hk = __builtin_popcount(q & LOWMASK) + s;
    const int hb = __builtin_popcount((q >> (R - 1)) & LOWMASK) + s;
    double wr = 0.0, wi = 0.0;
#pragma unroll
    for (int x = 0; x <= R; ++x)  // select the powers without dynamic register indexing
#pragma unroll
      for (int y = 0; y <= R; ++y)
        if (x == hk && y == hb) {
          wr = fma(pxr[x], pyr[y], -(pxi[x] * pyi[y]));
          wi = fma(pxr[x], pyi[y], pxi[x] * pyr[y]);
        }
    sr = fma(wr, v[e].x, fma(-wi, v[e].y, sr));
    si = fma(wr, v[e].y, fma(wi, v[e].x, si));
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (lane == 0) store_entry(a, i, j, fma(sr, sr, si * si), 2 * (acc - R * a.n));
}

// FP64 sweep of one pair per group of G = 2^LB lanes (reps <= 3, the pair
// uniform over the group): the M = 2^(2r-1) entries sit M / G per lane as
// in group_axis, every butterfly the one-lane sweep's operations and the
// renormalisation its power of two (the group's largest component), so the
// environment is bitwise the one-lane sweep's; for the closure the group's
// first lane gathers the M entries and sums them in the one-lane order, so
// the stored entry is bitwise the refinement's.  Generators of the next
// 2 PF sites in flight (the points of a pair list are scattered: each
// site's loads miss the caches).
template <int R, int LB, int PF>
__device__ __forceinline__ void fp64_pair_group(const SweepArgs& a, int64_t i, int64_t j, bool comp) {
  using D = DLayout<R>;
  constexpr int M = D::M, G = 1 << LB, E = M / G;
  static_assert(E >= 1, "a group holds at most M lanes");
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
  const int lane = threadIdx.x & 63, gl = lane & (G - 1);
  const float4* __restrict__ gA = a.gen_a;
  const float4* __restrict__ gB = a.gen_b;
  const float4* __restrict__ lA = a.gen_a + int64_t(a.n) * a.Na;  // Section L follows Section G
  const float4* __restrict__ lB = a.gen_b + int64_t(a.n) * a.Nb;
  const int64_t ic = (i >= 0 && i < a.Na) ? i : a.Na - 1;  // loads of idle groups stay in bounds
  const int64_t jc = (j >= 0 && j < a.Nb) ? j : a.Nb - 1;
  double2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = gl | (e << LB);
    const int s = (q >> D::S) & 1;
    const int par = dcol_sign_parity<R>(q & LOWMASK, s) ^ dcol_sign_parity<R>((q >> (R - 1)) & LOWMASK, s);
    v[e] = make_double2(par ? -1.0 : 1.0, 0.0);
  }
  int32_t acc = 0;
  int countdown = a.renorm_every;
  auto step = [&](const Gen64& cx, const Gen64& cy) {
    GAxes<R, LB, E, 1>::ket(v, lane, cx);
    GAxes<R, LB, E, 1>::bra(v, lane, cy);
    const double asr = fma(cx.ar, cy.ar, cx.ai * cy.ai);
    const double asi = fma(cx.ai, cy.ar, -(cx.ar * cy.ai));
    const double bsr = fma(cx.br, cy.br, cx.bi * cy.bi);
    const double bsi = fma(cx.bi, cy.br, -(cx.br * cy.bi));
    constexpr int SB1 = (R >= 2) ? D::ket_bit(R - 1) : -1;
    constexpr int SB2 = (R >= 2) ? D::bra_bit(R - 1) : -1;
    group_axis<E, LB, D::S, SB1, SB2>(v, lane, asr, asi, bsr, bsi);
    if (--countdown == 0) {
      double m = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) m = fmax(m, fmax(fabs(v[e].x), fabs(v[e].y)));
      if constexpr (G > 1) m = fmax(m, xor_lane<0>(m));
      if constexpr (G > 2) m = fmax(m, xor_lane<1>(m));
#pragma unroll
      for (int off = 4; off < G; off <<= 1) m = fmax(m, __shfl_xor(m, off, 64));
      int ex = 0;
      (void)frexp(m, &ex);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = make_double2(ldexp(v[e].x, -ex), ldexp(v[e].y, -ex));
      acc += ex;
      countdown = a.renorm_every;
    }
  };
  struct Raw {
    float4 xh, xl, yh, yl;
  };
  Raw buf[2][PF];
  auto load = [&](int k0, Raw(&g)[PF]) {
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      const int64_t kc = (k0 + d < a.n) ? k0 + d : a.n - 1;
      g[d].xh = gA[kc * a.Na + ic];
      g[d].xl = lA[kc * a.Na + ic];
      g[d].yh = gB[kc * a.Nb + jc];
      g[d].yl = lB[kc * a.Nb + jc];
    }
  };
  auto sweep = [&](int k0, const Raw(&g)[PF]) {
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      if (k0 + d >= a.n) break;  // uniform
      const Gen64 cx = {double(g[d].xh.x) + double(g[d].xl.x), double(g[d].xh.y) + double(g[d].xl.y),
                        double(g[d].xh.z) + double(g[d].xl.z), double(g[d].xh.w) + double(g[d].xl.w)};
      const Gen64 cy = {double(g[d].yh.x) + double(g[d].yl.x), double(g[d].yh.y) + double(g[d].yl.y),
                        double(g[d].yh.z) + double(g[d].yl.z), double(g[d].yh.w) + double(g[d].yl.w)};
      step(cx, cy);
    }
  };
  if (a.n > 1) {
    load(1, buf[0]);
    for (int k = 1; k < a.n; k += 2 * PF) {
      load(k + PF, buf[1]);
      sweep(k, buf[0]);
      if (k + PF >= a.n) break;
      load(k + 2 * PF, buf[0]);
      sweep(k + PF, buf[1]);
    }
  }
  // the M entries in q order, in every lane of the group
  double2 all[M];
  const int base = lane & ~(G - 1);
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int src = base | (q & (G - 1));
    all[q] = make_double2(__shfl(v[q >> LB].x, src, 64), __shfl(v[q >> LB].y, src, 64));
  }
  if (comp && gl == 0) {
    const Gen64 gx = gen64(gA, lA, ic), gy = gen64(gB, lB, jc);
    const double s2 = dclosure<R>(all, gx.ar, gx.ai, gy.ar, gy.ai);
    store_entry(a, i, j, s2, 2 * (acc - R * a.n));
  }
}

// FP64 entries of a device-resident pair list (reps <= 3): one pair per
// group of 2^LB lanes, 64 / 2^LB pairs per wave.  Chunks of a wave's pairs
// go to the blocks in turn (chunk c to block c % gridDim.x, wave
// c / gridDim.x) so a short list is spread over as many compute units as it
// has chunks.
template <int R, int LB>
__global__ void __launch_bounds__(256)
pairs_fp64_group_kernel(SweepArgs a, const int32_t* __restrict__ pairs, const int32_t* __restrict__ count,
                        int64_t max_pairs) {
  constexpr int P = 64 >> LB;  // pairs per wave
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n = listed_count(count, max_pairs);
  for (int64_t c = int64_t(wave) * gridDim.x + blockIdx.x; c * P < n; c += int64_t(gridDim.x) * 4) {  // wave-uniform
    int64_t i, j;
    const bool comp = listed_pair(a, pairs, n, c * P + (lane >> LB), i, j);
    if (!__builtin_amdgcn_ballot_w64(comp)) continue;
    fp64_pair_group<R, LB, 4>(a, i, j, comp);
  }
}

template <int R>
__global__ void __launch_bounds__(256)
refine_wave_kernel(SweepArgs a, double thresh, const uint32_t* __restrict__ list, const uint32_t* __restrict__ count) {
  const int wave = threadIdx.x >> 6;
  const uint64_t items = uint64_t(*count) * (kTile * kTile);
  for (uint64_t it = uint64_t(blockIdx.x) * 4 + wave; it < items; it += uint64_t(gridDim.x) * 4) {  // wave-uniform
    int32_t ti, tj;
    if (!decode_tile(a, list[it / (kTile * kTile)], ti, tj)) continue;
    const int pr = int(it % (kTile * kTile));
    const int64_t i = int64_t(ti) * kTile + pr / kTile, j = int64_t(tj) * kTile + pr % kTile;
    // the same pair in every lane; only entries above the threshold
    if (!pair_computed(a, i, j) || !(a.K[i * a.ldk + j] > thresh)) continue;
    fp64_pair_wave<R>(a, i, j);
  }
}

// FP64 entries of a device-resident pair list (reps >= 4): one pair per wave.
template <int R>
__global__ void __launch_bounds__(256)
pairs_fp64_wave_kernel(SweepArgs a, const int32_t* __restrict__ pairs, const int32_t* __restrict__ count,
                       int64_t max_pairs) {
  const int wave = threadIdx.x >> 6;
  const int64_t n = listed_count(count, max_pairs);
  // pair p to block p % gridDim.x (a short list spread over the compute units)
  for (int64_t p = int64_t(wave) * gridDim.x + blockIdx.x; p < n; p += int64_t(gridDim.x) * 4) {  // wave-uniform
    int64_t i, j;
    if (!listed_pair(a, pairs, n, p, i, j)) continue;
    fp64_pair_wave<R>(a, i, j);
  }
}

}  // namespace

hipError_t launch_pairs_fp64(const SweepArgs& a, int32_t reps, const int32_t* pairs, const int32_t* count,
                             int64_t max_pairs, int64_t resident_blocks, hipStream_t stream) {
  if (reps < 1 || reps > kMaxReps) return hipErrorInvalidValue;
  if (max_pairs <= 0) return hipSuccess;
  // one pair per group of 2 or 4 lanes (reps 1; 2 and 3) or per wave, at
  // most the resident blocks
  const int64_t per_block = (reps >= 4) ? 4 : 4 * (64 >> (reps == 1 ? 1 : 2));
  int64_t blocks = (max_pairs + per_block - 1) / per_block;
  if (blocks > resident_blocks) blocks = resident_blocks;
  if (blocks < 1) blocks = 1;
  const dim3 grid{unsigned(blocks)};
  switch (reps) {
    case 1: hipLaunchKernelGGL((pairs_fp64_group_kernel<1, 1>), grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
    case 2: hipLaunchKernelGGL((pairs_fp64_group_kernel<2, 2>), grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
    case 3: hipLaunchKernelGGL((pairs_fp64_group_kernel<3, 2>), grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
    case 4: hipLaunchKernelGGL(pairs_fp64_wave_kernel<4>, grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
    case 5: hipLaunchKernelGGL(pairs_fp64_wave_kernel<5>, grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
    default: hipLaunchKernelGGL(pairs_fp64_wave_kernel<6>, grid, dim3(256), 0, stream, a, pairs, count, max_pairs); break;
  }
  return hipGetLastError();
}

hipError_t launch_refine(const SweepArgs& a, int32_t reps, double thresh, uint32_t* list, uint32_t* count,
                         int64_t resident_blocks, hipStream_t stream) {
  if (reps < 1 || reps > kMaxReps) return hipErrorInvalidValue;
  const int64_t tiles = launch_tiles(a);
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_reset, dim3(1), dim3(64), 0, stream, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // a list whose length is read on the device may hold far fewer tiles than
  // its capacity: a bounded grid strides over whatever it holds
  const int64_t scan_cap = a.tile_count ? kScanBlocksDeviceCount : kMaxGridBlocks / 8 * 8;
  const int64_t scan_blocks = tiles < scan_cap ? tiles : scan_cap;
  hipLaunchKernelGGL(refine_scan_kernel, dim3(unsigned(scan_blocks)), dim3(256), 0, stream, a, thresh, list, count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // enough waves for every listed ket point (pair at reps >= 4), at most the
  // resident blocks
  int64_t blocks = tiles * (reps >= 4 ? kTile * kTile : kTile) / 4;
  if (blocks > resident_blocks) blocks = resident_blocks;
  if (blocks < 1) blocks = 1;
  if (reps >= 4) {
    const dim3 grid{unsigned(blocks)};
    switch (reps) {
      case 4: hipLaunchKernelGGL(refine_wave_kernel<4>, grid, dim3(256), 0, stream, a, thresh, list, count); break;
      case 5: hipLaunchKernelGGL(refine_wave_kernel<5>, grid, dim3(256), 0, stream, a, thresh, list, count); break;
      default: hipLaunchKernelGGL(refine_wave_kernel<6>, grid, dim3(256), 0, stream, a, thresh, list, count); break;
    }
    return hipGetLastError();
  }
  switch (reps) {
    case 1: hipLaunchKernelGGL(refine_kernel<1>, dim3(unsigned(blocks)), dim3(256), 0, stream, a, thresh, list, count); break;
    case 2: hipLaunchKernelGGL(refine_kernel<2>, dim3(unsigned(blocks)), dim3(256), 0, stream, a, thresh, list, count); break;
    default: hipLaunchKernelGGL(refine_kernel<3>, dim3(unsigned(blocks)), dim3(256), 0, stream, a, thresh, list, count); break;
  }
  return hipGetLastError();
}

hipError_t refine_resident_blocks(int32_t reps, int64_t* out) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) {
    switch (reps) {
      case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_kernel<1>, 256, 0); break;
      case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_kernel<2>, 256, 0); break;
      case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_kernel<3>, 256, 0); break;
      case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_wave_kernel<4>, 256, 0); break;
      case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_wave_kernel<5>, 256, 0); break;
      default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, refine_wave_kernel<6>, 256, 0); break;
    }
  }
  if (e != hipSuccess) return e;
  *out = int64_t(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

}  // namespace qsvm
