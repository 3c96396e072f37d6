// Butterfly sweep with each pair's environment split across two lanes, for
// bond dimensions whose environment does not fit one lane's registers
// (reps = 4: chi = 16, 2^(2r-1) = 128 complex entries per pair).
//
// The recursion, gauge and butterflies are those of the one-lane sweep
// (sweep_butterfly_item.h).  Lanes 2p and 2p+1 hold pair p; lane h keeps the
// entries whose shared (physical) bit s equals h, 2^(2r-2) of them.  The ket
// and bra bit axes act on bits below s, so they run inside each lane with
// the unchanged code.  Only the shared-bit axis pairs entries across the two
// lanes: (u0, u1) -> (u0 + as u1, nu (u0 + bs u1)) with as = a_x conj(a_y),
// bs = b_x conj(b_y) and nu = +-1 the sign pattern (a function of the
// lane's own index bits).  To give both lanes the same instruction stream,
// lane 1 stores its entries divided by a per-pair phase Phi: with Phi' =
// bs Phi,
//     lane 0:  u0 <- u0 + (as Phi) p        (p = lane 1's stored value)
//     lane 1:  u~1 <- nu (u~1 + (1/Phi') p)  (p = lane 0's value),
// after which Phi <- Phi'.  Both lanes compute "own + c * partner" with their
// own coefficient c; Phi is carried in FP64 and multiplies lane 1's part of
// the closure at the end.  The partner's values come from the neighbouring
// lane through the LDS crossbar (ds_swizzle, quad permutation [1, 0, 3, 2]),
// four entries per wait: that keeps the 128 exchanges per site off the
// VALU, where DPP moves measured about 8 extra issue cycles each (the sweep
// ran 1.1x slower with them).  Renormalisation takes the larger of the two
// lanes' maxima, so both halves share one power-of-two scale.
//
// Work layout: a tile is 64 ket x 64 bra points; a wave owns one ket point
// (wave-uniform, scalar loads) and 32 bra points (two lanes each); a block of
// 4 waves covers two ket points x 64 bra points, so a tile is 32 blocks.

#include "../../include/qsvm.h"
#include "sweep_butterfly_item.h"

namespace qsvm {
namespace {

// Value of x in the partner lane (lane ^ 1): DPP quad permutation [1, 0, 3, 2]
// (for the few values per site outside the shared-bit axis: the FP64 phase
// and the renormalisation maximum).
__device__ __forceinline__ float partner(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ double partner(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(uint64_t(b) >> 32)), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// Initial environment of lane h: the sign pattern of the entries with s = h.
template <int R, int ML>
__device__ __forceinline__ void init_split(float2 (&v)[ML], int h) {
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
#pragma unroll
  for (int q = 0; q < ML; ++q) {
    const int ket = q & LOWMASK;
    const int bra = (q >> (R - 1)) & LOWMASK;
    const int p0 = col_sign_parity<R>(ket, 0) ^ col_sign_parity<R>(bra, 0);
    const int p1 = col_sign_parity<R>(ket, 1) ^ col_sign_parity<R>(bra, 1);
    const int par = h ? p1 : p0;
    v[q] = make_float2(par ? -1.0f : 1.0f, 0.0f);
  }
}

// Partner (lane ^ 1) values of four entries through the LDS crossbar
// (ds_swizzle in quad-permute mode [1, 0, 3, 2], no LDS memory touched); one
// wait for all eight.  Written as one asm block so that the compiler cannot
// hoist the swizzles of a whole site ahead of their use (it does with the
// builtin, and the results then spill); the wait also covers any scalar loads
// still in flight.  Faster than batches of eight entries (529.5 vs 527 ms).
__device__ __forceinline__ void swizzle4(const float2& v0, const float2& v1, const float2& v2, const float2& v3,
                                         float (&p)[8]) {
  asm volatile(
      "ds_swizzle_b32 %0, %8 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %1, %9 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %2, %10 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %3, %11 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %4, %12 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %5, %13 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %6, %14 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "ds_swizzle_b32 %7, %15 offset:swizzle(QUAD_PERM,1,0,3,2)\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(p[0]), "=&v"(p[1]), "=&v"(p[2]), "=&v"(p[3]), "=&v"(p[4]), "=&v"(p[5]), "=&v"(p[6]), "=&v"(p[7])
      : "v"(v0.x), "v"(v0.y), "v"(v1.x), "v"(v1.y), "v"(v2.x), "v"(v2.y), "v"(v3.x), "v"(v3.y));
}

// Shared-bit axis across the lane pair: v <- sg(q) (v + c * partner(v)),
// where sg(q) = -1 for the entries whose sign bits are set, in lane 1 only
// (nsg = -1 in lane 1, +1 in lane 0).  Partner values arrive four entries
// at a time through the LDS crossbar.
template <int R, int ML>
__device__ __forceinline__ void cross_axis(float2 (&v)[ML], float cr, float ci, float nsg) {
  constexpr int SB1 = Layout<R>::ket_bit(R - 1);
  constexpr int SB2 = Layout<R>::bra_bit(R - 1);
#pragma unroll
  for (int c = 0; c < ML / 4; ++c) {
    float p[8];
    swizzle4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3], p);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = 4 * c + e;
      const float pr = p[2 * e], pim = p[2 * e + 1];
      float tr = fmaf(cr, pr, v[q].x);
      tr = fmaf(-ci, pim, tr);
      float ti = fmaf(cr, pim, v[q].y);
      ti = fmaf(ci, pr, ti);
      if (((q >> SB1) ^ (q >> SB2)) & 1) {
        tr *= nsg;
        ti *= nsg;
      }
      v[q] = make_float2(tr, ti);
    }
  }
}

// Closure of one lane: sum_q g_x^|c| conj(g_y)^|c'| v[q] over the entries with
// s = 0 (lane 1's entries carry one more factor g_x conj(g_y), applied by the
// caller), in FP64.  The weight depends only on (|c|, |c'|), so the entries
// of each of the R x R weight classes are summed first (in a fixed order)
// and each class sum is multiplied by its weight once.
template <int R, int ML>
__device__ __forceinline__ void closure_half(const float2 (&v)[ML], double gxr, double gxi, double gyr,
                                             double gyi, double& sr, double& si) {
  constexpr int LOWMASK = (1 << (R - 1)) - 1;
  double pxr[R], pxi[R], pyr[R], pyi[R];
  pxr[0] = 1.0; pxi[0] = 0.0; pyr[0] = 1.0; pyi[0] = 0.0;
#pragma unroll
  for (int m = 1; m < R; ++m) {
    pxr[m] = fma(pxr[m - 1], gxr, -(pxi[m - 1] * gxi));
    pxi[m] = fma(pxr[m - 1], gxi, pxi[m - 1] * gxr);
    pyr[m] = fma(pyr[m - 1], gyr, -(pyi[m - 1] * gyi));
    pyi[m] = fma(pyr[m - 1], gyi, pyi[m - 1] * gyr);
  }
  sr = 0.0;
  si = 0.0;
#pragma unroll
  for (int hk = 0; hk < R; ++hk) {
#pragma unroll
    for (int hb = 0; hb < R; ++hb) {
      double cr = 0.0, ci = 0.0;
#pragma unroll
      for (int q = 0; q < ML; ++q) {
        if (__builtin_popcount(q & LOWMASK) != hk || __builtin_popcount((q >> (R - 1)) & LOWMASK) != hb) continue;
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

// One work item: ket point i against bra points j0 .. j0+31 (two lanes each).
template <int R>
__device__ __forceinline__ void split_item(const SweepArgs& a, int64_t i, int64_t j0) {
  constexpr int ML = 1 << (2 * R - 2);  // entries per lane
  const int lane = threadIdx.x & 63;
  const int h = lane & 1;
  const int64_t j = j0 + (lane >> 1);

  const bool comp = pair_computed(a, i, j);
  const bool active = pair_active(a, i, j);
  if (!__builtin_amdgcn_ballot_w64(active)) return;

  const int64_t jc = (j < a.Nb) ? j : a.Nb - 1;  // clamp loads of idle lanes in bounds
  const int64_t ic = (i < a.Na) ? i : a.Na - 1;

  float2 v[ML];
  init_split<R>(v, h);
  int32_t acc = 0;
  double phr = 1.0, phi = 0.0;  // Phi of lane 1's entries (carried by both lanes)
  const float nsg = h ? -1.0f : 1.0f;

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
      Axes<R, 1>::ket(v, cx);
      Axes<R, 1>::bra(v, cy);
      // shared-bit coefficients as = a_x conj(a_y), bs = b_x conj(b_y) in FP64
      // (products of FP32 values are exact there); Phi' = bs Phi; lane 0
      // uses as Phi, lane 1 uses 1 / Phi', each rounded to FP32 once
      const double xar = cx.x, xai = cx.y, xbr = cx.z, xbi = cx.w;
      const double yar = cy.x, yai = cy.y, ybr = cy.z, ybi = cy.w;
      const double asr = fma(xar, yar, xai * yai), asi = fma(xai, yar, -(xar * yai));
      const double bsr = fma(xbr, ybr, xbi * ybi), bsi = fma(xbi, ybr, -(xbr * ybi));
      const double nr = fma(bsr, phr, -(bsi * phi));
      const double ni = fma(bsr, phi, bsi * phr);
      const double q = 1.0 / fma(nr, nr, ni * ni);
      const float c0r = float(fma(asr, phr, -(asi * phi)));
      const float c0i = float(fma(asr, phi, asi * phr));
      const float c1r = float(nr * q), c1i = float(-ni * q);
      cross_axis<R>(v, h ? c1r : c0r, h ? c1i : c0i, nsg);
      phr = nr;
      phi = ni;
      if (--countdown == 0) {
        float m = absmax(v);
        m = fmaxf(m, partner(m));
        acc += rescale(v, m);
        countdown = a.renorm_every;
      }
      cy = cy_next;
      cx = cx_next;
    }
  }

  // closure: lane h sums its entries; lane 1's carry g_x conj(g_y) Phi more
  const float4 gx4 = gA[ic];
  const float4 gy4 = gB[jc];
  const double gxr = gx4.x, gxi = gx4.y, gyr = gy4.x, gyi = -double(gy4.y);
  double sr, si;
  closure_half<R>(v, gxr, gxi, gyr, gyi, sr, si);
  if (h) {
    const double wr = fma(gxr, gyr, -(gxi * gyi));
    const double wi = fma(gxr, gyi, gxi * gyr);
    const double fr = fma(wr, phr, -(wi * phi));
    const double fi = fma(wr, phi, wi * phr);
    const double tr = fma(sr, fr, -(si * fi));
    const double ti = fma(sr, fi, si * fr);
    sr = tr;
    si = ti;
  }
  const double or_ = partner(sr), oi = partner(si);
  // the same order of addition in both lanes: lane 0's part + lane 1's part
  const double tr = h ? or_ + sr : sr + or_;
  const double ti = h ? oi + si : si + oi;
  if (h == 0 && active) {
    const double s2 = comp ? fma(tr, tr, ti * ti) : 1.0;
    // amp = closure * 2^(acc - R n)  =>  K = s2 * 2^(2 (acc - R n))
    store_entry(a, i, j, s2, 2 * (acc - R * a.n));
  }
}

// KB = ket points per block: a block's 4 waves cover KB ket points x 128/KB
// bra points of one tile (32 blocks per tile either way).  W = target waves
// per SIMD.
template <int R, int W, int KB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8)))
sweep_split_kernel(SweepArgs a) {
  const uint32_t L = xcd_logical_block();
  if (L >= a.num_blocks) return;
  const uint32_t tile = L / uint32_t(a.blocks_per_tile);
  const uint32_t sub = L % uint32_t(a.blocks_per_tile);
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t i, j0;
  if constexpr (KB == 2) {
    i = int64_t(ti) * kTile + int64_t(sub) * 2 + (wave >> 1);
    j0 = int64_t(tj) * kTile + 32 * (wave & 1);
  } else {
    i = int64_t(ti) * kTile + int64_t(sub >> 1) * 4 + wave;
    j0 = int64_t(tj) * kTile + 32 * int64_t(sub & 1);
  }
  split_item<R>(a, i, j0);
}

template <int R, int W, int KB>
hipError_t launch_split(const SweepArgs& a0, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = kTile / 2;
  return launch_chunked(a, a.blocks_per_tile, [&](SweepArgs c) {
    const int64_t blocks = launch_tiles(c) * c.blocks_per_tile;
    if (blocks <= 0) return hipSuccess;
    c.num_blocks = uint32_t(blocks);
    const uint32_t padded = uint32_t((blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((sweep_split_kernel<R, W, KB>), dim3(padded), dim3(256), 0, stream, c);
    return hipGetLastError();
  });
}

}  // namespace

// Variants of the split sweep (target waves per SIMD W, ket points per block
// KB); all compute bitwise identical results.  Variant 0 is the default (the
// fastest measured on MI355X at 784 qubits, 2048 points: 140.0 ms against
// 141.5 / 140.2 / 141.6 ms for variants 1..3).
hipError_t launch_sweep_split_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream) {
  switch (reps * 16 + variant) {
    case 64 + 0: return launch_split<4, 3, 2>(a, stream);
    case 64 + 1: return launch_split<4, 2, 2>(a, stream);
    case 64 + 2: return launch_split<4, 3, 4>(a, stream);
    case 64 + 3: return launch_split<4, 2, 4>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qsvm
