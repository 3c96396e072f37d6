// Device helpers shared by the two sweep kernels: tile decoding, the
// XCD-aware block order, and the FP64 finalize/store of one kernel entry.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "qsvm_internal.h"

namespace qsvm {

constexpr int kTile = 64;  // tile edge in points: one wave's lanes span the bra side

// Kernel arguments common to both sweeps (device-side copy of GramLaunch).
struct SweepArgs {
  const float4* gen_a;   // Section G of the ket set (butterfly sweep)
  const float4* gen_b;   // Section G of the bra set
  const float2* dense_a; // Section D of the ket set (dense sweep)
  const float2* dense_b; // Section D of the bra set
  double* K;
  double* log_k;
  int64_t Na, Nb, ldk;
  int64_t row_begin, row_end;
  int32_t n;
  int32_t renorm_every;
  int32_t sym, diag_mode;
  int32_t tile_row0;     // first tile row in the row range
  int32_t tile_rows;     // tile rows in the row range
  int32_t tiles_b;       // tile columns (ceil(Nb / 64))
  int32_t blocks_per_tile;
  uint32_t num_blocks;   // logical blocks (before padding to a multiple of 8)
  const int32_t* tile_list;  // optional device list of (ti, tj) tiles (symmetric only)
  const int32_t* tile_count; // optional: with tile_list, the list length is read here on the
                             // device, clamped to [0, tile_rows] (tile_rows = the list capacity)
};

// Tiles one launch covers: the list length, the upper triangle of the row
// range (symmetric) or the full row range x column grid (rectangular).
__host__ __device__ inline int64_t launch_tiles(const SweepArgs& a) {
  if (a.tile_list) return a.tile_rows;
  if (a.sym)
    return int64_t(a.tile_rows) * a.tiles_b - (int64_t(a.tile_rows) * (a.tile_rows - 1)) / 2 -
           int64_t(a.tile_rows) * a.tile_row0;
  return int64_t(a.tile_rows) * a.tiles_b;
}

// Tiles of the launch as the device sees them: launch_tiles, or the listed
// count when the list length lives in device memory.
__device__ __forceinline__ int64_t device_tiles(const SweepArgs& a) {
  const int64_t t = launch_tiles(a);
  if (!a.tile_count) return t;
  const int64_t c = *a.tile_count;
  return c < 0 ? 0 : (c < t ? c : t);
}

// A dispatch carries its grid size in work-items as a 32-bit number, so one
// launch of 256-thread blocks holds fewer than 2^24 blocks.
constexpr int64_t kMaxGridBlocks = (int64_t(1) << 24) - 8;

// Issue the tiles of `a` as one or more launches of at most kMaxGridBlocks
// blocks each: consecutive tile rows (the row range narrowed to them) or
// consecutive stretches of the tile list.  `one(chunk)` launches one chunk.
// A single tile row too wide for one launch is an error.
template <class F>
hipError_t launch_chunked(const SweepArgs& a, int64_t blocks_per_tile, F one) {
  const int64_t cap = kMaxGridBlocks / blocks_per_tile;  // tiles per launch
  if (a.tile_list) {
    for (int64_t off = 0; off < a.tile_rows; off += cap) {
      SweepArgs c = a;
      c.tile_list = a.tile_list + 2 * off;
      c.tile_rows = int32_t((a.tile_rows - off < cap) ? a.tile_rows - off : cap);
      const hipError_t e = one(c);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t t_end = int64_t(a.tile_row0) + a.tile_rows;
  for (int64_t t = a.tile_row0; t < t_end;) {
    // tiles of tile row u: the full grid, or the upper triangle from u on
    auto row_tiles = [&](int64_t u) { return a.sym ? a.tiles_b - u : int64_t(a.tiles_b); };
    if (row_tiles(t) > cap) return hipErrorInvalidConfiguration;
    int64_t m = 0, tiles = 0;
    while (t + m < t_end && tiles + row_tiles(t + m) <= cap) tiles += row_tiles(t + m++);
    SweepArgs c = a;
    c.tile_row0 = int32_t(t);
    c.tile_rows = int32_t(m);
    c.row_begin = (t * kTile > a.row_begin) ? t * kTile : a.row_begin;
    c.row_end = ((t + m) * kTile < a.row_end) ? (t + m) * kTile : a.row_end;
    const hipError_t e = one(c);
    if (e != hipSuccess) return e;
    t += m;
  }
  return hipSuccess;
}

// Map the hardware block index to a logical block so that the blocks of one
// tile run back to back on the same XCD (the dispatcher hands consecutive
// block indices to the 8 XCDs round robin).  The grid is padded to a
// multiple of 8; padded slots return num_blocks or more.
__device__ __forceinline__ uint32_t xcd_logical_block() {
  const uint32_t b = blockIdx.x;
  const uint32_t per_xcd = gridDim.x >> 3;
  return (b & 7u) * per_xcd + (b >> 3);
}

// Tile (row, column) of logical tile u.  Symmetric: upper triangle
// (row <= column) of tile rows [tile_row0, tile_row0 + tile_rows), row-major;
// or entry u of the tile list, when one is given.  Returns false for a list
// entry outside 0 <= ti <= tj < tiles_b (the work item is then skipped).
__device__ __forceinline__ bool decode_tile(const SweepArgs& a, uint32_t u, int32_t& ti, int32_t& tj) {
  if (a.tile_list) {
    ti = a.tile_list[2 * int64_t(u)];
    tj = a.tile_list[2 * int64_t(u) + 1];
    return ti >= 0 && ti <= tj && tj < a.tiles_b;
  }
  if (!a.sym) {
    ti = a.tile_row0 + int32_t(u / uint32_t(a.tiles_b));
    tj = int32_t(u % uint32_t(a.tiles_b));
    return true;
  }
  const int64_t T = a.tiles_b;
  // offset(t) = t*T - t*(t-1)/2 tiles precede tile row t
  auto offset = [T](int64_t t) { return t * T - (t * (t - 1)) / 2; };
  const int64_t U = int64_t(u) + offset(a.tile_row0);
  const double q = double(2 * T + 1);
  int64_t t = int64_t((q - sqrt(q * q - 8.0 * double(U))) * 0.5);
  if (t < 0) t = 0;
  while (t + 1 < T && offset(t + 1) <= U) ++t;
  while (t > 0 && offset(t) > U) --t;
  ti = int32_t(t);
  tj = int32_t(t + (U - offset(t)));
  return true;
}

// Finalize one pair: amp = s * 2^(e2/2) where |s|^2 = s2 and e2 = 2*(log2
// exponent); write K (and log K) with the symmetric mirror when asked.
__device__ __forceinline__ void store_entry(const SweepArgs& a, int64_t i, int64_t j, double s2,
                                            int32_t e2) {
  double kv, lk;
  if (a.sym && i == j && a.diag_mode == 0) {
    kv = 1.0;
    lk = 0.0;
  } else {
    kv = ldexp(s2, e2);
    lk = (s2 > 0.0) ? log(s2) + double(e2) * 0.69314718055994530942 : -INFINITY;
  }
  a.K[i * a.ldk + j] = kv;
  if (a.log_k) a.log_k[i * a.ldk + j] = lk;
  if (a.sym && i != j) {
    a.K[j * a.ldk + i] = kv;
    if (a.log_k) a.log_k[j * a.ldk + i] = lk;
  }
}

// Is pair (i, j) one this launch must write?
__device__ __forceinline__ bool pair_active(const SweepArgs& a, int64_t i, int64_t j) {
  if (i >= a.Na || j >= a.Nb) return false;
  if (i < a.row_begin || i >= a.row_end) return false;
  if (a.sym && j < i) return false;
  return true;
}

// Does the pair need a contraction (the symmetric diagonal may be assigned)?
__device__ __forceinline__ bool pair_computed(const SweepArgs& a, int64_t i, int64_t j) {
  return pair_active(a, i, j) && !(a.sym && i == j && a.diag_mode == 0);
}

}  // namespace qsvm
