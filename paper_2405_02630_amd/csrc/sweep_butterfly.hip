// Single-Gram launch of the butterfly sweep (device code of one work item in
// sweep_butterfly_item.h): one grid over the tiles of one Gram, blocks mapped
// XCD-aware, with the kernel variants the autotuner chooses among.

#include <atomic>

#include "sweep_butterfly_item.h"

namespace qsvm {
namespace {

// One launch over the tiles of one Gram.  W = target waves per SIMD (the
// register budget the compiler must fit: 512 / W VGPRs).
template <int R, int PI, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8)))
sweep_butterfly_kernel(SweepArgs a) {
  const uint32_t L = xcd_logical_block();
  if (L >= a.num_blocks) return;
  const uint32_t tile = L / uint32_t(a.blocks_per_tile);
  const uint32_t sub = L % uint32_t(a.blocks_per_tile);
  int32_t ti, tj;
  if (!decode_tile(a, tile, ti, tj)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i0 = int64_t(ti) * kTile + (int64_t(sub) * 4 + wave) * PI;  // wave-uniform
  butterfly_item<R, PI>(a, i0, int64_t(tj) * kTile);
}

template <int R, int PI, int W>
hipError_t launch_pi(const SweepArgs& a0, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = kTile / (4 * PI);
  return launch_chunked(a, a.blocks_per_tile, [&](SweepArgs c) {
    const int64_t blocks = launch_tiles(c) * c.blocks_per_tile;
    if (blocks <= 0) return hipSuccess;
    c.num_blocks = uint32_t(blocks);
    const uint32_t padded = uint32_t((blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((sweep_butterfly_kernel<R, PI, W>), dim3(padded), dim3(256), 0, stream, c);
    return hipGetLastError();
  });
}

// Persistent form for a tile list whose length is read on the device
// (a.tile_count): every block strides over the (tile, block of the tile)
// items in the XCD-aware order until the listed tiles are done.
template <int R, int PI, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8)))
sweep_butterfly_list_kernel(SweepArgs a) {
  const uint64_t bpt = uint64_t(a.blocks_per_tile);
  const uint64_t items = uint64_t(device_tiles(a)) * bpt;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint64_t L = xcd_logical_block(); L < items; L += gridDim.x) {
    const uint32_t tile = uint32_t(L / bpt);
    const uint32_t sub = uint32_t(L % bpt);
    int32_t ti, tj;
    if (!decode_tile(a, tile, ti, tj)) continue;
    const int64_t i0 = int64_t(ti) * kTile + (int64_t(sub) * 4 + wave) * PI;  // wave-uniform
    butterfly_item<R, PI>(a, i0, int64_t(tj) * kTile);
  }
}

// Blocks of the persistent form that fit the device at once (cached per
// device and kernel variant), a multiple of 8 for the XCD-aware order.
template <int R, int PI, int W>
hipError_t list_grid(int64_t* out) {
  static std::atomic<int64_t> cache[64];  // zero-initialised (static storage)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < 64) {
    const int64_t v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) {
      *out = v;
      return hipSuccess;
    }
  }
  int cus = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_butterfly_list_kernel<R, PI, W>, 256, 0);
  if (e != hipSuccess) return e;
  int64_t g = int64_t(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1) / 8 * 8;
  if (g < 8) g = 8;
  if (dev >= 0 && dev < 64) cache[dev].store(g, std::memory_order_relaxed);
  *out = g;
  return hipSuccess;
}

template <int R, int PI, int W>
hipError_t launch_list_pi(const SweepArgs& a0, hipStream_t stream) {
  SweepArgs a = a0;
  a.blocks_per_tile = kTile / (4 * PI);
  int64_t grid = 0;
  hipError_t e = list_grid<R, PI, W>(&grid);
  if (e != hipSuccess) return e;
  const int64_t most = launch_tiles(a) * a.blocks_per_tile;  // the list's capacity in blocks
  if (most <= 0) return hipSuccess;
  if (grid > most) grid = (most + 7) / 8 * 8;
  a.num_blocks = uint32_t(grid);
  hipLaunchKernelGGL((sweep_butterfly_list_kernel<R, PI, W>), dim3(unsigned(grid)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

// Kernel variants (ket points per lane PI, target waves per SIMD W); all
// compute bitwise identical results.  Variant 0 of each reps is the default:
// the fastest measured on MI355X for 784 qubits and 2048..4096 points.
hipError_t launch_sweep_butterfly_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream) {
  switch (reps * 16 + variant) {
    case 16 + 0: return launch_pi<1, 4, 4>(a, stream);
    case 16 + 1: return launch_pi<1, 4, 8>(a, stream);
    case 16 + 2: return launch_pi<1, 8, 4>(a, stream);
    case 16 + 3: return launch_pi<1, 8, 2>(a, stream);
    case 32 + 0: return launch_pi<2, 2, 4>(a, stream);
    case 32 + 1: return launch_pi<2, 4, 4>(a, stream);
    case 32 + 2: return launch_pi<2, 4, 2>(a, stream);
    case 32 + 3: return launch_pi<2, 2, 8>(a, stream);
    case 48 + 0: return launch_pi<3, 1, 2>(a, stream);
    case 48 + 1: return launch_pi<3, 2, 2>(a, stream);
    case 48 + 2: return launch_pi<3, 1, 3>(a, stream);
    case 48 + 3: return launch_pi<3, 1, 4>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

// Ket points per lane of a variant (the PI of the table above).
int32_t butterfly_variant_pi(int32_t reps, int32_t variant) {
  static constexpr int32_t kPi[3][4] = {{4, 4, 8, 8}, {2, 4, 4, 2}, {1, 2, 1, 1}};
  if (reps < 1 || reps > 3 || variant < 0 || variant >= kButterflyVariants) return 0;
  return kPi[reps - 1][variant];
}

}  // namespace qsvm

namespace qsvm {

// The persistent form over a tile list of device-resident length.  Inside
// the persistent loop the compiler keeps more values live than in the
// one-item kernel, so each reps uses one variant that compiles without
// register spills (results are bitwise those of every variant).
hipError_t launch_sweep_butterfly_counted(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream) {
  if (!a.tile_list || !a.tile_count || variant < 0 || variant >= kButterflyVariants) return hipErrorInvalidValue;
  switch (reps) {
    case 1: return launch_list_pi<1, 4, 4>(a, stream);
    case 2: return launch_list_pi<2, 2, 4>(a, stream);
    case 3: return launch_list_pi<3, 1, 2>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qsvm
