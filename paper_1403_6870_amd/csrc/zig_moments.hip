// Fused generate-and-reduce: the raw moment sums S_p = sum of x^p, p = 1..5,
// of the outputs a fill would write, with no output written to HBM.
//
// The summation order is part of the definition, so that the result is the
// same bits whatever the launch shape or scheduling:
//   - tiles of 2048 Philox blocks from the fill's first block; in a tile,
//     lane l (0..255) adds the outputs of blocks l, l + 256, ..., l + 1792
//     in order (the fill's own tile code, with the tile reduced instead of
//     stored), and the lane sums are reduced by halving;
//   - groups of 256 tiles are reduced the same way (the last group padded
//     with zeros);
//   - the total is +0 plus the group sums in order.
// A fill is processed in segments of 2^16 tiles (256 groups): the tile
// kernel writes per-tile sums, the group kernel per-group sums, and the
// total kernel continues the running total in `sums`.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

constexpr int kMomWG = 256;
constexpr int kMomS = 8;

template <uint32_t DIST, uint32_t DT, bool ACCEL>
__global__ void __launch_bounds__(kMomWG) moments_kernel(FillArgs a, double* tile_sums) {
  // the slow-path tables stay in device memory, as in the fill's 256 x 8
  // kernel: one more workgroup per CU
  __shared__ FillLds<DT, kMomWG, kMomS, kLdsLayers, !lean_shape(kMomWG, kMomS)> sh;
  const FillCtx c = load_tables<DIST, DT, kMomWG, kMomS, kLdsLayers, !lean_shape(kMomWG, kMomS)>(a, sh);
  TileLds tl;
  tl.stage = sh.stage;
  tl.slowmap = sh.slowmap;
  tl.prefix = sh.prefix;
  for (;;) {
    if (threadIdx.x == 0) sh.tile = atomicAdd(&a.counters[0], 1u);
    __syncthreads();
    const uint64_t t0 = (uint64_t)sh.tile * a.chunk;
    if (t0 >= a.tiles) break;
    const uint64_t t1 = t0 + a.chunk < a.tiles ? t0 + a.chunk : a.tiles;
    for (uint64_t t = t0; t < t1; ++t) {
      fill_tile<DIST, DT, kMomWG, kMomS, false, true, ACCEL>(a, c, tl, (uint32_t)t, tile_sums + 5 * t);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(&a.counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&a.counters[0], 0u);
      atomicExch(&a.counters[1], 0u);
    }
  }
}

// Group k = blockIdx.x: halving reduction of tile sums 256k .. 256k + 255.
__global__ void __launch_bounds__(256) group_kernel(const double* tile_sums, uint32_t tiles, double* group_sums) {
  __shared__ double red[5][256];
  const uint32_t tid = threadIdx.x;
  const uint32_t i = blockIdx.x * 256u + tid;
#pragma unroll
  for (int p = 0; p < 5; ++p) red[p][tid] = i < tiles ? tile_sums[(size_t)i * 5 + p] : 0.0;
  __syncthreads();
  for (uint32_t h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int p = 0; p < 5; ++p) red[p][tid] = red[p][tid] + red[p][tid + h];
    }
    __syncthreads();
  }
  if (tid < 5) group_sums[(size_t)blockIdx.x * 5 + tid] = red[tid][0];
}

// sums[p] = (running total or +0) + group sums in order; one lane per p.
__global__ void total_kernel(const double* group_sums, uint32_t groups, double* sums, uint32_t accumulate) {
  const uint32_t p = threadIdx.x;
  if (p >= 5) return;
  double t = accumulate ? sums[p] : 0.0;
  for (uint32_t k = 0; k < groups; ++k) t = t + group_sums[(size_t)k * 5 + p];
  sums[p] = t;
}

template <class K>
int resident(K kernel, int* out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair((const void*)kernel, dev);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return 0;
  }
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kMomWG, 0);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  if (per_cu < 1) return (int)hipErrorInvalidConfiguration;
  *out = cache[key] = per_cu * cus;
  return 0;
}

template <uint32_t DIST, uint32_t DT, bool ACCEL = false>
int launch_segment(const FillArgs& args, double* tile_sums, hipStream_t st) {
  auto kernel = moments_kernel<DIST, DT, ACCEL>;
  int groups = 0;
  int e = resident(kernel, &groups);
  if (e != 0) return e;
  FillArgs a = args;
  uint64_t chunk = a.tiles / (2ull * (uint64_t)groups);
  if (chunk > a.chunk) chunk = a.chunk;
  if (chunk < 1) chunk = 1;
  a.chunk = (uint32_t)chunk;
  const uint64_t steps = (a.tiles + chunk - 1) / chunk;
  const uint32_t grid = steps < (uint64_t)groups ? (uint32_t)steps : (uint32_t)groups;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(kMomWG), 0, st, a, tile_sums);
  return (int)hipGetLastError();
}

}  // namespace

int launch_moments_segment(uint32_t dist, uint32_t dtype, const FillArgs& a, double* tile_sums, double* group_sums,
                           double* sums, bool accumulate, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  int e;
  if (dist == kDistNormal && a.accel)
    e = dtype == kF64 ? launch_segment<kDistNormal, kF64, true>(a, tile_sums, st)
                      : launch_segment<kDistNormal, kF32, true>(a, tile_sums, st);
  else if (dist == kDistExp && dtype == kF64)
    e = launch_segment<kDistExp, kF64>(a, tile_sums, st);
  else if (dist == kDistExp && dtype == kF32)
    e = launch_segment<kDistExp, kF32>(a, tile_sums, st);
  else if (dist == kDistNormal && dtype == kF64)
    e = launch_segment<kDistNormal, kF64>(a, tile_sums, st);
  else
    e = launch_segment<kDistNormal, kF32>(a, tile_sums, st);
  if (e != 0) return e;
  const uint32_t ngroups = (uint32_t)((a.tiles + 255) / 256);
  hipLaunchKernelGGL(group_kernel, dim3(ngroups), dim3(256), 0, st, tile_sums, (uint32_t)a.tiles, group_sums);
  e = (int)hipGetLastError();
  if (e != 0) return e;
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, st, group_sums, ngroups, sums, accumulate ? 1u : 0u);
  return (int)hipGetLastError();
}

int launch_moments_zero(double* sums, void* stream) {
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), nullptr, 0u, sums, 0u);
  return (int)hipGetLastError();
}

}  // namespace zig
