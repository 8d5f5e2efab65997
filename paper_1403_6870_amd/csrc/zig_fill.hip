// Instantiations and launcher of the fill kernel (zig_fill_kernel.hpp).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

// Workgroups of one kernel variant resident on the whole device.
template <class K>
int resident_groups(K kernel, int wg, size_t lds, int* out) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t, int>, int> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  const auto key = std::make_tuple((const void*)kernel, wg, lds, dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return 0;
  }
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, wg, lds);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  if (per_cu < 1) return (int)hipErrorInvalidConfiguration;
  *out = per_cu * cus;
  cache[key] = *out;
  return 0;
}

template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE, bool ACCEL>
int launch_one(const FillArgs& args, hipStream_t st) {
  auto kernel = fill_kernel<DIST, DT, WG, S, TRACE, ACCEL>;
  int groups = 0;
  int e = resident_groups(kernel, WG, 0, &groups);
  if (e != 0) return e;
  FillArgs a = args;
  // tiles per counter step: as asked, but small enough that every resident
  // workgroup gets a couple of steps
  uint64_t chunk = a.tiles / (2ull * (uint64_t)groups);
  if (chunk > a.chunk) chunk = a.chunk;
  if (chunk < 1) chunk = 1;
  a.chunk = (uint32_t)chunk;
  const uint64_t steps = (a.tiles + chunk - 1) / chunk;
  const uint32_t grid = steps < (uint64_t)groups ? (uint32_t)steps : (uint32_t)groups;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(WG), 0, st, a);
  return (int)hipGetLastError();
}

template <uint32_t DIST, uint32_t DT, bool TRACE, bool ACCEL = false>
int launch_shape(uint32_t wg, uint32_t spl, const FillArgs& a, hipStream_t st) {
#define ZIG_SHAPE(W, S_) \
  if (wg == W && spl == S_) return launch_one<DIST, DT, W, S_, TRACE, ACCEL>(a, st);
  if constexpr (!TRACE) {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(64, 2) ZIG_SHAPE(64, 4) ZIG_SHAPE(64, 8)
    ZIG_SHAPE(128, 1) ZIG_SHAPE(128, 2) ZIG_SHAPE(128, 4) ZIG_SHAPE(128, 8)
    ZIG_SHAPE(256, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4) ZIG_SHAPE(256, 8)
    ZIG_SHAPE(512, 1) ZIG_SHAPE(512, 2) ZIG_SHAPE(512, 4)
    ZIG_SHAPE(1024, 1) ZIG_SHAPE(1024, 2)
  } else {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4)
  }
#undef ZIG_SHAPE
  return (int)hipErrorInvalidConfiguration;
}

}  // namespace

int launch_fill(uint32_t dist, uint32_t dtype, uint32_t wg, uint32_t spl, bool trace, const FillArgs& a,
                void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dist == kDistNormal && a.accel) {  // the accelerated overhang variant
    if (trace) {
      if (dtype == kF64) return launch_shape<kDistNormal, kF64, true, true>(wg, spl, a, st);
      if (dtype == kF32) return launch_shape<kDistNormal, kF32, true, true>(wg, spl, a, st);
    } else {
      if (dtype == kF64) return launch_shape<kDistNormal, kF64, false, true>(wg, spl, a, st);
      if (dtype == kF32) return launch_shape<kDistNormal, kF32, false, true>(wg, spl, a, st);
    }
    return (int)hipErrorInvalidValue;
  }
  if (trace) {
    if (dist == kDistExp && dtype == kF64) return launch_shape<kDistExp, kF64, true>(wg, spl, a, st);
    if (dist == kDistExp && dtype == kF32) return launch_shape<kDistExp, kF32, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF64) return launch_shape<kDistNormal, kF64, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF32) return launch_shape<kDistNormal, kF32, true>(wg, spl, a, st);
  } else {
    if (dist == kDistExp && dtype == kF64) return launch_shape<kDistExp, kF64, false>(wg, spl, a, st);
    if (dist == kDistExp && dtype == kF32) return launch_shape<kDistExp, kF32, false>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF64) return launch_shape<kDistNormal, kF64, false>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF32) return launch_shape<kDistNormal, kF32, false>(wg, spl, a, st);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace zig
