// Instantiations and launcher of the fill kernel (zig_fill_kernel.hpp).
#include <hip/hip_runtime.h>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

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
