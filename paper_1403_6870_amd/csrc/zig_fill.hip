// Instantiations and launcher of the fill kernel (zig_fill_kernel.hpp).
#include <hip/hip_runtime.h>

#include "zig_fill_kernel.hpp"

namespace zig {

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
