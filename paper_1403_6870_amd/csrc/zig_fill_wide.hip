// Instantiations and launcher of the fill kernel for tables of more than
// 256 layers (Appendix D item 1 names 1024): the fast-path table of up to
// 1024 entries in LDS, the slow-path tables read from device memory.
#include <hip/hip_runtime.h>

#include "zig_fill_kernel.hpp"

namespace zig {

int launch_fill_wide(uint32_t dist, uint32_t dtype, uint32_t wg, uint32_t spl, bool trace, const FillArgs& a,
                     void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.accel || a.ttab != nullptr) return (int)hipErrorInvalidValue;
  if (trace) {
    if (dist == kDistExp && dtype == kF64)
      return launch_shape<kDistExp, kF64, true, false, false, true>(wg, spl, a, st);
    if (dist == kDistExp && dtype == kF32)
      return launch_shape<kDistExp, kF32, true, false, false, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF64)
      return launch_shape<kDistNormal, kF64, true, false, false, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF32)
      return launch_shape<kDistNormal, kF32, true, false, false, true>(wg, spl, a, st);
  } else {
    if (dist == kDistExp && dtype == kF64)
      return launch_shape<kDistExp, kF64, false, false, false, true>(wg, spl, a, st);
    if (dist == kDistExp && dtype == kF32)
      return launch_shape<kDistExp, kF32, false, false, false, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF64)
      return launch_shape<kDistNormal, kF64, false, false, false, true>(wg, spl, a, st);
    if (dist == kDistNormal && dtype == kF32)
      return launch_shape<kDistNormal, kF32, false, false, false, true>(wg, spl, a, st);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace zig
