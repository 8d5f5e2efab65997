// Instantiations and launcher of the fill kernel running the traditional
// ziggurat (the comparison sampler of Table 1), FP64, on the same tile,
// compaction and store structure as the modified sampler.
#include <hip/hip_runtime.h>

#include "zig_fill_kernel.hpp"

namespace zig {

int launch_trad(uint32_t dist, uint32_t wg, uint32_t spl, const FillArgs& a, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.ttab == nullptr || a.tetab == nullptr) return (int)hipErrorInvalidValue;
  if (dist == kDistExp) return launch_shape<kDistExp, kF64, false, false, true>(wg, spl, a, st);
  if (dist == kDistNormal) return launch_shape<kDistNormal, kF64, false, false, true>(wg, spl, a, st);
  return (int)hipErrorInvalidValue;
}

}  // namespace zig
