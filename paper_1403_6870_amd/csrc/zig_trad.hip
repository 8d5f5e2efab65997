// Instantiations and launcher of the fill kernel running the traditional
// ziggurat (the comparison sampler of Table 1), FP64, on the same tile,
// compaction and store structure as the modified sampler.
#include <hip/hip_runtime.h>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

template <uint32_t DIST>
int launch_trad_shape(uint32_t wg, uint32_t spl, const FillArgs& a, hipStream_t st) {
#define ZIG_SHAPE(W, S_) \
  if (wg == W && spl == S_) return launch_one<DIST, kF64, W, S_, false, false, true>(a, st);
  ZIG_SHAPE(64, 1) ZIG_SHAPE(64, 2) ZIG_SHAPE(64, 4) ZIG_SHAPE(64, 8)
  ZIG_SHAPE(128, 1) ZIG_SHAPE(128, 2) ZIG_SHAPE(128, 4) ZIG_SHAPE(128, 8)
  ZIG_SHAPE(256, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4) ZIG_SHAPE(256, 8)
  ZIG_SHAPE(512, 1) ZIG_SHAPE(512, 2) ZIG_SHAPE(512, 4)
  ZIG_SHAPE(1024, 1) ZIG_SHAPE(1024, 2)
#undef ZIG_SHAPE
  return (int)hipErrorInvalidConfiguration;
}

}  // namespace

int launch_trad(uint32_t dist, uint32_t wg, uint32_t spl, const FillArgs& a, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.ttab == nullptr || a.tetab == nullptr) return (int)hipErrorInvalidValue;
  if (dist == kDistExp) return launch_trad_shape<kDistExp>(wg, spl, a, st);
  if (dist == kDistNormal) return launch_trad_shape<kDistNormal>(wg, spl, a, st);
  return (int)hipErrorInvalidValue;
}

}  // namespace zig
