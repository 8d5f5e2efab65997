// Launch-shape table of the fill kernels.
#include "zig_tune.hpp"

namespace zig {

bool shape_supported(uint32_t wg, uint32_t spl) {
  const bool w = wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024;
  const bool s = spl == 1 || spl == 2 || spl == 4 || spl == 8;
  return w && s && wg * spl <= 2048;
}

Shape tuned_shape(uint32_t dist, uint32_t dtype, uint64_t n) {
  (void)n;
  Shape s;
  // measured on MI355X at 2^30 outputs: the exponential prefers wide
  // workgroups, the normal distribution (heavier slow path, more
  // registers) longer tiles on narrower ones
  if (dist == 0) {
    s.wg = 512;
    s.spl = 4;
  } else {
    s.wg = 128;
    s.spl = 8;
  }
  (void)dtype;
  // about 16K blocks per step of the tile counter
  s.chunk = 16384 / (s.wg * s.spl);
  if (s.chunk < 1) s.chunk = 1;
  return s;
}

}  // namespace zig
