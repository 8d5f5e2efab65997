// Launch-shape table of the fill kernels.
#pragma once

#include <cstdint>

namespace zig {

struct Shape {
  uint32_t wg;   // lanes per workgroup
  uint32_t spl;    // Philox blocks per lane per tile
  uint32_t chunk;  // tiles per step of the tile counter
};

// shapes compiled into the library
bool shape_supported(uint32_t wg, uint32_t spl);

// shape for a fill of n outputs (tuned table, else the built-in default)
Shape tuned_shape(uint32_t dist, uint32_t dtype, uint64_t n);

}  // namespace zig
