// Launch-shape table of the fill and batch kernels, and the autotuner.
#pragma once

#include <cstdint>

namespace zig {

struct Shape {
  uint32_t wg;     // lanes per workgroup
  uint32_t spl;    // Philox blocks per lane per tile
  uint32_t chunk;  // tiles per step of the tile counter
};

constexpr uint32_t kSizeClasses = 4;  // n <= 2^17, <= 2^21, <= 2^25, larger

// shapes compiled into the library
bool shape_supported(uint32_t wg, uint32_t spl);

uint32_t size_class(uint64_t n);

// shape for a fill of n outputs on the current device: the tuned table if
// the device has one (measured, or loaded from the cache), else built in
Shape tuned_shape(uint32_t dist, uint32_t dtype, uint64_t n);

// default batch-kernel shape on the current device
void tuned_batch_shape(uint32_t* wg, uint32_t* spl);

// A fill with an explicit shape (zig_api.cpp); used by the tuner.
int fill_shaped(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double p0, double p1,
                void* out, void* stream, const Shape& shape);

}  // namespace zig
