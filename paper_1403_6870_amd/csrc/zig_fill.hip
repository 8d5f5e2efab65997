// Fill kernels of the modified ziggurat sampler for gfx950.
//
// One workgroup owns one tile of WG * S consecutive Philox blocks (2 FP64
// or 4 FP32 outputs per block) and writes it contiguously; workgroups are
// dispatched in tile order so the whole grid streams through HBM in address
// order.  Per tile:
//   A. every lane computes S blocks; each output takes its layer index and
//      magnitude from its fast word and, when the layer lies under the
//      density (i < L, Table 1 step 2), its value from one multiply by the
//      LDS-resident X_i 2^-53.  Outputs whose layer index is >= L are
//      appended to a per-workgroup LDS queue: one ballot per output slot,
//      one LDS atomic per wave, the lane's offset from mbcnt.
//   B. the workgroup drains the queue, one slow output per lane: region
//      draw, overhang box or tail (Table 1 steps 3-8) on that output's own
//      slow stream; results go back to LDS.
//   C. lanes patch their slow outputs from LDS (or compute them in place
//      when the queue overflowed), apply the location-scale epilogue and
//      issue one 16-byte store per block.
#include <hip/hip_runtime.h>

#include "zig_device.hpp"

namespace zig {
namespace {

template <uint32_t DT>
struct OutType;
template <>
struct OutType<kF64> {
  using T = double;
  static constexpr int per_block = 2;
};
template <>
struct OutType<kF32> {
  using T = float;
  static constexpr int per_block = 4;
};

template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE>
__global__ void __launch_bounds__(WG) fill_kernel(FillArgs a) {
  using OutT = typename OutType<DT>::T;
  constexpr int O = OutType<DT>::per_block;
  constexpr int TILE = WG * S;
  static_assert(S * O <= 32, "slot bitmasks hold 32 outputs per lane");

  __shared__ OutT xs[kMaxLayers];
  __shared__ uint32_t qcount;
  extern __shared__ double qres[];  // [queue] magnitudes, then [queue] u32 slots
  uint32_t* qslot = reinterpret_cast<uint32_t*>(qres + a.queue);

  const DevTable* tb = a.tab;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  for (uint32_t i = tid; i < kMaxLayers; i += WG) {
    if constexpr (DT == kF64)
      xs[i] = tb->XS[i];
    else
      xs[i] = tb->XS32[i];
  }
  if (tid == 0) qcount = 0;
  __syncthreads();

  const uint32_t L = tb->L;
  const uint32_t imask = tb->i_max - 1;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t tile0 = a.blk0 + (uint64_t)blockIdx.x * TILE;
  const double scale = a.scale, shift = a.shift;
  const float fscale = (float)scale, fshift = (float)shift;

  OutT val[S][O];
  uint32_t pos[S][O];
  uint32_t slowbits = 0, negbits = 0;

#pragma unroll
  for (int s = 0; s < S; ++s) {
    const uint64_t m = tile0 + (uint64_t)(s * WG) + tid;
    uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = (DT == kF64) ? 0u : 1u;
    dev::philox10(c0, c1, c2, c3, k0, k1);
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const uint64_t g = m * O + o;
      const bool live = (m <= a.blk_last) && (g >= a.first) && (g <= a.last);
      uint32_t i;
      OutT x;
      bool neg = false;
      if constexpr (DT == kF64) {
        const uint64_t w = (o == 0) ? ((uint64_t)c0 | ((uint64_t)c1 << 32)) : ((uint64_t)c2 | ((uint64_t)c3 << 32));
        i = (uint32_t)w & imask;
        x = (double)(w >> 11) * xs[i];
        if constexpr (DIST == kDistNormal) neg = (w >> 10) & 1u;
      } else {
        const uint32_t w = (o == 0) ? c0 : (o == 1) ? c1 : (o == 2) ? c2 : c3;
        i = w & imask;
        if constexpr (DIST == kDistExp) {
          x = (float)(w >> 8) * xs[i];
        } else {
          x = (float)(w >> 9) * xs[i];
          neg = (w >> 8) & 1u;
        }
      }
      const uint32_t bit = 1u << (s * O + o);
      if (neg) {
        x = -x;
        negbits |= bit;
      }
      if constexpr (DT == kF64)
        val[s][o] = __builtin_fma(scale, x, shift);
      else
        val[s][o] = __builtin_fmaf(fscale, x, fshift);
      const bool slow = live && (i >= L);
      const uint64_t mask = __ballot(slow);
      if (mask != 0) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if ((int)lane == leader) base = atomicAdd(&qcount, (uint32_t)__popcll(mask));
        base = __builtin_amdgcn_readlane(base, leader);
        if (slow) {
          const uint32_t p = base + dev::lanes_below(mask);
          pos[s][o] = p;
          slowbits |= bit;
          if (p < a.queue) qslot[p] = (uint32_t)((s * WG + tid) * O + o);
        }
      }
      if constexpr (TRACE) {
        if (live) {
          const uint64_t k = g - a.first;
          if (a.t_layer) a.t_layer[k] = i;
          if (!slow) {
            if (a.t_region) a.t_region[k] = -1;
            if (a.t_words) a.t_words[k] = 0;
            if (a.t_tests) a.t_tests[k] = 0;
          }
        }
      }
    }
  }
  __syncthreads();

  // B: drain the queue
  {
    const uint32_t cnt = min(qcount, a.queue);
    for (uint32_t e = tid; e < cnt; e += WG) {
      const uint32_t slot = qslot[e];
      const uint64_t g = (tile0 + slot / O) * O + (slot % O);
      int32_t region;
      uint32_t words, tests;
      qres[e] = dev::slow_magnitude<DIST>(tb, a.etab, g, k0, k1, region, words, tests);
      if constexpr (TRACE) {
        const uint64_t k = g - a.first;
        if (a.t_region) a.t_region[k] = region;
        if (a.t_words) a.t_words[k] = words;
        if (a.t_tests) a.t_tests[k] = tests;
      }
    }
  }
  __syncthreads();

  // C: patch slow outputs, store
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const uint64_t m = tile0 + (uint64_t)(s * WG) + tid;
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const uint32_t bit = 1u << (s * O + o);
      if (slowbits & bit) {
        const uint32_t p = pos[s][o];
        double mag;
        if (p < a.queue) {
          mag = qres[p];
        } else {
          const uint64_t g = m * O + o;
          int32_t region;
          uint32_t words, tests;
          mag = dev::slow_magnitude<DIST>(tb, a.etab, g, k0, k1, region, words, tests);
          if constexpr (TRACE) {
            const uint64_t k = g - a.first;
            if (a.t_region) a.t_region[k] = region;
            if (a.t_words) a.t_words[k] = words;
            if (a.t_tests) a.t_tests[k] = tests;
          }
        }
        OutT x = (OutT)mag;
        if (negbits & bit) x = -x;
        if constexpr (DT == kF64)
          val[s][o] = __builtin_fma(scale, x, shift);
        else
          val[s][o] = __builtin_fmaf(fscale, x, fshift);
      }
    }
    if (m > a.blk_last) continue;
    const uint64_t g0 = m * O;
    OutT* out = static_cast<OutT*>(a.out);
    if (a.aligned16 && g0 >= a.first && g0 + (O - 1) <= a.last) {
      if constexpr (DT == kF64) {
        double2 v;
        v.x = val[s][0];
        v.y = val[s][1];
        *reinterpret_cast<double2*>(out + (g0 - a.first)) = v;
      } else {
        float4 v;
        v.x = val[s][0];
        v.y = val[s][1];
        v.z = val[s][2];
        v.w = val[s][3];
        *reinterpret_cast<float4*>(out + (g0 - a.first)) = v;
      }
    } else {
#pragma unroll
      for (int o = 0; o < O; ++o) {
        const uint64_t g = g0 + o;
        if (g >= a.first && g <= a.last) out[g - a.first] = val[s][o];
      }
    }
  }
}

template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE>
int launch_one(uint64_t grid, const FillArgs& a, hipStream_t st) {
  const size_t lds = (size_t)a.queue * (sizeof(double) + sizeof(uint32_t));
  hipLaunchKernelGGL((fill_kernel<DIST, DT, WG, S, TRACE>), dim3((uint32_t)grid), dim3(WG), lds, st, a);
  return (int)hipGetLastError();
}

template <uint32_t DIST, uint32_t DT, bool TRACE>
int launch_shape(uint32_t wg, uint32_t spl, uint64_t grid, const FillArgs& a, hipStream_t st) {
#define ZIG_SHAPE(W, S_) \
  if (wg == W && spl == S_) return launch_one<DIST, DT, W, S_, TRACE>(grid, a, st);
  if constexpr (!TRACE) {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(64, 2) ZIG_SHAPE(64, 4) ZIG_SHAPE(64, 8)
    ZIG_SHAPE(128, 1) ZIG_SHAPE(128, 2) ZIG_SHAPE(128, 4) ZIG_SHAPE(128, 8)
    ZIG_SHAPE(256, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4) ZIG_SHAPE(256, 8)
    ZIG_SHAPE(512, 1) ZIG_SHAPE(512, 2) ZIG_SHAPE(512, 4) ZIG_SHAPE(512, 8)
  } else {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4)
  }
#undef ZIG_SHAPE
  return (int)hipErrorInvalidConfiguration;
}

}  // namespace

int launch_fill(uint32_t dist, uint32_t dtype, uint32_t wg, uint32_t spl, bool trace, uint64_t grid, const FillArgs& a,
                void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (trace) {
    if (dist == kDistExp && dtype == kF64) return launch_shape<kDistExp, kF64, true>(wg, spl, grid, a, st);
    if (dist == kDistExp && dtype == kF32) return launch_shape<kDistExp, kF32, true>(wg, spl, grid, a, st);
    if (dist == kDistNormal && dtype == kF64) return launch_shape<kDistNormal, kF64, true>(wg, spl, grid, a, st);
    if (dist == kDistNormal && dtype == kF32) return launch_shape<kDistNormal, kF32, true>(wg, spl, grid, a, st);
  } else {
    if (dist == kDistExp && dtype == kF64) return launch_shape<kDistExp, kF64, false>(wg, spl, grid, a, st);
    if (dist == kDistExp && dtype == kF32) return launch_shape<kDistExp, kF32, false>(wg, spl, grid, a, st);
    if (dist == kDistNormal && dtype == kF64) return launch_shape<kDistNormal, kF64, false>(wg, spl, grid, a, st);
    if (dist == kDistNormal && dtype == kF32) return launch_shape<kDistNormal, kF32, false>(wg, spl, grid, a, st);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace zig
