// Batch kernel: many fill requests of uneven sizes, mixed distributions,
// output types and parameters in one persistent launch.
//
// Every request is cut into tiles exactly as its own fill would be (tiles of
// WG * S Philox blocks from the request's first block), and the tiles of all
// requests form one flat space.  Persistent workgroups take chunks of that
// space from an atomic counter; wave 0 finds the request owning a tile with
// a 64-way search over the requests' first tiles (one ballot per level) and
// the workgroup runs the fill's own tile code with that request's seed,
// range, parameters and output.  Outputs are therefore bit-identical to the
// same requests filled one by one.  Both distributions' tables are copied
// into LDS once per workgroup.  For the serving loop, the last workgroup to
// finish also advances the per-client counters (an order-free max of every
// request's end index).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

// With FULL the slow-path tables (X, f, alias) of both distributions are
// staged here too; otherwise only the fast-path tables are, and the slow
// paths (a percent or two of the outputs) read the rest from device memory.
// The lean layout saves 18 KB, which lifts the 128 x 8 kernel from 2 to 4
// waves per SIMD: the better choice when a batch keeps the device busy for
// many tiles, since the tables then stay in L2.  A small batch starts with
// cold tables, and there the staged copy answers the drain's dependent
// reads faster.
template <int WG, int S, bool FULL>
struct BatchLds {
  static constexpr uint32_t SL = FULL ? kLdsLayers : 1;
  double xs64[2][kLdsLayers];
  float xs32[2][kLdsLayers];
  double X[2][SL + 1];
  double f[2][SL + 1];
  uint64_t TA[2][SL];
  double2 stage[WG * S];
  uint64_t slowmap[S * 4 * (WG / 64)];  // enough for 4 outputs per block
  uint32_t prefix[S * 4 * (WG / 64) + 1];
  uint32_t chunk;
  uint32_t req;
};

// Last request r in [0, count) whose first tile is <= t (wave-wide call).
__device__ __forceinline__ uint32_t find_request(const BatchReq* reqs, uint32_t count, uint32_t t) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t lo = 0, hi = count;  // reqs[lo].tile_start <= t < reqs[hi].tile_start (hi = count: end)
  while (hi - lo > 1) {
    const uint32_t stride = (hi - lo + 63) / 64;
    const uint32_t idx = lo + lane * stride;
    const bool pred = idx < hi && reqs[idx].tile_start <= t;
    const uint64_t m = __builtin_amdgcn_ballot_w64(pred);
    const uint32_t c = 63u - (uint32_t)__clzll((long long)m);
    lo = lo + c * stride;
    const uint32_t nh = lo + stride;
    hi = nh < hi ? nh : hi;
  }
  return lo;
}

template <int WG, int S, bool FULL>
__device__ __forceinline__ void batch_body(const BatchArgs& ba, const BatchHeader* hdr) {
  __shared__ BatchLds<WG, S, FULL> sh;
  const uint32_t tid = threadIdx.x;
  for (uint32_t d = 0; d < 2; ++d) {
    const DevTable* tb = ba.tabs + d;
    for (uint32_t i = tid; i < kLdsLayers; i += WG) {
      sh.xs64[d][i] = tb->XS[i];
      sh.xs32[d][i] = tb->XS32[i];
    }
    if constexpr (FULL) {
      for (uint32_t i = tid; i < kLdsLayers; i += WG) {
        sh.TA[d][i] = tb->TA[i];
      }
      for (uint32_t i = tid; i <= kLdsLayers; i += WG) {
        sh.X[d][i] = tb->X[i];
        sh.f[d][i] = tb->f[i];
      }
    }
  }
  dev::TabView vexp = dev::global_view(ba.tabs);
  vexp.XS = sh.xs64[0];
  dev::TabView vnorm = dev::global_view(ba.tabs + 1);
  vnorm.XS = sh.xs64[1];
  if constexpr (FULL) {
    vexp.X = sh.X[0];
    vexp.f = sh.f[0];
    vexp.TA = sh.TA[0];
    vnorm.X = sh.X[1];
    vnorm.f = sh.f[1];
    vnorm.TA = sh.TA[1];
  }
  TileLds tl;
  tl.stage = sh.stage;
  tl.slowmap = sh.slowmap;
  tl.prefix = sh.prefix;
  tl.list = nullptr;  // the batch kernel searches the prefix sums
  tl.marks = nullptr;

  const uint32_t count = hdr->count;
  const uint32_t total = hdr->total_tiles;
  const uint32_t step = hdr->chunk;
  const BatchReq* reqs = reinterpret_cast<const BatchReq*>(hdr + 1);

  for (;;) {
    if (tid == 0) sh.chunk = atomicAdd(&ba.counters[0], 1u);
    __syncthreads();
    const uint64_t t0 = (uint64_t)sh.chunk * step;
    if (t0 >= total) break;
    const uint32_t t1 = (uint32_t)(t0 + step < total ? t0 + step : total);
    if (tid < 64) {
      const uint32_t r = find_request(reqs, count, (uint32_t)t0);
      if (tid == 0) sh.req = r;
    }
    __syncthreads();
    uint32_t r = __builtin_amdgcn_readfirstlane(sh.req);
    for (uint32_t t = (uint32_t)t0; t < t1; ++t) {
      while (r + 1 < count && reqs[r + 1].tile_start <= t) ++r;
      const BatchReq& q = reqs[r];
      FillArgs a;
      a.seed = q.seed;
      a.first = q.first;
      a.last = q.last;
      a.blk0 = q.blk0;
      a.blk_last = q.blk_last;
      a.out = q.out;
      a.scale = q.scale;
      a.shift = q.shift;
      a.tab = ba.tabs + q.dist;
      a.etab = ba.tabs;
      a.counters = nullptr;
      a.tiles = q.tiles;
      a.chunk = 1;
      a.aligned16 = q.aligned16;
      a.has_full = q.has_full;
      a.full_lo = q.full_lo;
      a.full_hi = q.full_hi;
      a.accel = 0;
      a.pad = 0;
      a.t_layer = nullptr;
      a.t_region = nullptr;
      a.t_words = nullptr;
      a.t_tests = nullptr;
      a.ttab = nullptr;
      a.tetab = nullptr;
      FillCtx c;
      c.ex = vexp;
      c.k0 = (uint32_t)q.seed;
      c.k1 = (uint32_t)(q.seed >> 32);
      c.scale = q.scale;
      c.shift = q.shift;
      const uint32_t lt = t - q.tile_start;
      const uint32_t kind = (q.dist & 1) * 2 + (q.dtype & 1);
      if (kind == 0) {
        c.own = vexp;
        c.fast = sh.xs64[0];
        fill_tile<kDistExp, kF64, WG, S, false>(a, c, tl, lt);
      } else if (kind == 1) {
        c.own = vexp;
        c.fast = sh.xs32[0];
        fill_tile<kDistExp, kF32, WG, S, false>(a, c, tl, lt);
      } else if (kind == 2) {
        c.own = vnorm;
        c.fast = sh.xs64[1];
        fill_tile<kDistNormal, kF64, WG, S, false>(a, c, tl, lt);
      } else {
        c.own = vnorm;
        c.fast = sh.xs32[1];
        fill_tile<kDistNormal, kF32, WG, S, false>(a, c, tl, lt);
      }
      // no barrier between tiles (see fill_tile): a lane's stores read only
      // the staging places it wrote itself, whatever request a tile is of
    }
  }
  if (tid == 0) sh.req = atomicAdd(&ba.counters[1], 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (sh.req) {  // the last workgroup: every other one has taken its final step
    if (tid == 0) {
      atomicExch(&ba.counters[0], 0u);
      atomicExch(&ba.counters[1], 0u);
    }
    if (ba.client_next != nullptr) {
      for (uint32_t i = tid; i < count; i += WG)
        atomicMax(reinterpret_cast<unsigned long long*>(&ba.client_next[reqs[i].seed - ba.seed_base]),
                  (unsigned long long)(reqs[i].last + 1));
    }
  }
}

template <int WG, int S, bool FULL>
__global__ void __launch_bounds__(WG) batch_kernel(BatchArgs ba) {
  batch_body<WG, S, FULL>(ba, ba.hdr);
}

// A small batch with its descriptors in the kernel arguments: read in
// place from the argument segment, no copy to device memory first.
template <int WG, int S, bool FULL>
__global__ void __launch_bounds__(WG) batch_kernel_inline(BatchArgs ba, BatchInline inl) {
  batch_body<WG, S, FULL>(ba, &inl.hdr);
}

template <class K>
int groups_of(K kernel, int wg, uint32_t* out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, uint32_t> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair((const void*)kernel, dev);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return 0;
  }
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, wg, 0);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  if (per_cu < 1) return (int)hipErrorInvalidConfiguration;
  cache[key] = (uint32_t)(per_cu * cus);
  *out = cache[key];
  return 0;
}

}  // namespace

#define ZIG_BATCH_SHAPES(X) X(64, 4) X(128, 4) X(128, 8) X(256, 2) X(256, 4) X(512, 2)

bool batch_shape_supported(uint32_t wg, uint32_t spl) {
#define ZIG_B(W, S_) \
  if (wg == W && spl == S_) return true;
  ZIG_BATCH_SHAPES(ZIG_B)
#undef ZIG_B
  return false;
}

int batch_groups(uint32_t wg, uint32_t spl, bool full, uint32_t* groups) {
#define ZIG_B(W, S_)                                                     \
  if (wg == W && spl == S_) {                                            \
    if (full) return groups_of(batch_kernel<W, S_, true>, W, groups);    \
    return groups_of(batch_kernel<W, S_, false>, W, groups);             \
  }
  ZIG_BATCH_SHAPES(ZIG_B)
#undef ZIG_B
  return (int)hipErrorInvalidConfiguration;
}

int launch_batch(uint32_t wg, uint32_t spl, bool full, uint32_t grid, const BatchArgs& a, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
#define ZIG_B(W, S_)                                                                     \
  if (wg == W && spl == S_) {                                                            \
    if (full)                                                                            \
      hipLaunchKernelGGL((batch_kernel<W, S_, true>), dim3(grid), dim3(W), 0, st, a);  \
    else                                                                                 \
      hipLaunchKernelGGL((batch_kernel<W, S_, false>), dim3(grid), dim3(W), 0, st, a); \
    return (int)hipGetLastError();                                                       \
  }
  ZIG_BATCH_SHAPES(ZIG_B)
#undef ZIG_B
  return (int)hipErrorInvalidConfiguration;
}

int launch_batch_inline(uint32_t wg, uint32_t spl, bool full, uint32_t grid, const BatchArgs& a,
                        const BatchInline& inl, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
#define ZIG_B(W, S_)                                                                                 \
  if (wg == W && spl == S_) {                                                                        \
    if (full)                                                                                        \
      hipLaunchKernelGGL((batch_kernel_inline<W, S_, true>), dim3(grid), dim3(W), 0, st, a, inl);  \
    else                                                                                             \
      hipLaunchKernelGGL((batch_kernel_inline<W, S_, false>), dim3(grid), dim3(W), 0, st, a, inl); \
    return (int)hipGetLastError();                                                                   \
  }
  ZIG_BATCH_SHAPES(ZIG_B)
#undef ZIG_B
  return (int)hipErrorInvalidConfiguration;
}

namespace {
__global__ void raise_counters_kernel(uint64_t* counters, const uint64_t* ends, uint32_t count) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < count && ends[c] != 0)
    atomicMax(reinterpret_cast<unsigned long long*>(&counters[c]), (unsigned long long)ends[c]);
}
}  // namespace

int launch_raise_counters(uint64_t* counters, const uint64_t* ends, uint32_t count, void* stream) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(raise_counters_kernel, dim3((count + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     counters, ends, count);
  return (int)hipGetLastError();
}

}  // namespace zig
