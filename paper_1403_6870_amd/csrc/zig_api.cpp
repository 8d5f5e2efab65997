// C ABI of the sampler library: argument checking, table registry and
// device upload, launch-shape choice, launches.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zig.h"
#include "zig_internal.hpp"
#include "zig_ring.hpp"
#include "zig_tune.hpp"

namespace zig {
namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

struct HostPair {
  HostTable t[2];
};

std::mutex g_mu;
std::map<uint32_t, std::unique_ptr<HostPair>> g_host;           // by i_max
std::map<std::pair<int, uint32_t>, DevTable*> g_dev;               // (device, i_max) -> 2 tables

bool valid_imax(uint32_t i_max) { return i_max >= 8 && i_max <= kMaxLayers && (i_max & (i_max - 1)) == 0; }

// host tables of both distributions; caller holds g_mu
int host_tables_locked(uint32_t i_max, HostPair** out) {
  auto it = g_host.find(i_max);
  if (it != g_host.end()) {
    *out = it->second.get();
    return ZIG_OK;
  }
  std::unique_ptr<HostPair> hp(new HostPair());
  for (uint32_t d = 0; d < 2; ++d) {
    std::string err = build_host_table(d, i_max, &hp->t[d]);
    if (!err.empty()) return fail(ZIG_ENOTABLES, "table construction: " + err);
  }
  *out = hp.get();
  g_host[i_max] = std::move(hp);
  return ZIG_OK;
}

void to_device_layout(const HostTable& h, DevTable* d) {
  std::memset(d, 0, sizeof(*d));
  d->dist = h.dist;
  d->i_max = h.i_max;
  d->b = h.b;
  d->L = h.L;
  d->K_eps = h.K_eps;
  d->K_cvx = h.K_cvx;
  d->K_ccv = h.K_ccv;
  d->X0 = h.X0;
  d->invX0 = h.invX0;
  for (uint32_t i = 0; i < h.i_max; ++i) {
    d->XS[i] = h.XS[i];
    d->XS32[i] = h.XS32[i];
    const uint64_t cap = 1ull << (64 - h.b);
    const uint64_t t = h.T[i] < cap ? h.T[i] : cap - 1;
    d->TA[i] = (t << h.b) | h.A[i];
  }
  for (uint32_t j = 0; j <= h.L; ++j) {
    d->X[j] = h.X[j];
    d->f[j] = h.f[j];
    d->W[j] = h.W[j];
    d->H[j] = h.H[j];
  }
  if (h.dist == kDistNormal) {
    for (uint32_t j = 0; j <= h.L; ++j) {
      d->SQlo[j] = h.SQlo[j];
      d->SQhi[j] = h.SQhi[j];
    }
    // the fast-path table past the layers holds +inf for the normal: a
    // slow output's placeholder is then +-inf and carries its sign to the
    // slow path (NaN when its magnitude bits are all zero)
    for (uint32_t i = h.L; i < h.i_max; ++i) {
      d->XS[i] = HUGE_VAL;
      d->XS32[i] = HUGE_VALF;
    }
  }
}

constexpr const char* kNotBuilt =
    "tables of this i_max are not built on this device: call zig_build_tables first";

// device copy for the current device; returns the pair [exp, normal].
// With build false nothing is built, allocated or copied: tables missing on
// the device are an error (ZIG_ESTATE).
int device_tables(uint32_t i_max, const DevTable** out, bool build = true) {
  if (!valid_imax(i_max)) return fail(ZIG_EINVAL, "i_max must be a power of two in [8, 1024]");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, i_max);
  auto it = g_dev.find(key);
  if (it != g_dev.end()) {
    *out = it->second;
    return ZIG_OK;
  }
  if (!build) return fail(ZIG_ESTATE, kNotBuilt);
  HostPair* hp = nullptr;
  int r = host_tables_locked(i_max, &hp);
  if (r != ZIG_OK) return r;
  DevTable host[2];
  to_device_layout(hp->t[0], &host[0]);
  to_device_layout(hp->t[1], &host[1]);
  DevTable* d = nullptr;
  e = hipMalloc(&d, sizeof(host));
  if (e != hipSuccess) return fail(ZIG_ENOMEM, std::string("hipMalloc(tables): ") + hipGetErrorString(e));
  e = hipMemcpy(d, host, sizeof(host), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(ZIG_EHIP, std::string("hipMemcpy(tables): ") + hipGetErrorString(e));
  }
  g_dev[key] = d;
  *out = d;
  return ZIG_OK;
}

// Traditional sampler tables (the comparison of Table 1), host and device,
// built on first use like the modified ones.
struct TradPair {
  HostTrad t[2];
};
std::map<uint32_t, std::unique_ptr<TradPair>> g_thost;  // by i_max
std::map<std::pair<int, uint32_t>, DevTrad*> g_tdev;     // (device, i_max) -> [exp, normal]

int host_trad_locked(uint32_t i_max, TradPair** out) {
  auto it = g_thost.find(i_max);
  if (it != g_thost.end()) {
    *out = it->second.get();
    return ZIG_OK;
  }
  std::unique_ptr<TradPair> tp(new TradPair());
  for (uint32_t d = 0; d < 2; ++d) {
    std::string err = build_host_trad(d, i_max, &tp->t[d]);
    if (!err.empty()) return fail(ZIG_ENOTABLES, "traditional tables: " + err);
  }
  *out = tp.get();
  g_thost[i_max] = std::move(tp);
  return ZIG_OK;
}

int device_trad(uint32_t i_max, const DevTrad** out, bool build = true) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, i_max);
  auto it = g_tdev.find(key);
  if (it != g_tdev.end()) {
    *out = it->second;
    return ZIG_OK;
  }
  if (!build)
    return fail(ZIG_ESTATE,
                "traditional tables of this i_max are not on this device: run one uncaptured traditional fill first");
  TradPair* tp = nullptr;
  int r = host_trad_locked(i_max, &tp);
  if (r != ZIG_OK) return r;
  DevTrad host[2];
  std::memset(host, 0, sizeof(host));
  for (uint32_t d = 0; d < 2; ++d) {
    const HostTrad& h = tp->t[d];
    host[d].dist = h.dist;
    host[d].n = h.n;
    host[d].b = h.b;
    host[d].r = h.r;
    host[d].invr = h.invr;
    for (uint32_t i = 0; i < h.n; ++i) {
      host[d].WS[i] = h.WS[i];
      host[d].KQ[i] = h.KQ[i];
      host[d].f[i] = h.f[i];
    }
  }
  DevTrad* d = nullptr;
  e = hipMalloc(&d, sizeof(host));
  if (e != hipSuccess) return fail(ZIG_ENOMEM, std::string("hipMalloc(tables): ") + hipGetErrorString(e));
  e = hipMemcpy(d, host, sizeof(host), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(ZIG_EHIP, std::string("hipMemcpy(tables): ") + hipGetErrorString(e));
  }
  g_tdev[key] = d;
  *out = d;
  return ZIG_OK;
}

// HIP's streams and events for the scratch-slot rings (zig_ring.hpp).
struct HipRingOps {
  using Event = hipEvent_t;
  using Stream = void*;
  static int wait(void* s, hipEvent_t e) { return (int)hipStreamWaitEvent(static_cast<hipStream_t>(s), e, 0); }
  static int record(hipEvent_t e, void* s) { return (int)hipEventRecord(e, static_cast<hipStream_t>(s)); }
};
using HipSlotRing = SlotRing<HipRingOps>;

// Releases what a ring holds (a ring whose set-up failed part way).
void ring_release(HipSlotRing* r) {
  for (hipEvent_t e : r->ev)
    if (e) (void)hipEventDestroy(e);
  r->ev.clear();
  if (r->base) (void)hipFree(r->base);
  r->base = nullptr;
}

int ring_init(HipSlotRing* r, uint32_t slots, size_t slot_bytes) {
  hipError_t e = hipMalloc(&r->base, slots * slot_bytes);
  if (e != hipSuccess) {
    r->base = nullptr;
    return fail(ZIG_ENOMEM, std::string("hipMalloc(launch scratch): ") + hipGetErrorString(e));
  }
  e = hipMemset(r->base, 0, slots * slot_bytes);
  if (e != hipSuccess) {
    ring_release(r);
    return fail(ZIG_EHIP, std::string("hipMemset(launch scratch): ") + hipGetErrorString(e));
  }
  r->ev.assign(slots, nullptr);
  for (uint32_t k = 0; k < slots; ++k) {
    e = hipEventCreateWithFlags(&r->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      ring_release(r);
      return fail(ZIG_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  r->recorded.assign(slots, 0);
  r->slot_bytes = slot_bytes;
  r->slots = slots;
  return ZIG_OK;
}

constexpr uint32_t kCounterSlots = 64;
constexpr uint32_t kMomentSlots = 4;

struct DeviceScratch {
  HipSlotRing counters;  // 2 x uint32 per slot
  HipSlotRing moments;   // kMomMaxGroups x 5 doubles per slot
  int cus = 0;
};
std::mutex g_cmu;
std::map<int, std::unique_ptr<DeviceScratch>> g_scratch;

int device_scratch(DeviceScratch** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_cmu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *out = it->second.get();
    return ZIG_OK;
  }
  std::unique_ptr<DeviceScratch> d(new DeviceScratch());
  e = hipDeviceGetAttribute(&d->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
  int r = ring_init(&d->counters, kCounterSlots, 2 * sizeof(uint32_t));
  if (r != ZIG_OK) return r;
  r = ring_init(&d->moments, kMomentSlots, (size_t)kMomMaxGroups * 5 * sizeof(double));
  if (r != ZIG_OK) {
    ring_release(&d->counters);
    return r;
  }
  *out = d.get();
  g_scratch[dev] = std::move(d);
  return ZIG_OK;
}

// Whether `stream` is being captured into a graph (the legacy null stream
// cannot be).
int stream_capturing(void* stream, bool* capturing) {
  *capturing = false;
  if (stream == nullptr) return ZIG_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cs);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("hipStreamIsCapturing: ") + hipGetErrorString(e));
  *capturing = cs != hipStreamCaptureStatusNone;
  return ZIG_OK;
}

int check_params(uint32_t dist, double p0, double p1, double* scale, double* shift) {
  if (dist == kDistExp) {
    if (!std::isfinite(p0) || !(p0 > 0.0)) return fail(ZIG_EINVAL, "lambda must be finite and > 0");
    const double s = 1.0 / p0;
    if (!std::isfinite(s) || !(s > 0.0)) return fail(ZIG_EINVAL, "1/lambda must be finite and > 0");
    *scale = s;
    *shift = 0.0;
    return ZIG_OK;
  }
  if (dist == kDistNormal) {
    if (!std::isfinite(p0)) return fail(ZIG_EINVAL, "mu must be finite");
    if (!std::isfinite(p1) || !(p1 > 0.0)) return fail(ZIG_EINVAL, "sigma must be finite and > 0");
    *scale = p1;
    *shift = p0;
    return ZIG_OK;
  }
  return fail(ZIG_EINVAL, "unknown distribution");
}

int fill_impl(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double p0, double p1,
              void* out, void* stream, const zig_launch* launch, bool trace, uint32_t* t_layer, int32_t* t_region,
              uint32_t* t_words, uint32_t* t_tests, const Shape* forced, bool own = false,
              uint32_t* own_counters = nullptr) {
  g_error.clear();
  if (dist != kDistExp && dist != kDistNormal) return fail(ZIG_EINVAL, "unknown distribution");
  if (dtype != kF64 && dtype != kF32) return fail(ZIG_EINVAL, "unknown dtype");
  double scale = 0.0, shift = 0.0;
  int r = check_params(dist, p0, p1, &scale, &shift);
  if (r != ZIG_OK) return r;
  zig_launch cfg = {0, 0, 0, 0};
  if (launch) cfg = *launch;
  const uint32_t i_max = cfg.i_max ? cfg.i_max : 256;
  if (!valid_imax(i_max)) return fail(ZIG_EINVAL, "i_max must be a power of two in [8, 1024]");
  if (cfg.flags & ~(ZIG_LAUNCH_NORMAL_ACCEL | ZIG_LAUNCH_TRADITIONAL))
    return fail(ZIG_EINVAL, "unknown launch flags");
  const bool trad = (cfg.flags & ZIG_LAUNCH_TRADITIONAL) != 0;
  if (trad) {
    if (cfg.flags & ZIG_LAUNCH_NORMAL_ACCEL)
      return fail(ZIG_EINVAL, "ZIG_LAUNCH_TRADITIONAL does not combine with ZIG_LAUNCH_NORMAL_ACCEL");
    if (dtype != kF64) return fail(ZIG_EINVAL, "the traditional sampler is FP64 only");
    if (i_max > kLdsLayers) return fail(ZIG_EINVAL, "the traditional sampler takes i_max up to 256");
    if (trace) return fail(ZIG_EINVAL, "the traditional sampler has no trace");
  }
  const bool wide = i_max > kLdsLayers;
  if (wide && (cfg.flags & ZIG_LAUNCH_NORMAL_ACCEL))
    return fail(ZIG_EINVAL, "the accelerated normal variant takes i_max up to 256");
  if (n == 0) return ZIG_OK;
  if (out == nullptr) return fail(ZIG_EINVAL, "out is null");
  const uint64_t esize = dtype == kF64 ? 8 : 4;
  if (((uintptr_t)out) % esize != 0) return fail(ZIG_EINVAL, "out is not aligned to its element size");
  if (n - 1 > UINT64_MAX - first) return fail(ZIG_EINVAL, "first_index + n exceeds 2^64");

  Shape sh = forced ? *forced : tuned_shape(dist, dtype, n);
  if (cfg.wg) sh.wg = cfg.wg;
  if (cfg.spl) sh.spl = cfg.spl;
  if (cfg.wg || cfg.spl) sh.chunk = 16384 / (sh.wg * sh.spl) ? 16384 / (sh.wg * sh.spl) : 1;
  if (trace) {
    if (!((sh.wg == 64 && sh.spl == 1) || (sh.wg == 256 && (sh.spl == 2 || sh.spl == 4)))) {
      sh.wg = 256;
      sh.spl = 2;
    }
  }
  if (!shape_supported(sh.wg, sh.spl)) return fail(ZIG_EINVAL, "unsupported workgroup size / samples per lane");

  // A fill enqueued on a stream being captured allocates and copies
  // nothing (either would break or end the capture): its tables must be on
  // the device already, and its schedule needs no scratch.
  bool capturing = false;
  r = stream_capturing(stream, &capturing);
  if (r != ZIG_OK) return r;
  const DevTable* tabs = nullptr;
  r = device_tables(i_max, &tabs, !capturing);
  if (r != ZIG_OK) return r;
  const DevTrad* ttabs = nullptr;
  if (trad) {
    r = device_trad(i_max, &ttabs, !capturing);
    if (r != ZIG_OK) return r;
  }

  const uint64_t per_block = dtype == kF64 ? 2 : 4;
  const uint64_t last = first + (n - 1);
  FillArgs a;
  std::memset(&a, 0, sizeof(a));
  a.seed = seed;
  a.first = first;
  a.last = last;
  a.blk_last = last / per_block;
  a.out = out;
  a.scale = scale;
  a.shift = shift;
  a.tab = tabs + dist;
  a.etab = tabs + kDistExp;
  a.aligned16 = ((((uintptr_t)out) - first * esize) & 15u) == 0 ? 1u : 0u;
  a.accel = (dist == kDistNormal && (cfg.flags & ZIG_LAUNCH_NORMAL_ACCEL)) ? 1u : 0u;
  a.t_layer = t_layer;
  a.t_region = t_region;
  a.t_words = t_words;
  a.t_tests = t_tests;
  if (trad) {
    a.ttab = ttabs + dist;
    a.tetab = ttabs + kDistExp;
  }

  // blocks whose outputs all lie in [first, last]
  a.full_lo = first / per_block + (first % per_block != 0);
  if (last % per_block == per_block - 1) {
    a.full_hi = last / per_block;
    a.has_full = a.full_lo <= a.full_hi;
  } else {
    a.full_hi = last / per_block == 0 ? 0 : last / per_block - 1;
    a.has_full = last / per_block > 0 && a.full_lo <= a.full_hi;
  }

  const uint64_t blk0 = first / per_block;
  const uint64_t nblk = a.blk_last - blk0 + 1;
  const uint64_t tile = (uint64_t)sh.wg * sh.spl;
  const uint64_t tiles = nblk / tile + (nblk % tile != 0);
  // Tile schedule.  A fill of at most kStaticTilesPerCU tiles per compute
  // unit gives workgroup w the tiles w, w + G, ... (no counters, no set-up
  // cost: 2^20 FP64 outputs in 9.5 us against 15 us with counters).  A
  // larger one lets workgroups take chunks of tiles from an atomic counter,
  // which balances them (2^30 FP64 normal: 2.05 ms against 2.4 ms
  // statically).  A stream being captured always gets the static schedule,
  // so a graph holds no scratch and may be replayed on any stream.
  DeviceScratch* ds = nullptr;
  if (!capturing) {
    r = device_scratch(&ds);
    if (r != ZIG_OK) return r;
  }
  // a caller with its own counters (own) uses them, or the fixed schedule
  // when it has none
  const bool dynamic = !capturing && (!own || own_counters != nullptr) &&
                       tiles > (uint64_t)kStaticTilesPerCU * (uint64_t)ds->cus;
  const uint64_t chunk = 1ull << 30;  // tiles per launch: the counter stays far from 2^32
  for (uint64_t start = 0; start < tiles; start += chunk) {
    a.blk0 = blk0 + start * tile;
    a.tiles = (uint32_t)((tiles - start < chunk) ? tiles - start : chunk);
    a.chunk = sh.chunk;
    auto go = [&](void* counters) {
      FillArgs b = a;
      b.counters = static_cast<uint32_t*>(counters);
      return trad   ? launch_trad(dist, sh.wg, sh.spl, b, stream)
             : wide ? launch_fill_wide(dist, dtype, sh.wg, sh.spl, trace, b, stream)
                    : launch_fill(dist, dtype, sh.wg, sh.spl, trace, b, stream);
    };
    const int e = !dynamic ? go(nullptr) : own ? go(own_counters) : ring_launch(&ds->counters, stream, go);
    if (e != 0)
      return fail(ZIG_EHIP, std::string("fill launch: ") + hipGetErrorString(static_cast<hipError_t>(e)));
  }
  return ZIG_OK;
}

// Checked arguments of a moments call.
struct MomentsCall {
  double scale = 0.0, shift = 0.0;
  uint32_t i_max = 256, spl = 32;
  bool accel = false;
};

int moments_args(uint32_t dist, uint32_t dtype, uint64_t first_index, uint64_t n, double p0, double p1,
                 const double* sums, const zig_launch* launch, MomentsCall* mc) {
  if (dist > 1) return fail(ZIG_EINVAL, "unknown distribution");
  if (dtype > 1) return fail(ZIG_EINVAL, "unknown dtype");
  int r = check_params(dist, p0, p1, &mc->scale, &mc->shift);
  if (r != ZIG_OK) return r;
  zig_launch cfg = {0, 0, 0, 0};
  if (launch) cfg = *launch;
  mc->i_max = cfg.i_max ? cfg.i_max : 256;
  if (!valid_imax(mc->i_max)) return fail(ZIG_EINVAL, "i_max must be a power of two in [8, 1024]");
  if (cfg.flags & ZIG_LAUNCH_TRADITIONAL) return fail(ZIG_EINVAL, "the moments kernel runs the modified sampler only");
  if (mc->i_max > kLdsLayers) return fail(ZIG_EINVAL, "the moments kernel takes i_max up to 256");
  if (cfg.flags & ~ZIG_LAUNCH_NORMAL_ACCEL) return fail(ZIG_EINVAL, "unknown launch flags");
  mc->spl = cfg.spl ? cfg.spl : 32;
  if ((cfg.wg && cfg.wg != 256) || !moments_spl_supported(mc->spl))
    return fail(ZIG_EINVAL, "the moments kernel runs 256 lanes x 16, 32 or 64 blocks");
  mc->accel = dist == kDistNormal && (cfg.flags & ZIG_LAUNCH_NORMAL_ACCEL) != 0;
  if (sums == nullptr) return fail(ZIG_EINVAL, "sums is null");
  if (((uintptr_t)sums) % 8 != 0) return fail(ZIG_EINVAL, "sums is not 8-byte aligned");
  if (n > 0 && n - 1 > UINT64_MAX - first_index) return fail(ZIG_EINVAL, "first_index + n exceeds 2^64");
  return ZIG_OK;
}

int moments_zero(double* sums, void* stream) {
  const int e = launch_moments_zero(sums, stream);
  if (e != 0) return fail(ZIG_EHIP, std::string("moments launch: ") + hipGetErrorString((hipError_t)e));
  return ZIG_OK;
}

// Argument block and launch of the moments kernels (shared by the
// entry points with library-owned and with static scratch).
int moments_launch(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double scale,
                   double shift, const DevTable* tabs, uint32_t spl, bool accel, double* partial,
                   uint32_t max_groups, double* sums, void* stream) {
  const uint64_t per_block = dtype == kF64 ? 2 : 4;
  const uint64_t last = first_index + (n - 1);
  FillArgs a;
  std::memset(&a, 0, sizeof(a));
  a.seed = seed;
  a.first = first_index;
  a.last = last;
  a.blk_last = last / per_block;
  a.scale = scale;
  a.shift = shift;
  a.tab = tabs + dist;
  a.etab = tabs + kDistExp;
  a.accel = (dist == kDistNormal && accel) ? 1u : 0u;
  a.full_lo = first_index / per_block + (first_index % per_block != 0);
  if (last % per_block == per_block - 1) {
    a.full_hi = last / per_block;
    a.has_full = a.full_lo <= a.full_hi;
  } else {
    a.full_hi = last / per_block == 0 ? 0 : last / per_block - 1;
    a.has_full = last / per_block > 0 && a.full_lo <= a.full_hi;
  }
  a.blk0 = first_index / per_block;
  const uint64_t nblk = a.blk_last - a.blk0 + 1;
  const uint64_t tile = 256ull * spl;
  const uint64_t tiles = nblk / tile + (nblk % tile != 0);
  const int e = launch_moments(dist, dtype, spl, a, tiles, partial, max_groups, sums, stream);
  if (e != 0) return fail(ZIG_EHIP, std::string("moments launch: ") + hipGetErrorString((hipError_t)e));
  return ZIG_OK;
}

}  // namespace

int device_tables_for(uint32_t i_max, const DevTable** out) { return device_tables(i_max, out); }
int stream_capturing_for(void* stream, bool* capturing) { return stream_capturing(stream, capturing); }
int params_for(uint32_t dist, double p0, double p1, double* scale, double* shift) {
  return check_params(dist, p0, p1, scale, shift);
}
int fill_shaped(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double p0, double p1,
                void* out, void* stream, const Shape& shape) {
  return fill_impl(dist, dtype, seed, first, n, p0, p1, out, stream, nullptr, false, nullptr, nullptr, nullptr,
                   nullptr, &shape);
}
int fill_own_counters(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double p0,
                      double p1, void* out, void* stream, uint32_t* counters) {
  return fill_impl(dist, dtype, seed, first, n, p0, p1, out, stream, nullptr, false, nullptr, nullptr, nullptr,
                   nullptr, nullptr, true, counters);
}
void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

}  // namespace zig

extern "C" {

int zig_build_tables(uint32_t i_max) {
  zig::g_error.clear();
  const zig::DevTable* t = nullptr;
  return zig::device_tables(i_max, &t);
}

int zig_get_tables(uint32_t dist, uint32_t i_max, zig_table_view* out) {
  zig::g_error.clear();
  if (out == nullptr) return zig::fail(ZIG_EINVAL, "out is null");
  if (dist > 1) return zig::fail(ZIG_EINVAL, "unknown distribution");
  if (!zig::valid_imax(i_max)) return zig::fail(ZIG_EINVAL, "i_max must be a power of two in [8, 1024]");
  std::lock_guard<std::mutex> lk(zig::g_mu);
  zig::HostPair* hp = nullptr;
  int r = zig::host_tables_locked(i_max, &hp);
  if (r != ZIG_OK) return r;
  const zig::HostTable& t = hp->t[dist];
  out->dist = t.dist;
  out->i_max = t.i_max;
  out->b = t.b;
  out->L = t.L;
  out->X = t.X.data();
  out->f = t.f.data();
  out->XS = t.XS.data();
  out->XS32 = t.XS32.data();
  out->W = t.W.data();
  out->H = t.H.data();
  out->q = t.q.data();
  out->T = t.T.data();
  out->alias = t.A.data();
  out->eps = t.eps;
  out->K_eps = t.K_eps;
  out->X0 = t.X0;
  out->invX0 = t.invX0;
  out->eps_cvx = t.eps_cvx;
  out->del_ccv = t.del_ccv;
  out->K_cvx = t.K_cvx;
  out->K_ccv = t.K_ccv;
  out->sq_lo = t.SQlo.empty() ? nullptr : t.SQlo.data();
  out->sq_hi = t.SQhi.empty() ? nullptr : t.SQhi.data();
  return ZIG_OK;
}

int zig_get_trad_tables(uint32_t dist, uint32_t i_max, zig_trad_view* out) {
  zig::g_error.clear();
  if (out == nullptr) return zig::fail(ZIG_EINVAL, "out is null");
  if (dist > 1) return zig::fail(ZIG_EINVAL, "unknown distribution");
  if (!zig::valid_imax(i_max) || i_max > zig::kLdsLayers)
    return zig::fail(ZIG_EINVAL, "the traditional sampler takes i_max a power of two in [8, 256]");
  std::lock_guard<std::mutex> lk(zig::g_mu);
  zig::TradPair* tp = nullptr;
  int r = zig::host_trad_locked(i_max, &tp);
  if (r != ZIG_OK) return r;
  const zig::HostTrad& t = tp->t[dist];
  out->dist = t.dist;
  out->n = t.n;
  out->b = t.b;
  out->pad = 0;
  out->X = t.X.data();
  out->f = t.f.data();
  out->W = t.W.data();
  out->WS = t.WS.data();
  out->k = t.k.data();
  out->KQ = t.KQ.data();
  out->r = t.r;
  out->v = t.v;
  out->invr = t.invr;
  return ZIG_OK;
}

int zig_fill(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0, double p1,
             void* out, void* stream, const zig_launch* launch) {
  return zig::fill_impl(dist, dtype, seed, first_index, n, p0, p1, out, stream, launch, false, nullptr, nullptr,
                        nullptr, nullptr, nullptr);
}

int zig_fill_exp(uint64_t seed, uint64_t first_index, uint64_t n, uint32_t dtype, double lambda, void* out,
                 void* stream) {
  return zig::fill_impl(ZIG_EXP, dtype, seed, first_index, n, lambda, 0.0, out, stream, nullptr, false, nullptr,
                        nullptr, nullptr, nullptr, nullptr);
}

int zig_fill_normal(uint64_t seed, uint64_t first_index, uint64_t n, uint32_t dtype, double mu, double sigma,
                    void* out, void* stream) {
  return zig::fill_impl(ZIG_NORMAL, dtype, seed, first_index, n, mu, sigma, out, stream, nullptr, false, nullptr,
                        nullptr, nullptr, nullptr, nullptr);
}

int zig_fill_trace(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0,
                   double p1, void* out, uint32_t* layer, int32_t* region, uint32_t* words, uint32_t* tests,
                   void* stream, const zig_launch* launch) {
  return zig::fill_impl(dist, dtype, seed, first_index, n, p0, p1, out, stream, launch, true, layer, region, words,
                        tests, nullptr);
}

int zig_moments(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0, double p1,
                double* sums, void* stream, const zig_launch* launch) {
  zig::g_error.clear();
  zig::MomentsCall mc;
  int r = zig::moments_args(dist, dtype, first_index, n, p0, p1, sums, launch, &mc);
  if (r != ZIG_OK) return r;
  bool capturing = false;
  r = zig::stream_capturing(stream, &capturing);
  if (r != ZIG_OK) return r;
  if (capturing)
    return zig::fail(ZIG_EINVAL, "zig_moments cannot be captured into a graph: its scratch slot would be fixed");
  if (n == 0) return zig::moments_zero(sums, stream);
  const zig::DevTable* tabs = nullptr;
  r = zig::device_tables(mc.i_max, &tabs);
  if (r != ZIG_OK) return r;
  zig::DeviceScratch* ds = nullptr;
  r = zig::device_scratch(&ds);
  if (r != ZIG_OK) return r;
  int rr = ZIG_OK;
  const int e = zig::ring_launch(&ds->moments, stream, [&](void* partial) {
    rr = zig::moments_launch(dist, dtype, seed, first_index, n, mc.scale, mc.shift, tabs, mc.spl, mc.accel,
                             static_cast<double*>(partial), zig::kMomMaxGroups, sums, stream);
    return rr == ZIG_OK ? 0 : (int)hipErrorLaunchFailure;
  });
  if (rr != ZIG_OK) return rr;
  if (e != 0) return zig::fail(ZIG_EHIP, std::string("moments launch: ") + hipGetErrorString((hipError_t)e));
  return ZIG_OK;
}

int zig_moments_noalloc(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0,
                        double p1, double* sums, void* stream, const zig_launch* launch) {
  zig::g_error.clear();
  zig::MomentsCall mc;
  int r = zig::moments_args(dist, dtype, first_index, n, p0, p1, sums, launch, &mc);
  if (r != ZIG_OK) return r;
  if (n == 0) return zig::moments_zero(sums, stream);
  const zig::DevTable* tabs = nullptr;
  r = zig::device_tables(mc.i_max, &tabs, false);
  if (r != ZIG_OK) return r;
  double* partial = nullptr;
  const int e = zig::moments_static_scratch(&partial);
  if (e != 0)
    return zig::fail(ZIG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString((hipError_t)e));
  return zig::moments_launch(dist, dtype, seed, first_index, n, mc.scale, mc.shift, tabs, mc.spl, mc.accel, partial,
                             zig::kMomMaxGroups, sums, stream);
}

const char* zig_last_error(void) { return zig::g_error.c_str(); }

const char* zig_version(void) { return "zigrand 0.1 gfx950"; }

}  // extern "C"
