// Host side of zig_fill_batch: request checking, the flat tile space, the
// pinned descriptor ring and the hipGraph cache.
//
// A batch call writes its request descriptors into one of a ring of pinned
// host slots and replays a graph of (host-to-device copy of the
// descriptors, persistent batch kernel) captured for that slot and for the
// power-of-two bucket of the request count; the graph is launched on the
// caller's stream and an event marks when the slot may be rewritten.  Each
// slot owns its device buffer and tile counters, so graphs launched on
// different streams never share state.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zig.h"
#include "zig_internal.hpp"
#include "zig_tune.hpp"

namespace zig {
namespace {

constexpr int kSlots = 4;
constexpr uint32_t kMaxBatch = 1u << 20;

struct Slot {
  void* host = nullptr;       // pinned: header + requests
  void* dev = nullptr;        // device copy
  uint32_t* counters = nullptr;
  uint32_t cap = 0;           // requests the buffers hold
  hipEvent_t done = nullptr;  // last graph launch that read `host`
  bool used = false;
  std::map<std::tuple<uint32_t, uint32_t, uint32_t, bool>, hipGraphExec_t> graphs;  // (bucket, wg, spl, full)
};

struct DeviceBatch {
  std::mutex mu;
  Slot slots[kSlots];
  int next = 0;
  hipStream_t capture = nullptr;
};

std::mutex g_mu;
std::map<int, std::unique_ptr<DeviceBatch>> g_dev;

int fail(int code, const std::string& m) {
  set_error(m);
  return code;
}

int hip_fail(const char* what, hipError_t e) {
  return fail(ZIG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void free_slot(Slot& s) {
  for (auto& kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
  s.graphs.clear();
  if (s.host) (void)hipHostFree(s.host);
  if (s.dev) (void)hipFree(s.dev);
  s.host = s.dev = nullptr;
  s.cap = 0;
}

int ensure_capacity(Slot& s, uint32_t count) {
  if (s.cap >= count && s.host) return ZIG_OK;
  uint32_t cap = 64;
  while (cap < count) cap <<= 1;
  free_slot(s);
  const size_t bytes = sizeof(BatchHeader) + (size_t)cap * sizeof(BatchReq);
  hipError_t e = hipHostMalloc(&s.host, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return fail(ZIG_ENOMEM, std::string("hipHostMalloc(batch): ") + hipGetErrorString(e));
  e = hipMalloc(&s.dev, bytes);
  if (e != hipSuccess) return fail(ZIG_ENOMEM, std::string("hipMalloc(batch): ") + hipGetErrorString(e));
  if (!s.counters) {
    e = hipMalloc(&s.counters, 2 * sizeof(uint32_t));
    if (e != hipSuccess) return fail(ZIG_ENOMEM, std::string("hipMalloc(counters): ") + hipGetErrorString(e));
    e = hipMemset(s.counters, 0, 2 * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail("hipMemset(counters)", e);
  }
  if (!s.done) {
    e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail("hipEventCreate", e);
  }
  s.cap = cap;
  return ZIG_OK;
}

// Checks one request and fills its descriptor (tile fields are set by the
// caller, which knows the tile size).
int describe(const zig_request& r, BatchReq* d, uint32_t index) {
  if (r.dist > 1) return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": unknown distribution");
  if (r.dtype > 1) return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": unknown dtype");
  double scale = 0.0, shift = 0.0;
  if (params_for(r.dist, r.p0, r.p1, &scale, &shift) != ZIG_OK)
    return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": " + zig_last_error());
  if (r.n == 0) return ZIG_OK;
  if (r.out == nullptr) return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": out is null");
  const uint64_t esize = r.dtype == ZIG_F64 ? 8 : 4;
  if (((uintptr_t)r.out) % esize != 0)
    return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": out is not aligned to its element size");
  if (r.n - 1 > UINT64_MAX - r.first_index)
    return fail(ZIG_EINVAL, "request " + std::to_string(index) + ": first_index + n exceeds 2^64");
  make_descriptor(r.dist, r.dtype, r.seed, r.first_index, r.n, scale, shift, r.out, d);
  return ZIG_OK;
}

}  // namespace

void make_descriptor(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double scale,
                     double shift, void* out, BatchReq* d) {
  // outputs per Philox block: 2 (FP64) or 4 (FP32), as a shift and a mask
  const uint32_t sh = dtype == ZIG_F64 ? 1 : 2;
  const uint64_t mask = (1ull << sh) - 1;
  const uint64_t esize = dtype == ZIG_F64 ? 8 : 4;
  std::memset(d, 0, sizeof(*d));
  d->seed = seed;
  d->first = first;
  d->last = first + (n - 1);
  d->blk0 = d->first >> sh;
  d->blk_last = d->last >> sh;
  d->full_lo = (d->first >> sh) + ((d->first & mask) != 0);
  if ((d->last & mask) == mask) {
    d->full_hi = d->last >> sh;
    d->has_full = d->full_lo <= d->full_hi;
  } else {
    d->full_hi = (d->last >> sh) == 0 ? 0 : (d->last >> sh) - 1;
    d->has_full = (d->last >> sh) > 0 && d->full_lo <= d->full_hi;
  }
  d->out = out;
  d->scale = scale;
  d->shift = shift;
  d->dist = dist;
  d->dtype = dtype;
  d->aligned16 = ((((uintptr_t)out) - d->first * esize) & 15u) == 0 ? 1u : 0u;
}

// About 8K blocks per counter step, and every resident workgroup gets a few
// steps.  It travels in the header, so one graph serves every batch of a
// size bucket; workgroups with no step to take leave at once.
uint32_t batch_chunk(uint64_t total_tiles, uint32_t tile_blocks, uint32_t groups) {
  uint64_t chunk = 8192 / tile_blocks;
  if (chunk < 1) chunk = 1;
  const uint64_t cap_chunk = total_tiles / (2ull * groups);
  if (chunk > cap_chunk) chunk = cap_chunk < 1 ? 1 : cap_chunk;
  return (uint32_t)chunk;
}

// Fewer than four tiles per resident workgroup of the lean kernel: the
// batch is over before its tables would warm in L2, so the kernel that
// stages them in LDS is the faster one.
bool batch_full(uint64_t total_tiles, uint32_t lean_groups) { return total_tiles < 4ull * lean_groups; }

int fill_batch_impl(const zig_request* reqs, uint32_t count, void* stream, const zig_batch_opts* opts) {
  clear_error();
  if (count > 0 && reqs == nullptr) return fail(ZIG_EINVAL, "reqs is null");
  if (count > kMaxBatch) return fail(ZIG_EINVAL, "more than 2^20 requests in one batch");
  uint32_t wg = 0, spl = 0, flags = 0;
  tuned_batch_shape(&wg, &spl);
  if (opts) {
    if (opts->wg) wg = opts->wg;
    if (opts->spl) spl = opts->spl;
    flags = opts->flags;
  }
  if (!batch_shape_supported(wg, spl)) return fail(ZIG_EINVAL, "unsupported batch workgroup size / blocks per lane");
  if (flags & ~ZIG_BATCH_NO_GRAPH) return fail(ZIG_EINVAL, "unknown batch flags");
  const uint64_t tile_blocks = (uint64_t)wg * spl;
  // tiles of a request: a shift when the tile is a power of two blocks
  uint32_t tile_shift = 0;
  while ((1ull << tile_shift) < tile_blocks) ++tile_shift;
  const bool pow2 = (1ull << tile_shift) == tile_blocks;

  // A graph captured from here would hold one descriptor slot and its
  // counters, which later batches reuse while the graph may replay.
  bool capturing = false;
  int r = stream_capturing_for(stream, &capturing);
  if (r != ZIG_OK) return r;
  if (capturing)
    return fail(ZIG_EINVAL, "a batch cannot be captured into a graph: its descriptor slot would be fixed in it");

  // Validation and descriptors in one pass, written straight into the slot's
  // pinned buffer (or, for a few requests, the kernel-argument block); a
  // request that fails validation leaves the slot unlaunched and unused.
  const DevTable* tabs = nullptr;
  r = device_tables_for(256, &tabs);
  if (r != ZIG_OK) return r;
  uint32_t groups = 0;
  hipError_t e = (hipError_t)batch_groups(wg, spl, false, &groups);
  if (e != hipSuccess) return hip_fail("batch occupancy", e);

  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail("hipGetDevice", e);
  DeviceBatch* db;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& p = g_dev[dev];
    if (!p) p.reset(new DeviceBatch());
    db = p.get();
  }
  std::lock_guard<std::mutex> lk(db->mu);
  Slot& s = db->slots[db->next];
  if (s.used) {
    e = hipEventSynchronize(s.done);
    if (e != hipSuccess) return hip_fail("hipEventSynchronize(batch slot)", e);
  }
  r = ensure_capacity(s, count);
  if (r != ZIG_OK) return r;
  const bool inline_desc = count <= kInlineReqs;
  BatchInline inl;
  BatchHeader* h = inline_desc ? &inl.hdr : static_cast<BatchHeader*>(s.host);
  BatchReq* q = reinterpret_cast<BatchReq*>(h + 1);
  uint32_t m = 0;
  uint64_t total = 0;
  for (uint32_t i = 0; i < count; ++i) {
    r = describe(reqs[i], &q[m], i);
    if (r != ZIG_OK) return r;
    if (reqs[i].n == 0) continue;
    BatchReq& d = q[m];
    const uint64_t blocks = d.blk_last - d.blk0 + 1;
    const uint64_t t = pow2 ? (blocks + tile_blocks - 1) >> tile_shift : (blocks + tile_blocks - 1) / tile_blocks;
    if (total + t >= (1ull << 31)) return fail(ZIG_EINVAL, "batch too large (more than 2^31 tiles)");
    d.tiles = (uint32_t)t;
    d.tile_start = (uint32_t)total;
    total += t;
    ++m;
  }
  if (m == 0) return ZIG_OK;
  db->next = (db->next + 1) % kSlots;

  const bool full = batch_full(total, groups);
  if (full) {
    e = (hipError_t)batch_groups(wg, spl, true, &groups);
    if (e != hipSuccess) return hip_fail("batch occupancy", e);
  }
  const uint32_t chunk = batch_chunk(total, tile_blocks, groups);
  const uint32_t grid = groups;
  h->count = m;
  h->total_tiles = (uint32_t)total;
  h->chunk = chunk;
  h->pad = 0;

  BatchArgs ba;
  ba.hdr = static_cast<const BatchHeader*>(s.dev);
  ba.tabs = tabs;
  ba.counters = s.counters;
  ba.client_next = nullptr;
  ba.seed_base = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);

  if (inline_desc) {
    const int le = launch_batch_inline(wg, spl, full, grid, ba, inl, stream);
    if (le != 0) return hip_fail("batch launch", (hipError_t)le);
  } else if (flags & ZIG_BATCH_NO_GRAPH) {
    e = hipMemcpyAsync(s.dev, s.host, sizeof(BatchHeader) + (size_t)m * sizeof(BatchReq), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail("hipMemcpyAsync(batch)", e);
    int le = launch_batch(wg, spl, full, grid, ba, stream);
    if (le != 0) return hip_fail("batch launch", (hipError_t)le);
  } else {
    // the graph copies the bucket's worth of descriptors and launches the
    // device-filling grid
    uint32_t bucket = 64;
    while (bucket < m) bucket <<= 1;
    const auto key = std::make_tuple(bucket, wg, spl, full);
    auto it = s.graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it != s.graphs.end()) {
      exec = it->second;
    } else {
      if (!db->capture) {
        e = hipStreamCreateWithFlags(&db->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail("hipStreamCreate(capture)", e);
      }
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(db->capture, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail("hipStreamBeginCapture", e);
      const size_t bytes = sizeof(BatchHeader) + (size_t)bucket * sizeof(BatchReq);
      hipError_t e1 = hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, db->capture);
      int le = launch_batch(wg, spl, full, grid, ba, db->capture);
      e = hipStreamEndCapture(db->capture, &g);
      if (e1 != hipSuccess) return hip_fail("capture: hipMemcpyAsync", e1);
      if (le != 0) return hip_fail("capture: batch launch", (hipError_t)le);
      if (e != hipSuccess) return hip_fail("hipStreamEndCapture", e);
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail("hipGraphInstantiate", e);
      s.graphs[key] = exec;
    }
    e = hipGraphLaunch(exec, st);
    if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
  }
  e = hipEventRecord(s.done, st);
  if (e != hipSuccess) return hip_fail("hipEventRecord(batch slot)", e);
  s.used = true;
  return ZIG_OK;
}

}  // namespace zig

extern "C" int zig_fill_batch(const zig_request* reqs, uint32_t count, void* stream) {
  return zig::fill_batch_impl(reqs, count, stream, nullptr);
}

extern "C" int zig_fill_batch_ex(const zig_request* reqs, uint32_t count, void* stream, const zig_batch_opts* opts) {
  return zig::fill_batch_impl(reqs, count, stream, opts);
}

extern "C" int zig_fill_each(const zig_request* reqs, uint32_t count, void* stream) {
  if (count > 0 && reqs == nullptr) {
    zig::set_error("reqs is null");
    return ZIG_EINVAL;
  }
  for (uint32_t i = 0; i < count; ++i) {
    const zig_request& r = reqs[i];
    int e = zig_fill(r.dist, r.dtype, r.seed, r.first_index, r.n, r.p0, r.p1, r.out, stream, nullptr);
    if (e != ZIG_OK) return e;
  }
  return ZIG_OK;
}
