// Internal declarations shared by the library's host and device sources.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace zig {

constexpr uint32_t kMaxLayers = 1024;  // largest supported i_max
// Largest i_max whose slow-path tables the standard kernels keep in LDS;
// larger tables (Appendix D item 1's 1024 layers) run in the wide kernels,
// which keep only the fast-path table there.
constexpr uint32_t kLdsLayers = 256;
constexpr uint32_t kDistExp = 0;
constexpr uint32_t kDistNormal = 1;
constexpr uint32_t kF64 = 0;
constexpr uint32_t kF32 = 1;

// Tables of one distribution as the kernels read them (device memory).
// Layers i < L; X[L] = 0 and f[L] = 1 close the cap; box j (1..L) spans
// [X[j], X[j] + W[j]] x [f[j-1], f[j-1] + H[j]].
struct DevTable {
  uint32_t dist, i_max, b, L;
  uint64_t K_eps;
  uint64_t K_cvx, K_ccv;  // normal: chord-band thresholds of the accelerated overhang variant
  double X0, invX0;
  double XS[kMaxLayers];
  float XS32[kMaxLayers];
  double X[kMaxLayers + 1];
  double f[kMaxLayers + 1];
  double W[kMaxLayers + 1];
  double H[kMaxLayers + 1];
  // alias column c: its threshold in the high 64 - b bits (a full
  // column's, 2^(64-b), stored one less: it decides nothing, since such a
  // column is its own alias) and its alias in the low b bits
  uint64_t TA[kMaxLayers];
  // normal: per-box squeeze of the plain box test on k1 + k2 (the two
  //53-bit uniforms): below SQlo[j] the point is under the density, at or
  // above SQhi[j] it is over it, both with a margin far beyond rounding
  uint64_t SQlo[kMaxLayers + 1];
  uint64_t SQhi[kMaxLayers + 1];
};

// g++ builds the host side and hipcc the device side: both must agree
static_assert(sizeof(DevTable) == 53336 + 2 * 8 * (kMaxLayers + 1), "DevTable layout");

// Host copy with the same content plus the quantities only tests need.
struct HostTable {
  uint32_t dist = 0, i_max = 0, b = 0, L = 0;
  std::vector<double> X, f, XS, W, H;
  std::vector<float> XS32;
  std::vector<uint64_t> q, T;
  std::vector<uint32_t> A;
  double eps = 0.0, X0 = 0.0, invX0 = 0.0;
  uint64_t K_eps = 0;
  double eps_cvx = 0.0, del_ccv = 0.0;  // normal only
  uint64_t K_cvx = 0, K_ccv = 0;
  std::vector<uint64_t> SQlo, SQhi;  // normal only, index j = 1..L
};

// Builds one distribution's tables in binary128 (zig_tables.cpp).
// Returns an empty string on success, else a message.
std::string build_host_table(uint32_t dist, uint32_t i_max, HostTable* out);

// Tables of the traditional ziggurat (Marsaglia & Tsang), the comparison
// sampler of Table 1, as the kernels read them: n layers of equal area v;
// layer 0 is the rectangle [0, X_0] x [0, f_0] plus the tail beyond X_0
// (width W_0 = v / f_0), layer i >= 1 the rectangle [0, X_{i-1}] x
// [f_{i-1}, f_i] (width W_i = X_{i-1}); X_{n-1} = 0 and f_{n-1} = 1.  A draw
// with magnitude bits k (53 bits) in layer i has x = k W_i 2^-53 and lies
// wholly under the density when k < KQ[i] = ceil(2^53 X_i / W_i).
struct DevTrad {
  uint32_t dist, n, b, pad;
  double r, invr;
  double WS[kLdsLayers];
  uint64_t KQ[kLdsLayers];
  double f[kLdsLayers];
};
static_assert(sizeof(DevTrad) == 6176, "DevTrad layout");

struct HostTrad {
  uint32_t dist = 0, n = 0, b = 0;
  std::vector<double> X, f, W, WS, k;
  std::vector<uint64_t> KQ;
  double r = 0.0, v = 0.0, invr = 0.0;
};

// Builds the traditional stack of n <= kLdsLayers layers in binary128
// (zig_tables.cpp).
std::string build_host_trad(uint32_t dist, uint32_t n, HostTrad* out);

// Kernel-side argument block of a plain fill.
struct FillArgs {
  uint64_t seed;
  uint64_t first;     // first global output index
  uint64_t last;      // last global output index (inclusive)
  uint64_t blk0;      // first Philox block of this launch
  uint64_t blk_last;  // last Philox block of the whole fill
  void* out;          // element 0 of the caller's buffer (index `first`)
  double scale, shift;
  const DevTable* tab;   // tables of the distribution
  const DevTable* etab;  // exponential tables (normal tail)
  uint32_t* counters;    // [0] next tile step, [1] workgroups done, zero between launches;
                         // null: workgroup w takes tiles w, w + grid, ...
  uint32_t tiles;        // tiles of WG * S blocks in this launch
  uint32_t chunk;        // tiles taken per step of the counter
  uint32_t aligned16;    // 16-byte block stores are aligned
  uint32_t has_full;     // some block has all its outputs in range
  uint64_t full_lo, full_hi;  // first and last such block
  uint32_t accel;        // normal: accelerated overhang variant (chord bands)
  uint32_t pad;
  // trace arrays (trace build only), indexed by output - first
  uint32_t* t_layer;
  int32_t* t_region;
  uint32_t* t_words;
  uint32_t* t_tests;
  // traditional sampler only: its tables (distribution, exponential)
  const DevTrad* ttab;
  const DevTrad* tetab;
};

// Fills of at most this many tiles per compute unit use the static tile
// schedule (a.counters null); larger ones take tiles from a counter pair.
constexpr uint32_t kStaticTilesPerCU = 16;

// Launch of one (dist, dtype, wg, spl) variant over a.tiles tiles, with as
// many persistent workgroups as fit on the device; defined in zig_fill.hip.
// Returns 0 or a hipError_t value.
int launch_fill(uint32_t dist, uint32_t dtype, uint32_t wg, uint32_t spl, bool trace, const FillArgs& a,
                void* stream);

// The same for tables of more than kLdsLayers layers (zig_fill_wide.hip);
// no accelerated variant.
int launch_fill_wide(uint32_t dist, uint32_t dtype, uint32_t wg, uint32_t spl, bool trace, const FillArgs& a,
                     void* stream);

// The same for the traditional sampler, FP64 only (zig_trad.hip); a.ttab
// and a.tetab set.
int launch_trad(uint32_t dist, uint32_t wg, uint32_t spl, const FillArgs& a, void* stream);

// Raw moments (zig_moments.hip): a.tiles is unused; `tiles` tiles of
// 256 * spl Philox blocks from a.blk0.  At most max_groups workgroups run,
// each writing its 5 partial sums to partial[5 * w ..]; a second kernel
// writes their total to sums.  Returns 0 or a hipError_t value.
constexpr uint32_t kMomMaxGroups = 4096;
bool moments_spl_supported(uint32_t spl);
int launch_moments(uint32_t dist, uint32_t dtype, uint32_t spl, const FillArgs& a, uint64_t tiles, double* partial,
                   uint32_t max_groups, double* sums, void* stream);
// Device address of the file-scope partial-sum array of zig_moments_noalloc
// (kMomMaxGroups * 5 doubles) on the current device, looked up once per
// device.  Returns 0 or a hipError_t value.
int moments_static_scratch(double** out);
int launch_moments_zero(double* sums, void* stream);

// One request of a batch as the batch kernel reads it (device memory).
struct BatchReq {
  uint64_t seed, first, last, blk0, blk_last, full_lo, full_hi;
  void* out;
  double scale, shift;
  uint32_t dist, dtype, aligned16, has_full;
  uint32_t tile_start;  // first tile of this request in the batch's tile space
  uint32_t tiles;       // tiles of this request
};
static_assert(sizeof(BatchReq) == 104, "BatchReq layout");

// Device batch buffer: a header followed by `count` requests.
struct BatchHeader {
  uint32_t count;        // requests (all with n > 0)
  uint32_t total_tiles;  // tiles of all requests
  uint32_t chunk;        // tiles per step of the counter
  uint32_t pad;
};
static_assert(sizeof(BatchHeader) == 16, "BatchHeader layout");

struct BatchArgs {
  const BatchHeader* hdr;  // followed by the BatchReq array
  const DevTable* tabs;    // [exp, normal]
  uint32_t* counters;      // [0] next chunk, [1] workgroups done; zero between launches
  // Serving: when not null, the last workgroup to finish raises
  // client_next[seed - seed_base] to (last index + 1) of every request.
  uint64_t* client_next;
  uint64_t seed_base;
};

// A small batch whose header and requests travel in the kernel arguments
// (no descriptor copy): the requests follow the header as in device memory.
constexpr uint32_t kInlineReqs = 8;
struct BatchInline {
  BatchHeader hdr;
  BatchReq reqs[kInlineReqs];
};
static_assert(sizeof(BatchInline) == 16 + 104 * kInlineReqs, "BatchInline layout");

// counters[c] = max(counters[c], ends[c]) for c < count, on `stream`: the
// owed client counter raises of served requests that ran as plain fills.
int launch_raise_counters(uint64_t* counters, const uint64_t* ends, uint32_t count, void* stream);

// Descriptor of one checked request with n > 0; the tile fields are left
// for the caller, which knows the tile size (zig_batch.cpp).
void make_descriptor(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double scale,
                     double shift, void* out, BatchReq* d);
// Tiles per step of the batch kernel's work counter.
uint32_t batch_chunk(uint64_t total_tiles, uint32_t tile_blocks, uint32_t groups);

// Batch kernel launch of one (wg, spl) variant with `grid` workgroups
// (zig_batch.hip); returns 0 or a hipError_t value.  batch_groups gives the
// resident workgroup count of that variant on the current device.
// `full` selects the variant that stages every table in LDS (see
// batch_full); batch_groups gives each variant's resident count.
int launch_batch(uint32_t wg, uint32_t spl, bool full, uint32_t grid, const BatchArgs& a, void* stream);
// The same with the descriptors in the kernel arguments (a.hdr unused).
int launch_batch_inline(uint32_t wg, uint32_t spl, bool full, uint32_t grid, const BatchArgs& a,
                        const BatchInline& inl, void* stream);

int batch_groups(uint32_t wg, uint32_t spl, bool full, uint32_t* groups);

// The staged-table variant for batches too small to keep the lean one's
// resident workgroups busy for a few tiles each (zig_batch.cpp).
bool batch_full(uint64_t total_tiles, uint32_t lean_groups);
bool batch_shape_supported(uint32_t wg, uint32_t spl);

// zig_fill for callers that keep many fills queued on several streams of
// their own and own a counter pair per launch in flight (zig_api.cpp): a
// large fill takes its tiles from `counters` (zero at rest, left at zero)
// instead of the library's ring, so no event waits couple the streams;
// with counters null every size uses the fixed tile schedule.
int fill_own_counters(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first, uint64_t n, double p0,
                      double p1, void* out, void* stream, uint32_t* counters);

// Shared helpers of the C ABI implementation (zig_api.cpp).
int device_tables_for(uint32_t i_max, const DevTable** out);
int stream_capturing_for(void* stream, bool* capturing);  // whether stream is being captured into a graph
int params_for(uint32_t dist, double p0, double p1, double* scale, double* shift);
void set_error(const std::string& msg);
void clear_error();

}  // namespace zig
