/*
 * zig.h -- C ABI of the MI355X (gfx950) modified-ziggurat sampler.
 *
 * The method is McFarland's modified ziggurat (arXiv:1403.6870): equal-area
 * layers that lie wholly under the density are sampled by a single multiply
 * (section 2, Table 1 modified column, step 2); only the rare tail, overhang
 * and cap regions fall back to rejection or a tail sampler (Table 1 steps
 * 3-8, the paragraph after Table 1, Appendix C).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status (ZIG_OK = 0) and never throws.
 *    On a non-zero status, zig_last_error() returns a message describing it
 *    (thread-local, valid until the next call on the same thread).
 *  - Output buffers are device memory owned by the caller (hipMalloc'd or a
 *    framework allocation); capacity >= n * element size, aligned to the
 *    element size.  The library never frees or retains them.
 *  - `stream` is a hipStream_t passed as an opaque pointer; NULL is the
 *    default stream of the current device.  Fills are asynchronous: they
 *    return after enqueueing, launch failures return ZIG_EHIP, and a
 *    device fault surfaces at the caller's next synchronisation.
 *  - Determinism: the output at global index k is a pure function of
 *    (distribution, dtype, seed, k, parameters, i_max).  It does not depend
 *    on the stream, launch shape, batch composition or call splitting:
 *    fill(first, n) equals fill(first, a) followed by fill(first + a, n - a).
 *  - The uniform source is Philox4x32-10 keyed by (seed mod 2^32,
 *    seed >> 32).  Output k of an FP64 fill takes the 64-bit word
 *    (k even: words 0|1, k odd: words 2|3) of the block with counter
 *    (k>>1, 0, 0); an FP32 fill takes word k&3 of counter (k>>2, 0, 1); the
 *    rejection and tail work of output k draws words t = 0, 1, ... from
 *    counter (k, t>>1, 2).
 */
#ifndef ZIG_H
#define ZIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ZIG_OK 0
#define ZIG_EINVAL 1     /* invalid argument */
#define ZIG_ENOTABLES 2  /* table construction failed */
#define ZIG_EHIP 3       /* a HIP runtime call or kernel launch failed */
#define ZIG_ENOMEM 4     /* device or host allocation failed */
#define ZIG_EBUSY 5      /* server admission refused (non-blocking submit) */
#define ZIG_ESTATE 6     /* object in the wrong state (closed server, unknown ticket) */

/* distributions and output types */
#define ZIG_EXP 0u
#define ZIG_NORMAL 1u
#define ZIG_F64 0u
#define ZIG_F32 1u

/* Builds the layer, region and alias tables of both distributions with
 * i_max layers (section 2: equal-area layers solved from
 * X_i (P(X_i) - P(X_{i-1})) = 1/i_max, computed in 113-bit precision and
 * rounded to double as in Appendix B), and uploads them to the current
 * device.  i_max must be a power of two in [8, 256].  Idempotent and
 * thread-safe; the tables are immutable afterwards.  Fills call it
 * implicitly with the i_max they use (256 by default).
 * Errors: ZIG_EINVAL (bad i_max), ZIG_ENOTABLES, ZIG_EHIP, ZIG_ENOMEM. */
int zig_build_tables(uint32_t i_max);

/* Host-side read-only view of one distribution's tables, for inspection
 * and checking.  Pointers stay valid until the process ends.  Layers are
 * i = 0..L-1 bottom up, with X[L] = 0 and f[L] = 1 closing the top cap;
 * regions are j = 0 (tail), 1..L-1 (overhang right of layer j), L (cap).
 *   X, f      L+1 entries: layer lengths and heights f_i = P(X_i)
 *   XS        i_max entries: X_i * 2^-53 (0 for i >= L)
 *   XS32      i_max entries: RN32(X_i) * 2^-24 (exp) or 2^-23 (normal)
 *   W, H      L+1 entries, index 0 unused: box width X_{j-1} - X_j and
 *             height f_j - f_{j-1} of region j
 *   q         L+1 entries: integer region weights, sum 2^64
 *   T, alias  i_max entries: alias thresholds (units of 2^-(64-b),
 *             b = log2 i_max) and alias targets
 *   eps, K_eps  exponential only: the widest normalised band between a
 *             box's chord and the density, and floor((1 - eps) 2^53)
 *   X0, invX0 tail start and RN(1/X0).
 * Builds the tables if needed.  Errors: ZIG_EINVAL, ZIG_ENOTABLES. */
typedef struct {
  uint32_t dist, i_max, b, L;
  const double* X;
  const double* f;
  const double* XS;
  const float* XS32;
  const double* W;
  const double* H;
  const uint64_t* q;
  const uint64_t* T;
  const uint32_t* alias;
  double eps;
  uint64_t K_eps;
  double X0, invX0;
} zig_table_view;
int zig_get_tables(uint32_t dist, uint32_t i_max, zig_table_view* out);

/* out[k] = sample of Exp(lambda) at global index first_index + k, k < n:
 * x from the modified ziggurat for e^-x (Table 1; tail by recursion on
 * the memoryless tail; overhangs by the reflected three-region test of
 * Figure 2), then out = fma(RN(1/lambda), x, 0).  dtype ZIG_F64 (double
 * out) or ZIG_F32 (float out).  n = 0 is a no-op.
 * Errors: ZIG_EINVAL (null out with n > 0, bad dtype, lambda not finite
 * or <= 0, first_index + n > 2^64), ZIG_EHIP. */
int zig_fill_exp(uint64_t seed, uint64_t first_index, uint64_t n, uint32_t dtype, double lambda, void* out,
                 void* stream);

/* out[k] = sample of N(mu, sigma^2) at global index first_index + k:
 * magnitude from the modified ziggurat for e^-x^2/2 on x >= 0 (Table 1;
 * Marsaglia's tail on exponential draws; plain box rejection in the
 * overhangs), sign from a bit of the uniform word, then
 * out = fma(sigma, +-x, mu).  Errors as zig_fill_exp (sigma finite > 0,
 * mu finite). */
int zig_fill_normal(uint64_t seed, uint64_t first_index, uint64_t n, uint32_t dtype, double mu, double sigma,
                    void* out, void* stream);

/* Launch shape and table size for zig_fill.  Zero fields mean "pick":
 * i_max 256; wg/spl from the tuned table.  wg in {64,...,1024} lanes
 * per workgroup and spl in {1,2,4,8} Philox blocks per lane make a tile
 * of wg * spl blocks (at most 2048), which is also the depth of the
 * per-workgroup slow-output queue. */
typedef struct {
  uint32_t i_max;
  uint32_t wg;
  uint32_t spl;
} zig_launch;

/* Generic fill: dist ZIG_EXP (p0 = lambda, p1 ignored) or ZIG_NORMAL
 * (p0 = mu, p1 = sigma); launch may be NULL.  Same contract as above. */
int zig_fill(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0, double p1,
             void* out, void* stream, const zig_launch* launch);

/* Debug variant of zig_fill that also records, per output k (device
 * arrays of n entries each, any may be NULL):
 *   layer[k]  layer index i taken from the fast word,
 *   region[k] region j of the first alias draw, -1 on the fast path,
 *   words[k]  64-bit slow-stream words consumed,
 *   tests[k]  evaluations of the density in accept/reject tests.
 * Slower; for checking only. */
int zig_fill_trace(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0,
                   double p1, void* out, uint32_t* layer, int32_t* region, uint32_t* words, uint32_t* tests,
                   void* stream, const zig_launch* launch);

/* One request of a batch: dist ZIG_EXP (p0 = lambda) or ZIG_NORMAL (p0 = mu,
 * p1 = sigma), dtype, seed, first_index, n and a caller-owned device output
 * of n elements; the same contract as zig_fill for each request. */
typedef struct {
  uint32_t dist, dtype;
  uint64_t seed, first_index, n;
  double p0, p1;
  void* out;
} zig_request;

/* Batch options: launch shape (0 = default) and flags. */
#define ZIG_BATCH_NO_GRAPH 1u /* launch the copy and kernel directly instead of replaying a graph */
typedef struct {
  uint32_t wg, spl;
  uint32_t flags;
} zig_batch_opts;

/* Fills `count` requests (up to 2^20) of uneven sizes, mixed distributions,
 * dtypes and parameters in one persistent launch: the requests' tiles form
 * one flat space that the device's workgroups take in chunks from an atomic
 * counter.  Each request's output is bit-identical to zig_fill of the same
 * request.  The request descriptors are copied from a ring of pinned host
 * slots by a captured hipGraph (copy + kernel) that is replayed on `stream`;
 * `reqs` may be reused as soon as the call returns.  Outputs of different
 * requests must not overlap.  Requests with n = 0 are skipped; an invalid
 * request fails the whole call with ZIG_EINVAL (its index in the message)
 * before any device work. */
int zig_fill_batch(const zig_request* reqs, uint32_t count, void* stream);
int zig_fill_batch_ex(const zig_request* reqs, uint32_t count, void* stream, const zig_batch_opts* opts);

/* The same requests as zig_fill_batch, launched one zig_fill per request in
 * order on `stream` (the per-request baseline the batch is compared with).
 * Stops at the first failing request. */
int zig_fill_each(const zig_request* reqs, uint32_t count, void* stream);

/* Message for the last non-zero status on this thread ("" if none). */
const char* zig_last_error(void);

/* Library version string. */
const char* zig_version(void);

#ifdef __cplusplus
}
#endif
#endif
