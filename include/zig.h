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
 *    default stream of the current device (hipStreamPerThread is accepted
 *    too).  Fills are asynchronous: they return after enqueueing, launch
 *    failures return ZIG_EHIP, and a device fault surfaces at the caller's
 *    next synchronisation.  Work enqueued on hipStreamPerThread is
 *    synchronised by that thread (for instance with
 *    hipStreamSynchronize(hipStreamPerThread)) before the thread ends: a
 *    device-wide synchronisation afterwards need not wait for it.
 *  - Scratch: a fill of more than 16 tiles per compute unit takes its
 *    tiles from an atomic counter pair; the library owns a ring of 64 such
 *    pairs per device (allocated on first use, kept until the process
 *    ends) and gives each launch its own, behind an event, so concurrent
 *    fills on any streams and threads never share one.  Smaller fills, and
 *    every fill enqueued on a stream that is being captured into a graph,
 *    use a fixed tile-to-workgroup schedule with no scratch, so a captured
 *    graph may be replayed on several streams at once.
 *  - Graph capture: a fill enqueued on a capturing stream allocates and
 *    copies nothing, so its tables must already be on the device
 *    (zig_build_tables(i_max), or an earlier uncaptured fill with that
 *    i_max on that device; for the traditional sampler, an uncaptured
 *    traditional fill).  Otherwise it returns ZIG_ESTATE and enqueues
 *    nothing, and the capture stays usable.  zig_moments and the batch
 *    calls refuse a capturing stream (ZIG_EINVAL); zig_moments_noalloc
 *    may be captured.
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
#define ZIG_ESTATE 6     /* wrong state (closed server, unknown ticket, tables not built before capture) */

/* distributions and output types */
#define ZIG_EXP 0u
#define ZIG_NORMAL 1u
#define ZIG_F64 0u
#define ZIG_F32 1u

/* Builds the layer, region and alias tables of both distributions with
 * i_max layers (section 2: equal-area layers solved from
 * X_i (P(X_i) - P(X_{i-1})) = 1/i_max, computed in 113-bit precision and
 * rounded to double as in Appendix B), and uploads them to the current
 * device.  i_max must be a power of two in [8, 1024] (Appendix D item 1
 * names 1024; 256 is the paper's choice).  Idempotent and
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
 *   XS32      i_max entries: RN32(X_i) * 2^-(32-s) (exp) or 2^-(31-s)
 *             (normal), s = max(b, 8): 2^-24 / 2^-23 up to 256 layers
 *   W, H      L+1 entries, index 0 unused: box width X_{j-1} - X_j and
 *             height f_j - f_{j-1} of region j
 *   q         L+1 entries: integer region weights, sum 2^64
 *   T, alias  i_max entries: alias thresholds (units of 2^-(64-b),
 *             b = log2 i_max) and alias targets
 *   eps, K_eps  exponential only: the widest normalised band between a
 *             box's chord and the density, and floor((1 - eps) 2^53)
 *   X0, invX0 tail start and RN(1/X0).
 *   eps_cvx, del_ccv, K_cvx, K_ccv  normal only, for the accelerated
 *             overhang variant (ZIG_LAUNCH_NORMAL_ACCEL): the widest
 *             normalised chord-curve gap of the convex boxes (X_j >= 1)
 *             and of the concave ones (X_{j-1} <= 1), and the thresholds
 *             floor((1 - eps_cvx (1 + 2^-20)) 2^53) and
 *             ceil((1 + del_ccv (1 + 2^-20)) 2^53) on k1 + k2.
 *   sq_lo, sq_hi  normal only (NULL for the exponential), L+1 entries,
 *             index 0 unused: the squeeze of the plain box test of box j.
 *             With k1, k2 its two 53-bit uniforms, k1 + k2 < sq_lo[j]
 *             lies under the density and k1 + k2 >= sq_hi[j] over it, each
 *             with a margin of 2^-20 of the box (or of its chord gap), so
 *             the kernels decide such points without evaluating the
 *             density and with the same outcome.  Convex boxes (X_j >= 1):
 *             floor((1 - gap_j (1 + 2^-20)) 2^53) + 1 and 2^53 + 2^33;
 *             concave ones (X_{j-1} <= 1): 2^53 - 2^33 and
 *             ceil((1 + gap_j (1 + 2^-20)) 2^53); the box holding x = 1:
 *             0 and 2^55 (never).
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
  double eps_cvx, del_ccv;
  uint64_t K_cvx, K_ccv;
  const uint64_t* sq_lo;
  const uint64_t* sq_hi;
} zig_table_view;
int zig_get_tables(uint32_t dist, uint32_t i_max, zig_table_view* out);

/* Host-side view of the traditional ziggurat's tables (the comparison
 * sampler of Table 1), n = i_max layers of equal area v, built in
 * binary128 and rounded to double.  Layer 0 is the rectangle
 * [0, X_0] x [0, f_0] plus the tail beyond X_0 = r; layer i >= 1 is
 * [0, X_{i-1}] x [f_{i-1}, f_i]; X_{n-1} = 0, f_{n-1} = 1; r is fixed by
 * the top layer having area v too.  All arrays have n entries:
 *   X, f   layer corners (f_i = P(X_i))
 *   W      layer widths: W_0 = v / f_0, W_i = X_{i-1}
 *   WS     W_i * 2^-53
 *   k      X_i / W_i, the share of layer i wholly under the density
 *   KQ     ceil(2^53 k_i): magnitude bits below it quick-accept
 * Pointers stay valid until the process ends.  Errors: ZIG_EINVAL,
 * ZIG_ENOTABLES. */
typedef struct {
  uint32_t dist, n, b, pad;
  const double* X;
  const double* f;
  const double* W;
  const double* WS;
  const double* k;
  const uint64_t* KQ;
  double r, v, invr;
} zig_trad_view;
int zig_get_trad_tables(uint32_t dist, uint32_t i_max, zig_trad_view* out);

/* out[k] = sample of Exp(lambda) at global index first_index + k, k < n:
 * x from the modified ziggurat for e^-x (Table 1; tail by recursion on
 * the memoryless tail; overhangs by the reflected three-region test of
 * Figure 2), then out = fma(RN(1/lambda), x, 0).  dtype ZIG_F64 (double
 * out) or ZIG_F32 (float out).  n = 0 is a no-op.
 * Errors: ZIG_EINVAL (null out with n > 0, bad dtype, lambda not finite
 * or <= 0, first_index + n > 2^64), ZIG_ESTATE (capturing stream, tables
 * not yet on the device), ZIG_EHIP. */
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

/* Launch shape, table size and variant for zig_fill.  Zero fields mean
 * "pick": i_max 256; wg/spl from the tuned table.  wg in {64,...,1024}
 * lanes per workgroup and spl in {1,2,4,8} Philox blocks per lane make a
 * tile of wg * spl blocks (at most 2048; also wg 256 with spl 7 or 10,
 * 1792 or 2560 blocks), whose slow outputs the workgroup gathers and
 * finishes together.  The shape never changes the outputs.
 * i_max above 256 (512 or 1024 layers) takes b = log2 i_max index bits:
 * the FP64 word keeps its layout (sign bit 10, magnitude bits 11..63);
 * the FP32 word gives bits 0..b-1 to the index, the exponential's
 * magnitude bits b..31 (x = k RN32(X_i) 2^-(32-b)), the normal's sign bit b
 * and magnitude bits b+1..31 (2^-(31-b)).  Such tables run the plain
 * modified sampler only (no flags).
 * flags: ZIG_LAUNCH_NORMAL_ACCEL selects, for the normal distribution, an
 * accelerated overhang sampler that goes beyond the paper's text (which
 * gives the chord split for the exponential only, section 2): in the
 * boxes right of the inflection point x = 1 the density is convex, points
 * above the chord are reflected across it and points below the band
 * k1 + k2 <= K_cvx accepted without evaluating it; in the boxes left of
 * it (and the cap) the density is concave, points on or below the chord
 * are accepted and points with k1 + k2 > K_ccv rejected without
 * evaluating it; the box containing x = 1 keeps plain rejection.  Its
 * outputs are a different exact sample than the default's (the slow
 * outputs differ; fast-path and tail outputs are the same); the
 * exponential ignores the flag.
 * ZIG_LAUNCH_TRADITIONAL replaces the modified sampler with the
 * traditional ziggurat the paper compares against (Table 1, right
 * column; Marsaglia & Tsang's stack of i_max equal-area layers, tables as
 * zig_get_trad_tables describes): output g takes layer i and magnitude
 * bits k from its fast word exactly as the modified sampler does and
 * returns x = k W_i 2^-53 when k < KQ[i]; otherwise a wedge test draws
 * U2 from the output's slow stream (accept when
 * f_{i-1} + U2 (f_i - f_{i-1}) < P(x)), and each rejection takes a fresh
 * (i, k) word from the same stream; layer 0 past X_0 is the tail
 * (exponential: X_0 plus a fresh traditional exponential; normal:
 * Marsaglia's method on two traditional exponentials).  FP64 only, no
 * trace; not combinable with ZIG_LAUNCH_NORMAL_ACCEL.  It exists for the
 * comparison of Table 1. */
#define ZIG_LAUNCH_NORMAL_ACCEL 1u /* normal overhangs: the accelerated variant (see below) */
#define ZIG_LAUNCH_TRADITIONAL 2u  /* the traditional ziggurat, for comparison */
typedef struct {
  uint32_t i_max;
  uint32_t wg;
  uint32_t spl;
  uint32_t flags;
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

/* Fused generate-and-reduce: the raw moment sums S_p = sum over k of x_k^p,
 * p = 1..5, of the n outputs x_k that zig_fill with the same arguments
 * would write (as written: doubles, or floats widened to double), written
 * to sums[0..4] in device memory (caller-owned, 8-byte aligned); no output
 * is written to HBM.  This is the generate-and-aggregate form of the
 * paper's benchmark (section 3) and the statistic of Appendix B's
 * raw-moment table.
 * Each term is formed by double products (x*x, then its square; the odd
 * powers multiply by x fused with their addition) and added in an order
 * fixed by the launch: workgroup w of G takes the tiles w, w + G, ... of
 * 256 * spl Philox blocks from first_index / 2 (FP64) or / 4 (FP32); each
 * lane adds its own terms, at most 2 * spl * O per tile (O = 2 outputs per
 * block for FP64, 4 for FP32); lane sums are added over each wave by a
 * shuffle tree, over the 4 waves in order, and the G partial sums by 256
 * lanes in sequence and a halving tree.  G is the number of resident
 * workgroups of the kernel (at least min(tiles, compute units), at most
 * 4096), so a device gives the same bits on every run.  The result
 * therefore differs from the exact sum of the same terms by at most
 * gamma_h * sum |x_k^p| + 2^-53 sum |x_k^p|, gamma_h = h u / (1 - h u),
 * u = 2^-53, h = 2 spl O ceil(tiles / G) + ceil(G / 256) + 18.
 * launch may be NULL; launch->i_max (up to 256), launch->spl (16, 32 or
 * 64; default 32, with wg 0 or 256) and ZIG_LAUNCH_NORMAL_ACCEL are
 * honoured.  Asynchronous on `stream`; each launch takes one of 4
 * per-device scratch slots of 160 KB (partial sums), behind an event.  A
 * stream being captured is refused (ZIG_EINVAL): a graph would fix the
 * slot.  Errors: as zig_fill (sums in place of out). */
int zig_moments(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0, double p1,
                double* sums, void* stream, const zig_launch* launch);

/* zig_moments for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and summation order as zig_moments, but it calls
 * no allocating routine: the partial sums live in a static device array
 * of 4096 x 5 doubles (160 KB) that each GPU the library runs on holds
 * until the process ends, and the tables must already be built on the
 * current device (zig_build_tables(i_max) first, else ZIG_ESTATE).  The
 * array holds the most workgroups one launch uses, so no n is refused on
 * its account.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, concurrent replays of
 * a graph holding such a call) race and give wrong sums.  A capturing
 * stream is accepted.  Errors: as zig_moments, plus ZIG_ESTATE. */
int zig_moments_noalloc(uint32_t dist, uint32_t dtype, uint64_t seed, uint64_t first_index, uint64_t n, double p0,
                        double p1, double* sums, void* stream, const zig_launch* launch);

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
 * a batch of at most 8 requests instead passes them in the kernel
 * arguments and is launched directly.  `reqs` may be reused as soon as the
 * call returns.  Outputs of different
 * requests must not overlap.  Requests with n = 0 are skipped; an invalid
 * request or an unknown flag fails the whole call with ZIG_EINVAL (a
 * request's index in the message) before any device work, and so does a
 * stream being captured into a graph (the graph would hold one descriptor
 * slot, which later batches reuse). */
int zig_fill_batch(const zig_request* reqs, uint32_t count, void* stream);
int zig_fill_batch_ex(const zig_request* reqs, uint32_t count, void* stream, const zig_batch_opts* opts);

/* The same requests as zig_fill_batch, launched one zig_fill per request in
 * order on `stream` (the per-request baseline the batch is compared with).
 * Stops at the first failing request. */
int zig_fill_each(const zig_request* reqs, uint32_t count, void* stream);

/* Autotuner.  Times, on the current device, every compiled fill shape
 * (workgroup size x Philox blocks per lane, and for fills above 2^21
 * outputs the step of the work counter: 8K, 16K or 32K blocks) for each
 * distribution, output type and size class (n <= 2^17, <= 2^21, <= 2^25,
 * larger; timed at 2^16, 2^20, 2^24 and 2^28 outputs), and the batch
 * kernel's shapes on a fixed mix of 1024 requests; fills and batches on
 * that device then use the fastest (a candidate must beat the current
 * choice by 1 %).  Outputs never depend on the shape, only the speed does.
 * cache_path names a JSON file to load from and save to; NULL takes the
 * environment variable ZIG_AUTOTUNE_CACHE, or none.  A cache is used only
 * if it was written for the same architecture name and compute-unit count.
 * Flags: ZIG_TUNE_LOAD loads only (ZIG_ESTATE if no matching cache exists);
 * ZIG_TUNE_FORCE measures even if a matching cache exists.  Without any
 * call, the first fill on a device loads ZIG_AUTOTUNE_CACHE if it names a
 * matching file, else the built-in table (measured on MI355X) is used.
 * Measuring takes a few seconds and 2 GiB of device memory; other work on
 * the device meanwhile disturbs the timings, not the results.
 * Errors: ZIG_EINVAL (flags, unwritable path), ZIG_ESTATE, ZIG_EHIP,
 * ZIG_ENOMEM. */
#define ZIG_TUNE_LOAD 1u
#define ZIG_TUNE_FORCE 2u
int zig_autotune(const char* cache_path, uint32_t flags);

/* The shape a fill of (dist, dtype, n) uses on the current device; the
 * counter step in Philox blocks goes to *step_blocks (may be NULL). */
int zig_tuned_shape(uint32_t dist, uint32_t dtype, uint64_t n, zig_launch* out, uint32_t* step_blocks);

/* The batch-kernel shape zig_fill_batch uses when none is given. */
int zig_tuned_batch_shape(zig_batch_opts* out);

/* Drops the current device's tuned table (back to the built-in one). */
int zig_autotune_reset(void);

/* ---------------------------------------------------------------------
 * Serving loop: continuous batching of fill requests from many clients.
 *
 * Each client c owns a sample stream with seed seed_base + c and a
 * device-resident next index.  A submitted request of n samples is queued
 * FIFO; the scheduler admits requests in arrival order while their outputs
 * fit into an output arena of cap_bytes (256-byte granules, first fit),
 * gives each its first index from its client's counter in admission order,
 * and launches the admitted requests as one batch on the next free of
 * `streams` fill streams.  Several requests go as a copy of the batch
 * descriptors, then the persistent batch kernel of zig_fill_batch, whose
 * last workgroup raises the device counters to the ends of the batch's
 * requests; a lone request goes as the plain fill of that request, and
 * its client's device counter is raised before the counters are next
 * read (zig_server_counters, checkpoints).  A request's
 * samples are therefore the zig_fill output of (dist, dtype,
 * seed_base + c, first_index, n, p0, p1) whatever else it was batched
 * with; first_index is reported in its completion.  The output lives in
 * the arena until the caller releases the ticket.
 * --------------------------------------------------------------------- */
typedef struct zig_server zig_server;

#define ZIG_BACKEND_DEVICE 0u    /* the HIP path on the current device */
#define ZIG_BACKEND_HOST_FAKE 1u /* host threads only, no device calls: the scheduler under test */

/* Server configuration; zero fields take the stated defaults. */
typedef struct {
  uint32_t backend;         /* ZIG_BACKEND_* */
  uint32_t streams;         /* fill streams, 1..8 (default 4); two batches in flight per stream */
  uint32_t max_batch;       /* requests per batch, 1..4096 (default 1024) */
  uint32_t clients;         /* client ids 0..clients-1, at most 2^20 (default 64) */
  uint32_t window_us;       /* gathering window after the oldest queued arrival (default 0) */
  uint32_t fake_latency_us; /* host fake: time each batch takes */
  uint32_t fake_fail_every; /* host fake: every k-th request (count from 1) fails, 0 = never */
  uint32_t pad;
  uint64_t cap_bytes;       /* admission cap: bytes of admitted, unreleased outputs (required) */
  uint64_t seed_base;       /* client c draws from seed seed_base + c */
  void* arena;              /* device arena of cap_bytes supplied by the caller, or NULL to allocate */
} zig_server_cfg;

/* One request: dist/dtype/parameters as zig_fill (p0 = lambda, or p0 = mu,
 * p1 = sigma), n samples, and an optional arrival timestamp
 * (zig_server_now_ns clock) that latencies are measured from (0 = submit
 * time). */
typedef struct {
  uint32_t dist, dtype;
  uint64_t n;
  double p0, p1;
  uint64_t t_arrival_ns;
} zig_spec;

/* Completion record of one request.  Timestamps are zig_server_now_ns
 * values; t_done_ns is taken when the host observes the batch's
 * completion event. */
typedef struct {
  int32_t status;          /* ZIG_OK, or why the request did not run */
  uint32_t client, dist, dtype;
  uint64_t seed, first_index, n;
  void* out;               /* n outputs in the arena (NULL unless status is ZIG_OK) */
  uint64_t batch_id;
  uint32_t batch_size, pad;
  uint64_t t_arrival_ns, t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns;
} zig_completion;

typedef struct {
  uint64_t batches, requests, samples, failed_requests;
  uint64_t max_inflight_batches, max_bytes_in_use;
  uint64_t bytes_in_use, queued, inflight_batches;
} zig_server_stats;

/* Monotonic clock of the server's timestamps, in ns. */
uint64_t zig_server_now_ns(void);

/* Creates a server and starts its scheduler and completion threads.  The
 * device backend uses the current device, allocates the arena unless one
 * is supplied, and starts every client counter at 0.
 * Errors: ZIG_EINVAL (bad configuration), ZIG_ENOMEM, ZIG_EHIP, ZIG_ENOTABLES. */
int zig_server_create(const zig_server_cfg* cfg, zig_server** out);

/* Queues a request of `client`; never waits for admission.  With
 * ZIG_SUBMIT_NONBLOCK the request is refused with ZIG_EBUSY when the bytes
 * admitted or queued would then exceed cap_bytes.  n = 0 completes at once
 * without using an index.  *ticket identifies the request until released.
 * Errors: ZIG_EINVAL (client out of range, bad parameters, n * element size
 * above cap_bytes), ZIG_EBUSY, ZIG_ESTATE (server shutting down).  A request
 * whose indices would pass 2^64 - 2 (counter + n > 2^64 - 1) completes with
 * status ZIG_EINVAL at admission and leaves the counter where it was. */
#define ZIG_SUBMIT_NONBLOCK 1u
int zig_server_submit(zig_server* srv, uint32_t client, const zig_spec* spec, uint32_t flags, uint64_t* ticket);

/* Waits up to timeout_us (negative: no limit) for a request and copies its
 * completion record to *out (may be NULL).  Returns the request's status,
 * ZIG_EBUSY on timeout, ZIG_ESTATE for an unknown ticket. */
int zig_server_wait(zig_server* srv, uint64_t ticket, int64_t timeout_us, zig_completion* out);

/* Returns a completed request's output space to the arena and forgets the
 * ticket.  Errors: ZIG_ESTATE (unknown ticket or not complete). */
int zig_server_release(zig_server* srv, uint64_t ticket);

/* Client disconnect: its queued requests are cancelled (status ZIG_ESTATE,
 * no index used), its completed requests are released, and its requests in
 * flight are released when they complete.  *reclaimed (may be NULL)
 * receives the number of requests cancelled or released. */
int zig_server_drop_client(zig_server* srv, uint32_t client, uint64_t* reclaimed);

/* Snapshot of the device counters (next index) of clients 0..count-1 once
 * every launched batch has finished (checkpoint), and restore of them;
 * restore needs an idle server (nothing queued or in flight).  Errors:
 * ZIG_EINVAL, ZIG_ESTATE (restore on a busy server), ZIG_EHIP. */
int zig_server_counters(zig_server* srv, uint64_t* next_index, uint32_t count);
int zig_server_set_counters(zig_server* srv, const uint64_t* next_index, uint32_t count);

int zig_server_stats_get(zig_server* srv, zig_server_stats* out);

/* Open-loop replay of a request trace: request i is submitted at
 * t0 + arrival_ns[i] (t0 = the call's start), its latency counted from that
 * scheduled time, and released once complete; if copy_to[i] is not NULL its
 * output is first copied there (device memory of n elements).  out[i]
 * receives the completion record (its `out` field is then stale).  Blocks
 * until every request has completed.
 * ZIG_REPLAY_NAIVE replays the same trace on a naive server instead: each
 * request is launched at arrival as its own zig_fill on the next of the
 * server's fill streams (round robin), with its first index from host-side
 * counters that start at 0, and an event per request; the batching
 * scheduler stays idle.  Needs the device backend and an idle server. */
#define ZIG_REPLAY_NAIVE 1u
typedef struct {
  uint32_t client, pad;
  zig_spec spec;           /* spec.t_arrival_ns is the offset from t0 */
  void* copy_to;
} zig_trace_item;
int zig_server_replay(zig_server* srv, const zig_trace_item* items, uint64_t count, uint32_t flags,
                      zig_completion* out);

/* Stops the server: queued requests are cancelled, batches in flight are
 * waited for, every resource (arena included, unless supplied) is freed. */
int zig_server_destroy(zig_server* srv);

/* Message for the last non-zero status on this thread ("" if none). */
const char* zig_last_error(void);

/* Library version string. */
const char* zig_version(void);

#ifdef __cplusplus
}
#endif
#endif
