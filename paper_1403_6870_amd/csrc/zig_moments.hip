// Fused generate-and-reduce: the raw moment sums S_p = sum of x^p, p = 1..5,
// of the outputs a fill would write, with nothing written to HBM (the
// generate-and-aggregate form of the paper's benchmark, section 3, and the
// statistic of Appendix B's raw-moment table).
//
// Each lane keeps five running sums for the whole launch.  Workgroup w of
// G takes tiles w, w + G, w + 2G, ... (a fixed assignment, so the result is
// the same bits on every run with the same G, which depends only on the
// device).  Per tile:
//   A. every lane computes its S Philox blocks; an output on the fast path
//      (layer i < L) is added to the lane's sums at once; slow outputs are
//      recorded in an LDS bitmap by wave ballots (no staging tile);
//   B. wave 0 numbers the slow outputs by prefix sums over the bitmap, and
//      every lane takes a share of them, runs the slow path (region,
//      overhang box or tail) and adds the result to its own sums.
// The bitmap and its prefix sums are double-buffered by tile parity, so
// one barrier after phase A and one after the prefix suffice.  At the end
// the lane sums are reduced over each wave (shuffle tree), over the waves
// in order, and written per workgroup; a second kernel adds the G partial
// sums (256 lanes in sequence, then a halving tree).
//
// Every term is x^p formed from the output as written (FP32 widened to
// double) by products x*x, (x*x)*x, (x*x)^2, (x*x)^2*x, the multiplications
// by x of the odd powers fused with their addition.  A lane adds at most
// 2 S O terms per tile it takes (O outputs per block; S O of its own
// blocks and at most as many slow outputs), so the rounding error of S_p
// is at most gamma_h sum |x^p| + u sum |x^p| with
// h = 2 S O ceil(tiles / G) + 6 + WG / 64 + ceil(G / 256) + 8.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "zig_fill_kernel.hpp"

namespace zig {
namespace {

constexpr int kMomWG = 256;

// Tile of 256 lanes x S Philox blocks (no staging tile, so larger tiles
// than the fill's fit).
template <uint32_t DT, int S>
struct MomShape {
  using OutT = typename OutType<DT>::T;
  static constexpr int O = OutType<DT>::per_block;
  static constexpr int TILE = kMomWG * S;
  static constexpr int NWAVE = kMomWG / 64;
  static constexpr int NWORD = S * O * NWAVE;
  static_assert(NWORD <= 1024, "tile shape");
};

template <uint32_t DT, int S>
struct MomLds {
  using Sh = MomShape<DT, S>;
  typename Sh::OutT xs[kLdsLayers];  // fast-path table, 0 for i >= L
  double X[kLdsLayers + 1];
  double f[kLdsLayers + 1];
  uint64_t TA[kLdsLayers];
  uint64_t slowmap[2][Sh::NWORD];
  uint32_t prefix[2][Sh::NWORD + 1];
  double red[5][Sh::NWAVE];
};

__device__ __forceinline__ void add_powers(double (&acc)[5], double x) {
  const double q2 = x * x;
  const double q4 = q2 * q2;
  acc[0] = acc[0] + x;
  acc[1] = acc[1] + q2;
  acc[2] = __builtin_fma(q2, x, acc[2]);
  acc[3] = acc[3] + q4;
  acc[4] = __builtin_fma(q4, x, acc[4]);
}

// Five waves per SIMD, and phase A unrolled by two blocks rather than fully,
// which keeps the kernel near 90 registers with nothing spilled: measured
// at 2^32 FP64 outputs on 256 x 32 tiles against 256 x 8 fully unrolled
// (three waves), 572 -> 741 Gsamples/s for the exponential and 462 -> 616
// for the normal.  Six waves measured 3 % faster but spill to scratch.
template <uint32_t DIST, uint32_t DT, int S, bool ACCEL>
__global__ void __launch_bounds__(kMomWG) __attribute__((amdgpu_waves_per_eu(5)))
moments_kernel(FillArgs a, uint64_t tiles, double* partial) {
  using Sh = MomShape<DT, S>;
  using OutT = typename Sh::OutT;
  constexpr int WG = kMomWG;
  constexpr int O = Sh::O;
  constexpr int NWAVE = Sh::NWAVE;
  constexpr int NWORD = Sh::NWORD;
  constexpr int TILE = Sh::TILE;
  __shared__ MomLds<DT, S> sh;

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t wave = tid >> 6;
  const DevTable* tb = a.tab;
  const uint32_t L = tb->L;
  for (uint32_t i = tid; i < kLdsLayers; i += WG) {
    if constexpr (DT == kF64)
      sh.xs[i] = i < L ? tb->XS[i] : 0.0;
    else
      sh.xs[i] = i < L ? tb->XS32[i] : 0.0f;
    sh.TA[i] = tb->TA[i];
  }
  for (uint32_t i = tid; i <= kLdsLayers; i += WG) {
    sh.X[i] = tb->X[i];
    sh.f[i] = tb->f[i];
  }
  dev::TabView own = dev::global_view(tb);
  own.X = sh.X;
  own.f = sh.f;
  own.TA = sh.TA;
  const dev::TabView ex = dev::global_view(a.etab);
  const uint32_t imask = own.imask;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const double scale = a.scale;
  const float fscale = (float)a.scale;
  double shiftv = a.shift;
  float fshift = (float)a.shift;
  if constexpr (DIST == kDistNormal) asm volatile("" : "+v"(shiftv), "+v"(fshift));
  __syncthreads();

  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  uint32_t parity = 0;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x, parity ^= 1u) {
    const uint64_t tile0 = a.blk0 + t * TILE;
    const bool interior = a.has_full && tile0 >= a.full_lo && tile0 + (TILE - 1) <= a.full_hi;
    uint64_t* const slowmap = sh.slowmap[parity];
    uint32_t* const prefix = sh.prefix[parity];
    // this wave's first bitmap word, as an LDS address
    const uint32_t lds_word = dev::lds_address(slowmap + wave);

    // A: fast outputs into the sums, slow ones into the bitmap
    auto phase_a = [&](auto interior_tag) {
      constexpr bool IN = decltype(interior_tag)::value;
#pragma unroll 2
      for (int s = 0; s < S; ++s) {
        const uint64_t m = tile0 + (uint64_t)(s * WG) + tid;
        uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = (DT == kF64) ? 0u : 1u;
        dev::philox10(c0, c1, c2, c3, k0, k1);
#pragma unroll
        for (int o = 0; o < O; ++o) {
          const uint64_t g = m * O + o;
          bool live = true;
          if constexpr (!IN) live = (m <= a.blk_last) && (g >= a.first) && (g <= a.last);
          uint32_t i;
          OutT x;
          if constexpr (DT == kF64) {
            const uint32_t lo = (o == 0) ? c0 : c2, hi = (o == 0) ? c1 : c3;
            i = lo & imask;
            const double k = __builtin_fma((double)hi, 0x1p21, (double)(lo >> 11));
            x = k * sh.xs[i];
            if constexpr (DIST == kDistNormal) x = dev::with_sign_of(x, lo << 21);
          } else {
            const uint32_t w = (o == 0) ? c0 : (o == 1) ? c1 : (o == 2) ? c2 : c3;
            i = w & imask;
            if constexpr (DIST == kDistExp) {
              x = (float)(w >> 8) * sh.xs[i];
            } else {
              x = (float)(w >> 9) * sh.xs[i];
              x = dev::with_sign_of(x, w << 23);
            }
          }
          const bool miss = i >= L;
          const bool slow = live && miss;
          double v;
          // the exponential's slow placeholder is scale * 0 = +0, which
          // adds nothing; the normal's is mu and is masked out
          if constexpr (DIST == kDistExp) {
            if constexpr (DT == kF64)
              v = scale * x;
            else
              v = (double)(fscale * x);
            if constexpr (!IN) v = live ? v : 0.0;
          } else {
            if constexpr (DT == kF64)
              v = __builtin_fma(scale, x, shiftv);
            else
              v = (double)__builtin_fmaf(fscale, x, fshift);
            v = (live && !miss) ? v : 0.0;
          }
          add_powers(acc, v);
          const uint64_t mask = __builtin_amdgcn_ballot_w64(slow);
          dev::store_from_lane0(lds_word + (s * O + o) * NWAVE * 8, mask, 0);
        }
      }
    };
    if (interior)
      phase_a(std::true_type());
    else
      phase_a(std::false_type());
    __syncthreads();

    // B: number the slow outputs and share them out over every lane; the
    // prefix pass holds up the workgroup, and the drain the next tile, so
    // both take issue priority over the other workgroups' phase A
    __builtin_amdgcn_s_setprio(2);
    if (wave == 0) {
      constexpr int PER = (NWORD + 63) / 64;
      uint32_t cnt[PER];
      uint32_t mine = 0;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int w = lane * PER + k;
        cnt[k] = (w < NWORD) ? (uint32_t)__popcll(slowmap[w]) : 0u;
        mine += cnt[k];
      }
      const uint32_t incl = dev::wave_inclusive_sum(mine);
      uint32_t run = incl - mine;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int w = lane * PER + k;
        if (w < NWORD) prefix[w] = run;
        run += cnt[k];
      }
      if (lane == 63) prefix[NWORD] = incl;
    }
    __syncthreads();
    const uint32_t total = prefix[NWORD];
    for (uint32_t e = tid; e < total; e += WG) {
      uint32_t lo = 0, hi = NWORD;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= e)
          lo = mid;
        else
          hi = mid;
      }
      uint64_t bits = slowmap[lo];
      for (uint32_t r = e - prefix[lo]; r > 0; --r) bits &= bits - 1;
      const uint32_t ln = (uint32_t)__ffsll((unsigned long long)bits) - 1;
      const uint32_t so = lo / NWAVE, wv = lo % NWAVE;
      const uint32_t s = so / O, o = so % O;
      const uint64_t g = (tile0 + s * WG + wv * 64 + ln) * O + o;
      bool neg = false;
      if constexpr (DIST == kDistNormal) neg = dev::normal_sign<DT>(g, k0, k1, 8u);
      int32_t region;
      uint32_t words, tests;
      const double mag = dev::slow_magnitude<DIST, ACCEL>(own, ex, g, k0, k1, region, words, tests);
      OutT x = (OutT)mag;
      if (neg) x = -x;
      double v;
      if constexpr (DIST == kDistExp) {
        if constexpr (DT == kF64)
          v = scale * x;
        else
          v = (double)(fscale * x);
      } else {
        if constexpr (DT == kF64)
          v = __builtin_fma(scale, x, a.shift);
        else
          v = (double)__builtin_fmaf(fscale, x, fshift);
      }
      add_powers(acc, v);
    }
    __builtin_amdgcn_s_setprio(0);
    // no barrier: the next tile writes the other bitmap, and the one after
    // comes behind that tile's two barriers
  }

  // lane sums -> wave sums (shuffle tree) -> workgroup sums (waves in order)
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const double up = __shfl_down(acc[p], h);
      if ((int)lane < h) acc[p] = acc[p] + up;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < 5; ++p) sh.red[p][wave] = acc[p];
  }
  __syncthreads();
  if (tid < 5) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s = s + sh.red[tid][w];
    partial[(size_t)blockIdx.x * 5 + tid] = s;
  }
}

// sums[p] = the G partial sums of p added by 256 lanes in sequence (lane l
// takes partials l, l + 256, ...) and a halving tree over the lanes.
__global__ void __launch_bounds__(256) partials_kernel(const double* partial, uint32_t groups, double* sums) {
  __shared__ double red[5][256];
  const uint32_t tid = threadIdx.x;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (uint32_t g = tid; g < groups; g += 256) {
#pragma unroll
    for (int p = 0; p < 5; ++p) s[p] = s[p] + partial[(size_t)g * 5 + p];
  }
#pragma unroll
  for (int p = 0; p < 5; ++p) red[p][tid] = s[p];
  __syncthreads();
  for (uint32_t h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int p = 0; p < 5; ++p) red[p][tid] = red[p][tid] + red[p][tid + h];
    }
    __syncthreads();
  }
  if (tid < 5) sums[tid] = red[tid][0];
}

template <class K>
int resident(K kernel, int* out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
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
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kMomWG, 0);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  if (per_cu < 1) return (int)hipErrorInvalidConfiguration;
  *out = cache[key] = per_cu * cus;
  return 0;
}

template <uint32_t DIST, uint32_t DT, int S, bool ACCEL>
int launch_s(const FillArgs& a, uint64_t tiles, double* partial, uint32_t max_groups, double* sums,
             hipStream_t st) {
  auto kernel = moments_kernel<DIST, DT, S, ACCEL>;
  int groups = 0;
  int e = resident(kernel, &groups);
  if (e != 0) return e;
  uint64_t grid = (uint64_t)groups < tiles ? (uint64_t)groups : tiles;
  if (grid > max_groups) grid = max_groups;
  hipLaunchKernelGGL(kernel, dim3((uint32_t)grid), dim3(kMomWG), 0, st, a, tiles, partial);
  e = (int)hipGetLastError();
  if (e != 0) return e;
  hipLaunchKernelGGL(partials_kernel, dim3(1), dim3(256), 0, st, partial, (uint32_t)grid, sums);
  return (int)hipGetLastError();
}

template <uint32_t DIST, uint32_t DT, bool ACCEL>
int launch_d(uint32_t spl, const FillArgs& a, uint64_t tiles, double* partial, uint32_t max_groups, double* sums,
             hipStream_t st) {
  if (spl == 16) return launch_s<DIST, DT, 16, ACCEL>(a, tiles, partial, max_groups, sums, st);
  if (spl == 32) return launch_s<DIST, DT, 32, ACCEL>(a, tiles, partial, max_groups, sums, st);
  if (spl == 64) return launch_s<DIST, DT, 64, ACCEL>(a, tiles, partial, max_groups, sums, st);
  return (int)hipErrorInvalidConfiguration;
}

// Partial sums for zig_moments_noalloc: one slot of 5 doubles per
// workgroup, as many as a launch may use.  Host code must not pass this
// name to a kernel (in host code it is a stand-in, not a device address);
// it uses the address hipGetSymbolAddress gives on each device.
static __device__ __align__(256) double scratch[kMomMaxGroups * 5];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int moments_static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    double* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

bool moments_spl_supported(uint32_t spl) { return spl == 16 || spl == 32 || spl == 64; }

int launch_moments(uint32_t dist, uint32_t dtype, uint32_t spl, const FillArgs& a, uint64_t tiles, double* partial,
                   uint32_t max_groups, double* sums, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dist == kDistNormal && a.accel)
    return dtype == kF64 ? launch_d<kDistNormal, kF64, true>(spl, a, tiles, partial, max_groups, sums, st)
                         : launch_d<kDistNormal, kF32, true>(spl, a, tiles, partial, max_groups, sums, st);
  if (dist == kDistExp && dtype == kF64)
    return launch_d<kDistExp, kF64, false>(spl, a, tiles, partial, max_groups, sums, st);
  if (dist == kDistExp && dtype == kF32)
    return launch_d<kDistExp, kF32, false>(spl, a, tiles, partial, max_groups, sums, st);
  if (dist == kDistNormal && dtype == kF64)
    return launch_d<kDistNormal, kF64, false>(spl, a, tiles, partial, max_groups, sums, st);
  return launch_d<kDistNormal, kF32, false>(spl, a, tiles, partial, max_groups, sums, st);
}

int launch_moments_zero(double* sums, void* stream) {
  hipLaunchKernelGGL(partials_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), nullptr, 0u, sums);
  return (int)hipGetLastError();
}

}  // namespace zig
