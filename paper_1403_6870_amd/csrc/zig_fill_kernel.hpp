// The fill kernel of the modified ziggurat sampler for gfx950 (and, for
// the comparison of Table 1, of the traditional one; see fill_tile).
//
// Work is cut into tiles of WG * S consecutive Philox blocks (2 FP64 or 4
// FP32 outputs per block), each written contiguously by one workgroup.  A
// workgroup first copies the fast-path table X_i 2^-53 and the slow-path
// tables (X, f, alias) of its distribution into LDS.  Per tile:
//   A. every lane computes S blocks.  Each output takes its layer index and
//      magnitude from its fast word; when the layer lies under the density
//      (i < L, Table 1 step 2) its value is one multiply plus the
//      location-scale epilogue.  Values go to an LDS staging tile; for each
//      output slot the wave's ballot of slow lanes (i >= L) is written to an
//      LDS bitmap.
//   B. the slow outputs are numbered by prefix sums over the bitmap words
//      and shared out over all lanes: region draw, overhang box or tail
//      (Table 1 steps 3-8) on the output's own slow stream, tables from
//      LDS (a normal output's sign is re-derived from its fast block); each
//      result overwrites its staging place.
//   C. every lane copies its blocks from LDS to HBM with 16-byte stores.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "zig_device.hpp"

namespace zig {

template <uint32_t DT>
struct OutType;
template <>
struct OutType<kF64> {
  using T = double;
  using V = double2;
  static constexpr int per_block = 2;
};
template <>
struct OutType<kF32> {
  using T = float;
  using V = float4;
  static constexpr int per_block = 4;
};

template <uint32_t DT, int WG, int S>
struct FillShape {
  using OutT = typename OutType<DT>::T;
  using VecT = typename OutType<DT>::V;
  static constexpr int O = OutType<DT>::per_block;
  static constexpr int TILE = WG * S;
  static constexpr int NWAVE = WG / 64;
  static constexpr int NWORD = S * O * NWAVE;  // one 64-bit ballot word per (s, o, wave)
  static_assert(WG % 64 == 0 && NWORD <= 1024 && TILE * 16 <= 40960, "tile shape");
};

// LDS of one workgroup.  CAP is the largest table it serves.  With SLOWLDS
// the slow-path tables (X, f, alias) are staged here too; otherwise only
// the fast-path table is, and the slow paths, which serve one or two
// outputs in a hundred, read the rest from device memory (L2-resident).
// Wide tables always run that way, and so do the shapes for which the
// smaller footprint fits one more workgroup on a CU (lean_shape).
// The traditional sampler (TRAD) keeps its quick-accept thresholds and
// layer heights in T and f and has no use for X and A.
// A tile with at most kListCap slow outputs lists their staging places
// (LIST kernels), so that each drain lane finds its output with one LDS
// read instead of a search of the prefix sums.
constexpr uint32_t kListCap = 128;

template <uint32_t DT, int WG, int S, uint32_t CAP = kLdsLayers, bool SLOWLDS = (CAP <= kLdsLayers),
          bool TRAD = false, bool LIST = false>
struct FillLds {
  using Sh = FillShape<DT, WG, S>;
  static constexpr uint32_t SLOW_XA = SLOWLDS && !TRAD ? CAP : 1;
  static constexpr uint32_t SLOW_FT = SLOWLDS || TRAD ? CAP : 1;
  typename Sh::OutT xs[CAP];
  double X[SLOW_XA + 1];
  double f[SLOW_FT + 1];
  uint64_t T[SLOW_FT];  // packed alias columns, or the traditional sampler's thresholds
  typename Sh::VecT stage[Sh::TILE];
  uint64_t slowmap[Sh::NWORD];
  uint32_t prefix[Sh::NWORD + 1];
  uint16_t list[LIST ? kListCap : 1];
  uint32_t marks[LIST ? 1 : 64];  // kernels without the list: see fill_tile
  uint32_t tile;
};

// 128 x 8, 256 x 8 and 256 x 7 tiles: the staged slow tables (9 KB) are
// what keeps a fourth (256 x 7: fifth) workgroup off a CU's 160 KB of LDS;
// without them the normal fill runs at 4 instead of 3 waves per SIMD
// (2.40 -> 2.10 ms at 2^30 FP64 on 256 x 8).  Larger workgroups of the
// same tile size are limited by registers first and lose from the slower
// table reads.
constexpr bool lean_shape(int wg, int s) {
  return ((wg == 128 || wg == 256) && s == 8) || (wg == 256 && s == 7);
}

// Waves per SIMD the register allocator is asked to allow: 256 x 7 fits 5
// workgroups in LDS, and the normal kernel, at 103 registers by default,
// fits 5 waves in 87 without spilling when asked (2.10 -> 2.06 ms for the
// normal 2^30 FP64 fill, 1.37 -> 1.32 ms in FP32).  1 means no request.
constexpr int waves_hint(int wg, int s, bool plain) { return plain && wg == 256 && s == 7 ? 5 : 1; }

// Per-workgroup constants of one fill: table views, the fast-path table
// (X_i 2^-53 as double for FP64, RN32(X_i) 2^-24/2^-23 as float for FP32),
// the Philox key and the location-scale pair.
struct FillCtx {
  dev::TabView own, ex;
  dev::TradView tr, trex;  // the traditional sampler's tables (own in LDS)
  const void* fast;
  uint32_t k0, k1;
  double scale, shift;
};

// LDS a tile works in: the staging tile (16 bytes per Philox block), the
// slow-output bitmap and its prefix sums.
struct TileLds {
  void* stage;
  uint64_t* slowmap;
  uint32_t* prefix;
  uint16_t* list;   // LIST kernels only
  uint32_t* marks;  // MARKS kernels only
};

template <uint32_t DIST, uint32_t DT, int WG, int S, uint32_t CAP = kLdsLayers, bool SLOWLDS = (CAP <= kLdsLayers),
          bool LIST = false>
__device__ __forceinline__ FillCtx load_tables(const FillArgs& a, FillLds<DT, WG, S, CAP, SLOWLDS, false, LIST>& sh) {
  const DevTable* tb = a.tab;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < CAP; i += WG) {
    if constexpr (DT == kF64)
      sh.xs[i] = tb->XS[i];
    else
      sh.xs[i] = tb->XS32[i];
  }
  FillCtx c;
  c.own = dev::global_view(tb);
  if constexpr (SLOWLDS) {
    for (uint32_t i = tid; i < CAP; i += WG) {
      sh.T[i] = tb->TA[i];
    }
    for (uint32_t i = tid; i <= CAP; i += WG) {
      sh.X[i] = tb->X[i];
      sh.f[i] = tb->f[i];
    }
    c.own.X = sh.X;
    c.own.f = sh.f;
    c.own.TA = sh.T;
  }
  if constexpr (DT == kF64) c.own.XS = sh.xs;
  c.fast = sh.xs;
  c.ex = dev::global_view(a.etab);
  c.k0 = (uint32_t)a.seed;
  c.k1 = (uint32_t)(a.seed >> 32);
  c.scale = a.scale;
  c.shift = a.shift;
  return c;
}

// The traditional sampler's context (FP64): widths W_i 2^-53 in the fast
// table, quick-accept thresholds and layer heights in LDS, the exponential
// tables of the normal tail read from device memory.
template <uint32_t DIST, int WG, int S, bool SLOWLDS>
__device__ __forceinline__ FillCtx load_trad_tables(const FillArgs& a,
                                                    FillLds<kF64, WG, S, kLdsLayers, SLOWLDS, true>& sh) {
  const DevTrad* tb = a.ttab;
  for (uint32_t i = threadIdx.x; i < kLdsLayers; i += WG) {
    sh.xs[i] = tb->WS[i];
    sh.T[i] = tb->KQ[i];
    sh.f[i] = tb->f[i];
  }
  FillCtx c = {};
  c.tr = dev::trad_view(tb);
  c.tr.WS = sh.xs;
  c.tr.KQ = sh.T;
  c.tr.f = sh.f;
  c.trex = dev::trad_view(a.tetab);
  c.fast = sh.xs;
  c.k0 = (uint32_t)a.seed;
  c.k1 = (uint32_t)(a.seed >> 32);
  c.scale = a.scale;
  c.shift = a.shift;
  return c;
}

// One tile (tile index t of this launch).  Ends with the staging tile
// written out.  A lane's phase C reads only staging places it wrote in
// phase A, so consecutive tiles need no barrier between them.
//
// With TRAD set (FP64 only) the sampler is the traditional ziggurat: the
// fast word quick-accepts when its magnitude bits lie below the layer's
// threshold, and phase B runs the traditional slow path from that word.
//
// WIDE marks tables of more than 256 layers: a 32-bit word then gives
// s = b > 8 low bits to the index, so its magnitude starts at bit s (the
// normal's sign sits at bit s); otherwise s = 8.
//
// With LIST set, wave 0 also writes the staging places of a tile's slow
// outputs, in entry order, to sh.list when there are at most kListCap of
// them.  With MARKS set instead, when there are at most 64 (all in wave
// 0's drain), sh.marks[e] gives entry e's bitmap word and that word's
// first entry, so a drain lane reads them with one load instead of a
// binary search over the prefix sums.
template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE, bool ACCEL = false, bool TRAD = false,
          bool WIDE = false, bool LIST = false, bool MARKS = false, bool FRESH = false>
__device__ __forceinline__ void fill_tile(const FillArgs& a, const FillCtx& c, const TileLds& sh, uint32_t t) {
  using Sh = FillShape<DT, WG, S>;
  using OutT = typename Sh::OutT;
  using VecT = typename Sh::VecT;
  constexpr int O = Sh::O;
  constexpr int NWAVE = Sh::NWAVE;
  constexpr int NWORD = Sh::NWORD;
  constexpr int TILE = Sh::TILE;
  static_assert(!TRAD || (DT == kF64 && !TRACE && !ACCEL), "traditional sampler: plain FP64 fills");

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t wave = tid >> 6;
  const uint32_t L = TRAD ? 0u : c.own.L;
  const uint32_t imask = TRAD ? c.tr.imask : c.own.imask;
  const uint32_t s32 = WIDE ? (c.own.b > 8u ? c.own.b : 8u) : 8u;
  const float fscale = (float)c.scale;
  // the location sits in VGPRs for the whole tile: a VALU fma takes only
  // one scalar operand, and rematerialising it cost a move per output
  double shiftv = c.shift;
  float fshift = (float)c.shift;
  if constexpr (DIST == kDistNormal) asm volatile("" : "+v"(shiftv), "+v"(fshift));
  OutT* const out = static_cast<OutT*>(a.out);
  VecT* const stage = static_cast<VecT*>(sh.stage);
  OutT* const stage_s = static_cast<OutT*>(sh.stage);
  const OutT* const xs = static_cast<const OutT*>(c.fast);

  const uint64_t tile0 = a.blk0 + (uint64_t)t * TILE;
  const bool interior = a.has_full && tile0 >= a.full_lo && tile0 + (TILE - 1) <= a.full_hi;

  // this wave's first bitmap word, as an LDS address
  const uint32_t lds_word = dev::lds_address(sh.slowmap + wave);
  // A: fast path into the staging tile, slow outputs into the bitmap
  auto phase_a = [&](auto interior_tag) {
    constexpr bool IN = decltype(interior_tag)::value;
    // FRESH: the slices' block offsets are formed per tile.  Hoisted out
    // of the persistent loop they hold S register pairs, which left the
    // normal fill kernels at their register limit with a scratch spill
    // whose reloads missed L2; the batch kernel, held at 3 waves per SIMD
    // by its LDS, is faster with them hoisted.
    uint32_t tid_a = tid;
    if constexpr (FRESH) asm volatile("" : "+v"(tid_a));
    (void)tid_a;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t m =
          FRESH ? tile0 + (uint64_t)((uint32_t)(s * WG) + tid_a) : tile0 + (uint64_t)(s * WG) + tid;
      uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = (DT == kF64) ? 0u : 1u;
      dev::philox10(c0, c1, c2, c3, c.k0, c.k1);
      OutT v[O];
#pragma unroll
      for (int o = 0; o < O; ++o) {
        const uint64_t g = m * O + o;
        bool live = true;
        if constexpr (!IN) live = (m <= a.blk_last) && (g >= a.first) && (g <= a.last);
        uint32_t i;
        OutT x;
        bool miss;  // the fast word does not decide the output
        if constexpr (DT == kF64) {
          const uint32_t lo = (o == 0) ? c0 : c2, hi = (o == 0) ? c1 : c3;
          i = lo & imask;
          // the 53 magnitude bits k = hi 2^21 + (lo >> 11), converted
          // exactly (k < 2^53) by one fma of the two 32-bit conversions
          const double k = __builtin_fma((double)hi, 0x1p21, (double)(lo >> 11));
          x = k * xs[i];
          if constexpr (TRAD)
            miss = (((uint64_t)hi << 21) | (lo >> 11)) >= c.tr.KQ[i];
          else
            miss = i >= L;
          if constexpr (DIST == kDistNormal) x = dev::with_sign_of(x, lo << 21);
        } else {
          const uint32_t w = (o == 0) ? c0 : (o == 1) ? c1 : (o == 2) ? c2 : c3;
          i = w & imask;
          miss = i >= L;
          if constexpr (DIST == kDistExp) {
            x = (float)(w >> s32) * xs[i];
          } else {
            x = (float)(w >> (s32 + 1u)) * xs[i];
            x = dev::with_sign_of(x, w << (31u - s32));
          }
        }
        // a slow output's value here is a placeholder that phase B replaces;
        // for the exponential the shift is +0 and x >= 0, where
        // fma(scale, x, +0) is the rounded product
        const bool slow = live && miss;
        if constexpr (DIST == kDistExp) {
          if constexpr (DT == kF64)
            v[o] = c.scale * x;
          else
            v[o] = fscale * x;
        } else {
          if constexpr (DT == kF64)
            v[o] = __builtin_fma(c.scale, x, shiftv);
          else
            v[o] = __builtin_fmaf(fscale, x, fshift);
        }
        const uint64_t mask = __builtin_amdgcn_ballot_w64(slow);
        // the normal kernels run out of scalar registers, and the
        // compiler's lane-0 store then reloads its exec mask per output
        if constexpr (DIST == kDistNormal)
          dev::store_from_lane0(lds_word, mask, (s * O + o) * NWAVE * 8);
        else if (lane == 0)
          sh.slowmap[(s * O + o) * NWAVE + wave] = mask;
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
      VecT vv;
      if constexpr (DT == kF64) {
        vv.x = v[0];
        vv.y = v[1];
      } else {
        vv.x = v[0];
        vv.y = v[1];
        vv.z = v[2];
        vv.w = v[3];
      }
      stage[s * WG + tid] = vv;
    }
  };
  if (interior)
    phase_a(std::true_type());
  else
    phase_a(std::false_type());
  __syncthreads();

  // B: number the slow outputs (exclusive prefix over the bitmap words, by
  // wave 0) and share them out over every lane.  This is the tile's
  // critical path, run by one wave while the others wait: it takes issue
  // priority over the other workgroups' waves on its SIMD until the drain
  // ends.
  __builtin_amdgcn_s_setprio(2);
  if (wave == 0) {
    constexpr int PER = (NWORD + 63) / 64;
    uint32_t cnt[PER];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int w = lane * PER + k;
      cnt[k] = (w < NWORD) ? (uint32_t)__popcll(sh.slowmap[w]) : 0u;
      mine += cnt[k];
    }
    const uint32_t incl = dev::wave_inclusive_sum(mine);
    uint32_t run = incl - mine;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int w = lane * PER + k;
      if (w < NWORD) sh.prefix[w] = run;
      run += cnt[k];
    }
    if (lane == 63) sh.prefix[NWORD] = incl;
    if constexpr (MARKS) {
      // mark each word's first entry with (word + 1, entry) and carry the
      // marks to the word's later entries by a prefix maximum
      // (the lanes of wave 0 exchange the marks through LDS: volatile keeps
      // the compiler from taking a lane's own earlier store for the value
      // another lane wrote; LDS accesses of one wave complete in order)
      if ((uint32_t)__builtin_amdgcn_readlane((int)incl, 63) <= 64u) {
        typedef __attribute__((address_space(3))) volatile uint32_t LdsWord;
        LdsWord* const mk = (LdsWord*)sh.marks;
        mk[lane] = 0u;
        uint32_t pos = incl - mine;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int w = lane * PER + k;
          if (w < NWORD && cnt[k] > 0u) mk[pos] = ((uint32_t)(w + 1) << 8) | pos;
          pos += cnt[k];
        }
        const uint32_t here = mk[lane];
        mk[lane] = dev::wave_inclusive_max(here);
      }
    }
    if constexpr (LIST) {
      // each lane lists the set bits of its words, from its prefix on
      if (__shfl(incl, 63) <= kListCap) {
        uint32_t pos = incl - mine;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int w = lane * PER + k;
          uint64_t bits = (w < NWORD) ? sh.slowmap[w] : 0ull;
          const uint32_t so = (uint32_t)w / NWAVE, wv = (uint32_t)w % NWAVE;
          const uint32_t base = ((so / O) * WG + wv * 64) * O + so % O;
          while (bits) {
            const uint32_t ln = (uint32_t)__ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            sh.list[pos++] = (uint16_t)(base + ln * O);
          }
        }
      }
    }
  }
  __syncthreads();
  const uint32_t total = sh.prefix[NWORD];
  for (uint32_t e = tid; e < total; e += WG) {
    uint32_t blk, o;
    if (LIST && total <= kListCap) {
      const uint32_t pl = sh.list[e];
      blk = pl / O;
      o = pl % O;
    } else {
      // the word holding entry e: prefix[lo] <= e < prefix[lo + 1]
      uint32_t lo = 0, first;
      if (MARKS && total <= 64u) {
        const uint32_t m = sh.marks[e];
        lo = (m >> 8) - 1u;
        first = m & 255u;
      } else {
        uint32_t hi = NWORD;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (sh.prefix[mid] <= e)
            lo = mid;
          else
            hi = mid;
        }
        first = sh.prefix[lo];
      }
      uint64_t bits = sh.slowmap[lo];
      for (uint32_t r = e - first; r > 0; --r) bits &= bits - 1;
      const uint32_t ln = (uint32_t)__ffsll((unsigned long long)bits) - 1;
      const uint32_t so = lo / NWAVE, wv = lo % NWAVE;
      o = so % O;
      blk = (so / O) * WG + wv * 64 + ln;
    }
    const uint64_t g = (tile0 + blk) * O + o;
    OutT* place = stage_s + blk * O + o;
    bool neg = false;
    int32_t region = -1;
    uint32_t words, tests;
    double mag;
    if constexpr (TRAD) {
      mag = dev::trad_slow<DIST>(c.tr, c.trex, g, c.k0, c.k1, neg, words, tests);
    } else {
      if constexpr (DIST == kDistNormal) {
        // the placeholder is +-inf with the output's sign, or NaN when
        // its magnitude bits were all zero (then the fast block is redone)
        const OutT ph = *place;
        if (__builtin_isnan(ph))
          neg = dev::normal_sign<DT>(g, c.k0, c.k1, s32);
        else
          neg = __builtin_signbit(ph);
      }
      mag = dev::slow_magnitude<DIST, ACCEL>(c.own, c.ex, g, c.k0, c.k1, region, words, tests);
    }
    OutT x = (OutT)mag;
    if (neg) x = -x;
    if constexpr (DIST == kDistExp) {
      if constexpr (DT == kF64)
        *place = c.scale * x;
      else
        *place = fscale * x;
    } else {
      if constexpr (DT == kF64)
        *place = __builtin_fma(c.scale, x, c.shift);
      else
        *place = __builtin_fmaf(fscale, x, fshift);
    }
    if constexpr (TRACE) {
      const uint64_t k = g - a.first;
      if (a.t_region) a.t_region[k] = region;
      if (a.t_words) a.t_words[k] = words;
      if (a.t_tests) a.t_tests[k] = tests;
    }
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  // C: staging tile to HBM.  An interior tile with 16-byte aligned blocks
  // (the common case) stores from one uniform base pointer at lane offsets.
  if (interior && a.aligned16) {
    VecT* const dst = reinterpret_cast<VecT*>(out + (tile0 * O - a.first));
    // formed per tile, so the compiler does not keep one offset register
    // per slice alive across the whole persistent loop
    uint32_t lane_blk = tid;
    asm volatile("" : "+v"(lane_blk));
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s * WG + lane_blk] = stage[s * WG + tid];
    return;
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const uint64_t m = tile0 + (uint64_t)(s * WG) + tid;
    const uint64_t g0 = m * O;
    const VecT vv = stage[s * WG + tid];
    if (interior || (m <= a.blk_last && g0 >= a.first && g0 + (O - 1) <= a.last)) {
      if (a.aligned16) {
        *reinterpret_cast<VecT*>(out + (g0 - a.first)) = vv;
      } else {
        const OutT* pv = reinterpret_cast<const OutT*>(&vv);
#pragma unroll
        for (int o = 0; o < O; ++o) out[g0 + o - a.first] = pv[o];
      }
    } else if (m <= a.blk_last) {
      const OutT* pv = reinterpret_cast<const OutT*>(&vv);
#pragma unroll
      for (int o = 0; o < O; ++o) {
        const uint64_t g = g0 + o;
        if (g >= a.first && g <= a.last) out[g - a.first] = pv[o];
      }
    }
  }
}

// Persistent workgroups.  A large fill gives them chunks of `a.chunk`
// consecutive tiles per atomic step of its counter pair (one atomic per
// tile would serialise the device on that address), so the tiles in flight
// stay a window that sweeps through the output in address order and fast
// workgroups take more; the last workgroup to leave resets the pair.  A
// small fill (no counters) deals the tiles out round robin.
template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE, bool ACCEL = false, bool TRAD = false,
          bool WIDE = false>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(waves_hint(WG, S, !TRAD && !WIDE))))
fill_kernel(FillArgs a) {
  static_assert(!(WIDE && (TRAD || ACCEL)), "wide tables: the plain modified sampler");
  constexpr uint32_t CAP = WIDE ? kMaxLayers : kLdsLayers;
  constexpr bool SLOWLDS = !WIDE && !lean_shape(WG, S);
  // the slow-output list pays for the exponential (2^30 FP64: 1.57 ->
  // 1.53 ms) and, since the slice offsets stopped holding registers
  // across tiles, for the normal's large tiles (256 x 7: 0.3 % FP64, 0.6 %
  // FP32); in its smaller shapes the list's two registers cross a
  // register granule (6 -> 5 waves per SIMD; 512 x 4 at 2^30 FP64 went
  // from 1.97 to 2.65 ms), so those keep the entry marks
  constexpr bool LIST = !TRAD && !WIDE && (DIST == kDistExp || S >= 7);
  __shared__ FillLds<DT, WG, S, CAP, SLOWLDS, TRAD, LIST> sh;
  const FillCtx c = [&] {
    if constexpr (TRAD)
      return load_trad_tables<DIST, WG, S, SLOWLDS>(a, sh);
    else
      return load_tables<DIST, DT, WG, S, CAP, SLOWLDS, LIST>(a, sh);
  }();
  TileLds tl;
  tl.stage = sh.stage;
  tl.slowmap = sh.slowmap;
  tl.prefix = sh.prefix;
  tl.list = sh.list;
  tl.marks = sh.marks;
  // Tile schedule: with counters, chunks of a.chunk tiles taken from
  // counters[0]; without, workgroup w takes tiles w, w + G, ...
  const bool dynamic = a.counters != nullptr;
  uint64_t next = blockIdx.x;
  if (!dynamic) __syncthreads();  // the tables in LDS are complete
  for (;;) {
    uint64_t t0, t1;
    if (dynamic) {
      if (threadIdx.x == 0) sh.tile = atomicAdd(&a.counters[0], 1u);
      __syncthreads();
      t0 = (uint64_t)sh.tile * a.chunk;
      t1 = t0 + a.chunk < a.tiles ? t0 + a.chunk : a.tiles;
    } else {
      t0 = next;
      t1 = next + 1;
      next += gridDim.x;
    }
    if (t0 >= a.tiles) break;
    // No barrier between tiles: in phase C a lane reads only the staging
    // places it wrote itself in phase A, and the bitmap, prefix sums and
    // list are last read before the barrier that ends the drain, so the
    // next tile's phase A overwrites nothing another wave still reads.
    for (uint64_t t = t0; t < t1; ++t)
      fill_tile<DIST, DT, WG, S, TRACE, ACCEL, TRAD, WIDE, LIST, !LIST, true>(a, c, tl, (uint32_t)t);
  }
  // the last workgroup to leave resets the counters for the slot's next user
  if (dynamic && threadIdx.x == 0) {
    if (atomicAdd(&a.counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&a.counters[0], 0u);
      atomicExch(&a.counters[1], 0u);
    }
  }
}

// Workgroups of one kernel variant resident on the whole device.
template <class K>
int resident_groups(K kernel, int wg, size_t lds, int* out) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t, int>, int> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  const auto key = std::make_tuple((const void*)kernel, wg, lds, dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return 0;
  }
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, wg, lds);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  if (per_cu < 1) return (int)hipErrorInvalidConfiguration;
  *out = per_cu * cus;
  cache[key] = *out;
  return 0;
}

// Launch of one fill-kernel variant: as many persistent workgroups as are
// resident on the device, fewer when the launch has fewer counter steps.
template <uint32_t DIST, uint32_t DT, int WG, int S, bool TRACE, bool ACCEL = false, bool TRAD = false,
          bool WIDE = false>
int launch_one(const FillArgs& args, hipStream_t st) {
  auto kernel = fill_kernel<DIST, DT, WG, S, TRACE, ACCEL, TRAD, WIDE>;
  int groups = 0;
  int e = resident_groups(kernel, WG, 0, &groups);
  if (e != 0) return e;
  FillArgs a = args;
  if (a.counters == nullptr) {
    const uint32_t grid = a.tiles < (uint64_t)groups ? a.tiles : (uint32_t)groups;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(WG), 0, st, a);
    return (int)hipGetLastError();
  }
  // tiles per counter step: as asked, but small enough that every resident
  // workgroup gets a couple of steps
  uint64_t chunk = a.tiles / (2ull * (uint64_t)groups);
  if (chunk > a.chunk) chunk = a.chunk;
  if (chunk < 1) chunk = 1;
  a.chunk = (uint32_t)chunk;
  const uint64_t steps = (a.tiles + chunk - 1) / chunk;
  const uint32_t grid = steps < (uint64_t)groups ? (uint32_t)steps : (uint32_t)groups;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(WG), 0, st, a);
  return (int)hipGetLastError();
}

// Launch of the variant with workgroup size wg and spl blocks per lane:
// every power-of-two shape of up to 2048 blocks per tile plus 256 x 7
// (1792 blocks, 5 waves per SIMD) and 256 x 10 (2560 blocks, about 60 slow
// normal outputs: one full wave for the drain) for plain fills, three
// shapes for the trace build.
template <uint32_t DIST, uint32_t DT, bool TRACE, bool ACCEL = false, bool TRAD = false, bool WIDE = false>
int launch_shape(uint32_t wg, uint32_t spl, const FillArgs& a, hipStream_t st) {
#define ZIG_SHAPE(W, S_) \
  if (wg == W && spl == S_) return launch_one<DIST, DT, W, S_, TRACE, ACCEL, TRAD, WIDE>(a, st);
  if constexpr (!TRACE) {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(64, 2) ZIG_SHAPE(64, 4) ZIG_SHAPE(64, 8)
    ZIG_SHAPE(128, 1) ZIG_SHAPE(128, 2) ZIG_SHAPE(128, 4) ZIG_SHAPE(128, 8)
    ZIG_SHAPE(256, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4) ZIG_SHAPE(256, 7) ZIG_SHAPE(256, 8) ZIG_SHAPE(256, 10)
    ZIG_SHAPE(512, 1) ZIG_SHAPE(512, 2) ZIG_SHAPE(512, 4)
    ZIG_SHAPE(1024, 1) ZIG_SHAPE(1024, 2)
  } else {
    ZIG_SHAPE(64, 1) ZIG_SHAPE(256, 2) ZIG_SHAPE(256, 4)
  }
#undef ZIG_SHAPE
  return (int)hipErrorInvalidConfiguration;
}

}  // namespace zig
