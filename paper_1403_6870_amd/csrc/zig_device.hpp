// Device-side pieces of the modified ziggurat sampler for gfx950: the
// Philox4x32-10 uniform source, the per-output slow stream, the alias draw
// and the rejection/tail paths.  The fast path lives in the kernels.
//
// The slow paths read their tables through a TabView, a set of pointers
// that the kernels aim at LDS copies (the hot region, box and alias tables)
// or at the device tables (the rarely used ones); every function here is
// inlined so the compiler sees which address space each pointer lives in.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "zig_internal.hpp"

namespace zig {
namespace dev {

constexpr uint64_t kOne53 = 1ull << 53;

// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32->64 products,
// the high halves folded into the other pair of words with the round key;
// the key is bumped by the Weyl constants between rounds.  The key is the
// same for every lane, so its schedule stays in scalar registers.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input xor in one v_bitop3_b32 (truth table 0x96)
    const uint32_t a = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t b = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = a;
    c2 = b;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Word t of the slow stream of output g comes from the block with counter
// (g lo, g hi, t >> 1, 2): words 0|1 for even t, 2|3 for odd t.  One block
// serves two consecutive words.
struct SlowStream {
  uint32_t g0, g1, k0, k1;
  uint32_t t;
  uint32_t spare_lo, spare_hi;

  __device__ __forceinline__ SlowStream(uint64_t g, uint32_t key0, uint32_t key1)
      : g0((uint32_t)g), g1((uint32_t)(g >> 32)), k0(key0), k1(key1), t(0), spare_lo(0), spare_hi(0) {}

  __device__ __forceinline__ uint64_t next() {
    uint64_t w;
    if ((t & 1u) == 0) {
      uint32_t c0 = g0, c1 = g1, c2 = t >> 1, c3 = 2u;
      philox10(c0, c1, c2, c3, k0, k1);
      w = (uint64_t)c0 | ((uint64_t)c1 << 32);
      spare_lo = c2;
      spare_hi = c3;
    } else {
      w = (uint64_t)spare_lo | ((uint64_t)spare_hi << 32);
    }
    ++t;
    return w;
  }
};

// Tables of one distribution as the slow paths read them.  X[L] = 0 and
// f[L] = 1; box j spans [X[j], X[j-1]] x [f[j-1], f[j]], its width and
// height being the same double subtractions the table builder defines.
struct TabView {
  const double* X;
  const double* f;
  const uint64_t* TA;  // alias columns: threshold above the low b bits, alias in them
  const double* XS;
  uint32_t L, imask, b;
  uint64_t keps;
  uint64_t kcvx, kccv;  // normal: chord-band thresholds of the accelerated variant
  const uint64_t* sqlo;  // normal: per-box squeeze of the plain box test
  const uint64_t* sqhi;
  double X0, invX0;
};

__device__ __forceinline__ TabView global_view(const DevTable* t) {
  TabView v;
  v.X = t->X;
  v.f = t->f;
  v.TA = t->TA;
  v.XS = t->XS;
  v.L = t->L;
  v.imask = t->i_max - 1;
  v.b = t->b;
  v.keps = t->K_eps;
  v.kcvx = t->K_cvx;
  v.kccv = t->K_ccv;
  v.sqlo = t->SQlo;
  v.sqhi = t->SQhi;
  v.X0 = t->X0;
  v.invX0 = t->invX0;
  return v;
}

// Region draw: column c from the low b bits, compare the high 64-b bits
// with the column threshold, else take the column's alias; threshold and
// alias come in one word.
__device__ __forceinline__ uint32_t alias_region(const TabView& v, uint64_t r) {
  const uint32_t c = (uint32_t)r & v.imask;
  const uint64_t e = v.TA[c];
  return (r >> v.b) < (e >> v.b) ? c : (uint32_t)e & v.imask;
}

__device__ __forceinline__ double lattice53(uint64_t k) { return (double)k * 0x1p-53; }

// Exponential draw after its fast word failed (layer index >= L): region j
// from the alias table; the tail (j = 0) is X_0 plus a fresh exponential,
// whose own fast word is the next slow word (tail nesting adds X_0 once per
// level, innermost first); a box is sampled by reflection across the chord,
// the eps band shortcut and the exact test, retrying in the same box.
// `first_region` receives the first j drawn, `tests` counts exp() calls.
__device__ __forceinline__ double exp_slow(const TabView& E, SlowStream& s, int32_t& first_region, uint32_t& tests) {
  uint32_t nest = 0;
  double y = 0.0;
  bool first = true;
  for (;;) {
    const uint32_t j = alias_region(E, s.next());
    if (first) {
      first_region = (int32_t)j;
      first = false;
    }
    if (j == 0) {
      ++nest;
      const uint64_t w = s.next();
      const uint32_t i = (uint32_t)w & E.imask;
      if (i < E.L) {
        y = (double)(w >> 11) * E.XS[i];
        break;
      }
      continue;
    }
    const double left = E.X[j], right = E.X[j - 1];
    const double base = E.f[j - 1], top = E.f[j];
    const double width = right - left, height = top - base;
    for (;;) {
      uint64_t k1 = s.next() >> 11;
      uint64_t k2 = s.next() >> 11;
      if (k1 + k2 > kOne53) {
        const uint64_t r1 = kOne53 - k2;
        k2 = kOne53 - k1;
        k1 = r1;
      }
      const double x = __builtin_fma(lattice53(k1), width, left);
      if (k1 + k2 <= E.keps) {
        y = x;
        break;
      }
      const double yy = __builtin_fma(lattice53(k2), height, base);
      ++tests;
      if (yy < exp(-x)) {
        y = x;
        break;
      }
    }
    break;
  }
  for (uint32_t c = 0; c < nest; ++c) y = E.X0 + y;
  return y;
}

// The whole exponential sampler started from fast word w.
__device__ __forceinline__ double exp_from_word(const TabView& E, uint64_t w, SlowStream& s, uint32_t& tests) {
  const uint32_t i = (uint32_t)w & E.imask;
  if (i < E.L) return (double)(w >> 11) * E.XS[i];
  int32_t unused;
  return exp_slow(E, s, unused, tests);
}

// Normal magnitude after its fast word failed: region j; the tail uses
// Marsaglia's method with two exponential draws E1, E2 (t = E1 / X_0,
// accept when 2 E2 > t^2, return X_0 + t); a box is sampled by plain
// rejection against e^{-x^2/2}, retrying in the same box.
template <bool ACCEL>
__device__ __forceinline__ double normal_slow(const TabView& N, const TabView& E, SlowStream& s,
                                              int32_t& first_region, uint32_t& tests) {
  const uint32_t j = alias_region(N, s.next());
  first_region = (int32_t)j;
  if (j == 0) {
    for (;;) {
      const double e1 = exp_from_word(E, s.next(), s, tests);
      const double e2 = exp_from_word(E, s.next(), s, tests);
      const double t = e1 * N.invX0;
      if (e2 + e2 > t * t) return N.X0 + t;
    }
  }
  const double left = N.X[j], right = N.X[j - 1];
  const double base = N.f[j - 1], top = N.f[j];
  const double width = right - left, height = top - base;
  if constexpr (!ACCEL) {
    // plain rejection; the squeeze decides most points as the density
    // test would, so e^{-x^2/2} is evaluated only near the curve (tests
    // counts every decision)
    const uint64_t sq_lo = N.sqlo[j], sq_hi = N.sqhi[j];
    for (;;) {
      const uint64_t k1 = s.next() >> 11;
      const uint64_t k2 = s.next() >> 11;
      const double x = __builtin_fma(lattice53(k1), width, left);
      ++tests;
      const uint64_t sum = k1 + k2;
      if (sum < sq_lo) return x;
      if (sum >= sq_hi) continue;
      const double yy = __builtin_fma(lattice53(k2), height, base);
      if (yy < exp(-0.5 * (x * x))) return x;
    }
  }
  // accelerated variant: convex boxes (right of the inflection point, curve
  // below the chord) reflect points above the chord and accept below the
  // eps band; concave boxes (left of it, the cap included) accept below the
  // chord and reject above the delta band; the box straddling the
  // inflection point keeps plain rejection
  const uint32_t kind = left >= 1.0 ? 1u : right <= 1.0 ? 2u : 0u;
  for (;;) {
    uint64_t k1 = s.next() >> 11;
    uint64_t k2 = s.next() >> 11;
    if (kind == 1u && k1 + k2 > kOne53) {
      const uint64_t r1 = kOne53 - k2;
      k2 = kOne53 - k1;
      k1 = r1;
    }
    const double x = __builtin_fma(lattice53(k1), width, left);
    if (kind == 1u && k1 + k2 <= N.kcvx) return x;
    if (kind == 2u) {
      if (k1 + k2 <= kOne53) return x;
      if (k1 + k2 > N.kccv) continue;
    }
    const double yy = __builtin_fma(lattice53(k2), height, base);
    ++tests;
    if (yy < exp(-0.5 * (x * x))) return x;
  }
}

// Magnitude of output g on its slow path.  `own` is the distribution's
// table view, `ex` the exponential one (the normal tail).
template <uint32_t DIST, bool ACCEL = false>
__device__ __forceinline__ double slow_magnitude(const TabView& own, const TabView& ex, uint64_t g, uint32_t k0,
                                                 uint32_t k1, int32_t& region, uint32_t& words, uint32_t& tests) {
  SlowStream s(g, k0, k1);
  tests = 0;
  double m;
  if constexpr (DIST == kDistExp)
    m = exp_slow(own, s, region, tests);
  else
    m = normal_slow<ACCEL>(own, ex, s, region, tests);
  words = s.t;
  return m;
}

// Sign of normal output g (FP64: bit 10 of its fast word; FP32: bit s32,
// 8 unless the table has more than 256 layers), recomputed from its fast
// block for the rare outputs on the slow path.
template <uint32_t DT>
__device__ __forceinline__ bool normal_sign(uint64_t g, uint32_t k0, uint32_t k1, uint32_t s32) {
  if constexpr (DT == kF64) {
    const uint64_t m = g >> 1;
    uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = 0u;
    philox10(c0, c1, c2, c3, k0, k1);
    const uint32_t lo = (g & 1) ? c2 : c0;
    return (lo >> 10) & 1u;
  } else {
    const uint64_t m = g >> 2;
    uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = 1u;
    philox10(c0, c1, c2, c3, k0, k1);
    const uint32_t r = g & 3;
    const uint32_t w = r == 0 ? c0 : r == 1 ? c1 : r == 2 ? c2 : c3;
    return (w >> s32) & 1u;
  }
}

// ---- the traditional ziggurat (Table 1, right column), for comparison --

// Its tables as the slow path reads them: layer widths W_i 2^-53, the
// quick-accept thresholds on the 53 magnitude bits, the layer heights.
struct TradView {
  const double* WS;
  const uint64_t* KQ;
  const double* f;
  uint32_t imask;
  double r, invr;
};

__device__ __forceinline__ TradView trad_view(const DevTrad* t) {
  TradView v;
  v.WS = t->WS;
  v.KQ = t->KQ;
  v.f = t->f;
  v.imask = t->n - 1;
  v.r = t->r;
  v.invr = t->invr;
  return v;
}

// Traditional exponential from the word w: layer i from its low bits, the
// 53 magnitude bits k from bits 11..63, x = k W_i 2^-53.  Quick accept when
// k < KQ[i]; layer 0 beyond X_0 is the tail, X_0 plus a fresh traditional
// exponential (nesting added innermost first); any other layer tests
// f_{i-1} + U2 (f_i - f_{i-1}) < e^-x with U2 from the slow stream and on
// rejection starts over from a fresh word.
__device__ __forceinline__ double trad_exp(const TradView& E, uint64_t w, SlowStream& s, uint32_t& tests) {
  uint32_t nest = 0;
  double x;
  for (;;) {
    const uint32_t i = (uint32_t)w & E.imask;
    const uint64_t k = w >> 11;
    x = (double)k * E.WS[i];
    if (k < E.KQ[i]) break;
    if (i == 0) {
      ++nest;
      w = s.next();
      continue;
    }
    const double lo = E.f[i - 1];
    const double y = __builtin_fma(lattice53(s.next() >> 11), E.f[i] - lo, lo);
    ++tests;
    if (y < exp(-x)) break;
    w = s.next();
  }
  for (uint32_t c = 0; c < nest; ++c) x = E.r + x;
  return x;
}

// Traditional normal magnitude from the word w; the tail beyond X_0 = r
// uses Marsaglia's method on two traditional exponentials.
__device__ __forceinline__ double trad_normal(const TradView& N, const TradView& E, uint64_t w, SlowStream& s,
                                              uint32_t& tests) {
  for (;;) {
    const uint32_t i = (uint32_t)w & N.imask;
    const uint64_t k = w >> 11;
    const double x = (double)k * N.WS[i];
    if (k < N.KQ[i]) return x;
    if (i == 0) {
      for (;;) {
        const double e1 = trad_exp(E, s.next(), s, tests);
        const double e2 = trad_exp(E, s.next(), s, tests);
        const double t = e1 * N.invr;
        if (e2 + e2 > t * t) return N.r + t;
      }
    }
    const double lo = N.f[i - 1];
    const double y = __builtin_fma(lattice53(s.next() >> 11), N.f[i] - lo, lo);
    ++tests;
    if (y < exp(-0.5 * (x * x))) return x;
    w = s.next();
  }
}

// Output g (FP64) of the traditional sampler after its first word missed
// the quick test: the word is recomputed from the fast block (it also
// holds the normal sign, bit 10) and the sampler runs from it.
template <uint32_t DIST>
__device__ __forceinline__ double trad_slow(const TradView& own, const TradView& ex, uint64_t g, uint32_t k0,
                                            uint32_t k1, bool& neg, uint32_t& words, uint32_t& tests) {
  const uint64_t m = g >> 1;
  uint32_t c0 = (uint32_t)m, c1 = (uint32_t)(m >> 32), c2 = 0u, c3 = 0u;
  philox10(c0, c1, c2, c3, k0, k1);
  const uint64_t w = (g & 1) ? ((uint64_t)c2 | ((uint64_t)c3 << 32)) : ((uint64_t)c0 | ((uint64_t)c1 << 32));
  SlowStream s(g, k0, k1);
  tests = 0;
  double x;
  if constexpr (DIST == kDistExp) {
    neg = false;
    x = trad_exp(own, w, s, tests);
  } else {
    neg = (w >> 10) & 1u;
    x = trad_normal(own, ex, w, s, tests);
  }
  words = s.t;
  return x;
}

// -x when bit 31 of `bit` is set, else x: the bit xored into the sign
// (one three-input bitop, truth table of S0 ^ (S1 & S2), instead of a
// compare and select); -0.0 for x = +0.0, as negation gives.
__device__ __forceinline__ double with_sign_of(double x, uint32_t bit) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), bit, 0x80000000u, 0x78);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint32_t)b);
}
__device__ __forceinline__ float with_sign_of(float x, uint32_t bit) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  return __builtin_bit_cast(float, __builtin_amdgcn_bitop3_b32(b, bit, 0x80000000u, 0x78));
}

// Byte address in LDS of a pointer into shared memory.
template <class T>
__device__ __forceinline__ uint32_t lds_address(T* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) T*)p;
}

// Stores the wave-uniform v (a scalar register pair, such as a ballot) at
// LDS address addr + off from lane 0 alone: exec is set to that lane, v is
// moved into its vector registers and stored, and exec is restored, all in
// one block.  addr must hold the address in lane 0 (computed in uniform
// code); off must fold to a constant.  Written out because the compiler
// otherwise keeps a lane-0 exec mask for the whole kernel and, short of
// scalar registers, reloads it from a vector register twice per store.
__device__ __forceinline__ void store_from_lane0(uint32_t addr, uint64_t v, int off) {
  uint64_t saved, vd;
  asm volatile(
      "s_mov_b64 %0, exec\n\t"
      "s_mov_b64 exec, 1\n\t"
      "v_mov_b64 %1, %3\n\t"
      "ds_write_b64 %2, %1 offset:%4\n\t"
      "s_mov_b64 exec, %0"
      : "=&s"(saved), "=&v"(vd)
      : "v"(addr), "s"(v), "i"(off)
      : "memory");
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active): a
// Hillis-Steele scan inside each row of 16 lanes by DPP row shifts of 1, 2,
// 4 and 8 (lanes shifted in from outside the row read 0), then the totals
// of the rows below, read from lanes 15, 31 and 47.  No LDS round trips,
// which a shuffle-based scan pays six times in a row.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
  const uint32_t row = (threadIdx.x & 63u) >> 4;
  return x + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

// Inclusive prefix maximum over the 64 lanes of a wave (all lanes active),
// built like wave_inclusive_sum; lanes shifted in from outside a row read 0.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t x) {
  uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x = x > t ? x : t;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x = x > t ? x : t;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x = x > t ? x : t;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x = x > t ? x : t;
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
  const uint32_t row = (threadIdx.x & 63u) >> 4;
  uint32_t below = row >= 1 ? r0 : 0u;
  if (row >= 2 && r1 > below) below = r1;
  if (row >= 3 && r2 > below) below = r2;
  return x > below ? x : below;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace dev
}  // namespace zig
