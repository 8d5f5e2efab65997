// Host construction of the ziggurat tables in binary128 (__float128).
//
// Section 2 of McFarland's paper: layers of equal area 1/i_max of the total
// lie under the density, each with its upper-right corner (X_i, P(X_i)) on
// the curve and its lower-left corner at (0, P(X_{i-1})), so that
//   X_i (P(X_i) - P(X_{i-1})) = area,
// solved bottom up until no further layer fits.  The rest of the mass lies
// in the tail beyond X_0, in the overhang right of each layer and in the cap
// above the top layer; the sampler picks one of those regions with
// probability proportional to its area.  Appendix B: the tables are computed
// in 128-bit precision and rounded once to double.
//
// Each layer's length is found by a bracketed Newton iteration on the layer
// equation (bisection whenever a Newton step leaves the bracket), starting
// from the maximiser of X (P(X) - P(X_{i-1})), itself found the same way.
#include <quadmath.h>

#include <cmath>
#include <deque>

#include "zig_internal.hpp"

namespace zig {
namespace {

using q128 = __float128;

struct Density {
  uint32_t dist;
  q128 p(q128 x) const { return dist == kDistExp ? expq(-x) : expq(-0.5Q * x * x); }
  q128 dp(q128 x) const { return dist == kDistExp ? -expq(-x) : -x * expq(-0.5Q * x * x); }
  q128 d2p(q128 x) const { return dist == kDistExp ? expq(-x) : (x * x - 1) * expq(-0.5Q * x * x); }
  q128 total() const { return dist == kDistExp ? (q128)1 : sqrtq(M_PIq * 0.5Q); }
  // integral of p over [x, infinity)
  q128 upper(q128 x) const {
    if (dist == kDistExp) return expq(-x);
    return sqrtq(M_PIq * 0.5Q) * erfcq(x * M_SQRT1_2q);
  }
  // integral of p over [lo, hi]
  q128 between(q128 lo, q128 hi) const {
    if (dist == kDistExp) return expq(-lo) * -expm1q(lo - hi);
    if (lo >= 1) return upper(lo) - upper(hi);
    return sqrtq(M_PIq * 0.5Q) * (erfq(hi * M_SQRT1_2q) - erfq(lo * M_SQRT1_2q));
  }
};

// Root of fn in [lo, hi] (fn changes sign there) by Newton steps kept inside
// a shrinking bracket.
template <class F, class DF>
q128 bracketed_newton(F fn, DF dfn, q128 lo, q128 hi) {
  q128 flo = fn(lo);
  q128 xneg = lo, xpos = hi;  // fn(xneg) < 0 <= fn(xpos)
  if (flo >= 0) {
    xneg = hi;
    xpos = lo;
  }
  q128 x = 0.5Q * (lo + hi);
  q128 step_old = fabsq(hi - lo), step = step_old;
  q128 fx = fn(x), dfx = dfn(x);
  if (fx < 0)
    xneg = x;
  else
    xpos = x;
  for (int it = 0; it < 600; ++it) {
    const bool outside = ((x - xpos) * dfx - fx) * ((x - xneg) * dfx - fx) > 0;
    const bool slow = fabsq(2 * fx) > fabsq(step_old * dfx);
    q128 prev = x;
    if (outside || slow || dfx == 0) {
      step_old = step;
      step = 0.5Q * (xpos - xneg);
      x = xneg + step;
    } else {
      step_old = step;
      step = fx / dfx;
      x = x - step;
    }
    if (x == prev) break;  // the bracket cannot shrink any further
    if (fabsq(x - prev) <= fabsq(x) * 0x1p-112Q) break;  // Newton converged
    fx = fn(x);
    dfx = dfn(x);
    if (fx < 0)
      xneg = x;
    else
      xpos = x;
  }
  return x;
}

// round-half-even of a non-negative binary128 value below 2^64
uint64_t round_half_even(q128 v) {
  q128 fl = floorq(v);
  q128 frac = v - fl;
  uint64_t r = (uint64_t)fl;
  if (frac > 0.5Q || (frac == 0.5Q && (r & 1))) r += 1;
  return r;
}

}  // namespace

std::string build_host_table(uint32_t dist, uint32_t i_max, HostTable* out) {
  if (dist != kDistExp && dist != kDistNormal) return "unknown distribution";
  uint32_t b = 0;
  while (b < 31 && (1u << b) < i_max) ++b;
  if ((1u << b) != i_max || i_max < 8 || i_max > kMaxLayers) return "i_max must be a power of two in [8, 1024]";

  const Density P{dist};
  const q128 area = P.total() / i_max;
  std::vector<q128> Xq, fq;
  q128 f_below = 0;
  q128 X_below = 64;  // P is negligible there for both densities
  while (Xq.size() < i_max) {
    auto g = [&](q128 x) { return x * (P.p(x) - f_below); };
    auto dg = [&](q128 x) { return P.p(x) - f_below + x * P.dp(x); };
    auto d2g = [&](q128 x) { return 2 * P.dp(x) + x * P.d2p(x); };
    const q128 x_peak = bracketed_newton(dg, d2g, (q128)0, X_below);
    if (g(x_peak) < area) break;
    auto h = [&](q128 x) { return g(x) - area; };
    const q128 x_new = bracketed_newton(h, dg, x_peak, X_below);
    Xq.push_back(x_new);
    fq.push_back(P.p(x_new));
    f_below = fq.back();
    X_below = x_new;
  }
  const uint32_t L = (uint32_t)Xq.size();
  if (L < 1 || L >= i_max) return "layer construction failed";

  HostTable& t = *out;
  t = HostTable();
  t.dist = dist;
  t.i_max = i_max;
  t.b = b;
  t.L = L;
  t.X.assign(L + 1, 0.0);
  t.f.assign(L + 1, 1.0);
  for (uint32_t i = 0; i < L; ++i) {
    t.X[i] = (double)Xq[i];
    t.f[i] = (double)fq[i];
  }
  t.XS.assign(i_max, 0.0);
  t.XS32.assign(i_max, 0.0f);
  // the 32-bit word keeps its low s = max(b, 8) bits for the index: the
  // magnitude has 32 - s bits (exponential) or 31 - s after the sign bit s
  const int s32 = b > 8 ? (int)b : 8;
  const int e32 = dist == kDistExp ? s32 - 32 : s32 - 31;
  for (uint32_t i = 0; i < L; ++i) {
    t.XS[i] = std::ldexp(t.X[i], -53);
    t.XS32[i] = std::ldexp((float)Xq[i], e32);
  }
  t.W.assign(L + 1, 0.0);
  t.H.assign(L + 1, 0.0);
  for (uint32_t j = 1; j <= L; ++j) {
    t.W[j] = t.X[j - 1] - t.X[j];
    t.H[j] = t.f[j] - t.f[j - 1];
  }

  // region masses: tail, overhang right of each layer, cap
  std::vector<q128> mass(L + 1);
  mass[0] = P.upper(Xq[0]);
  for (uint32_t j = 1; j <= L; ++j) {
    const q128 right = Xq[j - 1];
    const q128 left = (j == L) ? (q128)0 : Xq[j];
    mass[j] = P.between(left, right) - fq[j - 1] * (right - left);
  }
  q128 msum = 0;
  for (q128 m : mass) msum += m;
  t.q.assign(L + 1, 0);
  unsigned __int128 used = 0;
  const q128 two64 = 18446744073709551616.0Q;
  for (uint32_t j = 0; j < L; ++j) {
    t.q[j] = round_half_even(mass[j] / msum * two64);
    used += t.q[j];
  }
  const unsigned __int128 total_weight = (unsigned __int128)1 << 64;
  if (used >= total_weight) return "region weights overflow";
  t.q[L] = (uint64_t)(total_weight - used);

  // alias table (Vose) in exact integers; small and large columns are
  // served first-in first-out in ascending column order
  const uint64_t cap = (uint64_t)1 << (64 - b);
  t.T.assign(i_max, 0);
  t.A.assign(i_max, 0);
  std::vector<uint64_t> rest(i_max, 0);
  for (uint32_t c = 0; c <= L; ++c) rest[c] = t.q[c];
  std::deque<uint32_t> small, large;
  for (uint32_t c = 0; c < i_max; ++c) {
    if (rest[c] < cap) {
      small.push_back(c);
    } else if (rest[c] > cap) {
      large.push_back(c);
    } else {
      t.T[c] = cap;
      t.A[c] = c;
    }
  }
  while (!small.empty()) {
    if (large.empty()) return "alias construction failed";
    const uint32_t s = small.front();
    small.pop_front();
    const uint32_t g = large.front();
    t.T[s] = rest[s];
    t.A[s] = g;
    rest[g] -= cap - rest[s];
    if (rest[g] <= cap) {
      large.pop_front();
      if (rest[g] < cap) {
        small.push_back(g);
      } else {
        t.T[g] = cap;
        t.A[g] = g;
      }
    }
  }
  if (!large.empty()) return "alias construction left weight";

  // exponential boxes: largest normalised gap between chord and curve;
  // in a box of width w the curve is (e^{-wu} - e^{-w}) / (1 - e^{-w})
  if (dist == kDistExp) {
    q128 eps = 0;
    for (uint32_t j = 1; j <= L; ++j) {
      const q128 w = Xq[j - 1] - ((j == L) ? (q128)0 : Xq[j]);
      const q128 one_minus = -expm1q(-w);  // 1 - e^{-w}
      const q128 slope = one_minus / w;    // e^{-w u*} where the gap peaks
      const q128 u_star = -logq(slope) / w;
      const q128 gap = 1 - u_star - (slope - expq(-w)) / one_minus;
      if (gap > eps) eps = gap;
    }
    t.eps = (double)eps;
    t.K_eps = (uint64_t)floorq((1 - eps) * 9007199254740992.0Q);
  }

  // normal boxes, for the accelerated overhang variant: the largest
  // normalised gap between chord and curve in the convex boxes (X_j >= 1,
  // curve below the chord) and in the concave ones (X_{j-1} <= 1, curve
  // above, the cap included), at the point where the curve's normalised
  // slope is -1: x e^{-x^2/2} = h / w.  Each is widened by 2^-20 and turned
  // into a threshold on k1 + k2.
  //
  // The same gaps box by box give the squeeze of the plain box test (it
  // decides the same points as the density test, only without evaluating
  // it): in a convex box the point is under the curve when
  // u + v <= 1 - gap_j (1 + 2^-20) and over it when u + v >= 1 + 2^-20; in a
  // concave box under it when u + v < 1 - 2^-20 and over it when
  // u + v >= 1 + gap_j (1 + 2^-20).  The margins (2^-20 of the box, or of
  // its gap) exceed by far the rounding of the computed test; the box
  // holding x = 1 is never squeezed.
  if (dist == kDistNormal) {
    q128 widest_below = 0, widest_above = 0;
    const uint64_t one53 = (uint64_t)1 << 53, margin = (uint64_t)1 << 33;
    t.SQlo.assign(L + 1, 0);
    t.SQhi.assign(L + 1, (uint64_t)1 << 55);
    for (uint32_t j = 1; j <= L; ++j) {
      const bool convex = t.X[j] >= 1.0, concave = t.X[j - 1] <= 1.0;
      if (!convex && !concave) continue;
      const q128 left = (j == L) ? (q128)0 : Xq[j], right = Xq[j - 1];
      const q128 base = fq[j - 1], top = (j == L) ? (q128)1 : fq[j];
      const q128 w = right - left, h = top - base, slope = h / w;
      auto fn = [&](q128 x) { return x * P.p(x) - slope; };
      auto dfn = [&](q128 x) { return (1 - x * x) * P.p(x); };
      const q128 xs = bracketed_newton(fn, dfn, left, right);
      const q128 u = (xs - left) / w, c = (P.p(xs) - base) / h;
      if (convex) widest_below = fmaxq(widest_below, (1 - u) - c);
      if (concave) widest_above = fmaxq(widest_above, c - (1 - u));
      const q128 gap = convex ? (1 - u) - c : c - (1 - u);
      const q128 wide_gap = gap * (1 + 0x1p-20Q);
      if (convex) {
        t.SQlo[j] = (uint64_t)floorq((1 - wide_gap) * 9007199254740992.0Q) + 1;
        t.SQhi[j] = one53 + margin;
      } else {
        t.SQlo[j] = one53 - margin;
        t.SQhi[j] = (uint64_t)ceilq((1 + wide_gap) * 9007199254740992.0Q);
      }
    }
    const q128 widen = 1 + 0x1p-20Q;
    t.eps_cvx = (double)widest_below;
    t.del_ccv = (double)widest_above;
    t.K_cvx = (uint64_t)floorq((1 - widest_below * widen) * 9007199254740992.0Q);
    t.K_ccv = (uint64_t)ceilq((1 + widest_above * widen) * 9007199254740992.0Q);
  }
  t.X0 = t.X[0];
  t.invX0 = (double)(1 / Xq[0]);
  return std::string();
}

// Traditional stack of n layers (Marsaglia & Tsang; the right column of
// Table 1).  Given the base X_0 = r, every layer has the area
// v = r P(r) + (mass beyond r); layer i >= 1 sits on f_{i-1} with width
// X_{i-1}, so f_i = f_{i-1} + v / X_{i-1} and X_i = P^{-1}(f_i).  The right r
// leaves for the top layer, of width X_{n-2} and height 1 - f_{n-2}, exactly
// the area v: a larger r leaves it too much, a smaller one too little (or
// the stack reaches P(0) = 1 early).  r is found by bisection down to
// adjacent binary128 values.
std::string build_host_trad(uint32_t dist, uint32_t n, HostTrad* out) {
  if (dist != kDistExp && dist != kDistNormal) return "unknown distribution";
  uint32_t b = 0;
  while (b < 31 && (1u << b) < n) ++b;
  if ((1u << b) != n || n < 8 || n > kLdsLayers)
    return "the traditional sampler takes i_max a power of two in [8, 256]";
  const Density P{dist};
  auto inverse = [&](q128 y) { return dist == kDistExp ? -logq(y) : sqrtq(-2 * logq(y)); };
  std::vector<q128> X(n), f(n);
  q128 v = 0;
  // +1: r too large (top layer too big); -1: r too small
  auto side = [&](q128 r) -> int {
    v = r * P.p(r) + P.upper(r);
    X[0] = r;
    f[0] = P.p(r);
    for (uint32_t i = 1; i + 1 < n; ++i) {
      f[i] = f[i - 1] + v / X[i - 1];
      if (f[i] >= 1) return -1;
      X[i] = inverse(f[i]);
    }
    return X[n - 2] * (1 - f[n - 2]) > v ? 1 : -1;
  };
  q128 small = 0.25Q, large = 64;
  if (side(small) != -1 || side(large) != 1) return "traditional stack: no bracket";
  for (;;) {
    const q128 mid = 0.5Q * (small + large);
    if (!(mid > small && mid < large)) break;
    if (side(mid) > 0)
      large = mid;
    else
      small = mid;
  }
  if (side(large) != 1) return "traditional stack: bisection failed";
  X[n - 1] = 0;
  f[n - 1] = 1;

  HostTrad& t = *out;
  t = HostTrad();
  t.dist = dist;
  t.n = n;
  t.b = b;
  t.X.resize(n);
  t.f.resize(n);
  t.W.resize(n);
  t.WS.resize(n);
  t.k.resize(n);
  t.KQ.resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    const q128 w = i == 0 ? v / f[0] : X[i - 1];
    t.X[i] = (double)X[i];
    t.f[i] = (double)f[i];
    t.W[i] = (double)w;
    t.WS[i] = std::ldexp(t.W[i], -53);
    t.k[i] = (double)(X[i] / w);
    // k U1 < k_i for the 53-bit lattice value U1 = k 2^-53 exactly when the
    // integer k is below ceil(2^53 k_i)
    t.KQ[i] = (uint64_t)std::ceil(std::ldexp(t.k[i], 53));
  }
  t.r = t.X[0];
  t.v = (double)v;
  t.invr = (double)(1 / X[0]);
  return std::string();
}

}  // namespace zig
