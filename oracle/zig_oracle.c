/*
 * Scalar CPU oracle for the modified ziggurat sampler of McFarland,
 * arXiv:1403.6870.
 *
 * TEST INFRASTRUCTURE ONLY: this is the correctness reference the GPU
 * library is checked against.  It shares no code with the library; the
 * product path never links, loads or calls it.
 *
 * Plain, slow and direct on purpose: every Philox block is recomputed
 * when needed, every sample is produced by one straight-line function,
 * and the tables are built by bisection in 113-bit binary128 arithmetic.
 *
 * What is computed, with the paper passage each step follows:
 *
 *  Layers (section 2, the layer equation): equal-area layers of area
 *    a = total/i_max lie under P.  Layer k (0 = bottom) has upper-right
 *    corner (X_k, f_k = P(X_k)) on the density and lower-left corner
 *    (0, f_{k-1}), f_{-1} = 0, so X_k (P(X_k) - f_{k-1}) = a.  Layers are
 *    solved by bisection until none fits.  Tables are computed in 128-bit
 *    precision and rounded once to double (Appendix B).
 *  Regions outside the layers (section 2, Figure 1): the tail beyond X_0,
 *    the overhang to the right of each layer, and the cap above the top
 *    layer; each is drawn with probability proportional to its area by an
 *    alias table (section 2, the O(1) discrete draw of j from A).
 *  Sampling (Table 1, modified column): draw U1 and i; if i < L return
 *    U1 X_i; else draw j; j = 0 samples the tail; otherwise sample a point
 *    in box j and accept it under P, retrying in the same box.
 *  Exponential tail: memorylessness, X_0 plus a fresh exponential draw
 *    (the paragraph after Table 1; Appendix C item 4).
 *  Normal tail: Marsaglia's method fed with exponential draws (same
 *    paragraph).
 *  Exponential overhang split (the paragraph after Table 1, Figure 2):
 *    points above the chord are reflected into the lower triangle
 *    (Appendix C item 5), points below the chord by more than a single
 *    global eps (Appendix D item 2) are accepted without evaluating P.
 *  Integer uniforms (Appendix C items 1 and 2): U is a 64-bit integer,
 *    its low bits give i (and j's column).
 *
 * Readings taken where the text is ambiguous or garbled:
 *  R1  The regions are j = 0..L: tail, L-1 overhangs, and the cap above
 *      layer L-1 (X_L := 0, f_L := 1).  The text's j in [0, L) omits the
 *      cap, which holds mass.
 *  R2  The layer root is the larger root of X(P(X) - f_{k-1}) = a (between
 *      the maximiser of the left side and X_{k-1}); construction stops
 *      when the maximum of the left side is below a.
 *  R3  Table 1 step 7 uses the box of j with offset: accept when
 *      f_{j-1} + U2 (f_j - f_{j-1}) < P(x).
 *  R4  A rejected point is redrawn in the same box j with fresh U1, U2.
 *  R5  The chord-gap eps is computed per box width w in normalised
 *      coordinates: eps(w) = 1 - u* - 1/w + 1/(e^w - 1) with
 *      u* = -ln((1 - e^-w)/w)/w; eps = max over the boxes.
 *  R6  The reflection maps (u, v) above the chord u + v = 1 to
 *      (1 - v, 1 - u); fast-accept when u + v <= 1 - eps.
 *  R7  Normal overhangs use plain rejection in the box (the split is
 *      stated for the exponential only).
 *  R8  Normal tail: t = E1 / X_0 (as E1 * RN(1/X_0)), accept when
 *      E2 + E2 > t * t, return X_0 + t; E1, E2 from the exponential
 *      sampler with the exponential tables of the same i_max.
 *  R9  Exponential tail nesting folds to the right: X_0 + (X_0 + (...)).
 *  R10 Bits of the 64-bit fast word: i = bits 0..b-1, normal sign = bit
 *      10, magnitude k = bits 11..63 (53 bits), U1 = k 2^-53; no bit is
 *      used twice, and the magnitude bits are not reused on the slow path.
 *  R11 The alias table is built with exact integers: region weights
 *      q_j = RNE(2^64 A_j / sum A) for j < L, q_L = 2^64 - sum; Vose's
 *      construction with FIFO small/large lists in ascending index order.
 *  R12 Uniform source: Philox4x32-10 in place of the Mersenne Twister
 *      (section 2 states the source can be substituted).  Key =
 *      (seed lo, seed hi).  FP64 fast word of output n: block
 *      (n>>1, 0, 0) words 0|1 (n even) or 2|3 (n odd); FP32 fast word:
 *      block (n>>2, 0, 1) word n&3; slow word t of output n: block
 *      (n, t>>1, 2) words 0|1 (t even) or 2|3 (t odd).
 *  R13 Single precision (Appendix D item 4 names it without a definition):
 *      i = bits 0..b-1 of the 32-bit word and s = max(b, 8); exp magnitude
 *      = bits s..31, x = k * RN32(X_i) 2^-(32-s); normal sign = bit s,
 *      magnitude bits s+1..31, x = k * RN32(X_i) 2^-(31-s) (for the
 *      default 256 layers: bits 8..31 and 2^-24, sign bit 8, bits 9..31 and
 *      2^-23; Appendix D item 1's 1024 layers take bits 10..31 and 2^-22,
 *      sign bit 10, bits 11..31 and 2^-21).  The slow path is the double
 *      one, rounded to float at the end.
 *  R14 Location-scale is one fused multiply-add after sampling:
 *      out = fma(scale, x, shift); exponential scale = RN(1/lambda).
 *  R15 Traditional sampler (Table 1, right column; comparison only): the
 *      first (i, U1) is the fast word of R10/R12; the wedge's U2 and each
 *      restart's fresh word are the output's slow words in order; tails as
 *      R8/R9 with traditional exponentials.
 */
#include "zig_oracle.h"

#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 hp;

uint64_t orc_tables_size(void) { return (uint64_t)sizeof(orc_tables); }

/* ------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of two 32x32->64 products and xors with a
 * Weyl-bumped key, as defined by Salmon et al. (SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static void seed_key(uint64_t seed, uint32_t key[2]) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
}

static uint64_t fast_word64(uint64_t seed, uint64_t n) {
  uint32_t key[2], ctr[4], x[4];
  uint64_t m = n >> 1;
  seed_key(seed, key);
  ctr[0] = (uint32_t)m;
  ctr[1] = (uint32_t)(m >> 32);
  ctr[2] = 0;
  ctr[3] = 0;
  orc_philox4x32_10(ctr, key, x);
  if ((n & 1) == 0) return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
  return (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

static uint32_t fast_word32(uint64_t seed, uint64_t n) {
  uint32_t key[2], ctr[4], x[4];
  uint64_t m = n >> 2;
  seed_key(seed, key);
  ctr[0] = (uint32_t)m;
  ctr[1] = (uint32_t)(m >> 32);
  ctr[2] = 0;
  ctr[3] = 1;
  orc_philox4x32_10(ctr, key, x);
  return x[n & 3];
}

/* The slow stream of one output: word t comes from block (n, t>>1, 2). */
typedef struct {
  uint32_t key[2];
  uint64_t n;
  uint64_t t;
  uint32_t tests;
} slow_stream;

static uint64_t next_word(slow_stream* s) {
  uint32_t ctr[4], x[4];
  ctr[0] = (uint32_t)s->n;
  ctr[1] = (uint32_t)(s->n >> 32);
  ctr[2] = (uint32_t)(s->t >> 1);
  ctr[3] = 2;
  orc_philox4x32_10(ctr, s->key, x);
  uint64_t w;
  if ((s->t & 1) == 0)
    w = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
  else
    w = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
  s->t += 1;
  return w;
}

/* ------------------------------------------------------------------ */
/* Tables.  P is the unnormalised density: e^-x, or e^-x^2/2 on x >= 0. */

static hp dens(int dist, hp x) {
  if (dist == ORC_EXP) return expq(-x);
  return expq(-(x * x) / 2);
}

static hp dens_slope(int dist, hp x) {
  if (dist == ORC_EXP) return -expq(-x);
  return -x * expq(-(x * x) / 2);
}

static hp dens_total(int dist) {
  if (dist == ORC_EXP) return 1;
  return sqrtq(M_PIq / 2);
}

/* integral of P from x to infinity */
static hp dens_upper(int dist, hp x) {
  if (dist == ORC_EXP) return expq(-x);
  return sqrtq(M_PIq / 2) * erfcq(x / sqrtq((hp)2));
}

static void hpstr(char* dst, hp v) { quadmath_snprintf(dst, 48, "%.36Qe", v); }

/* g(X) = X (P(X) - fprev) and its derivative */
static hp layer_g(int dist, hp X, hp fprev) { return X * (dens(dist, X) - fprev); }
static hp layer_dg(int dist, hp X, hp fprev) { return dens(dist, X) - fprev + X * dens_slope(dist, X); }

int orc_build_tables(int dist, uint32_t i_max, orc_tables* t) {
  if (dist != ORC_EXP && dist != ORC_NORMAL) return -1;
  uint32_t b = 0;
  while ((1u << b) < i_max) ++b;
  if ((1u << b) != i_max || b < 3 || b > 10) return -1;
  memset(t, 0, sizeof(*t));
  t->dist = dist;
  t->i_max = i_max;
  t->b = b;
  const int s32 = b > 8 ? (int)b : 8; /* R13 */

  static __thread hp Xh[ORC_MAX_IMAX + 1], fh[ORC_MAX_IMAX + 1], Ah[ORC_MAX_IMAX + 1];
  const hp total = dens_total(dist);
  const hp area = total / i_max;

  /* layer recursion, bottom up */
  uint32_t L = 0;
  hp fprev = 0, Xprev = 64; /* P(64) is far below any layer height */
  for (;;) {
    if (L >= i_max) return -1;
    /* maximiser of g: g' falls through zero once on (0, Xprev) */
    hp lo = 0, hi = Xprev;
    for (int it = 0; it < 1000; ++it) {
      hp mid = (lo + hi) / 2;
      if (mid <= lo || mid >= hi) break;
      if (layer_dg(dist, mid, fprev) > 0)
        lo = mid;
      else
        hi = mid;
    }
    hp xm = lo;
    if (layer_g(dist, xm, fprev) < area) break; /* no further layer fits */
    /* the larger root: g decreases from g(xm) >= a to g(Xprev) < a */
    lo = xm;
    hi = Xprev;
    for (int it = 0; it < 1000; ++it) {
      hp mid = (lo + hi) / 2;
      if (mid <= lo || mid >= hi) break;
      if (layer_g(dist, mid, fprev) >= area)
        lo = mid;
      else
        hi = mid;
    }
    Xh[L] = lo;
    fh[L] = dens(dist, lo);
    fprev = fh[L];
    Xprev = lo;
    ++L;
  }
  if (L < 1) return -1;
  t->L = L;
  Xh[L] = 0;
  fh[L] = 1;

  for (uint32_t k = 0; k <= L; ++k) {
    t->X[k] = (double)Xh[k];
    t->f[k] = (double)fh[k];
    hpstr(t->hpX[k], Xh[k]);
    hpstr(t->hpf[k], fh[k]);
  }
  t->X[L] = 0.0;
  t->f[L] = 1.0;
  for (uint32_t i = 0; i < i_max; ++i) {
    if (i < L) {
      t->XS[i] = ldexp(t->X[i], -53);
      t->XS32[i] = ldexpf((float)Xh[i], dist == ORC_EXP ? s32 - 32 : s32 - 31);
    } else {
      t->XS[i] = 0.0;
      t->XS32[i] = 0.0f;
    }
  }
  for (uint32_t j = 1; j <= L; ++j) {
    t->W[j] = t->X[j - 1] - t->X[j];
    t->H[j] = t->f[j] - t->f[j - 1];
  }

  /* region masses: tail, overhangs right of each layer, cap */
  Ah[0] = dens_upper(dist, Xh[0]);
  for (uint32_t j = 1; j <= L; ++j) {
    hp under = dens_upper(dist, Xh[j]) - dens_upper(dist, Xh[j - 1]);
    Ah[j] = under - fh[j - 1] * (Xh[j - 1] - Xh[j]);
  }
  hp sumA = 0;
  for (uint32_t j = 0; j <= L; ++j) sumA += Ah[j];
  for (uint32_t j = 0; j <= L; ++j) hpstr(t->hpA[j], Ah[j]);
  hpstr(t->hp_area, area);
  hpstr(t->hp_total, total);

  /* integer weights summing to 2^64 */
  unsigned __int128 acc = 0;
  const hp two64 = ldexpq(1, 64);
  for (uint32_t j = 0; j < L; ++j) {
    hp v = rintq(Ah[j] / sumA * two64);
    t->q[j] = (uint64_t)v;
    acc += t->q[j];
  }
  unsigned __int128 full = (unsigned __int128)1 << 64;
  if (acc >= full) return -1;
  t->q[L] = (uint64_t)(full - acc);

  /* alias table, exact integers, FIFO order */
  {
    const uint64_t cap = (uint64_t)1 << (64 - b);
    static __thread uint64_t w[ORC_MAX_IMAX];
    static __thread uint32_t small[ORC_MAX_IMAX], large[ORC_MAX_IMAX];
    uint32_t sh = 0, st = 0, lh = 0, lt = 0;
    for (uint32_t c = 0; c < i_max; ++c) w[c] = (c <= L) ? t->q[c] : 0;
    for (uint32_t c = 0; c < i_max; ++c) {
      if (w[c] < cap)
        small[st++] = c;
      else if (w[c] > cap)
        large[lt++] = c;
      else {
        t->T[c] = cap;
        t->A[c] = c;
      }
    }
    while (sh < st) {
      if (lh >= lt) return -1;
      uint32_t s = small[sh++];
      uint32_t g = large[lh];
      t->T[s] = w[s];
      t->A[s] = g;
      w[g] -= cap - w[s];
      if (w[g] < cap) {
        ++lh;
        small[st++] = g;
      } else if (w[g] == cap) {
        ++lh;
        t->T[g] = cap;
        t->A[g] = g;
      }
    }
    if (lh != lt) return -1;
  }

  /* chord gap of the exponential boxes */
  if (dist == ORC_EXP) {
    hp eps = 0;
    for (uint32_t j = 1; j <= L; ++j) {
      hp wd = Xh[j - 1] - Xh[j];
      hp ustar = -logq(-expm1q(-wd) / wd) / wd;
      hp e = 1 - ustar - 1 / wd + 1 / expm1q(wd);
      if (e > eps) eps = e;
    }
    t->eps = (double)eps;
    t->K_eps = (uint64_t)floorq((1 - eps) * ldexpq(1, 53));
    hpstr(t->hp_eps, eps);
  }
  /* chord bands of the normal boxes, for the accelerated overhang variant.
   * In a box's normalised coordinates the curve runs from (0, 1) to (1, 0)
   * and the chord is u + v = 1.  Right of the inflection point (X_j >= 1)
   * the curve is convex and lies below the chord, left of it (X_{j-1} <= 1,
   * the cap included) concave and above; the gap is largest where the
   * curve's normalised slope is -1, i.e. where x e^{-x^2/2} = h / w, the
   * only such point in the box (x e^{-x^2/2} is monotone on either side
   * of 1).  The box straddling 1 has no band. */
  if (dist == ORC_NORMAL) {
    hp ecvx = 0, dccv = 0;
    for (uint32_t j = 1; j <= L; ++j) {
      const int convex = t->X[j] >= 1.0, concave = t->X[j - 1] <= 1.0;
      if (!convex && !concave) continue;
      const hp left = Xh[j], right = Xh[j - 1], w = right - left;
      const hp base = fh[j - 1], top = fh[j], h = top - base;
      const hp target = h / w;
      hp lo = left, hi = right;
      for (int it = 0; it < 1000; ++it) {
        const hp mid = (lo + hi) / 2;
        if (mid <= lo || mid >= hi) break;
        const hp ph = mid * expq(-mid * mid / 2) - target;
        if (convex ? ph > 0 : ph < 0)
          lo = mid;
        else
          hi = mid;
      }
      const hp u = (lo - left) / w;
      const hp c = (expq(-lo * lo / 2) - base) / h;
      const hp gap = convex ? (1 - u) - c : c - (1 - u);
      if (convex && gap > ecvx) ecvx = gap;
      if (concave && gap > dccv) dccv = gap;
    }
    const hp widen = 1 + ldexpq(1, -20);
    t->eps_cvx = (double)ecvx;
    t->del_ccv = (double)dccv;
    t->K_cvx = (uint64_t)floorq((1 - ecvx * widen) * ldexpq(1, 53));
    t->K_ccv = (uint64_t)ceilq((1 + dccv * widen) * ldexpq(1, 53));
    hpstr(t->hp_eps_cvx, ecvx);
    hpstr(t->hp_del_ccv, dccv);
  }
  t->X0 = t->X[0];
  t->invX0 = (double)(1 / Xh[0]);
  return 0;
}

uint32_t orc_alias_draw(const orc_tables* t, uint64_t r) {
  uint32_t c = (uint32_t)(r & (t->i_max - 1));
  uint64_t h = r >> t->b;
  return (h < t->T[c]) ? c : t->A[c];
}

/* ------------------------------------------------------------------ */
/* Sampling */

static const uint64_t ONE53 = (uint64_t)1 << 53;

static double unif53(uint64_t k) { return (double)k * 0x1p-53; }

static double box_left(const orc_tables* t, uint32_t j) { return t->X[j]; /* X[L] = 0 */ }

/* One attempt in box j.  Exponential: reflect across the chord, accept
 * below the eps band without evaluating P, else compare with P(x).
 * Normal: compare with P(x); in the accelerated variant, first the chord
 * bands of the convex and concave boxes. */
static int box_try(const orc_tables* t, uint32_t j, uint64_t k1, uint64_t k2, double* x, uint32_t* tests) {
  if (t->dist == ORC_EXP) {
    if (k1 + k2 > ONE53) {
      uint64_t r1 = ONE53 - k2;
      uint64_t r2 = ONE53 - k1;
      k1 = r1;
      k2 = r2;
    }
    double xv = fma(unif53(k1), t->W[j], box_left(t, j));
    if (k1 + k2 <= t->K_eps) {
      *x = xv;
      return 1;
    }
    double y = fma(unif53(k2), t->H[j], t->f[j - 1]);
    *tests += 1;
    if (y < exp(-xv)) {
      *x = xv;
      return 1;
    }
    return 0;
  }
  if (t->accel) {
    /* accelerated variant: reflection and the eps band in convex boxes,
     * accept below the chord and reject above the delta band in concave
     * ones, plain rejection in the box straddling the inflection point */
    if (t->X[j] >= 1.0) {
      if (k1 + k2 > ONE53) {
        uint64_t r1 = ONE53 - k2;
        uint64_t r2 = ONE53 - k1;
        k1 = r1;
        k2 = r2;
      }
      double xv = fma(unif53(k1), t->W[j], box_left(t, j));
      if (k1 + k2 <= t->K_cvx) {
        *x = xv;
        return 1;
      }
      double y = fma(unif53(k2), t->H[j], t->f[j - 1]);
      *tests += 1;
      if (y < exp(-0.5 * (xv * xv))) {
        *x = xv;
        return 1;
      }
      return 0;
    }
    if (t->X[j - 1] <= 1.0) {
      double xv = fma(unif53(k1), t->W[j], box_left(t, j));
      if (k1 + k2 <= ONE53) {
        *x = xv;
        return 1;
      }
      if (k1 + k2 > t->K_ccv) return 0;
      double y = fma(unif53(k2), t->H[j], t->f[j - 1]);
      *tests += 1;
      if (y < exp(-0.5 * (xv * xv))) {
        *x = xv;
        return 1;
      }
      return 0;
    }
  }
  double xv = fma(unif53(k1), t->W[j], box_left(t, j));
  double y = fma(unif53(k2), t->H[j], t->f[j - 1]);
  *tests += 1;
  if (y < exp(-0.5 * (xv * xv))) {
    *x = xv;
    return 1;
  }
  return 0;
}

int orc_box_attempt(const orc_tables* t, uint32_t j, uint64_t k1, uint64_t k2, double* x) {
  uint32_t tests = 0;
  if (j < 1 || j > t->L || k1 >= ONE53 || k2 >= ONE53) return -1;
  return box_try(t, j, k1, k2, x, &tests);
}

int orc_box_grid(const orc_tables* t, uint32_t j, uint32_t g, uint32_t shift, uint8_t* accept, double* x) {
  if (j < 1 || j > t->L || shift > 53 || ((uint64_t)g << shift) > ONE53) return -1;
  for (uint64_t a = 0; a < g; ++a)
    for (uint64_t c = 0; c < g; ++c) {
      uint32_t tests = 0;
      double xv = 0.0;
      int r = box_try(t, j, a << shift, c << shift, &xv, &tests);
      accept[a * g + c] = (uint8_t)r;
      x[a * g + c] = r ? xv : 0.0;
    }
  return 0;
}

static double exp_region(const orc_tables* ex, uint32_t j, slow_stream* s);

/* the exponential sampler started from fast word w, continuing on s */
static double exp_from_word(const orc_tables* ex, uint64_t w, slow_stream* s) {
  uint32_t i = (uint32_t)(w & (ex->i_max - 1));
  if (i < ex->L) return (double)(w >> 11) * ex->XS[i];
  uint64_t r = next_word(s);
  return exp_region(ex, orc_alias_draw(ex, r), s);
}

static double exp_region(const orc_tables* ex, uint32_t j, slow_stream* s) {
  if (j == 0) {
    uint64_t w = next_word(s);
    double rest = exp_from_word(ex, w, s);
    return ex->X0 + rest;
  }
  for (;;) {
    uint64_t k1 = next_word(s) >> 11;
    uint64_t k2 = next_word(s) >> 11;
    double x;
    if (box_try(ex, j, k1, k2, &x, &s->tests)) return x;
  }
}

static double normal_region(const orc_tables* nt, const orc_tables* ex, uint32_t j, slow_stream* s) {
  if (j == 0) {
    for (;;) {
      uint64_t w1 = next_word(s);
      double e1 = exp_from_word(ex, w1, s);
      uint64_t w2 = next_word(s);
      double e2 = exp_from_word(ex, w2, s);
      double tt = e1 * nt->invX0;
      if (e2 + e2 > tt * tt) return nt->X0 + tt;
    }
  }
  for (;;) {
    uint64_t k1 = next_word(s) >> 11;
    uint64_t k2 = next_word(s) >> 11;
    double x;
    if (box_try(nt, j, k1, k2, &x, &s->tests)) return x;
  }
}

typedef struct {
  uint32_t layer;
  int32_t region;
  uint32_t words;
  uint32_t tests;
} trace_rec;

/* magnitude from the slow path of output n (first alias draw, then region) */
static double slow_magnitude(int dist, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t n,
                             trace_rec* tr) {
  slow_stream s;
  seed_key(seed, s.key);
  s.n = n;
  s.t = 0;
  s.tests = 0;
  const orc_tables* t = (dist == ORC_EXP) ? ex : nt;
  uint32_t j = orc_alias_draw(t, next_word(&s));
  double x = (dist == ORC_EXP) ? exp_region(ex, j, &s) : normal_region(nt, ex, j, &s);
  tr->region = (int32_t)j;
  tr->words = (uint32_t)s.t;
  tr->tests = s.tests;
  return x;
}

static double sample64(int dist, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t n, double scale,
                       double shift, trace_rec* tr) {
  const orc_tables* t = (dist == ORC_EXP) ? ex : nt;
  uint64_t w = fast_word64(seed, n);
  uint32_t i = (uint32_t)(w & (t->i_max - 1));
  double x;
  tr->layer = i;
  tr->region = -1;
  tr->words = 0;
  tr->tests = 0;
  if (i < t->L)
    x = (double)(w >> 11) * t->XS[i];
  else
    x = slow_magnitude(dist, ex, nt, seed, n, tr);
  if (dist == ORC_NORMAL && ((w >> 10) & 1)) x = -x;
  return fma(scale, x, shift);
}

static float sample32(int dist, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t n, double scale,
                      double shift, trace_rec* tr) {
  const orc_tables* t = (dist == ORC_EXP) ? ex : nt;
  uint32_t w = fast_word32(seed, n);
  uint32_t i = w & (t->i_max - 1);
  const uint32_t s32 = t->b > 8 ? t->b : 8; /* R13 */
  float x;
  tr->layer = i;
  tr->region = -1;
  tr->words = 0;
  tr->tests = 0;
  if (dist == ORC_EXP) {
    if (i < t->L)
      x = (float)(w >> s32) * t->XS32[i];
    else
      x = (float)slow_magnitude(dist, ex, nt, seed, n, tr);
  } else {
    if (i < t->L)
      x = (float)(w >> (s32 + 1)) * t->XS32[i];
    else
      x = (float)slow_magnitude(dist, ex, nt, seed, n, tr);
    if ((w >> s32) & 1) x = -x;
  }
  return fmaf((float)scale, x, (float)shift);
}

static int check_args(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t first, uint64_t n,
                      const void* out) {
  if (dist != ORC_EXP && dist != ORC_NORMAL) return -1;
  if (dtype != ORC_F64 && dtype != ORC_F32) return -1;
  if (ex == NULL || ex->dist != ORC_EXP) return -1;
  if (dist == ORC_NORMAL && (nt == NULL || nt->dist != ORC_NORMAL)) return -1;
  if (n > 0 && out == NULL) return -1;
  if (n > 0 && first + (n - 1) < first) return -1;
  return 0;
}

int orc_fill_trace(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t first,
                   uint64_t n, double scale, double shift, void* out, uint32_t* layer, int32_t* region,
                   uint32_t* words, uint32_t* tests) {
  if (check_args(dist, dtype, ex, nt, first, n, out)) return -1;
  for (uint64_t k = 0; k < n; ++k) {
    trace_rec tr;
    if (dtype == ORC_F64)
      ((double*)out)[k] = sample64(dist, ex, nt, seed, first + k, scale, shift, &tr);
    else
      ((float*)out)[k] = sample32(dist, ex, nt, seed, first + k, scale, shift, &tr);
    if (layer) layer[k] = tr.layer;
    if (region) region[k] = tr.region;
    if (words) words[k] = tr.words;
    if (tests) tests[k] = tr.tests;
  }
  return 0;
}

typedef struct {
  int dist, dtype;
  const orc_tables *ex, *nt;
  uint64_t seed, first, lo, hi;
  double scale, shift;
  void* out;
} fill_job;

static void* fill_worker(void* arg) {
  fill_job* jb = (fill_job*)arg;
  for (uint64_t k = jb->lo; k < jb->hi; ++k) {
    trace_rec tr;
    if (jb->dtype == ORC_F64)
      ((double*)jb->out)[k] = sample64(jb->dist, jb->ex, jb->nt, jb->seed, jb->first + k, jb->scale, jb->shift, &tr);
    else
      ((float*)jb->out)[k] = sample32(jb->dist, jb->ex, jb->nt, jb->seed, jb->first + k, jb->scale, jb->shift, &tr);
  }
  return NULL;
}

int orc_fill(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t first,
             uint64_t n, double scale, double shift, void* out, int threads) {
  if (check_args(dist, dtype, ex, nt, first, n, out)) return -1;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((uint64_t)threads > n) threads = (n > 0) ? (int)n : 1;
  fill_job jobs[256];
  pthread_t tid[256];
  for (int k = 0; k < threads; ++k) {
    jobs[k].dist = dist;
    jobs[k].dtype = dtype;
    jobs[k].ex = ex;
    jobs[k].nt = nt;
    jobs[k].seed = seed;
    jobs[k].first = first;
    jobs[k].lo = n * (uint64_t)k / (uint64_t)threads;
    jobs[k].hi = n * (uint64_t)(k + 1) / (uint64_t)threads;
    jobs[k].scale = scale;
    jobs[k].shift = shift;
    jobs[k].out = out;
  }
  if (threads == 1) {
    fill_worker(&jobs[0]);
    return 0;
  }
  for (int k = 0; k < threads; ++k) pthread_create(&tid[k], NULL, fill_worker, &jobs[k]);
  for (int k = 0; k < threads; ++k) pthread_join(tid[k], NULL);
  return 0;
}

/* ---- raw moments (Appendix B's test statistic; section 3's
 * generate-and-aggregate benchmark) -------------------------------------
 * S_p = sum of x^p, p = 1..5, over the outputs x of a fill of (dist,
 * dtype, seed, first, n, scale, shift), each x taken as the fill writes
 * it (a float widened to double) and its powers formed by double
 * multiplications q2 = x*x, q3 = q2*x, q4 = q2*q2, q5 = q4*x.  The sum is
 * the exact sum of those terms rounded once to double (to nearest, ties
 * to even), so it depends on no order of addition; the absolute sums
 * sum |q_p| are formed the same way (they bound any other order's
 * rounding error). */

/* Exact sum of doubles.  A finite double is m 2^(e - 1075) with m an
 * integer below 2^53 and e its biased exponent field (a subnormal counts
 * as e = 1 without the hidden bit).  Bucket e holds the signed sum of the
 * m of all terms with that field, so the sum is sum_e bucket[e] 2^(e-1075)
 * exactly; a 128-bit bucket takes 2^74 terms before it could overflow. */
#define XS_BUCKETS 2047
typedef struct {
  __int128 b[XS_BUCKETS];
  int nonfinite;
} exact_sum;

static void xs_add(exact_sum* s, double x) {
  uint64_t u;
  memcpy(&u, &x, sizeof(u));
  uint32_t e = (uint32_t)(u >> 52) & 0x7ffu;
  int64_t m = (int64_t)(u & ((1ull << 52) - 1));
  if (e == 0x7ffu) {
    s->nonfinite = 1;
    return;
  }
  if (e == 0)
    e = 1;
  else
    m |= (int64_t)1 << 52;
  if (u >> 63)
    s->b[e] -= m;
  else
    s->b[e] += m;
}

static void xs_merge(exact_sum* into, const exact_sum* from) {
  for (int e = 0; e < XS_BUCKETS; ++e) into->b[e] += from->b[e];
  into->nonfinite |= from->nonfinite;
}

/* Unsigned big integers of XS_LIMBS 64-bit limbs, least significant
 * first, counting units of 2^-1074: bucket e weighs 2^(e-1). */
#define XS_LIMBS 36

static void big_add_shifted(uint64_t* big, unsigned __int128 v, uint32_t sh) {
  const uint32_t q = sh / 64, r = sh % 64;
  const uint64_t v0 = (uint64_t)v, v1 = (uint64_t)(v >> 64);
  uint64_t w[3];
  w[0] = v0 << r;
  w[1] = r ? (v1 << r) | (v0 >> (64 - r)) : v1;
  w[2] = r ? v1 >> (64 - r) : 0;
  unsigned __int128 carry = 0;
  for (uint32_t k = q; k < XS_LIMBS; ++k) {
    const unsigned __int128 t = (unsigned __int128)big[k] + (k - q < 3 ? w[k - q] : 0) + carry;
    big[k] = (uint64_t)t;
    carry = t >> 64;
    if (k - q >= 2 && carry == 0) break;
  }
}

static int big_cmp(const uint64_t* a, const uint64_t* b) {
  for (int k = XS_LIMBS - 1; k >= 0; --k)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}

static void big_sub(uint64_t* a, const uint64_t* b) { /* a -= b, a >= b */
  uint64_t borrow = 0;
  for (int k = 0; k < XS_LIMBS; ++k) {
    const uint64_t bk = b[k] + borrow;
    const uint64_t nb = (bk < borrow) || (a[k] < bk);
    a[k] -= bk;
    borrow = nb;
  }
}

static int big_bit(const uint64_t* a, int pos) { return (int)((a[pos / 64] >> (pos % 64)) & 1u); }

/* The exact sum rounded to double, to nearest with ties to even (an
 * exact zero gives +0; a non-finite term gives NaN). */
static double xs_round(const exact_sum* s) {
  if (s->nonfinite) return NAN;
  uint64_t pos[XS_LIMBS], neg[XS_LIMBS];
  memset(pos, 0, sizeof(pos));
  memset(neg, 0, sizeof(neg));
  for (uint32_t e = 1; e < XS_BUCKETS; ++e) {
    const __int128 v = s->b[e];
    if (v > 0) big_add_shifted(pos, (unsigned __int128)v, e - 1);
    if (v < 0) big_add_shifted(neg, (unsigned __int128)0 - (unsigned __int128)v, e - 1);
  }
  double sign = 1.0;
  const int c = big_cmp(pos, neg);
  if (c == 0) return 0.0;
  if (c > 0) {
    big_sub(pos, neg);
  } else {
    big_sub(neg, pos);
    memcpy(pos, neg, sizeof(pos));
    sign = -1.0;
  }
  int top = XS_LIMBS * 64 - 1;
  while (!big_bit(pos, top)) --top;
  if (top < 53) return sign * ldexp((double)pos[0], -1074); /* exact */
  uint64_t mant = 0;
  for (int k = top; k > top - 53; --k) mant = (mant << 1) | (uint64_t)big_bit(pos, k);
  const int rbit = big_bit(pos, top - 53);
  int sticky = 0;
  for (int k = top - 54; k >= 0 && !sticky; --k) {
    if (k % 64 == 63 && pos[k / 64] == 0) {
      k -= 63;
      continue;
    }
    sticky = big_bit(pos, k);
  }
  if (rbit && (sticky || (mant & 1u))) ++mant; /* mant may reach 2^53: still exact */
  return sign * ldexp((double)mant, top - 52 - 1074);
}

int orc_exact_sum(const double* x, uint64_t n, double* sum) {
  if (sum == NULL || (n > 0 && x == NULL)) return -1;
  exact_sum* s = (exact_sum*)calloc(1, sizeof(exact_sum));
  if (s == NULL) return -1;
  for (uint64_t k = 0; k < n; ++k) xs_add(s, x[k]);
  *sum = xs_round(s);
  free(s);
  return 0;
}

typedef struct {
  int dist, dtype;
  const orc_tables *ex, *nt;
  uint64_t seed, first, lo, hi;
  double scale, shift;
  exact_sum* acc; /* [10]: S_1..S_5, then |.| sums */
} mom_job;

static void* mom_worker(void* arg) {
  mom_job* jb = (mom_job*)arg;
  for (uint64_t k = jb->lo; k < jb->hi; ++k) {
    trace_rec tr;
    double x;
    if (jb->dtype == ORC_F64)
      x = sample64(jb->dist, jb->ex, jb->nt, jb->seed, jb->first + k, jb->scale, jb->shift, &tr);
    else
      x = (double)sample32(jb->dist, jb->ex, jb->nt, jb->seed, jb->first + k, jb->scale, jb->shift, &tr);
    const double q2 = x * x, q3 = q2 * x, q4 = q2 * q2, q5 = q4 * x;
    const double q[5] = {x, q2, q3, q4, q5};
    for (int p = 0; p < 5; ++p) {
      xs_add(&jb->acc[p], q[p]);
      xs_add(&jb->acc[5 + p], fabs(q[p]));
    }
  }
  return NULL;
}

int orc_moments(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t first,
                uint64_t n, double scale, double shift, double sums[5], double abs_sums[5], int threads) {
  double dummy;
  if (check_args(dist, dtype, ex, nt, first, n, &dummy) || sums == NULL) return -1;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((uint64_t)threads > n) threads = n > 0 ? (int)n : 1;
  exact_sum* acc = (exact_sum*)calloc((size_t)threads * 10, sizeof(exact_sum));
  if (acc == NULL) return -1;
  mom_job jobs[256];
  pthread_t tid[256];
  for (int k = 0; k < threads; ++k) {
    mom_job* jb = &jobs[k];
    jb->dist = dist;
    jb->dtype = dtype;
    jb->ex = ex;
    jb->nt = nt;
    jb->seed = seed;
    jb->first = first;
    jb->lo = n * (uint64_t)k / (uint64_t)threads;
    jb->hi = n * (uint64_t)(k + 1) / (uint64_t)threads;
    jb->scale = scale;
    jb->shift = shift;
    jb->acc = acc + (size_t)k * 10;
  }
  if (threads == 1) {
    mom_worker(&jobs[0]);
  } else {
    for (int k = 0; k < threads; ++k) pthread_create(&tid[k], NULL, mom_worker, &jobs[k]);
    for (int k = 0; k < threads; ++k) pthread_join(tid[k], NULL);
  }
  for (int k = 1; k < threads; ++k)
    for (int p = 0; p < 10; ++p) xs_merge(&acc[p], &acc[(size_t)k * 10 + p]);
  for (int p = 0; p < 5; ++p) {
    sums[p] = xs_round(&acc[p]);
    if (abs_sums) abs_sums[p] = xs_round(&acc[5 + p]);
  }
  free(acc);
  return 0;
}

/* ---- traditional ziggurat ------------------------------------------- */

static hp dens_inverse(int dist, hp y) { return dist == ORC_EXP ? -logq(y) : sqrtq(-2 * logq(y)); }

/* Builds the stack from X_0 = r; returns f_{n-1} - P(0) (the closure
 * residual, decreasing in r), or +1 if the stack reaches P(0) early. */
static hp trad_stack(int dist, uint32_t n, hp r, hp* X, hp* f, hp* v_out) {
  const hp v = r * dens(dist, r) + dens_upper(dist, r);
  X[0] = r;
  f[0] = dens(dist, r);
  for (uint32_t i = 1; i < n; ++i) {
    f[i] = f[i - 1] + v / X[i - 1];
    if (i == n - 1) break;
    if (f[i] >= 1) return 1;
    X[i] = dens_inverse(dist, f[i]);
  }
  *v_out = v;
  return f[n - 1] - 1;
}

int orc_build_trad(int dist, uint32_t n, orc_trad* t) {
  if (dist != ORC_EXP && dist != ORC_NORMAL) return -1;
  uint32_t b = 0;
  while ((1u << b) < n) ++b;
  if ((1u << b) != n || b < 3 || b > 10) return -1;
  memset(t, 0, sizeof(*t));
  t->dist = dist;
  t->n = n;
  t->b = b;
  static __thread hp X[ORC_MAX_IMAX + 1], f[ORC_MAX_IMAX + 1];
  hp lo = 0.5, hi = 40, v = 0;
  for (int it = 0; it < 2000; ++it) {
    const hp mid = (lo + hi) / 2;
    if (mid <= lo || mid >= hi) break;
    if (trad_stack(dist, n, mid, X, f, &v) > 0)
      lo = mid;
    else
      hi = mid;
  }
  if (trad_stack(dist, n, hi, X, f, &v) > 0) return -1;
  X[n - 1] = 0;
  f[n - 1] = 1;
  for (uint32_t i = 0; i < n; ++i) {
    t->X[i] = (double)X[i];
    t->f[i] = (double)f[i];
    const hp w = (i == 0) ? v / f[0] : X[i - 1];
    t->W[i] = (double)w;
    t->WS[i] = ldexp(t->W[i], -53);
    t->k[i] = (double)(X[i] / w);
  }
  t->v = (double)v;
  t->r = (double)X[0];
  t->invr = (double)(1 / X[0]);
  hpstr(t->hp_r, X[0]);
  hpstr(t->hp_v, v);
  return 0;
}

uint64_t orc_trad_size(void) { return sizeof(orc_trad); }

/* The traditional exponential sampler from a (U1, i) word w: returns x
 * with the tails nested as X_0 + (X_0 + (... + y)). */
static double trad_exp_from(const orc_trad* E, uint64_t w, slow_stream* s) {
  uint32_t nest = 0;
  double x;
  for (;;) {
    const uint32_t i = (uint32_t)(w & (E->n - 1));
    const uint64_t k = w >> 11;
    x = (double)k * E->WS[i];
    if (unif53(k) < E->k[i]) break; /* step 3 */
    if (i == 0) {                   /* step 4: the tail, by memorylessness */
      ++nest;
      w = next_word(s);
      continue;
    }
    const double y = fma(unif53(next_word(s) >> 11), E->f[i] - E->f[i - 1], E->f[i - 1]); /* steps 5-6 */
    s->tests += 1;
    if (y < exp(-x)) break;
    w = next_word(s); /* step 7 */
  }
  for (uint32_t c = 0; c < nest; ++c) x = E->r + x;
  return x;
}

static double trad_normal_from(const orc_trad* N, const orc_trad* E, uint64_t w, slow_stream* s) {
  for (;;) {
    const uint32_t i = (uint32_t)(w & (N->n - 1));
    const uint64_t k = w >> 11;
    const double x = (double)k * N->WS[i];
    if (unif53(k) < N->k[i]) return x;
    if (i == 0) {
      for (;;) {
        const double e1 = trad_exp_from(E, next_word(s), s);
        const double e2 = trad_exp_from(E, next_word(s), s);
        const double tt = e1 * N->invr;
        if (e2 + e2 > tt * tt) return N->r + tt;
      }
    }
    const double y = fma(unif53(next_word(s) >> 11), N->f[i] - N->f[i - 1], N->f[i - 1]);
    s->tests += 1;
    if (y < exp(-0.5 * (x * x))) return x;
    w = next_word(s);
  }
}

typedef struct {
  int dist;
  const orc_trad *ex, *nt;
  uint64_t seed, first, lo, hi;
  double scale, shift;
  double* out;
  uint32_t* words;
} trad_job;

static void* trad_worker(void* arg) {
  trad_job* jb = (trad_job*)arg;
  for (uint64_t k = jb->lo; k < jb->hi; ++k) {
    const uint64_t g = jb->first + k;
    const uint64_t w = fast_word64(jb->seed, g);
    slow_stream s;
    seed_key(jb->seed, s.key);
    s.n = g;
    s.t = 0;
    s.tests = 0;
    double x;
    if (jb->dist == ORC_EXP) {
      x = trad_exp_from(jb->ex, w, &s);
    } else {
      x = trad_normal_from(jb->nt, jb->ex, w, &s);
      if ((w >> 10) & 1) x = -x;
    }
    jb->out[k] = fma(jb->scale, x, jb->shift);
    if (jb->words) jb->words[k] = (uint32_t)s.t;
  }
  return NULL;
}

int orc_trad_fill(int dist, const orc_trad* ex, const orc_trad* nt, uint64_t seed, uint64_t first, uint64_t n,
                  double scale, double shift, double* out, uint32_t* words, int threads) {
  if (dist != ORC_EXP && dist != ORC_NORMAL) return -1;
  if (ex == NULL || ex->dist != ORC_EXP || (dist == ORC_NORMAL && (nt == NULL || nt->dist != ORC_NORMAL)))
    return -1;
  if (n > 0 && (out == NULL || first + (n - 1) < first)) return -1;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((uint64_t)threads > n) threads = n > 0 ? (int)n : 1;
  trad_job jobs[256];
  pthread_t tid[256];
  for (int k = 0; k < threads; ++k) {
    trad_job* jb = &jobs[k];
    jb->dist = dist;
    jb->ex = ex;
    jb->nt = nt;
    jb->seed = seed;
    jb->first = first;
    jb->lo = n * (uint64_t)k / (uint64_t)threads;
    jb->hi = n * (uint64_t)(k + 1) / (uint64_t)threads;
    jb->scale = scale;
    jb->shift = shift;
    jb->out = out;
    jb->words = words;
  }
  if (threads == 1) {
    trad_worker(&jobs[0]);
    return 0;
  }
  for (int k = 0; k < threads; ++k) pthread_create(&tid[k], NULL, trad_worker, &jobs[k]);
  for (int k = 0; k < threads; ++k) pthread_join(tid[k], NULL);
  return 0;
}

int orc_sample_region(const orc_tables* ex, const orc_tables* nt, int dist, uint32_t j, uint64_t seed, uint64_t index0,
                      uint64_t n, double* out) {
  const orc_tables* t = (dist == ORC_EXP) ? ex : nt;
  if (t == NULL || ex == NULL || j > t->L) return -1;
  for (uint64_t k = 0; k < n; ++k) {
    slow_stream s;
    seed_key(seed, s.key);
    s.n = index0 + k;
    s.t = 0;
    s.tests = 0;
    out[k] = (dist == ORC_EXP) ? exp_region(ex, j, &s) : normal_region(nt, ex, j, &s);
  }
  return 0;
}
