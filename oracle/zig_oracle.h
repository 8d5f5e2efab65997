/*
 * Scalar CPU oracle for the modified ziggurat sampler (McFarland,
 * "A modified ziggurat algorithm for generating exponentially- and
 * normally-distributed pseudorandom numbers", arXiv:1403.6870).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the correctness reference that
 * the GPU library is checked against.  It shares no source with the GPU
 * library and must never be linked into, loaded by or called from the
 * product path.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.
 *
 * Every quantity here is written straight from the paper's definitions
 * (section 2, its layer equation, Table 1, the overhang split after Table 1
 * and Appendices B and C), with the ambiguous points resolved as listed in
 * zig_oracle.c's header comment.
 */
#ifndef ZIG_ORACLE_H
#define ZIG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EXP = 0, ORC_NORMAL = 1 };
enum { ORC_F64 = 0, ORC_F32 = 1 };

#define ORC_MAX_IMAX 1024

/* Tables of one distribution at one i_max.  Index conventions:
 *   layers   i = 0..L-1 (0 = bottom layer, whose lower-left corner is the
 *            origin), X[L] := 0 and f[L] := 1 close the top cap;
 *   regions  j = 0..L: 0 = tail, 1..L-1 = overhang right of layer j,
 *            L = cap above the top layer;
 *   alias    columns c = 0..i_max-1 with 64-bit thresholds T[c] in units
 *            of 2^-(64-b) and alias index A[c]. */
typedef struct {
  int dist;
  uint32_t i_max, b, L;
  double X[ORC_MAX_IMAX + 1];
  double f[ORC_MAX_IMAX + 1];
  double XS[ORC_MAX_IMAX];     /* X_i * 2^-53, zero for i >= L */
  float XS32[ORC_MAX_IMAX];    /* RN32(X_i) * 2^-(32-s) (exp) or 2^-(31-s) (normal), s = max(b, 8) */
  double W[ORC_MAX_IMAX + 1];  /* box widths  W_j = X_{j-1} - X_j, j = 1..L */
  double H[ORC_MAX_IMAX + 1];  /* box heights H_j = f_j - f_{j-1}, j = 1..L */
  uint64_t q[ORC_MAX_IMAX + 1];/* integer region weights, sum = 2^64 */
  uint64_t T[ORC_MAX_IMAX];
  uint32_t A[ORC_MAX_IMAX];
  double eps;                  /* exp only: max normalised chord gap */
  uint64_t K_eps;              /* exp only: floor((1 - eps) * 2^53) */
  double X0, invX0;
  /* normal only, for the accelerated overhang variant: the largest
   * normalised gap between chord and curve in the convex boxes (X_j >= 1,
   * curve below the chord) and in the concave boxes (X_{j-1} <= 1, curve
   * above), each widened by 2^-20 relatively, as integer thresholds on
   * k1 + k2: K_cvx = floor((1 - eps_cvx) 2^53), K_ccv = ceil((1 + del_ccv) 2^53). */
  double eps_cvx, del_ccv;
  uint64_t K_cvx, K_ccv;
  /* normal only: 1 selects the accelerated overhang variant (set by the
   * caller after building; 0 = plain rejection, the default) */
  int accel;
  /* decimal strings (36 significant digits) of the 113-bit values, for
   * the tests that check the construction in higher precision */
  char hpX[ORC_MAX_IMAX + 1][48];
  char hpf[ORC_MAX_IMAX + 1][48];
  char hpA[ORC_MAX_IMAX + 1][48];
  char hp_area[48], hp_total[48], hp_eps[48], hp_eps_cvx[48], hp_del_ccv[48];
} orc_tables;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Builds the tables of `dist` for i_max in {8,16,32,64,128,256}.
 * Returns 0 on success, -1 on an unsupported argument. */
int orc_build_tables(int dist, uint32_t i_max, orc_tables* t);

/* Fills out[k] (double or float, by dtype) with the sample of global index
 * first + k for k < n, scaled as out = fma(scale, x, shift).  `ex` is the
 * exponential table set (used by the normal tail as well), `nt` the normal
 * one (may be NULL for dist == ORC_EXP).  Uses `threads` POSIX threads over
 * contiguous index ranges; the output does not depend on it. */
int orc_fill(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed,
             uint64_t first, uint64_t n, double scale, double shift, void* out, int threads);

/* Same as orc_fill, single thread, plus a per-output trace:
 *   layer[k] = layer index i drawn from the fast word,
 *   region[k] = region j of the first alias draw (-1 on the fast path),
 *   words[k]  = 64-bit slow-stream words consumed,
 *   tests[k]  = exp() accept/reject evaluations performed.
 * Any trace pointer may be NULL. */
int orc_fill_trace(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed,
                   uint64_t first, uint64_t n, double scale, double shift, void* out, uint32_t* layer,
                   int32_t* region, uint32_t* words, uint32_t* tests);

/* Raw moment sums S_p = sum of x^p, p = 1..5, over the outputs a fill of
 * the same arguments writes (powers by double multiplication: x*x, then
 * *x, squared, *x), each the exact sum rounded once to double, so no order
 * of addition enters; abs_sums (may be NULL) receives sum |x^p| the same
 * way.  Uses `threads` POSIX threads over contiguous index ranges; the
 * result does not depend on it. */
int orc_moments(int dist, int dtype, const orc_tables* ex, const orc_tables* nt, uint64_t seed, uint64_t first,
                uint64_t n, double scale, double shift, double sums[5], double abs_sums[5], int threads);

/* The exact sum of x[0..n-1] rounded once to double (to nearest, ties to
 * even; +0 for an exact zero, NaN if a term is not finite). */
int orc_exact_sum(const double* x, uint64_t n, double* sum);

/* One rejection attempt in overhang/cap box j (1..L) with injected
 * 53-bit integers k1, k2.  Returns 1 and sets *x on acceptance. */
int orc_box_attempt(const orc_tables* t, uint32_t j, uint64_t k1, uint64_t k2, double* x);

/* All attempts of box j on the lattice k1 = a << shift, k2 = c << shift,
 * a, c < g: accept[a*g + c] and the returned x (0 when rejected). */
int orc_box_grid(const orc_tables* t, uint32_t j, uint32_t g, uint32_t shift, uint8_t* accept, double* x);

/* Samples region j (0..L) directly, drawing from the slow stream of
 * (seed, index) from its first word (no alias draw).  Used to test the
 * tail and overhang samplers in isolation.  Writes n draws for the
 * indices index0 .. index0+n-1. */
int orc_sample_region(const orc_tables* ex, const orc_tables* nt, int dist, uint32_t j, uint64_t seed,
                      uint64_t index0, uint64_t n, double* out);

/* The alias draw j(r) for a 64-bit word r. */
uint32_t orc_alias_draw(const orc_tables* t, uint64_t r);

/* ---- traditional ziggurat (Table 1, right column), for the A/B test --
 * n layers of equal area v covering P: layer 0 is the rectangle
 * [0, X_0] x [0, f_0] plus the tail beyond X_0 (width W_0 = v / f_0),
 * layer i >= 1 the rectangle [0, X_{i-1}] x [f_{i-1}, f_i] (width
 * W_i = X_{i-1}), with f_i = P(X_i) and X_{n-1} = 0, f_{n-1} = P(0) = 1;
 * X_0 = r is solved so that the stack closes at the top.  k_i = X_i / W_i
 * is the fraction of layer i that lies wholly under P. */
typedef struct {
  int dist;
  uint32_t n, b;
  double X[ORC_MAX_IMAX + 1];
  double f[ORC_MAX_IMAX + 1];
  double W[ORC_MAX_IMAX];
  double WS[ORC_MAX_IMAX];  /* W_i * 2^-53 */
  double k[ORC_MAX_IMAX];
  double v, r, invr;
  char hp_r[48], hp_v[48];
} orc_trad;

int orc_build_trad(int dist, uint32_t n, orc_trad* t);

/* FP64 fill with the traditional sampler on the same uniform streams as
 * the modified one: output g takes its first (U1, i) from its fast word
 * (index bits 0..b-1, normal sign bit 10, U1 from bits 11..63); a layer's
 * wedge test draws U2, and every restart a new (U1, i), from the output's
 * slow stream, as do the tails (exponential: X_0 plus a fresh traditional
 * exponential; normal: Marsaglia's method on two traditional
 * exponentials).  `words` (may be NULL) receives the slow words used per
 * output. */
int orc_trad_fill(int dist, const orc_trad* ex, const orc_trad* nt, uint64_t seed, uint64_t first, uint64_t n,
                  double scale, double shift, double* out, uint32_t* words, int threads);
uint64_t orc_trad_size(void);

/* Size of orc_tables, so that foreign callers can allocate it. */
uint64_t orc_tables_size(void);

#ifdef __cplusplus
}
#endif
#endif
