/* Runs the oracle's entry points on small inputs, for a sanitizer build by
 * test_host_sanitizers.py: every table size of both distributions, fills
 * of both output types with 1 and 4 threads (which must agree), the traced
 * fill, box attempts and a box lattice.  Prints "ok" on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/zig_oracle.h"

int main(void) {
  static orc_tables ex, nt;
  const uint32_t sizes[] = {8, 16, 32, 64, 128, 256};
  for (int s = 0; s < 6; ++s) {
    if (orc_build_tables(ORC_EXP, sizes[s], &ex) || orc_build_tables(ORC_NORMAL, sizes[s], &nt)) {
      printf("FAIL tables %u\n", sizes[s]);
      return 1;
    }
    const uint64_t n = 5000;
    double* a = malloc(n * sizeof(double));
    double* b = malloc(n * sizeof(double));
    uint32_t* layer = malloc(n * sizeof(uint32_t));
    int32_t* region = malloc(n * sizeof(int32_t));
    uint32_t* words = malloc(n * sizeof(uint32_t));
    uint32_t* tests = malloc(n * sizeof(uint32_t));
    for (int dist = 0; dist < 2; ++dist)
      for (int dtype = 0; dtype < 2; ++dtype) {
        memset(a, 0, n * sizeof(double));
        memset(b, 0, n * sizeof(double));
        orc_fill(dist, dtype, &ex, &nt, 99, 12345, n, 1.5, -0.5, a, 1);
        orc_fill(dist, dtype, &ex, &nt, 99, 12345, n, 1.5, -0.5, b, 4);
        if (memcmp(a, b, n * (dtype ? 4 : 8)) != 0) {
          printf("FAIL thread count changed the output\n");
          return 1;
        }
        orc_fill_trace(dist, dtype, &ex, &nt, 99, 12345, n, 1.5, -0.5, b, layer, region, words, tests);
        if (memcmp(a, b, n * (dtype ? 4 : 8)) != 0) {
          printf("FAIL trace fill differs\n");
          return 1;
        }
      }
    free(a);
    free(b);
    free(layer);
    free(region);
    free(words);
    free(tests);
  }
  double x = 0.0;
  for (uint32_t j = 1; j <= ex.L; j += 17) orc_box_attempt(&ex, j, (uint64_t)j << 40, (uint64_t)j << 41, &x);
  uint8_t acc[64 * 64];
  double xs[64 * 64];
  orc_box_grid(&nt, 5, 64, 47, acc, xs);
  printf("ok\n");
  return 0;
}
