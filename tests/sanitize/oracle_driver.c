/* Drives the CPU oracle (oracle/ht_oracle.c, compiled into the same program) over small grids,
 * ragged grids, sector grids and degenerate hits, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, leak-free misuse or undefined operation
 * in the oracle aborts the program. It also checks a few facts that hold whatever the inputs
 * (the vote total equals the matrix sum, peaks are sorted, at or above the threshold and at
 * most the capacity). Exit status 0 when everything ran clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_grid {
  int32_t n_theta, n_phi, n_a, n_b;
  float a_min, a_max, b_min, b_max;
  uint32_t threshold;
  int32_t phi_sectors;
} oracle_grid;

int oracle_check_grid(const oracle_grid* g);
int oracle_tables(const oracle_grid* g, float* a2, float* inv_db, float* phi_cs, float* th_cs);
int oracle_hit_info(const oracle_grid* g, const float* x, const float* y, const float* z,
                    int64_t n, int32_t* info, float* vals, int32_t* cells_tp);
int64_t oracle_fill(const oracle_grid* g, const float* x, const float* y, const float* z,
                    int64_t n, uint32_t* M);
int64_t oracle_peaks(const oracle_grid* g, const uint32_t* M, uint32_t* out_cell,
                     uint32_t* out_votes, int64_t capacity);
int oracle_readout(const oracle_grid* g, const uint32_t* cells, int64_t n, double* out);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(double lo, double hi)
{
  /* xorshift64*: a small counter-free generator for the driver's inputs */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  const uint64_t r = rng_state * 2685821657736338717ull;
  return lo + (hi - lo) * ((double)(r >> 11) / 9007199254740992.0);
}

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      exit(2);                                                        \
    }                                                                 \
  } while (0)

static void run_grid(oracle_grid g, int n_hits)
{
  CHECK(oracle_check_grid(&g) == 0);
  const int64_t cells = (int64_t)g.n_theta * g.n_phi * g.n_a * g.n_b;
  float* x = malloc(sizeof(float) * (size_t)(n_hits + 1));
  float* y = malloc(sizeof(float) * (size_t)(n_hits + 1));
  float* z = malloc(sizeof(float) * (size_t)(n_hits + 1));
  for (int i = 0; i < n_hits; ++i) {
    x[i] = (float)uniform(-1200.0, 1200.0);
    y[i] = (float)uniform(-1200.0, 1200.0);
    z[i] = (float)uniform(-3000.0, 3000.0);
    switch (i % 17) { /* degenerate hits: they vote nothing */
      case 3: x[i] = NAN; break;
      case 5: y[i] = 0.0f; break;
      case 7: z[i] = INFINITY; break;
      case 11: x[i] = 0.0f; y[i] = -0.0f; break;
      case 13: x[i] = 3.0e38f; y[i] = 3.0e38f; break; /* r2 overflows */
      default: break;
    }
  }
  uint32_t* M = malloc(sizeof(uint32_t) * (size_t)cells);
  const int64_t votes = oracle_fill(&g, x, y, z, n_hits, M);
  CHECK(votes >= 0);
  int64_t sum = 0;
  for (int64_t c = 0; c < cells; ++c) sum += M[c];
  CHECK(sum == votes);
  const int64_t cap = 64;
  uint32_t* pc = malloc(sizeof(uint32_t) * (size_t)cap);
  uint32_t* pv = malloc(sizeof(uint32_t) * (size_t)cap);
  const int64_t found = oracle_peaks(&g, M, pc, pv, cap);
  CHECK(found >= 0);
  const int64_t k = found < cap ? found : cap;
  for (int64_t i = 0; i < k; ++i) {
    CHECK(pv[i] >= g.threshold && pv[i] == M[pc[i]]);
    if (i) CHECK(pc[i] > pc[i - 1]);
  }
  CHECK(oracle_peaks(&g, M, NULL, NULL, 0) == found);
  double* ro = malloc(sizeof(double) * 9 * (size_t)(k + 1));
  CHECK(oracle_readout(&g, pc, k, ro) == 0);
  int32_t* info = malloc(sizeof(int32_t) * 4 * (size_t)(n_hits + 1));
  float* vals = malloc(sizeof(float) * 3 * (size_t)(n_hits + 1));
  int32_t* tp = malloc(sizeof(int32_t) * 8 * (size_t)(n_hits + 1));
  CHECK(oracle_hit_info(&g, x, y, z, n_hits, info, vals, tp) == 0);
  float* a2 = malloc(sizeof(float) * (size_t)g.n_a);
  float* phi = malloc(sizeof(float) * 4 * (size_t)g.n_phi);
  float* th = malloc(sizeof(float) * (4 * (size_t)g.n_theta + 2));
  float inv_db = 0.0f;
  CHECK(oracle_tables(&g, a2, &inv_db, phi, th) == 0);
  free(a2); free(phi); free(th);
  free(info); free(vals); free(tp); free(ro);
  free(pc); free(pv); free(M); free(x); free(y); free(z);
}

int main(void)
{
  const oracle_grid base = {4, 16, 64, 64, -2000.f, 2000.f, -2000.f, 2000.f, 8, 0};
  run_grid(base, 250);
  run_grid(base, 0);
  oracle_grid g = base;
  g.n_theta = 3; g.n_phi = 5; g.n_a = 7; g.n_b = 9; g.threshold = 2;
  g.a_min = -1500.f; g.a_max = 1300.f; g.b_min = -1100.f; g.b_max = 1700.f;
  run_grid(g, 300);
  g = base; g.n_theta = 1; g.n_phi = 3; g.n_a = 1; g.n_b = 1; g.threshold = 1;
  run_grid(g, 40);
  g = base; g.n_phi = 4; g.phi_sectors = 1; g.threshold = 3;
  run_grid(g, 200);
  g = base; g.n_phi = 1; g.phi_sectors = 1; g.n_theta = 2; g.threshold = 2;
  run_grid(g, 100);
  g = base; g.n_a = 3; g.n_b = 20000; g.n_theta = 2; g.n_phi = 4; g.threshold = 2;
  run_grid(g, 60);
  /* invalid grids are refused */
  oracle_grid bad = base;
  bad.n_phi = 2;
  CHECK(oracle_check_grid(&bad) != 0);
  bad = base; bad.a_min = NAN;
  CHECK(oracle_check_grid(&bad) != 0);
  bad = base; bad.threshold = 0;
  CHECK(oracle_check_grid(&bad) != 0);
  bad = base; bad.n_a = 1 << 25;
  CHECK(oracle_check_grid(&bad) != 0);
  bad = base; bad.n_theta = 1024; bad.n_phi = 1024; bad.n_a = 1024; bad.n_b = 1024;
  CHECK(oracle_check_grid(&bad) != 0);
  CHECK(oracle_fill(&base, NULL, NULL, NULL, -1, NULL) < 0);
  CHECK(oracle_peaks(&base, NULL, NULL, NULL, -1) < 0);
  printf("oracle driver: clean\n");
  return 0;
}
