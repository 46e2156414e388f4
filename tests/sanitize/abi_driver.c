/* Drives the host side of libht.so's C ABI, for a build of the library's host code with
 * AddressSanitizer and UndefinedBehaviorSanitizer: table and tiling queries, launch-shape
 * settings, batch plans, and argument validation of every entry point with invalid arguments.
 * Every call made here returns before any device work, so the program needs no GPU. Any
 * out-of-bounds access or undefined operation in that host code aborts the program; a wrong
 * status code fails a check. Exit status 0 when everything ran clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ht.h"
#include "ht_debug.h"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      exit(2);                                                        \
    }                                                                 \
  } while (0)

#define EXPECT_EINVAL(call)                  \
  do {                                       \
    CHECK((call) == HT_EINVAL);              \
    CHECK(strlen(ht_last_error()) > 0);      \
  } while (0)

static void tables_of(const ht_grid* g)
{
  float* a2 = malloc(sizeof(float) * (size_t)g->n_a);
  float* phi = malloc(sizeof(float) * 4 * (size_t)g->n_phi);
  float* th = malloc(sizeof(float) * (4 * (size_t)g->n_theta + 2));
  float inv = 0.0f;
  CHECK(ht_tables(g, a2, &inv, phi, th) == HT_OK);
  CHECK(isfinite(inv) && inv > 0.0f);
  for (int i = 1; i < g->n_a; ++i) CHECK(a2[i] > a2[i - 1]);
  free(a2);
  free(phi);
  free(th);
}

int main(void)
{
  const ht_grid paper = {4, 16, 1024, 1024, -2000.f, 2000.f, -2000.f, 2000.f, 9, 0};
  const ht_grid small = {4, 16, 64, 64, -2000.f, 2000.f, -2000.f, 2000.f, 8, 0};
  const ht_grid stress = {8, 32, 2048, 2048, -2000.f, 2000.f, -2000.f, 2000.f, 9, 0};
  const ht_grid sectors = {4, 4, 1024, 1024, -2000.f, 2000.f, -2000.f, 2000.f, 9, 1};
  const ht_grid wide = {1, 3, 8, 65536, -2000.f, 2000.f, -2000.f, 2000.f, 2, 0};
  const ht_grid ragged = {3, 5, 7, 9, -1500.f, 1300.f, -1100.f, 1700.f, 2, 0};
  const ht_grid* grids[] = {&paper, &small, &stress, &sectors, &wide, &ragged};

  for (size_t i = 0; i < sizeof(grids) / sizeof(grids[0]); ++i) {
    tables_of(grids[i]);
    int32_t rows = 0, n_tiles = 0, cap = 0, lds = 0;
    CHECK(ht_tiling(grids[i], &rows, &n_tiles, &cap, &lds) == HT_OK);
    CHECK(rows >= 1 && n_tiles >= 1 && cap >= 1);
    ht_tuning t;
    CHECK(ht_get_tuning(grids[i], &t) == HT_OK);
  }
  CHECK(ht_tiling(&wide, NULL, NULL, NULL, NULL) == HT_OK);

  /* invalid grids */
  ht_grid bad = small;
  bad.n_phi = 2;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.a_max = NAN;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.b_min = bad.b_max;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.threshold = 0;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.n_a = (1 << 24) + 1;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.n_theta = 64; bad.n_phi = 65;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = stress; bad.n_b = 16384;  /* 2^33 cells */
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  bad = small; bad.phi_sectors = 2;
  EXPECT_EINVAL(ht_tiling(&bad, NULL, NULL, NULL, NULL));
  EXPECT_EINVAL(ht_tiling(NULL, NULL, NULL, NULL, NULL));
  EXPECT_EINVAL(ht_tables(&small, NULL, NULL, NULL, NULL));

  /* launch shapes */
  ht_tuning tu = {4, 32, 128, 2, 16};
  CHECK(ht_set_tuning(&paper, &tu) == HT_OK);
  ht_tuning got;
  CHECK(ht_get_tuning(&paper, &got) == HT_OK);
  CHECK(got.rows == 4 && got.group_tiles == 32 && got.cand_cap == 128 && got.nt_store == 2 &&
        got.tiles_per_block == 16);
  const ht_tuning bad_tunings[] = {{3, 0, 0, -1, 0}, {128, 0, 0, -1, 0}, {0, 24, 0, -1, 0},
                                   {0, 0, 100, -1, 0}, {0, 0, 8192, -1, 0}, {0, 0, 0, 3, 0},
                                   {0, 0, 0, -2, 0}, {0, 0, 0, -1, 3}, {0, 0, 0, -1, 128},
                                   {-1, 0, 0, -1, 0}};
  for (size_t i = 0; i < sizeof(bad_tunings) / sizeof(bad_tunings[0]); ++i)
    EXPECT_EINVAL(ht_set_tuning(&paper, &bad_tunings[i]));
  CHECK(ht_set_tuning(&paper, NULL) == HT_OK);
  EXPECT_EINVAL(ht_get_tuning(&paper, NULL));

  /* batch plans: the paper grid keeps direct lists, sixteen stress events take the counting sort */
  ht_event evs[100];
  for (int i = 0; i < 100; ++i) {
    evs[i].hit_offset = 0;
    evs[i].n_hits = 1000 + 70 * i;
    evs[i].peak_offset = 0;
    evs[i].peak_capacity = 0;
  }
  int32_t direct = -1;
  int64_t bytes = 0;
  CHECK(ht_debug_batch_plan(&paper, evs, 100, &direct, &bytes) == HT_OK && direct == 1 && bytes > 0);
  for (int i = 0; i < 16; ++i) evs[i].n_hits = 105600;
  CHECK(ht_debug_batch_plan(&stress, evs, 16, &direct, &bytes) == HT_OK && direct == 0);
  evs[0].n_hits = 0;
  CHECK(ht_debug_batch_plan(&small, evs, 1, &direct, &bytes) == HT_OK);
  evs[0].n_hits = -1;
  EXPECT_EINVAL(ht_debug_batch_plan(&small, evs, 1, &direct, &bytes));
  evs[0].n_hits = ((int64_t)1 << 28) + 1;
  EXPECT_EINVAL(ht_debug_batch_plan(&small, evs, 1, &direct, &bytes));
  EXPECT_EINVAL(ht_debug_batch_plan(&small, evs, 0, &direct, &bytes));
  EXPECT_EINVAL(ht_debug_batch_plan(&small, NULL, 1, &direct, &bytes));

  /* argument checks that come before any device work */
  float dummy[4];
  uint32_t acc[4];
  ht_peak out[4];
  int64_t nf[1];
  EXPECT_EINVAL(ht_fill(&small, dummy, dummy, dummy, -1, acc, NULL));
  EXPECT_EINVAL(ht_fill(&small, dummy, dummy, dummy, 4, NULL, NULL));
  EXPECT_EINVAL(ht_fill(&small, NULL, dummy, dummy, 4, acc, NULL));
  EXPECT_EINVAL(ht_fill(&small, dummy, dummy, dummy, ((int64_t)1 << 28) + 1, acc, NULL));
  EXPECT_EINVAL(ht_fill(&bad, dummy, dummy, dummy, 4, acc, NULL));
  EXPECT_EINVAL(ht_fill_atomic(&small, dummy, dummy, dummy, -5, acc, NULL));
  EXPECT_EINVAL(ht_peaks(&small, acc, out, -1, nf, NULL));
  EXPECT_EINVAL(ht_peaks(&small, acc, NULL, 4, nf, NULL));
  EXPECT_EINVAL(ht_peaks(&small, acc, out, 4, NULL, NULL));
  EXPECT_EINVAL(ht_fill_peaks(&small, dummy, dummy, dummy, -1, acc, out, 4, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_noalloc(&small, dummy, dummy, dummy, -1, acc, out, 4, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_noalloc(&small, dummy, dummy, dummy, 4, NULL, out, 4, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_noalloc(&small, dummy, dummy, dummy, 4, acc, out, -1, nf, NULL));
  ht_grid many_a = small;
  many_a.n_a = 32768;
  EXPECT_EINVAL(ht_fill_peaks_noalloc(&many_a, dummy, dummy, dummy, 4, acc, out, 4, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_batch(&small, evs, -1, dummy, dummy, dummy, acc, out, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_batch(&small, evs, 65536, dummy, dummy, dummy, acc, out, nf, NULL));
  EXPECT_EINVAL(ht_fill_peaks_batch(&small, NULL, 1, dummy, dummy, dummy, acc, out, nf, NULL));
  evs[0].n_hits = 4;
  evs[0].hit_offset = -1;
  EXPECT_EINVAL(ht_fill_peaks_batch(&small, evs, 1, dummy, dummy, dummy, acc, out, nf, NULL));
  evs[0].hit_offset = 0;
  EXPECT_EINVAL(ht_fill_peaks_batch(&small, evs, 1, NULL, NULL, NULL, acc, out, nf, NULL));
  CHECK(ht_fill_peaks_batch(&small, evs, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == HT_OK);
  EXPECT_EINVAL(ht_readout(&small, NULL, nf, -1, NULL, NULL));
  EXPECT_EINVAL(ht_readout(&small, NULL, NULL, 0, NULL, NULL));

  /* request loop: invalid options and handles */
  ht_serve_opts o = {1 << 30, 1024, 5000, 8, 2, 16, 0};
  ht_server* sv = (ht_server*)1;
  EXPECT_EINVAL(ht_serve_create(&small, &o, NULL));
  o.max_batch = 0;
  EXPECT_EINVAL(ht_serve_create(&small, &o, &sv));
  CHECK(sv == NULL);
  o.max_batch = 8;
  o.n_streams = 17;
  EXPECT_EINVAL(ht_serve_create(&small, &o, &sv));
  o.n_streams = 2;
  o.queue_depth = 0;
  EXPECT_EINVAL(ht_serve_create(&small, &o, &sv));
  o.queue_depth = 16;
  o.hbm_budget_bytes = 0;
  EXPECT_EINVAL(ht_serve_create(&small, &o, &sv));
  EXPECT_EINVAL(ht_serve_create(&bad, &o, &sv));
  uint64_t ticket = 0;
  EXPECT_EINVAL(ht_serve_submit(NULL, dummy, dummy, dummy, 4, &ticket));
  EXPECT_EINVAL(ht_serve_poll(NULL, 1, out, 4, nf, NULL));
  CHECK(ht_serve_destroy(NULL) == HT_OK);

  /* diagnostics */
  EXPECT_EINVAL(ht_profile_enable(3));
  double ms = 0.0;
  int64_t count = 0;
  EXPECT_EINVAL(ht_profile_read(NULL, &ms, &count, 0));
  int32_t kind = 0;
  EXPECT_EINVAL(ht_debug_pointer_kind(NULL, &kind));
  EXPECT_EINVAL(ht_debug_unary(dummy, dummy, dummy, -1, NULL));
  CHECK(ht_debug_unary(NULL, NULL, NULL, 0, NULL) == HT_OK);
  int32_t info[4];
  int32_t slabs[4];
  EXPECT_EINVAL(ht_debug_hit_values(&small, dummy, dummy, dummy, -1, info, dummy, slabs, NULL));
  CHECK(ht_bench_hbm_write(NULL, 16, 0, NULL) == HT_EINVAL);
  CHECK(ht_bench_hbm_write(dummy, 15, 0, NULL) == HT_EINVAL);
  CHECK(ht_bench_hbm_write(dummy, 16 * 1024 + 16, 3, NULL) == HT_EINVAL);  /* tiles: whole 16 KiB */
  CHECK(ht_bench_hbm_write(dummy, 16 * 1024, 5, NULL) == HT_EINVAL);
  CHECK(ht_bench_atomic_rand(acc, 0, 1, NULL) == HT_EINVAL);
  CHECK(ht_bench_lds_atomic(0, 1, acc, NULL) == HT_EINVAL);
  printf("abi driver: clean\n");
  return 0;
}
