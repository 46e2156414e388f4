/*
 * ht_debug.h -- diagnostic entry points of libht.so, for parity tests of intermediate values.
 * They run the same device code as the product path and are not needed to use the library.
 */
#ifndef HT_DEBUG_H_
#define HT_DEBUG_H_

#include <stdint.h>

#include "ht.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ht_debug_hit_values: the per-hit steps of the bin rule (validity, r2, r = sqrt(r2),
 * k = 1/(2y), theta and phi half-sectors, (theta, phi) cells; see ht.h) computed by the same
 * device function the fill uses, for n_hits hits.
 * x, y, z: device float[n_hits]. info: device int32[4*n_hits] = {valid, s_theta, s_phi, n_cells};
 * vals: device float[3*n_hits] = {r2, r, k} (zeros for invalid hits); slabs: device
 * int32[4*n_hits], the cells as slab indices t*n_phi + p, padded with -1. Asynchronous on stream.
 * Errors: HT_EINVAL, HT_EDEVICE. */
int ht_debug_hit_values(const ht_grid* grid, const float* x, const float* y, const float* z,
                        int64_t n_hits, int32_t* info, float* vals, int32_t* slabs, void* stream);

/* ht_debug_unary: the two correctly rounded operations of the per-hit values (bin rule O2),
 * computed by the same device functions the preparation uses: root[i] = sqrtf(v[i]) and
 * inv2[i] = 1.0f / (v[i] + v[i]), each one IEEE binary32 operation rounded to nearest even (v + v
 * is exact below overflow). Meant for checking them against the host over every binary32 input.
 * v, root, inv2: float[n], device memory or mapped pinned host memory, caller-owned.
 * Asynchronous on stream. Errors: HT_EINVAL (n < 0, NULL or unusable pointers), HT_EDEVICE. */
int ht_debug_unary(const float* v, float* root, float* inv2, int64_t n, void* stream);

/* ht_debug_pointer_kind: how the library classifies a pointer given as a peak output, from the
 * HIP runtime's attributes (host only, no device work): 0 = refused (not usable by a kernel,
 * e.g. unregistered host memory), 1 = device memory, 2 = pinned host memory mapped into the
 * device, 3 = managed memory. Errors: HT_EINVAL for NULL arguments. */
int ht_debug_pointer_kind(const void* ptr, int32_t* kind);

/* ht_fill_atomic: step 1 through the plain kernel (zero the matrix, then one global atomicAdd
 * per vote, one block per hit with its threads over the A bins, as the paper's first kernel is
 * organised). Same contract and results as ht_fill; kept as the baseline it is measured against. */
int ht_fill_atomic(const ht_grid* grid, const float* x, const float* y, const float* z,
                   int64_t n_hits, uint32_t* acc, void* stream);

/* ht_tiling: the tile shape the library uses for a grid: rows = A rows per tile,
 * n_tiles = tiles over the whole matrix, cand_cap = candidate slots per tile,
 * lds_fill = 1 when the fill goes through LDS tiles. Host only. */
int ht_tiling(const ht_grid* grid, int32_t* rows, int32_t* n_tiles, int32_t* cand_cap,
              int32_t* lds_fill);

/* ht_debug_batch_plan: the slab-list layout ht_fill_peaks_batch picks for these events on this
 * grid at the current launch shape, computed on the host with the same code (no device work):
 * *direct = 1 for direct per-slab lists, 0 for the counting sort into packed lists (used when
 * an event's direct lists would pass 512 MiB or all events' scratch would pass 8 GiB);
 * *scratch_bytes = the device scratch the batch needs. events: host ht_event[n_events].
 * Errors: HT_EINVAL (grid, events, n_events outside [1, 65535], NULL outputs). */
int ht_debug_batch_plan(const ht_grid* grid, const ht_event* events, int32_t n_events,
                        int32_t* direct, int64_t* scratch_bytes);

/* ht_profile_enable: per-stage timing of later calls. mode 1: a HIP event (created without the
 * system-scope fence) is recorded on the call's stream before and after each stage ("prep",
 * "fill", "fill_atomic", "candidates", "peaks"); mode 2: around the fill stages only ("fill",
 * "fill_atomic"); 0 turns it off. Graph-captured calls are not timed. Host only; HT_EINVAL for
 * another mode. */
int ht_profile_enable(int mode);

/* ht_profile_read: waits for the recorded events of stage `name` and returns their summed
 * duration (*total_ms) and count; reset != 0 then drops all records. Errors: HT_EINVAL,
 * HT_EDEVICE. */
int ht_profile_read(const char* name, double* total_ms, int64_t* count, int reset);

/* Roofline microbenchmarks: one launch each on `stream` (the caller times it); device buffers.
 * They measure the ceilings the fill and the peak search are compared with.
 * ht_bench_hbm_write: stores over buf[bytes] (bytes a multiple of 16); mode 0: non-temporal
 *   16-byte stores, 1: ordinary 16-byte stores, 2: ordinary 4-byte stores, all three in a
 *   grid-stride loop; 3 (non-temporal) and 4 (ordinary): 16-byte stores tile by tile, one
 *   workgroup per 16 KiB tile as the fill writes the matrix (bytes a multiple of 16 KiB).
 * ht_bench_hbm_read: non-temporal 16-byte loads over buf[bytes]; sink: device uint32[1].
 * ht_bench_copy: dst[bytes] = src[bytes]; the reference kernel for hardware byte counters.
 * ht_bench_atomic_rand: n_ops no-return atomicAdd(+1) on 32-bit words at hashed-uniform
 *   indices of buf[n_words] (n_words <= 2^32 - 1).
 * ht_bench_lds_atomic: `blocks` workgroups of 256 threads, each thread doing `iters` LDS
 *   ds_add_u32 at pseudo-random addresses of a 32 KiB array; sink: device uint32[1].
 * Errors: HT_EINVAL for bad sizes or null pointers, HT_EDEVICE for a failed launch. */
int ht_bench_hbm_write(void* buf, int64_t bytes, int32_t mode, void* stream);
int ht_bench_hbm_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream);
int ht_bench_copy(void* dst, const void* src, int64_t bytes, void* stream);
int ht_bench_atomic_rand(uint32_t* buf, int64_t n_words, int64_t n_ops, void* stream);
int ht_bench_lds_atomic(int32_t blocks, int32_t iters, uint32_t* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HT_DEBUG_H_ */
