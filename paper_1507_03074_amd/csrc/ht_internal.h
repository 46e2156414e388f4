// ht_internal.h -- types shared by the translation units of libht.so (kernels, C ABI, server).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "ht.h"

namespace ht {

// Largest number of (theta, phi) cells (slabs); their counters live in LDS during the prep.
constexpr int kMaxSlabs = 4096;
// Per-event slab counters: a pair of arrays used alternately by successive calls. A call counts
// into the array that is zero and clears the other one for the next call, so no call needs a
// separate clearing launch. They live in memory of their own, cleared once when allocated.
// Each array holds kMaxSlabs slab counters followed by the candidate-pool cursor, the marker
// of the one pool reservation that crosses the pool's end (pool_cap + 1 - its start, 0 if
// none) and the number of tiles whose candidates did not fit.
constexpr int kCounterWords = kMaxSlabs + 64;
constexpr int kPoolCounter = kMaxSlabs;
constexpr int kPoolCut = kMaxSlabs + 1;
constexpr int kOvfCounter = kMaxSlabs + 2;
constexpr size_t kCounterBytes = 2 * sizeof(uint32_t) * kCounterWords;
// tile_off value of a tile whose candidates did not fit the pool (searched densely instead)
constexpr uint32_t kTileOverflow = 0xffffffffu;
// Direct slab lists (one fixed-capacity list per slab, capacity = the event's hit count) are
// used while they need at most this many bytes per event; above it, a counting sort.
constexpr size_t kDirectListMax = (size_t)1 << 29;
// A batch uses direct lists only while the scratch of all its events stays within this.
constexpr size_t kBatchDirectMax = (size_t)8 << 30;

// Grid constants and tables as the kernels see them (passed by value as a kernel argument).
struct DevGrid {
  int32_t n_theta, n_phi, n_a, n_b;
  float b_min;
  float inv_db;     // (float)(n_b / (b_max - b_min))
  float nb_f;       // (float)n_b, exact because n_b <= 2^24
  uint32_t threshold;
  int32_t n_slabs;         // n_theta * n_phi: one (A, B) slab per (theta, phi) cell
  int32_t rows;            // A rows per tile; a tile is rows x n_b contiguous cells of one slab
  int32_t tiles_per_slab;  // ceil(n_a / rows)
  int32_t n_tiles;         // n_slabs * tiles_per_slab
  int32_t cand_cap;        // candidate-pool entries per tile (the pool is shared by all tiles)
  int32_t lds_fill;        // 1: fill through an LDS tile; 0: global atomics (very wide B rows)
  int32_t group_tiles;     // tiles per workgroup of the peak search (16, 32 or 64)
  int32_t nt_store;        // fill store kind: 0 16-byte, 1 non-temporal 16-byte, 2 4-byte
  int32_t fill_tiles;      // fill tiles per workgroup (filled in turn)
  int32_t pool_bound;      // 1: large events get a candidate pool sized by their vote bound
  int32_t phi_sectors;     // 1: phi cells are independent sectors (no phi widening or neighbours)
  int32_t packed_lists;    // 1: always the counting-sort (packed) slab lists, never direct ones
  int32_t test_blocks;     // workgroups per event of the candidate test
  int32_t dense_w;         // 1: the stencil peak search is available on this grid (0: not)
  int32_t dense_rows;      // A rows per workgroup of the stencil peak search (a multiple of 12)
  int32_t dense_hits;      // events with at least this many hits take the stencil (0: never)
  const float* a2;         // device [n_a]
  const float* phi_cs;     // device [2 * 2 n_phi] (cos, sin)
  const float* th_cs;      // device [2 * (2 n_theta + 1)] (cos, sin)
};

// One event's inputs, outputs and scratch (device pointers).
struct EvDesc {
  const float* x;
  const float* y;
  const float* z;
  int64_t n_hits;
  uint32_t* acc;        // [cells]
  ht_peak* out;         // [cap]
  int64_t cap;
  int64_t* n_found;     // [1]
  // scratch
  uint32_t* slab_cnt;       // [n_slabs] counters of this call, zero on entry (kCounterBytes)
  uint32_t* slab_cnt_next;  // [n_slabs] the other counter array, cleared by this call
  int64_t list_cap;         // > 0: direct lists, list_cap records per slab; 0: counting sort
  uint32_t* slab_off;       // [n_slabs + 1] (counting sort)
  int32_t* hit_slab;    // [4 n_hits] slab of each (hit, cell) or -1
  uint32_t* hit_pos;    // [4 n_hits] position of the (hit, cell) in its slab list
  float4* hit_rec;      // [n_hits] (x, r2, k, 0)
  float4* list;         // hit records bucketed by slab: [n_slabs * list_cap] or [4 n_hits]
  uint32_t* tile_cnt;   // [n_tiles] candidates (cells >= threshold) per tile
  uint32_t* tile_off;   // [n_tiles] first pool entry of each tile's candidates, or kTileOverflow
  uint2* pool;          // [pool_cap] (cell, votes) of the candidates, ascending within a tile
  uint32_t pool_cap;    // entries: at least n_tiles * cand_cap, more for large events
  uint8_t* pk_flag;     // [pool_cap] 1 if the pool entry is a peak
  uint32_t* ovf_list;   // [n_tiles] tiles whose candidates did not fit the pool
  uint32_t* tile_pk;    // [n_tiles] peaks per tile
  uint32_t* group_pk;   // [n_groups] peaks per group of tiles
  int32_t dense;        // 1: peaks from the stencil over the matrix (crowded events), not the pool
  uint8_t* pk_mask;     // 64-bit words of peak bits of a dense event, kChunkCells cells per
                        // (slab, row, chunk) word, stored by the stencil's workgroups
};

// B columns tested per wave of the stencil peak search: a wave64 holds them and the cell on
// either side.
constexpr int kChunkCells = 62;

// Launch shape of one grid (ht_tuning resolved against the defaults).
struct Tiling {
  int32_t rows, tiles_per_slab, n_tiles, cand_cap, lds_fill, group_tiles, nt_store, fill_tiles;
  int32_t pool_bound;
  int32_t packed_lists;
  int32_t dense_w, dense_rows, dense_hits;  // stencil peak search (DevGrid fields of these names)
};
Tiling choose_tiling(const ht_grid& g);

// Device copies of the bin-rule tables of one grid.
struct DevTables {
  float* a2 = nullptr;
  float* phi = nullptr;
  float* th = nullptr;
  float inv_db = 0.0f;
};
// Floats of each table: a2[n_a], phi (cos, sin)[2 n_phi], theta (cos, sin)[2 n_theta + 1].
inline size_t a2_floats(const ht_grid& g) { return (size_t)g.n_a; }
inline size_t phi_floats(const ht_grid& g) { return 4 * (size_t)g.n_phi; }
inline size_t th_floats(const ht_grid& g) { return 2 * (2 * (size_t)g.n_theta + 1); }
// The tables computed on the host in double and rounded once to float, into caller arrays of
// the sizes above.
void host_tables_into(const ht_grid& g, float* a2, float* inv_db, float* phi, float* th);
DevGrid make_devgrid(const ht_grid& g, const DevTables& t, const Tiling& tl);

// Whether an event of n_hits hits uses direct slab lists (see kDirectListMax).
bool direct_lists(const DevGrid& g, int64_t n_hits);
// Whether the fused fill + peaks of an event of n_hits hits searches its peaks with the stencil
// over the matrix (crowded events) instead of the candidate pool.
bool dense_peaks(const DevGrid& g, int64_t n_hits);
// What an event's peak-search scratch holds: the candidate pool, the stencil's peak mask, or
// both (request-loop slots, which serve events of either kind).
enum PeakScratch { kPeakPool = 1, kPeakMask = 2 };
// Bytes of per-event scratch for a grid tiling and an event size, and the carving of it.
size_t event_scratch_bytes(const DevGrid& g, int64_t n_hits, bool direct, int peaks = kPeakPool);
void carve_event_scratch(const DevGrid& g, int64_t n_hits, bool direct, char* base, EvDesc* ev,
                         int peaks = kPeakPool);

// Kernel launchers (ht_kernels.hip). `evs` is a device array of n_ev descriptors, or nullptr
// for a single event passed by value in `ev0`. `max_hits` bounds n_hits over the events.
hipError_t launch_prep(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                       int64_t max_hits, bool direct, hipStream_t s);
hipError_t launch_fill(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                       bool emit_candidates, int64_t max_hits, hipStream_t s);
hipError_t launch_candidates(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                             hipStream_t s);
hipError_t launch_peaks(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                        hipStream_t s);
// Stencil peak search and ordered write of the events marked dense (others are skipped).
hipError_t launch_peaks_dense(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                              hipStream_t s);
// Plain fill: zero the matrix, then one global atomicAdd per vote (reference path and the
// fallback for B rows too wide for an LDS tile).
hipError_t launch_fill_atomic(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                              int64_t max_hits, hipStream_t s);

hipError_t launch_readout(const DevGrid& g, const ht_peak* peaks, const int64_t* n_found, int64_t cap,
                          ht_track* tracks, double b_min, double db, hipStream_t s);

size_t fill_lds_bytes(const DevGrid& g);
int n_groups(const DevGrid& g);

// Host helpers (ht_api.cpp).
// 0: not usable by a kernel; 1: device memory; 2: pinned host memory mapped into the device;
// 3: managed memory.
int pointer_kind(const void* ptr);
int check_accessible(const void* ptr, const char* what);
// Enqueues one event's stages on s: prep (counting into ev.slab_cnt and clearing
// ev.slab_cnt_next), then the fill, then the peak search, as do_fill / do_peaks ask; `atomic`
// takes the global-atomic fill and a candidate scan of the matrix. *counters_used is set once
// a kernel that uses the counter pair is on the stream (the caller then flips to the other
// array for its next call). `timed` records the stage timers of ht_profile_enable.
int enqueue_event(const DevGrid& g, const EvDesc& ev, int64_t n_hits, bool direct, bool atomic,
                  bool do_fill, bool do_peaks, bool timed, hipStream_t s, bool* counters_used);
int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);
int validate_grid(const ht_grid* g);
uint64_t n_cells(const ht_grid& g);
// Validates the grid, uploads its tables once per device and picks the tiling.
int make_device_grid(const ht_grid& g, int dev, DevGrid* out);
// The whole batched pipeline (prep, fill with candidates, peaks) for n_ev events whose
// descriptors are already in device memory.
// *prep_enqueued is set once the preparation (which counts into and clears the events' counter
// arrays) is on the stream.
// A batch split into runs of events whose peak searches run on a side stream beside the next
// run's fill (pieces <= kMaxPieces; pieces 1: no split).
constexpr int kMaxPieces = 8;
struct BatchSplit {
  int pieces;
  hipStream_t side;
  hipEvent_t filled[kMaxPieces];  // recorded on the launch stream after each run's fill
  hipEvent_t done;                // recorded on the side stream after the last peak search
};
// any_pool / any_dense: whether some event searches its peaks through the candidate pool /
// the stencil (only the kernels needed are launched). split: NULL, or how to overlap.
int launch_batch(const DevGrid& g, const EvDesc* d_ev, int n_ev, int64_t max_hits, bool direct,
                 bool any_pool, bool any_dense, hipStream_t s, bool* prep_enqueued,
                 const BatchSplit* split = nullptr);

}  // namespace ht
