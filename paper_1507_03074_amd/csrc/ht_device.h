// ht_device.h -- device code shared by the kernel translation units of libht.so: memory
// helpers, wave and block scans, the candidate pooling of an LDS tile, and the fill kernel
// template (its row counts are instantiated in separate translation units so that they compile
// in parallel).
//
// Every floating-point step of the bin rule is one binary32 operation, rounded to nearest even,
// in the documented order: contraction is off wherever this header is included.
#pragma once

#include "ht_internal.h"

#pragma clang fp contract(off)

namespace ht {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
static_assert(kBlock == 256, "candidate emission splits a tile over four wave64s");
constexpr int kGroupTiles = 64;  // largest group of tiles per peak workgroup (g.group_tiles)
constexpr int kWalkChunks = 4;   // chunks of kBlock pool entries per round of the ordered peak walk

// A launch's event descriptor: the kernel argument for one event, else evs[blockIdx.y]. The
// descriptor array is read through the constant address space: both sources are then
// scalar-loaded (a generic pointer chosen between the two would make every field a vector
// memory load, one more round trip before each workgroup's first real load).
#define CONSTANT __attribute__((address_space(4)))
__device__ __forceinline__ EvDesc load_ev(const EvDesc& ev0, const EvDesc* evs)
{
#if defined(__HIP_DEVICE_COMPILE__)
  if (evs) return ((const CONSTANT EvDesc*)evs)[blockIdx.y];
#else
  if (evs) return evs[blockIdx.y];  // the host pass only parses device functions
#endif
  return ev0;
}

// ---------------------------------------------------------------------------------------------
// Memory helpers. Pointers reached through descriptors are generic to the compiler, which then
// emits FLAT instructions: those count against the LDS counter too, so every LDS wait would also
// wait for outstanding global stores, and the compiler must assume they may alias LDS. gp()
// states that a pointer is global memory (device memory or host memory mapped into the GPU's
// address space). lds_barrier() synchronises the workgroup for LDS only: no workgroup here reads
// global data written by another of its threads in the same launch, so outstanding global
// stores need not complete before a barrier.
// ---------------------------------------------------------------------------------------------
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gp(T* p)
{
  return (GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const GLOBAL T* gp(const T* p)
{
  return (const GLOBAL T*)p;
}
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// (x, r2, k) of a record: three 4-byte loads the compiler merges into one 12-byte load (the
// unused fourth word is not loaded, so it cannot hold up a register)
__device__ __forceinline__ void ld_xyz(const float4* p, size_t i, float* x, float* r2, float* k)
{
  const GLOBAL float* q = (const GLOBAL float*)p + 4 * i;
  *x = q[0];
  *r2 = q[1];
  *k = q[2];
}
__device__ __forceinline__ void st_rec(float4* p, size_t i, float4 v)
{
  const f32x4 w = {v.x, v.y, v.z, v.w};
  ((GLOBAL f32x4*)p)[i] = w;
}
__device__ __forceinline__ uint2 ld_cand(const uint2* p, size_t i)
{
  const u32x2 v = ((const GLOBAL u32x2*)p)[i];
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void st_cand(uint2* p, size_t i, uint32_t cell, uint32_t votes)
{
  const u32x2 w = {cell, votes};
  ((GLOBAL u32x2*)p)[i] = w;
}
// an output peak: one 8-byte store when the caller's array is 8-byte aligned (a wave's peaks
// then go out as one contiguous run, which matters when the array is host memory mapped into
// the GPU: every store becomes a bus write), else two 4-byte stores (the array need only be
// 4-byte aligned). a8 is uniform.
__device__ __forceinline__ void st_peak(ht_peak* p, int64_t i, uint32_t cell, uint32_t votes, bool a8)
{
  if (a8) {
    const u32x2 w = {cell, votes};
    ((GLOBAL u32x2*)p)[i] = w;
    return;
  }
  GLOBAL uint32_t* q = (GLOBAL uint32_t*)p + 2 * i;
  q[0] = cell;
  q[1] = votes;
}
__device__ __forceinline__ uint32_t gatomic_add(uint32_t* p, uint32_t v)
{
  return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lds_barrier()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------------------------
// Wave / block scans (wave64)
// ---------------------------------------------------------------------------------------------
// Inclusive scan over a wave64 with DPP moves, which stay in the VALU (no LDS round trips):
// Hillis-Steele shifts inside each row of 16 lanes, then the last lane of row 0 is added to
// row 1 and row 3, and that of row 1 (lane 31) to rows 2 and 3. A lane whose source lies
// outside its row is masked off and adds 0. Every lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v)
{
  return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum over a wave64 (every lane active); the result is uniform.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

// Exclusive scan over the block (blockDim a multiple of 64, at most 1024). smem: >= 17 words.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* smem, uint32_t* total)
{
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) smem[w] = inc;
  lds_barrier();
  if (threadIdx.x < 64) {
    uint32_t s = threadIdx.x < (unsigned)nw ? smem[threadIdx.x] : 0u;
    uint32_t si = wave_incl_scan(s);
    if (threadIdx.x < (unsigned)nw) smem[threadIdx.x] = si - s;
    if (threadIdx.x == (unsigned)nw - 1) smem[16] = si;
  }
  lds_barrier();
  uint32_t res = smem[w] + inc - v;
  *total = smem[16];
  lds_barrier();
  return res;
}

__device__ uint32_t block_sum(uint32_t v, uint32_t* smem)
{
  uint32_t total;
  block_excl_scan(v, smem, &total);
  return total;
}


// ---------------------------------------------------------------------------------------------
// Candidates (cells >= threshold) of one tile held in LDS. Each wave takes a quarter of the tile
// (in 16-byte units when VEC, the tile then being a multiple of 4 cells): count_candidates
// leaves each wave's count in s_small[wave]; after a barrier, emit_candidates reserves the
// tile's chunk of the event's candidate pool with one atomic and each wave writes the
// candidates of its quarter in cell order (ballot compaction), so every tile's chunk is sorted
// by cell index. A tile whose candidates do not fit the pool is recorded as overflowed
// (searched densely). The LDS tile is left as it was. (Dropping here the cells that lose to a
// neighbour inside the tile cut the peak test but cost the fill more than it saved.)
// Both are called by the whole block; s_small: >= 9 words. emit_candidates ends with a barrier
// when the tile holds candidates, so the caller may then overwrite the tile.
// ---------------------------------------------------------------------------------------------
template <bool VEC>
__device__ __forceinline__ void tile_quarter(uint32_t L, int wave, uint32_t* q0, uint32_t* q1)
{
  const uint32_t n = VEC ? L / 4u : L;  // 16-byte units or cells
  const uint32_t seg = (n + 3u) / 4u;
  *q0 = min(n, (uint32_t)wave * seg);
  *q1 = min(n, *q0 + seg);
}

template <bool VEC>
__device__ void count_candidates(const uint32_t* s_tile, uint32_t L, uint32_t T, uint32_t* s_small)
{
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t q0, q1;
  tile_quarter<VEC>(L, wave, &q0, &q1);
  uint32_t cnt = 0;  // uniform: sums of ballots
  if (VEC) {
    const u32x4* s4 = reinterpret_cast<const u32x4*>(s_tile);
    const u32x4 zero4 = {0u, 0u, 0u, 0u};
    for (uint32_t b = q0; b < q1; b += 4 * 64) {
      u32x4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {  // four reads in flight, then the compares
        const uint32_t i = b + (uint32_t)(k * 64 + lane);
        v[k] = i < q1 ? s4[i] : zero4;  // T >= 1, so a zero is never a candidate
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        cnt += (uint32_t)(__popcll(__ballot(v[k].x >= T)) + __popcll(__ballot(v[k].y >= T)) +
                          __popcll(__ballot(v[k].z >= T)) + __popcll(__ballot(v[k].w >= T)));
    }
  } else {
    for (uint32_t b = q0; b < q1; b += 64) {
      const uint32_t i = b + lane;
      cnt += (uint32_t)__popcll(__ballot(i < q1 && s_tile[i] >= T));
    }
  }
  if (lane == 0) s_small[wave] = cnt;
}

template <bool VEC>
__device__ void emit_candidates(const DevGrid& g, const EvDesc& e, int tile, uint32_t cell0,
                                const uint32_t* s_tile, uint32_t L, uint32_t* s_small)
{
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t T = g.threshold;
  const uint32_t w0 = s_small[0], w1 = s_small[1], w2 = s_small[2];
  const uint32_t total = w0 + w1 + w2 + s_small[3];
  if (total == 0) {  // uniform
    if (threadIdx.x == 0) {
      // peak counts start at zero; the candidate test (a later launch) adds to them
      gp(e.tile_pk)[tile] = 0u;
      if (tile % g.group_tiles == 0) gp(e.group_pk)[tile / g.group_tiles] = 0u;
      gp(e.tile_cnt)[tile] = 0u;
      gp(e.tile_off)[tile] = 0u;
    }
    return;
  }
  if (threadIdx.x == 0) {
    uint32_t base = gatomic_add(e.slab_cnt + kPoolCounter, total);
    if (base > e.pool_cap || total > e.pool_cap - base) {
      // reservations are contiguous, so at most one starts inside the pool and crosses its
      // end: it marks where the written entries stop
      if (base <= e.pool_cap) gp(e.slab_cnt)[kPoolCut] = e.pool_cap - base + 1u;
      gp(e.ovf_list)[gatomic_add(e.slab_cnt + kOvfCounter, 1u)] = (uint32_t)tile;
      base = kTileOverflow;
    }
    s_small[8] = base;
    gp(e.tile_cnt)[tile] = total;
    gp(e.tile_off)[tile] = base;
    gp(e.tile_pk)[tile] = 0u;
    if (tile % g.group_tiles == 0) gp(e.group_pk)[tile / g.group_tiles] = 0u;
  }
  lds_barrier();
  const uint32_t base = s_small[8];
  if (base != kTileOverflow) {  // uniform
    uint32_t q0, q1;
    tile_quarter<VEC>(L, wave, &q0, &q1);
    // candidates of the earlier quarters
    uint32_t run = base + (wave > 0 ? w0 : 0u) + (wave > 1 ? w1 : 0u) + (wave > 2 ? w2 : 0u);
    // a lane's rank among the ballot's set lanes below it: mbcnt adds the count of set bits below
    // the lane in one half of the mask to its second operand
    auto rank = [](uint64_t m, uint32_t base) {
      return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
    };
    if (VEC) {
      const u32x4* s4 = reinterpret_cast<const u32x4*>(s_tile);
      const u32x4 zero4 = {0u, 0u, 0u, 0u};
      for (uint32_t b = q0; b < q1; b += 2 * 64) {
        u32x4 v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t i = b + (uint32_t)(k * 64 + lane);
          v[k] = i < q1 ? s4[i] : zero4;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          // cells 4i .. 4i+3 of lane l precede those of lane l+1
          const uint32_t c = cell0 + 4u * (b + (uint32_t)(k * 64 + lane));
          const bool c0 = v[k].x >= T, c1 = v[k].y >= T, c2 = v[k].z >= T, c3 = v[k].w >= T;
          const uint64_t m0 = __ballot(c0), m1 = __ballot(c1), m2 = __ballot(c2), m3 = __ballot(c3);
          uint32_t r = rank(m3, rank(m2, rank(m1, rank(m0, run))));
          if (c0) st_cand(e.pool, r++, c, v[k].x);
          if (c1) st_cand(e.pool, r++, c + 1u, v[k].y);
          if (c2) st_cand(e.pool, r++, c + 2u, v[k].z);
          if (c3) st_cand(e.pool, r, c + 3u, v[k].w);
          run += (uint32_t)(__popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3));
        }
      }
    } else {
      for (uint32_t b = q0; b < q1; b += 64) {
        const uint32_t i = b + lane;
        const uint32_t v = i < q1 ? s_tile[i] : 0u;
        const bool c = v >= T;
        const uint64_t m = __ballot(c);
        if (c) st_cand(e.pool, rank(m, run), cell0 + i, v);
        run += (uint32_t)__popcll(m);
      }
    }
  }
  lds_barrier();
}

// ---------------------------------------------------------------------------------------------
// Fill through an LDS tile of ROWS x n_b counters. The grid holds ceil(n_tiles / fill_tiles)
// workgroups; workgroup w fills tiles w, w + G, w + 2G, ... (G workgroups), so at any moment the
// workgroups write one contiguous stretch of the matrix. Per tile: the slab's record list is
// read (with direct lists the first CACHE records per thread are loaded together with the list
// length, in one memory round trip; longer lists come in further chunks of CACHE records per
// thread, each chunk's loads issued together), the votes go to LDS, the tile's candidates are
// pooled, the tile is written out once, and the LDS tile is left all zero. CACHE is 2 for short
// lists (few registers, so eight waves fit on each SIMD) and 8 for long ones, where the LDS
// tile, not the registers, limits how many workgroups fit.
// ---------------------------------------------------------------------------------------------
template <int ROWS, bool VEC, bool EMIT, bool NT, int CACHE>
__global__ __launch_bounds__(kBlock) void k_fill(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  extern __shared__ uint32_t smem[];
  EvDesc e = load_ev(ev0, evs);
  const uint32_t nb = (uint32_t)g.n_b;
  const uint32_t Lpad = ((uint32_t)ROWS * nb + 3u) & ~3u;
  uint32_t* s_tile = smem;
  uint32_t* s_small = smem + Lpad;  // 16 words
  // long lists only: one word per lane past the small words, where a vote outside the row goes
  uint32_t* const s_spill = smem + Lpad + 16u + (threadIdx.x & 63u);
  u32x4* s4 = reinterpret_cast<u32x4*>(s_tile);
  const u32x4 zero4 = {0u, 0u, 0u, 0u};
  for (uint32_t i = threadIdx.x; i < Lpad / 4; i += kBlock) s4[i] = zero4;

  const float b_min = g.b_min, inv_db = g.inv_db, nb_f = g.nb_f;
  const uint32_t nb_bits = __float_as_uint(nb_f);
  const uint32_t T = g.threshold;
  // Workgroups are dealt to the eight XCDs in turn, so consecutive tiles land on different
  // XCDs and a slab's record list is fetched into every XCD's L2. Giving each XCD one
  // contiguous range of tiles instead measured 11% slower on the paper grid (eight separate
  // write streams); the plain order is kept.
  //
  // With long lists and several tiles per workgroup, a workgroup instead fills consecutive
  // tiles, the A rows of one slab in turn, and keeps the slab's records in registers from one
  // tile to the next when they all fit (no list load after the first tile).
  const bool consecutive = CACHE == 8 && g.fill_tiles > 1;  // uniform
  const int t_begin = consecutive ? (int)blockIdx.x * g.fill_tiles : (int)blockIdx.x;
  const int t_end = consecutive ? min(t_begin + g.fill_tiles, g.n_tiles) : g.n_tiles;
  const int t_step = consecutive ? 1 : (int)gridDim.x;
  int held_slab = -1;  // slab whose whole record list is in registers, or -1
  size_t beg = 0;
  uint32_t n = 0;
  float cx[CACHE], cr2[CACHE], ck[CACHE];
  for (int tile = t_begin; tile < t_end; tile += t_step) {  // uniform
    const int slab = tile / g.tiles_per_slab;
    const int a0 = (tile - slab * g.tiles_per_slab) * ROWS;
    const int rows = min(ROWS, g.n_a - a0);
    const uint32_t L = (uint32_t)rows * nb;
    if (CACHE != 8 || slab != held_slab) {  // the short-list variant never holds a list
      uint32_t last;  // last readable record (before n is known)
      if (e.list_cap > 0) {
        beg = (size_t)slab * (size_t)e.list_cap;
        n = gp(e.slab_cnt)[slab];
        last = (uint32_t)e.list_cap - 1u;
      } else {
        // the packed list has one record of slack past its end, so beg is always readable
        const uint32_t o = gp(e.slab_off)[slab];
        beg = o;
        n = gp(e.slab_off)[slab + 1] - o;
        last = n > 0 ? n - 1u : 0u;
      }
      // unconditional loads from clamped indices: no branch, so the values land straight in
      // the registers the votes read, and the loads overlap the list-length load
#pragma unroll
      for (int c = 0; c < CACHE; ++c)
        ld_xyz(e.list, beg + min(threadIdx.x + (uint32_t)c * kBlock, last), &cx[c], &cr2[c], &ck[c]);
      held_slab = (consecutive && n <= (uint32_t)(CACHE * kBlock)) ? slab : -1;
    }
    float a2r[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) a2r[r] = g.a2[min(a0 + r, g.n_a - 1)];
    // the LDS tile is zero: set at the start, restored at the end of every tile
    lds_barrier();
    // Long lists (crowded events) vote with no branch: every row, and a vote outside the row
    // adds to the lane's spill word instead (rows past a short last tile are cleared after it).
    // In range means 0 <= f < n_b: adding +0 turns -0 into +0 and leaves every other value as
    // it is, and the bit patterns of non-negative binary32 values order as the values do, while
    // negative values, NaN and infinity all have patterns at or above that of n_b. This measured
    // 11% faster on the long-list fill of a 40k-hit event and 4% slower on the short-list fill
    // of the paper event, which keeps the branch.
    auto vote = [&](float x, float r2, float k) {
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (CACHE == 8 || r < rows) {
          float ax = a2r[r] * x;
          float num = r2 - ax;
          float B = num * k;
          float d = B - b_min;
          float f = d * inv_db;
          if (CACHE == 8) {
            const float f0 = f + 0.0f;
            const bool in = __float_as_uint(f0) < nb_bits;
            atomicAdd(in ? &s_tile[(uint32_t)r * nb + (uint32_t)(int)f0] : s_spill, 1u);
          } else if (f >= 0.0f && f < nb_f) {
            atomicAdd(&s_tile[(uint32_t)r * nb + (uint32_t)(int)f], 1u);
          }
        }
      }
    };
#pragma unroll
    for (int c = 0; c < CACHE; ++c)
      if (threadIdx.x + (uint32_t)c * kBlock < n) vote(cx[c], cr2[c], ck[c]);
    // longer lists: further chunks of CACHE records per thread, each chunk's loads issued
    // together (one round trip per chunk)
    for (uint32_t base = CACHE * kBlock; base < n; base += CACHE * kBlock) {  // uniform
#pragma unroll
      for (int c = 0; c < CACHE; ++c)
        ld_xyz(e.list, beg + min(base + threadIdx.x + (uint32_t)c * kBlock, n - 1u), &cx[c], &cr2[c], &ck[c]);
#pragma unroll
      for (int c = 0; c < CACHE; ++c)
        if (base + threadIdx.x + (uint32_t)c * kBlock < n) vote(cx[c], cr2[c], ck[c]);
    }
    lds_barrier();

    const uint32_t cell0 = ((uint32_t)slab * (uint32_t)g.n_a + (uint32_t)a0) * nb;
    if (EMIT && e.dense) {
      // crowded event: its peaks come from the stencil over the written matrix, which only
      // needs the group's peak count cleared
      if (threadIdx.x == 0 && tile % g.group_tiles == 0) gp(e.group_pk)[tile / g.group_tiles] = 0u;
    } else if (EMIT) {
      // candidates are pooled before the tile is written, so the wait for the pool reservation
      // never falls behind this tile's stores (the memory counter a wave waits on counts stores
      // too); each pass keeps several 16-byte LDS reads in flight per lane
      count_candidates<VEC>(s_tile, L, T, s_small);
      lds_barrier();
      emit_candidates<VEC>(g, e, tile, cell0, s_tile, L, s_small);
    }

    // write the tile out once, clearing LDS on the way
    GLOBAL uint32_t* dst = gp(e.acc) + cell0;
    if (VEC) {
      GLOBAL u32x4* d4 = reinterpret_cast<GLOBAL u32x4*>(dst);
      for (uint32_t i = threadIdx.x; i < L / 4; i += kBlock) {
        const u32x4 v = s4[i];
        if (NT) __builtin_nontemporal_store(v, d4 + i);
        else d4[i] = v;
        s4[i] = zero4;
      }
    } else {
      for (uint32_t i = threadIdx.x; i < L; i += kBlock) {
        const uint32_t v = s_tile[i];
        if (NT) __builtin_nontemporal_store(v, dst + i);
        else dst[i] = v;
        s_tile[i] = 0u;
      }
    }
    if (CACHE == 8 && L < Lpad)  // uniform: the rows past a short last tile took votes
      for (uint32_t i = L + threadIdx.x; i < Lpad; i += kBlock) s_tile[i] = 0u;
    // the LDS tile is all zero again; the next tile's votes start after its first barrier
  }
}

template <int ROWS, bool NT, int CACHE>
hipError_t launch_fill_cache(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                             bool vec, bool emit, size_t lds, hipStream_t s)
{
  dim3 grid((g.n_tiles + g.fill_tiles - 1) / g.fill_tiles, n_ev);  // interleaved tiles
  if (vec) {
    if (emit) hipLaunchKernelGGL((k_fill<ROWS, true, true, NT, CACHE>), grid, dim3(kBlock), lds, s, g, ev0, evs);
    else hipLaunchKernelGGL((k_fill<ROWS, true, false, NT, CACHE>), grid, dim3(kBlock), lds, s, g, ev0, evs);
  } else {
    if (emit) hipLaunchKernelGGL((k_fill<ROWS, false, true, NT, CACHE>), grid, dim3(kBlock), lds, s, g, ev0, evs);
    else hipLaunchKernelGGL((k_fill<ROWS, false, false, NT, CACHE>), grid, dim3(kBlock), lds, s, g, ev0, evs);
  }
  return hipGetLastError();
}

template <int ROWS, bool NT>
hipError_t launch_fill_rows(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                            bool vec, bool emit, bool long_lists, size_t lds, hipStream_t s)
{
  // long-list variant only where tiles are narrow enough for it to matter (rows <= 8)
  if (ROWS <= 8 && long_lists) return launch_fill_cache<ROWS, NT, 8>(g, ev0, evs, n_ev, vec, emit, lds, s);
  return launch_fill_cache<ROWS, NT, 2>(g, ev0, evs, n_ev, vec, emit, lds, s);
}
}  // namespace

// Fill launch for one A-row count per tile (ht_fill_rows.hip instantiates each).
template <int ROWS>
hipError_t launch_fill_for_rows(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev, bool nt,
                                bool vec, bool emit, bool long_lists, size_t lds, hipStream_t s);

}  // namespace ht
