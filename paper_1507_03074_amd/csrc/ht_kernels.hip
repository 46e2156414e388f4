// ht_kernels.hip -- gfx950 kernels of the Hough-transform fill and peak search.
//
// Pipeline (paper section 2: every hit votes along its circles through the interaction point,
// then the local maxima above a threshold are the track candidates). Every kernel takes a batch
// of events (grid.y = event), so one launch per stage serves a single event or a whole batch:
//   k_prep_direct per hit: validity, r2, k = 1/(2y), theta/phi half-sectors and the 2-4
//                 (theta, phi) cells; the (hit, cell) records go to fixed-capacity per-slab lists
//                 (one slab = the A x B plane of one (theta, phi) cell), their positions reserved
//                 with LDS-aggregated atomics. Very large events use a counting sort instead:
//                 k_prep counts, then k_bucket scans the counts in LDS and scatters.
//   k_fill        one workgroup per (slab, tile of A rows): the slab's records vote into an LDS
//                 tile (ds_add), the cells >= threshold go to the event's candidate pool as
//                 sorted per-tile chunks (cell, votes), then every cell of the tile is written to
//                 HBM once with coalesced 16-byte stores (so the matrix needs no memset)
//   k_peak_test   the pooled candidates spread evenly over the workgroups: each takes the strict
//                 3^4 test against its 80 neighbours (a cell below the threshold can never beat a
//                 candidate, so only candidates need testing); peaks are counted per tile and
//                 per group of 16-64 tiles
//   k_peak_write  per group: its output offset from the earlier groups' totals; the ordered
//                 peak list
//   crowded events (at least dense_hits hits) skip the candidate pool: the fill only writes
//   the matrix, k_peak_stencil tests every cell in one read of it (one wave per phi cell, the
//   theta cells in its registers, the phi neighbours through LDS) into 64-bit peak words, and
//   k_peak_write_dense writes the ordered peak list from them
// ht_peaks on an arbitrary matrix replaces prep and fill with k_cand_scan (one read of it).
// No kernel synchronises workgroups with each other: on this multi-XCD part an agent-scope
// release costs an L2 write-back, while a kernel boundary is cheap.
//
// Every floating-point step of the bin rule is one binary32 operation, rounded to nearest even,
// in the documented order: contraction is off for this file, sqrtf and the division are the
// correctly rounded forms.
#include <cstdlib>

#include "ht_device.h"

#pragma clang fp contract(off)

namespace ht {
namespace {

// ---------------------------------------------------------------------------------------------
// Per-hit preparation (validity, per-hit values, half-sectors, cells)
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int half_plane(float c, float s, float vx, float vy)
{
  float lhs = c * vy;
  float rhs = s * vx;
  float d = lhs - rhs;
  return d >= 0.0f ? 1 : 0;
}

// The two correctly rounded operations of the per-hit values: r = sqrt(r2) and k = 1/(2y)
// (2y is exact). Shared by the preparation and by ht_debug_unary, which checks them against
// the host over every binary32 input.
__device__ __forceinline__ float hit_root(float r2) { return sqrtf(r2); }
__device__ __forceinline__ float hit_inv2(float y)
{
  float ty = y + y;
  return 1.0f / ty;
}

struct HitPrep {
  int n;  // number of (theta, phi) cells, 0 when the hit votes nothing
  int slab[4];
  int s_theta, s_phi;
  float x, r2, r, k;
};

// phi_cs, th_cs: the boundary tables (g.phi_cs, g.th_cs or a copy of them in LDS).
__device__ HitPrep prep_hit(const DevGrid& g, const float* phi_cs, const float* th_cs, float x,
                            float y, float z)
{
  HitPrep h;
  h.n = 0;
  h.s_theta = h.s_phi = 0;
  h.x = x;
  h.r2 = h.r = h.k = 0.0f;
  // one test of all three coordinates (no short cut), so the load of z is not held back until
  // x and y have been checked
  if (!(isfinite(x) & isfinite(y) & isfinite(z)) | (y == 0.0f)) return h;
  float xx = x * x;
  float yy = y * y;
  float r2 = xx + yy;
  if (!(r2 > 0.0f) || isinf(r2)) return h;
  float r = hit_root(r2);
  float k = hit_inv2(y);
  int s_phi;
  if (y > 0.0f) {
    s_phi = 0;
    for (int m = 1; m < g.n_phi; ++m) s_phi += half_plane(phi_cs[2 * m], phi_cs[2 * m + 1], x, y);
  } else {
    s_phi = g.n_phi;
    for (int m = g.n_phi + 1; m < 2 * g.n_phi; ++m)
      s_phi += half_plane(phi_cs[2 * m], phi_cs[2 * m + 1], x, y);
  }
  int s_th = 0;
  for (int m = 1; m < 2 * g.n_theta; ++m) s_th += half_plane(th_cs[2 * m], th_cs[2 * m + 1], z, r);
  const int p0 = s_phi >> 1;
  const int p1 = (s_phi & 1) ? (p0 + 1 == g.n_phi ? 0 : p0 + 1) : (p0 == 0 ? g.n_phi - 1 : p0 - 1);
  const int t0 = s_th >> 1;
  const int t1 = (s_th & 1) ? t0 + 1 : t0 - 1;
  if (g.phi_sectors) {
    // section 4: the hit's own sector only
    h.slab[0] = t0 * g.n_phi + p0;
    h.n = 1;
    if (t1 >= 0 && t1 < g.n_theta) {
      h.slab[1] = t1 * g.n_phi + p0;
      h.n = 2;
    }
  } else {
    h.slab[0] = t0 * g.n_phi + p0;
    h.slab[1] = t0 * g.n_phi + p1;
    h.n = 2;
    if (t1 >= 0 && t1 < g.n_theta) {
      h.slab[2] = t1 * g.n_phi + p0;
      h.slab[3] = t1 * g.n_phi + p1;
      h.n = 4;
    }
  }
  h.s_theta = s_th;
  h.s_phi = s_phi;
  h.r2 = r2;
  h.r = r;
  h.k = k;
  return h;
}

// The boundary tables copied into LDS (dynamic shared memory): the sector counts then read
// them at LDS latency instead of one scalar load after another. The caller's next barrier makes
// the copy visible. Without LDS_TABLES (grids whose tables exceed kLdsTableBytes) the tables are
// read from global memory.
constexpr size_t kLdsTableBytes = 16384;

template <bool LDS_TABLES>
__device__ __forceinline__ void tables_to_lds(const DevGrid& g, float* s_tab, const float** tab_phi,
                                              const float** tab_th)
{
  if (!LDS_TABLES) {
    *tab_phi = g.phi_cs;
    *tab_th = g.th_cs;
    return;
  }
  const int n_phi = 4 * g.n_phi, n_th = 2 * (2 * g.n_theta + 1);
  for (int i = threadIdx.x; i < n_phi + n_th; i += kBlock)
    s_tab[i] = i < n_phi ? gp(g.phi_cs)[i] : gp(g.th_cs)[i - n_phi];
  *tab_phi = s_tab;
  *tab_th = s_tab + n_phi;
}

// Direct lists: counts per slab in LDS per workgroup, one global atomic per (workgroup, slab)
// reserves the workgroup's range of each slab's fixed-capacity list, then the records are
// written there. slab_cnt is zero on entry and ends holding the list lengths; workgroup 0 clears
// the other counter array for the next call.
template <bool LDS_TABLES>
__global__ __launch_bounds__(kBlock) void k_prep_direct(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  __shared__ uint32_t lcnt[kMaxSlabs];
  extern __shared__ float s_tab[];
  EvDesc e = load_ev(ev0, evs);
  // clear all of the other array: an earlier call on a grid with more slabs may have used
  // entries past this grid's n_slabs
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kCounterWords; i += kBlock) gp(e.slab_cnt_next)[i] = 0u;
  if ((int64_t)blockIdx.x * kBlock >= e.n_hits) return;  // uniform: whole block idle
  const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  // the hit's coordinates are loaded first, so their round trip overlaps the table copy
  const int64_t hc = min(h, e.n_hits - 1);
  const float hx = gp(e.x)[hc], hy = gp(e.y)[hc], hz = gp(e.z)[hc];
  const float *tab_phi, *tab_th;
  tables_to_lds<LDS_TABLES>(g, s_tab, &tab_phi, &tab_th);
  for (int i = threadIdx.x; i < g.n_slabs; i += kBlock) lcnt[i] = 0u;
  lds_barrier();
  HitPrep p;
  p.n = 0;
  uint32_t local[4] = {0u, 0u, 0u, 0u};
  if (h < e.n_hits) {
    p = prep_hit(g, tab_phi, tab_th, hx, hy, hz);
    // constant indices keep p.slab and local in registers (a runtime index would put them in
    // scratch memory)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < p.n) local[q] = atomicAdd(&lcnt[p.slab[q]], 1u);
  }
  lds_barrier();
  for (int i = threadIdx.x; i < g.n_slabs; i += kBlock) {
    uint32_t c = lcnt[i];
    if (c) lcnt[i] = gatomic_add(e.slab_cnt + i, c);
  }
  lds_barrier();
  if (h < e.n_hits) {
    const float4 rec = make_float4(p.x, p.r2, p.k, 0.0f);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < p.n) st_rec(e.list, (size_t)p.slab[q] * (size_t)e.list_cap + lcnt[p.slab[q]] + local[q], rec);
  }
}

// Counting sort, first pass: counts per slab (LDS, then one global atomic per workgroup and
// slab) and each record's position within its slab. Workgroup 0 clears the other counter array.
template <bool LDS_TABLES>
__global__ __launch_bounds__(kBlock) void k_prep(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  __shared__ uint32_t lcnt[kMaxSlabs];
  extern __shared__ float s_tab[];
  EvDesc e = load_ev(ev0, evs);
  // clear all of the other array: an earlier call on a grid with more slabs may have used
  // entries past this grid's n_slabs
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kCounterWords; i += kBlock) e.slab_cnt_next[i] = 0u;
  if ((int64_t)blockIdx.x * kBlock >= e.n_hits) return;  // uniform: whole block idle
  const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t hc = min(h, e.n_hits - 1);
  const float hx = gp(e.x)[hc], hy = gp(e.y)[hc], hz = gp(e.z)[hc];
  const float *tab_phi, *tab_th;
  tables_to_lds<LDS_TABLES>(g, s_tab, &tab_phi, &tab_th);
  for (int i = threadIdx.x; i < g.n_slabs; i += kBlock) lcnt[i] = 0u;
  lds_barrier();
  HitPrep p;
  p.n = 0;
  uint32_t local[4] = {0u, 0u, 0u, 0u};
  if (h < e.n_hits) {
    p = prep_hit(g, tab_phi, tab_th, hx, hy, hz);
    e.hit_rec[h] = make_float4(p.x, p.r2, p.k, 0.0f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int s = q < p.n ? p.slab[q] : -1;
      e.hit_slab[4 * h + q] = s;
      if (s >= 0) local[q] = atomicAdd(&lcnt[s], 1u);
    }
  }
  lds_barrier();
  for (int i = threadIdx.x; i < g.n_slabs; i += kBlock) {
    uint32_t c = lcnt[i];
    if (c) lcnt[i] = atomicAdd(&e.slab_cnt[i], c);
  }
  lds_barrier();
  if (h < e.n_hits)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < p.n) e.hit_pos[4 * h + q] = lcnt[p.slab[q]] + local[q];
}

// Every workgroup scans the slab counts into LDS (they are few); workgroup 0 also publishes the
// offsets for the fill. Then each hit's records go to their slab lists.
__global__ __launch_bounds__(kBlock) void k_bucket(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  __shared__ uint32_t s_off[kMaxSlabs];
  __shared__ uint32_t smem[32];
  EvDesc e = load_ev(ev0, evs);
  if (blockIdx.x > 0 && (int64_t)blockIdx.x * kBlock >= e.n_hits) return;
  const int ns = g.n_slabs;
  const int per = (ns + kBlock - 1) / kBlock;
  const int beg = min(ns, (int)threadIdx.x * per);
  const int end = min(ns, beg + per);
  uint32_t sum = 0;
  for (int i = beg; i < end; ++i) sum += e.slab_cnt[i];
  uint32_t total;
  uint32_t run = block_excl_scan(sum, smem, &total);
  for (int i = beg; i < end; ++i) {
    const uint32_t c = e.slab_cnt[i];
    s_off[i] = run;
    if (blockIdx.x == 0) e.slab_off[i] = run;
    run += c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) e.slab_off[ns] = total;
  lds_barrier();
  const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (h >= e.n_hits) return;
  const float4 rec = e.hit_rec[h];
  for (int q = 0; q < 4; ++q) {
    const int s = e.hit_slab[4 * h + q];
    if (s < 0) break;
    e.list[s_off[s] + e.hit_pos[4 * h + q]] = rec;
  }
}

// Candidates of an arbitrary matrix: one coalesced read of each tile into LDS, then the same
// count and ordered emission as the fill's. Workgroup 0 clears the other counter array for the
// next call.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_cand_scan(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  extern __shared__ uint32_t smem[];
  EvDesc e = load_ev(ev0, evs);
  const int tile = blockIdx.x;
  if (tile == 0)
    for (int i = threadIdx.x; i < kCounterWords; i += kBlock) gp(e.slab_cnt_next)[i] = 0u;
  const int slab = tile / g.tiles_per_slab;
  const int a0 = (tile - slab * g.tiles_per_slab) * g.rows;
  const int rows = min(g.rows, g.n_a - a0);
  const uint32_t nb = (uint32_t)g.n_b;
  const uint32_t L = (uint32_t)rows * nb;
  const uint32_t Lpad = ((uint32_t)g.rows * nb + 3u) & ~3u;
  uint32_t* s_tile = smem;
  uint32_t* s_small = smem + Lpad;
  const uint32_t cell0 = ((uint32_t)slab * (uint32_t)g.n_a + (uint32_t)a0) * nb;
  const GLOBAL uint32_t* src = gp(e.acc) + cell0;
  if (VEC) {
    const GLOBAL u32x4* s4 = reinterpret_cast<const GLOBAL u32x4*>(src);
    u32x4* l4 = reinterpret_cast<u32x4*>(s_tile);
    for (uint32_t i = threadIdx.x; i < L / 4; i += kBlock) l4[i] = __builtin_nontemporal_load(s4 + i);
  } else {
    for (uint32_t i = threadIdx.x; i < L; i += kBlock) s_tile[i] = src[i];
  }
  lds_barrier();
  count_candidates<VEC>(s_tile, L, g.threshold, s_small);
  lds_barrier();
  emit_candidates<VEC>(g, e, tile, cell0, s_tile, L, s_small);
}

// ---------------------------------------------------------------------------------------------
// Peak test: strict maximum under (votes, -index) over the 3^4 box, phi periodic.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void cell_coords(const DevGrid& g, uint32_t c, uint32_t* t, uint32_t* p,
                                            uint32_t* a, uint32_t* b)
{
  const uint32_t nb = (uint32_t)g.n_b, na = (uint32_t)g.n_a, np = (uint32_t)g.n_phi;
  *b = c % nb;
  uint32_t q = c / nb;
  *a = q % na;
  q /= na;
  *p = q % np;
  *t = q / np;
}


// The 27 neighbour rows are taken one theta slice (9 rows of three cells, one 12-byte load each)
// at a time, its own theta first: the nine loads of a slice are issued together, and a
// candidate beaten in one slice skips the rest (most candidates are beaten early). The window
// of a row starts at min(max(b, 1) - 1, n_b - 3), so it stays inside the row; absent rows
// (outside theta or A, or phi neighbours across sectors) read the candidate's own row and are
// masked out.
__device__ bool is_peak(const DevGrid& g, const uint32_t* __restrict__ acc, uint32_t c, uint32_t v)
{
  const uint32_t nb = (uint32_t)g.n_b, na = (uint32_t)g.n_a, np = (uint32_t)g.n_phi;
  uint32_t t, p, a, b;
  cell_coords(g, c, &t, &p, &a, &b);
  const uint32_t pm = p == 0 ? np - 1 : p - 1;
  const uint32_t pp1 = p + 1 == np ? 0 : p + 1;
  if (nb < 3) {
    // narrow rows: one load per neighbour
    bool beaten = false;
    for (int k = 0; k < 27; ++k) {
      const int dt = k / 9 - 1, dp = (k / 3) % 3 - 1, da = k % 3 - 1;
      const int tt = (int)t + dt, aa = (int)a + da;
      if (tt < 0 || tt >= g.n_theta || aa < 0 || aa >= (int)na) continue;
      if (g.phi_sectors && dp != 0) continue;
      const uint32_t pp = dp < 0 ? pm : (dp > 0 ? pp1 : p);
      const uint32_t rowc = (((uint32_t)tt * np + pp) * na + (uint32_t)aa) * nb;
      for (int db = -1; db <= 1; ++db) {
        const int bb = (int)b + db;
        if (bb < 0 || bb >= (int)nb || (dt == 0 && dp == 0 && da == 0 && db == 0)) continue;
        const uint32_t n = rowc + (uint32_t)bb;
        const uint32_t w = gp(acc)[n];
        beaten |= w > v || (w == v && n < c);
      }
    }
    return !beaten;
  }
  const uint32_t w0 = min(max(b, 1u) - 1u, nb - 3u);
#pragma unroll
  for (int slice = 0; slice < 3; ++slice) {
    const int dt = slice == 0 ? 0 : (slice == 1 ? -1 : 1);
    const int tt = (int)t + dt;
    if (tt < 0 || tt >= g.n_theta) continue;
    uint32_t row[9][3];
    uint32_t base[9];
    bool rv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int dp = k / 3 - 1, da = k % 3 - 1;
      const int aa = (int)a + da;
      rv[k] = aa >= 0 && aa < (int)na && !(g.phi_sectors && dp != 0);
      const uint32_t pp = dp < 0 ? pm : (dp > 0 ? pp1 : p);
      base[k] = (rv[k] ? (((uint32_t)tt * np + pp) * na + (uint32_t)aa) * nb : c - b) + w0;
      const GLOBAL uint32_t* rw = gp(acc) + base[k];
      row[k][0] = rw[0];
      row[k][1] = rw[1];
      row[k][2] = rw[2];
    }
    bool beaten = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const bool centre_row = dt == 0 && k == 4;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const uint32_t bb = w0 + (uint32_t)q;
        // inside the window; neighbour iff |bb - b| <= 1 and not the candidate itself
        const bool near = bb + 1u >= b && bb <= b + 1u && !(centre_row && bb == b);
        const uint32_t n = base[k] + (uint32_t)q;
        beaten |= rv[k] && near && (row[k][q] > v || (row[k][q] == v && n < c));
      }
    }
    if (beaten) return false;
  }
  return true;
}

__device__ __forceinline__ void tile_range(const DevGrid& g, int tile, uint32_t* cell0, uint32_t* L)
{
  const int slab = tile / g.tiles_per_slab;
  const int a0 = (tile - slab * g.tiles_per_slab) * g.rows;
  const int rows = min(g.rows, g.n_a - a0);
  *cell0 = ((uint32_t)slab * (uint32_t)g.n_a + (uint32_t)a0) * (uint32_t)g.n_b;
  *L = (uint32_t)rows * (uint32_t)g.n_b;
}

// Candidates of an arbitrary matrix whose B rows are too wide for an LDS tile (grids that also
// fill through global atomics; a tile is then one row of up to 2^24 cells): the same count and
// ordered emission as k_cand_scan, read straight from the matrix, so the row is read twice.
// Workgroup 0 clears the other counter array for the next call.
__global__ __launch_bounds__(kBlock) void k_cand_scan_wide(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  __shared__ uint32_t s_small[16];
  EvDesc e = load_ev(ev0, evs);
  const int tile = blockIdx.x;
  if (tile == 0)
    for (int i = threadIdx.x; i < kCounterWords; i += kBlock) gp(e.slab_cnt_next)[i] = 0u;
  uint32_t cell0, L;
  tile_range(g, tile, &cell0, &L);
  const uint32_t* src = e.acc + cell0;
  count_candidates<false>(src, L, g.threshold, s_small);
  lds_barrier();
  emit_candidates<false>(g, e, tile, cell0, src, L, s_small);
}

// Largest t with pre[t] <= f, given pre[0] <= f < pre[kGroupTiles] and pre non-decreasing: a
// fixed number of halving steps, with no branch.
__device__ __forceinline__ int group_tile_of(const uint32_t* pre, uint32_t f)
{
  static_assert((kGroupTiles & (kGroupTiles - 1)) == 0, "halving search over a power of two");
  int lo = 0;
#pragma unroll
  for (int step = kGroupTiles / 2; step > 0; step >>= 1) lo += pre[lo + step] <= f ? step : 0;
  return lo;
}

// Whether any cell of neighbour row k (0..26: dt, dp, da in {-1, 0, 1}, row-major) of candidate
// c with v votes beats it under (votes, -index). Rows outside theta or A are absent; phi wraps.
// Loads one 12-byte window of three cells; the window of a row starts at
// min(max(b, 1) - 1, n_b - 3), so it stays inside the row.
__device__ bool row_beats(const DevGrid& g, const uint32_t* __restrict__ acc, uint32_t c, uint32_t v, int k)
{
  const uint32_t nb = (uint32_t)g.n_b, na = (uint32_t)g.n_a, np = (uint32_t)g.n_phi;
  uint32_t t, p, a, b;
  cell_coords(g, c, &t, &p, &a, &b);
  const int dt = k / 9 - 1, dp = (k / 3) % 3 - 1, da = k % 3 - 1;
  const int tt = (int)t + dt, aa = (int)a + da;
  if (tt < 0 || tt >= g.n_theta || aa < 0 || aa >= (int)na) return false;
  if (g.phi_sectors && dp != 0) return false;  // sectors have no phi neighbours
  const uint32_t pp = dp < 0 ? (p == 0 ? np - 1 : p - 1) : (dp > 0 ? (p + 1 == np ? 0 : p + 1) : p);
  const uint32_t rowc = (((uint32_t)tt * np + pp) * na + (uint32_t)aa) * nb;
  const bool centre_row = k == 13;
  if (nb < 3) {
    bool beaten = false;
    for (uint32_t bb = b == 0 ? 0 : b - 1; bb <= b + 1 && bb < nb; ++bb) {
      if (centre_row && bb == b) continue;
      const uint32_t n = rowc + bb;
      const uint32_t w = gp(acc)[n];
      beaten |= w > v || (w == v && n < c);
    }
    return beaten;
  }
  const uint32_t w0 = min(max(b, 1u) - 1u, nb - 3u);
  const GLOBAL uint32_t* rw = gp(acc) + rowc + w0;
  const uint32_t vals[3] = {rw[0], rw[1], rw[2]};
  bool beaten = false;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint32_t bb = w0 + (uint32_t)q;
    const bool near = bb + 1u >= b && bb <= b + 1u && !(centre_row && bb == b);
    const uint32_t n = rowc + bb;
    beaten |= near && (vals[q] > v || (vals[q] == v && n < c));
  }
  return beaten;
}

__device__ __forceinline__ void count_peak(const DevGrid& g, const EvDesc& e, uint32_t c)
{
  // (slab, a) from the row index c / n_b: a slab of one cell row by 2^32 cells (n_a n_b = 2^32)
  // would wrap a 32-bit slab size
  const uint32_t row = c / (uint32_t)g.n_b;
  const uint32_t slab = row / (uint32_t)g.n_a;
  const uint32_t a = row - slab * (uint32_t)g.n_a;
  const uint32_t tile = slab * (uint32_t)g.tiles_per_slab + a / (uint32_t)g.rows;
  gatomic_add(e.tile_pk + tile, 1u);
  gatomic_add(e.group_pk + tile / (uint32_t)g.group_tiles, 1u);
}

// Peak test of every pooled candidate, spread evenly over the grid whatever tiles they came
// from. Few candidates (at most two passes of the grid): half a wave (32 lanes) per candidate,
// one lane per neighbour row, so a candidate costs one load per lane and a ballot, and the
// whole test is about one memory round trip. Many candidates: one thread per candidate, its 27
// row loads issued back to back; each workgroup takes one contiguous run of the pool (whole
// waves), so the waves of a CU test neighbouring cells and share their rows in the L1, and the
// runs of one XCD are adjacent, so its L2 holds one region. Each result goes to pk_flag; a
// peak adds one to its tile's and its group's counts. Tiles whose candidates did not fit the
// pool are counted densely, one wave per tile.
__global__ __launch_bounds__(kBlock) void k_peak_test(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  EvDesc e = load_ev(ev0, evs);
  if (e.dense) return;  // uniform: searched by the stencil
  const int lane = threadIdx.x & 63, half = lane >> 5, k = lane & 31;
  // workgroups are dealt to the 8 XCDs in turn: give each XCD one contiguous run of blocks
  const uint32_t blk =
      gridDim.x % 8u ? blockIdx.x : (blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
  const uint32_t wave = blk * (kBlock / 64) + (threadIdx.x >> 6);
  const uint32_t n_waves = gridDim.x * (kBlock / 64);
  // this half-wave's first entry is loaded before the entry count is known (an index inside
  // the pool is always readable), so the count and the entry cost one round trip
  const uint32_t i_first = 2u * wave + (uint32_t)half;
  uint2 cv_first = make_uint2(0u, 0u);
  if (i_first < e.pool_cap) cv_first = ld_cand(e.pool, i_first);
  // the three counters load together (none waits for another)
  const uint32_t cut = gp(e.slab_cnt)[kPoolCut];
  const uint32_t reserved = gp(e.slab_cnt)[kPoolCounter];
  const uint32_t n_ovf = gp(e.slab_cnt)[kOvfCounter];
  const uint32_t n_valid = min(cut ? e.pool_cap + 1u - cut : reserved, e.pool_cap);
  const uint32_t* acc = e.acc;
  if (n_valid <= 4u * n_waves) {
    for (uint32_t i0 = 2u * wave; i0 < n_valid; i0 += 2u * n_waves) {  // wave-uniform
      const uint32_t i = i0 + (uint32_t)half;
      const bool live = i < n_valid;
      uint2 cv = make_uint2(0u, 0u);
      bool beaten = false;
      if (live) {
        cv = i == i_first ? cv_first : ld_cand(e.pool, i);
        if (k < 27) beaten = row_beats(g, acc, cv.x, cv.y, k);
      }
      const uint64_t m = __ballot(beaten);
      const uint32_t hm = (uint32_t)(m >> (32 * half));
      if (live && k == 0) {
        const bool pk = hm == 0u;
        gp(e.pk_flag)[i] = pk ? 1 : 0;
        if (pk) count_peak(g, e, cv.x);
      }
    }
  } else {
    // the run length is a whole number of waves; the last runs may be short or empty. Bounds
    // and index are 64-bit: the pool may hold nearly 2^32 entries.
    const uint64_t per = (((uint64_t)n_valid + gridDim.x - 1u) / gridDim.x + 63u) & ~(uint64_t)63u;
    const uint64_t i_end = min((uint64_t)n_valid, (uint64_t)(blk + 1u) * per);
    for (uint64_t i = (uint64_t)blk * per + threadIdx.x; i < i_end; i += kBlock) {
      const uint2 cv = ld_cand(e.pool, i);
      const bool pk = is_peak(g, acc, cv.x, cv.y);
      gp(e.pk_flag)[i] = pk ? 1 : 0;
      if (pk) count_peak(g, e, cv.x);
    }
  }
  for (uint32_t j = wave; j < n_ovf; j += n_waves) {
    const int tile = (int)gp(e.ovf_list)[j];
    uint32_t cell0, L;
    tile_range(g, tile, &cell0, &L);
    uint32_t mine = 0;
    for (uint32_t q = (uint32_t)lane; q < L; q += 64) {
      const uint32_t c = cell0 + q;
      const uint32_t v = gp(acc)[c];
      if (v >= g.threshold && is_peak(g, acc, c, v)) ++mine;
    }
    mine = wave_sum(mine);
    if (lane == 0 && mine) {
      gatomic_add(e.tile_pk + tile, mine);
      gatomic_add(e.group_pk + tile / g.group_tiles, mine);
    }
  }
}

// One workgroup per group of tiles: its output offset is the sum of the earlier groups' peak
// counts; the group's pooled candidates are walked in order (tile by tile, each tile's chunk
// ascending, kWalkChunks * kBlock of them per memory round trip) and the flagged ones written
// out; tiles that did not fit the pool are re-scanned densely.
__global__ __launch_bounds__(kBlock) void k_peak_write(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  __shared__ uint32_t s_pre[kGroupTiles + 1];
  __shared__ uint32_t s_out[kGroupTiles + 1];
  __shared__ uint32_t s_ovf[kGroupTiles];
  __shared__ uint32_t s_off[kGroupTiles];
  __shared__ uint32_t s_first[kGroupTiles];
  __shared__ uint32_t smem[32];
  EvDesc e = load_ev(ev0, evs);
  if (e.dense) return;  // uniform: written by k_peak_write_dense
  const int G = blockIdx.x;
  const int t0 = G * g.group_tiles;
  const bool a8 = ((uintptr_t)e.out & 7u) == 0;
  const int nt = min(g.group_tiles, g.n_tiles - t0);
  // every load that does not depend on another is issued first: the earlier groups' peak
  // counts (all threads), the group's candidate counts and pool offsets (wave 0) and its peak
  // counts (wave 1)
  const int ti = (int)(threadIdx.x & 63);
  uint32_t t_cnt = 0, t_off = 0, t_pk = 0;
  if (threadIdx.x < 64 && ti < nt) {
    t_cnt = gp(e.tile_cnt)[t0 + ti];
    t_off = gp(e.tile_off)[t0 + ti];
  } else if (threadIdx.x >= 64 && threadIdx.x < 128 && ti < nt) {
    t_pk = gp(e.tile_pk)[t0 + ti];
  }
  // four loads in flight per thread and round (groups past G read as zero)
  uint32_t part = 0;
  for (int i0 = 0; i0 < G; i0 += 4 * kBlock) {  // uniform
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k * kBlock + (int)threadIdx.x;
      w[k] = i < G ? gp(e.group_pk)[i] : 0u;
    }
    part += w[0] + w[1] + w[2] + w[3];
  }
  const uint32_t base32 = block_sum(part, smem);
  const int64_t base = (int64_t)base32;
  if (G == (int)gridDim.x - 1 && threadIdx.x == 0) *gp(e.n_found) = base + gp(e.group_pk)[G];
  if (base >= e.cap) return;  // uniform
  static_assert(kGroupTiles == 64, "one wave holds a group's tiles");
  if (threadIdx.x < 64) {
    // tiles nt..63 count zero, so s_pre[nt..64] all equal the group's candidate total; tiles
    // whose candidates did not fit the pool count zero here (they are scanned densely)
    const uint32_t ovf = t_off == kTileOverflow ? 1u : 0u;
    s_ovf[ti] = ovf;
    s_off[ti] = t_off;
    const uint32_t inc = wave_incl_scan(ovf ? 0u : t_cnt);
    s_pre[ti + 1] = inc;
    if (ti == 0) s_pre[0] = 0u;
  } else if (threadIdx.x < 128) {
    // prefix of the peak counts of all the group's tiles
    const uint32_t inc = wave_incl_scan(t_pk);
    s_out[ti + 1] = inc;
    if (ti == 0) s_out[0] = 0u;
  }
  lds_barrier();
  const uint32_t total = s_pre[kGroupTiles];
  uint32_t run = 0;
  // kWalkChunks chunks of kBlock candidates per round: the flags and entries of all of them are
  // loaded, with no branch between the loads, before the first chunk is scanned, so a round
  // costs one memory round trip. Positions past the group's total load its first candidate
  // (always readable) and count as no peak.
  for (uint32_t b0 = 0; b0 < total; b0 += kWalkChunks * kBlock) {  // uniform
    uint32_t flag[kWalkChunks];
    int tl[kWalkChunks];
    uint2 cv[kWalkChunks];
#pragma unroll
    for (int k = 0; k < kWalkChunks; ++k) {
      const uint32_t f = b0 + (uint32_t)k * kBlock + threadIdx.x;
      const uint32_t fc = f < total ? f : 0u;
      tl[k] = group_tile_of(s_pre, fc);
      const size_t idx = (size_t)s_off[tl[k]] + (fc - s_pre[tl[k]]);
      flag[k] = gp(e.pk_flag)[idx];
      cv[k] = ld_cand(e.pool, idx);
    }
#pragma unroll
    for (int k = 0; k < kWalkChunks; ++k) {
      const uint32_t f0 = b0 + (uint32_t)k * kBlock;
      if (f0 >= total) break;  // uniform
      const uint32_t f = f0 + threadIdx.x;
      const bool pk = f < total && flag[k] != 0u;
      uint32_t tot;
      const uint32_t pos = run + block_excl_scan(pk ? 1u : 0u, smem, &tot);
      // the first candidate of a tile records how many of the group's pooled peaks precede it
      if (f < total && f == s_pre[tl[k]]) s_first[tl[k]] = pos;
      lds_barrier();
      if (pk) {
        const int64_t o = base + s_out[tl[k]] + (pos - s_first[tl[k]]);
        if (o < e.cap) st_peak(e.out, o, cv[k].x, cv[k].y, a8);
      }
      run += tot;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t* acc = e.acc;
  for (int tl = wave; tl < nt; tl += kBlock / 64) {
    if (!s_ovf[tl]) continue;
    uint32_t cell0, L;
    tile_range(g, t0 + tl, &cell0, &L);
    uint32_t r = 0;
    for (uint32_t b0 = 0; b0 < L; b0 += 64) {
      const uint32_t i = b0 + lane;
      bool pk = false;
      uint32_t c = 0, v = 0;
      if (i < L) {
        c = cell0 + i;
        v = gp(acc)[c];
        pk = v >= g.threshold && is_peak(g, acc, c, v);
      }
      const uint64_t m = __ballot(pk);
      const int64_t o = base + s_out[tl] + r + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (pk && o < e.cap) st_peak(e.out, o, c, v, a8);
      r += (uint32_t)__popcll(m);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Peak search of crowded events: an LDS-halo stencil over the whole matrix (one read of it), in
// place of the candidate pool. A workgroup owns one chunk of kChunkCells B columns of every
// (theta, phi) slab and walks down a segment of S A rows. Wave p holds phi cell p of every theta
// cell, so its theta neighbours are in its own registers: lane j holds cell b = base + j - 1 of
// slab (t, p) for each t, where base = kChunkCells * chunk. Lanes 1..62 are tested; lanes 0 and
// 63 hold the cells just outside the chunk, so that every tested cell's B neighbours are in the
// wave (neighbouring chunks overlap by those two cells).
//
// The strict maximum under (votes, -index) splits the 80 neighbours of a cell c into those of
// lower index ("before": theta cell t - 1, the phi cell of lower index in theta cell t, the row
// above in its own slab, the cell left of it) and the others ("after"). A before-neighbour w
// beats c iff w >= v(c); an after-neighbour iff w > v(c). With Mb and Ma the maxima over the
// before- and after-neighbours (absent cells count 0),
//   c is a peak  iff  v(c) >= T,  v(c) >= Mb + 1  and  v(c) >= Ma.
// Per row a a wave forms, for each t, R3(a, b) = the maximum over b-1..b+1 (neighbour lanes by
// DPP wave shifts), then W9(a-1, b) = the maximum of R3 over rows a-2..a (the 3 x 3 (A, B)
// window), and puts W9 into LDS. After one barrier it reads the W9 of its two phi neighbours,
// P3 = the maximum of the three phi cells' W9, and tests row a-1: the own slab's parts come from
// registers, theta cell t - 1 gives P3(t - 1) (before), t + 1 gives P3(t + 1) (after), and the
// two phi neighbours in theta cell t join the before- or after-neighbours by their index (phi
// wraps: phi cell 0's left neighbour is the last one, an after-neighbour; the last one's right
// neighbour is phi cell 0, a before-neighbour). With phi sectors there are no phi neighbours,
// no LDS exchange and no barrier.
//
// Rows are read with buffer loads, one resource per row spanning that row of every theta cell's
// slab: a lane whose cell lies outside the row, or a row outside the segment's rows
// a_beg - 1 .. a_end (or outside the matrix), reads zero without touching memory. Each row is
// loaded kStAhead rows before its step into a ring of kStAhead + 1 register slots; the step loop
// is unrolled by kStUnroll, a multiple of the ring slots, of the three rows of R3 history and of
// the two LDS buffers, so all of them are fixed registers and offsets. The test of a row is a
// ballot; its bits 1..62 are the chunk's peak bits, one 64-bit peak word per (slab, row, chunk),
// staged in LDS and stored once per segment. The words are counted when they are stored, and each
// wave adds one count per group of tiles its words fall in (a segmented scan over its lanes): a
// count kept per row in scalar registers cost 35 scalar registers and about a tenth of the
// kernel's time.
// ---------------------------------------------------------------------------------------------
constexpr int kStAhead = 3;
constexpr int kStSlots = kStAhead + 1;
constexpr int kStUnroll = 12;
static_assert(kStUnroll % kStSlots == 0 && kStUnroll % 3 == 0, "ring slots, R3 history and LDS buffers must align");
// the fourth word of a buffer resource on gfx9-family parts: 32-bit data format, no swizzle
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint64_t kTestedLanes = 0x7ffffffffffffffeull;  // lanes 1..62
constexpr uint32_t kStOutside = 0x80000000u;                // a load offset past every resource
constexpr int kStWholeRows = 48;  // segments up to this many rows keep all their peak words in LDS

__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) { return max(a, max(b, c)); }
// lane j - 1's value (wave_shr:1; lane 0 gets 0)
__device__ __forceinline__ uint32_t lane_left(uint32_t v)
{
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);
}
// lane j + 1's value (wave_shl:1; lane 63 gets 0)
__device__ __forceinline__ uint32_t lane_right(uint32_t v)
{
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);
}

// Inclusive maximum over a wave64, with the DPP steps of the inclusive sum (a lane whose source
// lies outside its row takes the maximum with 0). Every lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_max(uint32_t v)
{
  return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v)
{
  v = dpp_max<0x111, 0xf>(v);
  v = dpp_max<0x112, 0xf>(v);
  v = dpp_max<0x114, 0xf>(v);
  v = dpp_max<0x118, 0xf>(v);
  v = dpp_max<0x142, 0xa>(v);
  v = dpp_max<0x143, 0xc>(v);
  return v;
}

// Adds the peaks of one 64-bit peak word per lane to the peak counts of their groups of tiles.
// The words a wave holds are in (theta cell, row) order, so the lanes of one group form one run:
// a scan of the counts and a maximum-scan of the runs' starting sums give each run's total, which
// its last lane adds with one atomic. A lane with valid false (no word, or a row past the
// matrix) adds nothing and splits runs. Every lane of the wave must be active.
__device__ __forceinline__ void add_group_counts(uint32_t* group_pk, bool valid, uint32_t grp, uint64_t word)
{
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t gv = valid ? grp : 0xffffffffu;  // group numbers are below 2^31
  const uint32_t c = valid ? (uint32_t)__builtin_popcountll(word) : 0u;
  const uint32_t incl = wave_incl_scan(c);
  // the neighbours' groups are read by every lane (no short-circuit: a DPP read of a lane that
  // is switched off returns 0)
  const uint32_t gl = lane_left(gv), gr = lane_right(gv);
  const bool start = (lane == 0u) | (gl != gv);
  const bool last = (lane == 63u) | (gr != gv);
  const uint32_t run0 = wave_incl_max(start ? incl - c : 0u);
  if (valid && last && incl != run0) gatomic_add(group_pk + grp, incl - run0);
}

// Block b of a grid of G runs on XCD b % 8 (workgroups are dealt to the eight XCDs in turn); the
// number this returns is a bijection of [0, G) under which XCD x runs one contiguous range of
// numbers: the first G % 8 XCDs take ceil(G / 8) of them, the others floor(G / 8).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t G)
{
  const uint32_t x = b & 7u, i = b >> 3, q = G >> 3, r = G & 7u;
  return x < r ? x * (q + 1u) + i : r * (q + 1u) + (x - r) * q + i;
}

template <int NT, bool SECT>
__global__ __launch_bounds__(1024) void k_peak_stencil(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  // two buffers of W9, each [theta cell][16 phi slots][64 lanes]: fixed strides, so every LDS
  // address is one of three lane addresses plus a constant
  extern __shared__ uint32_t s_w9[];
  constexpr uint32_t kTBytes = 16u * 256u, kBufBytes = NT * kTBytes;
  EvDesc e = load_ev(ev0, evs);
  if (!e.dense) return;  // uniform: this event's peaks come from the candidate pool
  const uint32_t nb = (uint32_t)g.n_b;
  const int na = g.n_a, np = g.n_phi, S = g.dense_rows;
  const uint32_t lane = threadIdx.x & 63u;
  const int p = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nch = (int)((nb + kChunkCells - 1) / kChunkCells);
  // Workgroups are dealt to the eight XCDs in turn; renumbered so that each XCD takes one
  // contiguous range (adjacent chunks of the same rows, then the next rows), the cache lines that
  // neighbouring workgroups share (chunk edges overlap by two cells, segment edges by two rows)
  // are fetched into one L2. The row bounds are uniform (read from the first lane), so the row
  // loop and its tests stay scalar.
  const uint32_t lb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int chunk = __builtin_amdgcn_readfirstlane((int)lb % nch);
  const int a_beg = __builtin_amdgcn_readfirstlane(((int)lb / nch) * S);
  const int a_end = min(a_beg + S, na);
  const uint32_t base = (uint32_t)chunk * kChunkCells;
  const uint32_t row_bytes = nb * 4u;
  // The next row to load (row a_beg - 1 first), as a byte address in slab (0, p). One buffer
  // resource per row covers the NT rows of slabs (0..NT-1, p), theta cell t's row t t_bytes
  // further (a scalar offset). A lane's offset is its cell's, or kStOutside for cells outside the
  // row (the cell left of B = 0, cells past n_b), which the range check turns into zeros (with
  // or without the scalar offset counted in it: kStOutside is past the resource either way), as
  // it does every load of a row outside the segment's rows a_beg - 1 .. a_end or the matrix (an
  // empty resource). The address is never dereferenced outside the rows read.
  const uintptr_t slab_bytes = (uintptr_t)na * row_bytes;
  const uint32_t t_bytes = (uint32_t)((uintptr_t)np * slab_bytes);  // (NT-1) t_bytes + row_bytes < 2^31
  const uint32_t span = (uint32_t)(NT - 1) * t_bytes + row_bytes;
  const bool cell_in = !(base == 0u && lane == 0u) && base + lane - 1u < nb;
  const uint32_t off = cell_in ? (base + lane - 1u) * 4u : kStOutside;
  uintptr_t rp = (uintptr_t)e.acc + (uintptr_t)p * slab_bytes + (uintptr_t)a_beg * row_bytes - row_bytes;
  int ra = a_beg - 1;  // the row of the next load
  const uint32_t own_a = (uint32_t)p * 256u + 4u * lane;
  const uint32_t pm_a = (uint32_t)(p == 0 ? np - 1 : p - 1) * 256u + 4u * lane;
  const uint32_t pq_a = (uint32_t)(p + 1 == np ? 0 : p + 1) * 256u + 4u * lane;
  const bool p_mid = p > 0 && p + 1 < np;  // phi neighbours: one before, one after
  const uint32_t T = g.threshold;
  const uint32_t rows_log2 = (uint32_t)__ffs(g.rows) - 1u;
  const uint32_t gt_log2 = (uint32_t)__ffs(g.group_tiles) - 1u;
  // The peak word of (slab sl, row a = seg S + r, chunk c) is at ((sl n_seg + seg) nch + c) S + r:
  // a wave's words of one theta cell form one contiguous run of S words, and the words of a
  // group of tiles (rows of one or two slabs) lie close together for the writer. A wave's words
  // wait in its own LDS staging slots, [row][theta cell] after the W9 buffers: for the whole
  // segment when it has at most kStWholeRows rows (the default), and go out at the end; else for
  // a block of kStUnroll rows, and go out after each block. Stores of peak words are slow to
  // complete, and every one is waited for with the loads of the rows that follow it, so a wave
  // stores as few times as it can.
  // (the word's position, computed where the words are stored: kept out of the step loop's
  // scalar registers)
#define HT_ST_MW()                                                                             \
  const uint32_t n_seg_ = ((uint32_t)na + (uint32_t)S - 1u) / (uint32_t)S;                     \
  GLOBAL uint64_t* const mw = reinterpret_cast<GLOBAL uint64_t*>(gp(e.pk_mask)) +              \
      (((size_t)p * n_seg_ + (size_t)(lb / (uint32_t)nch)) * (size_t)nch + (size_t)chunk) * (size_t)S; \
  const uint32_t mt_words = (uint32_t)np * n_seg_ * (uint32_t)nch * (uint32_t)S  /* t to t + 1 */
  constexpr uint32_t kStageStep = NT * 8u;  // bytes per row in a wave's slots
  const bool whole = S <= kStWholeRows;     // uniform
  const uint32_t slot_rows = whole ? (uint32_t)S : (uint32_t)kStUnroll;
  char* const stage_w = reinterpret_cast<char*>(s_w9) + (SECT ? 0u : 2u * kBufBytes) +
                        (uint32_t)p * slot_rows * kStageStep;
  // slot (row u, t) is at stage_w + 8 (u NT + t): written by lane 0, read back by the flush
  char* stage_blk = stage_w;  // lane 0's slots of the block's first row
  // group of tiles of theta cell t's row a (a below n_a)
  auto group_of = [&](uint32_t t, uint32_t a) {
    return ((t * (uint32_t)np + (uint32_t)p) * (uint32_t)g.tiles_per_slab + (a >> rows_log2)) >> gt_log2;
  };
  uint32_t ring[kStSlots][NT], hist[3][NT];

  // The next row (rows outside [a_beg - 1, a_end] or the matrix read zeros) into ring slot
  // slot_ (a constant).
#define HT_ST_LOAD(slot_)                                                                      \
  do {                                                                                         \
    const int nr_ = (ra >= 0 && ra <= a_end && ra < na) ? (int)span : 0;                      \
    const __amdgpu_buffer_rsrc_t r_ = __builtin_amdgcn_make_buffer_rsrc((void*)rp, 0, nr_, kRsrcWord3); \
    _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_)                                          \
      ring[slot_][t_] = __builtin_amdgcn_raw_buffer_load_b32(r_, off, (uint32_t)t_ * t_bytes, 0); \
    rp += row_bytes;                                                                           \
    ++ra;                                                                                      \
  } while (0)
  // R3 of step kc_'s row (kc_ a constant congruent to the step modulo kStUnroll) into history
  // slot kc_ % 3
#define HT_ST_R3(kc_)                                                                          \
  do {                                                                                         \
    _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_) {                                        \
      const uint32_t v_ = ring[(kc_) % kStSlots][t_];                                          \
      hist[(kc_) % 3][t_] = max(max(lane_left(v_), v_), lane_right(v_));                       \
    }                                                                                          \
  } while (0)
  // The test of the row in ring slot vs_ (R3 above in h0_, below in h2_) for every theta cell.
  // Its phi neighbours in the own theta cell join the before- or after-neighbours by the wave's
  // class c_ (a constant; uniform per wave): 0 phi cells 1 .. n_phi - 2 (phi - 1 before, phi + 1
  // after; also sectors, which have none), 1 phi cell 0 (both after: phi - 1 wraps to the last),
  // 2 the last phi cell (both before: phi + 1 wraps to 0).
#define HT_ST_TEST(c_)                                                                         \
  do {                                                                                         \
    _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_) {                                        \
      const uint32_t vm_ = ring[vs_][t_];                                                      \
      uint32_t mb_ = max(lane_left(vm_), hist[h0_][t_]);                                       \
      uint32_t ma_ = max(lane_right(vm_), hist[h2_][t_]);                                      \
      const uint32_t pb_ = t_ > 0 ? p3_[t_ > 0 ? t_ - 1 : 0] : 0u;                             \
      const uint32_t pa_ = t_ + 1 < NT ? p3_[t_ + 1 < NT ? t_ + 1 : 0] : 0u;                   \
      if (SECT) {                                                                              \
        mb_ = max(mb_, pb_);                                                                   \
        ma_ = max(ma_, pa_);                                                                   \
      } else if ((c_) == 0) {                                                                  \
        mb_ = max3u(mb_, pb_, wm_[t_]);                                                        \
        ma_ = max3u(ma_, pa_, wq_[t_]);                                                        \
      } else if ((c_) == 1) {                                                                  \
        mb_ = max(mb_, pb_);                                                                   \
        ma_ = max3u(ma_, pa_, max(wm_[t_], wq_[t_]));                                          \
      } else {                                                                                 \
        mb_ = max3u(mb_, pb_, max(wm_[t_], wq_[t_]));                                          \
        ma_ = max(ma_, pa_);                                                                   \
      }                                                                                        \
      pk_[t_] = __builtin_amdgcn_ballot_w64(vm_ >= max3u(mb_ + 1u, ma_, T)) & kTestedLanes;   \
    }                                                                                          \
  } while (0)
  // Step kb_ + kc_ (kc_ >= 2 a constant, kb_ a multiple of kStUnroll): R3 of its row completes W9
  // of the row before; W9 goes to LDS buffer kc_ % 2, and after one barrier the phi neighbours'
  // are read and the row before is tested; then the row kStAhead steps on is loaded into the
  // slot of that tested row.
#define HT_ST_STEP(kc_, kb_)                                                                   \
  do {                                                                                         \
    HT_ST_R3(kc_);                                                                             \
    constexpr int h0_ = ((kc_) + 1) % 3, h1_ = ((kc_) + 2) % 3, h2_ = (kc_) % 3;               \
    constexpr int vs_ = ((kc_) + kStSlots - 1) % kStSlots;                                     \
    uint32_t w9_[NT], p3_[NT], wm_[NT], wq_[NT];                                               \
    _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_)                                          \
      w9_[t_] = max3u(hist[h0_][t_], hist[h1_][t_], hist[h2_][t_]);                            \
    if (!SECT) {                                                                               \
      char* B_ = reinterpret_cast<char*>(s_w9) + ((kc_) % 2) * kBufBytes;                      \
      _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_)                                        \
        *reinterpret_cast<uint32_t*>(B_ + t_ * kTBytes + own_a) = w9_[t_];                     \
      lds_barrier();                                                                           \
      _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_) {                                      \
        wm_[t_] = *reinterpret_cast<const uint32_t*>(B_ + t_ * kTBytes + pm_a);                \
        wq_[t_] = *reinterpret_cast<const uint32_t*>(B_ + t_ * kTBytes + pq_a);                \
        p3_[t_] = max3u(wm_[t_], w9_[t_], wq_[t_]);                                            \
      }                                                                                        \
    } else {                                                                                   \
      _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_) p3_[t_] = wm_[t_] = wq_[t_] = w9_[t_]; \
    }                                                                                          \
    uint64_t pk_[NT];                                                                          \
    if (SECT || p_mid) HT_ST_TEST(0);                                                          \
    else if (p == 0) HT_ST_TEST(1);                                                            \
    else HT_ST_TEST(2);                                                                        \
    if (lane == 0u) { /* lane 0 puts the words into the wave's staging slots */               \
      _Pragma("unroll") for (int t_ = 0; t_ < NT; ++t_)                                        \
        *reinterpret_cast<uint64_t*>(stage_blk + ((kc_) - 2) * kStageStep + 8 * t_) = pk_[t_]; \
    }                                                                                          \
    HT_ST_LOAD(vs_);                                                                           \
  } while (0)

  // steps 0 and 1 (rows a_beg - 1 and a_beg) only start the R3 history
#pragma unroll
  for (int k = 0; k < kStAhead; ++k) HT_ST_LOAD(k);
  HT_ST_R3(0);
  HT_ST_LOAD(kStAhead % kStSlots);
  HT_ST_R3(1);
  HT_ST_LOAD((1 + kStAhead) % kStSlots);
  // steps 2 .. S + 1 test rows a_beg .. a_beg + S - 1 (S is a multiple of kStUnroll)
  for (int kb = 0; kb < S; kb += kStUnroll) {  // uniform
    HT_ST_STEP(2, kb);
    HT_ST_STEP(3, kb);
    HT_ST_STEP(4, kb);
    HT_ST_STEP(5, kb);
    HT_ST_STEP(6, kb);
    HT_ST_STEP(7, kb);
    HT_ST_STEP(8, kb);
    HT_ST_STEP(9, kb);
    HT_ST_STEP(10, kb);
    HT_ST_STEP(11, kb);
    HT_ST_STEP(12, kb);
    HT_ST_STEP(13, kb);
    if (whole) {  // uniform
      stage_blk += kStUnroll * kStageStep;
    } else {
      // the block's words leave the staging slots: lane t kStUnroll + u stores theta cell t's
      // word of the block's u-th row (runs of kStUnroll words). Lane 0 wrote the slots: the
      // fence keeps these reads after its writes (with phi sectors no barrier orders them).
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
      HT_ST_MW();
      const bool in = lane < (uint32_t)(kStUnroll * NT);
      const uint32_t t = in ? lane / kStUnroll : 0u, u = in ? lane - t * kStUnroll : 0u;
      const uint64_t w = *reinterpret_cast<const uint64_t*>(stage_w + 8u * (u * NT + t));
      if (in) mw[(size_t)t * mt_words + (size_t)kb + u] = w;
      const uint32_t a = (uint32_t)(a_beg + kb) + u;
      add_group_counts(e.group_pk, in && a < (uint32_t)na, group_of(t, a), w);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    }
  }
  if (whole) {  // uniform: the segment's words, a run of S per theta cell
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    HT_ST_MW();
    const uint32_t n_w = (uint32_t)S * NT;
    for (uint32_t j0 = 0; j0 < n_w; j0 += 64u) {  // uniform: every lane counts
      const uint32_t j = j0 + lane;
      const bool in = j < n_w;
      const uint32_t t = in ? j / (uint32_t)S : 0u, r = in ? j - t * (uint32_t)S : 0u;
      const uint64_t w = *reinterpret_cast<const uint64_t*>(stage_w + 8u * (r * NT + t));
      if (in) mw[(size_t)t * mt_words + r] = w;
      const uint32_t a = (uint32_t)a_beg + r;
      add_group_counts(e.group_pk, in && a < (uint32_t)na, group_of(t, a), w);
    }
  }
#undef HT_ST_STEP
#undef HT_ST_TEST
#undef HT_ST_MW
#undef HT_ST_R3
#undef HT_ST_LOAD
}

// Ordered output of a dense event: one workgroup per group of tiles (a contiguous range of rows
// of the matrix, so of peak-mask words); its output offset is the sum of the earlier groups'
// peak counts. Thread t takes the t-th of 256 equal, contiguous pieces of the group's words, all
// loaded at once; one block scan of the pieces' peak counts gives each thread where its peaks
// go, in cell order (words in row, then chunk order; bits 1..62 of a word are the chunk's cells
// in B order).
constexpr int kWriteStage = 4096;  // peaks of a group staged in LDS by the dense writer

__global__ __launch_bounds__(kBlock) void k_peak_write_dense(DevGrid g, EvDesc ev0, const EvDesc* evs,
                                                               uint32_t stage_cap)
{
  __shared__ uint32_t smem[32];
  __shared__ uint32_t s_cells[kWriteStage];
  EvDesc e = load_ev(ev0, evs);
  if (!e.dense) return;
  const int G = blockIdx.x;
  const int t0 = G * g.group_tiles;
  const int nt = min(g.group_tiles, g.n_tiles - t0);
  const bool a8 = ((uintptr_t)e.out & 7u) == 0;
  uint32_t c_beg, L0, c_last, L1;
  tile_range(g, t0, &c_beg, &L0);
  tile_range(g, t0 + nt - 1, &c_last, &L1);
  const uint32_t nb = (uint32_t)g.n_b, nch = (nb + kChunkCells - 1) / kChunkCells;
  // The group's rows [c_beg / nb, (c_last + L1) / nb) of the slab-major row order, so its words
  // in cell order ("logical" words w = (slab n_a + a) nch + chunk). The stencil stored the word
  // of (slab sl, row a = seg S + r, chunk c) at ((sl n_seg + seg) nch + c) S + r; a thread walks
  // its logical words with that position kept up to date.
  const uint32_t w0 = (c_beg / nb) * nch, w1 = (uint32_t)(((uint64_t)c_last + L1) / nb) * nch;
  const uint32_t per = (w1 - w0 + kBlock - 1) / kBlock;
  const uint32_t lo = min(w1, w0 + per * threadIdx.x), hi = min(w1, lo + per);
  const GLOBAL uint64_t* mw = reinterpret_cast<const GLOBAL uint64_t*>(gp((const uint8_t*)e.pk_mask));
  const uint32_t na = (uint32_t)g.n_a, S = (uint32_t)g.dense_rows;
  const uint32_t n_seg = (na + S - 1u) / S;
  uint32_t ch = lo % nch, a = (lo / nch) % na, sl = lo / nch / na;
  uint32_t seg = a / S, r = a - seg * S;
  auto rewind = [&]() {
    ch = lo % nch;
    a = (lo / nch) % na;
    sl = lo / nch / na;
    seg = a / S;
    r = a - seg * S;
  };
  auto phys = [&]() { return ((sl * n_seg + seg) * nch + ch) * S + r; };
  auto next = [&]() {
    if (++ch == nch) {
      ch = 0;
      if (++r == S) {
        r = 0;
        ++seg;
      }
      if (++a == na) {
        a = 0;
        seg = 0;
        r = 0;
        ++sl;
      }
    }
  };
  constexpr int kMaxW = 16;  // up to 16 words per thread held in registers
  uint64_t wv[kMaxW];
  uint32_t cnt = 0;
  const int nw = (int)(hi - lo);
  if (per <= (uint32_t)kMaxW) {  // uniform
#pragma unroll
    for (int k = 0; k < kMaxW; ++k) {
      wv[k] = k < nw ? mw[phys()] : 0ull;
      next();
    }
  }
  // the earlier groups' peak counts give the output offset (loaded while the words arrive)
  uint32_t part = 0;
  for (int i0 = 0; i0 < G; i0 += 4 * kBlock) {  // uniform
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k * kBlock + (int)threadIdx.x;
      w[k] = i < G ? gp(e.group_pk)[i] : 0u;
    }
    part += w[0] + w[1] + w[2] + w[3];
  }
  const int64_t base = (int64_t)block_sum(part, smem);
  if (G == (int)gridDim.x - 1 && threadIdx.x == 0) *gp(e.n_found) = base + gp(e.group_pk)[G];
  if (base >= e.cap) return;  // uniform
  if (per <= (uint32_t)kMaxW) {  // uniform
#pragma unroll
    for (int k = 0; k < kMaxW; ++k) cnt += (uint32_t)__builtin_popcountll(wv[k]);
  } else {
    for (uint32_t w = lo; w < hi; ++w) {
      cnt += (uint32_t)__builtin_popcountll(mw[phys()]);
      next();
    }
  }
  uint32_t tot;
  const uint32_t lo_pk = block_excl_scan(cnt, smem, &tot);  // the thread's first peak in the group
  // Cell of bit j of word w: row w / nch, chunk w % nch, B = chunk * kChunkCells + j - 1. A group
  // of at most kWriteStage peaks (the common case) first lists its cells in LDS, in order; then
  // every thread loads the votes of every 256th of them at once and stores those peaks, so the
  // group's vote loads take one round trip whichever threads own the crowded words, and the
  // stores are contiguous. A larger group emits each thread's peaks itself, loading the votes of
  // up to four at a time.
#define HT_FOR_PEAKS(w_, bits_, body_)                                                         \
  do {                                                                                         \
    uint64_t b_ = (bits_);                                                                     \
    if (b_) {                                                                                  \
      const uint32_t row_ = (w_) / nch;                                                        \
      const uint32_t c0_ = row_ * nb + ((w_) - row_ * nch) * kChunkCells - 1u;                 \
      while (b_) {                                                                             \
        const uint32_t c_ = c0_ + (uint32_t)__builtin_ctzll(b_);                               \
        b_ &= b_ - 1ull;                                                                       \
        body_;                                                                                 \
      }                                                                                        \
    }                                                                                          \
  } while (0)
  if (tot <= stage_cap) {  // uniform (stage_cap <= kWriteStage)
    uint32_t i = lo_pk;
    if (per <= (uint32_t)kMaxW) {  // uniform
#pragma unroll
      for (int k = 0; k < kMaxW; ++k) HT_FOR_PEAKS(lo + (uint32_t)k, wv[k], s_cells[i++] = c_);
    } else {
      rewind();
      for (uint32_t w = lo; w < hi; ++w) {
        HT_FOR_PEAKS(w, mw[phys()], s_cells[i++] = c_);
        next();
      }
    }
    lds_barrier();
    constexpr int kRounds = kWriteStage / kBlock;
    uint32_t c[kRounds], v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t k = (uint32_t)r * kBlock + threadIdx.x;
      c[r] = s_cells[k < tot ? k : 0u];
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
      if ((uint32_t)r * kBlock < tot) v[r] = gp(e.acc)[c[r]];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t k = (uint32_t)r * kBlock + threadIdx.x;
      if (k < tot && base + (int64_t)k < e.cap) st_peak(e.out, base + (int64_t)k, c[r], v[r], a8);
    }
    return;
  }
  int64_t o = base + (int64_t)lo_pk;
  if (o >= e.cap || cnt == 0) return;
#define HT_EMIT_WORD(w_, bits_)                                                                \
  do {                                                                                         \
    uint64_t b_ = (bits_);                                                                     \
    if (b_) {                                                                                  \
      const uint32_t row_ = (w_) / nch;                                                        \
      const uint32_t c0_ = row_ * nb + ((w_) - row_ * nch) * kChunkCells - 1u;                 \
      while (b_) {                                                                             \
        uint32_t c_[4], v_[4];                                                                 \
        int n_ = 0;                                                                            \
        _Pragma("unroll") for (int q_ = 0; q_ < 4; ++q_) {                                     \
          c_[q_] = c0_ + (b_ ? (uint32_t)__builtin_ctzll(b_) : 1u);                            \
          n_ += b_ ? 1 : 0;                                                                    \
          b_ &= b_ - 1ull;                                                                     \
        }                                                                                      \
        _Pragma("unroll") for (int q_ = 0; q_ < 4; ++q_) v_[q_] = gp(e.acc)[c_[q_]];          \
        _Pragma("unroll") for (int q_ = 0; q_ < 4; ++q_) {                                     \
          if (q_ < n_ && o < e.cap) st_peak(e.out, o, c_[q_], v_[q_], a8);                     \
          o += q_ < n_ ? 1 : 0;                                                                \
        }                                                                                      \
      }                                                                                        \
    }                                                                                          \
  } while (0)
  if (per <= (uint32_t)kMaxW) {  // uniform
#pragma unroll
    for (int k = 0; k < kMaxW; ++k) HT_EMIT_WORD(lo + (uint32_t)k, wv[k]);
  } else {
    rewind();
    for (uint32_t w = lo; w < hi; ++w) {
      HT_EMIT_WORD(w, mw[phys()]);
      next();
    }
  }
#undef HT_EMIT_WORD
#undef HT_FOR_PEAKS
}

// ---------------------------------------------------------------------------------------------
// Plain fill: zero the matrix, then one global atomicAdd per vote. One block per hit, its
// threads over the A bins (the decomposition the paper describes, kept as a baseline).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_zero_acc(DevGrid g, EvDesc ev0, const EvDesc* evs,
                                                     uint64_t cells)
{
  EvDesc e = load_ev(ev0, evs);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < cells; i += stride)
    e.acc[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_fill_atomic(DevGrid g, EvDesc ev0, const EvDesc* evs)
{
  EvDesc e = load_ev(ev0, evs);
  const int64_t h = blockIdx.x;
  if (h >= e.n_hits) return;
  int slabs[4];
  int ns = 0;
  for (int q = 0; q < 4; ++q) {
    int s = e.hit_slab[4 * h + q];
    if (s >= 0) slabs[ns++] = s;
  }
  if (ns == 0) return;
  const float4 rec = e.hit_rec[h];
  const float x = rec.x, r2 = rec.y, k = rec.z;
  for (int i = threadIdx.x; i < g.n_a; i += kBlock) {
    float ax = g.a2[i] * x;
    float num = r2 - ax;
    float B = num * k;
    float d = B - g.b_min;
    float f = d * g.inv_db;
    if (f >= 0.0f && f < g.nb_f) {
      const uint32_t j = (uint32_t)(int)f;
      for (int q = 0; q < ns; ++q)
        atomicAdd(&e.acc[((uint64_t)slabs[q] * g.n_a + i) * g.n_b + j], 1u);
    }
  }
}

// Track parameters of each peak: bin indices, bin-centre (A, B), rho, phi, theta in double.
__global__ __launch_bounds__(kBlock) void k_readout(DevGrid g, const ht_peak* peaks, const int64_t* n_found,
                                                    int64_t cap, ht_track* tracks, double b_min,
                                                    double db)
{
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = min(*n_found, cap);
  if (i >= n) return;
  const ht_peak pk = peaks[i];
  uint32_t t, p, a, b;
  cell_coords(g, pk.cell, &t, &p, &a, &b);
  const double A = 0.5 * (double)g.a2[a];
  const double B = b_min + ((double)b + 0.5) * db;
  double phi = atan2(B, A);
  if (phi < 0.0) phi += 2.0 * 3.14159265358979323846;
  ht_track tr;
  tr.cell = pk.cell;
  tr.votes = pk.votes;
  tr.t = (int32_t)t;
  tr.p = (int32_t)p;
  tr.a = (int32_t)a;
  tr.b = (int32_t)b;
  tr.A = (float)A;
  tr.B = (float)B;
  tr.rho = (float)sqrt(A * A + B * B);
  tr.phi = (float)phi;
  tr.theta = (float)(((double)t + 0.5) * 3.14159265358979323846 / (double)g.n_theta);
  tracks[i] = tr;
}

__global__ __launch_bounds__(kBlock) void k_debug_hits(DevGrid g, const float* x, const float* y,
                                                       const float* z, int64_t n, int32_t* info,
                                                       float* vals, int32_t* slabs)
{
  const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (h >= n) return;
  HitPrep p = prep_hit(g, g.phi_cs, g.th_cs, x[h], y[h], z[h]);
  info[4 * h + 0] = p.n > 0;
  info[4 * h + 1] = p.s_theta;
  info[4 * h + 2] = p.s_phi;
  info[4 * h + 3] = p.n;
  vals[3 * h + 0] = p.r2;
  vals[3 * h + 1] = p.r;
  vals[3 * h + 2] = p.k;
  for (int q = 0; q < 4; ++q) slabs[4 * h + q] = q < p.n ? p.slab[q] : -1;
}

__global__ __launch_bounds__(kBlock) void k_debug_unary(const float* v, float* root, float* inv2,
                                                        int64_t n)
{
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const float a = v[i];
    root[i] = hit_root(a);
    inv2[i] = hit_inv2(a);
  }
}
hipError_t launch_fill_nt(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev, bool nt,
                          bool vec, bool emit, bool long_lists, size_t lds, hipStream_t s)
{
  switch (g.rows) {
    case 1: return launch_fill_for_rows<1>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 2: return launch_fill_for_rows<2>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 4: return launch_fill_for_rows<4>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 8: return launch_fill_for_rows<8>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 16: return launch_fill_for_rows<16>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 32: return launch_fill_for_rows<32>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    case 64: return launch_fill_for_rows<64>(g, ev0, evs, n_ev, nt, vec, emit, long_lists, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int n_groups(const DevGrid& g) { return (g.n_tiles + g.group_tiles - 1) / g.group_tiles; }

size_t fill_lds_bytes(const DevGrid& g)
{
  const size_t lpad = (((size_t)g.rows * g.n_b) + 3) & ~(size_t)3;
  return (lpad + 16) * sizeof(uint32_t);
}

hipError_t launch_prep(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                       int64_t max_hits, bool direct, hipStream_t s)
{
  const unsigned blocks = (unsigned)std::max<int64_t>(1, (max_hits + kBlock - 1) / kBlock);
  // the boundary tables: 4 n_phi + 2 (2 n_theta + 1) floats (about 300 B for the paper grid)
  const size_t tab = (size_t)(4 * g.n_phi + 2 * (2 * g.n_theta + 1)) * sizeof(float);
  const bool lds = tab <= kLdsTableBytes;
  if (direct) {
    if (lds) hipLaunchKernelGGL(k_prep_direct<true>, dim3(blocks, n_ev), dim3(kBlock), tab, s, g, ev0, evs);
    else hipLaunchKernelGGL(k_prep_direct<false>, dim3(blocks, n_ev), dim3(kBlock), 0, s, g, ev0, evs);
    return hipGetLastError();
  }
  if (lds) hipLaunchKernelGGL(k_prep<true>, dim3(blocks, n_ev), dim3(kBlock), tab, s, g, ev0, evs);
  else hipLaunchKernelGGL(k_prep<false>, dim3(blocks, n_ev), dim3(kBlock), 0, s, g, ev0, evs);
  hipLaunchKernelGGL(k_bucket, dim3(blocks, n_ev), dim3(kBlock), 0, s, g, ev0, evs);
  return hipGetLastError();
}

hipError_t launch_fill(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                       bool emit, int64_t max_hits, hipStream_t s)
{
  // more than two records per thread expected per slab (a hit has at most four cells, about
  // three on average): load eight per thread per round trip
  const bool long_lists = max_hits * 3 > (int64_t)2 * kBlock * g.n_slabs;
  // store kind 2: 4-byte stores (the dword path), otherwise 16-byte stores where rows allow
  const bool vec = (g.n_b % 4) == 0 && g.nt_store != 2;
  // long lists: 64 spill words past the tile (one per lane) for votes outside the row
  const size_t lds = fill_lds_bytes(g) + (long_lists ? 64 * sizeof(uint32_t) : 0);
  return launch_fill_nt(g, ev0, evs, n_ev, g.nt_store == 1, vec, emit, long_lists, lds, s);
}

hipError_t launch_candidates(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                             hipStream_t s)
{
  dim3 grid(g.n_tiles, n_ev);
  if (!g.lds_fill) {
    // rows wider than an LDS tile (up to 2^24 cells): read from the matrix directly
    hipLaunchKernelGGL(k_cand_scan_wide, grid, dim3(kBlock), 0, s, g, ev0, evs);
    return hipGetLastError();
  }
  const size_t lds = fill_lds_bytes(g);
  if (g.n_b % 4 == 0) hipLaunchKernelGGL(k_cand_scan<true>, grid, dim3(kBlock), lds, s, g, ev0, evs);
  else hipLaunchKernelGGL(k_cand_scan<false>, grid, dim3(kBlock), lds, s, g, ev0, evs);
  return hipGetLastError();
}

hipError_t launch_peaks(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                        hipStream_t s)
{
  hipLaunchKernelGGL(k_peak_test, dim3(g.test_blocks, n_ev), dim3(kBlock), 0, s, g, ev0, evs);
  hipLaunchKernelGGL(k_peak_write, dim3(n_groups(g), n_ev), dim3(kBlock), 0, s, g, ev0, evs);
  return hipGetLastError();
}

int dense_blocks(const DevGrid& g)
{
  return ((g.n_b + kChunkCells - 1) / kChunkCells) * ((g.n_a + g.dense_rows - 1) / g.dense_rows);
}

hipError_t launch_peaks_dense(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                              hipStream_t s)
{
  // one wave per phi cell; two LDS buffers of 16 phi slots of 64 window maxima per theta cell
  // (none with sectors), then every wave's staging slots for the peak words of its segment's
  // rows (or of 12 rows when the segment is longer than kStWholeRows)
  const dim3 grid(dense_blocks(g), n_ev), block(64 * g.n_phi);
  const int slot_rows = g.dense_rows <= kStWholeRows ? g.dense_rows : kStUnroll;
  const size_t lds = (g.phi_sectors ? 0 : 2 * (size_t)g.n_theta * 16 * 256) +
                     (size_t)g.n_phi * slot_rows * g.n_theta * 8;
#define HT_ST_CASE(nt_)                                                                        \
  case nt_:                                                                                    \
    if (g.phi_sectors) hipLaunchKernelGGL((k_peak_stencil<nt_, true>), grid, block, lds, s, g, ev0, evs); \
    else hipLaunchKernelGGL((k_peak_stencil<nt_, false>), grid, block, lds, s, g, ev0, evs);  \
    break
  switch (g.n_theta) {
    HT_ST_CASE(1);
    HT_ST_CASE(2);
    HT_ST_CASE(3);
    HT_ST_CASE(4);
    default: return hipErrorInvalidValue;  // the tiling offers the stencil for 1-4 theta cells only
  }
#undef HT_ST_CASE
  // HT_DENSE_STAGE (tests): stage at most that many peaks of a group in LDS, so that smaller
  // groups take the writer's other path
  uint32_t stage_cap = kWriteStage;
  if (const char* v = std::getenv("HT_DENSE_STAGE")) {
    const long c = std::strtol(v, nullptr, 10);
    if (c >= 0 && c < kWriteStage) stage_cap = (uint32_t)c;
  }
  hipLaunchKernelGGL(k_peak_write_dense, dim3(n_groups(g), n_ev), dim3(kBlock), 0, s, g, ev0, evs, stage_cap);
  return hipGetLastError();
}

hipError_t launch_fill_atomic(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs, int n_ev,
                              int64_t max_hits, hipStream_t s)
{
  const uint64_t cells = (uint64_t)g.n_slabs * g.n_a * g.n_b;
  hipLaunchKernelGGL(k_zero_acc, dim3(4096, n_ev), dim3(kBlock), 0, s, g, ev0, evs, cells);
  hipLaunchKernelGGL(k_fill_atomic, dim3((unsigned)std::max<int64_t>(max_hits, 1), n_ev), dim3(kBlock), 0,
                     s, g, ev0, evs);
  return hipGetLastError();
}

hipError_t launch_readout(const DevGrid& g, const ht_peak* peaks, const int64_t* n_found, int64_t cap,
                          ht_track* tracks, double b_min, double db, hipStream_t s)
{
  if (cap > 0)
    hipLaunchKernelGGL(k_readout, dim3((unsigned)((cap + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g,
                       peaks, n_found, cap, tracks, b_min, db);
  return hipGetLastError();
}

hipError_t launch_debug_hits(const DevGrid& g, const float* x, const float* y, const float* z,
                             int64_t n, int32_t* info, float* vals, int32_t* slabs, hipStream_t s)
{
  if (n > 0)
    hipLaunchKernelGGL(k_debug_hits, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       g, x, y, z, n, info, vals, slabs);
  return hipGetLastError();
}

hipError_t launch_debug_unary(const float* v, float* root, float* inv2, int64_t n, hipStream_t s)
{
  if (n > 0) {
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL(k_debug_unary, dim3((unsigned)blocks), dim3(kBlock), 0, s, v, root, inv2, n);
  }
  return hipGetLastError();
}

}  // namespace ht