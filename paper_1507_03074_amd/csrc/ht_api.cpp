// ht_api.cpp -- C ABI of libht.so: validation, bin-rule tables, tiling, scratch, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ht_debug.h"
#include "ht_internal.h"

namespace ht {
hipError_t launch_debug_hits(const DevGrid& g, const float* x, const float* y, const float* z,
                             int64_t n, int32_t* info, float* vals, int32_t* slabs, hipStream_t s);
hipError_t launch_debug_unary(const float* v, float* root, float* inv2, int64_t n, hipStream_t s);

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what)
{
  return fail(e == hipErrorOutOfMemory ? HT_ENOMEM : HT_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

static const double kPi = 3.14159265358979323846;

int validate_grid(const ht_grid* g)
{
  if (!g) return fail(HT_EINVAL, "grid is NULL");
  if (g->phi_sectors != 0 && g->phi_sectors != 1) return fail(HT_EINVAL, "phi_sectors must be 0 or 1");
  if (g->n_theta < 1 || g->n_phi < (g->phi_sectors ? 1 : 3) || g->n_a < 1 || g->n_b < 1)
    return fail(HT_EINVAL, "grid needs n_theta >= 1, n_phi >= 3 (>= 1 with phi sectors), n_a >= 1, n_b >= 1");
  if (g->n_a > (1 << 24) || g->n_b > (1 << 24)) return fail(HT_EINVAL, "n_a and n_b must be <= 2^24");
  if ((int64_t)g->n_theta * g->n_phi > kMaxSlabs) return fail(HT_EINVAL, "n_theta*n_phi must be <= 4096");
  if (!std::isfinite(g->a_min) || !std::isfinite(g->a_max) || !std::isfinite(g->b_min) ||
      !std::isfinite(g->b_max))
    return fail(HT_EINVAL, "grid ranges must be finite");
  if (!(g->a_min < g->a_max) || !(g->b_min < g->b_max))
    return fail(HT_EINVAL, "grid ranges need min < max");
  if (g->threshold < 1) return fail(HT_EINVAL, "threshold must be >= 1");
  const double cells = (double)g->n_theta * g->n_phi * (double)g->n_a * (double)g->n_b;
  if (cells > 4294967296.0) return fail(HT_EINVAL, "more than 2^32 cells");
  return HT_OK;
}

uint64_t n_cells(const ht_grid& g) { return (uint64_t)g.n_theta * g.n_phi * g.n_a * g.n_b; }

// Bin-rule tables, computed in double and rounded once to float.
void host_tables_into(const ht_grid& g, float* a2, float* inv_db, float* phi, float* th)
{
  const double da = ((double)g.a_max - (double)g.a_min) / (double)g.n_a;
  for (int32_t i = 0; i < g.n_a; ++i)
    a2[i] = (float)(2.0 * (double)g.a_min + (double)(2 * (int64_t)i + 1) * da);
  *inv_db = (float)((double)g.n_b / ((double)g.b_max - (double)g.b_min));
  for (int32_t m = 0; m < 2 * g.n_phi; ++m) {
    const double ang = ((double)m * kPi) / (double)g.n_phi;
    phi[2 * m] = (float)std::cos(ang);
    phi[2 * m + 1] = (float)std::sin(ang);
  }
  for (int32_t m = 0; m <= 2 * g.n_theta; ++m) {
    const double ang = ((double)m * kPi) / (double)(2 * g.n_theta);
    th[2 * m] = (float)std::cos(ang);
    th[2 * m + 1] = (float)std::sin(ang);
  }
}

void host_tables(const ht_grid& g, std::vector<float>& a2, float& inv_db, std::vector<float>& phi,
                 std::vector<float>& th)
{
  a2.resize(a2_floats(g));
  phi.resize(phi_floats(g));
  th.resize(th_floats(g));
  host_tables_into(g, a2.data(), &inv_db, phi.data(), th.data());
}

// ---------------------------------------------------------------------------------------------
// Tiling
// ---------------------------------------------------------------------------------------------
static int env_int(const char* name, int def)
{
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : def;
}

// Largest power-of-two row count (<= 64) whose u32 tile fits the LDS budget; the candidate
// slots per tile scale with the tile (1/32 of its cells, 64..1024).
// Per-grid launch shapes set through ht_set_tuning (keyed by dimensions and ranges).
typedef std::tuple<int32_t, int32_t, int32_t, int32_t, uint32_t, uint32_t, uint32_t, uint32_t> TuneKey;
static std::mutex g_tune_mu;
static std::map<TuneKey, ht_tuning> g_tune;

static uint32_t fbits(float f);

static TuneKey tune_key(const ht_grid& g)
{
  return TuneKey{g.n_theta, g.n_phi, g.n_a, g.n_b, fbits(g.a_min), fbits(g.a_max), fbits(g.b_min),
                 fbits(g.b_max)};
}

static const int64_t kLdsTileMax = 65536 - 8192;  // bytes of an LDS tile (leaves room for the small scratch words)

Tiling choose_tiling(const ht_grid& g)
{
  Tiling t;
  const int64_t row_bytes = (int64_t)g.n_b * 4;
  const int64_t budget = env_int("HT_FILL_LDS_BYTES", 32768);
  const int64_t lds_max = kLdsTileMax;
  t.lds_fill = row_bytes <= lds_max ? 1 : 0;
  int rows = 1;
  if (t.lds_fill) {
    while (rows < 64 && (int64_t)(rows * 2) * row_bytes <= std::max<int64_t>(budget, row_bytes) &&
           rows < g.n_a)
      rows *= 2;
    const int forced = env_int("HT_FILL_ROWS", 0);
    if (forced > 0 && (forced & (forced - 1)) == 0 && forced <= 64 &&
        (int64_t)forced * row_bytes <= lds_max)
      rows = forced;
  }
  // keep the tile count inside a 32-bit grid dimension
  while (rows < 64 && (int64_t)g.n_theta * g.n_phi * ((g.n_a + rows - 1) / rows) > 0x7fffffffLL) rows *= 2;
  t.rows = rows;
  t.tiles_per_slab = (g.n_a + rows - 1) / rows;
  t.n_tiles = g.n_theta * g.n_phi * t.tiles_per_slab;
  const int64_t tile_cells = (int64_t)rows * g.n_b;
  int cap = 64;
  while (cap < 1024 && cap * 32 < tile_cells) cap *= 2;
  const int forced_cap = env_int("HT_CAND_CAP", 0);
  if (forced_cap >= 2 && forced_cap <= 4096 && (forced_cap & (forced_cap - 1)) == 0) cap = forced_cap;
  t.cand_cap = cap;
  // peak-search groups: small groups spread clustered candidates over more workgroups; the
  // write kernel sums the earlier groups' totals, so keep the group count moderate
  int gt = 16;
  while (gt < 64 && ((int64_t)t.n_tiles + gt - 1) / gt > 2048) gt *= 2;
  const int forced_gt = env_int("HT_GROUP_TILES", 0);
  if (forced_gt == 16 || forced_gt == 32 || forced_gt == 64) gt = forced_gt;
  t.group_tiles = gt;
  t.nt_store = std::min(2, std::max(0, env_int("HT_FILL_NT", 0)));
  // fill tiles per workgroup: one by default (measured fastest on the paper grid: many short
  // workgroups hide the record-load latency better than fewer workgroups looping over tiles)
  int ft = 1;
  const int forced_ft = env_int("HT_FILL_TILES", 0);
  if (forced_ft > 0 && forced_ft <= 64 && (forced_ft & (forced_ft - 1)) == 0) ft = forced_ft;
  t.fill_tiles = ft;
  // HT_POOL_BOUND=0: the pool holds n_tiles * cand_cap entries only (tests force overflow so)
  t.pool_bound = env_int("HT_POOL_BOUND", 1) != 0 ? 1 : 0;
  // HT_PACKED_LISTS=1: every event takes the counting sort into packed slab lists, the layout
  // that large batches and very large events use, so that tests reach it on small grids
  t.packed_lists = env_int("HT_PACKED_LISTS", 0) != 0 ? 1 : 0;
  ht_tuning tu;
  std::memset(&tu, 0, sizeof(tu));
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(g));
    if (it != g_tune.end()) {
      tu = it->second;
      have = true;
    }
  }
  if (have) {
    if (tu.rows > 0 && t.lds_fill) t.rows = tu.rows;
    if (tu.group_tiles > 0) t.group_tiles = tu.group_tiles;
    if (tu.cand_cap > 0) t.cand_cap = tu.cand_cap;
    if (tu.nt_store >= 0) t.nt_store = tu.nt_store;
    if (tu.tiles_per_block > 0) t.fill_tiles = tu.tiles_per_block;
    t.tiles_per_slab = (g.n_a + t.rows - 1) / t.rows;
    t.n_tiles = g.n_theta * g.n_phi * t.tiles_per_slab;
  }
  // Stencil peak search of crowded events: a workgroup holds kChunkCells B columns of every
  // slab, one wave per phi cell with every theta cell in its registers (so at most 16 phi cells
  // and 4 theta cells), and walks dense_rows A rows (a multiple of 12, its unrolled step loop).
  // It needs LDS tiles for the fill (whose candidate pass it replaces). By default the segments
  // are as long as lets every workgroup run at once, two per CU (256 CUs).
  // One buffer resource spans a row of every theta cell's slab: under 2^31 bytes.
  const bool st_offsets = ((uint64_t)(g.n_theta - 1) * g.n_phi * g.n_a + 1) * g.n_b * 4 < (1ull << 31);
  t.dense_w = (t.lds_fill && g.n_theta <= 4 && g.n_phi <= 16 && st_offsets) ? 1 : 0;
  {
    const int n_chunks = (g.n_b + kChunkCells - 1) / kChunkCells;
    const int segs = std::max(1, 512 / n_chunks);
    int s_rows = (g.n_a + segs - 1) / segs;
    const int forced = env_int("HT_DENSE_ROWS", 0);
    if (forced > 0) s_rows = std::min(forced, 4096);
    t.dense_rows = std::max(12, ((s_rows + 11) / 12) * 12);
  }
  // default: events with at least n_slabs n_b / 4 hits, a quarter of a hit per (theta, phi, B)
  // cell, where the stencil's one pass over the matrix measured faster than the candidate pool
  // (on the 4x16x1024x1024 grid: 16384 hits; the pool won up to 15k hits, the stencil from 18k);
  // -1 never
  int64_t dh = ((int64_t)g.n_theta * g.n_phi * g.n_b + 3) / 4;
  const int forced_dh = env_int("HT_DENSE_HITS", 0);
  if (forced_dh != 0) dh = forced_dh;
  if (have && tu.dense_hits != 0) dh = tu.dense_hits;
  t.dense_hits = (t.dense_w > 0 && dh > 0) ? (int32_t)std::min<int64_t>(dh, 1 << 28) : 0;
  return t;
}

int check_tuning(const ht_grid& g, const ht_tuning& tu)
{
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (tu.rows < 0 || (tu.rows > 0 && (!pow2(tu.rows) || tu.rows > 64 ||
                                      (int64_t)tu.rows * g.n_b * 4 > kLdsTileMax)))
    return fail(HT_EINVAL, "tuning.rows must be a power of two <= 64 with rows*n_b*4 <= %lld",
                (long long)kLdsTileMax);
  if ((int64_t)g.n_theta * g.n_phi * ((g.n_a + std::max(tu.rows, 1) - 1) / std::max(tu.rows, 1)) >
      0x7fffffffLL)
    return fail(HT_EINVAL, "tuning.rows gives too many tiles");
  if (tu.group_tiles != 0 && tu.group_tiles != 16 && tu.group_tiles != 32 && tu.group_tiles != 64)
    return fail(HT_EINVAL, "tuning.group_tiles must be 16, 32 or 64");
  if (tu.cand_cap < 0 || (tu.cand_cap > 0 && (!pow2(tu.cand_cap) || tu.cand_cap > 4096)))
    return fail(HT_EINVAL, "tuning.cand_cap must be a power of two <= 4096");
  if (tu.nt_store < -1 || tu.nt_store > 2) return fail(HT_EINVAL, "tuning.nt_store must be -1, 0, 1 or 2");
  if (tu.tiles_per_block < 0 || (tu.tiles_per_block > 0 && (!pow2(tu.tiles_per_block) || tu.tiles_per_block > 64)))
    return fail(HT_EINVAL, "tuning.tiles_per_block must be a power of two <= 64");
  if (tu.dense_hits < -1) return fail(HT_EINVAL, "tuning.dense_hits must be -1, 0 or a hit count");
  return HT_OK;
}

// ---------------------------------------------------------------------------------------------
// Device tables, cached per (device, grid)
// ---------------------------------------------------------------------------------------------
static std::mutex g_mu;
typedef std::tuple<int, int32_t, int32_t, int32_t, int32_t, uint32_t, uint32_t, uint32_t, uint32_t>
    TabKey;
static std::map<TabKey, DevTables> g_tables;

static uint32_t fbits(float f)
{
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

int get_tables(const ht_grid& g, int dev, DevTables* out)
{
  TabKey key{dev, g.n_theta, g.n_phi, g.n_a, g.n_b, fbits(g.a_min), fbits(g.a_max), fbits(g.b_min),
             fbits(g.b_max)};
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    *out = it->second;
    return HT_OK;
  }
  std::vector<float> a2, phi, th;
  DevTables t;
  host_tables(g, a2, t.inv_db, phi, th);
  hipError_t e;
  if ((e = hipMalloc(&t.a2, a2.size() * 4)) != hipSuccess) return fail_hip(e, "hipMalloc(tables)");
  if ((e = hipMalloc(&t.phi, phi.size() * 4)) != hipSuccess) return fail_hip(e, "hipMalloc(tables)");
  if ((e = hipMalloc(&t.th, th.size() * 4)) != hipSuccess) return fail_hip(e, "hipMalloc(tables)");
  if ((e = hipMemcpy(t.a2, a2.data(), a2.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(t.phi, phi.data(), phi.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(t.th, th.data(), th.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return fail_hip(e, "hipMemcpy(tables)");
  g_tables[key] = t;
  *out = t;
  return HT_OK;
}

DevGrid make_devgrid(const ht_grid& g, const DevTables& t, const Tiling& tl)
{
  DevGrid d;
  std::memset(&d, 0, sizeof(d));  // padding too: the bytes key the graph cache
  d.n_theta = g.n_theta;
  d.n_phi = g.n_phi;
  d.n_a = g.n_a;
  d.n_b = g.n_b;
  d.b_min = g.b_min;
  d.inv_db = t.inv_db;
  d.nb_f = (float)g.n_b;
  d.threshold = g.threshold;
  d.n_slabs = g.n_theta * g.n_phi;
  d.rows = tl.rows;
  d.tiles_per_slab = tl.tiles_per_slab;
  d.n_tiles = tl.n_tiles;
  d.cand_cap = tl.cand_cap;
  d.lds_fill = tl.lds_fill;
  d.group_tiles = tl.group_tiles;
  d.nt_store = tl.nt_store;
  d.fill_tiles = tl.fill_tiles;
  d.pool_bound = tl.pool_bound;
  d.phi_sectors = g.phi_sectors;
  d.packed_lists = tl.packed_lists;
  // candidate test: enough workgroups to spread a few thousand candidates over the whole chip
  // in one pass (two candidates per wave), few enough that a near-empty event exits at once
  d.test_blocks = std::max(16, std::min(1024, (tl.n_tiles + 15) / 16));
  d.dense_w = tl.dense_w;
  d.dense_rows = tl.dense_rows;
  d.dense_hits = tl.dense_hits;
  d.a2 = t.a2;
  d.phi_cs = t.phi;
  d.th_cs = t.th;
  return d;
}

// ---------------------------------------------------------------------------------------------
// Per-event scratch
// ---------------------------------------------------------------------------------------------
static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

bool dense_peaks(const DevGrid& g, int64_t n)
{
  return g.dense_w > 0 && g.dense_hits > 0 && n >= g.dense_hits;
}

bool direct_lists(const DevGrid& g, int64_t n)
{
  return g.lds_fill && !g.packed_lists &&
         (size_t)g.n_slabs * (size_t)std::max<int64_t>(n, 1) * 16 <= kDirectListMax;
}

// Candidate-pool entries for an event of up to n hits: cand_cap per tile, and at least a
// quarter of the bound on the cells that can reach the threshold (a hit's records vote at most
// once per A row, into at most four (theta, phi) cells, two with phi sectors: votes <= 4 n n_a,
// candidates <= votes / T). Large events have far more candidates than cand_cap per tile (a
// 40k-hit event on the paper grid about 2.6M, against 0.25 of its bound of 18M); a tile whose
// candidates do not fit is searched densely, which is exact but slow.
size_t pool_entries(const DevGrid& g, int64_t n)
{
  const size_t by_tiles = (size_t)g.n_tiles * (size_t)g.cand_cap;
  const size_t cells = (size_t)g.n_theta * g.n_phi * g.n_a * g.n_b;
  const size_t bound = g.pool_bound ? (size_t)std::max<int64_t>(n, 0) * (g.phi_sectors ? 2 : 4) *
                                          (size_t)g.n_a / (size_t)g.threshold
                                    : 0;
  return std::min<size_t>(std::max(by_tiles, std::min(cells, bound / 4)), 0xfffffff0u);
}

static size_t mask_bytes(const DevGrid& g)
{
  // one 64-bit word per (slab, row, chunk of kChunkCells columns), rows padded to whole segments
  // of dense_rows (the stencil's waves store their segments whole)
  const size_t n_chunks = ((size_t)g.n_b + kChunkCells - 1) / kChunkCells;
  const size_t rows = (((size_t)g.n_a + g.dense_rows - 1) / g.dense_rows) * g.dense_rows;
  return 8 * (size_t)g.n_slabs * rows * n_chunks;
}

size_t event_scratch_bytes(const DevGrid& g, int64_t n, bool direct, int peaks)
{
  const size_t nn = (size_t)std::max<int64_t>(n, 0);
  size_t b = 0;
  b += al(4 * ((size_t)g.n_slabs + 1));       // slab_off
  if (direct) {
    b += al(16 * (size_t)g.n_slabs * std::max<size_t>(nn, 1));  // list
  } else {
    b += al(16 * nn);                         // hit_slab
    b += al(16 * nn);                         // hit_pos
    b += al(16 * nn);                         // hit_rec
    b += al(64 * nn + 16);                    // list (+1 record of slack for the fill)
  }
  b += al(4 * (size_t)g.n_tiles);             // tile_cnt
  b += al(4 * (size_t)g.n_tiles);             // tile_off
  const size_t pe = (peaks & kPeakPool) ? pool_entries(g, n) : 0;
  b += al(8 * pe);                            // pool
  b += al(pe);                                // pk_flag
  if (peaks & kPeakMask) b += al(mask_bytes(g));  // pk_mask
  b += al(4 * (size_t)g.n_tiles);               // ovf_list
  b += al(4 * (size_t)g.n_tiles);             // tile_pk
  b += al(4 * (size_t)n_groups(g));           // group_pk
  return b;
}

void carve_event_scratch(const DevGrid& g, int64_t n, bool direct, char* p, EvDesc* ev, int peaks)
{
  const size_t nn = (size_t)std::max<int64_t>(n, 0);
  auto take = [&p](size_t bytes) {
    char* r = p;
    p += al(bytes);
    return r;
  };
  ev->slab_off = (uint32_t*)take(4 * ((size_t)g.n_slabs + 1));
  if (direct) {
    ev->list_cap = (int64_t)std::max<size_t>(nn, 1);
    ev->list = (float4*)take(16 * (size_t)g.n_slabs * (size_t)ev->list_cap);
    ev->hit_slab = nullptr;
    ev->hit_pos = nullptr;
    ev->hit_rec = nullptr;
  } else {
    ev->list_cap = 0;
    ev->hit_slab = (int32_t*)take(16 * nn);
    ev->hit_pos = (uint32_t*)take(16 * nn);
    ev->hit_rec = (float4*)take(16 * nn);
    ev->list = (float4*)take(64 * nn + 16);
  }
  ev->tile_cnt = (uint32_t*)take(4 * (size_t)g.n_tiles);
  ev->tile_off = (uint32_t*)take(4 * (size_t)g.n_tiles);
  ev->pool_cap = (peaks & kPeakPool) ? (uint32_t)pool_entries(g, n) : 0u;
  ev->pool = (uint2*)take(8 * (size_t)ev->pool_cap);
  ev->pk_flag = (uint8_t*)take((size_t)ev->pool_cap);
  ev->pk_mask = (peaks & kPeakMask) ? (uint8_t*)take(mask_bytes(g)) : nullptr;
  ev->ovf_list = (uint32_t*)take(4 * (size_t)g.n_tiles);
  ev->tile_pk = (uint32_t*)take(4 * (size_t)g.n_tiles);
  ev->group_pk = (uint32_t*)take(4 * (size_t)n_groups(g));
}

// Scratch owned by the library, one per (device, stream). Calls on one stream are ordered on
// the device, so they may reuse the same scratch; growing it waits for the stream first.
struct Workspace {
  char* dev = nullptr;
  size_t bytes = 0;
  uint32_t* ctr = nullptr;  // zeroed slab counter pairs, kCounterBytes per event slot
  int ctr_events = 0;
  std::vector<uint8_t> parity;  // which array of each pair the next call counts into
  EvDesc* h_ev = nullptr;   // pinned staging of batch descriptors
  EvDesc* d_ev = nullptr;
  int ev_cap = 0;
  hipEvent_t ev_copied = nullptr;
  hipStream_t capture = nullptr;  // private stream used only to capture batch graphs
  hipStream_t side = nullptr;     // side stream of split batches (eager launches)
  hipStream_t capture_side = nullptr;  // side stream of split batches under capture
  hipEvent_t split_ev[kMaxPieces + 1] = {};
  struct Graph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
};

static std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

int get_workspace(int dev, hipStream_t s, size_t bytes, Workspace** out)
{
  Workspace* w;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace*& slot = g_ws[{dev, s}];
    if (!slot) slot = new Workspace();
    w = slot;
  }
  if (bytes > w->bytes) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    if (w->dev) (void)hipFree(w->dev);
    w->dev = nullptr;
    w->bytes = 0;
    const size_t want = std::max(bytes, (size_t)1 << 20);
    if ((e = hipMalloc(&w->dev, want)) != hipSuccess) return fail_hip(e, "hipMalloc(scratch)");
    w->bytes = want;
  }
  *out = w;
  return HT_OK;
}

int ensure_counters(Workspace* w, int n_ev, hipStream_t s)
{
  if (n_ev <= w->ctr_events) return HT_OK;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  if (w->ctr) (void)hipFree(w->ctr);
  w->ctr = nullptr;
  w->ctr_events = 0;
  const int want = std::max(n_ev, 16);
  if ((e = hipMalloc((void**)&w->ctr, kCounterBytes * want)) != hipSuccess)
    return fail_hip(e, "hipMalloc(counters)");
  if ((e = hipMemset(w->ctr, 0, kCounterBytes * want)) != hipSuccess) return fail_hip(e, "hipMemset(counters)");
  w->ctr_events = want;
  w->parity.assign(want, 0);
  return HT_OK;
}

// Counter arrays of event slot i for this call: count into the zero one, clear the other.
void use_counters(Workspace* w, int i, EvDesc* d)
{
  uint32_t* pair = w->ctr + (size_t)i * (kCounterBytes / 4);
  d->slab_cnt = pair + (w->parity[i] ? kCounterWords : 0);
  d->slab_cnt_next = pair + (w->parity[i] ? 0 : kCounterWords);
}

void flip_counters(Workspace* w, int n) { for (int i = 0; i < n; ++i) w->parity[i] ^= 1; }

int ensure_ev_staging(Workspace* w, int n_ev, hipStream_t s)
{
  if (n_ev <= w->ev_cap) {
    if (w->ev_copied) {
      hipError_t e = hipEventSynchronize(w->ev_copied);
      if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
    }
    return HT_OK;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  if (w->h_ev) (void)hipHostFree(w->h_ev);
  if (w->d_ev) (void)hipFree(w->d_ev);
  w->h_ev = nullptr;
  w->d_ev = nullptr;
  w->ev_cap = 0;
  int cap = std::max(n_ev, 16);
  if ((e = hipHostMalloc((void**)&w->h_ev, sizeof(EvDesc) * cap, hipHostMallocDefault)) != hipSuccess)
    return fail_hip(e, "hipHostMalloc(descriptors)");
  if ((e = hipMalloc((void**)&w->d_ev, sizeof(EvDesc) * cap)) != hipSuccess)
    return fail_hip(e, "hipMalloc(descriptors)");
  if (!w->ev_copied && (e = hipEventCreateWithFlags(&w->ev_copied, hipEventDisableTiming)) != hipSuccess)
    return fail_hip(e, "hipEventCreate");
  w->ev_cap = cap;
  return HT_OK;
}

int make_device_grid(const ht_grid& g, int dev, DevGrid* out)
{
  int rc = validate_grid(&g);
  if (rc) return rc;
  DevTables t;
  if ((rc = get_tables(g, dev, &t))) return rc;
  *out = make_devgrid(g, t, choose_tiling(g));
  return HT_OK;
}

// ---------------------------------------------------------------------------------------------
// Stage profiler: HIP events recorded on the launch stream around each stage.
// ---------------------------------------------------------------------------------------------
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static int g_prof_mode = 0;  // 0 off, 1 every stage, 2 the fill stages only
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_prof_pool;

static thread_local bool t_capturing = false;

static hipEvent_t prof_event()
{
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  // timing events without the system-scope fence: they order nothing for the host, and the
  // fence (a cache writeback) would add to what they measure
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

struct StageTimer {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(const char* n, hipStream_t st) : name(n), s(st)
  {
    if (!name) return;  // untimed call
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof_mode == 0 || t_capturing) return;
    if (g_prof_mode == 2 && std::strncmp(name, "fill", 4) != 0) return;
    a = prof_event();
    if (a) (void)hipEventRecord(a, s);
  }
  ~StageTimer()
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!a) return;
    hipEvent_t b = prof_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_prof.push_back({name, a, b});
  }
};

struct Prepared {
  DevGrid g;
  int dev;
  hipStream_t s;
};

int prepare(const ht_grid* grid, void* stream, Prepared* p)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  hipError_t e = hipGetDevice(&p->dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if ((rc = make_device_grid(*grid, p->dev, &p->g))) return rc;
  p->s = (hipStream_t)stream;
  return HT_OK;
}

int check_launch(hipError_t e, const char* what)
{
  if (e != hipSuccess) return fail_hip(e, what);
  return HT_OK;
}

// Failure injection for tests of the error paths: with HT_TEST_FAIL_STAGE set to a stage name
// ("prep", "fill" or "peaks"), that stage's launch is not made and the call fails as a failed
// launch would (HT_EDEVICE), with the earlier stages already on the stream.
int injected_failure(const char* stage)
{
  const char* v = std::getenv("HT_TEST_FAIL_STAGE");
  if (v && std::strcmp(v, stage) == 0)
    return fail(HT_EDEVICE, "injected failure before the %s launch (HT_TEST_FAIL_STAGE)", stage);
  return HT_OK;
}

int launch_batch(const DevGrid& g, const EvDesc* d_ev, int n_ev, int64_t max_hits, bool direct,
                 bool any_pool, bool any_dense, hipStream_t s, bool* prep_enqueued, const BatchSplit* split)
{
  EvDesc none;
  std::memset(&none, 0, sizeof(none));
  int rc;
  *prep_enqueued = false;
  {
    StageTimer t("prep", s);
    if ((rc = injected_failure("prep")) ||
        (rc = check_launch(launch_prep(g, none, d_ev, n_ev, max_hits, direct && g.lds_fill, s), "prep launch")))
      return rc;
    *prep_enqueued = true;
  }
  if ((rc = injected_failure("fill"))) return rc;
  const int pieces = split && g.lds_fill ? std::min(split->pieces, n_ev) : 1;
  if (pieces > 1) {
    // The batch in `pieces` runs of consecutive events: the fill of run i + 1 (on s) overlaps
    // the peak search of run i (on the side stream, after an event recorded when run i's fill
    // is done): the fill is bound by HBM writes, the candidate test by memory latency. s waits
    // for the side stream at the end, so the call's completion on s covers everything.
    hipError_t e;
    for (int i = 0; i < pieces; ++i) {
      const int e0 = (int)((int64_t)n_ev * i / pieces), e1 = (int)((int64_t)n_ev * (i + 1) / pieces);
      if ((rc = check_launch(launch_fill(g, none, d_ev + e0, e1 - e0, true, max_hits, s), "fill launch")))
        return rc;
      if ((e = hipEventRecord(split->filled[i], s)) != hipSuccess) return fail_hip(e, "hipEventRecord");
      if ((e = hipStreamWaitEvent(split->side, split->filled[i], 0)) != hipSuccess)
        return fail_hip(e, "hipStreamWaitEvent");
      if (i == 0 && (rc = injected_failure("peaks"))) return rc;
      if (any_pool && (rc = check_launch(launch_peaks(g, none, d_ev + e0, e1 - e0, split->side), "peak launch")))
        return rc;
      if (any_dense &&
          (rc = check_launch(launch_peaks_dense(g, none, d_ev + e0, e1 - e0, split->side), "stencil peak launch")))
        return rc;
    }
    if ((e = hipEventRecord(split->done, split->side)) != hipSuccess) return fail_hip(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(s, split->done, 0)) != hipSuccess) return fail_hip(e, "hipStreamWaitEvent");
    return HT_OK;
  }
  if (g.lds_fill) {
    StageTimer t("fill", s);
    if ((rc = check_launch(launch_fill(g, none, d_ev, n_ev, true, max_hits, s), "fill launch"))) return rc;
  } else {
    {
      StageTimer t("fill_atomic", s);
      if ((rc = check_launch(launch_fill_atomic(g, none, d_ev, n_ev, max_hits, s), "fill launch")))
        return rc;
    }
    StageTimer t("candidates", s);
    if ((rc = check_launch(launch_candidates(g, none, d_ev, n_ev, s), "candidate launch"))) return rc;
  }
  if ((rc = injected_failure("peaks"))) return rc;
  StageTimer t("peaks", s);
  if (any_pool && (rc = check_launch(launch_peaks(g, none, d_ev, n_ev, s), "peak launch"))) return rc;
  if (any_dense && (rc = check_launch(launch_peaks_dense(g, none, d_ev, n_ev, s), "stencil peak launch")))
    return rc;
  return HT_OK;
}

// Outputs (peak list, count) may live in device memory or in pinned host memory that is
// mapped into the device's address space; anything else would fault on the device, so it is
// rejected here, on the host, before any launch.
// 0: not usable by a kernel; 1: device memory; 2: host memory mapped into the device; 3: managed.
// Only what the runtime positively reports as device-accessible is accepted: unregistered host
// memory (malloc, numpy, unpinned tensors) is reported as a successful query of type
// hipMemoryTypeUnregistered and must be refused.
int pointer_kind(const void* ptr)
{
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (attr.type == hipMemoryTypeDevice) return 1;
  if (attr.type == hipMemoryTypeHost && attr.devicePointer) return 2;
  if (attr.type == hipMemoryTypeManaged) return 3;
  return 0;
}

int check_accessible(const void* ptr, const char* what)
{
  if (!ptr) return HT_OK;
  if (pointer_kind(ptr) == 0)
    return fail(HT_EINVAL, "%s is neither device memory nor mapped pinned host memory", what);
  return HT_OK;
}

// Scratch layout of a batch: direct slab lists for every event when each event allows them and
// their scratch totals at most 8 GiB, else the counting sort for all (the 16-event batch of
// 105600-hit events on the 8x32x2048x2048 grid takes the counting sort). Returns whether the
// lists are direct; offs[i] is event i's scratch offset, *total the bytes of all of them.
bool plan_batch(const DevGrid& g, const ht_event* events, int n_events, std::vector<size_t>* offs,
                size_t* total, int64_t* max_hits)
{
  auto layout = [&g](int64_t n) { return dense_peaks(g, n) ? kPeakMask : kPeakPool; };
  bool direct = g.lds_fill != 0;
  size_t direct_bytes = 0;
  for (int i = 0; i < n_events; ++i) {
    direct = direct && direct_lists(g, events[i].n_hits);
    direct_bytes += event_scratch_bytes(g, events[i].n_hits, true, layout(events[i].n_hits));
  }
  if (direct_bytes > kBatchDirectMax) direct = false;
  offs->assign((size_t)n_events, 0);
  *total = 0;
  *max_hits = 0;
  for (int i = 0; i < n_events; ++i) {
    *max_hits = std::max(*max_hits, events[i].n_hits);
    (*offs)[i] = *total;
    *total += event_scratch_bytes(g, events[i].n_hits, direct, layout(events[i].n_hits));
  }
  return direct;
}

int enqueue_event(const DevGrid& g, const EvDesc& ev, int64_t nh, bool direct, bool atomic,
                  bool do_fill, bool do_peaks, bool timed, hipStream_t s, bool* counters_used)
{
  // stage timers only where asked for (they may create HIP events); a null name times nothing
#define HT_STAGE(var, name) StageTimer var(timed ? name : nullptr, s)
  int rc;
  *counters_used = false;
  if (do_fill) {
    {
      HT_STAGE(t, "prep");
      if ((rc = injected_failure("prep")) ||
          (rc = check_launch(launch_prep(g, ev, nullptr, 1, nh, direct, s), "prep launch")))
        return rc;
      *counters_used = true;
    }
    if ((rc = injected_failure("fill"))) return rc;
    if (atomic) {
      HT_STAGE(t, "fill_atomic");
      if ((rc = check_launch(launch_fill_atomic(g, ev, nullptr, 1, nh, s), "fill launch"))) return rc;
    } else {
      HT_STAGE(t, "fill");
      if ((rc = check_launch(launch_fill(g, ev, nullptr, 1, do_peaks, nh, s), "fill launch"))) return rc;
    }
  }
  if (do_peaks) {
    if (!do_fill || atomic) {
      HT_STAGE(t, "candidates");
      if ((rc = check_launch(launch_candidates(g, ev, nullptr, 1, s), "candidate launch"))) return rc;
      *counters_used = true;
    }
    if ((rc = injected_failure("peaks"))) return rc;
    HT_STAGE(t, "peaks");
    if (ev.dense) {
      if ((rc = check_launch(launch_peaks_dense(g, ev, nullptr, 1, s), "stencil peak launch"))) return rc;
    } else if ((rc = check_launch(launch_peaks(g, ev, nullptr, 1, s), "peak launch"))) {
      return rc;
    }
  }
#undef HT_STAGE
  return HT_OK;
}

int run_event(const ht_grid* grid, const float* x, const float* y, const float* z, int64_t n,
              uint32_t* acc, ht_peak* out, int64_t cap, int64_t* n_found, void* stream,
              bool do_fill, bool do_peaks, bool force_atomic)
{
  if (n < 0) return fail(HT_EINVAL, "n_hits < 0");
  if (!acc) return fail(HT_EINVAL, "acc is NULL");
  if (do_fill && n > 0 && (!x || !y || !z)) return fail(HT_EINVAL, "hit arrays are NULL");
  if (do_peaks && (cap < 0 || !n_found || (cap > 0 && !out)))
    return fail(HT_EINVAL, "peak output arguments are invalid");
  if (n > ((int64_t)1 << 28)) return fail(HT_EINVAL, "n_hits must be <= 2^28");
  Prepared p;
  int rc = prepare(grid, stream, &p);
  if (rc) return rc;
  if (do_peaks && ((rc = check_accessible(out, "out")) || (rc = check_accessible(n_found, "n_found"))))
    return rc;
  const int64_t nh = do_fill ? n : 0;
  const bool atomic = force_atomic || !p.g.lds_fill;
  const bool direct = !atomic && direct_lists(p.g, nh);
  // crowded events of the fused call: peaks from the stencil over the written matrix
  const bool dense = do_fill && do_peaks && !atomic && dense_peaks(p.g, nh);
  const int layout = dense ? kPeakMask : kPeakPool;
  Workspace* w;
  if ((rc = get_workspace(p.dev, p.s, event_scratch_bytes(p.g, nh, direct, layout), &w))) return rc;
  if ((rc = ensure_counters(w, 1, p.s))) return rc;
  EvDesc ev;
  std::memset(&ev, 0, sizeof(ev));
  carve_event_scratch(p.g, nh, direct, w->dev, &ev, layout);
  ev.dense = dense ? 1 : 0;
  use_counters(w, 0, &ev);
  ev.x = x;
  ev.y = y;
  ev.z = z;
  ev.n_hits = nh;
  ev.acc = acc;
  ev.out = out;
  ev.cap = cap;
  ev.n_found = n_found;
  bool used = false;
  rc = enqueue_event(p.g, ev, nh, direct, atomic, do_fill, do_peaks, true, p.s, &used);
  // the next call counts into the other array only if a kernel of this call counts into this
  // one and clears that one (a launch that failed before it leaves both as they were)
  if (used) flip_counters(w, 1);
  return rc;
}

}  // namespace ht

using namespace ht;

extern "C" {

int ht_tables(const ht_grid* grid, float* a2, float* inv_db, float* phi_cs, float* th_cs)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!a2 || !inv_db || !phi_cs || !th_cs) return fail(HT_EINVAL, "table pointers are NULL");
  host_tables_into(*grid, a2, inv_db, phi_cs, th_cs);
  return HT_OK;
}

int ht_tiling(const ht_grid* grid, int32_t* rows, int32_t* n_tiles, int32_t* cand_cap,
              int32_t* lds_fill)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  Tiling t = choose_tiling(*grid);
  if (rows) *rows = t.rows;
  if (n_tiles) *n_tiles = t.n_tiles;
  if (cand_cap) *cand_cap = t.cand_cap;
  if (lds_fill) *lds_fill = t.lds_fill;
  return HT_OK;
}

int ht_fill(const ht_grid* grid, const float* x, const float* y, const float* z, int64_t n_hits,
            uint32_t* acc, void* stream)
{
  return run_event(grid, x, y, z, n_hits, acc, nullptr, 0, nullptr, stream, true, false, false);
}

int ht_fill_atomic(const ht_grid* grid, const float* x, const float* y, const float* z,
                   int64_t n_hits, uint32_t* acc, void* stream)
{
  return run_event(grid, x, y, z, n_hits, acc, nullptr, 0, nullptr, stream, true, false, true);
}

int ht_peaks(const ht_grid* grid, const uint32_t* acc, ht_peak* out, int64_t capacity,
             int64_t* n_found, void* stream)
{
  return run_event(grid, nullptr, nullptr, nullptr, 0, const_cast<uint32_t*>(acc), out, capacity,
                   n_found, stream, false, true, false);
}

int ht_fill_peaks(const ht_grid* grid, const float* x, const float* y, const float* z,
                  int64_t n_hits, uint32_t* acc, ht_peak* out, int64_t capacity,
                  int64_t* n_found, void* stream)
{
  return run_event(grid, x, y, z, n_hits, acc, out, capacity, n_found, stream, true, true, false);
}

int ht_fill_peaks_batch(const ht_grid* grid, const ht_event* events, int32_t n_events,
                        const float* x, const float* y, const float* z, uint32_t* acc,
                        ht_peak* out, int64_t* n_found, void* stream)
{
  if (n_events < 0 || n_events > 65535) return fail(HT_EINVAL, "n_events must be in [0, 65535]");
  if (n_events == 0) return HT_OK;
  if (!events || !acc || !n_found) return fail(HT_EINVAL, "NULL batch argument");
  int64_t max_hits = 0;
  int rc = validate_grid(grid);
  if (rc) return rc;
  for (int32_t i = 0; i < n_events; ++i) {
    const ht_event& ev = events[i];
    if (ev.n_hits < 0 || ev.n_hits > ((int64_t)1 << 28) || ev.hit_offset < 0 || ev.peak_capacity < 0 ||
        ev.peak_offset < 0)
      return fail(HT_EINVAL, "event %d has invalid offsets or sizes", i);
    if (ev.n_hits > 0 && (!x || !y || !z)) return fail(HT_EINVAL, "hit arrays are NULL");
    if (ev.peak_capacity > 0 && !out) return fail(HT_EINVAL, "out is NULL");
  }
  Prepared p;
  if ((rc = prepare(grid, stream, &p))) return rc;
  if ((rc = check_accessible(out, "out")) || (rc = check_accessible(n_found, "n_found"))) return rc;
  std::vector<size_t> offs;
  size_t total_scratch = 0;
  const bool direct = plan_batch(p.g, events, n_events, &offs, &total_scratch, &max_hits);
  Workspace* w;
  if ((rc = get_workspace(p.dev, p.s, total_scratch, &w))) return rc;
  if ((rc = ensure_ev_staging(w, n_events, p.s))) return rc;
  if ((rc = ensure_counters(w, n_events, p.s))) return rc;
  const uint64_t cells = n_cells(*grid);
  bool any_pool = false, any_dense = false;
  for (int32_t i = 0; i < n_events; ++i) {
    const ht_event& ev = events[i];
    EvDesc& d = w->h_ev[i];
    std::memset(&d, 0, sizeof(d));
    const bool dense = p.g.lds_fill && dense_peaks(p.g, ev.n_hits);
    any_pool = any_pool || !dense;
    any_dense = any_dense || dense;
    carve_event_scratch(p.g, ev.n_hits, direct, w->dev + offs[i], &d, dense ? kPeakMask : kPeakPool);
    d.dense = dense ? 1 : 0;
    use_counters(w, i, &d);
    d.x = x ? x + ev.hit_offset : nullptr;
    d.y = y ? y + ev.hit_offset : nullptr;
    d.z = z ? z + ev.hit_offset : nullptr;
    d.n_hits = ev.n_hits;
    d.acc = acc + (size_t)i * cells;
    d.out = out ? out + ev.peak_offset : nullptr;
    d.cap = ev.peak_capacity;
    d.n_found = n_found + i;
  }
  // prep grids are sized for a power-of-two bucket of workgroups, so batches of one size share
  // a graph (workgroups past an event's hits return at once)
  int64_t blocks = 1;
  while (blocks * 256 < max_hits) blocks *= 2;
  const int64_t max_hits_b = max_hits > 0 ? blocks * 256 : 0;
  hipError_t e;
  // overlap of the peak searches with the fills of later events: the batch in `pieces` runs
  const int pieces = std::max(1, std::min(std::min(env_int("HT_BATCH_PIECES", 1), kMaxPieces), (int)n_events));
  BatchSplit split;
  std::memset(&split, 0, sizeof(split));
  split.pieces = pieces;
  const bool graph_mode = env_int("HT_BATCH_GRAPH", 1) != 0;
  if (pieces > 1) {
    hipStream_t& side = graph_mode ? w->capture_side : w->side;
    if (!side && (e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking)) != hipSuccess)
      return fail_hip(e, "hipStreamCreate(side)");
    for (int i = 0; i <= kMaxPieces; ++i)
      if (!w->split_ev[i] && (e = hipEventCreateWithFlags(&w->split_ev[i], hipEventDisableTiming)) != hipSuccess)
        return fail_hip(e, "hipEventCreate(split)");
    split.side = side;
    for (int i = 0; i < kMaxPieces; ++i) split.filled[i] = w->split_ev[i];
    split.done = w->split_ev[kMaxPieces];
  }
  // The descriptors above hold this call's counter arrays. The next call switches to the other
  // arrays only once this call's preparation (which counts into these and clears those) is on
  // the stream; a call that fails before that leaves the counters as they were.
  if (!graph_mode) {
    e = hipMemcpyAsync(w->d_ev, w->h_ev, sizeof(EvDesc) * n_events, hipMemcpyHostToDevice, p.s);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync(descriptors)");
    if ((e = hipEventRecord(w->ev_copied, p.s)) != hipSuccess) return fail_hip(e, "hipEventRecord");
    bool prep_enqueued = false;
    rc = launch_batch(p.g, w->d_ev, n_events, max_hits_b, direct, any_pool, any_dense, p.s, &prep_enqueued,
                      pieces > 1 ? &split : nullptr);
    if (prep_enqueued) flip_counters(w, n_events);
    return rc;
  }
  // graph key: everything the captured launches depend on besides the descriptor contents
  std::vector<unsigned char> key(sizeof(DevGrid) + 4 * sizeof(int64_t) + 2 * sizeof(void*));
  {
    unsigned char* q = key.data();
    std::memcpy(q, &p.g, sizeof(DevGrid));
    q += sizeof(DevGrid);
    const int64_t ints[4] = {n_events, max_hits_b, p.dev,
                             (direct ? 1 : 0) | (any_pool ? 2 : 0) | (any_dense ? 4 : 0) | (pieces << 3)};
    std::memcpy(q, ints, sizeof(ints));
    q += sizeof(ints);
    const void* ptrs[2] = {w->d_ev, w->h_ev};
    std::memcpy(q, ptrs, sizeof(ptrs));
  }
  hipGraphExec_t exec = nullptr;
  for (auto& gr : w->graphs)
    if (gr.key == key) exec = gr.exec;
  if (!exec) {
    if (!w->capture && (e = hipStreamCreateWithFlags(&w->capture, hipStreamNonBlocking)) != hipSuccess)
      return fail_hip(e, "hipStreamCreate(capture)");
    // the capture stream must not start before earlier work on the caller's stream is done
    // with the descriptor staging; capturing records work without running it
    if ((e = hipStreamBeginCapture(w->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return fail_hip(e, "hipStreamBeginCapture");
    t_capturing = true;
    e = hipMemcpyAsync(w->d_ev, w->h_ev, sizeof(EvDesc) * n_events, hipMemcpyHostToDevice, w->capture);
    bool captured_prep = false;
    int lrc = e == hipSuccess
                  ? launch_batch(p.g, w->d_ev, n_events, max_hits_b, direct, any_pool, any_dense, w->capture,
                                 &captured_prep, pieces > 1 ? &split : nullptr)
                  : HT_EDEVICE;
    t_capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(w->capture, &graph);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync(descriptors, capture)");
    if (lrc != HT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return lrc;
    }
    if (e2 != hipSuccess) return fail_hip(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
    if (w->graphs.size() >= 16) {
      (void)hipGraphExecDestroy(w->graphs.front().exec);
      w->graphs.erase(w->graphs.begin());
    }
    w->graphs.push_back({key, exec});
  }
  {
    StageTimer t("batch", p.s);
    if ((e = hipGraphLaunch(exec, p.s)) != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  }
  flip_counters(w, n_events);
  if ((e = hipEventRecord(w->ev_copied, p.s)) != hipSuccess) return fail_hip(e, "hipEventRecord");
  return HT_OK;
}

int ht_set_tuning(const ht_grid* grid, const ht_tuning* tuning)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!tuning) {
    g_tune.erase(tune_key(*grid));
    return HT_OK;
  }
  if ((rc = check_tuning(*grid, *tuning))) return rc;
  g_tune[tune_key(*grid)] = *tuning;
  return HT_OK;
}

int ht_get_tuning(const ht_grid* grid, ht_tuning* tuning)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!tuning) return fail(HT_EINVAL, "tuning is NULL");
  Tiling t = choose_tiling(*grid);
  tuning->rows = t.rows;
  tuning->group_tiles = t.group_tiles;
  tuning->cand_cap = t.cand_cap;
  tuning->nt_store = t.nt_store;
  tuning->tiles_per_block = t.fill_tiles;
  tuning->dense_hits = t.dense_w > 0 && t.dense_hits > 0 ? t.dense_hits : -1;
  return HT_OK;
}

int ht_readout(const ht_grid* grid, const ht_peak* peaks, const int64_t* n_found, int64_t capacity,
               ht_track* tracks, void* stream)
{
  if (capacity < 0 || capacity > ((int64_t)1 << 31)) return fail(HT_EINVAL, "capacity out of range");
  if (!n_found || (capacity > 0 && (!peaks || !tracks))) return fail(HT_EINVAL, "NULL readout argument");
  Prepared p;
  int rc = prepare(grid, stream, &p);
  if (rc) return rc;
  if ((rc = check_accessible(peaks, "peaks")) || (rc = check_accessible(n_found, "n_found")) ||
      (rc = check_accessible(tracks, "tracks")))
    return rc;
  const double db = ((double)grid->b_max - (double)grid->b_min) / (double)grid->n_b;
  return check_launch(launch_readout(p.g, peaks, n_found, capacity, tracks, (double)grid->b_min, db, p.s),
                      "readout launch");
}

int ht_debug_pointer_kind(const void* ptr, int32_t* kind)
{
  if (!ptr || !kind) return fail(HT_EINVAL, "NULL argument");
  *kind = pointer_kind(ptr);
  return HT_OK;
}

int ht_debug_hit_values(const ht_grid* grid, const float* x, const float* y, const float* z,
                        int64_t n_hits, int32_t* info, float* vals, int32_t* slabs, void* stream)
{
  if (n_hits < 0) return fail(HT_EINVAL, "n_hits < 0");
  if (n_hits > 0 && (!x || !y || !z || !info || !vals || !slabs)) return fail(HT_EINVAL, "NULL pointer");
  Prepared p;
  int rc = prepare(grid, stream, &p);
  if (rc) return rc;
  return check_launch(launch_debug_hits(p.g, x, y, z, n_hits, info, vals, slabs, p.s), "debug launch");
}

int ht_debug_unary(const float* v, float* root, float* inv2, int64_t n, void* stream)
{
  if (n < 0) return fail(HT_EINVAL, "n < 0");
  if (n == 0) return HT_OK;
  if (!v || !root || !inv2) return fail(HT_EINVAL, "NULL pointer");
  if (pointer_kind(v) == 0 || pointer_kind(root) == 0 || pointer_kind(inv2) == 0)
    return fail(HT_EINVAL, "an array is not device-accessible memory");
  return check_launch(launch_debug_unary(v, root, inv2, n, (hipStream_t)stream), "debug launch");
}

int ht_debug_batch_plan(const ht_grid* grid, const ht_event* events, int32_t n_events,
                        int32_t* direct, int64_t* scratch_bytes)
{
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!events || !direct || !scratch_bytes || n_events < 1 || n_events > 65535)
    return fail(HT_EINVAL, "invalid batch-plan arguments");
  for (int32_t i = 0; i < n_events; ++i)
    if (events[i].n_hits < 0 || events[i].n_hits > ((int64_t)1 << 28))
      return fail(HT_EINVAL, "event %d has an invalid size", i);
  // the tiling alone decides the layout; the tables (device memory) are not needed
  const DevGrid g = make_devgrid(*grid, DevTables(), choose_tiling(*grid));
  std::vector<size_t> offs;
  size_t total = 0;
  int64_t max_hits = 0;
  *direct = plan_batch(g, events, n_events, &offs, &total, &max_hits) ? 1 : 0;
  *scratch_bytes = (int64_t)total;
  return HT_OK;
}

int ht_profile_enable(int mode)
{
  if (mode < 0 || mode > 2) return fail(HT_EINVAL, "profile mode must be 0, 1 or 2");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mode = mode;
  return HT_OK;
}

int ht_profile_read(const char* name, double* total_ms, int64_t* count, int reset)
{
  if (!name || !total_ms || !count) return fail(HT_EINVAL, "NULL profile argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (const ProfRec& r : g_prof) {
    if (std::strcmp(r.name, name) != 0) continue;
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize(profile)");
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, r.a, r.b)) != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  if (reset) {
    for (const ProfRec& r : g_prof) {
      (void)hipEventSynchronize(r.b);
      g_prof_pool.push_back(r.a);
      g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
  }
  return HT_OK;
}

const char* ht_last_error(void) { return g_err.c_str(); }

}  // extern "C"
