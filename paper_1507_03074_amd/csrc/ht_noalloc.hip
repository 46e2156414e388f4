// ht_noalloc.hip -- ht_fill_peaks_noalloc: the fused fill and peak search of one event with all
// of the library's device scratch in one fixed array of this file, so the call allocates no
// device memory.
//
// The array `scratch` (kNoAllocBytes, 256-byte aligned, zero when the code object is loaded)
// holds, on each device the library runs on:
//   [0, kCounterBytes)            the pair of slab-counter arrays (one counts, one is cleared)
//   [kTabOff, kTabOff + kTabBytes) the bin-rule tables of the grid last used on the device
//   [kEvOff, kNoAllocBytes)       the event scratch (slab lists, candidate pool, peak counts)
// Host code never passes the array's name to a kernel or a copy: its host-side symbol is only
// a stand-in. The device address of each device's copy is looked up once, with that device
// current, and kept in g_ptr[device].
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "ht_internal.h"

// 64 MiB: the largest event scratch of the call (see kNoAllocBytes below)
static __device__ __align__(256) unsigned char scratch[(size_t)64 << 20];

namespace ht {
namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;
// tables: a2 up to kNoAllocMaxA floats, phi up to 4 * 4096, theta up to 2 * (2 * 4096 + 1)
constexpr size_t kNoAllocMaxA = 16384;
constexpr size_t kTabOff = (kCounterBytes + 255) & ~(size_t)255;
constexpr size_t kTabBytes = (size_t)256 << 10;
constexpr size_t kEvOff = kTabOff + kTabBytes;
static_assert(4 * (kNoAllocMaxA + 4 * kMaxSlabs + 2 * (2 * kMaxSlabs + 1)) + 3 * 256 <= kTabBytes,
              "the largest tables fit their region");

static_assert(sizeof(scratch) == kNoAllocBytes, "the array is kNoAllocBytes long");

std::mutex g_na_mu;
char* g_ptr[kNoAllocMaxDevices];          // device address of each device's scratch, or null
uint8_t g_parity[kNoAllocMaxDevices];     // which counter array the next call counts into
bool g_tab_valid[kNoAllocMaxDevices];     // the table region holds the tables of g_tab_grid
ht_grid g_tab_grid[kNoAllocMaxDevices];
// host staging of the tables (a fixed array, so no host allocation either)
float g_tab_host[kTabBytes / 4];

bool same_tables(const ht_grid& a, const ht_grid& b)
{
  return a.n_theta == b.n_theta && a.n_phi == b.n_phi && a.n_a == b.n_a && a.n_b == b.n_b &&
         std::memcmp(&a.a_min, &b.a_min, 4) == 0 && std::memcmp(&a.a_max, &b.a_max, 4) == 0 &&
         std::memcmp(&a.b_min, &b.b_min, 4) == 0 && std::memcmp(&a.b_max, &b.b_max, 4) == 0;
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace
}  // namespace ht

using namespace ht;

extern "C" int ht_fill_peaks_noalloc(const ht_grid* grid, const float* x, const float* y,
                                     const float* z, int64_t n_hits, uint32_t* acc, ht_peak* out,
                                     int64_t capacity, int64_t* n_found, void* stream)
{
  if (n_hits < 0) return fail(HT_EINVAL, "n_hits < 0");
  if (!acc) return fail(HT_EINVAL, "acc is NULL");
  if (n_hits > 0 && (!x || !y || !z)) return fail(HT_EINVAL, "hit arrays are NULL");
  if (capacity < 0 || !n_found || (capacity > 0 && !out))
    return fail(HT_EINVAL, "peak output arguments are invalid");
  if (n_hits > ((int64_t)1 << 28)) return fail(HT_EINVAL, "n_hits must be <= 2^28");
  int rc = validate_grid(grid);
  if (rc) return rc;
  if ((size_t)grid->n_a > kNoAllocMaxA)
    return fail(HT_EINVAL, "ht_fill_peaks_noalloc: n_a = %d exceeds its table limit of %zu A bins",
                grid->n_a, kNoAllocMaxA);
  if ((rc = check_accessible(out, "out")) || (rc = check_accessible(n_found, "n_found"))) return rc;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(HT_EINVAL, "ht_fill_peaks_noalloc supports device ordinals below %d", kNoAllocMaxDevices);
  hipStream_t s = (hipStream_t)stream;

  // the layout: direct slab lists when they fit, else the counting sort (the same results);
  // an event that fits neither is refused before any device work
  const Tiling tl = choose_tiling(*grid);
  DevGrid g = make_devgrid(*grid, DevTables(), tl);
  const bool atomic = !g.lds_fill;
  const bool dense = !atomic && dense_peaks(g, n_hits);
  const int layout = dense ? kPeakMask : kPeakPool;
  const size_t room = kNoAllocBytes - kEvOff;
  bool direct = !atomic && direct_lists(g, n_hits) && event_scratch_bytes(g, n_hits, true, layout) <= room;
  const size_t need = event_scratch_bytes(g, n_hits, direct, layout);
  if (need > room)
    return fail(HT_EINVAL,
                "ht_fill_peaks_noalloc: this event needs %zu bytes of scratch; the fixed scratch "
                "holds %zu (use ht_fill_peaks)", need, room);

  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_ptr[dev]) {
    // once per device, with the device current: the address of this device's copy
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
      return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(HT_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[dev] = (char*)ptr;
  }
  char* base = g_ptr[dev];
  // bin-rule tables: uploaded when the grid differs from the one whose tables the region holds
  // (a synchronous copy on the caller's stream)
  const size_t a2_off = 0;
  const size_t phi_off = al256(4 * a2_floats(*grid));
  const size_t th_off = phi_off + al256(4 * phi_floats(*grid));
  const size_t tab_bytes = th_off + 4 * th_floats(*grid);
  float inv_db = 0.0f;
  host_tables_into(*grid, g_tab_host + a2_off / 4, &inv_db, g_tab_host + phi_off / 4,
                   g_tab_host + th_off / 4);
  if (!g_tab_valid[dev] || !same_tables(g_tab_grid[dev], *grid)) {
    g_tab_valid[dev] = false;
    if ((e = hipMemcpyAsync(base + kTabOff, g_tab_host, tab_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail_hip(e, "hipMemcpyAsync(tables)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(e, "hipStreamSynchronize(tables)");
    g_tab_grid[dev] = *grid;
    g_tab_valid[dev] = true;
  }
  DevTables t;
  t.a2 = (float*)(base + kTabOff + a2_off);
  t.phi = (float*)(base + kTabOff + phi_off);
  t.th = (float*)(base + kTabOff + th_off);
  t.inv_db = inv_db;
  g = make_devgrid(*grid, t, tl);

  EvDesc ev;
  std::memset(&ev, 0, sizeof(ev));
  carve_event_scratch(g, n_hits, direct, base + kEvOff, &ev, layout);
  ev.dense = dense ? 1 : 0;
  uint32_t* pair = (uint32_t*)base;
  ev.slab_cnt = pair + (g_parity[dev] ? kCounterWords : 0);
  ev.slab_cnt_next = pair + (g_parity[dev] ? 0 : kCounterWords);
  ev.x = x;
  ev.y = y;
  ev.z = z;
  ev.n_hits = n_hits;
  ev.acc = acc;
  ev.out = out;
  ev.cap = capacity;
  ev.n_found = n_found;
  bool used = false;
  rc = enqueue_event(g, ev, n_hits, direct, atomic, true, true, false, s, &used);
  if (used) g_parity[dev] ^= 1;
  return rc;
}
