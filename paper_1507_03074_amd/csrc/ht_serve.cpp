// ht_serve.cpp -- request loop for events that arrive one by one (continuous batching).
//
// Submitted events wait in a FIFO with their hits in pinned host staging. A background thread
// admits them while device slots are free -- a slot is the device memory one event needs (its
// vote matrix, scratch, hits and peak list), and the number of slots is what the HBM budget
// holds -- groups whatever is admitted (up to max_batch) into one batched launch, and puts
// successive batches on different streams so that they overlap on the GPU. When a batch's
// completion event fires, its peak lists (written by the peak kernel straight into mapped,
// coherent pinned host memory) are handed to the requests and the slots go back to the pool,
// so later arrivals are admitted while earlier batches are still running.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ht_internal.h"

namespace ht {
namespace {

double now_s()
{
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  int stage = -1;  // pinned staging buffer holding x[n], y[n], z[n] back to back
  int slot = -1;
  ht_timing t{};
  bool done = false;
  int status = HT_OK;
  int64_t n_found = 0;
  std::vector<ht_peak> peaks;
};

struct Slot {
  uint32_t* ctr;      // slab counter pair (see kCounterBytes)
  int parity;         // which array of the pair the next batch counts into
  uint32_t* acc;
  char* scratch;
  float* hits;
  ht_peak* h_out;     // pinned host peak list, written by the kernels through d_out
  int64_t* h_nfound;  // pinned host count, written through d_nfound
  ht_peak* d_out;     // device addresses of h_out / h_nfound
  int64_t* d_nfound;
};

struct Batch {
  int stream;
  std::vector<Request*> reqs;
};

}  // namespace
}  // namespace ht

using namespace ht;

struct ht_server {
  ht_grid grid;
  ht_serve_opts opts;
  DevGrid g;
  int dev = 0;
  uint64_t cells = 0;
  size_t scratch_bytes = 0;
  bool direct = false;
  int layout = kPeakPool;       // slots hold a candidate pool, and a peak mask when events can be crowded
  char* arena = nullptr;        // device: all slots
  uint32_t* ctr = nullptr;      // device: slab counters of all slots
  char* host_out = nullptr;     // pinned: per-slot peak lists and counts
  float* stage_pool = nullptr;  // pinned: per-request hit staging
  std::vector<Slot> slots;
  std::vector<int> free_slots;
  std::vector<int> free_stage;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done_ev;
  std::vector<EvDesc*> h_ev, d_ev;
  std::vector<int> stream_busy;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::map<uint64_t, Request*> reqs;
  std::vector<Batch> inflight;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
};

namespace {

void complete_batch(ht_server* sv, Batch& b, int status)
{
  const double t = now_s();
  for (Request* r : b.reqs) {
    Slot& s = sv->slots[r->slot];
    if (status == HT_OK) {
      r->n_found = *s.h_nfound;
      const int64_t k = std::min<int64_t>(r->n_found, sv->opts.peak_capacity);
      r->peaks.assign(s.h_out, s.h_out + std::max<int64_t>(k, 0));
    }
    r->status = status;
    r->t.t_done = t;
    r->done = true;
    sv->free_slots.push_back(r->slot);
    sv->free_stage.push_back(r->stage);
    r->slot = -1;
    r->stage = -1;
  }
  sv->stream_busy[b.stream] = 0;
}

// Enqueue the copies and kernels of one batch on its stream (called without the lock).
int launch(ht_server* sv, Batch& b)
{
  hipStream_t s = sv->streams[b.stream];
  const int64_t mh = sv->opts.max_hits;
  int64_t max_n = 0;
  bool any_pool = false, any_dense = false;
  hipError_t e;
  for (size_t i = 0; i < b.reqs.size(); ++i) {
    Request* r = b.reqs[i];
    Slot& sl = sv->slots[r->slot];
    const float* stage = sv->stage_pool + (size_t)r->stage * 3 * mh;
    if (r->n > 0 &&
        (e = hipMemcpyAsync(sl.hits, stage, 12 * (size_t)r->n, hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail_hip(e, "hipMemcpyAsync(hits)");
    EvDesc& d = sv->h_ev[b.stream][i];
    std::memset(&d, 0, sizeof(d));
    carve_event_scratch(sv->g, mh, sv->direct, sl.scratch, &d, sv->layout);
    // crowded events search their peaks with the stencil (the slot holds both layouts)
    d.dense = (sv->layout & kPeakMask) && dense_peaks(sv->g, r->n) ? 1 : 0;
    any_pool = any_pool || !d.dense;
    any_dense = any_dense || d.dense;
    d.slab_cnt = sl.ctr + (sl.parity ? kCounterWords : 0);
    d.slab_cnt_next = sl.ctr + (sl.parity ? 0 : kCounterWords);
    d.x = sl.hits;
    d.y = sl.hits + r->n;
    d.z = sl.hits + 2 * r->n;
    d.n_hits = r->n;
    d.acc = sl.acc;
    d.out = sl.d_out;  // mapped pinned host memory: the kernels write the peaks to the host
    d.cap = sv->opts.peak_capacity;
    d.n_found = sl.d_nfound;
    max_n = std::max(max_n, r->n);
  }
  if ((e = hipMemcpyAsync(sv->d_ev[b.stream], sv->h_ev[b.stream], sizeof(EvDesc) * b.reqs.size(),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_hip(e, "hipMemcpyAsync(descriptors)");
  bool prep_enqueued = false;
  int rc = launch_batch(sv->g, sv->d_ev[b.stream], (int)b.reqs.size(), max_n, sv->direct, any_pool,
                        any_dense, s, &prep_enqueued);
  // a slot switches counter arrays only once the preparation that counts into this one and
  // clears the other is on the stream
  if (prep_enqueued)
    for (Request* r : b.reqs) sv->slots[r->slot].parity ^= 1;
  if (rc) return rc;
  if ((e = hipEventRecord(sv->done_ev[b.stream], s)) != hipSuccess) return fail_hip(e, "hipEventRecord");
  return HT_OK;
}

void loop(ht_server* sv)
{
  (void)hipSetDevice(sv->dev);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // completions
    for (size_t i = 0; i < sv->inflight.size();) {
      hipError_t q = hipEventQuery(sv->done_ev[sv->inflight[i].stream]);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      complete_batch(sv, sv->inflight[i], q == hipSuccess ? HT_OK : HT_EDEVICE);
      sv->inflight.erase(sv->inflight.begin() + i);
      sv->cv.notify_all();
    }
    // admission and launch: one batch per free stream
    while (!sv->stop && !sv->pending.empty() && !sv->free_slots.empty()) {
      int st = -1;
      for (size_t k = 0; k < sv->stream_busy.size(); ++k)
        if (!sv->stream_busy[k]) {
          st = (int)k;
          break;
        }
      if (st < 0) break;
      Batch b;
      b.stream = st;
      const double t = now_s();
      while (!sv->pending.empty() && !sv->free_slots.empty() &&
             (int)b.reqs.size() < sv->opts.max_batch) {
        Request* r = sv->pending.front();
        sv->pending.pop_front();
        r->slot = sv->free_slots.back();
        sv->free_slots.pop_back();
        r->t.t_admit = t;
        b.reqs.push_back(r);
      }
      sv->stream_busy[st] = 1;
      lk.unlock();
      const double tl = now_s();
      for (Request* r : b.reqs) r->t.t_launch = tl;
      int rc = launch(sv, b);
      // a launch that failed part way may have left copies into the batch's slots in flight:
      // let them finish before the slots go back to the pool
      if (rc != HT_OK) (void)hipStreamSynchronize(sv->streams[st]);
      lk.lock();
      if (rc != HT_OK) {
        complete_batch(sv, b, rc);
        sv->cv.notify_all();
      } else {
        sv->inflight.push_back(std::move(b));
      }
    }
    if (sv->stop && sv->inflight.empty()) break;
    if (sv->inflight.empty())
      sv->cv.wait(lk, [sv] { return sv->stop || (!sv->pending.empty() && !sv->free_slots.empty()); });
    else
      sv->cv.wait_for(lk, std::chrono::microseconds(20));
  }
}

void free_server(ht_server* sv)
{
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : sv->done_ev) (void)hipEventDestroy(e);
  for (EvDesc* p : sv->h_ev) (void)hipHostFree(p);
  for (EvDesc* p : sv->d_ev) (void)hipFree(p);
  if (sv->arena) (void)hipFree(sv->arena);
  if (sv->ctr) (void)hipFree(sv->ctr);
  if (sv->host_out) (void)hipHostFree(sv->host_out);
  if (sv->stage_pool) (void)hipHostFree(sv->stage_pool);
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

}  // namespace

extern "C" {

int ht_serve_create(const ht_grid* grid, const ht_serve_opts* opts, ht_server** out)
{
  if (!out) return fail(HT_EINVAL, "server output pointer is NULL");
  *out = nullptr;
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!opts || opts->hbm_budget_bytes <= 0 || opts->peak_capacity <= 0 || opts->max_hits <= 0 ||
      opts->max_hits > ((int64_t)1 << 28) || opts->max_batch < 1 || opts->max_batch > 4096 ||
      opts->n_streams < 1 || opts->n_streams > 16 || opts->queue_depth < 1)
    return fail(HT_EINVAL, "invalid server options");
  hipError_t e = hipSetDevice(opts->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  ht_server* sv = new ht_server();
  sv->grid = *grid;
  sv->opts = *opts;
  sv->dev = opts->device;
  if ((rc = make_device_grid(*grid, sv->dev, &sv->g))) {
    delete sv;
    return rc;
  }
  sv->cells = n_cells(*grid);
  sv->direct = direct_lists(sv->g, opts->max_hits);
  sv->layout = kPeakPool | (dense_peaks(sv->g, opts->max_hits) ? kPeakMask : 0);
  sv->scratch_bytes = event_scratch_bytes(sv->g, opts->max_hits, sv->direct, sv->layout);
  const size_t slot_bytes = al(4 * sv->cells) + al(sv->scratch_bytes) + al(12 * (size_t)opts->max_hits);
  const int64_t n_slots = std::min<int64_t>(opts->hbm_budget_bytes / (int64_t)slot_bytes, 4096);
  if (n_slots < 1) {
    delete sv;
    return fail(HT_EINVAL, "hbm_budget_bytes holds no event (one needs %zu bytes)", slot_bytes);
  }
  auto bail = [&](int code) {
    free_server(sv);
    return code;
  };
  if ((e = hipMalloc(&sv->arena, slot_bytes * (size_t)n_slots)) != hipSuccess)
    return bail(fail_hip(e, "hipMalloc(server slots)"));
  if ((e = hipMalloc(&sv->ctr, kCounterBytes * (size_t)n_slots)) != hipSuccess)
    return bail(fail_hip(e, "hipMalloc(server counters)"));
  if ((e = hipMemset(sv->ctr, 0, kCounterBytes * (size_t)n_slots)) != hipSuccess)
    return bail(fail_hip(e, "hipMemset(server counters)"));
  const size_t host_slot = al(sizeof(ht_peak) * (size_t)opts->peak_capacity) + al(8);
  if ((e = hipHostMalloc((void**)&sv->host_out, host_slot * (size_t)n_slots,
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return bail(fail_hip(e, "hipHostMalloc(server results)"));
  if ((e = hipHostMalloc((void**)&sv->stage_pool, 12 * (size_t)opts->max_hits * opts->queue_depth,
                         hipHostMallocDefault)) != hipSuccess)
    return bail(fail_hip(e, "hipHostMalloc(server staging)"));
  for (int64_t i = 0; i < n_slots; ++i) {
    char* p = sv->arena + (size_t)i * slot_bytes;
    Slot s;
    s.ctr = sv->ctr + (size_t)i * (kCounterBytes / 4);
    s.parity = 0;
    s.acc = (uint32_t*)p;
    p += al(4 * sv->cells);
    s.scratch = p;
    p += al(sv->scratch_bytes);
    s.hits = (float*)p;
    char* h = sv->host_out + (size_t)i * host_slot;
    s.h_out = (ht_peak*)h;
    s.h_nfound = (int64_t*)(h + al(sizeof(ht_peak) * (size_t)opts->peak_capacity));
    void* dp = nullptr;
    if ((e = hipHostGetDevicePointer(&dp, s.h_out, 0)) != hipSuccess || !dp)
      return bail(fail_hip(e, "hipHostGetDevicePointer(results)"));
    s.d_out = (ht_peak*)dp;
    if ((e = hipHostGetDevicePointer(&dp, s.h_nfound, 0)) != hipSuccess || !dp)
      return bail(fail_hip(e, "hipHostGetDevicePointer(results)"));
    s.d_nfound = (int64_t*)dp;
    sv->slots.push_back(s);
    sv->free_slots.push_back((int)(n_slots - 1 - i));
  }
  for (int i = 0; i < opts->queue_depth; ++i) sv->free_stage.push_back(opts->queue_depth - 1 - i);
  for (int i = 0; i < opts->n_streams; ++i) {
    hipStream_t s;
    hipEvent_t ev;
    EvDesc *h, *d;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
      return bail(fail_hip(e, "hipStreamCreate"));
    sv->streams.push_back(s);
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return bail(fail_hip(e, "hipEventCreate"));
    sv->done_ev.push_back(ev);
    if ((e = hipHostMalloc((void**)&h, sizeof(EvDesc) * opts->max_batch, hipHostMallocDefault)) != hipSuccess)
      return bail(fail_hip(e, "hipHostMalloc(descriptors)"));
    sv->h_ev.push_back(h);
    if ((e = hipMalloc((void**)&d, sizeof(EvDesc) * opts->max_batch)) != hipSuccess)
      return bail(fail_hip(e, "hipMalloc(descriptors)"));
    sv->d_ev.push_back(d);
    sv->stream_busy.push_back(0);
  }
  sv->th = std::thread(loop, sv);
  *out = sv;
  return HT_OK;
}

int ht_serve_submit(ht_server* sv, const float* x, const float* y, const float* z, int64_t n,
                    uint64_t* ticket)
{
  if (!sv || !ticket) return fail(HT_EINVAL, "NULL server or ticket");
  if (n < 0 || n > sv->opts.max_hits) return fail(HT_EINVAL, "n_hits outside [0, max_hits]");
  if (n > 0 && (!x || !y || !z)) return fail(HT_EINVAL, "hit arrays are NULL");
  const double t = now_s();
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->free_stage.empty()) return fail(HT_EAGAIN, "queue_depth requests outstanding");
  Request* r = new Request();
  r->ticket = sv->next_ticket++;
  r->n = n;
  r->stage = sv->free_stage.back();
  sv->free_stage.pop_back();
  r->t.t_submit = t;
  float* st = sv->stage_pool + (size_t)r->stage * 3 * sv->opts.max_hits;
  std::memcpy(st, x, 4 * (size_t)n);
  std::memcpy(st + n, y, 4 * (size_t)n);
  std::memcpy(st + 2 * n, z, 4 * (size_t)n);
  sv->reqs[r->ticket] = r;
  sv->pending.push_back(r);
  *ticket = r->ticket;
  lk.unlock();
  sv->cv.notify_all();
  return HT_OK;
}

int ht_serve_poll(ht_server* sv, uint64_t ticket, ht_peak* out, int64_t capacity, int64_t* n_found,
                  ht_timing* timing)
{
  if (!sv || !n_found || capacity < 0 || (capacity > 0 && !out))
    return fail(HT_EINVAL, "invalid poll arguments");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(HT_EINVAL, "unknown or released ticket");
  Request* r = it->second;
  if (!r->done) return HT_EAGAIN;
  int status = r->status;
  *n_found = r->n_found;
  if (timing) *timing = r->t;
  if (status == HT_OK) {
    const int64_t k = std::min<int64_t>((int64_t)r->peaks.size(), capacity);
    if (k > 0) std::memcpy(out, r->peaks.data(), sizeof(ht_peak) * (size_t)k);
    if (r->n_found > (int64_t)r->peaks.size() || r->n_found > capacity) {
      status = HT_EOVERFLOW;
      fail(HT_EOVERFLOW, "ticket %llu: %lld peaks do not fit the capacity", (unsigned long long)ticket,
           (long long)r->n_found);
    }
  } else {
    fail(status, "ticket %llu failed on the device", (unsigned long long)ticket);
  }
  sv->reqs.erase(it);
  delete r;
  return status;
}

int ht_serve_destroy(ht_server* sv)
{
  if (!sv) return HT_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  for (hipStream_t s : sv->streams) (void)hipStreamSynchronize(s);
  free_server(sv);
  return HT_OK;
}

}  // extern "C"
