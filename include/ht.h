/*
 * ht.h -- C ABI of the MI355X Hough-transform track-finding library (libht.so).
 *
 * The library computes the two steps of the track finder of Rinaldi et al., "GPGPU for track
 * finding in High Energy Physics" (arXiv:1507.03074):
 *
 *   1. Fill (section 2; kernel decomposition in section 3): every hit (x_H, y_H, z_H) votes
 *      for the circles x^2 + y^2 - 2Ax - 2By = 0 through the interaction point and the hit; for
 *      each A bin the matching B is evaluated and the element M_H(A, B, theta, phi) of every
 *      (theta, phi) cell that holds the hit is incremented by one.
 *   2. Peak search (section 2, second step; neighbour comparison in section 3): the elements
 *      that are local maxima of M_H and reach a threshold are the track candidates.
 *
 * Bin rule. The paper fixes neither the binning of theta and phi nor how a real B becomes a
 * bin index. This library uses the following rule, in IEEE-754 binary32 with one rounding per
 * operation, in the order written, nothing fused (it is the rule the CPU oracle follows, so
 * results are bit-exact):
 *   - tables, computed on the host in double and rounded once to float:
 *       A2[i]  = (float)(2*a_min + (2i+1)*((a_max - a_min)/n_a))        (twice the A-bin centre)
 *       invdB  = (float)(n_b / (b_max - b_min))
 *       Uphi[m] = ((float)cos(m*pi/n_phi), (float)sin(m*pi/n_phi)),          m in [0, 2 n_phi)
 *       Uth[m]  = ((float)cos(m*pi/(2 n_theta)), (float)sin(m*pi/(2 n_theta))), m in [0, 2 n_theta]
 *   - a hit votes nothing unless x, y, z are finite, y != 0 and r2 = x*x + y*y is finite and > 0;
 *   - r = sqrtf(r2), k = 1/(y + y), both correctly rounded;
 *   - half-plane test P(u; v) := u.cos*v.y - u.sin*v.x >= 0;
 *     phi half-sector: y > 0: s = #{m in [1, n_phi): P(Uphi[m]; (x,y))},
 *                      y < 0: s = n_phi + #{m in [n_phi+1, 2 n_phi): P(Uphi[m]; (x,y))};
 *     theta half-sector: s = #{m in [1, 2 n_theta): P(Uth[m]; (z,r))};
 *     each cell's range is widened by half a bin on both sides, so the hit lies in phi cells
 *     s>>1 and (s odd ? s>>1 + 1 : s>>1 - 1) mod n_phi, and in theta cell s>>1 plus
 *     (s odd ? +1 : -1) from it when that is inside [0, n_theta);
 *   - per A bin i: num = r2 - A2[i]*x; B = num*k; f = (B - b_min)*invdB; the hit votes iff
 *     f >= 0 and f < n_b, at B bin j = (int)f, in every (theta, phi) cell it lies in;
 *   - cell c is a peak iff M[c] >= threshold and, for every neighbour n in its 3^4 box (theta,
 *     A and B are not periodic, phi is), M[c] > M[n] or (M[c] == M[n] and c < n).
 *
 * Layout. The vote matrix is uint32 [n_theta][n_phi][n_a][n_b], B fastest; the cell index is
 * c = ((t*n_phi + p)*n_a + a)*n_b + b. Peaks are listed by ascending cell index.
 *
 * Conventions for every call:
 *   - return value: HT_OK (0) or a negative ht_status; ht_last_error() describes the last
 *     failure of the calling thread. No exception crosses the ABI.
 *   - argument validation happens on the host, before any device work, and fails synchronously.
 *   - "device pointer" arguments are GPU memory owned by the caller (e.g. torch tensors); the
 *     library never frees them. Work is enqueued on `stream` (a hipStream_t, NULL for the null
 *     stream) and is asynchronous unless stated otherwise.
 *   - the peak outputs (out, n_found, and ht_readout's arrays) may also be pinned host memory
 *     mapped into the device (hipHostMalloc): the kernels then write the results straight to
 *     the host, with no copy afterwards. Any other host pointer there is rejected (HT_EINVAL).
 *   - device failures are reported as HT_EDEVICE by the call that observes them.
 *   - the library keeps per-(device, stream) scratch memory; calls on one stream are ordered,
 *     calls on different streams never share scratch. Host threads may call concurrently on
 *     different streams; calls on one stream must come from one host thread at a time (they
 *     share that stream's scratch and its small host-side state).
 *   - ht_set_tuning affects calls that start after it returns; it is safe to call from any
 *     thread.
 */
#ifndef HT_H_
#define HT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ht_status {
  HT_OK = 0,
  HT_EINVAL = -1,     /* invalid argument (grid, sizes, null pointer) */
  HT_ENOMEM = -2,     /* device or pinned-host allocation failed */
  HT_EOVERFLOW = -3,  /* more peaks than the output capacity (server poll only) */
  HT_EAGAIN = -4,     /* not ready / queue full (server only) */
  HT_EDEVICE = -5     /* a HIP runtime call failed */
} ht_status;

/* Binning of the vote matrix. Limits: n_theta >= 1, n_phi >= 3 (>= 1 with phi_sectors),
 * n_theta*n_phi <= 4096, 1 <= n_a, n_b <= 2^24, n_theta*n_phi*n_a*n_b <= 2^32, finite ranges
 * with min < max, threshold >= 1, phi_sectors 0 or 1. A and B are in the units of the hit
 * coordinates (mm); ranges are half-open.
 * phi_sectors = 0: the 4-D transform of section 2: phi cells widened by half a bin (two per
 *   hit), phi periodic in the peak search.
 * phi_sectors = 1: the sector variant of section 4: the n_phi phi cells are sectors of the
 *   transverse plane transformed independently, one M_H(A, B, theta) each: a hit votes in its
 *   own sector only, and a peak is compared with its (theta, A, B) neighbours in that sector
 *   only (3^3 box); the peak list is the merge of all sectors' peaks by ascending cell. */
typedef struct ht_grid {
  int32_t n_theta, n_phi, n_a, n_b;
  float a_min, a_max, b_min, b_max;
  uint32_t threshold;
  int32_t phi_sectors;
} ht_grid;

/* One local maximum: its cell index and vote count. */
typedef struct ht_peak {
  uint32_t cell;
  uint32_t votes;
} ht_peak;

/* Launch shape of the kernels for one grid. Results never depend on it (every shape gives
 * bit-identical matrices and peak lists); only speed does. Zero (or -1 for nt_store) means the
 * library's default for that field. */
typedef struct ht_tuning {
  int32_t rows;         /* A rows per fill tile: a power of two <= 64 whose rows x n_b uint32
                           counters fit in 56 KiB of LDS */
  int32_t group_tiles;  /* tiles per workgroup of the peak search: 16, 32 or 64 */
  int32_t cand_cap;     /* candidate-pool entries per tile, a power of two <= 4096: the cells
                           at or above the threshold of all tiles share a pool of at least
                           n_tiles * cand_cap entries (more for large events: a quarter of the
                           bound 4 n_hits n_a / threshold, at most the cell count); tiles that
                           do not fit are searched densely (slower, same results) */
  int32_t nt_store;     /* store kind of the fill's single write of the matrix: 0 ordinary
                           16-byte stores, 1 non-temporal 16-byte stores, 2 ordinary 4-byte
                           stores */
  int32_t tiles_per_block; /* fill tiles per workgroup, filled in turn with one LDS tile (the
                              slab's hit records are read once): a power of two <= 64 */
  int32_t dense_hits;   /* crowded events: a fused fill + peak search of an event with at least
                           this many hits finds its peaks with a stencil over the whole matrix
                           (one read of it, cost independent of the number of candidates)
                           instead of the candidate pool; -1 never. The default is
                           n_theta n_phi n_b / 4 hits (16384 on the 4x16x1024x1024 grid), about
                           where the stencil starts to beat the pool. The stencil needs LDS
                           fill tiles, at most 4 theta and 16 phi cells (one wave per phi cell
                           holds every theta cell's row), and theta cell 0's row and the last
                           one's less than 2^31 bytes apart; ht_get_tuning reports -1 where it
                           is unavailable. */
} ht_tuning;

/* ht_set_tuning: use `tuning` for every later call on grids with these dimensions and ranges
 * (the threshold is ignored); NULL restores the defaults. Host only.
 * Errors: HT_EINVAL for an invalid grid or a field outside its range. */
int ht_set_tuning(const ht_grid* grid, const ht_tuning* tuning);

/* ht_get_tuning: the launch shape the library will use for `grid` (defaults filled in). */
int ht_get_tuning(const ht_grid* grid, ht_tuning* tuning);

/* ht_tables: the bin-rule tables above, computed on the host (no device work). Host pointers:
 * a2[n_a], inv_db[1], phi_cs[2*(2*n_phi)] and th_cs[2*(2*n_theta+1)] as (cos, sin) pairs.
 * Errors: HT_EINVAL for an invalid grid or a null pointer. */
int ht_tables(const ht_grid* grid, float* a2, float* inv_db, float* phi_cs, float* th_cs);

/* ht_fill: step 1 (paper section 2) for one event.
 * x, y, z: device float[n_hits], the hit coordinates (structure of arrays).
 * acc: device uint32[n_theta*n_phi*n_a*n_b]; every element is overwritten (no pre-zeroing).
 * n_hits may be 0 (acc becomes all zeros).
 * Errors: HT_EINVAL (grid, n_hits < 0, null pointers with n_hits > 0 or acc null),
 * HT_ENOMEM (scratch), HT_EDEVICE. */
int ht_fill(const ht_grid* grid, const float* x, const float* y, const float* z, int64_t n_hits,
            uint32_t* acc, void* stream);

/* ht_peaks: step 2 (paper section 2; neighbour comparison of section 3) on any vote matrix.
 * acc: device uint32 matrix in the layout above (read only).
 * out: device ht_peak[capacity]; receives the first min(found, capacity) peaks by ascending cell.
 * n_found: device int64[1]; receives the total number of peaks, which may exceed capacity
 * (truncation is detected by the caller after synchronising: *n_found > capacity).
 * capacity may be 0 (out may then be NULL).
 * Errors: HT_EINVAL, HT_ENOMEM, HT_EDEVICE. */
int ht_peaks(const ht_grid* grid, const uint32_t* acc, ht_peak* out, int64_t capacity,
             int64_t* n_found, void* stream);

/* ht_fill_peaks: both steps for one event in one call. Same arguments and results as ht_fill
 * followed by ht_peaks on the same acc; the peak search takes its candidates from the fill, so
 * the matrix is written once and not read back in full. */
int ht_fill_peaks(const ht_grid* grid, const float* x, const float* y, const float* z,
                  int64_t n_hits, uint32_t* acc, ht_peak* out, int64_t capacity,
                  int64_t* n_found, void* stream);

/* ht_fill_peaks_noalloc: ht_fill_peaks for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid hipMalloc). Same arguments
 * and results as ht_fill_peaks (bit-identical matrix, peak list and count), but all of the
 * library's scratch for the call (slab lists, candidate pool, counters, tables) lives in one
 * fixed 64 MiB device array that each GPU the library runs on holds until the process ends;
 * the call makes no hipMalloc, hipFree or other allocating call.
 * Limits: n_a <= 16384, and the event's scratch must fit the array: direct slab lists are used
 * while they fit, else the counting sort; about 25 MB for 5000 hits on the 4x16x1024x1024 grid,
 * where events of up to about 500 000 hits fit (crowded events need no candidate pool). A larger
 * event is refused with HT_EINVAL before any device work, and ht_last_error() states the bytes
 * it needed (use ht_fill_peaks for it).
 * Sharing: every call on one GPU uses that GPU's array, which keeps the last call's contents.
 * Calls on one GPU must not overlap (on different streams or host threads they race on the
 * array); calls are serialised on the host by a lock, so overlap only arises from work still
 * running on the device when a call on another stream starts. The first call with a grid whose
 * tables differ from the last one's uploads the tables with a synchronous copy on `stream`, so
 * make that first call outside any graph capture.
 * Errors: as ht_fill_peaks. */
int ht_fill_peaks_noalloc(const ht_grid* grid, const float* x, const float* y, const float* z,
                          int64_t n_hits, uint32_t* acc, ht_peak* out, int64_t capacity,
                          int64_t* n_found, void* stream);

/* Track parameters of one peak (paper section 2: the centre (A, B) of the circle gives
 * rho = sqrt(A^2 + B^2) and phi = tan^-1(B/A)). */
typedef struct ht_track {
  uint32_t cell, votes;   /* the peak */
  int32_t t, p, a, b;     /* its theta, phi, A and B bin indices */
  float A, B;             /* centres of its A and B bins (mm): the circle centre */
  float rho;              /* sqrt(A^2 + B^2): the circle radius, proportional to p_T */
  float phi;              /* atan2(B, A) in [0, 2 pi): azimuth of the centre */
  float theta;            /* centre of its theta cell (rad) */
} ht_track;

/* ht_readout: track parameters of a peak list (NEXT to the peak search, paper section 2).
 * peaks: device ht_peak[capacity] as written by ht_peaks / ht_fill_peaks; n_found: device int64,
 * the count written by that call (entries past min(*n_found, capacity) are not read);
 * tracks: device ht_track[capacity], entry i filled for i < min(*n_found, capacity).
 * Values are computed in double and rounded once to float. Asynchronous on stream.
 * Errors: HT_EINVAL, HT_EDEVICE. */
int ht_readout(const ht_grid* grid, const ht_peak* peaks, const int64_t* n_found, int64_t capacity,
               ht_track* tracks, void* stream);

/* One event of a batch: its hits are x/y/z[hit_offset, hit_offset + n_hits) of the concatenated
 * arrays; its peaks go to out[peak_offset, peak_offset + peak_capacity). */
typedef struct ht_event {
  int64_t hit_offset;
  int64_t n_hits;
  int64_t peak_offset;
  int64_t peak_capacity;
} ht_event;

/* ht_fill_peaks_batch: both steps for n_events independent events of uneven sizes. The stages
 * (prep, fill, peak search) each run as one launch over the whole batch; the sequence, with the
 * upload of the event descriptors, is captured once per batch shape into a HIP graph and
 * replayed, so a batch costs one graph launch on the host.
 * events: HOST ht_event[n_events] (copied before the call returns).
 * x, y, z: device float arrays holding all events' hits.
 * acc: device uint32[n_events * cells]; event e's matrix is acc + e*cells, fully overwritten.
 * out: device ht_peak array covering every event's [peak_offset, peak_offset + peak_capacity).
 * n_found: device int64[n_events]; total peaks per event (may exceed its capacity).
 * Results are bit-identical to ht_fill_peaks on each event alone.
 * Errors: HT_EINVAL, HT_ENOMEM, HT_EDEVICE. */
int ht_fill_peaks_batch(const ht_grid* grid, const ht_event* events, int32_t n_events,
                        const float* x, const float* y, const float* z, uint32_t* acc,
                        ht_peak* out, int64_t* n_found, void* stream);

/* ------------------------------------------------------------------------------------------
 * Serving: a request loop on a background thread. Events are submitted from the host as they
 * arrive; the server admits them while device memory for their vote matrices is available
 * (hbm_budget_bytes), groups whatever is admitted into batches, runs them on n_streams streams
 * so that batches overlap on the device, and hands peak lists back by ticket.
 * ------------------------------------------------------------------------------------------ */
typedef struct ht_serve_opts {
  int64_t hbm_budget_bytes;   /* device bytes for vote matrices, hits and scratch (> 0) */
  int64_t peak_capacity;      /* per event (> 0) */
  int64_t max_hits;           /* largest event accepted (> 0) */
  int32_t max_batch;          /* events per launched batch (>= 1) */
  int32_t n_streams;          /* device streams used for overlapping batches (>= 1) */
  int32_t queue_depth;        /* requests submitted and not yet completed (>= 1); each holds
                                 a pinned staging buffer of max_hits hits until it completes */
  int32_t device;             /* HIP device ordinal */
} ht_serve_opts;

/* Host monotonic timestamps (seconds, CLOCK_MONOTONIC) of one request's life. */
typedef struct ht_timing {
  double t_submit, t_admit, t_launch, t_done;
} ht_timing;

typedef struct ht_server ht_server;

/* ht_serve_create: allocates the server's device memory and starts its thread.
 * Errors: HT_EINVAL, HT_ENOMEM, HT_EDEVICE; *server is NULL on failure. */
int ht_serve_create(const ht_grid* grid, const ht_serve_opts* opts, ht_server** server);

/* ht_serve_submit: HOST x, y, z[n_hits]; copied into the server's pinned staging before the
 * call returns (the caller may reuse its buffers at once). *ticket identifies the request.
 * Errors: HT_EINVAL (n_hits < 0 or > max_hits), HT_EAGAIN (queue_depth requests submitted and
 * not yet completed: retry after some complete). */
int ht_serve_submit(ht_server* server, const float* x, const float* y, const float* z,
                    int64_t n_hits, uint64_t* ticket);

/* ht_serve_poll: non-blocking. HT_EAGAIN while the request is in flight. When done, copies
 * min(found, capacity) peaks to the HOST array out, sets *n_found (host) to the total, fills
 * *timing if non-NULL, releases the ticket and returns HT_OK, or HT_EOVERFLOW if the peaks did
 * not fit the server's peak_capacity or the caller's capacity (the first ones are still
 * delivered). An unknown or already released ticket gives HT_EINVAL. */
int ht_serve_poll(ht_server* server, uint64_t ticket, ht_peak* out, int64_t capacity,
                  int64_t* n_found, ht_timing* timing);

/* ht_serve_destroy: waits for in-flight batches, stops the thread and frees everything.
 * Unpolled results are discarded. NULL is accepted. */
int ht_serve_destroy(ht_server* server);

/* Message for the last failure on the calling thread ("" if none). Valid until the next call. */
const char* ht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HT_H_ */
