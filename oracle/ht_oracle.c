/*
 * ht_oracle.c -- CPU oracle for the Hough-transform vote fill and local-maxima search.
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow, single-threaded reference that the GPU
 * library is checked against. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it. It shares no source, header, table or constant generator with the
 * GPU library: both sides compute the grid tables independently and a test compares them bit
 * for bit.
 *
 * What it computes (paper section 2, "Tracking with the Hough Transform"):
 *   - every hit (x_H, y_H, z_H) votes for the circles through the interaction point and the hit,
 *     x^2 + y^2 - 2Ax - 2By = 0, whose centre (A, B) lies on the (A, B) grid; the matrix element
 *     M_H(A, B, theta, phi) of each such circle is incremented by one, for the (theta, phi) cells
 *     the hit belongs to;
 *   - after all hits, the elements that are local maxima and reach the threshold are the track
 *     candidates (the second step of the same section; the neighbour comparison of section 3).
 * Section 3 adds that for each A bin the matching B is evaluated, i.e. one vote per (hit, cell,
 * A bin).
 *
 * The paper does not fix how a real B becomes a bin index, nor how theta and phi are binned. The
 * rule below is this project's reading, written out so that the oracle and the GPU kernels can
 * agree bit for bit. Every floating-point step is ONE IEEE-754 binary32 operation rounded to
 * nearest-even, in the order written; nothing is fused or reassociated. Build with
 * -O2 -ffp-contract=off -fno-fast-math on x86-64 (SSE2 float arithmetic, no FMA).
 *
 *   Grid: n_theta x n_phi x n_a x n_b cells, layout [theta][phi][A][B] with B fastest,
 *         cell index c = ((t*n_phi + p)*n_a + a)*n_b + b.  A in [a_min,a_max), B in [b_min,b_max).
 *   O0 tables (computed in double, rounded once to float):
 *         dA = (a_max - a_min)/n_a;  A2[i] = (float)(2*a_min + (2i+1)*dA)   (twice the A-bin centre)
 *         invdB = (float)(n_b/(b_max - b_min))
 *         phi half-bin boundary directions, m in [0, 2 n_phi):
 *             Uphi[m] = ((float)cos(m*pi/n_phi), (float)sin(m*pi/n_phi))
 *         theta half-bin boundary directions in the (z, r) plane, m in [0, 2 n_theta]:
 *             Uth[m]  = ((float)cos(m*pi/(2 n_theta)), (float)sin(m*pi/(2 n_theta)))
 *   O1 a hit votes nothing unless x, y, z are finite, y != 0 and r2 is finite and > 0.
 *   O2 r2 = x*x + y*y;  r = sqrtf(r2);  k = 1/(y + y)              (correctly rounded)
 *   O3 half-plane test P(u; v) := u.c*v.y - u.s*v.x >= 0  (v at or counter-clockwise of u)
 *         phi half-sector s_phi in [0, 2 n_phi):
 *             y > 0:  s_phi = #{ m in [1, n_phi)          : P(Uphi[m]; (x, y)) }
 *             y < 0:  s_phi = n_phi + #{ m in [n_phi+1, 2n_phi) : P(Uphi[m]; (x, y)) }
 *         theta half-sector s_th in [0, 2 n_theta):
 *             s_th = #{ m in [1, 2n_theta) : P(Uth[m]; (z, r)) }
 *         A cell widened by half a bin on each side holds the hit when the hit lies in one of
 *         the cell's own two half-sectors or in the adjacent half-sector of a neighbour:
 *             phi cells: s_phi>>1, and (s_phi odd ? +1 : -1) from it, modulo n_phi (always two);
 *             theta cells: s_th>>1, and (s_th odd ? +1 : -1) from it when inside [0, n_theta).
 *   O4 per A bin i:  num = r2 - A2[i]*x;  B = num*k;  f = (B - b_min)*invdB
 *   O5 vote iff f >= 0 and f < (float)n_b (NaN votes nothing); j = (int)f; for every cell (t,p)
 *      of the hit: M[t][p][i][j] += 1.
 *   O6 cell c is a peak iff M[c] >= T and, for each of its up to 80 neighbours n in the 3^4 box
 *      (theta, A and B are not periodic, so neighbours outside the range are absent; phi wraps
 *      around), M[c] > M[n] or (M[c] == M[n] and c < n).  Peaks are listed by ascending c.
 *
 * Sector variant (paper section 4, phi_sectors = 1): the transverse plane is split into n_phi
 * sectors that are read out and transformed independently, one M_H(A, B, theta) per sector, and
 * the results are merged. Each phi cell is then a sector:
 *   O3' a hit belongs to the one sector holding its azimuth, s_phi>>1 (no widening in phi);
 *       theta cells are as in O3;
 *   O6' the neighbourhood is the 3^3 box in (theta, A, B) inside the peak's own sector (no phi
 *       neighbours); the merged list is every sector's peaks by ascending c.
 *
 * Grid limits: n_theta >= 1, n_phi >= 3 (>= 1 with phi_sectors), 1 <= n_a, n_b <= 2^24,
 * n_theta*n_phi*n_a*n_b <= 2^32, finite ranges with min < max, threshold >= 1, phi_sectors 0 or 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

typedef struct oracle_grid {
  int32_t n_theta, n_phi, n_a, n_b;
  float a_min, a_max, b_min, b_max;
  uint32_t threshold;
  int32_t phi_sectors; /* 0: widened, periodic phi cells; 1: independent phi sectors */
} oracle_grid;

static const double kPi = 3.14159265358979323846;

int oracle_check_grid(const oracle_grid* g)
{
  if (!g) return ORACLE_EINVAL;
  if (g->phi_sectors != 0 && g->phi_sectors != 1) return ORACLE_EINVAL;
  if (g->n_theta < 1 || g->n_phi < (g->phi_sectors ? 1 : 3) || g->n_a < 1 || g->n_b < 1)
    return ORACLE_EINVAL;
  if (g->n_a > (1 << 24) || g->n_b > (1 << 24)) return ORACLE_EINVAL;
  if (!isfinite(g->a_min) || !isfinite(g->a_max) || !isfinite(g->b_min) || !isfinite(g->b_max))
    return ORACLE_EINVAL;
  if (!(g->a_min < g->a_max) || !(g->b_min < g->b_max)) return ORACLE_EINVAL;
  if (g->threshold < 1) return ORACLE_EINVAL;
  double cells = (double)g->n_theta * g->n_phi * (double)g->n_a * (double)g->n_b;
  if (cells > 4294967296.0) return ORACLE_EINVAL;
  return ORACLE_OK;
}

/* O0. a2: n_a floats; inv_db: 1 float; phi_cs: 2*(2*n_phi) floats (cos, sin pairs);
 * th_cs: 2*(2*n_theta+1) floats (cos, sin pairs). */
int oracle_tables(const oracle_grid* g, float* a2, float* inv_db, float* phi_cs, float* th_cs)
{
  if (oracle_check_grid(g) != ORACLE_OK) return ORACLE_EINVAL;
  double da = ((double)g->a_max - (double)g->a_min) / (double)g->n_a;
  for (int32_t i = 0; i < g->n_a; ++i)
    a2[i] = (float)(2.0 * (double)g->a_min + (double)(2 * (int64_t)i + 1) * da);
  *inv_db = (float)((double)g->n_b / ((double)g->b_max - (double)g->b_min));
  for (int32_t m = 0; m < 2 * g->n_phi; ++m) {
    double ang = ((double)m * kPi) / (double)g->n_phi;
    phi_cs[2 * m] = (float)cos(ang);
    phi_cs[2 * m + 1] = (float)sin(ang);
  }
  for (int32_t m = 0; m <= 2 * g->n_theta; ++m) {
    double ang = ((double)m * kPi) / (double)(2 * g->n_theta);
    th_cs[2 * m] = (float)cos(ang);
    th_cs[2 * m + 1] = (float)sin(ang);
  }
  return ORACLE_OK;
}

/* P(u; v): v lies on or counter-clockwise of direction u (both in one half-plane). */
static int half_plane(float uc, float us, float vx, float vy)
{
  float lhs = uc * vy;
  float rhs = us * vx;
  return (lhs - rhs) >= 0.0f;
}

typedef struct hit_state {
  int valid;
  float x, r2, r, k;
  int32_t s_theta, s_phi;
  int32_t n_cells;
  int32_t cell_t[4], cell_p[4];
} hit_state;

/* O1-O3 for one hit. */
static void prepare_hit(const oracle_grid* g, const float* phi_cs, const float* th_cs, float x,
                        float y, float z, hit_state* h)
{
  memset(h, 0, sizeof(*h));
  if (!isfinite(x) || !isfinite(y) || !isfinite(z) || y == 0.0f) return;
  float xx = x * x;
  float yy = y * y;
  float r2 = xx + yy;
  if (!(r2 > 0.0f) || isinf(r2)) return;
  h->valid = 1;
  h->x = x;
  h->r2 = r2;
  h->r = sqrtf(r2);
  float twice_y = y + y;
  h->k = 1.0f / twice_y;

  /* O3: phi half-sector by counting the boundaries the hit is at or past. */
  int32_t s_phi;
  if (y > 0.0f) {
    s_phi = 0;
    for (int32_t m = 1; m < g->n_phi; ++m)
      s_phi += half_plane(phi_cs[2 * m], phi_cs[2 * m + 1], x, y);
  } else {
    s_phi = g->n_phi;
    for (int32_t m = g->n_phi + 1; m < 2 * g->n_phi; ++m)
      s_phi += half_plane(phi_cs[2 * m], phi_cs[2 * m + 1], x, y);
  }
  /* O3: theta half-sector in the (z, r) plane, r > 0. */
  int32_t s_th = 0;
  for (int32_t m = 1; m < 2 * g->n_theta; ++m)
    s_th += half_plane(th_cs[2 * m], th_cs[2 * m + 1], z, h->r);
  h->s_theta = s_th;
  h->s_phi = s_phi;

  int32_t pc[2], tc[2], nt = 0;
  const int32_t np_cells = g->phi_sectors ? 1 : 2; /* O3': a sector holds the hit alone */
  pc[0] = s_phi >> 1;
  pc[1] = (s_phi & 1) ? (pc[0] + 1) % g->n_phi : (pc[0] - 1 + g->n_phi) % g->n_phi;
  tc[nt++] = s_th >> 1;
  {
    int32_t other = (s_th & 1) ? (s_th >> 1) + 1 : (s_th >> 1) - 1;
    if (other >= 0 && other < g->n_theta) tc[nt++] = other;
  }
  h->n_cells = 0;
  for (int32_t a = 0; a < nt; ++a)
    for (int32_t b = 0; b < np_cells; ++b) {
      h->cell_t[h->n_cells] = tc[a];
      h->cell_p[h->n_cells] = pc[b];
      h->n_cells++;
    }
}

/* O1-O3 per hit, exposed for tests. info[4*h] = {valid, s_theta, s_phi, n_cells};
 * vals[3*h] = {r2, r, k}; cells_tp[8*h] = up to four (t, p) pairs, padded with -1. */
int oracle_hit_info(const oracle_grid* g, const float* x, const float* y, const float* z,
                    int64_t n, int32_t* info, float* vals, int32_t* cells_tp)
{
  if (oracle_check_grid(g) != ORACLE_OK) return ORACLE_EINVAL;
  float* a2 = (float*)malloc(sizeof(float) * (size_t)g->n_a);
  float* phi_cs = (float*)malloc(sizeof(float) * 4 * (size_t)g->n_phi);
  float* th_cs = (float*)malloc(sizeof(float) * (4 * (size_t)g->n_theta + 2));
  float inv_db;
  oracle_tables(g, a2, &inv_db, phi_cs, th_cs);
  for (int64_t i = 0; i < n; ++i) {
    hit_state h;
    prepare_hit(g, phi_cs, th_cs, x[i], y[i], z[i], &h);
    info[4 * i + 0] = h.valid;
    info[4 * i + 1] = h.s_theta;
    info[4 * i + 2] = h.s_phi;
    info[4 * i + 3] = h.n_cells;
    vals[3 * i + 0] = h.r2;
    vals[3 * i + 1] = h.r;
    vals[3 * i + 2] = h.k;
    for (int c = 0; c < 4; ++c) {
      cells_tp[8 * i + 2 * c] = c < h.n_cells ? h.cell_t[c] : -1;
      cells_tp[8 * i + 2 * c + 1] = c < h.n_cells ? h.cell_p[c] : -1;
    }
  }
  free(a2);
  free(phi_cs);
  free(th_cs);
  return ORACLE_OK;
}

/* O1-O5: overwrites all of M (n_theta*n_phi*n_a*n_b uint32) and returns the number of votes
 * cast, or ORACLE_EINVAL. */
int64_t oracle_fill(const oracle_grid* g, const float* x, const float* y, const float* z,
                    int64_t n, uint32_t* M)
{
  if (oracle_check_grid(g) != ORACLE_OK || n < 0) return ORACLE_EINVAL;
  const int64_t n_a = g->n_a, n_b = g->n_b, n_phi = g->n_phi;
  const int64_t cells = (int64_t)g->n_theta * n_phi * n_a * n_b;
  memset(M, 0, sizeof(uint32_t) * (size_t)cells);
  float* a2 = (float*)malloc(sizeof(float) * (size_t)n_a);
  float* phi_cs = (float*)malloc(sizeof(float) * 4 * (size_t)n_phi);
  float* th_cs = (float*)malloc(sizeof(float) * (4 * (size_t)g->n_theta + 2));
  float inv_db;
  oracle_tables(g, a2, &inv_db, phi_cs, th_cs);
  const float b_min = g->b_min;
  const float nb_f = (float)g->n_b;
  int64_t votes = 0;
  for (int64_t h = 0; h < n; ++h) {
    hit_state s;
    prepare_hit(g, phi_cs, th_cs, x[h], y[h], z[h], &s);
    if (!s.valid) continue;
    for (int64_t i = 0; i < n_a; ++i) {
      float ax = a2[i] * s.x;
      float num = s.r2 - ax;
      float B = num * s.k;
      float d = B - b_min;
      float f = d * inv_db;
      if (!(f >= 0.0f && f < nb_f)) continue;
      int64_t j = (int64_t)f;
      for (int32_t c = 0; c < s.n_cells; ++c) {
        int64_t slab = (int64_t)s.cell_t[c] * n_phi + s.cell_p[c];
        M[(slab * n_a + i) * n_b + j] += 1u;
        votes++;
      }
    }
  }
  free(a2);
  free(phi_cs);
  free(th_cs);
  return votes;
}

/* O6: writes up to `capacity` peaks in ascending cell order and returns the total number found,
 * or ORACLE_EINVAL. */
int64_t oracle_peaks(const oracle_grid* g, const uint32_t* M, uint32_t* out_cell,
                     uint32_t* out_votes, int64_t capacity)
{
  if (oracle_check_grid(g) != ORACLE_OK || capacity < 0) return ORACLE_EINVAL;
  const int64_t n_t = g->n_theta, n_p = g->n_phi, n_a = g->n_a, n_b = g->n_b;
  const int64_t cells = n_t * n_p * n_a * n_b;
  const uint32_t T = g->threshold;
  const int dp_max = g->phi_sectors ? 0 : 1; /* O6': no neighbours across sectors */
  int64_t found = 0;
  for (int64_t c = 0; c < cells; ++c) {
    uint32_t v = M[c];
    if (v < T) continue;
    int64_t b = c % n_b;
    int64_t a = (c / n_b) % n_a;
    int64_t p = (c / (n_b * n_a)) % n_p;
    int64_t t = c / (n_b * n_a * n_p);
    int is_peak = 1;
    for (int dt = -1; dt <= 1 && is_peak; ++dt)
      for (int dp = -dp_max; dp <= dp_max && is_peak; ++dp)
        for (int da = -1; da <= 1 && is_peak; ++da)
          for (int db = -1; db <= 1 && is_peak; ++db) {
            if (dt == 0 && dp == 0 && da == 0 && db == 0) continue;
            int64_t tt = t + dt, aa = a + da, bb = b + db;
            if (tt < 0 || tt >= n_t || aa < 0 || aa >= n_a || bb < 0 || bb >= n_b) continue;
            int64_t pp = (p + dp + n_p) % n_p;
            int64_t nb = ((tt * n_p + pp) * n_a + aa) * n_b + bb;
            uint32_t w = M[nb];
            if (w > v || (w == v && nb < c)) is_peak = 0;
          }
    if (!is_peak) continue;
    if (found < capacity) {
      out_cell[found] = (uint32_t)c;
      out_votes[found] = v;
    }
    found++;
  }
  return found;
}

/* Track parameters of peaks (paper section 2: the circle centre (A, B) of a maximum gives
 * rho = sqrt(A^2 + B^2) and the azimuth phi = tan^-1(B/A) of the centre, taken in [0, 2 pi)
 * with atan2 so that the quadrant is kept). A and B are the centres of the peak's A and B bins,
 * A = A2[a] / 2 and B = b_min + (b + 1/2) (b_max - b_min) / n_b; theta is the centre of the
 * peak's theta cell. Computed in double. out[9*i] = {t, p, a, b, A, B, rho, phi, theta} with the
 * four indices as doubles; n_out = n. */
int oracle_readout(const oracle_grid* g, const uint32_t* cells, int64_t n, double* out)
{
  if (oracle_check_grid(g) != ORACLE_OK || n < 0) return ORACLE_EINVAL;
  float* a2 = (float*)malloc(sizeof(float) * (size_t)g->n_a);
  float* phi_cs = (float*)malloc(sizeof(float) * 4 * (size_t)g->n_phi);
  float* th_cs = (float*)malloc(sizeof(float) * (4 * (size_t)g->n_theta + 2));
  float inv_db;
  oracle_tables(g, a2, &inv_db, phi_cs, th_cs);
  const int64_t n_b = g->n_b, n_a = g->n_a, n_p = g->n_phi;
  const double db = ((double)g->b_max - (double)g->b_min) / (double)g->n_b;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t c = cells[i];
    const int64_t b = c % n_b, a = (c / n_b) % n_a, p = (c / (n_b * n_a)) % n_p;
    const int64_t t = c / (n_b * n_a * n_p);
    const double A = 0.5 * (double)a2[a];
    const double B = (double)g->b_min + ((double)b + 0.5) * db;
    double phi = atan2(B, A);
    if (phi < 0.0) phi += 2.0 * kPi;
    double* o = out + 9 * i;
    o[0] = (double)t;
    o[1] = (double)p;
    o[2] = (double)a;
    o[3] = (double)b;
    o[4] = A;
    o[5] = B;
    o[6] = sqrt(A * A + B * B);
    o[7] = phi;
    o[8] = ((double)t + 0.5) * kPi / (double)g->n_theta;
  }
  free(a2);
  free(phi_cs);
  free(th_cs);
  return ORACLE_OK;
}
