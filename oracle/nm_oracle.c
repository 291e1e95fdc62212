/*
 * nm_oracle.c -- brute-force CPU reference ("oracle") for the non-metric
 * neighbour lists and the Vicsek alignment step of
 *   D. M. Sussman, "Non-metric interaction rules in models of active matter"
 *   (arXiv:2103.10239).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * with the HIP path.
 *
 * Everything here is the plain definition written out:
 *   - neighbour lists by evaluating all N^2 pairs (the naive O(N^2) cost the
 *     paper names in Sec. I);
 *   - the metric rule "all pairs within r_0" (Sec. III);
 *   - the topological rule "the k nearest neighbours" (Sec. III);
 *   - the alignment rule Eq. (2) and the Euler move Eq. (1), in fp64;
 *   - Philox4x32-10 from Salmon, Moraes, Dror & Shaw, "Parallel random
 *     numbers: as easy as 1, 2, 3" (SC'11), for the noise vector of Eq. (2).
 *
 * Conventions the paper leaves open (each is a documented reading):
 *   - periodic square box of side L, integer coordinates in [0, L), minimum
 *     image with delta in [-L/2, L/2), squared distance in int64;
 *   - ties at equal distance are broken by the smaller particle index, i.e.
 *     candidates are ordered by the pair (d^2, j);
 *   - a particle is never its own neighbour; duplicates (d^2 = 0) are valid
 *     neighbours;
 *   - the metric rule is inclusive: d^2 <= r_c^2;
 *   - the alignment average optionally includes the particle's own heading
 *     (include_self), the zero vector keeps the old heading, and the move uses
 *     the heading at time t (Eq. 1), rounded to the integer grid with
 *     round-half-even;
 *   - two variants of the step, from the Vicsek-model family the alignment
 *     rule belongs to (flags in `variant`): angular noise (bit 0), where the
 *     new heading is the direction of the average plus eta times the noise
 *     angle, wrapped into [-pi, pi) (the particle's own heading stands in for
 *     the direction of a zero average); and the move with the new heading
 *     n_i(t+1) (bit 1);
 *   - the polar order parameter |sum_i n_i| / N of the headings;
 *   - a field-of-view topological rule: the k nearest among the particles
 *     inside a cone around the heading (see orc_knn_fov for its exact test);
 *   - noise word for particle i at step t of system s is word (i mod 4) of
 *     Philox4x32-10(counter = (i / 4, t mod 2^32, t >> 32, s),
 *                   key = (seed mod 2^32, seed >> 32)),
 *     and the noise angle is phi = fl(fl(u * 2^-32) * 2pi) - pi.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 * Floating-point contraction must stay off so that every operation above is
 * a separately rounded IEEE fp64 operation.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_CAPACITY (-3)
#define ORC_E_NOMEM (-4)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 5): ten rounds of the Philox
 * S-box/P-box, with the Weyl-sequence key schedule between rounds.          */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u; /* multiplier applied to word 0 */
static const uint32_t PHILOX_M1 = 0xCD9E8D57u; /* multiplier applied to word 2 */
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden-ratio key increment   */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3)-1 key increment      */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Noise word u_i of particle i at step `step` of system `sys_id`. */
uint32_t orc_noise_word(uint64_t seed, uint32_t sys_id, uint64_t step, int64_t i) {
  uint32_t ctr[4] = {(uint32_t)(i / 4), (uint32_t)step, (uint32_t)(step >> 32), sys_id};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[i % 4];
}

/* Angle of the random unit vector xi_i of Eq. (2): uniform in [-pi, pi). */
double orc_noise_angle(uint64_t seed, uint32_t sys_id, uint64_t step, int64_t i) {
  uint32_t u = orc_noise_word(seed, sys_id, step, i);
  double unit = (double)u * 0x1p-32;   /* exact: u < 2^32 */
  double turn = unit * (2.0 * M_PI);   /* one rounding    */
  return turn - M_PI;                  /* one rounding    */
}

/* ------------------------------------------------------------------------ */
/* Geometry: periodic minimum image, squared distance.                      */
/* ------------------------------------------------------------------------ */
static int64_t min_image(int64_t delta, int64_t box) {
  if (2 * delta >= box) delta -= box;
  if (2 * delta < -box) delta += box;
  return delta;
}

int64_t orc_d2(int32_t xa, int32_t ya, int32_t xb, int32_t yb, int32_t box) {
  int64_t dx = min_image((int64_t)xb - (int64_t)xa, box);
  int64_t dy = min_image((int64_t)yb - (int64_t)ya, box);
  return dx * dx + dy * dy;
}

static int check_coords(const int32_t* x, const int32_t* y, int32_t n, int32_t box) {
  for (int32_t i = 0; i < n; ++i)
    if (x[i] < 0 || x[i] >= box || y[i] < 0 || y[i] >= box) return ORC_E_RANGE;
  return ORC_OK;
}

/* Candidate ordering: by squared distance, then by particle index. */
typedef struct {
  int64_t d2;
  int32_t j;
} cand_t;

static int cand_less(cand_t a, cand_t b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.j < b.j);
}

static int cand_cmp(const void* pa, const void* pb) {
  cand_t a = *(const cand_t*)pa, b = *(const cand_t*)pb;
  if (cand_less(a, b)) return -1;
  if (cand_less(b, a)) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Topological rule: the k nearest neighbours of each particle.             */
/* rows == NULL: every particle, output row r is particle r.                */
/* rows != NULL: output row r is particle rows[r] (sampled rows).           */
/* nbr: int32[nrows * k]; d2: int64[nrows * k] or NULL.                     */
/* ------------------------------------------------------------------------ */
int orc_knn(const int32_t* x, const int32_t* y, int32_t n, int32_t box, int32_t k,
            const int32_t* rows, int32_t nrows, int32_t* nbr, int64_t* d2) {
  if (n < 2 || box < 1 || k < 1 || k > n - 1) return ORC_E_INVAL;
  if (check_coords(x, y, n, box) != ORC_OK) return ORC_E_RANGE;
  int32_t count = rows ? nrows : n;
  if (rows)
    for (int32_t r = 0; r < nrows; ++r)
      if (rows[r] < 0 || rows[r] >= n) return ORC_E_INVAL;
  int failed = 0;
#pragma omp parallel
  {
    cand_t* best = (cand_t*)malloc(sizeof(cand_t) * (size_t)k);
    if (!best) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int32_t r = 0; r < count; ++r) {
      if (!best) continue;
      int32_t i = rows ? rows[r] : r;
      int32_t have = 0; /* best[0..have) holds the smallest keys seen, ascending */
      for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        cand_t c = {orc_d2(x[i], y[i], x[j], y[j], box), j};
        if (have == k && !cand_less(c, best[k - 1])) continue;
        int32_t pos = (have < k) ? have++ : k - 1;
        while (pos > 0 && cand_less(c, best[pos - 1])) {
          best[pos] = best[pos - 1];
          --pos;
        }
        best[pos] = c;
      }
      for (int32_t t = 0; t < k; ++t) {
        nbr[(int64_t)r * k + t] = best[t].j;
        if (d2) d2[(int64_t)r * k + t] = best[t].d2;
      }
    }
    free(best);
  }
  return failed ? ORC_E_NOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Field-of-view topological rule: the k nearest among the particles inside */
/* a cone around the particle's heading (the topological rule of Sec. III,  */
/* restricted to what the particle faces).  The heading vector is          */
/* h = (rint(4096 cos theta), rint(4096 sin theta)) in fp64 from the fp32   */
/* heading; the cone's half angle alpha is given by cos alpha = c / 4096.   */
/* With d the minimum-image displacement to j, j is visible when d = 0 or   */
/* 4096 (d . h) >= c |d| |h|, decided exactly on squares in 128-bit         */
/* integers.  Fewer than k visible particles is an error (ORC_E_RANGE).     */
/* ------------------------------------------------------------------------ */
int orc_fov_visible(int64_t dx, int64_t dy, int64_t hx, int64_t hy, int32_t c) {
  if (dx == 0 && dy == 0) return 1;
  int64_t p = 4096 * (dx * hx + dy * hy);                /* |p| < 2^45 */
  unsigned __int128 p2 = (unsigned __int128)(p < 0 ? -p : p) * (unsigned __int128)(p < 0 ? -p : p);
  unsigned __int128 q2 = (unsigned __int128)(uint64_t)(dx * dx + dy * dy) *
                         (unsigned __int128)(uint64_t)(hx * hx + hy * hy) *
                         (unsigned __int128)(uint64_t)((int64_t)c * c);
  if (c >= 0) return p >= 0 && p2 >= q2;
  return p >= 0 || p2 <= q2;
}

int orc_knn_fov(const int32_t* x, const int32_t* y, const float* theta, int32_t n, int32_t box,
                int32_t k, int32_t c, const int32_t* rows, int32_t nrows, int32_t* nbr) {
  if (n < 2 || box < 1 || k < 1 || k > n - 1 || c < -4096 || c > 4096) return ORC_E_INVAL;
  if (check_coords(x, y, n, box) != ORC_OK) return ORC_E_RANGE;
  int32_t count = rows ? nrows : n;
  if (rows)
    for (int32_t r = 0; r < nrows; ++r)
      if (rows[r] < 0 || rows[r] >= n) return ORC_E_INVAL;
  int failed = 0, short_rows = 0;
#pragma omp parallel
  {
    cand_t* best = (cand_t*)malloc(sizeof(cand_t) * (size_t)k);
    if (!best) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int32_t r = 0; r < count; ++r) {
      if (!best) continue;
      int32_t i = rows ? rows[r] : r;
      int64_t hx = (int64_t)rint(4096.0 * cos((double)theta[i]));
      int64_t hy = (int64_t)rint(4096.0 * sin((double)theta[i]));
      int32_t have = 0;
      for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        int64_t dx = min_image((int64_t)x[j] - x[i], box), dy = min_image((int64_t)y[j] - y[i], box);
        if (!orc_fov_visible(dx, dy, hx, hy, c)) continue;
        cand_t cd = {dx * dx + dy * dy, j};
        if (have == k && !cand_less(cd, best[k - 1])) continue;
        int32_t pos = (have < k) ? have++ : k - 1;
        while (pos > 0 && cand_less(cd, best[pos - 1])) {
          best[pos] = best[pos - 1];
          --pos;
        }
        best[pos] = cd;
      }
      if (have < k) {
#pragma omp atomic write
        short_rows = 1;
      }
      for (int32_t t = 0; t < k; ++t) nbr[(int64_t)r * k + t] = t < have ? best[t].j : -1;
    }
    free(best);
  }
  if (failed) return ORC_E_NOMEM;
  return short_rows ? ORC_E_RANGE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Metric rule: all j != i with d^2(i, j) <= rc2, ascending by (d^2, j).    */
/* Pass 1 (orc_metric_count) writes the row lengths; the caller forms the   */
/* CSR offsets (exclusive prefix sum); pass 2 (orc_metric_fill) fills rows. */
/* ------------------------------------------------------------------------ */
int orc_metric_count(const int32_t* x, const int32_t* y, int32_t n, int32_t box,
                     int64_t rc2, const int32_t* rows, int32_t nrows, int64_t* counts) {
  if (n < 1 || box < 1 || rc2 < 0) return ORC_E_INVAL;
  if (check_coords(x, y, n, box) != ORC_OK) return ORC_E_RANGE;
  int32_t count = rows ? nrows : n;
  if (rows)
    for (int32_t r = 0; r < nrows; ++r)
      if (rows[r] < 0 || rows[r] >= n) return ORC_E_INVAL;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t r = 0; r < count; ++r) {
    int32_t i = rows ? rows[r] : r;
    int64_t m = 0;
    for (int32_t j = 0; j < n; ++j)
      if (j != i && orc_d2(x[i], y[i], x[j], y[j], box) <= rc2) ++m;
    counts[r] = m;
  }
  return ORC_OK;
}

int orc_metric_fill(const int32_t* x, const int32_t* y, int32_t n, int32_t box,
                    int64_t rc2, const int32_t* rows, int32_t nrows,
                    const int64_t* offsets, int32_t* idx, int64_t* d2) {
  if (n < 1 || box < 1 || rc2 < 0) return ORC_E_INVAL;
  if (check_coords(x, y, n, box) != ORC_OK) return ORC_E_RANGE;
  int32_t count = rows ? nrows : n;
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t r = 0; r < count; ++r) {
    int32_t i = rows ? rows[r] : r;
    int64_t m = offsets[r + 1] - offsets[r];
    cand_t* row = (cand_t*)malloc(sizeof(cand_t) * (size_t)(m > 0 ? m : 1));
    if (!row) {
#pragma omp atomic write
      failed = 1;
      continue;
    }
    int64_t have = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      int64_t dd = orc_d2(x[i], y[i], x[j], y[j], box);
      if (dd <= rc2 && have < m) {
        row[have].d2 = dd;
        row[have].j = j;
        ++have;
      }
    }
    qsort(row, (size_t)have, sizeof(cand_t), cand_cmp);
    for (int64_t t = 0; t < have; ++t) {
      idx[offsets[r] + t] = row[t].j;
      if (d2) d2[offsets[r] + t] = row[t].d2;
    }
    free(row);
  }
  return failed ? ORC_E_NOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One Vicsek step for the listed particles, Eq. (2) then Eq. (1):          */
/*   theta'_i = arg( eta * xi_i + (1/m_i) * sum_j n_j ),  n_j = (cos, sin)  */
/*   r'_i     = r_i + rint(v0 * n_i(t))  (mod L)                            */
/* The neighbour list of output row r is either nbr[r*k .. r*k+k) (fixed k, */
/* offsets == NULL) or idx[offsets[r] .. offsets[r+1]) (CSR).               */
/* Headings of neighbours are read from the full theta array (time t).      */
/* ------------------------------------------------------------------------ */
int orc_align_step(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                   int32_t box, const int32_t* nbr, const int64_t* offsets, int32_t k,
                   int32_t v0, float eta, uint64_t seed, uint32_t sys_id,
                   int32_t include_self, uint64_t step, const int32_t* rows,
                   int32_t nrows, int32_t* x_out, int32_t* y_out, float* theta_out,
                   uint32_t variant) {
  if (n < 1 || box < 1 || (variant & ~3u) != 0) return ORC_E_INVAL;
  if (!offsets && k < 0) return ORC_E_INVAL;
  if (check_coords(x, y, n, box) != ORC_OK) return ORC_E_RANGE;
  int32_t count = rows ? nrows : n;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int32_t r = 0; r < count; ++r) {
    int32_t i = rows ? rows[r] : r;
    int64_t begin = offsets ? offsets[r] : (int64_t)r * k;
    int64_t end = offsets ? offsets[r + 1] : (int64_t)r * k + k;

    /* Sum of neighbour unit vectors, fp64 from the fp32 headings. */
    double sx = 0.0, sy = 0.0;
    for (int64_t t = begin; t < end; ++t) {
      int32_t j = nbr[t];
      if (j == -1 && !offsets) { /* a fixed-k row padded after its last neighbour */
        end = t;
        break;
      }
      if (j < 0 || j >= n) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
      sx += cos((double)theta[j]);
      sy += sin((double)theta[j]);
    }
    double own_c = cos((double)theta[i]);
    double own_s = sin((double)theta[i]);
    if (include_self) {
      sx += own_c;
      sy += own_s;
    }
    int64_t m = (end - begin) + (include_self ? 1 : 0);
    double ax = 0.0, ay = 0.0;
    if (m > 0) {
      ax = sx / (double)m;
      ay = sy / (double)m;
    }

    double phi = orc_noise_angle(seed, sys_id, step, i);
    double e = (double)eta;
    float th_new = theta[i];
    if (variant & 1u) {
      /* Angular noise: the direction of the average (the old heading when
       * the average vanishes) turned by eta * phi, then brought back into
       * [-pi, pi) by whole turns. */
      double base = (ax == 0.0 && ay == 0.0) ? (double)theta[i] : atan2(ay, ax);
      double t = base + e * phi;
      double turn = 2.0 * M_PI;
      th_new = (float)(t - turn * floor((t + M_PI) / turn));
    } else {
      /* Vectorial noise: eta times a random unit vector xi_i. */
      double vx = ax + e * cos(phi);
      double vy = ay + e * sin(phi);
      /* Normalisation: only the direction matters; the zero vector keeps theta. */
      if (!(vx == 0.0 && vy == 0.0)) th_new = (float)atan2(vy, vx);
    }

    /* Euler move on the integer grid, with the heading at time t (Eq. 1) or,
     * in the variant, the new one. */
    double mc = own_c, ms = own_s;
    if (variant & 2u) {
      mc = cos((double)th_new);
      ms = sin((double)th_new);
    }
    int64_t dx = (int64_t)rint((double)v0 * mc);
    int64_t dy = (int64_t)rint((double)v0 * ms);
    int64_t nx = ((int64_t)x[i] + dx) % box;
    int64_t ny = ((int64_t)y[i] + dy) % box;
    if (nx < 0) nx += box;
    if (ny < 0) ny += box;

    x_out[r] = (int32_t)nx;
    y_out[r] = (int32_t)ny;
    theta_out[r] = th_new;
  }
  return bad ? ORC_E_INVAL : ORC_OK;
}

/* Polar order parameter: |sum_i (cos theta_i, sin theta_i)| / n, summed in
 * index order in fp64. */
double orc_polar_order(const float* theta, int32_t n) {
  if (n < 1) return -1.0;
  double c = 0.0, s = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    c += cos((double)theta[i]);
    s += sin((double)theta[i]);
  }
  return sqrt(c * c + s * s) / (double)n;
}

/* Number of OpenMP threads the oracle runs on (for reporting). */
int orc_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
