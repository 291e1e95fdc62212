/*
 * voronoi_oracle.c -- brute-force CPU reference for the Voronoi (Delaunay)
 * neighbour lists and the Voronoi-model forces of
 *   D. M. Sussman, "Non-metric interaction rules in models of active matter"
 *   (arXiv:2103.10239), Sec. III (neighbours = edges of a Delaunay
 *   triangulation), Sec. IV (empty circumcircles, the Voronoi dual, "do I need
 *   to recompute the Voronoi diagram?") and Sec. V (Eqs. 3 and 5-19).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; it shares no code, header, table or constant with the HIP
 * path.
 *
 * Neighbour relation (plain definition, Sec. IV).  The Voronoi cell of a
 * particle is the set of points nearer to it than to any other particle, and
 * the Delaunay triangulation is its dual: i and j are neighbours when their
 * cells share an edge.  Written out: i and j are neighbours iff the
 * perpendicular bisector of i and j holds a point strictly nearer to i (and
 * j) than to every other particle.  Where four or more particles are
 * co-circular (a square lattice) two cells may touch in a single point; that
 * pair is not a neighbour pair, so the relation is unique for every input
 * (it is the set of edges common to all Delaunay triangulations).
 *
 * Periodic box and coincident particles (readings):
 *   - positions are integers in [0, L), vectors are minimum images with each
 *     component in [-L/2, L/2), as for the other neighbour rules;
 *   - particles at the same position share one site: the diagram is that of
 *     the distinct positions, and a particle's neighbours are the other
 *     particles at its own site and every particle at each neighbouring site
 *     (the paper's rule assumes distinct points; two coincident particles
 *     have no bisector, and are each other's nearest possible neighbours);
 *   - the lists are defined when every Voronoi vertex lies strictly within
 *     L/8 of its site (then only minimum images can shape a cell, every
 *     Delaunay edge is shorter than L/4, and the minimum images of a
 *     triangle's three edges agree); otherwise the oracle reports E_RANGE.
 *
 * Row order: first the other particles at the particle's own site, by index;
 * then the neighbouring sites counter-clockwise by the direction of the
 * minimum-image vector from the particle, starting at the +x axis
 * (directions with dy > 0, or dy = 0 and dx > 0, come first; within a half
 * plane by the sign of the cross product), the particles of one site by
 * index.  Two neighbouring sites never share a direction, so the order is
 * exact and unique.
 *
 * The bisector test works on exact integers: for the bisector of 0 and d,
 * x(t) = d/2 + t (-d_y, d_x), every other particle q bounds t by the linear
 * inequality 2 t (d_perp . q) < |q|^2 - d . q, and the pair is a neighbour
 * pair iff the largest lower bound is below the smallest upper bound.  The
 * bounds are fractions of integers below 2^41, compared by 128-bit cross
 * multiplication.
 *
 * Forces (Sec. V) are fp64 on real-valued positions (integers for the
 * lists; the finite-difference checks move them by fractions of a unit).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_CAPACITY (-3)
#define ORC_E_NOMEM (-4)

typedef __int128 i128;

static int64_t vmin_image(int64_t delta, int64_t box) {
  if (2 * delta >= box) delta -= box;
  if (2 * delta < -box) delta += box;
  return delta;
}

/* A bound on the bisector parameter t: the fraction num / den, den > 0. */
typedef struct {
  int64_t num, den;
  int set;
} bound_t;

static int frac_lt(int64_t an, int64_t ad, int64_t bn, int64_t bd) {
  return (i128)an * bd < (i128)bn * ad;
}

/* Bisector of the origin and d against the points q[0..m) (vectors relative
 * to the particle; entry `skip` is d itself and is left out).  Returns 1 if
 * some point of the bisector is strictly nearer to 0 and d than to every q,
 * with the interval's ends (unset = unbounded) in *lo and *hi. */
static int bisector_open(int64_t dx, int64_t dy, const int64_t* qx, const int64_t* qy, int32_t m,
                         int32_t skip, bound_t* lo, bound_t* hi) {
  bound_t l = {0, 1, 0}, h = {0, 1, 0};
  for (int32_t s = 0; s < m; ++s) {
    if (s == skip || (qx[s] == dx && qy[s] == dy)) continue; /* d itself, or its site */
    if (qx[s] == 0 && qy[s] == 0) continue;                   /* the particle's own site */
    const int64_t num = qx[s] * qx[s] + qy[s] * qy[s] - (dx * qx[s] + dy * qy[s]);
    const int64_t den = 2 * (-dy * qx[s] + dx * qy[s]);
    if (den == 0) {
      if (num <= 0) return 0; /* q on the segment from 0 to d: the bisector is never nearer */
      continue;
    }
    if (den > 0) { /* t < num / den */
      if (!h.set || frac_lt(num, den, h.num, h.den)) h = (bound_t){num, den, 1};
    } else { /* t > num / den = (-num) / (-den) */
      if (!l.set || frac_lt(l.num, l.den, -num, -den)) l = (bound_t){-num, -den, 1};
    }
    if (l.set && h.set && !frac_lt(l.num, l.den, h.num, h.den)) return 0;
  }
  *lo = l;
  *hi = h;
  return 1;
}

/* |x(t)|^2 < r2 / 4 for the bisector point at t = b.num / b.den, exactly:
 * |x(t)|^2 = |d|^2 (1/4 + t^2), so 4|x|^2 < r2 <=> |d|^2 (den^2 + 4 num^2) < r2 den^2. */
static int vertex_within(int64_t dx, int64_t dy, bound_t b, int64_t r2) {
  const i128 d2 = (i128)dx * dx + (i128)dy * dy;
  const i128 den2 = (i128)b.den * b.den;
  const i128 lhs = d2 * (den2 + 4 * (i128)b.num * b.num);
  return lhs < (i128)r2 * den2;
}

static int half_plane(int64_t dx, int64_t dy) { return (dy > 0 || (dy == 0 && dx > 0)) ? 0 : 1; }

/* counter-clockwise from the +x axis */
static int ccw_before(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int ha = half_plane(ax, ay), hb = half_plane(bx, by);
  if (ha != hb) return ha < hb;
  return (i128)ax * by - (i128)ay * bx > 0;
}

/* The neighbours of particle i among the m points q (relative vectors, the
 * particle itself excluded; id[s] is the index of q[s]): appended
 * counter-clockwise to row[0..dmax), count in *deg.  r2 (> 0) is the squared
 * radius within which every cell vertex must lie, times 4 (i.e. the vertex
 * bound is sqrt(r2) / 2).  Returns ORC_OK, ORC_E_RANGE (a vertex outside the
 * bound, an unbounded cell, a coincident particle) or ORC_E_CAPACITY. */
static int cell_of(const int64_t* qx, const int64_t* qy, const int32_t* id, int32_t m, int64_t r2,
                   int32_t dmax, int32_t* row, int32_t* deg) {
  int64_t* rx = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)dmax);
  if (!rx) return ORC_E_NOMEM;
  int64_t* ry = rx + dmax;
  int32_t cnt = 0;
  int rc = ORC_OK;
  /* the other particles at the particle's own site, by index (candidates come
   * in ascending index) */
  int32_t own = 0;
  for (int32_t s = 0; s < m; ++s)
    if (qx[s] == 0 && qy[s] == 0) {
      if (own == dmax) {
        rc = ORC_E_CAPACITY;
        break;
      }
      row[own++] = id[s];
    }
  cnt = own;
  for (int32_t s = 0; s < m && rc == ORC_OK; ++s) {
    if (qx[s] == 0 && qy[s] == 0) continue;
    bound_t lo, hi;
    if (!bisector_open(qx[s], qy[s], qx, qy, m, s, &lo, &hi)) continue;
    if (!lo.set || !hi.set || !vertex_within(qx[s], qy[s], lo, r2) ||
        !vertex_within(qx[s], qy[s], hi, r2)) {
      rc = ORC_E_RANGE;
      break;
    }
    if (cnt == dmax) {
      rc = ORC_E_CAPACITY;
      break;
    }
    /* insertion into the counter-clockwise order (after the own site's
     * particles, and after the particles of the same site met before) */
    int32_t pos = cnt++;
    while (pos > own && ccw_before(qx[s], qy[s], rx[pos - 1], ry[pos - 1])) {
      row[pos] = row[pos - 1];
      rx[pos] = rx[pos - 1];
      ry[pos] = ry[pos - 1];
      --pos;
    }
    row[pos] = id[s];
    rx[pos] = qx[s];
    ry[pos] = qy[s];
  }
  free(rx);
  /* a bounded cell has at least three edges (with none, the cell is the whole
   * plane); sites count once however many particles they hold */
  int32_t sites = 0;
  for (int32_t u = own; u < cnt; ++u)
    if (u == own || rx[u] != rx[u - 1] || ry[u] != ry[u - 1]) ++sites;
  if (rc == ORC_OK && sites < 3) rc = ORC_E_RANGE;
  *deg = cnt;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Voronoi neighbour lists of the particles rows[0..nrows) (or of every     */
/* particle when rows == NULL), by the bisector test against all n - 1     */
/* other particles.  ring: int32[nrows * dmax], deg: int32[nrows].          */
/* ------------------------------------------------------------------------ */
int orc_voronoi(const int32_t* x, const int32_t* y, int32_t n, int32_t box, const int32_t* rows,
                int32_t nrows, int32_t dmax, int32_t* ring, int32_t* deg) {
  if (n < 3 || box < 8 || dmax < 1) return ORC_E_INVAL;
  for (int32_t i = 0; i < n; ++i)
    if (x[i] < 0 || x[i] >= box || y[i] < 0 || y[i] >= box) return ORC_E_RANGE;
  const int32_t count = rows ? nrows : n;
  const int64_t r2 = ((int64_t)box / 4) * ((int64_t)box / 4); /* vertices within L/8 */
  int status = ORC_OK;
#pragma omp parallel
  {
    int64_t* qx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* qy = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* id = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 4)
    for (int32_t r = 0; r < count; ++r) {
      if (!qx || !qy || !id) {
#pragma omp atomic write
        status = ORC_E_NOMEM;
        continue;
      }
      const int32_t i = rows ? rows[r] : r;
      int32_t m = 0;
      for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        qx[m] = vmin_image((int64_t)x[j] - x[i], box);
        qy[m] = vmin_image((int64_t)y[j] - y[i], box);
        id[m++] = j;
      }
      const int rc = cell_of(qx, qy, id, m, r2, dmax, ring + (int64_t)r * dmax, deg + r);
      if (rc != ORC_OK) {
#pragma omp critical
        if (status == ORC_OK || rc == ORC_E_RANGE) status = rc;
      }
    }
    free(qx);
    free(qy);
    free(id);
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* The same lists for sampled rows of a large system.  Only particles within */
/* a radius rho of the particle take part in the bisector test; a particle   */
/* q farther than twice a vertex's distance from the particle is nearer to   */
/* the particle than to q at that vertex (triangle inequality), so once     */
/* every vertex lies within rho / 2 the farther particles cannot change the */
/* cell.  rho starts at rho0 and doubles until that holds (up to L/4, the   */
/* bound of the lists' domain).  A coincident particle anywhere in the      */
/* system is not looked for (only within rho).                              */
/* ------------------------------------------------------------------------ */
int orc_voronoi_local(const int32_t* x, const int32_t* y, int32_t n, int32_t box, const int32_t* rows,
                      int32_t nrows, int32_t rho0, int32_t dmax, int32_t* ring, int32_t* deg) {
  if (n < 3 || box < 8 || dmax < 1 || rows == NULL || rho0 < 1) return ORC_E_INVAL;
  for (int32_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= n) return ORC_E_INVAL;
  for (int32_t i = 0; i < n; ++i)
    if (x[i] < 0 || x[i] >= box || y[i] < 0 || y[i] >= box) return ORC_E_RANGE;
  int status = ORC_OK;
#pragma omp parallel
  {
    int64_t* qx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* qy = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* id = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
    for (int32_t r = 0; r < nrows; ++r) {
      if (!qx || !qy || !id) {
#pragma omp atomic write
        status = ORC_E_NOMEM;
        continue;
      }
      const int32_t i = rows[r];
      int rc = ORC_E_RANGE;
      for (int64_t rho = rho0;; rho *= 2) {
        if (rho > box / 4) rho = box / 4;
        int32_t m = 0;
        for (int32_t j = 0; j < n; ++j) {
          if (j == i) continue;
          const int64_t dx = vmin_image((int64_t)x[j] - x[i], box);
          const int64_t dy = vmin_image((int64_t)y[j] - y[i], box);
          if (dx * dx + dy * dy > rho * rho) continue;
          qx[m] = dx;
          qy[m] = dy;
          id[m++] = j;
        }
        rc = cell_of(qx, qy, id, m, rho * rho, dmax, ring + (int64_t)r * dmax, deg + r);
        if (rc != ORC_E_RANGE || rho >= box / 4) break;
      }
      if (rc != ORC_OK) {
#pragma omp critical
        if (status == ORC_OK || rc == ORC_E_RANGE) status = rc;
      }
    }
    free(qx);
    free(qy);
    free(id);
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* Voronoi model (Sec. V): cell areas and perimeters, the energy of Eq. (3),
 * the vertex forces of Eqs. (5)-(8) and the particle forces of Eqs. (9)-(19).
 *
 * Input: real positions x, y (fp64, periodic box L) and the Voronoi rings of
 * every particle as CSR (offsets int64[n + 1], idx), counter-clockwise.
 * Vertex t of cell i is the circumcentre h_t of the triangle
 * (i, a_t, a_{t+1}) of consecutive ring neighbours (Sec. IV: Voronoi
 * vertices are the circumcentres of the Delaunay triangles).
 *
 * Readings of Sec. V where the printed formulas disagree with the quantities
 * they define (the forces are the gradient of Eq. (3) either way; finite
 * differences of the energy decide):
 *   - Eq. (8): with t_ij = h_ijk - h_gij and t_ik = h_ikl - h_ijk, the
 *     derivative of the perimeter is t^_ij - t^_ik (the printed sign of the
 *     second term is flipped);
 *   - Eqs. (15) and (19): c is the cross product r_ij x r_jk (Eq. 19 holds
 *     for this c; Eq. 15 prints r_kj, which flips c's sign and leaves d = 2c^2
 *     unchanged);
 *   - Eq. (18): the second term is -|r_ij|^2 r_jk (the derivative of
 *     r_ik . r_jk with respect to r_i is -r_jk).
 * Vectors r_ab point from a to b (minimum image).  The circumcentre relative
 * to i is z / d with z = (beta d) r_ij + (gamma d) r_ik (Eqs. 15-16).
 *
 * Outputs (each may be NULL): area[n], perim[n], fx[n], fy[n] (force on each
 * particle, Eq. 9), energy (Eq. 3, one double); per ring slot s of cell i
 * (slot of a_t): hx[s], hy[s] = h_t relative to particle i, and vfx[s],
 * vfy[s] = the force -dE/dh_t on that vertex (Eq. 5).
 * ------------------------------------------------------------------------ */
typedef struct {
  double x, y;
} v2;

static v2 vsub(v2 a, v2 b) { return (v2){a.x - b.x, a.y - b.y}; }
static v2 vadd(v2 a, v2 b) { return (v2){a.x + b.x, a.y + b.y}; }
static v2 vscale(v2 a, double s) { return (v2){a.x * s, a.y * s}; }
static double vdot(v2 a, v2 b) { return a.x * b.x + a.y * b.y; }
static double vcross(v2 a, v2 b) { return a.x * b.y - a.y * b.x; }
static double vnorm(v2 a) { return sqrt(vdot(a, a)); }

static double fmin_image(double delta, double box) {
  if (2.0 * delta >= box) delta -= box;
  if (2.0 * delta < -box) delta += box;
  return delta;
}

/* Circumcentre of (i, j, k) relative to i, from r_ij and r_ik (Eqs. 15-16). */
static v2 circumcentre(v2 rij, v2 rik) {
  const v2 rjk = vsub(rik, rij);
  const double c = vcross(rij, rjk);
  const double d = 2.0 * c * c;
  const double bd = -vdot(rik, rik) * vdot(rij, rjk);
  const double gd = vdot(rij, rij) * vdot(rik, rjk);
  const v2 z = vadd(vscale(rij, bd), vscale(rik, gd));
  return vscale(z, 1.0 / d);
}

/* dh/dr_i of the circumcentre of (i, j, k) (Eqs. 16-19): J[nu][lambda] =
 * d h_nu / d r_i,lambda. */
static void circumcentre_jacobian(v2 rij, v2 rik, double J[2][2]) {
  const v2 rjk = vsub(rik, rij);
  const double c = vcross(rij, rjk);
  const double d = 2.0 * c * c;
  const double bd = -vdot(rik, rik) * vdot(rij, rjk);
  const double gd = vdot(rij, rij) * vdot(rik, rjk);
  const v2 z = vadd(vscale(rij, bd), vscale(rik, gd));
  /* Eq. 17 */
  const v2 dbd = vadd(vscale(rik, 2.0 * vdot(rij, rjk)), vscale(rjk, vdot(rik, rik)));
  /* Eq. 18 (reading: -|r_ij|^2 r_jk) */
  const v2 dgd = vsub(vscale(rij, -2.0 * vdot(rik, rjk)), vscale(rjk, vdot(rij, rij)));
  /* Eq. 19: (1/d) dd/dr_i = (2/c) (-r_jk,y, r_jk,x) */
  const v2 dd = vscale((v2){-rjk.y, rjk.x}, 2.0 / c);
  const double a[2] = {rij.x, rij.y}, b[2] = {rik.x, rik.y}, zz[2] = {z.x, z.y};
  const double gb[2] = {dbd.x, dbd.y}, gg[2] = {dgd.x, dgd.y}, gdd[2] = {dd.x, dd.y};
  for (int nu = 0; nu < 2; ++nu)
    for (int la = 0; la < 2; ++la) {
      const double delta = nu == la ? 1.0 : 0.0;
      const double inner = a[nu] * gb[la] + b[nu] * gg[la] - (bd + gd) * delta - zz[nu] * gdd[la];
      J[nu][la] = delta + inner / d;
    }
}

/* Eqs. (6)-(8): dE_c/dh for the vertex h of cell c with its counter-clockwise
 * predecessor hp and successor hn, the cell's area A and perimeter P. */
static v2 cell_vertex_grad(v2 hp, v2 h, v2 hn, double A, double P, double ka, double kp, double a0,
                           double p0) {
  const v2 tij = vsub(h, hp); /* t_ij = h_ijk - h_gij */
  const v2 tik = vsub(hn, h); /* t_ik = h_ikl - h_ijk */
  const double lij = vnorm(tij), lik = vnorm(tik);
  /* l n^ of each edge: the edge vector turned by -90 degrees (outward for a
   * counter-clockwise cell) */
  const v2 ln_ij = (v2){tij.y, -tij.x};
  const v2 ln_ik = (v2){tik.y, -tik.x};
  const v2 dA = vscale(vadd(ln_ij, ln_ik), 0.5);                        /* Eq. 7 */
  const v2 dP = vsub(vscale(tij, 1.0 / lij), vscale(tik, 1.0 / lik));  /* Eq. 8 (reading) */
  return vadd(vscale(dA, 2.0 * ka * (A - a0)), vscale(dP, 2.0 * kp * (P - p0))); /* Eq. 6 */
}

static int64_t ring_pos(const int64_t* off, const int32_t* idx, int32_t c, int32_t who) {
  for (int64_t s = off[c]; s < off[c + 1]; ++s)
    if (idx[s] == who) return s;
  return -1;
}

int orc_voronoi_forces(const double* x, const double* y, int32_t n, double box, const int64_t* off,
                       const int32_t* idx, double ka, double kp, double a0, double p0, const int32_t* rows,
                       int32_t nrows, double* area, double* perim, double* fx, double* fy, double* energy,
                       double* hx, double* hy, double* vfx, double* vfy) {
  if (n < 3 || !(box > 0.0)) return ORC_E_INVAL;
  /* rows == NULL: every particle (every row must hold a cell).  Otherwise
   * only the forces of particles rows[0..nrows) (output index r), from the
   * rows given (a particle with fewer than three entries has no cell: its
   * area and perimeter are NaN, and so is any force that needs them). */
  if (!rows)
    for (int32_t i = 0; i < n; ++i)
      if (off[i + 1] - off[i] < 3) return ORC_E_INVAL;
  const int32_t count = rows ? nrows : n;
  const int64_t nnz = off[n];
  double* A = (double*)malloc(sizeof(double) * (size_t)n);
  double* P = (double*)malloc(sizeof(double) * (size_t)n);
  v2* H = (v2*)malloc(sizeof(v2) * (size_t)nnz); /* h_t of cell i at slot off[i] + t, relative to i */
  if (!A || !P || !H) {
    free(A);
    free(P);
    free(H);
    return ORC_E_NOMEM;
  }
  int status = ORC_OK;
  /* pass 1: vertices, areas, perimeters */
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t b = off[i], m = off[i + 1] - off[i];
    double a2 = 0.0, per = 0.0;
    if (m < 3) {
      A[i] = P[i] = NAN;
      continue;
    }
    /* the model gives each particle its own cell: coincident particles have none */
    for (int64_t t = 0; t < m; ++t) {
      const int32_t j = idx[b + t];
      if (x[j] == x[i] && y[j] == y[i]) {
#pragma omp atomic write
        status = ORC_E_RANGE;
      }
    }
    for (int64_t t = 0; t < m; ++t) {
      const int32_t j = idx[b + t], k = idx[b + (t + 1) % m];
      const v2 rij = {fmin_image(x[j] - x[i], box), fmin_image(y[j] - y[i], box)};
      const v2 rik = {fmin_image(x[k] - x[i], box), fmin_image(y[k] - y[i], box)};
      H[b + t] = circumcentre(rij, rik);
    }
    for (int64_t t = 0; t < m; ++t) {
      const v2 h0 = H[b + t], h1 = H[b + (t + 1) % m];
      a2 += vcross(h0, h1);
      per += vnorm(vsub(h1, h0));
    }
    A[i] = 0.5 * a2;
    P[i] = per;
  }
  if (status != ORC_OK) { /* coincident particles: no model */
    free(A);
    free(P);
    free(H);
    return status;
  }
  /* pass 2: dE/dh of every vertex (three cells, Eq. 5) and the forces (Eq. 9) */
#pragma omp parallel for schedule(static)
  for (int32_t r = 0; r < count; ++r) {
    const int32_t i = rows ? rows[r] : r;
    const int64_t b = off[i], m = off[i + 1] - off[i];
    v2 F = {0.0, 0.0};
    for (int64_t t = 0; t < m; ++t) {
      const int32_t j = idx[b + t], k = idx[b + (t + 1) % m];
      const v2 rij = {fmin_image(x[j] - x[i], box), fmin_image(y[j] - y[i], box)};
      const v2 rik = {fmin_image(x[k] - x[i], box), fmin_image(y[k] - y[i], box)};
      const v2 h = H[b + t];
      const v2 hprev = H[b + (t + m - 1) % m];
      const v2 hnext = H[b + (t + 1) % m];
      /* the vertex across the edge between cells j and k: the circumcentre
       * of (j, mm, k), mm the neighbour of j just before k */
      const int64_t sk = ring_pos(off, idx, j, k);
      const int64_t mj = off[j + 1] - off[j];
      if (sk < 0 || mj < 3 || idx[off[j] + ((sk - off[j]) + 1) % mj] != i) {
#pragma omp atomic write
        status = ORC_E_INVAL; /* the rings are not one triangulation */
        continue;
      }
      const int32_t mm = idx[off[j] + ((sk - off[j]) + mj - 1) % mj];
      const v2 rjm = {fmin_image(x[mm] - x[j], box), fmin_image(y[mm] - y[j], box)};
      const v2 rjk = {fmin_image(x[k] - x[j], box), fmin_image(y[k] - y[j], box)};
      const v2 hacross = vadd(rij, circumcentre(rjm, rjk)); /* relative to i */
      v2 g = cell_vertex_grad(hprev, h, hnext, A[i], P[i], ka, kp, a0, p0);
      g = vadd(g, cell_vertex_grad(hacross, h, hprev, A[j], P[j], ka, kp, a0, p0));
      g = vadd(g, cell_vertex_grad(hnext, h, hacross, A[k], P[k], ka, kp, a0, p0));
      if (hx) hx[b + t] = h.x;
      if (hy) hy[b + t] = h.y;
      if (vfx) vfx[b + t] = -g.x;
      if (vfy) vfy[b + t] = -g.y;
      double J[2][2];
      circumcentre_jacobian(rij, rik, J);
      F.x -= g.x * J[0][0] + g.y * J[1][0];
      F.y -= g.x * J[0][1] + g.y * J[1][1];
    }
    if (fx) fx[r] = F.x;
    if (fy) fy[r] = F.y;
  }
  if (area) memcpy(area, A, sizeof(double) * (size_t)n);
  if (perim) memcpy(perim, P, sizeof(double) * (size_t)n);
  if (energy && !rows) {
    double e = 0.0;
    for (int32_t i = 0; i < n; ++i) e += ka * (A[i] - a0) * (A[i] - a0) + kp * (P[i] - p0) * (P[i] - p0);
    *energy = e;
  }
  free(A);
  free(P);
  free(H);
  return status;
}
