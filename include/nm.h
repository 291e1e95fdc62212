/*
 * nm.h -- C ABI of the MI355X (gfx950) library for non-metric neighbour
 * lists and the Vicsek alignment step.
 *
 * Method: D. M. Sussman, "Non-metric interaction rules in models of active
 * matter", arXiv:2103.10239.  One time step of the fundamental loop (Alg. 1)
 * rebuilds the neighbour lists and applies the interactions:
 *   - cell lists make neighbour finding O(N) and parallel (Sec. I);
 *   - topological neighbours: the k nearest of each particle (Sec. III);
 *   - metric neighbours: every particle within r_0 (Sec. III);
 *   - alignment with vectorial noise, Eq. (2), and the Euler move, Eq. (1).
 *
 * Conventions (readings of points the paper leaves open):
 *   - 2D periodic square box of side L; coordinates are int32 in [0, L);
 *     L is a power of two, 2 <= L <= 2^20; distances use the minimum image
 *     with each axis offset in [-L/2, L/2), squared distances are exact
 *     integers (int64).
 *   - Neighbours are ordered by the pair (d^2, j): ties at equal distance go
 *     to the smaller particle index.  A particle is never its own neighbour;
 *     coincident particles (d^2 = 0) are valid neighbours.
 *   - The metric rule is inclusive: d^2 <= rc2.
 *   - Eq. (2): theta'_i = arg(eta * xi_i + (1/m_i) sum_j n_j), where the sum
 *     runs over the list of i plus i itself when include_self = 1
 *     (m_i = |list| + include_self).  If the argument is exactly the zero
 *     vector, theta'_i = theta_i.  xi_i = (cos phi_i, sin phi_i) with
 *     phi_i = (u_i * 2^-32) * 2pi - pi (fp64, each operation rounded), and
 *     u_i is word (i mod 4) of Philox4x32-10 (Salmon et al., SC'11) at
 *     counter (i / 4, step mod 2^32, step >> 32, sys_id), key (seed mod 2^32,
 *     seed >> 32).
 *   - Eq. (1) with the heading at time t and dt = 1:
 *     x'_i = (x_i + rint(v0 cos theta_i)) mod L, likewise y with sin,
 *     rint rounding half to even, evaluated in fp64.
 *   - Headings are fp32; neighbour lists and positions are exact, headings
 *     agree with an fp64 evaluation of Eq. (2) to well within 1e-5 rad.
 *
 * Memory and ownership.  Every pointer argument named x, y, theta, nbr, d2,
 * offsets, idx, *_out or ws is a DEVICE pointer owned by the caller; nm_grid
 * and nm_params are HOST pointers read during the call only.  `stream` is a
 * hipStream_t (0 = the null stream).  Calls enqueue work on `stream` and
 * return without synchronising unless documented otherwise; they never
 * allocate device memory.  Host-detectable argument errors return NM_E_INVAL
 * before anything is enqueued.  Data-dependent errors found on the device
 * (a coordinate outside [0, L), an out-of-range neighbour index, a metric
 * list over capacity) are recorded in the workspace's error word and
 * reported by nm_check(); the affected outputs are then unspecified.  Calls
 * that share a workspace must be ordered on one stream; calls with distinct
 * workspaces are independent.
 */
#ifndef NM_H_
#define NM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every call (no exceptions cross the ABI). */
#define NM_OK 0
#define NM_E_INVAL (-1)    /* invalid argument (host) or index/grid mismatch (device) */
#define NM_E_RANGE (-2)    /* a coordinate outside [0, L) reached the device          */
#define NM_E_CAPACITY (-3) /* metric list longer than the caller's capacity           */
#define NM_E_NOMEM (-4)    /* served form: a job can never fit the memory budget      */
#define NM_E_DEVICE (-5)   /* HIP launch/runtime failure                              */

/* Largest k the topological search supports (register-resident lists). */
#define NM_MAX_K 32

/* Geometry of one system's cell grid (Sec. I: a grid of cells of width w). */
typedef struct nm_grid {
  int32_t n;      /* particles, 2 <= n <= 2^24                                     */
  int32_t box;    /* L, power of two in [2, 2^20]                                  */
  int32_t cell_w; /* w, power of two in [1, L]; (L/w)^2 <= 2^28 cells              */
  int32_t block;  /* k-NN fast-path block side in cells: 0 = chosen from n, L, w   */
                  /* and k; 3..15 = that side; -1 = exact ring search only.  With */
                  /* NM_BLOCK_SUBSTRIPS or-ed into 0 or a side, a strip of cells  */
                  /* whose halo overflows the on-chip staging buffer runs as      */
                  /* sub-strips staged in turn instead of searching global memory */
                  /* (faster on strongly clustered states, slower elsewhere: a    */
                  /* separate kernel).  The lists are identical for every choice; */
                  /* only speed differs.                                          */
} nm_grid;

#define NM_BLOCK_SUBSTRIPS 0x100

/* Variants of the step (nm_params.variant), from the Vicsek-model family the
 * paper's alignment rule belongs to (Sec. III); 0 is Eq. (2) and Eq. (1) as
 * written:
 *   NM_NOISE_SCALAR      angular noise instead of Eq. (2)'s random unit
 *                        vector: theta' = arg(A) + eta * phi, A the average of
 *                        the unit vectors (theta itself when A = 0), phi the
 *                        same Philox noise angle in [-pi, pi); the result is
 *                        wrapped into [-pi, pi)
 *   NM_MOVE_NEW_HEADING  Eq. (1) with the new heading n_i(t+1) instead of
 *                        n_i(t) */
#define NM_NOISE_SCALAR 1u
#define NM_MOVE_NEW_HEADING 2u

/* Parameters of Eq. (1) and Eq. (2). */
typedef struct nm_params {
  int32_t box;          /* L, same rules as nm_grid.box                            */
  int32_t v0;           /* displacement per step in grid units, |v0| < L/2         */
  float eta;            /* noise strength, finite and >= 0                         */
  int32_t include_self; /* 1: own heading joins the average, 0: it does not       */
  uint64_t seed;        /* Philox key                                              */
  uint32_t sys_id;      /* Philox counter word 3 (system identity)                 */
  uint32_t variant;     /* 0, or NM_NOISE_SCALAR and/or NM_MOVE_NEW_HEADING         */
} nm_params;

/* Human-readable name of a status code (static string). */
const char* nm_status_str(int status);

/* Bytes of device workspace a grid needs (cell table, sorted particle copy,
 * scan state, error word).  Returns < 0 (an NM_E_* code) if the grid is
 * invalid.  The workspace must be 256-byte aligned (hipMalloc/torch are). */
int64_t nm_workspace_bytes(const nm_grid* g);

/* A cell width for n particles in a box of side L: the power of two w that
 * puts about `per_cell` particles in a cell on average (uniform density).
 * Host-only helper; the batched/served forms refine it by measurement. */
int32_t nm_suggest_cell_w(int32_t n, int32_t box, double per_cell);

/* Prepare a freshly allocated workspace: zero the cell histogram and stamp
 * the header.  Call once per workspace (and again after reuse for another
 * grid).  Enqueued on `stream`. */
int nm_workspace_init(const nm_grid* g, void* ws, size_t ws_bytes, void* stream);

/* Cell binning (Sec. I, cell lists): counting sort of the particles by cell.
 *   x, y   int32[n]  positions at time t, each in [0, L)
 *   ws     workspace of nm_workspace_bytes(g) bytes, initialised
 * Writes the per-cell start table and a cell-ordered copy of the particles
 * into `ws`.  Particles with a coordinate outside [0, L) are left out and
 * flag NM_E_RANGE. */
int nm_build_cells(const nm_grid* g, const int32_t* x, const int32_t* y, void* ws,
                   size_t ws_bytes, void* stream);

/* Topological neighbour list (Sec. III, "the k nearest neighbours"), from
 * the cells built by nm_build_cells/nm_step on the same grid.
 *   k      1 <= k <= min(NM_MAX_K, n - 1)
 *   nbr    int32[n * k], row i = the k nearest neighbours of particle i,
 *          ascending by (d^2, j), indices in the caller's particle order
 *   d2     int64[n * k] or NULL: the matching squared distances */
int nm_knn(const nm_grid* g, const void* ws, int32_t k, int32_t* nbr, int64_t* d2,
           void* stream);

/* Host-only description of the strip kernel that nm_knn, nm_knn_align and
 * nm_step run for grid g and list length k (no device work; for tests and
 * tuning reports).  out: HOST int32[10] =
 *   [0] kernel: 0 = no staging (one row of queries per strip, searched in
 *       global memory), 1 = staged strips (default kernel), 2 = staged
 *       strips with the sub-strip kernel (NM_BLOCK_SUBSTRIPS)
 *   [1] strip width tw, [2] strip height th (cells)
 *   [3] halo columns hx, [4] halo rows hy (cells on each side)
 *   [5] fixed block side (0: chosen per query)
 *   [6] 1 if staged offsets are int32 pairs with 64-bit distances, 0 if
 *       packed 16-bit offsets
 *   [7] tallest block the halo supports (rows)
 *   [8] strips across, [9] strips down
 * The layout depends on n, box, cell_w, block and k only. */
int nm_knn_layout(const nm_grid* g, int32_t k, int32_t* out);

/* Metric neighbour list (Sec. III, "all pairs within r_0") as CSR rows in
 * the caller's particle order, each row ascending by (d^2, j).
 *   rc2      r_0^2 in grid units^2, 0 <= rc2 < 2^40
 *   offsets  int32[n + 1]: always written; offsets[n] = nnz
 *   idx      int32[cap] or NULL.  NULL: count pass only.  Otherwise rows are
 *            filled if nnz <= cap; if nnz > cap nothing is written to idx and
 *            NM_E_CAPACITY is recorded (and returned when nnz_host != NULL)
 *   nnz_host host int64* or NULL.  Non-NULL: the call synchronises `stream`
 *            and stores nnz there (the two-call protocol: count, allocate,
 *            fill).  NULL: no synchronisation.
 * nnz must stay below 2^31 (else NM_E_CAPACITY). */
int nm_metric_list(const nm_grid* g, void* ws, int64_t rc2, int32_t* offsets, int32_t* idx,
                   int64_t cap, int64_t* nnz_host, void* stream);

/* Alignment and move for every particle, Eq. (2) then Eq. (1), from time-t
 * state (Alg. 1: lists and headings at t give theta(t+1); positions at t
 * and headings at t give r(t+1)).
 *   x, y, theta     int32/int32/fp32 [n], time t
 *   nbr             fixed-k lists int32[n * k] (offsets == NULL), k >= 0, or
 *                   CSR column indices int32[nnz_cap] (offsets != NULL); a
 *                   fixed-k row may end early, padded with -1 after its last
 *                   neighbour (rows of varying length such as nm_voronoi's)
 *   offsets         int32[n + 1] CSR row starts, or NULL
 *   nnz_cap         length of the CSR index array (ignored for fixed k)
 *   x_out, y_out, theta_out  [n], time t+1; must not alias the inputs
 * Neighbour indices outside [0, n) or malformed CSR rows are skipped and
 * flag NM_E_INVAL in `ws_err` (a workspace, or NULL to skip reporting). */
int nm_align_step(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                  const int32_t* nbr, const int32_t* offsets, int32_t k, int64_t nnz_cap,
                  const nm_params* p, uint64_t step, int32_t* x_out, int32_t* y_out,
                  float* theta_out, void* ws_err, void* stream);

/* Field-of-view topological lists (the topological rule of Sec. III
 * restricted to a cone around each particle's heading): for every particle
 * the k nearest, by (d^2, index), among the particles it sees.  The heading
 * vector is h = (rint(4096 cos theta), rint(4096 sin theta)) in fp64 from
 * the fp32 heading, and the cone's half angle alpha is given by
 * cos alpha = cos_q / 4096 (-4096 <= cos_q <= 4096; -4096 sees everything,
 * 0 the half plane ahead).  With d the minimum-image displacement to j, j is
 * seen when d = 0 or 4096 (d . h) >= cos_q |d| |h|, decided exactly.
 *   ws     built by nm_build_cells or nm_bin_step for these positions
 *   theta  device fp32[n], headings in the caller's particle order
 *   nbr    device int32[n * k], row-major in the caller's order
 *   k      1 <= k <= min(NM_MAX_K, n - 1)
 * A particle that sees fewer than k others makes nm_check() report
 * NM_E_RANGE (its row is then unspecified).  g->block >= 0 runs the strip
 * kernel of nm_knn with the cone as a candidate filter; -1 one lane per
 * particle with the exact ring search.  The lists are the same. */
int nm_knn_fov(const nm_grid* g, const void* ws, int32_t k, const float* theta, int32_t cos_q,
               int32_t* nbr, void* stream);

/* ------------------------------------------------------------------------
 * Voronoi (Delaunay) neighbour lists: the topological rule of Sec. III in
 * which neighbours are the edges of a Delaunay triangulation, through its
 * dual, the Voronoi diagram (Sec. IV).  i and j are neighbours when their
 * Voronoi cells share an edge of positive length; where four or more
 * particles are co-circular (a square lattice) cells that touch in a single
 * point are not neighbours, so the lists are unique for every input and
 * reciprocal.  Particles at the same position share one site: the diagram
 * is that of the distinct positions, and a particle's neighbours are the
 * other particles of its own site and every particle of each neighbouring
 * site.  Positions as for the other rules (minimum images in the periodic
 * box).  The lists are defined when every site's cell lies within L/8 of
 * it; otherwise nm_check() reports NM_E_RANGE and the affected rows are
 * unspecified.
 *
 * Rows: ring int32[n * dmax], row i = the other particles at particle i's
 * position by index, then the neighbouring sites counter-clockwise by the
 * direction of the minimum-image offset, starting at the +x axis (offsets
 * with dy > 0, or dy = 0 and dx > 0, first), each site's particles by index;
 * padded with -1; deg int32[n] = the row lengths.  Consecutive sites a_t,
 * a_{t+1} of row i are the triangles (i, a_t, a_{t+1}) of the Delaunay
 * triangulation, whose circumcentres are the cell's vertices.  A row longer
 * than dmax records NM_E_CAPACITY (the row keeps its first dmax entries).
 * ------------------------------------------------------------------------ */
#define NM_VORONOI_MAX_DEG 64

/* Voronoi lists from the cells built in ws (nm_build_cells or nm_bin_step).
 *   dmax   3 <= dmax <= NM_VORONOI_MAX_DEG (16 holds any row of a uniform
 *          system with overwhelming probability)
 * The workspace's Voronoi list and counters are used as scratch (ws is not
 * const).  Enqueued on `stream`. */
int nm_voronoi(const nm_grid* g, void* ws, int32_t dmax, int32_t* ring, int32_t* deg, void* stream);

/* "Do I need to recompute the Voronoi diagram?" (Sec. IV), as a test of the
 * triangulation held in (ring, deg) -- rows built for earlier positions --
 * against the positions x, y (device int32[n], caller order): every
 * triangle of consecutive row entries must still turn counter-clockwise,
 * the three rows of each triangle must agree, every row must wind once
 * around its particle with offsets below L/4, and every edge must be
 * strictly locally Delaunay (the fourth particle strictly outside the
 * circumcircle).  If all hold, the rows are still exactly the Voronoi
 * lists of x, y, up to the start of each row.
 *   stale  device uint8[n], out: 1 for every particle whose own test failed
 *          and every particle of its row (the rows a flip may change)
 *   nfail  device int32 or NULL, out: how many particles failed; 0 means
 *          no recomputation is needed
 * ws (grid g, n particles) holds the counters only. */
int nm_voronoi_check(const nm_grid* g, void* ws, const int32_t* x, const int32_t* y, int32_t dmax,
                     const int32_t* ring, const int32_t* deg, uint8_t* stale, int32_t* nfail,
                     void* stream);

/* Bring rows built for earlier positions up to date for the positions
 * x, y, whose cells ws must hold (nm_build_cells / nm_bin_step with x, y):
 * twice, nm_voronoi_check, then the stale rows recomputed and the others
 * rotated to start at the +x axis again; then the check once more, and if
 * any row still fails, every row recomputed.  Afterwards (ring, deg) equal
 * what nm_voronoi gives for x, y.  nfail (device int32 or NULL) receives
 * the first check's count.  stale: device uint8[n] scratch. */
int nm_voronoi_update(const nm_grid* g, void* ws, const int32_t* x, const int32_t* y, int32_t dmax,
                      int32_t* ring, int32_t* deg, uint8_t* stale, int32_t* nfail, void* stream);

/* Voronoi model of dense tissue (Sec. V): each particle owns its Voronoi
 * cell and the energy is Eq. (3), E = sum_i K_A (A_i - A_0)^2 +
 * K_P (P_i - P_0)^2, in grid units (areas in units^2, lengths in units). */
typedef struct nm_vm_params {
  double ka, kp; /* area and perimeter moduli K_A, K_P                      */
  double a0, p0; /* preferred area A_0 and perimeter P_0                    */
} nm_vm_params;

/* Cell areas and perimeters, the force on every particle, -dE/dr_i (Eq. 9,
 * by the chain rule through the cell vertices, Eqs. 10-19), and optionally
 * the energy and the vertex forces -dE/dh (Eqs. 5-8), all fp64, from the
 * rows of nm_voronoi (ring int32[n * dmax], deg int32[n]) for positions
 * x, y (device int32[n] in [0, box)).  The printed formulas are read as the
 * gradient of Eq. (3): Eq. (8) dP/dh = t_ij/|t_ij| - t_ik/|t_ik|, c =
 * r_ij x r_jk in Eqs. (15) and (19), Eq. (18) ending in -|r_ij|^2 r_jk.
 *   area, perim, fx, fy  device double[n], out (area and perim required)
 *   energy               device double or NULL: Eq. (3), summed in a fixed order
 *   vertex               device double[n * dmax * 4] or NULL: for slot t of
 *                        row i, vertex t of cell i (the circumcentre of
 *                        (i, a_t, a_{t+1}), relative to particle i) and the
 *                        force -dE/dh on it: (hx, hy, fx, fy)
 *   ws_err               workspace whose error word receives NM_E_INVAL for
 *                        rows that are not one triangulation and NM_E_RANGE
 *                        for coincident particles (the model needs a cell per
 *                        particle), or NULL
 * box is L (power of two, 8 <= L <= 2^20). */
int nm_voronoi_forces(const int32_t* x, const int32_t* y, int32_t n, int32_t box, int32_t dmax,
                      const int32_t* ring, const int32_t* deg, const nm_vm_params* vp, double* area,
                      double* perim, double* fx, double* fy, double* energy, double* vertex,
                      void* ws_err, void* stream);

/* Polar order parameter of the headings (Sec. III: the ordered, flocking
 * phase is the one whose headings agree), into the caller's DEVICE
 * double[3]: sums[0] = sum_i cos theta_i, sums[1] = sum_i sin theta_i (fp64)
 * and sums[2] = |(sums[0], sums[1])| / n, the order parameter.  theta:
 * device fp32[n], n >= 1.  Enqueued on `stream` without synchronising; the
 * summation order varies between calls (the sums agree to fp64 rounding). */
int nm_polar_order(const float* theta, int32_t n, double* sums, void* stream);

/* One full step of the topological model (Alg. 1) = nm_bin_step followed by
 * nm_knn_align.  Same results as nm_build_cells + nm_knn + nm_align_step
 * with the same k and parameters: identical lists, positions and headings.
 * The cells left in `ws` describe the time-t positions and can feed
 * nm_metric_list / nm_knn afterwards.  p->box must equal g->box. */
int nm_step(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta,
            int32_t k, const nm_params* p, uint64_t step, void* ws, size_t ws_bytes,
            int32_t* nbr, int32_t* x_out, int32_t* y_out, float* theta_out, void* stream);

/* First stage of nm_step: the cell binning of nm_build_cells, which in the
 * same pass stores, beside each particle's cell-ordered copy, its Philox
 * noise word for `step` (Eq. 2) and the fp64 unit vector of its heading.
 *   theta  fp32[n], headings at time t */
int nm_bin_step(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta,
                const nm_params* p, uint64_t step, void* ws, size_t ws_bytes, void* stream);

/* Second stage of nm_step: the k-NN lists (as nm_knn) fused with Eq. (2) and
 * Eq. (1) for every particle, from cells written by nm_bin_step with the
 * same parameters.  `theta` is the time-t heading array given to nm_bin_step
 * (read only where the alignment vector is exactly zero).  Outputs as nm_step. */
int nm_knn_align(const nm_grid* g, const void* ws, int32_t k, const nm_params* p,
                 const float* theta, int32_t* nbr, int32_t* x_out, int32_t* y_out,
                 float* theta_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): nm_step
 * with the workspace in a file-scope device array of the library instead of
 * a caller buffer.  Same arguments and results as nm_step without ws and
 * ws_bytes; the grid's nm_workspace_bytes must not exceed
 * NM_STEP_NOALLOC_MAX_BYTES (32 MiB, about 3e5 particles at one per cell),
 * else NM_E_NOMEM before anything is enqueued.  Device-side errors (a
 * coordinate outside [0, L)) are written to *err (device int32, NM_OK or the
 * first error of this call; err may be NULL) on `stream`, without
 * synchronising.  The array is looked up once per device with that device
 * current (call with the stream's device current); each device holds its own
 * copy until the process ends.  Every call on a device shares that array and
 * re-initialises it: calls that overlap on one device (concurrent streams or
 * host threads) race and must be serialised by the caller.  Calls no
 * hipMalloc, hipFree or allocating library routine. */
#define NM_STEP_NOALLOC_MAX_BYTES (32ll << 20)
int nm_step_noalloc(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta, int32_t k,
                    const nm_params* p, uint64_t step, int32_t* nbr, int32_t* x_out, int32_t* y_out,
                    float* theta_out, int32_t* err, void* stream);

/* Synchronise `stream`, return the first error recorded in `ws` since the
 * last check (NM_OK if none) and clear it. */
int nm_check(void* ws, void* stream);

/* Autotuner of the one-system step: for each of the ncand candidate grids
 * (same n and box; cell width and block may differ) time `reps` steps of
 * nm_bin_step + nm_knn_align on the given state (after one untimed step) and
 * store the index of the fastest in *best and, if ms_out != NULL, the mean
 * milliseconds per step of each candidate in ms_out[ncand].  `ws` must hold
 * nm_workspace_bytes of every candidate; it is left initialised for the
 * chosen grid.  The outputs are scratch (they receive tuning steps).
 * Synchronises `stream`. */
int nm_tune_grid(const nm_grid* cand, int32_t ncand, const int32_t* x, const int32_t* y,
                 const float* theta, int32_t k, const nm_params* p, uint64_t step, void* ws,
                 size_t ws_bytes, int32_t* nbr, int32_t* x_out, int32_t* y_out, float* theta_out,
                 int32_t reps, int32_t* best, float* ms_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent systems of uneven size, all advanced by
 * the step of nm_step (Alg. 1 with the k-NN rule, Eq. (2), Eq. (1)), one
 * persistent launch per stage for the whole batch, the step replayable from
 * a HIP graph.  Every system's lists, positions and headings are identical
 * to those of nm_step on that system alone with the same parameters, the
 * system's own sys_id and its own step count (the Philox stream is keyed by
 * system, never by its place in the batch).
 *
 * State lives in caller-owned concatenated arrays: system s owns particles
 * [offset_s, offset_s + n_s) (offsets are the prefix sums of n in system
 * order) and list rows [offset_s * k, (offset_s + n_s) * k) of nbr.  The
 * state is double-buffered: after a total of t steps since nm_batch_bind the
 * current positions and headings are in buffer t mod 2.
 * ------------------------------------------------------------------------ */
#define NM_BATCH_MAX_SYS 65536

typedef struct nm_batch nm_batch; /* host-side plan (opaque) */

typedef struct nm_batch_io {
  int32_t* x[2];     /* device, int32[total]: positions, buffers 0 and 1       */
  int32_t* y[2];
  float* theta[2];   /* device, fp32[total]: headings, buffers 0 and 1         */
  int32_t* nbr;      /* device, int32[total * k]: the lists of the last step   */
} nm_batch_io;

/* Plan a batch: nsys systems with n[s] particles each (host array,
 * k + 1 <= n[s] <= 2^24, total < 2^31) in boxes of side `box`, k nearest
 * neighbours, step parameters p (p->box == box; p->sys_id is ignored) and
 * per-system Philox identities sys_ids (host array, or NULL for 0..nsys-1).
 * Returns the host plan in *out and the device workspace size in *ws_bytes.
 * Allocates host memory only; free the plan with nm_batch_destroy. */
int nm_batch_plan(int32_t nsys, const int32_t* n, int32_t box, int32_t k, const nm_params* p,
                  const uint32_t* sys_ids, nm_batch** out, int64_t* ws_bytes);

/* Attach device memory and state buffers to a plan: `ws` (256-byte aligned,
 * at least *ws_bytes bytes) holds the per-system descriptors, the work-item
 * tables and every system's workspace; io names the state arrays (buffer 0
 * holds the initial state).  The next step of every system is `step0`.
 * Uploads the tables and initialises the workspaces on `stream`, then
 * synchronises it.  Rebinding resets the step count. */
int nm_batch_bind(nm_batch* b, void* ws, size_t ws_bytes, const nm_batch_io* io, uint64_t step0,
                  void* stream);

/* Advance every system by nsteps steps.  use_graph = 1: the first call
 * captures one step into a HIP graph (on a private stream) and every step is
 * a launch of that graph on `stream`; 0: the stage kernels are launched
 * directly.  Enqueues only; does not synchronise or allocate device memory. */
int nm_batch_step(nm_batch* b, int32_t nsteps, int32_t use_graph, void* stream);

/* Autotuner: for each size class (systems with equal floor(log2 n)), time
 * `reps` steps of the class alone under each candidate cell width (about
 * 0.5, 1, 2 and 4 particles per cell, blocks chosen per query) and keep the
 * fastest; then, at that width, the k-NN block choice (per query, fixed
 * sides 4 and 6, or the sub-strip kernel: nm_grid.block), which also sets
 * the strip shape.  The tuning steps read the current state and write only
 * the other buffer and nbr, and do not advance the step count.  The lists
 * are the same for every choice.  Synchronises; drops the captured graph. */
int nm_batch_tune(nm_batch* b, int32_t reps, void* stream);

/* Sets every system's k-NN block choice (nm_grid.block: 0, a side 3..15,
 * -1, optionally with NM_BLOCK_SUBSTRIPS), keeping the tuned cell widths:
 * for callers that know their workload.  The lists are the same for every
 * choice.  NM_E_INVAL for a value nm_grid does not accept.  Synchronises;
 * drops the captured graph. */
int nm_batch_set_block(nm_batch* b, int32_t block, void* stream);

/* The grid chosen for system s (cell width, block) and its particle offset. */
int nm_batch_system(const nm_batch* b, int32_t s, nm_grid* g, int32_t* offset);

/* Steps taken since nm_batch_bind (the current state is in buffer
 * nm_batch_steps_done(b) mod 2). */
int64_t nm_batch_steps_done(const nm_batch* b);

/* Synchronise `stream` and return the first error recorded by any system
 * since the last check (then cleared), NM_OK if none. */
int nm_batch_check(nm_batch* b, void* stream);

void nm_batch_destroy(nm_batch* b);

/* ------------------------------------------------------------------------
 * Served form: a request loop over jobs of different sizes.  Each job is a
 * system (n particles, k nearest neighbours, nsteps steps of nm_step from its
 * initial state, its own Philox seed and sys_id, step counter from 0).  The
 * server keeps admitted jobs' state on the device and advances all of them
 * together, one step per engine iteration (continuous batching: jobs that
 * arrive while others run join at the next iteration, finished jobs leave).
 * Admission is FIFO under a byte budget of device memory counted per job as
 * nm_server_job_bytes (workspace, double-buffered state, list).  A job's
 * results equal those of nm_step on that job alone: lists and positions
 * bit-exact, headings bit-exact as well (same kernels and arithmetic).
 * The server runs two host threads of its own and two HIP streams on the
 * device current at nm_server_create; it allocates device memory in slabs
 * (1 GiB or one job) that it keeps until destroyed.
 * ------------------------------------------------------------------------ */
typedef struct nm_server nm_server; /* opaque */

typedef struct nm_job {
  int32_t n;          /* particles, k + 1 <= n <= 2^24                          */
  int32_t k;          /* 1 <= k <= NM_MAX_K                                     */
  int32_t nsteps;     /* >= 1                                                   */
  int32_t want_nbr;   /* 1: keep the lists of the last step for nm_server_wait */
  nm_params p;        /* Eq. (1)-(2) parameters, box, seed, sys_id              */
  const int32_t* x;   /* HOST int32[n], initial positions in [0, box)           */
  const int32_t* y;
  const float* theta; /* HOST fp32[n], initial headings                         */
} nm_job;

typedef struct nm_job_result {
  int32_t status;     /* NM_OK or the first error of the job                    */
  int32_t steps;      /* steps taken                                            */
  double submit_s;    /* seconds since nm_server_create: submitted,             */
  double admit_s;     /*   admitted to the device,                              */
  double done_s;      /*   final state copied back to the host                  */
} nm_job_result;

typedef struct nm_server_info {
  int64_t submitted, completed, iterations;
  int64_t budget_bytes, used_bytes, peak_used_bytes; /* ledger                  */
  int64_t reserved_bytes;                            /* device slabs held       */
  int32_t active, peak_active, queued, status;       /* status: engine errors   */
  double now_s;
} nm_server_info;

/* Ledger bytes of a job (its admission cost), or < 0 if invalid. */
int64_t nm_server_job_bytes(int32_t n, int32_t k, int32_t box);

/* Start a server with a device-memory budget and at most max_slots jobs on
 * the device at once. */
int nm_server_create(int64_t budget_bytes, int32_t max_slots, nm_server** out);

/* Queue a job (its host inputs are copied before returning).  NM_E_NOMEM if
 * the job alone exceeds the budget; *id names it for poll/wait. */
int nm_server_submit(nm_server* s, const nm_job* job, int64_t* id);

/* 1 if job id has finished, 0 if not yet, NM_E_INVAL if unknown. */
int nm_server_poll(nm_server* s, int64_t id);

/* Block until job id finishes, copy its final state (and lists) into the
 * HOST arrays given (each may be NULL), fill *r (may be NULL) and forget the
 * job.  Returns the job's status. */
int nm_server_wait(nm_server* s, int64_t id, int32_t* x, int32_t* y, float* theta, int32_t* nbr,
                   nm_job_result* r);

/* Counters and ledger of the server (a snapshot). */
int nm_server_stats(nm_server* s, nm_server_info* out);

/* Finish every queued and running job, then stop the threads and release
 * the device memory.  Results not collected are dropped. */
void nm_server_destroy(nm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* NM_H_ */
