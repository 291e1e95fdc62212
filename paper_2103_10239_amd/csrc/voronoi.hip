// voronoi.hip -- Voronoi (Delaunay) neighbour lists: the topological rule of
// Sec. III in which neighbours are the edges of a Delaunay triangulation,
// built through its dual, the Voronoi diagram (Sec. IV), plus the test of
// Sec. IV that asks whether the diagram must be recomputed after a move,
// posed as an empty-circumcircle test of the old triangulation.
//
// Every particle's Voronoi cell is built on its own, so the work is
// embarrassingly parallel (the global consistency that Sec. IV warns serial
// algorithms about follows from the exactness of each cell): one lane per
// particle, particles taken in cell order so that a wavefront's lanes read
// the same cells.  The lane starts from a square around its particle and
// clips it by the bisector of every candidate found on rings of cells around
// the home cell.  A candidate farther than twice the farthest cell vertex
// cannot cut the cell, so the walk stops after the first ring whose outer
// bound certifies that; candidates inside the rings but that far are skipped
// without a test.
//
// Exactness.  All predicates are exact integers on minimum-image offsets
// from the particle:
//   - vertex t of the cell is the circumcentre of (0, g_t, g_{t+1}) for
//     consecutive clipping particles g (counter-clockwise);
//   - candidate c removes that vertex when it lies strictly inside the circle
//     through 0, g_t and g_{t+1}: D(g_t, g_{t+1}, c) < 0 with
//     D(a, b, c) = |a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b);
//   - removed vertices form one cyclic run; the candidate's edge replaces
//     the clipping particles strictly between them.
// Distances to vertices (for the stop test and the skip) are only compared
// with margins that absorb their rounding.  At the end, a clipping particle
// whose edge has shrunk to a point (D(g_{t-1}, g_t, g_{t+1}) = 0: four
// co-circular particles) is dropped: its cell touches this one in a vertex
// only, so it is not a neighbour.  The row then lists the remaining ones
// counter-clockwise from the +x axis.
//
// Two kernels.  The narrow one keeps offsets below 2^14 (16-bit pairs in
// LDS, D in 64-bit integers) and a cell of at most 16 edges at any time;
// cells it cannot finish within that range (sparse regions, long clipping
// histories) are listed for the wide one (32-bit offsets, D in 128-bit
// integers, 64 edges, rings out to the box).  Rows whose cell reaches L/8
// or more from its particle are outside the lists' domain: NM_E_RANGE.
//
// Coincident particles share one site (the diagram is that of the distinct
// positions): a candidate at the particle's own position is skipped, and a
// candidate at the position of a clipping particle never cuts (it lies on
// that particle's bisector).  The row then lists the other particles of the
// own site, then every particle of each neighbouring site, by index within
// a site (found in the site's grid cell).
#include "nm_internal.h"

namespace nm {

namespace {

constexpr int kVnBlock = 256;  // lanes per workgroup, narrow kernel
constexpr int kVnCap = 16;     // cell edges, narrow kernel (power of two)
constexpr int kVnSpan = 1 << 14;
constexpr int kVwBlock = 64;   // lanes per workgroup, wide kernel
constexpr int kVwCap = 64;     // cell edges, wide kernel (power of two)
constexpr int kVwGrid = 512;   // workgroups of the wide kernel

// ---------------------------------------------------------------------------
// exact predicates
// ---------------------------------------------------------------------------
// Sign of D(a, b, c) with |coordinates| <= 2^14: every product below 2^58.
__device__ __forceinline__ int inc_sign_n(int ax, int ay, int bx, int by, int cx, int cy) {
  const int na = ax * ax + ay * ay, nb = bx * bx + by * by, nc = cx * cx + cy * cy;
  const int bc = bx * cy - by * cx, ca = cx * ay - cy * ax, ab = ax * by - ay * bx;
  const long long d = static_cast<long long>(na) * bc + static_cast<long long>(nb) * ca +
                      static_cast<long long>(nc) * ab;
  return (d > 0) - (d < 0);
}

// Sign of D(a, b, c) with |coordinates| < 2^20: products below 2^80.
__device__ __forceinline__ int inc_sign_w(int ax, int ay, int bx, int by, int cx, int cy) {
  const long long na = static_cast<long long>(ax) * ax + static_cast<long long>(ay) * ay;
  const long long nb = static_cast<long long>(bx) * bx + static_cast<long long>(by) * by;
  const long long nc = static_cast<long long>(cx) * cx + static_cast<long long>(cy) * cy;
  const long long bc = static_cast<long long>(bx) * cy - static_cast<long long>(by) * cx;
  const long long ca = static_cast<long long>(cx) * ay - static_cast<long long>(cy) * ax;
  const long long ab = static_cast<long long>(ax) * by - static_cast<long long>(ay) * bx;
  const __int128 d = static_cast<__int128>(na) * bc + static_cast<__int128>(nb) * ca +
                     static_cast<__int128>(nc) * ab;
  return (d > 0) - (d < 0);
}

// Counter-clockwise from the +x axis: a strictly before b.
__device__ __forceinline__ bool ccw_before(int ax, int ay, int bx, int by) {
  const int ha = (ay > 0 || (ay == 0 && ax > 0)) ? 0 : 1;
  const int hb = (by > 0 || (by == 0 && bx > 0)) ? 0 : 1;
  if (ha != hb) return ha < hb;
  return static_cast<long long>(ax) * by - static_cast<long long>(ay) * bx > 0;
}

// Squared distance from the particle to the circumcentre of (0, a, b):
// |a|^2 |b|^2 |a - b|^2 / (4 (a x b)^2), in fp64 (relative error ~1e-15).
__device__ __forceinline__ double vertex_r2(int ax, int ay, int bx, int by) {
  const double na = static_cast<double>(ax) * ax + static_cast<double>(ay) * ay;
  const double nb = static_cast<double>(bx) * bx + static_cast<double>(by) * by;
  const double dx = static_cast<double>(ax) - bx, dy = static_cast<double>(ay) - by;
  const double cr = static_cast<double>(ax) * by - static_cast<double>(ay) * bx;
  return na * nb * (dx * dx + dy * dy) / (4.0 * cr * cr);
}

// |v|^2 < (L/8)^2 for the circumcentre v of (0, a, b), exactly:
// 16 |a|^2 |b|^2 |a - b|^2 < L^2 (a x b)^2.  Offsets are minimum images
// (|coordinates| <= 2^19), so the left side stays below 2^123 and the
// right side below 2^118.
__device__ __forceinline__ bool vertex_inside_domain(int ax, int ay, int bx, int by, int box) {
  const unsigned long long na = static_cast<unsigned long long>(static_cast<long long>(ax) * ax +
                                                                static_cast<long long>(ay) * ay);
  const unsigned long long nb = static_cast<unsigned long long>(static_cast<long long>(bx) * bx +
                                                                static_cast<long long>(by) * by);
  const long long dx = static_cast<long long>(ax) - bx, dy = static_cast<long long>(ay) - by;
  const unsigned long long nd = static_cast<unsigned long long>(dx * dx + dy * dy);
  long long cr = static_cast<long long>(ax) * by - static_cast<long long>(ay) * bx;
  if (cr < 0) cr = -cr;
  const unsigned __int128 lhs = static_cast<unsigned __int128>(na) * nb * nd * 16u;
  const unsigned __int128 rhs = static_cast<unsigned __int128>(cr) * static_cast<unsigned long long>(cr) *
                                (static_cast<unsigned long long>(box) * static_cast<unsigned long long>(box));
  return lhs < rhs;
}

// ---------------------------------------------------------------------------
// The cell: the list of its clipping particles, counter-clockwise, in LDS
// (one column per lane: entry t of lane l at [t][l], so a wavefront's lanes
// hit distinct banks), entries h .. h+m-1 of a ring buffer of CAP slots.
// Narrow cells pack each offset as two 16-bit halves.
// ---------------------------------------------------------------------------
template <int CAP, int BLK, bool WIDE>
struct Cell {
  int* xy;  // narrow: packed (x, y); wide: x
  int* yy;  // wide: y
  int* id;  // particle index, or -1 for the bounding square
  int h, m;

  __device__ __forceinline__ int slot(int t) const { return ((h + t) & (CAP - 1)) * BLK; }
  __device__ __forceinline__ void get(int t, int& x, int& y) const {
    const int p = slot(t);
    if (WIDE) {
      x = xy[p];
      y = yy[p];
    } else {
      const int v = xy[p];
      x = static_cast<int>(static_cast<short>(v & 0xFFFF));
      y = v >> 16;
    }
  }
  __device__ __forceinline__ void put(int t, int x, int y, int who) {
    const int p = slot(t);
    if (WIDE) {
      xy[p] = x;
      yy[p] = y;
    } else {
      xy[p] = static_cast<int>((static_cast<uint32_t>(x) & 0xFFFFu) | (static_cast<uint32_t>(y) << 16));
    }
    id[p] = who;
  }
  __device__ __forceinline__ void move(int from, int to) {
    const int p = slot(from), q = slot(to);
    xy[q] = xy[p];
    if (WIDE) yy[q] = yy[p];
    id[q] = id[p];
  }
  __device__ __forceinline__ int inc(int ax, int ay, int bx, int by, int cx, int cy) const {
    return WIDE ? inc_sign_w(ax, ay, bx, by, cx, cy) : inc_sign_n(ax, ay, bx, by, cx, cy);
  }

  // A square of half side `half` around the particle, cut by four virtual
  // particles (id -1) at distance 2 * half.
  __device__ void init(int half) {
    h = 0;
    m = 4;
    put(0, 2 * half, 0, -1);
    put(1, 0, 2 * half, -1);
    put(2, -2 * half, 0, -1);
    put(3, 0, -2 * half, -1);
  }

  // Largest squared vertex distance (narrow cells in fp32: |values| < 2^88,
  // relative error below 1e-6, absorbed by the callers' margin).
  __device__ double max_r2() const {
    if (!WIDE) {
      float r = 0.0f;
      int ax, ay, fx, fy;
      get(0, ax, ay);
      fx = ax;
      fy = ay;
      for (int t = 0; t < m; ++t) {
        int bx, by;
        if (t + 1 < m) get(t + 1, bx, by); else { bx = fx; by = fy; }
        const float na = static_cast<float>(ax * ax + ay * ay), nb = static_cast<float>(bx * bx + by * by);
        const float dx = static_cast<float>(ax - bx), dy = static_cast<float>(ay - by);
        const float cr = static_cast<float>(ax * by - ay * bx);
        r = fmaxf(r, na * nb * (dx * dx + dy * dy) / (4.0f * cr * cr));
        ax = bx;
        ay = by;
      }
      return static_cast<double>(r);
    }
    double r = 0.0;
    int ax, ay, fx, fy;
    get(0, ax, ay);
    fx = ax;
    fy = ay;
    for (int t = 0; t < m; ++t) {
      int bx, by;
      if (t + 1 < m) get(t + 1, bx, by); else { bx = fx; by = fy; }
      r = fmax(r, vertex_r2(ax, ay, bx, by));
      ax = bx;
      ay = by;
    }
    return r;
  }

  // Clip by the bisector of candidate (cx, cy).  1: the cell changed,
  // 0: no vertex lies strictly on the candidate's side, -1: no room.
  __device__ int clip(int cx, int cy, int who) {
    unsigned long long mask = 0ull;
    int ax, ay, fx, fy;
    get(0, ax, ay);
    fx = ax;
    fy = ay;
    for (int t = 0; t < m; ++t) {
      int bx, by;
      if (t + 1 < m) get(t + 1, bx, by); else { bx = fx; by = fy; }
      if (inc(ax, ay, bx, by, cx, cy) < 0) mask |= 1ull << t;
      ax = bx;
      ay = by;
    }
    if (mask == 0ull) return 0;
    const unsigned long long full = m == 64 ? ~0ull : ((1ull << m) - 1ull);
    const unsigned long long prev = ((mask << 1) | (mask >> (m - 1))) & full;  // bit t: vertex t-1 removed
    const unsigned long long first = mask & ~prev;                           // run starts
    if (first == 0ull) return 0;  // every vertex removed: impossible for a cell around its particle
    const int s = __builtin_ctzll(first);
    const int nr = __popcll(mask) - 1;  // clipping particles strictly inside the run
    if (s + nr <= m - 1) {
      // The removed ones are s+1 .. s+nr: the candidate goes to s+1 and the
      // tail moves to close the gap (or to open one, nr = 0).
      if (nr == 0) {
        if (m == CAP) return -1;
        for (int t = m - 1; t > s; --t) move(t, t + 1);
        m += 1;
      } else {
        for (int t = s + nr + 1; t < m; ++t) move(t, t - nr + 1);
        m -= nr - 1;
      }
      put(s + 1, cx, cy, who);
    } else {
      // The removed ones are s+1 .. m-1 and 0 .. e: the kept ones e+1 .. s
      // stay where they are, the candidate takes slot e before them.
      const int e = s + nr - m;
      h = (h + e) & (CAP - 1);
      m = s - e + 1;
      put(0, cx, cy, who);
    }
    return 1;
  }
};

// Outcome of building one cell.
enum : int { kCellDone = 0, kCellWide = 1, kCellFail = 2 };

// Build the Voronoi cell of the particle in slot s (position px, py).
template <int CAP, int BLK, bool WIDE>
__device__ int build_cell(const DevWs& w, Cell<CAP, BLK, WIDE>& cell, int s, int px, int py,
                          int total) {
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom q(px, py, w);
  // bounding square: narrow cells stay within 2^13 of the particle, wide
  // ones start at L/8 (a vertex there is already outside the domain)
  cell.init(WIDE ? (w.box >> 3) : (kVnSpan >> 1));
  // vertex distances are within ~1e-6 (narrow, fp32) or ~1e-15 (wide, fp64)
  // relative: the margin keeps every skip and the stop test on the safe side
  constexpr double margin = WIDE ? 1.0 + 1e-9 : 1.0 + 1e-4;
  double bound = 4.0 * cell.max_r2() * margin;  // candidates beyond cannot cut
  int outcome = -1;
  for (int r = 0; r <= q.rmax && outcome < 0; ++r) {
    if (!WIDE && (static_cast<long long>(r + 1) << w.log2_w) > kVnSpan) {
      outcome = kCellWide;
      break;
    }
    for_ring(r, q.lo, q.hi, [&](int dx, int dy) {
      if (outcome >= 0) return;
      const double gx = axis_gap(dx, q.ox, cw, sh);
      const double gy = axis_gap(dy, q.oy, cw, sh);
      if (gx * gx + gy * gy >= bound) return;
      const int64_t c = static_cast<int64_t>((q.hy + dy) & gm) * w.G + ((q.hx + dx) & gm);
      const int beg = w.start[c];
      const int end = min(w.start[c + 1], total);
      for (int t = beg; t < end && outcome < 0; ++t) {
        if (t == s) continue;
        const int4 e = w.sorted[t];
        const int ex = wrap_axis(e.x - px, sh);
        const int ey = wrap_axis(e.y - py, sh);
        if (ex == 0 && ey == 0) continue;  // the particle's own site
        const double d2 = static_cast<double>(ex) * ex + static_cast<double>(ey) * ey;
        if (d2 >= bound) continue;
        const int rc = cell.clip(ex, ey, e.z);
        if (rc < 0) {
          outcome = WIDE ? kCellFail : kCellWide;
          if (WIDE) set_err(w.hdr, NM_E_CAPACITY);
        } else if (rc > 0) {
          bound = 4.0 * cell.max_r2() * margin;
        }
      }
    });
    if (outcome < 0 && (r == q.rmax || static_cast<double>(q.ring_bound(r, cw)) >= bound))
      outcome = kCellDone;
  }
  if (outcome != kCellDone) return outcome < 0 ? kCellDone : outcome;
  // The bounding square must be gone and every vertex inside L/8.
  int ax, ay, fx, fy;
  cell.get(0, ax, ay);
  fx = ax;
  fy = ay;
  for (int t = 0; t < cell.m; ++t) {
    int bx, by;
    if (t + 1 < cell.m) cell.get(t + 1, bx, by); else { bx = fx; by = fy; }
    const bool virt = cell.id[cell.slot(t)] < 0;
    if (virt || !vertex_inside_domain(ax, ay, bx, by, w.box)) {
      if (!WIDE) return kCellWide;
      set_err(w.hdr, NM_E_RANGE);
      return kCellFail;
    }
    ax = bx;
    ay = by;
  }
  return kCellDone;
}

// Append the particles at position (sx, sy), in ascending index, except
// `skip`, to row[*cnt ..] (each found by a scan of the position's grid cell).
__device__ __forceinline__ void site_members(const DevWs& w, int sx, int sy, int skip, int total,
                                             int32_t* __restrict__ row, int dmax, int& cnt) {
  const int64_t c = static_cast<int64_t>(sy >> w.log2_w) * w.G + (sx >> w.log2_w);
  const int beg = w.start[c];
  const int end = min(w.start[c + 1], total);
  int last = -1;
  for (;;) {
    int best = 0x7FFFFFFF, left = 0;  // the next index, and how many remain
    for (int t = beg; t < end; ++t) {
      const int4 e = w.sorted[t];
      if (e.x == sx && e.y == sy && e.z > last && e.z != skip) {
        ++left;
        best = min(best, e.z);
      }
    }
    if (left == 0) break;
    if (cnt < dmax) row[cnt] = best;
    ++cnt;
    last = best;
    if (left == 1) break;  // that was the last one (no second scan for a lone particle)
  }
}

// Write the cell's row: the other particles of the own site, then the
// clipping particles whose edge has positive length, counter-clockwise from
// the +x axis, each expanded to all particles of its site.
template <int CAP, int BLK, bool WIDE>
__device__ void write_row(const DevWs& w, const Cell<CAP, BLK, WIDE>& cell, int who, int px, int py,
                          int total, int dmax, int32_t* __restrict__ ring, int32_t* __restrict__ deg) {
  const int m = cell.m;
  const int mask = w.box - 1;
  // start: the clipping particle with the smallest angle from +x
  int t0 = 0, bx0, by0;
  cell.get(0, bx0, by0);
  for (int t = 1; t < m; ++t) {
    int x, y;
    cell.get(t, x, y);
    if (ccw_before(x, y, bx0, by0)) {
      t0 = t;
      bx0 = x;
      by0 = y;
    }
  }
  int32_t* row = ring + static_cast<long long>(who) * dmax;
  int cnt = 0;
  site_members(w, px, py, who, total, row, dmax, cnt);
  int qx, qy, cx, cy, nx, ny;
  cell.get((t0 + m - 1) % m, qx, qy);
  cell.get(t0, cx, cy);
  for (int u = 0; u < m; ++u) {
    cell.get((t0 + u + 1) % m, nx, ny);
    if (cell.inc(qx, qy, cx, cy, nx, ny) != 0)
      site_members(w, (px + cx) & mask, (py + cy) & mask, -1, total, row, dmax, cnt);
    qx = cx;
    qy = cy;
    cx = nx;
    cy = ny;
  }
  if (cnt > dmax) set_err(w.hdr, NM_E_CAPACITY);
  for (int u = cnt; u < dmax; ++u) row[u] = -1;
  deg[who] = min(cnt, dmax);
}

__device__ __forceinline__ bool cells_built(const DevWs& w) {
  const WsHeader* hd = w.hdr;
  return hd->built == kBuilt && hd->n == w.n && hd->box == w.box && hd->cell_w == w.cell_w;
}

// Append slot s to the wide kernel's list (one atomic per wavefront).
__device__ __forceinline__ void list_wide(const DevWs& w, bool go, int s) {
  const unsigned long long b = __ballot(go);
  if (b == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(static_cast<long long>(b)) - 1;
  uint32_t base = 0u;
  if (lane == leader) base = atomicAdd(&w.hdr->nvwide, static_cast<uint32_t>(__popcll(b)));
  base = __shfl(base, leader, 64);
  const uint32_t at = base + static_cast<uint32_t>(__popcll(b & ((1ull << lane) - 1ull)));
  if (go && at < static_cast<uint32_t>(w.n)) w.vlist[at] = s;
}

// Narrow kernel over slots: every slot (list == nullptr) or the slots listed
// in `list` (count at *count).
// With `gate`, nothing runs unless *gate != 0.
__global__ __launch_bounds__(kVnBlock) void k_voronoi(DevWs w, int dmax, int32_t* __restrict__ ring,
                                                      int32_t* __restrict__ deg,
                                                      const int32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ count,
                                                      const uint32_t* __restrict__ gate) {
  __shared__ int sxy[kVnCap * kVnBlock];
  __shared__ int sid[kVnCap * kVnBlock];
  if (gate && *gate == 0u) return;
  if (!cells_built(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int nwork = list ? static_cast<int>(min<uint32_t>(*count, static_cast<uint32_t>(w.n))) : total;
  const int base = (list ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x)) * kVnBlock;
  if (base >= nwork) return;
  const int k = base + threadIdx.x;
  bool wide = false;
  int s = -1;
  if (k < nwork) {
    s = list ? list[k] : k;
    const int4 e = w.sorted[s];
    Cell<kVnCap, kVnBlock, false> cell{sxy + threadIdx.x, nullptr, sid + threadIdx.x, 0, 0};
    const int rc = build_cell(w, cell, s, e.x, e.y, total);
    if (rc == kCellDone) write_row(w, cell, e.z, e.x, e.y, total, dmax, ring, deg);
    wide = rc == kCellWide;
  }
  list_wide(w, wide, s);
}

// Wide kernel over the listed slots; the last workgroup empties the list.
__global__ __launch_bounds__(kVwBlock) void k_voronoi_wide(DevWs w, int dmax, int32_t* __restrict__ ring,
                                                           int32_t* __restrict__ deg) {
  __shared__ int sx[kVwCap * kVwBlock];
  __shared__ int sy[kVwCap * kVwBlock];
  __shared__ int sid[kVwCap * kVwBlock];
  const int total = min(w.start[w.C], w.n);
  const int nl = static_cast<int>(min<uint32_t>(w.hdr->nvwide, static_cast<uint32_t>(w.n)));
  for (int k = blockIdx.x * kVwBlock + threadIdx.x; k - threadIdx.x < nl; k += gridDim.x * kVwBlock) {
    if (k >= nl) continue;
    const int s = w.vlist[k];
    const int4 e = w.sorted[s];
    Cell<kVwCap, kVwBlock, true> cell{sx + threadIdx.x, sy + threadIdx.x, sid + threadIdx.x, 0, 0};
    if (build_cell(w, cell, s, e.x, e.y, total) == kCellDone) write_row(w, cell, e.z, e.x, e.y, total, dmax, ring, deg);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&w.hdr->nvdone, 1u) == gridDim.x - 1) {
      w.hdr->nvwide = 0u;
      w.hdr->nvdone = 0u;
    }
  }
}

// ---------------------------------------------------------------------------
// "Do I need to recompute the Voronoi diagram?" (Sec. IV), as a test of the
// old triangulation against the new positions.  Particle i's row
// a_0 .. a_{m-1} (counter-clockwise) stands for the triangles
// (i, a_t, a_{t+1}).  The rows are still exactly the neighbour lists when,
// for every particle and every t,
//   - each offset a_t - i has both components below L/4 (so the minimum
//     images of a triangle's edges agree),
//   - the triangle (i, a_t, a_{t+1}) turns counter-clockwise,
//   - the row winds once around i (one wrap past the +x axis),
//   - a_t's row holds a_{t+1} directly followed by i (the three rows agree
//     on the triangle),
//   - a_{t+2} lies strictly outside the circle through i, a_t, a_{t+1}
//     (the edge i - a_{t+1} is locally Delaunay, strictly),
// where a_t are the row's sites (runs of particles at one position, the
// own site's particles left out), and every particle listed at the own site
// lists this one back.
// and, over all rows, the cross products a_t x a_{t+1} sum to exactly 6 L^2
// (each triangle is counted from its three corners: the triangles cover the
// box once).  Then the rows form a triangulation of the torus that is
// locally Delaunay at every edge, hence the unique Delaunay triangulation,
// and no four of its particles are co-circular on an empty circle, so every
// edge is a neighbour pair.  A particle that finds a failure marks itself and
// its row's particles stale and counts itself in nvfail; a wrong total sets
// nvfail's top bit (no row can be trusted).  A zero count certifies the rows;
// rows of co-circular particles (a square lattice) never pass, so such
// systems are always recomputed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_vor_clear(WsHeader* hdr, uint8_t* __restrict__ stale, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) stale[i] = 0;
  if (i == 0) {
    hdr->nvfail = 0u;
    hdr->nvstale = 0u;
    hdr->varea2 = 0ull;
  }
}

// Rows of up to this many entries are read whole when searched.
constexpr int kRowRead = 8;

// Rows hold sites: a prefix of particles at the row's own position, then
// runs of particles sharing a position.  These helpers walk a row site by
// site; entries are valid indices (checked before).  A row of up to
// kRowRead entries is held in registers with its entries' positions (read
// together, not as a chain of index and position reads per step).
struct RowView {
  const int32_t* row;
  int m;
  int own;  // length of the own-site prefix
  const int32_t* x;
  const int32_t* y;
  bool whole;
  int rw[kRowRead], px[kRowRead], py[kRowRead];
  __device__ static __forceinline__ int sel(const int (&a)[kRowRead], int t) {
    int v = 0;
#pragma unroll
    for (int u = 0; u < kRowRead; ++u)
      if (u == t) v = a[u];
    return v;
  }
  __device__ __forceinline__ int idx(int t) const { return whole ? sel(rw, t) : row[t]; }
  __device__ __forceinline__ int xat(int t) const { return whole ? sel(px, t) : x[row[t]]; }
  __device__ __forceinline__ int yat(int t) const { return whole ? sel(py, t) : y[row[t]]; }
  __device__ __forceinline__ bool same(int t, int u) const { return xat(t) == xat(u) && yat(t) == yat(u); }
  // the first entry of the site after the one entry t belongs to (cyclic over
  // the site part of the row)
  __device__ __forceinline__ int next_site(int t) const {
    int u = t;
    for (int guard = 0; guard < m; ++guard) {
      u = u + 1 < m ? u + 1 : own;
      if (!same(u, t)) return u;
    }
    return t;
  }
  // the first entry of the site that entry t belongs to
  __device__ __forceinline__ int site_start(int t) const {
    int u = t;
    for (int guard = 0; guard < m; ++guard) {
      const int v = u > own ? u - 1 : m - 1;
      if (!same(v, t)) return u;
      u = v;
    }
    return t;
  }
};

// `dmax`: the rows' stride (a row is read whole only within it).
__device__ __forceinline__ RowView row_view(const int32_t* row, int m, int self, const int32_t* x,
                                            const int32_t* y, int dmax) {
  RowView r;
  r.row = row;
  r.m = m;
  r.own = 0;
  r.x = x;
  r.y = y;
  r.whole = m <= kRowRead && dmax >= kRowRead;
  if (r.whole) {
#pragma unroll
    for (int u = 0; u < kRowRead; ++u) r.rw[u] = row[u];
#pragma unroll
    for (int u = 0; u < kRowRead; ++u) {
      r.px[u] = u < m ? x[r.rw[u]] : 0;
      r.py[u] = u < m ? y[r.rw[u]] : 0;
    }
  }
  const int sx = x[self], sy = y[self];
  while (r.own < m && r.xat(r.own) == sx && r.yat(r.own) == sy) ++r.own;
  return r;
}

// Row `rv` (of particle a) holds the site at (bxp, byp) followed directly by
// the site at (ixp, iyp).
__device__ __forceinline__ bool row_holds_then(const RowView& rv, int bxp, int byp, int ixp, int iyp) {
  for (int t = rv.own; t < rv.m; ++t) {
    if (rv.xat(t) == bxp && rv.yat(t) == byp) {
      const int u = rv.next_site(t);
      return rv.xat(u) == ixp && rv.yat(u) == iyp;
    }
  }
  return false;
}

__global__ __launch_bounds__(kBlock) void k_vor_check(const int32_t* __restrict__ x,
                                                      const int32_t* __restrict__ y, int n, int log2_box,
                                                      int dmax, const int32_t* __restrict__ ring,
                                                      const int32_t* __restrict__ deg,
                                                      uint8_t* __restrict__ stale, WsHeader* hdr) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  bool fail = false;
  long long area2 = 0;
  if (i < n) {
    const int sh = 32 - log2_box;
    const int quarter = 1 << (log2_box - 2);
    const int m = deg[i];
    const int32_t* row = ring + static_cast<long long>(i) * dmax;
    if (m < 3 || m > dmax) fail = true;
    for (int t = 0; t < m && !fail; ++t) {  // indices first: only valid ones are read through
      const int j = row[t];
      if (static_cast<unsigned>(j) >= static_cast<unsigned>(n) || j == i) fail = true;
    }
    if (!fail) {
      const int xi = x[i], yi = y[i];
      const RowView rv = row_view(row, m, i, x, y, dmax);
      // the own site counts once in the area total: from its lowest index;
      // and every particle listed at the own site lists this one back
      bool lowest = true;
      for (int t = 0; t < rv.own && !fail; ++t) {
        const int p = row[t];
        lowest = lowest && p > i;
        const int mp = deg[p];
        bool back = false;
        if (mp >= 1 && mp <= dmax) {
          const int32_t* rowp = ring + static_cast<long long>(p) * dmax;
          for (int u = 0; u < mp; ++u) {
            const int q = rowp[u];
            if (static_cast<unsigned>(q) >= static_cast<unsigned>(n) || x[q] != xi || y[q] != yi) break;
            back = back || q == i;
          }
        }
        if (!back) fail = true;
      }
      if (m - rv.own < 3) fail = true;
      auto off = [&](int t, int& ox, int& oy) {  // entry t's offset
        ox = wrap_axis(rv.xat(t) - xi, sh);
        oy = wrap_axis(rv.yat(t) - yi, sh);
      };
      const int t0 = fail ? 0 : rv.site_start(rv.own);
      int ta = t0, tb = fail ? 0 : rv.next_site(t0);
      int ax, ay, bx, by;
      if (!fail) {
        off(ta, ax, ay);
        off(tb, bx, by);
      }
      int wraps = 0, nsites = 0;
      for (int guard = 0; guard < m && !fail; ++guard) {
        const int tc = rv.next_site(tb);
        int cx, cy;
        off(tc, cx, cy);
        if (abs(ax) >= quarter || abs(ay) >= quarter || (ax == 0 && ay == 0)) {
          fail = true;
          break;
        }
        const long long cr = static_cast<long long>(ax) * by - static_cast<long long>(ay) * bx;
        if (cr <= 0) fail = true;
        area2 += cr;
        if (!ccw_before(ax, ay, bx, by)) ++wraps;
        if (inc_sign_w(ax, ay, bx, by, cx, cy) <= 0) fail = true;
        const int a = rv.idx(ta);
        const int ma = deg[a];
        if (ma < 3 || ma > dmax) {
          fail = true;
        } else {
          // a's row must hold b's site directly followed by i's site.  When it
          // lists b directly followed by i the sites are adjacent (b and i lie
          // at different positions) and no position is needed; otherwise the
          // row is walked site by site.
          const int32_t* rowa = ring + static_cast<long long>(a) * dmax;
          const int b = rv.idx(tb);
          bool okidx = true, adjacent = false;
          if (ma <= kRowRead && dmax >= kRowRead) {
            // the usual short row: its first kRowRead entries read together
            // (rows are dmax long), instead of one read per step
            int ra[kRowRead];
#pragma unroll
            for (int u = 0; u < kRowRead; ++u) ra[u] = rowa[u];
#pragma unroll
            for (int u = 0; u < kRowRead; ++u) {
              if (u < ma) {
                const int nx = u + 1 < ma ? ra[u + 1 < kRowRead ? u + 1 : 0] : ra[0];
                okidx = okidx && static_cast<unsigned>(ra[u]) < static_cast<unsigned>(n);
                adjacent = adjacent || (ra[u] == b && nx == i);
              }
            }
          } else {
            for (int u = 0; u < ma; ++u) {
              const int q = rowa[u];
              okidx = okidx && static_cast<unsigned>(q) < static_cast<unsigned>(n);
              adjacent = adjacent || (q == b && rowa[u + 1 < ma ? u + 1 : 0] == i);
            }
          }
          if (!okidx || (!adjacent && !row_holds_then(row_view(rowa, ma, a, x, y, dmax), rv.xat(tb), rv.yat(tb), xi, yi)))
            fail = true;
        }
        ++nsites;
        ta = tb;
        ax = bx;
        ay = by;
        tb = tc;
        bx = cx;
        by = cy;
        if (ta == t0) break;
      }
      if (wraps != 1 || nsites < 3) fail = true;
      if (!lowest) area2 = 0;
    }
    if (fail) {
      stale[i] = 1;
      const int m2 = min(max(m, 0), dmax);  // deg out of range: mark what the row holds
      for (int t = 0; t < m2; ++t) {
        const int j = row[t];
        if (static_cast<unsigned>(j) < static_cast<unsigned>(n)) stale[j] = 1;
      }
    }
  }
  const unsigned long long bal = __ballot(fail);
  if (bal != 0ull && (threadIdx.x & 63) == __ffsll(static_cast<long long>(bal)) - 1)
    atomicAdd(&hdr->nvfail, static_cast<uint32_t>(__popcll(bal)));
  // the area total: a wavefront's sum, one atomic (only counted while no row fails)
  if (fail) area2 = 0;
  for (int o = 32; o > 0; o >>= 1) area2 += __shfl_xor(area2, o, 64);
  if ((threadIdx.x & 63) == 0 && area2 != 0) atomicAdd(&hdr->varea2, static_cast<unsigned long long>(area2));
}

// Rows that passed: rotate the site part to start at the +x axis again
// (positions moved).  Stale rows: list the particle's slot for recomputation.
__global__ __launch_bounds__(kBlock) void k_vor_sweep(DevWs w, const int32_t* __restrict__ x,
                                                      const int32_t* __restrict__ y, int dmax,
                                                      int32_t* __restrict__ ring,
                                                      const int32_t* __restrict__ deg,
                                                      const uint8_t* __restrict__ stale) {
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  bool go = false;
  if (s < total) {
    const int i = w.sorted[s].z;
    if (stale[i]) {
      go = true;
    } else {
      const int sh = 32 - w.log2_box;
      const int m = deg[i];
      int32_t* row = ring + static_cast<long long>(i) * dmax;
      const RowView rv = row_view(row, m, i, x, y, dmax);
      const int xi = x[i], yi = y[i];
      // the first entry of the site with the smallest angle
      int t0 = rv.own;
      int bx = wrap_axis(rv.xat(t0) - xi, sh), by = wrap_axis(rv.yat(t0) - yi, sh);
      for (int t = rv.own + 1; t < m; ++t) {
        const int ox = wrap_axis(rv.xat(t) - xi, sh), oy = wrap_axis(rv.yat(t) - yi, sh);
        if (ccw_before(ox, oy, bx, by)) {
          t0 = t;
          bx = ox;
          by = oy;
        }
      }
      t0 = rv.site_start(t0);
      if (t0 != rv.own) {  // rotate the site part left by t0 - own: three reversals
        auto rev = [&](int lo, int hi) {
          for (--hi; lo < hi; ++lo, --hi) {
            const int v = row[lo];
            row[lo] = row[hi];
            row[hi] = v;
          }
        };
        rev(rv.own, t0);
        rev(t0, m);
        rev(rv.own, m);
      }
    }
  }
  const unsigned long long b = __ballot(go);
  if (b == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(static_cast<long long>(b)) - 1;
  uint32_t base = 0u;
  if (lane == leader) base = atomicAdd(&w.hdr->nvstale, static_cast<uint32_t>(__popcll(b)));
  base = __shfl(base, leader, 64);
  const uint32_t at = base + static_cast<uint32_t>(__popcll(b & ((1ull << lane) - 1ull)));
  if (go && at < static_cast<uint32_t>(w.n)) w.rank[at] = s;
}

// After k_vor_check: a total other than 6 L^2 distrusts every row.
__global__ void k_vor_total(WsHeader* hdr, int log2_box, int32_t* out) {
  const unsigned long long want = 6ull << (2 * log2_box);
  if (hdr->nvfail == 0u && hdr->varea2 != want) hdr->nvfail = 0x80000000u;
  if (out) *out = static_cast<int32_t>(min(hdr->nvfail, 0x7FFFFFFFu));
}

}  // namespace

hipError_t launch_voronoi(const DevWs& w, int dmax, int32_t* ring, int32_t* deg, hipStream_t s) {
  const int nb = (w.n + kVnBlock - 1) / kVnBlock;
  hipLaunchKernelGGL(k_voronoi, dim3(nb), dim3(kVnBlock), 0, s, w, dmax, ring, deg, nullptr, nullptr,
                     nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_voronoi_wide, dim3(kVwGrid), dim3(kVwBlock), 0, s, w, dmax, ring, deg);
  return hipGetLastError();
}

hipError_t launch_voronoi_check(const DevWs& w, const int32_t* x, const int32_t* y, int dmax,
                                const int32_t* ring, const int32_t* deg, uint8_t* stale, int32_t* nfail,
                                hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_vor_clear, dim3(nb), dim3(kBlock), 0, s, w.hdr, stale, w.n);
  hipLaunchKernelGGL(k_vor_check, dim3(nb), dim3(kBlock), 0, s, x, y, w.n, w.log2_box, dmax, ring, deg,
                     stale, w.hdr);
  hipLaunchKernelGGL(k_vor_total, dim3(1), dim3(1), 0, s, w.hdr, w.log2_box, nfail);
  return hipGetLastError();
}

hipError_t launch_voronoi_update(const DevWs& w, const int32_t* x, const int32_t* y, int dmax,
                                 int32_t* ring, int32_t* deg, uint8_t* stale, int32_t* nfail, int rounds,
                                 hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  const int nv = (w.n + kVnBlock - 1) / kVnBlock;
  hipError_t e = hipSuccess;
  for (int r = 0; r < rounds && e == hipSuccess; ++r) {
    e = launch_voronoi_check(w, x, y, dmax, ring, deg, stale, r == 0 ? nfail : nullptr, s);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_vor_sweep, dim3(nb), dim3(kBlock), 0, s, w, x, y, dmax, ring, deg, stale);
    hipLaunchKernelGGL(k_voronoi, dim3(nv), dim3(kVnBlock), 0, s, w, dmax, ring, deg, w.rank,
                       &w.hdr->nvstale, nullptr);
    hipLaunchKernelGGL(k_voronoi_wide, dim3(kVwGrid), dim3(kVwBlock), 0, s, w, dmax, ring, deg);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // final certificate; anything still stale: every row again
  e = launch_voronoi_check(w, x, y, dmax, ring, deg, stale, rounds == 0 ? nfail : nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_voronoi, dim3(nv), dim3(kVnBlock), 0, s, w, dmax, ring, deg, nullptr, nullptr,
                     &w.hdr->nvfail);
  hipLaunchKernelGGL(k_voronoi_wide, dim3(kVwGrid), dim3(kVwBlock), 0, s, w, dmax, ring, deg);
  return hipGetLastError();
}

}  // namespace nm
