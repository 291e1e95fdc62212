// knn.hip -- topological neighbour lists (Sec. III: each particle interacts
// with its k nearest neighbours) and the fused step kernel.
//
// One lane per query, queries taken in cell order so that a wavefront's
// queries are spatial neighbours and read the same cached cells.
//
// Fast path: the lane scans a B x B block of cells around the query (a few
// contiguous slot ranges) and pushes every candidate through a branch-free
// insertion network of 32-bit keys (v_med3_u32), which keeps the k+1 best.
// The result is certified exact when the k+1 best have distinct distances
// and the k-th distance is strictly inside the block (no point outside can
// be as near); this holds for the great majority of queries.
//
// Exact path (the rest): rings of cells outward from the home cell, skipping
// cells whose nearest point is already farther than the current k-th
// neighbour, with 64-bit (d^2, index) keys.  It stops after ring r once the
// k-th squared distance is strictly below the squared distance to the edge of
// the scanned block: an equal distance in the next ring could still carry a
// smaller index, so equality does not stop the walk.
//
// The fused kernel then evaluates Eq. (2) and Eq. (1) for the query from the
// fp64 unit vectors stored beside the cell-ordered copy (the neighbours'
// entries sit in the cells just scanned, so they are cache hits) and writes
// the list, the new position and the new heading at the particle's index.
#include "nm_internal.h"

namespace nm {

namespace {

// Exact ring search (64-bit keys), filling `slot` with the k nearest.
template <int KMAX>
__device__ __forceinline__ bool knn_exact(const DevWs& w, int s, int qx, int qy, int k, int total,
                                          int (&slot)[KMAX]) {
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom q(qx, qy, w);
  TopK<KMAX, true> top;
  top.init(k);
  for (int r = 0; r <= q.rmax; ++r) {
    for_ring(r, q.lo, q.hi, [&](int dx, int dy) {
      const long long gx = axis_gap(dx, q.ox, cw, sh);
      const long long gy = axis_gap(dy, q.oy, cw, sh);
      if (gx * gx + gy * gy > key_bound_d2(top.worst())) return;
      const int64_t c = static_cast<int64_t>((q.hy + dy) & gm) * w.G + ((q.hx + dx) & gm);
      const int beg = w.start[c];
      const int end = min(w.start[c + 1], total);
      for (int t = beg; t < end; ++t) {
        if (t == s) continue;
        const int4 e = w.sorted[t];
        const int ex = wrap_axis(e.x - qx, sh);
        const int ey = wrap_axis(e.y - qy, sh);
        const long long d2 = static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey;
        const unsigned long long kk = pack_key(d2, e.z);
        if (kk < top.worst()) top.push(kk, t);
      }
    });
    if (key_bound_d2(top.worst()) < q.ring_bound(r, cw)) break;
  }
#pragma unroll
  for (int t = 0; t < KMAX; ++t) slot[t] = top.slot[t];
  return top.worst() != ~0ull;
}

// Reorder the k neighbour slots by exact (d^2, index): used when two of them
// share a distance field of the 32-bit keys (rare).
template <int KMAX>
__device__ __forceinline__ void sort_exact(const DevWs& w, int qx, int qy, int k, int (&slot)[KMAX]) {
  const int sh = 32 - w.log2_box;
  unsigned long long kk[KMAX];
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    kk[t] = ~0ull;
    if (t >= KMAX - k) {
      const int4 e = w.sorted[slot[t]];
      const int ex = wrap_axis(e.x - qx, sh), ey = wrap_axis(e.y - qy, sh);
      kk[t] = pack_key(static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey, e.z);
    }
  }
  // insertion sort over the static positions (the unused prefix holds ~0)
#pragma unroll
  for (int i = 1; i < KMAX; ++i) {
#pragma unroll
    for (int j = i; j > 0; --j) {
      const bool swap = kk[j] < kk[j - 1];
      const unsigned long long a = kk[j - 1], c = kk[j];
      const int sa = slot[j - 1], sc = slot[j];
      kk[j - 1] = swap ? c : a;
      kk[j] = swap ? a : c;
      slot[j - 1] = swap ? sc : sa;
      slot[j] = swap ? sa : sc;
    }
  }
  // the ~0 entries of the unused prefix sorted to the end: rotate them back
  if (k < KMAX) {
    int tmp[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) tmp[t] = slot[t];
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
      if (t >= KMAX - k) slot[t] = tmp[t - (KMAX - k)];
  }
}

// Block side for a query: its edge should sit `reach` mean k-th-neighbour
// radii away, r_k^2 = k / (pi rho), with the density rho estimated from the
// occupancy of the (up to) 3 x 3 cells around the home cell.
__device__ __forceinline__ int pick_block(const DevWs& w, const FastCfg& f, int k, int qx, int qy) {
  if (f.bfix > 0) return f.bfix;
  const int G = w.G;
  const int hx = qx >> w.log2_w, hy = qy >> w.log2_w;
  const int c0 = max(hx - 1, 0), c1 = min(hx + 1, G - 1);
  int n9 = 0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    const int64_t row = static_cast<int64_t>((hy + dy) & (G - 1)) * G;
    n9 += w.start[row + c1 + 1] - w.start[row + c0];
  }
  const float cells = 3.0f * static_cast<float>(c1 - c0 + 1);
  const float rk = sqrtf(static_cast<float>(k) * cells / (3.14159265f * fmaxf(static_cast<float>(n9), 0.5f)));
  const int B = static_cast<int>(ceilf(2.0f * f.reach * rk)) + 1;
  return min(max(B, 3), f.bmax);
}

// Fast block search; true (and `slot` filled) only when certified exact.
template <int KMAX>
__device__ __forceinline__ bool knn_fast(const DevWs& w, const FastCfg& f, int s, int qx, int qy,
                                         int k, int total, int (&slot)[KMAX]) {
  constexpr int KT = KMAX + 1;
  if (f.bmax == 0) return false;
  int B = pick_block(w, f, k, qx, qy);
  for (int attempt = 0; attempt < 2; ++attempt) {
    const QBlock b = make_qblock(w, qx, qy, B);
    uint32_t key[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) key[t] = (t < KT - (k + 1)) ? 0u : kKey32Inf;
    const uint32_t clampd = static_cast<uint32_t>(b.bound);
    const int sh = b.sh;
    const bool ok = walk_block(w, b, s, qx, qy, total,
                               [&](int x, int y, int qxi, int qyi, int tag, bool valid) {
                                 const int dx = x - qxi, dy = y - qyi;
                                 const uint32_t d2 = static_cast<uint32_t>(__mul24(dx, dx)) +
                                                     static_cast<uint32_t>(__mul24(dy, dy));
                                 const uint32_t kk = ((min(d2, clampd) >> sh) << 13) | static_cast<uint32_t>(tag);
                                 net_insert(key, valid ? kk : kKey32Inf);
                               });
    if (!ok) return false;
    const uint32_t kth = key[KT - 2];
    const long long dmax = (static_cast<long long>(key32_d(kth) + 1) << sh) - 1;
    if (kth == kKey32Inf || dmax >= b.bound) {  // the k-th may lie outside: widen once
      if (attempt == 0 && B < f.bmax) {
        B = min(B + 2, f.bmax);
        continue;
      }
      return false;
    }
    // The k nearest form the set {d^2 >> sh <= that of the k-th} only if the
    // (k+1)-th has a larger distance field; otherwise the exact search decides.
    if (key32_d(kth) >= key32_d(key[KT - 1])) return false;
    bool tied = false;
#pragma unroll
    for (int t = 0; t < KT - 2; ++t)
      if (t >= KT - (k + 1)) tied = tied || (key32_d(key[t]) == key32_d(key[t + 1]));
    bool mapped = true;
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
      if (t >= KMAX - k) {
        slot[t] = tag_slot(w, b, key[t] & 0x1FFFu, qx, qy);
        mapped = mapped && static_cast<uint32_t>(slot[t]) < static_cast<uint32_t>(total);
      }
    }
    if (mapped && tied) sort_exact<KMAX>(w, qx, qy, k, slot);
    return mapped;
  }
  return false;
}

__device__ __forceinline__ bool ws_ready(const DevWs& w) {
  const WsHeader* h = w.hdr;
  return h->built == kBuilt && h->n == w.n && h->box == w.box && h->cell_w == w.cell_w;
}

struct AlignArgs {
  int32_t v0;
  float eta;
  int32_t include_self;
  const float* theta;
  int32_t* x_out;
  int32_t* y_out;
  float* theta_out;
};

// Outputs of one query from the slots of its k neighbours: the list row (and
// squared distances), and for the fused step Eq. (2) and Eq. (1).
template <int KMAX, bool kAlign>
__device__ __forceinline__ void finish_query(const DevWs& w, int s, const int4& q, const int (&slot)[KMAX],
                                             int k, int32_t* __restrict__ nbr,
                                             long long* __restrict__ d2out, const AlignArgs& a) {
  int32_t* row = nbr + static_cast<int64_t>(q.z) * k;
  const int sh = 32 - w.log2_box;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    if (t >= KMAX - k) {
      const int4 e = w.sorted[slot[t]];
      row[t - (KMAX - k)] = e.z;
      if (!kAlign && d2out) {
        const int ex = wrap_axis(e.x - q.x, sh), ey = wrap_axis(e.y - q.y, sh);
        d2out[static_cast<int64_t>(q.z) * k + t - (KMAX - k)] =
            static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey;
      }
      if (kAlign) {
        const double2 u = w.cs[2 * slot[t]];
        sx += u.x;
        sy += u.y;
      }
    }
  }
  if (!kAlign) return;

  // Eq. (2): average of the neighbours' unit vectors (plus the particle's own),
  // vectorial noise, normalisation (only the direction is kept).
  const double2 own = w.cs[2 * s];
  const double2 xi = w.cs[2 * s + 1];
  if (a.include_self) {
    sx += own.x;
    sy += own.y;
  }
  const double m = static_cast<double>(k + (a.include_self ? 1 : 0));
  const double ax = sx / m, ay = sy / m;
  const double e = static_cast<double>(a.eta);
  const double vx = ax + e * xi.x;
  const double vy = ay + e * xi.y;
  const float th = (vx == 0.0 && vy == 0.0) ? a.theta[q.z] : vec_angle(vx, vy, 0.0f);

  // Eq. (1): move with the heading at time t, rounded to the grid (half to even).
  const int ddx = static_cast<int>(rint(static_cast<double>(a.v0) * own.x));
  const int ddy = static_cast<int>(rint(static_cast<double>(a.v0) * own.y));
  const int mask = w.box - 1;
  a.x_out[q.z] = (q.x + ddx) & mask;
  a.y_out[q.z] = (q.y + ddy) & mask;
  a.theta_out[q.z] = th;
}

// ---------------------------------------------------------------------------
// Tiles.  A workgroup owns `tc` consecutive cells of one cell row; its queries
// (the particles of those cells) are one contiguous range of cell-ordered
// slots.  It stages the halo of (2h + 1) x (tc + 2h) cells around the tile
// into LDS -- the cell start table and every particle's position, shifted
// into the tile's periodic image -- and each lane then runs the block search
// on LDS only.  A tile whose halo holds more than kTilePts particles (a dense
// cluster) searches global memory instead.  Queries that are not certified go
// to the tile's segment of the queue for the exact kernel.
// ---------------------------------------------------------------------------
constexpr int kTileCells = 2048;
constexpr int kTilePts = 2048;

struct TileCfg {
  int tc;    // tile width in cells
  int h;     // halo in cells (0: no staging)
  int ntx;   // tiles per cell row
  int bmax;  // largest block side the halo supports
};

__device__ __forceinline__ int tile_index(int b, int nb) { return xcd_tile(b, nb); }

// Block search on the staged tile.  jh: home column in staged coordinates,
// self: the query's LDS index.
template <int KMAX>
__device__ __forceinline__ bool knn_lds(const DevWs& w, const FastCfg& f, const TileCfg& tc,
                                        const int* lcell, const int2* lpos, const int* lslot, int W,
                                        int jh, int self, int qx, int qy, int k, int (&slot)[KMAX]) {
  constexpr int KT = KMAX + 1;
  const int h = tc.h;
  int B = f.bfix;
  if (B == 0) {
    int n9 = 0;
#pragma unroll
    for (int dr = -1; dr <= 1; ++dr) n9 += lcell[(h + dr) * W + jh + 2] - lcell[(h + dr) * W + jh - 1];
    const float rk = sqrtf(static_cast<float>(k) * 9.0f / (3.14159265f * fmaxf(static_cast<float>(n9), 0.5f)));
    B = static_cast<int>(ceilf(2.0f * f.reach * rk)) + 1;
    B = max(B, 3);
  }
  if (B > tc.bmax) return false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const QBlock b = make_qblock(w, qx, qy, B);
    uint32_t key[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) key[t] = (t < KT - (k + 1)) ? 0u : kKey32Inf;
    const uint32_t clampd = static_cast<uint32_t>(b.bound);
    const int sh = b.sh;
    // The block's rows as one flat sequence of LDS indices: a single loop over
    // every candidate of every row (the row switch is a predicated update), so
    // a wavefront runs as many iterations as its longest query, not as the sum
    // of its longest rows.  The query itself gets the key INF.
    const int j0 = jh + b.lo_x;
    const int row0 = (h + b.lo_y) * W + j0;
    int ncand = 0;
    for (int r = 0; r < B; ++r) ncand += lcell[row0 + r * W + B] - lcell[row0 + r * W];
    int r = 0, i = lcell[row0], e = lcell[row0 + B];
    while (i == e && r + 1 < B) {
      ++r;
      i = lcell[row0 + r * W];
      e = lcell[row0 + r * W + B];
    }
    int2 p = lpos[min(i, kTilePts - 1)];  // (no candidate at all: a harmless in-bounds read)
    for (int c = 0; c < ncand; ++c) {
      const int icur = i;
      const int2 pc = p;
      // advance to the next candidate (next row when this one is exhausted)
      ++i;
      while (i == e && r + 1 < B) {
        ++r;
        i = lcell[row0 + r * W];
        e = lcell[row0 + r * W + B];
      }
      p = lpos[min(i, kTilePts - 1)];
      const int dx = pc.x - qx, dy = pc.y - qy;
      const uint32_t d2 = static_cast<uint32_t>(__mul24(dx, dx)) + static_cast<uint32_t>(__mul24(dy, dy));
      const uint32_t kk = ((min(d2, clampd) >> sh) << 13) | static_cast<uint32_t>(icur);
      net_insert(key, icur == self ? kKey32Inf : kk);
    }
    const uint32_t kth = key[KT - 2];
    const long long dmax = (static_cast<long long>(key32_d(kth) + 1) << sh) - 1;
    if (kth == kKey32Inf || dmax >= b.bound) {
      if (attempt == 0 && B + 2 <= tc.bmax) {
        B += 2;
        continue;
      }
      return false;
    }
    if (key32_d(kth) >= key32_d(key[KT - 1])) return false;
    bool tied = false;
#pragma unroll
    for (int t = 0; t < KT - 2; ++t)
      if (t >= KT - (k + 1)) tied = tied || (key32_d(key[t]) == key32_d(key[t + 1]));
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
      if (t >= KMAX - k) slot[t] = lslot[key[t] & 0x1FFFu];
    if (tied) sort_exact<KMAX>(w, qx, qy, k, slot);
    return true;
  }
  return false;
}

template <int KMAX, bool kAlign>
__global__ __launch_bounds__(kBlock) void k_knn(DevWs w, FastCfg f, TileCfg tc, int k,
                                                int32_t* __restrict__ nbr,
                                                long long* __restrict__ d2out, AlignArgs a) {
  __shared__ int lcell[kTileCells + 1];
  __shared__ int2 lpos[kTilePts];
  __shared__ int lslot[kTilePts];
  __shared__ int s_part[kBlock / 64];
  __shared__ int s_defer;
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int tile = tile_index(blockIdx.x, gridDim.x);
  const int G = w.G, L = w.box, gm = G - 1;
  const int ty = tile / tc.ntx, tx0 = (tile - ty * tc.ntx) * tc.tc;
  const int tce = min(tc.tc, G - tx0);
  const int total = min(w.start[w.C], w.n);
  const int64_t rowbase = static_cast<int64_t>(ty) * G;
  const int q_beg = w.start[rowbase + tx0];
  const int q_end = min(w.start[rowbase + tx0 + tce], total);
  if (q_beg >= q_end) {
    if (threadIdx.x == 0) w.qcnt[tile] = 0;
    return;
  }
  const int h = tc.h, W = tce + 2 * h, R = 2 * h + 1, ncells = R * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_defer = 0;
  __syncthreads();  // s_defer is live before any lane can defer a query
  bool staged = h > 0 && ncells <= kTileCells;
  if (staged) {
    // Cell counts of the halo, row-major over (rho, j), prefix-summed into lcell.
    constexpr int kPer = (kTileCells + kBlock - 1) / kBlock;
    const int c0 = threadIdx.x * kPer;
    int cnt[kPer];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      cnt[i] = 0;
      const int c = c0 + i;
      if (c < ncells) {
        const int rho = c / W, j = c - rho * W;
        const int64_t cell = static_cast<int64_t>((ty - h + rho) & gm) * G + ((tx0 - h + j) & gm);
        cnt[i] = w.start[cell + 1] - w.start[cell];
      }
      sum += cnt[i];
    }
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) s_part[wave] = incl;
    __syncthreads();
    int run = incl - sum, grand = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      if (q < wave) run += s_part[q];
      grand += s_part[q];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      if (c0 + i < ncells) lcell[c0 + i] = run;
      run += cnt[i];
    }
    if (threadIdx.x == 0) lcell[ncells] = grand;
    staged = grand <= kTilePts;
    __syncthreads();
    if (staged) {
      // Copy each halo row as its (up to three) physically contiguous pieces.
      for (int rho = 0; rho < R; ++rho) {
        const int v = ty - h + rho;
        const int sy = v < 0 ? -L : (v >= G ? L : 0);
        const int64_t prow = static_cast<int64_t>(v & gm) * G;
        const int uL = tx0 - h, uR = tx0 + tce + h - 1;
        int p0 = uL;
        while (p0 <= uR) {
          const int p1 = p0 < 0 ? min(uR, -1) : (p0 < G ? min(uR, G - 1) : uR);
          const int sx = p0 < 0 ? -L : (p0 >= G ? L : 0);
          const int ga = w.start[prow + (p0 & gm)];
          const int ge = w.start[prow + (p1 & gm) + 1];
          const int lo = lcell[rho * W + (p0 - uL)];
          for (int i = threadIdx.x; i < ge - ga; i += kBlock) {
            const int4 e = w.sorted[ga + i];
            lpos[lo + i] = make_int2(e.x + sx, e.y + sy);
            lslot[lo + i] = ga + i;
          }
          p0 = p1 + 1;
        }
      }
    }
    __syncthreads();
  }

  const int lhome = staged ? lcell[h * W + h] : 0;
  for (int s = q_beg + static_cast<int>(threadIdx.x); s < q_end; s += kBlock) {
    const int4 q = w.sorted[s];
    int slot[KMAX];
    bool ok;
    if (staged) {
      const int jh = (q.x >> w.log2_w) - tx0 + h;
      ok = knn_lds<KMAX>(w, f, tc, lcell, lpos, lslot, W, jh, lhome + (s - q_beg), q.x, q.y, k, slot);
    } else {
      ok = knn_fast<KMAX>(w, f, s, q.x, q.y, k, total, slot);
    }
    if (ok) {
      finish_query<KMAX, kAlign>(w, s, q, slot, k, nbr, d2out, a);
    } else {
      w.queue[q_beg + atomicAdd(&s_defer, 1)] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) w.qcnt[tile] = s_defer;
}

// Cell (dx, dy) number q of ring r (q < 8r; the single cell of ring 0),
// walking the perimeter from (-r, -r) as the exact lane search does.
__device__ __forceinline__ void ring_cell(int r, int q, int& dx, int& dy) {
  if (r == 0) {
    dx = dy = 0;
    return;
  }
  const int side = q / (2 * r), p = q - side * 2 * r;
  dx = side == 0 ? -r + p : (side == 1 ? r : (side == 2 ? r - p : -r));
  dy = side == 0 ? -r : (side == 1 ? -r + p : (side == 2 ? r : r - p));
}

// One deferred query searched by a whole wavefront: for each ring the 64
// lanes take up to 64 cells at a time, skip cells whose nearest point is
// farther than the current k-th neighbour, flatten the candidates of the rest
// across the lanes and evaluate 64 per round; candidates that beat the
// current k-th are merged one by one (their keys broadcast to every lane,
// which all hold the same list).  Same stop rule as the lane search.
template <int KMAX>
__device__ __forceinline__ bool knn_wave(const DevWs& w, int s, const int4& q, int k, int total,
                                         int (&slot)[KMAX]) {
  const int lane = threadIdx.x & 63;
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom g(q.x, q.y, w);
  TopK<KMAX, true> top;
  top.init(k);
  for (int r = 0; r <= g.rmax; ++r) {
    const int ncell = r == 0 ? 1 : 8 * r;
    for (int c0 = 0; c0 < ncell; c0 += 64) {
      int beg = 0, cnt = 0;
      if (c0 + lane < ncell) {
        int dx, dy;
        ring_cell(r, c0 + lane, dx, dy);
        if (dx >= g.lo && dx <= g.hi && dy >= g.lo && dy <= g.hi) {
          const long long gx = axis_gap(dx, g.ox, cw, sh), gy = axis_gap(dy, g.oy, cw, sh);
          if (gx * gx + gy * gy <= key_bound_d2(top.worst())) {
            const int64_t c = static_cast<int64_t>((g.hy + dy) & gm) * w.G + ((g.hx + dx) & gm);
            beg = w.start[c];
            cnt = max(min(w.start[c + 1], total) - beg, 0);
          }
        }
      }
      int incl = cnt;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
      }
      const int ntot = __shfl(incl, 63, 64);
      const int excl = incl - cnt;
      for (int j0 = 0; j0 < ntot; j0 += 64) {
        const int j = j0 + lane;
        int lo = 0;  // owner lane of flattened candidate j: last lane with excl <= j
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int probe = lo + step;
          const int e = __shfl(excl, probe < 64 ? probe : 63, 64);
          if (probe < 64 && e <= j) lo = probe;
        }
        const int ob = __shfl(beg, lo, 64), oe = __shfl(excl, lo, 64);
        unsigned long long kk = ~0ull;
        int t = -1;
        if (j < ntot) {
          t = ob + (j - oe);
          if (t != s) {
            const int4 e = w.sorted[t];
            const int ex = wrap_axis(e.x - q.x, sh), ey = wrap_axis(e.y - q.y, sh);
            kk = pack_key(static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey, e.z);
          }
        }
        unsigned long long better = __ballot(kk < top.worst());
        while (better) {
          const int l = __ffsll(static_cast<long long>(better)) - 1;
          better &= better - 1;
          const unsigned long long bk = __shfl(kk, l, 64);
          const int bt = __shfl(t, l, 64);
          if (bk < top.worst()) top.push(bk, bt);
        }
      }
    }
    if (key_bound_d2(top.worst()) < g.ring_bound(r, cw)) break;
  }
#pragma unroll
  for (int t = 0; t < KMAX; ++t) slot[t] = top.slot[t];
  return top.worst() != ~0ull;
}

// The deferred queries, tile by tile: a tile with many of them gives each
// lane one (exact lane search); a tile with a few searches each with the whole
// wavefront, so that a single long search is not one lane's serial chain.
template <int KMAX, bool kAlign>
__global__ __launch_bounds__(kBlock) void k_knn_rest(DevWs w, TileCfg tc, int ntiles, int k,
                                                     int32_t* __restrict__ nbr,
                                                     long long* __restrict__ d2out, AlignArgs a) {
  if (!ws_ready(w)) return;
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (kBlock / 64);
  const int total = min(w.start[w.C], w.n);
  for (int tile = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); tile < ntiles; tile += waves) {
    const int cnt = w.qcnt[tile];
    if (cnt <= 0) continue;
    const int ty = tile / tc.ntx, tx0 = (tile - ty * tc.ntx) * tc.tc;
    const int base = w.start[static_cast<int64_t>(ty) * w.G + tx0];
    if (cnt >= 16) {
      for (int i = lane; i < cnt; i += 64) {
        const int s = w.queue[base + i];
        if (static_cast<uint32_t>(s) >= static_cast<uint32_t>(total)) continue;
        const int4 q = w.sorted[s];
        int slot[KMAX];
        if (!knn_exact<KMAX>(w, s, q.x, q.y, k, total, slot)) {
          set_err(w.hdr, NM_E_RANGE);  // fewer than k other particles were binned
          continue;
        }
        finish_query<KMAX, kAlign>(w, s, q, slot, k, nbr, d2out, a);
      }
    } else {
      for (int i = 0; i < cnt; ++i) {
        const int s = w.queue[base + i];
        if (static_cast<uint32_t>(s) >= static_cast<uint32_t>(total)) continue;
        const int4 q = w.sorted[s];
        int slot[KMAX];
        const bool ok = knn_wave<KMAX>(w, s, q, k, total, slot);
        if (lane == 0) {
          if (ok)
            finish_query<KMAX, kAlign>(w, s, q, slot, k, nbr, d2out, a);
          else
            set_err(w.hdr, NM_E_RANGE);
        }
      }
    }
  }
}

// Tile geometry: a halo of h cells supports blocks up to 2h + 1 cells (the
// staged frame is the minimum image while G >= 2h + 2); the tile width aims at
// about 224 queries per tile and a halo of at most ~1800 particles at the mean
// density.
TileCfg tile_cfg(const DevWs& w, const FastCfg& f) {
  TileCfg t{1, 0, w.G, 0};
  const double rho = static_cast<double>(w.n) / static_cast<double>(w.C);  // particles per cell
  int h = f.bmax > 0 ? min(4, (f.bmax + 1) / 2) : 0;
  while (h > 0 && w.G < 2 * h + 2) --h;
  int tc = static_cast<int>(224.0 / (rho > 1e-9 ? rho : 1e-9));
  if (h > 0) {
    const int R = 2 * h + 1;
    const int by_cells = kTileCells / R - 2 * h;
    const int by_pts = static_cast<int>(1800.0 / (R * (rho > 1e-9 ? rho : 1e-9))) - 2 * h;
    tc = min(tc, min(by_cells, by_pts));
  }
  tc = max(1, min(tc, w.G));
  t.tc = tc;
  t.h = (h > 0 && (2 * h + 1) * (tc + 2 * h) <= kTileCells) ? h : 0;
  t.ntx = (w.G + tc - 1) / tc;
  t.bmax = t.h > 0 ? min(2 * t.h + 1, f.bmax) : 0;
  return t;
}

template <int KMAX, bool kAlign>
hipError_t launch_t(const DevWs& w, const FastCfg& f, int k, int32_t* nbr, long long* d2,
                    const AlignArgs& a, hipStream_t s) {
  const TileCfg tc = tile_cfg(w, f);
  const int ntiles = w.G * tc.ntx;
  hipLaunchKernelGGL((k_knn<KMAX, kAlign>), dim3(ntiles), dim3(kBlock), 0, s, w, f, tc, k, nbr, d2, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nr = min((ntiles + 3) / 4, 1024);
  hipLaunchKernelGGL((k_knn_rest<KMAX, kAlign>), dim3(nr), dim3(kBlock), 0, s, w, tc, ntiles, k, nbr,
                     d2, a);
  return hipGetLastError();
}

// Register list sizes compiled; a request for k uses the smallest KMAX >= k.
template <class F>
hipError_t dispatch_k(int k, F&& f) {
  if (k <= 1) return f(std::integral_constant<int, 1>{});
  if (k <= 2) return f(std::integral_constant<int, 2>{});
  if (k <= 4) return f(std::integral_constant<int, 4>{});
  if (k <= 6) return f(std::integral_constant<int, 6>{});
  if (k <= 7) return f(std::integral_constant<int, 7>{});
  if (k <= 8) return f(std::integral_constant<int, 8>{});
  if (k <= 12) return f(std::integral_constant<int, 12>{});
  if (k <= 16) return f(std::integral_constant<int, 16>{});
  if (k <= 20) return f(std::integral_constant<int, 20>{});
  if (k <= 24) return f(std::integral_constant<int, 24>{});
  return f(std::integral_constant<int, 32>{});
}

}  // namespace

// Fast-path limits for a grid: block sides up to the largest B whose
// offsets keep 32-bit squared distances exact ((B / 2 + 1) w < 2^15) and whose
// block cannot meet itself around the box (B + 2 <= G).  `block` > 0 fixes the
// side, 0 picks it per query, < 0 disables the fast path.
FastCfg fast_cfg(const DevWs& w, int k, int block) {
  (void)k;
  FastCfg f{0, 0, 1.6f};
  if (block < 0) return f;
  int bmax = kMaxB;
  while (bmax >= 3 && ((static_cast<long long>((bmax >> 1) + 1) << w.log2_w) >= 32768 || bmax + 2 > w.G))
    --bmax;
  if (bmax < 3) return f;
  f.bmax = bmax;
  if (block > 0) {
    if (block > bmax) return FastCfg{0, 0, 1.6f};
    f.bfix = block;
  }
  return f;
}

hipError_t launch_knn(const DevWs& w, int k, int block, int32_t* nbr, long long* d2, hipStream_t s) {
  const FastCfg f = fast_cfg(w, k, block);
  AlignArgs a{};
  return dispatch_k(k, [&](auto km) { return launch_t<decltype(km)::value, false>(w, f, k, nbr, d2, a, s); });
}

hipError_t launch_knn_align(const DevWs& w, int k, int block, const nm_params* p, const float* theta,
                            int32_t* nbr, int32_t* x_out, int32_t* y_out, float* theta_out,
                            hipStream_t s) {
  const FastCfg f = fast_cfg(w, k, block);
  AlignArgs a{p->v0, p->eta, p->include_self, theta, x_out, y_out, theta_out};
  return dispatch_k(k, [&](auto km) {
    return launch_t<decltype(km)::value, true>(w, f, k, nbr, nullptr, a, s);
  });
}

}  // namespace nm
