// knn.hip -- topological neighbour lists (Sec. III: each particle interacts
// with its k nearest neighbours), the fused step kernel and the field-of-view
// lists.
//
// The kernels work on strips of cells staged in LDS (see "Strips" below);
// queries that a strip cannot serve from LDS run the global-memory paths
// here, one lane per query, queries taken in cell order so that a
// wavefront's queries are spatial neighbours and read the same cached cells.
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
#include "fov.h"
#include "strip.h"

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

// Exact squared distance from a staged query (packed position pq, or x and
// y) to staged particle i: the 16-bit differences are exact inside a block.
template <bool kWide>
__device__ __forceinline__ long long staged_d2(const int* lpos, int i, int pq, int pqy) {
  if (kWide) {
    const int2 c = reinterpret_cast<const int2*>(lpos)[i];
    const long long dx = c.x - pq, dy = c.y - pqy;
    return dx * dx + dy * dy;
  }
  return rel_d2(lpos[i], pq);
}

// sort_exact for staged neighbours (LDS indices), from the staged positions
// and particle indices.
template <int KMAX, bool kWide>
__device__ __forceinline__ void sort_exact_lds(const int* lpos, const int* lidx, int pq, int pqy, int k,
                                               int (&lds)[KMAX]) {
  unsigned long long kk[KMAX];
#pragma unroll
  for (int t = 0; t < KMAX; ++t)
    kk[t] = t >= KMAX - k ? pack_key(staged_d2<kWide>(lpos, lds[t], pq, pqy), lidx[lds[t]]) : 0ull;
  // the unused prefix holds 0, below every real key, so it stays in front
#pragma unroll
  for (int i = 1; i < KMAX; ++i) {
#pragma unroll
    for (int j = i; j > 0; --j) {
      const bool swap = kk[j] < kk[j - 1];
      const unsigned long long a = kk[j - 1], c = kk[j];
      const int sa = lds[j - 1], sc = lds[j];
      kk[j - 1] = swap ? c : a;
      kk[j] = swap ? a : c;
      lds[j - 1] = swap ? sc : sa;
      lds[j] = swap ? sa : sc;
    }
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

// Outputs of one query from the slots of its k neighbours: the list row (and
// squared distances), and for the fused step Eq. (2) and Eq. (1).
template <int KMAX, bool kAlign>
__device__ __forceinline__ void finish_query(const DevWs& w, int s, const int4& q, const int (&slot)[KMAX],
                                             int k, int32_t* __restrict__ nbr,
                                             long long* __restrict__ d2out, const AlignArgs& a) {
  int32_t* row = nbr + static_cast<int64_t>(q.z) * k;
  const int sh = 32 - w.log2_box;
  double sx = 0.0, sy = 0.0;
  int rv[KMAX];
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    rv[t] = 0;
    if (t >= KMAX - k) {
      const int4 e = w.sorted[slot[t]];
      if constexpr (kRowVec<KMAX>)
        rv[t] = e.z;
      else
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
  if constexpr (kRowVec<KMAX>) store_row<KMAX>(row, rv, k);
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
  const float th = heading_update(ax, ay, xi.x, xi.y, noise_angle(static_cast<uint32_t>(q.w)), a.eta,
                                  a.theta + q.z, a.variant);

  // Eq. (1): move with the heading at time t (or the new one), rounded to the grid.
  int ddx, ddy;
  move_step(a.v0, own.x, own.y, th, a.variant, ddx, ddy);
  const int mask = w.box - 1;
  a.x_out[q.z] = (q.x + ddx) & mask;
  a.y_out[q.z] = (q.y + ddy) & mask;
  a.theta_out[q.z] = th;
}

// ---------------------------------------------------------------------------
// Strips.  A workgroup owns a strip of tw x th cells (tw = 1 to 16 columns,
// about 256 queries) and stages the halo of W = tw + 2 hx columns by
// R = th + 2 hy rows into LDS: the LDS offset of each halo row, and every
// particle's position in the strip's periodic image relative to the halo
// corner, with its particle index.  A query's block is all W columns of
// Bq consecutive halo rows around its own, so its candidates are one
// contiguous LDS range, read several at a time.  Positions are a packed pair
// of 16-bit offsets whose differences are taken in 16-bit wrap-around
// arithmetic (exact: every block spans under 2^15 units), so that a squared
// distance is one packed subtract and one 16-bit dot product; where a block
// spans more (sparse systems) they are int32 pairs with 64-bit distances.
// A strip whose halo holds more particles than fit searches global memory,
// or, in the sub-strip kernel, runs as sub-strips staged in turn.
// Uncertified queries are finished at the end of the strip by the exact
// search.
// ---------------------------------------------------------------------------
constexpr int kDeferCap = 128;    // uncertified queries listed in LDS per strip
constexpr double kReachX = 1.25;  // strip half width, in mean k-th-neighbour radii
constexpr double kReachY = 1.2;   // halo height over the expected block height


// Block height for a staged query: fixed, or such that the block edge sits
// `reach` mean k-th-neighbour radii away, the density taken from the three
// halo rows around the query's (3 W cells).
__device__ __forceinline__ int strip_block_rows(const FastCfg& f, const int* rbase, int W, int cy,
                                                int k) {
  if (f.bfix > 0) return f.bfix;
  const int n3 = rbase[cy + 2] - rbase[cy - 1];
  const float rk = sqrtf(static_cast<float>(k) * static_cast<float>(3 * W) /
                         (3.14159265f * fmaxf(static_cast<float>(n3), 0.5f)));
  return max(static_cast<int>(ceilf(2.0f * f.reach * rk)) + 1, 1);
}

// Geometry of a query's block in a strip: halo rows [r0, r0 + Bq), all W
// columns; squared distance to the nearest point outside it, and the shift
// that fits that bound in the distance field of a 32-bit key.
struct StripBlock {
  int r0;
  long long bound;
  int sh;
};

__device__ __forceinline__ StripBlock strip_block(int rx, int oy, int cy, int Bq, int W, int lw) {
  const int cw = 1 << lw;
  const int half = Bq >> 1;
  const int lo = (Bq & 1) ? -half : -half + (oy >= (cw >> 1) ? 1 : 0);
  StripBlock b;
  b.r0 = cy + lo;
  const int gl = rx + 1, gr = W * cw - rx;
  const int gd = oy - lo * cw + 1, gu = (lo + Bq) * cw - oy;
  const long long m = min(min(gl, gr), min(gd, gu));
  b.bound = m * m;
  const int bits = 64 - __clzll(b.bound);
  b.sh = bits > kDBits ? bits - kDBits : 0;
  return b;
}

// Candidate filters of the strip search: every staged particle, or those
// inside the query's field of view.
struct NoFilter {
  static constexpr bool kActive = false;
};

struct FovFilter {
  static constexpr bool kActive = true;
  FovHeading h;
  __device__ bool visible_short(int dx, int dy, int d2) const { return fov_visible_short(dx, dy, d2, h); }
  __device__ bool visible(long long dx, long long dy) const { return fov_visible(dx, dy, h); }
};

// Certified search of one staged query over LDS.  self: the query's LDS
// index; (pq, pqy): its relative position (narrow: packed pair in pq);
// (rx, oy): its x offset from the halo corner and y offset in its cell; cy:
// its halo row.  True with `lds` filled (LDS indices of the k nearest that
// pass `filt`, in order) when they are certified.  Anything outside the
// block is farther than its edge whatever the filter, so the certificate
// holds for the filtered lists too.
template <int KMAX, bool kWide, class Filter>
__device__ __forceinline__ bool strip_search(const DevWs& w, const TileCfg& tc, const int* rbase,
                                             const int* lpos, const int* lidx, int W, int self,
                                             int pq, int pqy, int rx, int oy, int cy, int k, int Bq,
                                             const Filter& filt, int (&lds)[KMAX]) {
  constexpr int KT = KMAX + 1;
  // Without a filter the query's own key (distance 0, its LDS index) goes
  // through the network with the others, one more list entry, and is taken
  // out at the end: cheaper than masking every candidate against it.
  constexpr bool kWithSelf = !Filter::kActive;
  constexpr int KS = kWithSelf ? KT + 1 : KT;
  const int2* lpos2 = reinterpret_cast<const int2*>(lpos);
  if (Bq > tc.bmax) return false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const StripBlock b = strip_block(rx, oy, cy, Bq, W, w.log2_w);
    uint32_t kl[KS];
#pragma unroll
    for (int t = 0; t < KS; ++t) kl[t] = (t < KS - (k + 1 + (kWithSelf ? 1 : 0))) ? 0u : kKey32Inf;
    const int sh = b.sh;
    // wide strips: the bound rounded down to fp32 (so that a clamped field
    // stays below 2^19) and the exact scale 2^-sh
    float boundf = static_cast<float>(b.bound);
    if (static_cast<long long>(boundf) > b.bound) boundf = nextafterf(boundf, 0.0f);
    const float scale = ldexpf(1.0f, -sh);
    const int a = rbase[b.r0], e = rbase[b.r0 + Bq];
    // One round: candidates i .. i + kUnroll - 1.  Only the last round of a
    // block (tail) can pass its end; it masks what lies beyond.
    auto round = [&](int i, bool tail) {
      uint32_t kk[kUnroll];
      if (kWide) {
        // fp32 squared distances: the offsets are exact (below 2^24), the
        // square and the sum round twice (relative error below 2^-23, an
        // eighth of a distance-field unit), so every field is within one of
        // the exact one; the certificate below widens its margins to match.
        int2 pc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) pc[u] = lpos2[i + u];  // (buffer padded by kUnroll)
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int dxi = pc[u].x - pq, dyi = pc[u].y - pqy;
          const float dx = static_cast<float>(dxi), dy = static_cast<float>(dyi);
          const float d2 = fmaf(dy, dy, dx * dx);
          kk[u] = (static_cast<uint32_t>(fminf(d2, boundf) * scale) << 13) | static_cast<uint32_t>(i + u);
          if constexpr (Filter::kActive)
            if (!filt.visible(static_cast<long long>(dxi), static_cast<long long>(dyi))) kk[u] = kKey32Inf;
        }
      } else {
        int pc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) pc[u] = lpos[i + u];  // (buffer padded by kUnroll)
        const uint32_t clampd = static_cast<uint32_t>(b.bound);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t d2 = rel_d2_u(pc[u], pq);
          kk[u] = ((min(d2, clampd) >> sh) << 13) | static_cast<uint32_t>(i + u);
          if constexpr (Filter::kActive) {
            const short2v dd = __builtin_bit_cast(short2v, pc[u]) - __builtin_bit_cast(short2v, pq);
            if (!filt.visible_short(dd[0], dd[1], static_cast<int>(d2))) kk[u] = kKey32Inf;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        uint32_t c = kk[u];
        if (!kWithSelf && i + u == self) c = kKey32Inf;
        if (tail && i + u >= e) c = kKey32Inf;
        net_insert(kl, c);
      }
    };
    const int full = a + ((e - a) & ~(kUnroll - 1));
    for (int i = a; i < full; i += kUnroll) round(i, false);
    if (full < e) round(full, true);
    uint32_t key[KT];
    if constexpr (kWithSelf) {
      // the first entry not below the query's own key is that key (it is in
      // the list unless more than KS duplicates of lower index precede it)
      const uint32_t selfkey = static_cast<uint32_t>(self);
#pragma unroll
      for (int t = 0; t < KT; ++t) key[t] = kl[t] < selfkey ? kl[t] : kl[t + 1];
    } else {
#pragma unroll
      for (int t = 0; t < KT; ++t) key[t] = kl[t];
    }
    // Certificate (fields exact, or within one of exact on wide strips: M = 2):
    // the k-th lies inside the block, the (k+1)-th is strictly farther than
    // the k-th, and fields closer than M + 1 inside the k are re-sorted by
    // the exact (d^2, index).
    constexpr uint32_t M = kWide ? 2u : 0u;
    const uint32_t kth = key[KT - 2];
    const long long dmax = (static_cast<long long>(key32_d(kth) + 1 + M / 2) << sh) - 1;
    if (kth == kKey32Inf || dmax >= b.bound) {
      if (attempt == 0 && Bq + 2 <= tc.bmax) {
        Bq += 2;
        continue;
      }
      return false;
    }
    if (key32_d(kth) + M >= key32_d(key[KT - 1])) return false;
    bool tied = false;
#pragma unroll
    for (int t = 0; t < KT - 2; ++t)
      if (t >= KT - (k + 1)) tied = tied || (key32_d(key[t + 1]) - key32_d(key[t]) <= M);
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
      if (t >= KMAX - k) lds[t] = static_cast<int>(key[t] & 0x1FFFu);
    if (tied) sort_exact_lds<KMAX, kWide>(lpos, lidx, pq, pqy, k, lds);
    return true;
  }
  return false;
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
// current k-th are merged one by one (each broadcast to every lane; the list
// itself is spread over the lanes).  Same stop rule as the lane search.
// Candidates that fail `filt` are skipped.
template <int KMAX, class Filter = NoFilter>
__device__ __forceinline__ bool knn_wave(const DevWs& w, int s, const int4& q, int k, int total,
                                         int (&slot)[KMAX], const Filter& filt = Filter{}) {
  const int lane = threadIdx.x & 63;
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom g(q.x, q.y, w);
  // The list is spread over the wave: lane t < k holds the t-th nearest so
  // far (key and slot), so an insertion costs each lane one compare with its
  // own entry and its left neighbour's instead of a pass over a whole list.
  unsigned long long mine = ~0ull;
  int mslot = -1;
  unsigned long long worst = ~0ull;  // the k-th entry, in every lane
  for (int r = 0; r <= g.rmax; ++r) {
    const int ncell = r == 0 ? 1 : 8 * r;
    for (int c0 = 0; c0 < ncell; c0 += 64) {
      int beg = 0, cnt = 0;
      if (c0 + lane < ncell) {
        int dx, dy;
        ring_cell(r, c0 + lane, dx, dy);
        if (dx >= g.lo && dx <= g.hi && dy >= g.lo && dy <= g.hi) {
          const long long gx = axis_gap(dx, g.ox, cw, sh), gy = axis_gap(dy, g.oy, cw, sh);
          if (gx * gx + gy * gy <= key_bound_d2(worst)) {
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
            bool keep = true;
            if constexpr (Filter::kActive) keep = filt.visible(ex, ey);
            if (keep) kk = pack_key(static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey, e.z);
          }
        }
        unsigned long long better = __ballot(kk < worst);
        while (better) {
          const int l = __ffsll(static_cast<long long>(better)) - 1;
          better &= better - 1;
          const unsigned long long bk = __shfl(kk, l, 64);
          const int bt = __shfl(t, l, 64);
          if (bk < worst) {
            const unsigned long long left = __shfl_up(mine, 1, 64);
            const int lslot = __shfl_up(mslot, 1, 64);
            if (lane < k && bk < mine) {
              const bool shift = lane > 0 && bk < left;  // the new key lands before this entry
              mine = shift ? left : bk;
              mslot = shift ? lslot : bt;
            }
            worst = __shfl(mine, k - 1, 64);
          }
        }
      }
    }
    if (key_bound_d2(worst) < g.ring_bound(r, cw)) break;
  }
  // the list in every lane, in the lane search's layout (nearest first at
  // KMAX - k)
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    const int src = t - (KMAX - k);
    const int v = __shfl(mslot, src < 0 ? 0 : src, 64);
    slot[t] = src < 0 ? -1 : v;
  }
  return worst != ~0ull;
}

// One uncertified query searched by its own lane (exact ring search).
template <int KMAX, bool kAlign>
__device__ __forceinline__ void exact_lane(const DevWs& w, int s, int k, int total,
                                           int32_t* __restrict__ nbr, long long* __restrict__ d2out,
                                           const AlignArgs& a) {
  const int4 q = w.sorted[s];
  int slot[KMAX];
  if (knn_exact<KMAX>(w, s, q.x, q.y, k, total, slot))
    finish_query<KMAX, kAlign>(w, s, q, slot, k, nbr, d2out, a);
  else
    set_err(w.hdr, NM_E_RANGE);  // fewer than k other particles were binned
}

// Cells of strip `tile`: columns [x0, x0 + tw), rows [y0, y0 + ty).
struct StripBox {
  int x0, y0, ty;
};

__device__ __forceinline__ StripBox strip_box(const DevWs& w, const TileCfg& tc, int tile) {
  StripBox b;
  const int tyi = tile / tc.ntx, txi = tile - tyi * tc.ntx;
  b.x0 = txi * tc.tw;
  b.y0 = tyi * tc.th;
  b.ty = min(tc.th, w.G - b.y0);
  return b;
}


// What a strip does when its halo holds more particles than LDS.  The two
// are compiled as separate kernels: the sub-strip loop costs the common
// (fitting) strips some 10% when it shares their kernel, so the choice is a
// grid parameter that the autotuner weighs like the cell width.
enum StripMode {
  kOverflowGlobal = 0,  // search its queries in global memory (fast block search)
  kOverflowSplit = 1,   // run it as sub-strips of whole rows, each staged in turn
  kFieldOfView = 2,     // field-of-view lists (a.theta, a.cone); such a strip's
                        // queries and the uncertified ones take the exact search
};

template <int KMAX, bool kAlign, int kMode>
__device__ __forceinline__ void knn_tile_body(const DevWs& w, const FastCfg& f, const TileCfg& tc,
                                              int k, int32_t* __restrict__ nbr,
                                              long long* __restrict__ d2out, const AlignArgs& a,
                                              int tile) {
  // packed 16-bit pairs, or int32 pairs (wide); padded so that a round of
  // kUnroll reads past a block's last candidate stays inside the buffer
  __shared__ int2 lpos_store[kStripPts / 2 + kUnroll];
  __shared__ int lidx[kStripPts];          // particle index of each staged particle
  __shared__ int s_rbase[kStripRows + 1];  // LDS offset of each halo row
  __shared__ int s_ga0[kStripRows];        // first slot of the row's first piece
  __shared__ int s_n0[kStripRows];         // particles in the row's first piece
  __shared__ int s_ga1[kStripRows];        // first slot of its second piece (x wrap)
  __shared__ int s_qoff[kStripRows + 1];   // query prefix over the strip's rows
  __shared__ int s_tself[kStripRows];      // LDS index of each strip row's first query
  __shared__ int s_wsum[kBlock / 64];
  __shared__ int s_defer;
  __shared__ int s_dq[kDeferCap];  // slots of the strip's uncertified queries
  __shared__ uint8_t s_rowid[kStripPts];   // halo row of each staged particle
  __shared__ uint16_t s_qmap[kStripPts];   // LDS index of each of the strip's queries
  __shared__ int s_sub[kStripRows + 1];    // sub-strip rows (kOverflowSplit)
  __shared__ int s_nsub;
  int* lpos = reinterpret_cast<int*>(lpos_store);
  if (!ws_ready(w)) {
    if (tile == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const StripBox tb = strip_box(w, tc, tile);
  const int G = w.G, lw = w.log2_w;
  const int total = min(w.start[w.C], w.n);
  const int tw = tc.tw, hy = tc.hy;
  // The sub-strip kernel (chosen for clustered systems) takes each strip's
  // halo width from the strip's own density, never wider than the grid's:
  // dense strips get narrower blocks (6% less time at k = 20 on the clustered
  // state; the extra pass over the strip's rows costs the default kernel 7%
  // on uniform systems, which keep the grid's width).
  int hx = tc.hx;
  if (kMode == kOverflowSplit && hx > 1) {
    int q = 0;
    if (static_cast<int>(threadIdx.x) < tb.ty) {
      const int64_t prow = static_cast<int64_t>(tb.y0 + threadIdx.x) * G;
      q = max(min(w.start[prow + tb.x0 + tw], total) - w.start[prow + tb.x0], 0);
    }
    int nqs;
    (void)block_exclusive_scan(q, s_wsum, &nqs);
    if (nqs > 0) {
      const float rho = static_cast<float>(nqs) / static_cast<float>(tw * tb.ty);
      int hs = static_cast<int>(
          ceilf(static_cast<float>(kReachX) * sqrtf(static_cast<float>(k) / (3.14159265f * rho))));
      if (f.bfix > 0) hs = max(hs, f.bfix / 2);
      hx = max(1, min(hs, tc.hx));
    }
  }
  const int W = tw + 2 * hx;
  const int uL = tb.x0 - hx;
  const int lane = threadIdx.x & 63;
  const int ox0 = uL << lw;  // halo corner x (strip image)
  // the (sub-)strip being run: first row, rows, halo corner y (strip image)
  int y0_cur = tb.y0, ty_cur = tb.ty, oy0 = (tb.y0 - hy) << lw;
  const bool wide = tc.wide != 0;

  StripGeo geo{tb.x0, tb.y0, tb.ty, tw, hx, hy, wide};
  // built at each use: an aggregate of LDS addresses shared by the lambdas
  // below would become a constant global, which the target cannot express
  auto strip_lds = [&]() {
    return StripLds{lpos_store, lidx, s_rbase, s_ga0, s_n0, s_ga1, s_qoff, s_tself, s_wsum, s_rowid, s_qmap};
  };
  if (threadIdx.x == 0) s_defer = 0;

  auto defer = [&](int slot_s) {
    const int pos = atomicAdd(&s_defer, 1);
    if (pos < kDeferCap)
      s_dq[pos] = slot_s;
    else
      w.dflag[slot_s] = 1;  // overflow of the list: found again below by its flag
  };
  auto row_of = [&](int qi) {  // strip row of query qi
    int r = 0;
#pragma unroll
    for (int step = kRowStep; step > 0; step >>= 1)
      if (r + step < ty_cur && s_qoff[r + step] <= qi) r += step;
    return r;
  };
  // One staged query (LDS index self, halo row cy): the certified search over
  // LDS, then its outputs with the neighbours' indices from LDS and their
  // unit vectors gathered by slot; otherwise it is deferred to the exact search.
  auto staged_query = [&](int self, int cy) {
    int rx, oy, pq, pqy;
    if (wide) {
      const int2 p2 = lpos_store[self];
      pq = p2.x;
      pqy = p2.y;
      rx = p2.x;
      oy = p2.y & ((1 << lw) - 1);
    } else {
      pq = lpos[self];
      pqy = 0;
      rx = pq & 0xFFFF;
      oy = (pq >> 16) & ((1 << lw) - 1);
    }
    const int Bq = strip_block_rows(f, s_rbase, W, cy, k);
    int nb[KMAX];
    bool ok;
    if constexpr (kMode == kFieldOfView) {
      const FovFilter filt{fov_heading(a.theta[lidx[self]], a.cone)};
      ok = wide ? strip_search<KMAX, true>(w, tc, s_rbase, lpos, lidx, W, self, pq, pqy, rx, oy, cy, k, Bq,
                                           filt, nb)
                : strip_search<KMAX, false>(w, tc, s_rbase, lpos, lidx, W, self, pq, pqy, rx, oy, cy, k, Bq,
                                            filt, nb);
    } else {
      ok = wide ? strip_search<KMAX, true>(w, tc, s_rbase, lpos, lidx, W, self, pq, pqy, rx, oy, cy, k, Bq,
                                           NoFilter{}, nb)
                : strip_search<KMAX, false>(w, tc, s_rbase, lpos, lidx, W, self, pq, pqy, rx, oy, cy, k, Bq,
                                            NoFilter{}, nb);
    }
    const int s = strip_slot(strip_lds(), self);
    if (!ok) {
      defer(s);
      return;
    }
    const int qi = lidx[self];
    int32_t* row = nbr + static_cast<int64_t>(qi) * k;
    double sx = 0.0, sy = 0.0;
    int rv[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
      rv[t] = 0;
      if (t >= KMAX - k) {
        const int i = nb[t];
        if constexpr (kRowVec<KMAX>)
          rv[t] = lidx[i];
        else
          row[t - (KMAX - k)] = lidx[i];
        if (!kAlign && d2out)
          d2out[static_cast<int64_t>(qi) * k + t - (KMAX - k)] =
              wide ? staged_d2<true>(lpos, i, pq, pqy) : staged_d2<false>(lpos, i, pq, pqy);
        if (kAlign) {
          const double2 u = w.cs[2 * strip_slot(strip_lds(), i)];
          sx += u.x;
          sy += u.y;
        }
      }
    }
    if constexpr (kRowVec<KMAX>) store_row<KMAX>(row, rv, k);
    if (kAlign) {
      // Eq. (2) and Eq. (1) as in finish_query, the position from the staged copy
      const double2 own = w.cs[2 * s];
      const double2 xi = w.cs[2 * s + 1];
      if (a.include_self) {
        sx += own.x;
        sy += own.y;
      }
      const double m = static_cast<double>(k + (a.include_self ? 1 : 0));
      const double phi = (a.variant & NM_NOISE_SCALAR) ? noise_angle(static_cast<uint32_t>(w.sorted[s].w)) : 0.0;
      const float th = heading_update(sx / m, sy / m, xi.x, xi.y, phi, a.eta, a.theta + qi, a.variant);
      int ddx, ddy;
      move_step(a.v0, own.x, own.y, th, a.variant, ddx, ddy);
      const int qx = rx + ox0, qy = ((cy << lw) | oy) + oy0;  // strip-image coordinates
      const int mask = w.box - 1;
      a.x_out[qi] = (qx + ddx) & mask;
      a.y_out[qi] = (qy + ddy) & mask;
      a.theta_out[qi] = th;
    }
  };

  // The queries of the (sub-)strip just staged, or searched in global memory
  // (the fast block search) when its halo could not be staged.
  auto global_query = [&](int qi, int r) {
    int slot[KMAX];
    const int s = w.start[static_cast<int64_t>(y0_cur + r) * G + tb.x0] + (qi - s_qoff[r]);
    const int4 q = w.sorted[s];
    if constexpr (kMode == kFieldOfView) {
      fov_exact<KMAX>(w, s, q, fov_heading(a.theta[q.z], a.cone), k, total, nbr);
      return;
    }
    if (knn_fast<KMAX>(w, f, s, q.x, q.y, k, total, slot))
      finish_query<KMAX, kAlign>(w, s, q, slot, k, nbr, d2out, a);
    else
      defer(s);
  };
  if constexpr (kMode != kOverflowSplit) {
    int npts, nq;
    // Staging is a chain of global reads and barriers: its waves issue first
    // (wave priority), so that other strips' searches fill the gaps.
    __builtin_amdgcn_s_setprio(3);
    const bool staged = strip_stage<true>(w, geo, strip_lds(), total, npts, nq);
    __builtin_amdgcn_s_setprio(0);
    if (nq == 0) return;
    for (int qi = threadIdx.x; qi < nq; qi += kBlock) {
      if (staged) {
        const int self = s_qmap[qi];
        staged_query(self, s_rowid[self]);
      } else {
        global_query(qi, row_of(qi));
      }
    }
  } else {
    // The strip is staged whole when its halo fits LDS.  Otherwise it runs
    // as sub-strips of whole rows, each as tall as fits, staged one after
    // another; a row whose own halo does not fit (bit 30) is searched in
    // global memory.  One staging site keeps a single copy of that code.
    int next = -1, nsub = 0;  // the sub-strip to stage next (-1: none planned)
    for (;;) {
      int np_cur, nq_cur;
      __builtin_amdgcn_s_setprio(3);
      const bool st = strip_stage<true>(w, geo, strip_lds(), total, np_cur, nq_cur);
      __builtin_amdgcn_s_setprio(0);
      nq_cur = __builtin_amdgcn_readfirstlane(nq_cur);  // block-uniform: keep it scalar
      bool plan = false;
      if (next < 0) {
        if (nq_cur == 0) return;
        plan = !st && hx > 0;
      }
      if (plan) {
        const int cap = wide ? kStripPts / 2 : kStripPts;
        if (threadIdx.x == 0) {
          int ns = 0;
          for (int r0 = 0; r0 < tb.ty;) {
            const bool fits = s_rbase[r0 + 2 * hy + 1] - s_rbase[r0] <= cap;
            int r1 = r0 + 1;
            if (fits)
              while (r1 < tb.ty && s_rbase[r1 + 2 * hy + 1] - s_rbase[r0] <= cap) ++r1;
            s_sub[ns++] = r0 | (fits ? 0 : 1 << 30);
            r0 = r1;
          }
          s_sub[ns] = tb.ty;
          s_nsub = ns;
        }
        __syncthreads();
        nsub = __builtin_amdgcn_readfirstlane(s_nsub);
        next = 0;
      } else {
        if (st) {
          for (int qi = threadIdx.x; qi < nq_cur; qi += kBlock) {
            const int self = s_qmap[qi];
            staged_query(self, s_rowid[self]);
          }
        } else {
          for (int qi = threadIdx.x; qi < nq_cur; qi += kBlock) global_query(qi, row_of(qi));
        }
        if (next < 0 || next >= nsub) break;
        __syncthreads();  // this sub-strip's queries are done with LDS
      }
      const int e = __builtin_amdgcn_readfirstlane(s_sub[next]);
      const int r0 = e & 0xFFFF, r1 = __builtin_amdgcn_readfirstlane(s_sub[next + 1]) & 0xFFFF;
      y0_cur = tb.y0 + r0;
      ty_cur = r1 - r0;
      oy0 = (y0_cur - hy) << lw;
      geo = StripGeo{tb.x0, y0_cur, ty_cur, tw, (e >> 30) == 0 ? hx : 0, hy, wide};
      ++next;
    }
  }
  __syncthreads();
  const int nd = s_defer;
  if (nd == 0) return;

  // The strip's uncertified queries, by the exact ring search.  With many
  // (over 48), each lane searches its own; otherwise a wavefront searches one
  // at a time, so that a single long search is not one lane's serial chain
  // (on the clustered 2^22 state, from 16 to 48: 3-8% faster).
  const int nl = min(nd, kDeferCap);
  if (kMode == kFieldOfView && nl > 16) {
    for (int j = threadIdx.x; j < nl; j += kBlock) {
      const int sq = s_dq[j];
      const int4 q = w.sorted[sq];
      fov_exact<KMAX>(w, sq, q, fov_heading(a.theta[q.z], a.cone), k, total, nbr);
    }
  } else if (kMode != kFieldOfView && nl > 48) {
    for (int j = threadIdx.x; j < nl; j += kBlock) exact_lane<KMAX, kAlign>(w, s_dq[j], k, total, nbr, d2out, a);
  } else {
    for (int j = threadIdx.x >> 6; j < nl; j += kBlock / 64) {
      const int sq = s_dq[j];
      const int4 q = w.sorted[sq];
      int slot[KMAX];
      bool ok;
      if constexpr (kMode == kFieldOfView)
        ok = knn_wave<KMAX>(w, sq, q, k, total, slot, FovFilter{fov_heading(a.theta[q.z], a.cone)});
      else
        ok = knn_wave<KMAX>(w, sq, q, k, total, slot);
      if (lane == 0) {
        if (ok)
          finish_query<KMAX, kAlign>(w, sq, q, slot, k, nbr, d2out, a);
        else
          set_err(w.hdr, NM_E_RANGE);  // fewer than k other (visible) particles were binned
      }
    }
  }
  if (nd > kDeferCap) {
    for (int r = 0; r < tb.ty; ++r) {
      const int64_t row = static_cast<int64_t>(tb.y0 + r) * G;
      const int a0 = w.start[row + tb.x0];
      const int a1 = max(min(w.start[row + tb.x0 + tw], total), a0);
      for (int sq = a0 + threadIdx.x; sq < a1; sq += kBlock) {
        if (w.dflag[sq]) {
          w.dflag[sq] = 0;
          if constexpr (kMode == kFieldOfView) {
            const int4 q = w.sorted[sq];
            fov_exact<KMAX>(w, sq, q, fov_heading(a.theta[q.z], a.cone), k, total, nbr);
          } else {
            exact_lane<KMAX, kAlign>(w, sq, k, total, nbr, d2out, a);
          }
        }
      }
    }
  }
}

// Waves per SIMD asked of the compiler: five for the short lists (96 VGPRs,
// which the LDS of a strip also allows), four for KMAX 12-20, whose insertion
// networks would otherwise take the kernel to three or two; the spills these
// limits add (cold for k <= 12) cost less than the waves they gain.  The
// batched kernel, which also holds its system's descriptors, spills at five
// and takes four.
template <int KMAX>
constexpr int kKnnWaves = (KMAX >= 12 && KMAX <= 20) ? 4 : (KMAX <= 8 ? 5 : 1);
template <int KMAX>
constexpr int kBatchKnnWaves = KMAX <= 8 ? 4 : kKnnWaves<KMAX>;

template <int KMAX, bool kAlign, int kMode>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kKnnWaves<KMAX>))) void k_knn(DevWs w, FastCfg f, TileCfg tc, int k,
                                                int32_t* __restrict__ nbr,
                                                long long* __restrict__ d2out, AlignArgs a) {
  knn_tile_body<KMAX, kAlign, kMode>(w, f, tc, k, nbr, d2out, a, xcd_tile(blockIdx.x, gridDim.x));
}

// Field-of-view lists over the same strips (a.theta: headings, a.cone: the
// cone's cos(half angle) * 4096).
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_knn_fov_strip(DevWs w, FastCfg f, TileCfg tc, int k,
                                                          int32_t* __restrict__ nbr, AlignArgs a) {
  knn_tile_body<KMAX, false, kFieldOfView>(w, f, tc, k, nbr, nullptr, a, xcd_tile(blockIdx.x, gridDim.x));
}

template <int KMAX>
hipError_t launch_fov_strip_t(const DevWs& w, const FastCfg& f, const TileCfg& tc, int k, int32_t* nbr,
                              const AlignArgs& a, hipStream_t s) {
  const int ntiles = tc.ntx * tc.nty;
  hipLaunchKernelGGL(k_knn_fov_strip<KMAX>, dim3(ntiles), dim3(kBlock), 0, s, w, f, tc, k, nbr, a);
  return hipGetLastError();
}

// Batched k-NN + alignment.  Items of the tile stage are (system, tile); the
// hardware item order is remapped so that each XCD walks one contiguous run of
// items (consecutive tiles of a system share halo cells in that XCD's L2).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<T*>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ AlignArgs uniform_load_align(const BatchSys* d) {
  const int p = __builtin_amdgcn_readfirstlane(d->parity);
  AlignArgs a;
  a.v0 = __builtin_amdgcn_readfirstlane(d->v0);
  a.eta = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, d->eta)));
  a.include_self = __builtin_amdgcn_readfirstlane(d->include_self);
  a.variant = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(d->variant)));
  a.theta = uniform_ptr(d->th[p]);
  a.x_out = uniform_ptr(d->x[1 - p]);
  a.y_out = uniform_ptr(d->y[1 - p]);
  a.theta_out = uniform_ptr(d->th[1 - p]);
  return a;
}

template <int KMAX, int kMode>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kBatchKnnWaves<KMAX>))) void k_bb_knn(BatchRef b, int k) {
  constexpr int kSt = kMode == kOverflowSplit ? kStKnnSplit : kStKnn;
  const int ni = b.begin[kSt + 1] - b.begin[kSt];
  const int per = gridDim.x & ~7;  // whole rounds of the 8 XCDs
  for (int hw = blockIdx.x; hw < ni; hw += gridDim.x) {
    // Neighbouring strips on one XCD (one L2): over all items when each
    // workgroup takes one, else within the rounds that every workgroup of a
    // multiple-of-8 grid takes.
    int it = hw;
    const int round_base = (hw / gridDim.x) * gridDim.x;
    if (static_cast<int>(gridDim.x) == ni)
      it = xcd_tile(hw, ni);
    else if (per == static_cast<int>(gridDim.x) && round_base + per <= ni)
      it = round_base + xcd_tile(hw - round_base, per);
    const BatchSys* g = b.sys + b.items[b.begin[kSt] + it];
    const DevWs w = uniform_load(&g->w);
    const FastCfg f = uniform_load(&g->f);
    const TileCfg tc = uniform_load(&g->tc);
    const AlignArgs a = uniform_load_align(g);
    const int li = it - __builtin_amdgcn_readfirstlane(g->base[kSt]);
    knn_tile_body<KMAX, true, kMode>(w, f, tc, k, uniform_ptr(g->nbr), nullptr, a, li);
    __syncthreads();
  }
}

// Strip geometry.  Block rows: up to the expected block height plus one
// widening step (hy); block width: all W = tw + 2 hx columns, hx the expected
// half width.  The strip height aims at about 256 queries; the halo must fit
// the staging buffer and the row table, W <= G (a block never meets itself
// around the box), and narrow strips keep every block under 2^15 units.
TileCfg tile_cfg_impl(const DevWs& w, const FastCfg& f, int k, bool narrow_strips) {
  TileCfg t{1, 1, 0, 0, w.G, w.G, 0, 0};
  const double rho = static_cast<double>(w.n) / static_cast<double>(w.C);  // particles per cell
  const double rr = rho > 1e-12 ? rho : 1e-12;
  const double rk = sqrt(static_cast<double>(k) / (3.141592653589793 * rr));
  const int bmax_all = max(f.bmax, f.bmax_w);
  auto plain = [&]() {  // no staging: one row of queries per strip, global search
    t.tw = 1;
    t.hx = t.hy = 0;
    t.th = max(1, min(w.G, static_cast<int>(lround(256.0 / (rr * 1.0)))));
    t.th = min(t.th, kStripRows);
    t.ntx = w.G;
    t.nty = (w.G + t.th - 1) / t.th;
    t.bmax = 0;
    return t;
  };
  if (bmax_all < 1) return plain();
  // Halo rows: for a block kReachY times the expected height (queries in
  // sparse rows choose taller blocks; 1 with `narrow_strips`), plus one
  // widening step.
  const double ry = narrow_strips ? 1.0 : kReachY;
  const int bq = f.bfix > 0 ? f.bfix : static_cast<int>(ceil(2.0 * ry * f.reach * rk)) + 1;
  int hy = min((bq + 2) / 2, 15);  // (hy <= 15: block heights fit 5 bits)
  // The block width is fixed per strip, so it covers the tail of the k-th
  // neighbour distance, not only its mean.
  int hx = min(max(1, static_cast<int>(ceil(kReachX * rk))), 15);
  if (f.bfix > 0) hx = min(max(hx, f.bfix / 2), 15);
  // Strip width: wider as the halo widens (hx 2: two columns, hx >= 3: four,
  // or two for lists of up to 8, where a block's candidates (its rows times
  // W = tw + 2 hx) cost more than the extra staging: 93 -> 88 us for k = 7 at
  // w = 1024, block 6, while k = 12 loses 4%), and at least the narrowest
  // power of two whose strips reach ~256 queries within the row limit.  Wider
  // strips stage each particle fewer times and leave fewer queries near a
  // strip's side.  `narrow_strips` (two columns
  // only from hx 3, and halo rows for the expected block height) serves the
  // sub-strip kernel, whose larger halos overflow LDS more often, and the
  // field-of-view lists, whose blocks span every column of the strip.
  int tw = narrow_strips ? (hx >= 3 ? 2 : 1) : (hx >= 3 ? (k <= 8 ? 2 : 4) : (hx >= 2 ? 2 : 1));
  while (tw < 16 && 2 * tw <= w.G && 256.0 / (tw * rr) > 1.1 * (kTwRows - 2 * hy)) tw *= 2;
  while (hx > 1 && tw + 2 * hx > w.G) --hx;
  while (hy > 1 && 2 * hy + 1 > w.G) --hy;
  if (tw + 2 * hx > w.G || 2 * hy + 1 > w.G) return plain();
  const int W = tw + 2 * hx;
  const bool narrow = (static_cast<long long>(W) << w.log2_w) < 32768 &&
                      (static_cast<long long>(2 * hy + 1) << w.log2_w) < 32768;
  const int cap = narrow ? kStripPts : kStripPts / 2;
  int th = static_cast<int>(ceil(256.0 / (tw * rr)));
  th = max(1, min(th, w.G));
  while (th > 1 && (th + 2 * hy > kStripRows || (th + 2 * hy) * W * rho > 0.75 * cap)) --th;
  if (th + 2 * hy > kStripRows) return plain();
  t.tw = tw;
  t.th = th;
  t.hx = hx;
  t.hy = hy;
  t.ntx = w.G / tw;
  t.nty = (w.G + th - 1) / th;
  t.bmax = min(2 * hy + 1, w.G);
  t.wide = narrow ? 0 : 1;
  return t;
}

template <int KMAX, bool kAlign>
hipError_t launch_t(const DevWs& w, const FastCfg& f, int k, int32_t* nbr, long long* d2,
                    const AlignArgs& a, hipStream_t s) {
  const TileCfg tc = tile_cfg_impl(w, f, k, f.split != 0);
  const int ntiles = tc.ntx * tc.nty;
  if (f.split && tc.hx > 0)
    hipLaunchKernelGGL((k_knn<KMAX, kAlign, kOverflowSplit>), dim3(ntiles), dim3(kBlock), 0, s, w, f,
                       tc, k, nbr, d2, a);
  else
    hipLaunchKernelGGL((k_knn<KMAX, kAlign, kOverflowGlobal>), dim3(ntiles), dim3(kBlock), 0, s, w, f,
                       tc, k, nbr, d2, a);
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

TileCfg tile_cfg(const DevWs& w, const FastCfg& f, int k) { return tile_cfg_impl(w, f, k, f.split != 0); }

// The tiles of the plain-strip systems, then those of the sub-strip systems
// (each launch only when it has items).
hipError_t launch_batch_knn(const BatchRef& b, int k, hipStream_t s) {
  const int nt = b.begin[kStKnn + 1] - b.begin[kStKnn];
  const int ns = b.begin[kStKnnSplit + 1] - b.begin[kStKnnSplit];
  return dispatch_k(k, [&](auto km) {
    constexpr int KM = decltype(km)::value;
    if (nt > 0) {
      const int g = nt;  // one workgroup per strip: uneven strips balance over the CUs
      hipLaunchKernelGGL((k_bb_knn<KM, kOverflowGlobal>), dim3(g), dim3(kBlock), 0, s, b, k);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (ns > 0) {
      const int g = ns;
      hipLaunchKernelGGL((k_bb_knn<KM, kOverflowSplit>), dim3(g), dim3(kBlock), 0, s, b, k);
      return hipGetLastError();
    }
    return hipSuccess;
  });
}

// Fast-path limits for a grid: block sides up to the largest B whose
// offsets keep 32-bit squared distances exact ((B / 2 + 1) w < 2^15) and whose
// block cannot meet itself around the box (B + 2 <= G).  `block` > 0 fixes the
// side, 0 picks it per query, < 0 disables the fast path; NM_BLOCK_SUBSTRIPS
// in it selects the sub-strip kernel.
FastCfg fast_cfg(const DevWs& w, int k, int block) {
  (void)k;
  FastCfg f{0, 0, 1.25f, 0, 0};
  if (block < 0) return f;
  f.split = (block & NM_BLOCK_SUBSTRIPS) ? 1 : 0;
  block &= ~NM_BLOCK_SUBSTRIPS;
  int bw = kMaxB;  // any span (64-bit distances): the block must not meet itself
  while (bw >= 3 && bw + 2 > w.G) --bw;
  if (bw < 3) return f;
  int bmax = bw;
  while (bmax >= 3 && (static_cast<long long>((bmax >> 1) + 1) << w.log2_w) >= 32768) --bmax;
  if (bmax < 3) bmax = 0;
  if (block > 0) {
    if (block > bw) return f;
    f.bfix = block;
    if (block > bmax) bmax = 0;
  }
  f.bmax = bmax;
  f.bmax_w = bw;
  return f;
}

// A cone of half angle alpha sees the fraction alpha / pi of the directions,
// so its k nearest visible lie about as far as the k / (alpha / pi) nearest
// of all: the strips and blocks are sized for that many.
hipError_t launch_knn_fov_strips(const DevWs& w, int block, const float* theta, int k, int c,
                                 int32_t* nbr, hipStream_t s) {
  FastCfg f = fast_cfg(w, k, block);
  const double alpha = acos(fmax(-1.0, fmin(1.0, c / 4096.0)));
  const double frac = fmax(alpha / 3.141592653589793, 1.0 / 64.0);
  const int ks = static_cast<int>(ceil(k / frac));
  const TileCfg tc = tile_cfg_impl(w, f, ks, true);
  f.reach = static_cast<float>(f.reach * sqrt(static_cast<double>(ks) / k));
  AlignArgs a{};
  a.theta = theta;
  a.cone = c;
  if (k <= 4) return launch_fov_strip_t<4>(w, f, tc, k, nbr, a, s);
  if (k <= 8) return launch_fov_strip_t<8>(w, f, tc, k, nbr, a, s);
  if (k <= 12) return launch_fov_strip_t<12>(w, f, tc, k, nbr, a, s);
  if (k <= 16) return launch_fov_strip_t<16>(w, f, tc, k, nbr, a, s);
  if (k <= 24) return launch_fov_strip_t<24>(w, f, tc, k, nbr, a, s);
  return launch_fov_strip_t<32>(w, f, tc, k, nbr, a, s);
}

void knn_layout(const DevWs& w, int k, int block, int32_t out[10]) {
  const FastCfg f = fast_cfg(w, k, block);
  const TileCfg tc = tile_cfg_impl(w, f, k, f.split != 0);
  // kernel: 0 = one row of queries per strip, searched in global memory;
  // 1 = staged strips (default kernel); 2 = staged strips, sub-strip kernel
  out[0] = tc.hx == 0 ? 0 : (f.split ? 2 : 1);
  out[1] = tc.tw;
  out[2] = tc.th;
  out[3] = tc.hx;
  out[4] = tc.hy;
  out[5] = f.bfix;
  out[6] = tc.wide;
  out[7] = tc.bmax;
  out[8] = tc.ntx;
  out[9] = tc.nty;
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
  AlignArgs a{p->v0, p->eta, p->include_self, p->variant, theta, x_out, y_out, theta_out};
  return dispatch_k(k, [&](auto km) {
    return launch_t<decltype(km)::value, true>(w, f, k, nbr, nullptr, a, s);
  });
}

}  // namespace nm
