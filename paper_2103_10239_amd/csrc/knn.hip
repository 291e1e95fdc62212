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

// Fast block search; true (and `slot` filled) only when certified exact.
template <int KMAX>
__device__ __forceinline__ bool knn_fast(const DevWs& w, const FastCfg& f, int s, int qx, int qy,
                                         int k, int total, int (&slot)[KMAX]) {
  constexpr int KT = KMAX + 1;
  if (f.B == 0) return false;
  uint32_t key[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) key[t] = (t < KT - (k + 1)) ? 0u : kKey32Inf;
  BlockSegs sg;
  long long bound;
  int ncand;
  const int sh = f.sh;
  const bool ok = scan_block(w, f, s, qx, qy, total, sg, bound, ncand,
                             [&](int x, int y, int qxi, int qyi, int ord) {
                               const int dx = x - qxi, dy = y - qyi;
                               const uint32_t d2 = static_cast<uint32_t>(__mul24(dx, dx)) +
                                                   static_cast<uint32_t>(__mul24(dy, dy));
                               net_insert(key, ((d2 >> sh) << 8) | static_cast<uint32_t>(ord));
                             });
  if (!ok || ncand > 255) return false;
  const uint32_t kth = key[KT - 2];
  if (kth == kKey32Inf) return false;
  bool good = true;
#pragma unroll
  for (int t = 0; t < KT - 1; ++t)
    if (t >= KT - (k + 1)) good = good && (key32_d(key[t]) < key32_d(key[t + 1]));
  const long long dmax = (static_cast<long long>(key32_d(kth) + 1) << sh) - 1;
  if (!good || dmax >= bound) return false;
#pragma unroll
  for (int t = 0; t < KMAX; ++t)
    if (t >= KMAX - k) slot[t] = seg_slot(sg, key32_ord(key[t]));
  return true;
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

template <int KMAX, bool kAlign>
__global__ __launch_bounds__(kBlock) void k_knn(DevWs w, FastCfg f, int k, int32_t* __restrict__ nbr,
                                                long long* __restrict__ d2out, AlignArgs a) {
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  int slot[KMAX];
  if (!knn_fast<KMAX>(w, f, s, q.x, q.y, k, total, slot)) {
    if (!knn_exact<KMAX>(w, s, q.x, q.y, k, total, slot)) {
      set_err(w.hdr, NM_E_RANGE);  // fewer than k other particles were binned
      return;
    }
  }
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
        const double2 u = w.cs[slot[t]];
        sx += u.x;
        sy += u.y;
      }
    }
  }
  if (!kAlign) return;

  // Eq. (2): average of the neighbours' unit vectors (plus the particle's own),
  // vectorial noise, normalisation (only the direction is kept).
  const double2 own = w.cs[s];
  if (a.include_self) {
    sx += own.x;
    sy += own.y;
  }
  const double m = static_cast<double>(k + (a.include_self ? 1 : 0));
  const double ax = sx / m, ay = sy / m;
  double sp, cp;
  sincos(noise_angle(static_cast<uint32_t>(q.w)), &sp, &cp);
  const double e = static_cast<double>(a.eta);
  const double vx = ax + e * cp;
  const double vy = ay + e * sp;
  const float th = (vx == 0.0 && vy == 0.0) ? a.theta[q.z] : static_cast<float>(atan2(vy, vx));

  // Eq. (1): move with the heading at time t, rounded to the grid (half to even).
  const int ddx = static_cast<int>(rint(static_cast<double>(a.v0) * own.x));
  const int ddy = static_cast<int>(rint(static_cast<double>(a.v0) * own.y));
  const int mask = w.box - 1;
  a.x_out[q.z] = (q.x + ddx) & mask;
  a.y_out[q.z] = (q.y + ddy) & mask;
  a.theta_out[q.z] = th;
}

template <int KMAX, bool kAlign>
hipError_t launch_t(const DevWs& w, const FastCfg& f, int k, int32_t* nbr, long long* d2,
                    const AlignArgs& a, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_knn<KMAX, kAlign>), dim3(nb), dim3(kBlock), 0, s, w, f, k, nbr, d2, a);
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

// Fast-path block for a grid: the odd or even side B whose block edge sits
// about two mean k-th-neighbour distances from the query, limited so that
// 32-bit squared distances cannot overflow and the block cannot wrap onto
// itself.  `block` = 0 chooses automatically, < 0 disables the fast path.
FastCfg fast_cfg(const DevWs& w, int k, int block) {
  FastCfg f{0, 0};
  if (block < 0) return f;
  int B = block;
  if (B == 0) {
    // cells per k-th-neighbour radius: r_k^2 ~ k / (pi rho), rho = n / L^2
    const double cw = static_cast<double>(1 << w.log2_w);
    const double rk = sqrt(static_cast<double>(k) / (3.141592653589793 * w.n)) * w.box;
    const double want = 1.6 * rk;  // distance from the query to the block edge
    // odd B: edge >= (B-1)/2 cells; even B: edge >= (B-1)/2 cells as well
    B = static_cast<int>(ceil(2.0 * want / cw)) + 1;
    if (B < 3) B = 3;
  }
  if (B > kMaxB) return f;
  const long long ext = static_cast<long long>((B >> 1) + 1) << w.log2_w;  // max |offset|
  if (ext >= 32768 || B + 2 > w.G) return f;
  const long long dmax = 2 * ext * ext;
  int sh = 0;
  while ((dmax >> sh) >= (1ll << 24) - 1) ++sh;  // keeps every real key below kKey32Inf
  f.B = B;
  f.sh = sh;
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
