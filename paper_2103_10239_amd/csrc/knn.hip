// knn.hip -- topological neighbour lists (Sec. III: "each particle interacts
// with its k nearest neighbours") and the fused step kernel.
//
// One lane per query, queries taken in cell order so that a wavefront's
// queries are spatial neighbours and share cached cells.  Each lane walks
// rings of cells outward from its home cell, skips cells whose nearest point
// is already farther than its current k-th neighbour, and keeps the k best
// (d^2, index) keys in registers.  It stops after ring r once the k-th
// squared distance is strictly below the squared distance to the edge of the
// scanned block: an equal distance in the next ring could still carry a
// smaller index, so equality does not stop the walk.
//
// The fused kernel then evaluates Eq. (2) and Eq. (1) for the query from the
// fp64 unit vectors stored beside the cell-ordered copy (the neighbours'
// entries sit in the cells just scanned, so they are cache hits), and
// scatters the list, the new position and the new heading to the particle's
// own index.
#include "nm_internal.h"

namespace nm {

namespace {

template <int KMAX, bool kSlots>
__device__ __forceinline__ void knn_search(const DevWs& w, int s, int qx, int qy, int k,
                                           int total, TopK<KMAX, kSlots>& top) {
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom q(qx, qy, w);
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
}

__device__ __forceinline__ bool ws_ready(const DevWs& w) {
  const WsHeader* h = w.hdr;
  return h->built == kBuilt && h->n == w.n && h->box == w.box && h->cell_w == w.cell_w;
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_knn(DevWs w, int k, int32_t* __restrict__ nbr,
                                                long long* __restrict__ d2out) {
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  TopK<KMAX, false> top;
  knn_search(w, s, q.x, q.y, k, total, top);
  if (top.worst() == ~0ull) {  // fewer than k other particles were binned
    set_err(w.hdr, NM_E_RANGE);
    return;
  }
  int32_t* row = nbr + static_cast<int64_t>(q.z) * k;
  long long* drow = d2out ? d2out + static_cast<int64_t>(q.z) * k : nullptr;
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    if (t >= KMAX - k) {
      row[t - (KMAX - k)] = key_index(top.key[t]);
      if (drow) drow[t - (KMAX - k)] = key_d2(top.key[t]);
    }
  }
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

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_knn_align(DevWs w, int k, int32_t* __restrict__ nbr,
                                                      AlignArgs a) {
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  TopK<KMAX, true> top;
  knn_search(w, s, q.x, q.y, k, total, top);
  if (top.worst() == ~0ull) {
    set_err(w.hdr, NM_E_RANGE);
    return;
  }

  // Eq. (2): average of the neighbours' unit vectors (plus the particle's own).
  int32_t* row = nbr + static_cast<int64_t>(q.z) * k;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    if (t >= KMAX - k) {
      row[t - (KMAX - k)] = key_index(top.key[t]);
      const double2 u = w.cs[top.slot[t]];
      sx += u.x;
      sy += u.y;
    }
  }
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

template <int KMAX>
hipError_t launch_knn_t(const DevWs& w, int k, int32_t* nbr, long long* d2, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_knn<KMAX>, dim3(nb), dim3(kBlock), 0, s, w, k, nbr, d2);
  return hipGetLastError();
}

template <int KMAX>
hipError_t launch_knn_align_t(const DevWs& w, int k, int32_t* nbr, const AlignArgs& a,
                              hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_knn_align<KMAX>, dim3(nb), dim3(kBlock), 0, s, w, k, nbr, a);
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

hipError_t launch_knn(const DevWs& w, int k, int32_t* nbr, long long* d2, hipStream_t s) {
  return dispatch_k(k, [&](auto km) { return launch_knn_t<decltype(km)::value>(w, k, nbr, d2, s); });
}

hipError_t launch_knn_align(const DevWs& w, int k, const nm_params* p, const float* theta,
                            int32_t* nbr, int32_t* x_out, int32_t* y_out, float* theta_out,
                            hipStream_t s) {
  AlignArgs a{p->v0, p->eta, p->include_self, theta, x_out, y_out, theta_out};
  return dispatch_k(k, [&](auto km) { return launch_knn_align_t<decltype(km)::value>(w, k, nbr, a, s); });
}

}  // namespace nm
