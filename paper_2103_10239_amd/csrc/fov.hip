// fov.hip -- field-of-view topological lists: for every particle, the k
// nearest (by (d^2, index)) among the particles inside a cone around its
// heading (the topological rule of Sec. III restricted to what the particle
// faces).
//
// The heading vector is h = (rint(4096 cos theta), rint(4096 sin theta)) in
// fp64 from the fp32 heading; the cone's half angle alpha is given by
// cos alpha = c / 4096.  With d the minimum-image displacement to j, j is
// visible when d = 0 or 4096 (d . h) >= c |d| |h|, decided exactly on
// squares in 128-bit integers (|4096 d.h| < 2^45, c^2 |d|^2 |h|^2 < 2^89).
//
// One lane per query, in cell order: rings of cells around the home cell,
// nearest first, each candidate tested for visibility and pushed into the
// register list of 64-bit keys; a ring ends the search once the k-th visible
// key lies strictly inside it (the cone does not change that bound).
#include "nm_internal.h"

namespace nm {

namespace {

__device__ __forceinline__ bool fov_visible(long long dx, long long dy, long long hx, long long hy,
                                            unsigned long long h2c2, int c) {
  if (dx == 0 && dy == 0) return true;
  const long long p = 4096 * (dx * hx + dy * hy);
  const unsigned long long ap = static_cast<unsigned long long>(p < 0 ? -p : p);
  const unsigned __int128 p2 = static_cast<unsigned __int128>(ap) * ap;
  const unsigned __int128 q2 = static_cast<unsigned __int128>(static_cast<unsigned long long>(dx * dx + dy * dy)) *
                               h2c2;
  if (c >= 0) return p >= 0 && p2 >= q2;
  return p >= 0 || p2 <= q2;
}

template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_knn_fov(DevWs w, const float* __restrict__ theta, int k, int c,
                                                    int32_t* __restrict__ nbr) {
  const WsHeader* hd = w.hdr;
  if (!(hd->built == kBuilt && hd->n == w.n && hd->box == w.box && hd->cell_w == w.cell_w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  double sn, cs;
  sincos(static_cast<double>(theta[q.z]), &sn, &cs);
  const long long hx = static_cast<long long>(rint(4096.0 * cs));
  const long long hy = static_cast<long long>(rint(4096.0 * sn));
  // |h|^2 c^2 < 2^25 * 2^24 fits 64 bits
  const unsigned long long h2c2 = static_cast<unsigned long long>(hx * hx + hy * hy) *
                                  static_cast<unsigned long long>(static_cast<long long>(c) * c);
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom g(q.x, q.y, w);
  TopK<KMAX, true> top;
  top.init(k);
  for (int r = 0; r <= g.rmax; ++r) {
    for_ring(r, g.lo, g.hi, [&](int dx, int dy) {
      const long long gx = axis_gap(dx, g.ox, cw, sh);
      const long long gy = axis_gap(dy, g.oy, cw, sh);
      if (gx * gx + gy * gy > key_bound_d2(top.worst())) return;
      const int64_t cell = static_cast<int64_t>((g.hy + dy) & gm) * w.G + ((g.hx + dx) & gm);
      const int beg = w.start[cell];
      const int end = min(w.start[cell + 1], total);
      for (int t = beg; t < end; ++t) {
        if (t == s) continue;
        const int4 e = w.sorted[t];
        const int ex = wrap_axis(e.x - q.x, sh);
        const int ey = wrap_axis(e.y - q.y, sh);
        if (!fov_visible(ex, ey, hx, hy, h2c2, c)) continue;
        const long long d2 = static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey;
        const unsigned long long kk = pack_key(d2, e.z);
        if (kk < top.worst()) top.push(kk, t);
      }
    });
    if (key_bound_d2(top.worst()) < g.ring_bound(r, cw)) break;
  }
  if (top.worst() == ~0ull) {
    set_err(w.hdr, NM_E_RANGE);  // fewer than k visible particles
    return;
  }
  int32_t* row = nbr + static_cast<int64_t>(q.z) * k;
#pragma unroll
  for (int t = 0; t < KMAX; ++t)
    if (t >= KMAX - k) row[t - (KMAX - k)] = key_index(top.key[t]);
}

template <int KMAX>
hipError_t launch_fov_t(const DevWs& w, const float* theta, int k, int c, int32_t* nbr, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_knn_fov<KMAX>, dim3(nb), dim3(kBlock), 0, s, w, theta, k, c, nbr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_knn_fov(const DevWs& w, const float* theta, int k, int c, int32_t* nbr, hipStream_t s) {
  if (k <= 4) return launch_fov_t<4>(w, theta, k, c, nbr, s);
  if (k <= 8) return launch_fov_t<8>(w, theta, k, c, nbr, s);
  if (k <= 12) return launch_fov_t<12>(w, theta, k, c, nbr, s);
  if (k <= 16) return launch_fov_t<16>(w, theta, k, c, nbr, s);
  if (k <= 24) return launch_fov_t<24>(w, theta, k, c, nbr, s);
  return launch_fov_t<32>(w, theta, k, c, nbr, s);
}

}  // namespace nm
