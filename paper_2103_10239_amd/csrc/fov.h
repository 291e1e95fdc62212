// fov.h -- the field-of-view test and the exact per-query field-of-view
// search, shared by the ring-search kernel (fov.hip) and the strip kernel
// (knn.hip).
//
// The heading vector is h = (rint(4096 cos theta), rint(4096 sin theta)) in
// fp64 from the fp32 heading; the cone's half angle alpha is given by
// cos alpha = c / 4096.  With d the minimum-image displacement to j, j is
// visible when d = 0 or 4096 (d . h) >= c |d| |h|, decided exactly on
// squares in 128-bit integers (|4096 d.h| < 2^45, c^2 |d|^2 |h|^2 < 2^89).
#pragma once
#include "nm_internal.h"

namespace nm {

struct FovHeading {
  long long hx, hy;
  unsigned long long h2c2;  // |h|^2 c^2 (< 2^25 * 2^24)
  float h2c2f;              // the same, rounded to fp32
  int c;
  bool all;                 // c = -4096: every particle is visible
};

__device__ __forceinline__ FovHeading fov_heading(float theta, int c) {
  double sn, cs;
  sincos(static_cast<double>(theta), &sn, &cs);
  FovHeading f;
  f.hx = static_cast<long long>(rint(4096.0 * cs));
  f.hy = static_cast<long long>(rint(4096.0 * sn));
  f.h2c2 = static_cast<unsigned long long>(f.hx * f.hx + f.hy * f.hy) *
           static_cast<unsigned long long>(static_cast<long long>(c) * c);
  f.h2c2f = static_cast<float>(f.h2c2);
  f.c = c;
  f.all = c <= -4096;
  return f;
}

__device__ __forceinline__ bool fov_visible(long long dx, long long dy, const FovHeading& h) {
  if (dx == 0 && dy == 0) return true;
  const long long p = 4096 * (dx * h.hx + dy * h.hy);
  const unsigned long long ap = static_cast<unsigned long long>(p < 0 ? -p : p);
  const unsigned __int128 p2 = static_cast<unsigned __int128>(ap) * ap;
  const unsigned __int128 q2 =
      static_cast<unsigned __int128>(static_cast<unsigned long long>(dx * dx + dy * dy)) * h.h2c2;
  if (h.c >= 0) return p >= 0 && p2 >= q2;
  return p >= 0 || p2 <= q2;
}

// The same decision for a displacement of under 2^15 units per axis, whose
// squared length d2 is given.  d . h fits 29 bits; the sign settles most
// candidates, and the squares 2^24 (d . h)^2 and d2 |h|^2 c^2 are compared
// in fp32 (relative error below 2^-21 each), in 128-bit integers only when
// they lie within 2^-20 of each other.
__device__ __forceinline__ bool fov_visible_short(int dx, int dy, int d2, const FovHeading& h) {
  if (h.all) return true;
  const int p = dx * static_cast<int>(h.hx) + dy * static_cast<int>(h.hy);
  const bool front = p >= 0;
  if (h.c >= 0 ? !front : front) return front;  // behind a narrow cone / ahead of a wide one
  const float pf = static_cast<float>(p);
  const float lhs = pf * pf * 16777216.0f;
  const float rhs = static_cast<float>(d2) * h.h2c2f;
  if (lhs > rhs * (1.0f + 0x1p-20f)) return h.c >= 0;
  if (lhs < rhs * (1.0f - 0x1p-20f)) return h.c < 0;
  return fov_visible(dx, dy, h);
}

// Exact field-of-view list of the particle in slot s (position q): rings of
// cells around its home cell, nearest first; each visible candidate enters
// the register list of 64-bit (d^2, index) keys; the search ends once the
// k-th visible key lies strictly inside the ring (the cone does not change
// that bound).  Writes the row, or records NM_E_RANGE when fewer than k
// particles are visible.
template <int KMAX>
__device__ __forceinline__ void fov_exact(const DevWs& w, int s, const int4& q, const FovHeading& h, int k,
                                          int total, int32_t* __restrict__ nbr) {
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
        if (!fov_visible(ex, ey, h)) continue;
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

}  // namespace nm
