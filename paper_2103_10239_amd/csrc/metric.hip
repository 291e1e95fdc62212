// metric.hip -- metric neighbour lists (Sec. III: all pairs of particles
// within a distance r_0 count as neighbours), from the same cells as the
// topological lists, as CSR rows in the caller's particle order, each row
// ascending by (d^2, index).
//
// Three kernels: count the row lengths (one lane per query, cell order),
// prefix-sum them into the row offsets (the scan of cells.hip), and fill the
// rows.  The fill selects a row in chunks of kChunk keys: each pass over the
// candidates keeps the kChunk smallest keys above the last key written.
//
// Fast path: when a B x B block of cells around the query contains the whole
// disk of radius r_c (odd B, centred), the lane scans just that block, and
// the fill uses the 32-bit keys and branch-free insertion network of the k-NN
// fast path; the row is certified when no two of its entries have the same
// d^2 >> sh.  Otherwise (or when certification fails) the lane walks rings of
// cells with exact 64-bit keys.
#include "nm_internal.h"

namespace nm {

namespace {

constexpr int kChunk = 16;

__device__ __forceinline__ bool ws_ready(const DevWs& w) {
  const WsHeader* h = w.hdr;
  return h->built == kBuilt && h->n == w.n && h->box == w.box && h->cell_w == w.cell_w;
}

// Exact walk: every particle t != s of the cells that can hold a point within
// rc2 of the query; f(t, d2, index) for those with d2 <= rc2.
template <class F>
__device__ __forceinline__ void for_each_within(const DevWs& w, int s, int qx, int qy,
                                                long long rc2, int total, F&& f) {
  const int sh = 32 - w.log2_box;
  const int cw = 1 << w.log2_w;
  const int gm = w.G - 1;
  const QueryGeom q(qx, qy, w);
  for (int r = 0; r <= q.rmax; ++r) {
    for_ring(r, q.lo, q.hi, [&](int dx, int dy) {
      const long long gx = axis_gap(dx, q.ox, cw, sh);
      const long long gy = axis_gap(dy, q.oy, cw, sh);
      if (gx * gx + gy * gy > rc2) return;
      const int64_t c = static_cast<int64_t>((q.hy + dy) & gm) * w.G + ((q.hx + dx) & gm);
      const int beg = w.start[c];
      const int end = min(w.start[c + 1], total);
      for (int t = beg; t < end; ++t) {
        if (t == s) continue;
        const int4 e = w.sorted[t];
        const int ex = wrap_axis(e.x - qx, sh);
        const int ey = wrap_axis(e.y - qy, sh);
        const long long d2 = static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey;
        if (d2 <= rc2) f(t, d2, e.z);
      }
    });
    if (rc2 < q.ring_bound(r, cw)) break;
  }
}

__device__ __forceinline__ uint32_t d2_32(int x, int y, int qx, int qy) {
  const int dx = x - qx, dy = y - qy;
  return static_cast<uint32_t>(__mul24(dx, dx)) + static_cast<uint32_t>(__mul24(dy, dy));
}

__global__ __launch_bounds__(kBlock) void k_metric_count(DevWs w, FastCfg f, long long rc2,
                                                         int32_t* __restrict__ offsets) {
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < w.nb_scan_m; t += blockDim.x) w.scan_m->flags[t] = 0ull;
    if (threadIdx.x == 0) w.scan_m->ticket = 0u;
  }
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  int cnt = 0;
  bool fast = false;
  if (f.bfix > 0) {
    const QBlock b = make_qblock(w, q.x, q.y, f.bfix);
    const uint32_t r32 = static_cast<uint32_t>(rc2);
    if (rc2 < b.bound) {
      walk_block(w, b, s, q.x, q.y, total, [&](int x, int y, int qx, int qy, int, bool valid) {
        cnt += (valid && d2_32(x, y, qx, qy) <= r32) ? 1 : 0;
      });
      fast = true;
    }
  }
  if (!fast) {
    cnt = 0;
    for_each_within(w, s, q.x, q.y, rc2, total, [&](int, long long, int) { ++cnt; });
  }
  offsets[q.z] = cnt;
}

// Fill the row of query s through the fast block; false if not certified.
__device__ __forceinline__ bool fill_fast(const DevWs& w, const FastCfg& f, int s, int qx, int qy,
                                          long long rc2, int total, long long m,
                                          int32_t* __restrict__ out) {
  const QBlock b = make_qblock(w, qx, qy, f.bfix);
  if (rc2 >= b.bound) return false;
  const uint32_t r32 = static_cast<uint32_t>(rc2);
  int sh = 0;
  while ((rc2 >> sh) >= (1ll << kDBits) - 1) ++sh;
  uint32_t last = 0u;
  long long written = 0;
  uint32_t prev_d = 0xFFFFFFFFu;  // distance field of the last entry written
  while (written < m) {
    const int need = static_cast<int>(min<long long>(kChunk, m - written));
    uint32_t key[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) key[t] = (t < kChunk - need) ? 0u : kKey32Inf;
    const bool ok = walk_block(w, b, s, qx, qy, total,
                               [&](int x, int y, int qxi, int qyi, int tag, bool valid) {
                                 const uint32_t d2 = d2_32(x, y, qxi, qyi);
                                 const uint32_t kk = ((d2 >> sh) << 13) | static_cast<uint32_t>(tag);
                                 net_insert(key, (valid && d2 <= r32 && kk > last) ? kk : kKey32Inf);
                               });
    if (!ok || key[kChunk - 1] == kKey32Inf) return false;
    bool good = prev_d == 0xFFFFFFFFu || key32_d(key[kChunk - need]) != prev_d;
#pragma unroll
    for (int t = 0; t < kChunk - 1; ++t)
      if (t >= kChunk - need) good = good && key32_d(key[t]) != key32_d(key[t + 1]);
    if (!good) return false;
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      if (t >= kChunk - need) {
        const int slot = tag_slot(w, b, key[t] & 0x1FFFu, qx, qy);
        if (static_cast<uint32_t>(slot) >= static_cast<uint32_t>(total)) return false;
        out[written + t - (kChunk - need)] = w.sorted[slot].z;
      }
    }
    written += need;
    last = key[kChunk - 1];
    prev_d = key32_d(last);
  }
  return true;
}

__global__ __launch_bounds__(kBlock) void k_metric_fill(DevWs w, FastCfg f, long long rc2,
                                                        const int32_t* __restrict__ offsets,
                                                        int32_t* __restrict__ idx, long long cap) {
  if (!ws_ready(w)) return;
  const long long nnz = offsets[w.n];
  if (nnz > cap || nnz < 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_CAPACITY);
    return;
  }
  const int total = min(w.start[w.C], w.n);
  const int s = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (s >= total) return;
  const int4 q = w.sorted[s];
  const long long base = offsets[q.z];
  const long long m = static_cast<long long>(offsets[q.z + 1]) - base;
  if (base < 0 || m < 0 || base + m > nnz) {
    set_err(w.hdr, NM_E_INVAL);
    return;
  }
  int32_t* out = idx + base;
  if (m == 0 || (f.bfix > 0 && fill_fast(w, f, s, q.x, q.y, rc2, total, m, out))) return;
  long long written = 0;
  unsigned long long last = 0ull;  // every real key is >= 1
  while (written < m) {
    const int need = static_cast<int>(min<long long>(kChunk, m - written));
    TopK<kChunk, false> top;
    top.init(need);
    for_each_within(w, s, q.x, q.y, rc2, total, [&](int t, long long d2, int j) {
      const unsigned long long kk = pack_key(d2, j);
      if (kk > last && kk < top.worst()) top.push(kk, t);
    });
    if (top.worst() == ~0ull) {  // row shorter than counted: inconsistent input
      set_err(w.hdr, NM_E_INVAL);
      return;
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t)
      if (t >= kChunk - need) out[written + t - (kChunk - need)] = key_index(top.key[t]);
    written += need;
    last = top.worst();
  }
}

// Block of odd side B centred on the home cell that contains the disk of
// radius r_c for every query: (B - 1) / 2 cells >= r_c + 1, within the limits
// of the k-NN fast path.
FastCfg metric_cfg(const DevWs& w, long long rc2) {
  const FastCfg lim = fast_cfg(w, 1, 0);
  const double rc = sqrt(static_cast<double>(rc2));
  const int cw = 1 << w.log2_w;
  const int B = 2 * static_cast<int>(ceil((rc + 1.0) / cw)) + 1;
  if (lim.bmax == 0 || B > lim.bmax) return FastCfg{0, 0, 0.0f, 0};
  return FastCfg{lim.bmax, B, 0.0f, 0};
}

}  // namespace

hipError_t launch_metric_count(const DevWs& w, long long rc2, int32_t* offsets, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_metric_count, dim3(nb), dim3(kBlock), 0, s, w, metric_cfg(w, rc2), rc2,
                     offsets);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_rows(offsets, w.n, w.scan_m, w.nb_scan_m, w.hdr, s);
}

hipError_t launch_metric_fill(const DevWs& w, long long rc2, const int32_t* offsets, int32_t* idx,
                              long long cap, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_metric_fill, dim3(nb), dim3(kBlock), 0, s, w, metric_cfg(w, rc2), rc2,
                     offsets, idx, cap);
  return hipGetLastError();
}

}  // namespace nm
