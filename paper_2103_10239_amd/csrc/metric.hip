// metric.hip -- metric neighbour lists (Sec. III: all pairs of particles
// within a distance r_0 count as neighbours), from the same cells as the
// topological lists, as CSR rows in the caller's particle order, each row
// ascending by (d^2, index).
//
// Three kernels: count the row lengths, prefix-sum them into the row offsets
// (the scan of cells.hip), and fill the rows.  Both passes work on strips of
// cells staged in LDS with a halo of h = ceil((r_c + 1) / w) cells (the strip
// staging of strip.h, with particle indices beside the positions): the disk of
// radius r_c around any query lies inside the W halo columns of the 2h + 1
// halo rows around its own, one contiguous LDS range, so no search is needed.
// The fill appends the LDS index of each hit to the lane's column of an LDS
// buffer in one pass over the range, then orders the column by 32-bit keys
// in a sorting network; rows too long for the column are selected in chunks
// of kChunk, a pass over the range keeping the kChunk smallest exact
// (d^2, index) keys above the last one written.
// Strips whose halo does not fit LDS walk rings of cells in global memory.
#include "strip.h"

namespace nm {

namespace {

constexpr int kChunk = 16;

__device__ __forceinline__ bool ws_ready(const DevWs& w) {
  const WsHeader* h = w.hdr;
  return h->built == kBuilt && h->n == w.n && h->box == w.box && h->cell_w == w.cell_w;
}

// Cells that can hold a point within rc2 of (qx, qy), nearest rings first:
// f(beg, end) with the cell's slot range.
template <class F>
__device__ __forceinline__ void for_each_cell_within(const DevWs& w, int qx, int qy, long long rc2,
                                                     int total, F&& f) {
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
      f(w.start[c], min(w.start[c + 1], total));
    });
    if (rc2 < q.ring_bound(r, cw)) break;
  }
}

// Squared distance (min image) from (qx, qy) to the particle in slot t.
__device__ __forceinline__ long long slot_d2(const DevWs& w, int t, int qx, int qy, int& j) {
  const int sh = 32 - w.log2_box;
  const int4 e = w.sorted[t];
  const int ex = wrap_axis(e.x - qx, sh);
  const int ey = wrap_axis(e.y - qy, sh);
  j = e.z;
  return static_cast<long long>(ex) * ex + static_cast<long long>(ey) * ey;
}

// Exact walk by one thread: f(d2, index) for every particle t != s within rc2.
template <class F>
__device__ __forceinline__ void for_each_within(const DevWs& w, int s, int qx, int qy,
                                                long long rc2, int total, F&& f) {
  for_each_cell_within(w, qx, qy, rc2, total, [&](int beg, int end) {
    for (int t = beg; t < end; ++t) {
      if (t == s) continue;
      int j;
      const long long d2 = slot_d2(w, t, qx, qy, j);
      if (d2 <= rc2) f(d2, j);
    }
  });
}

// Strip geometry of the metric lists: halo h from r_c, width and height for
// about 256 queries per strip within the LDS limits.
struct MetricCfg {
  int tw, th, h, ntx, nty, wide, stage;
};

MetricCfg metric_cfg(const DevWs& w, long long rc2) {
  MetricCfg m{1, 1, 0, w.G, 0, 0, 0};
  const double rho = static_cast<double>(w.n) / static_cast<double>(w.C);
  const double rr = rho > 1e-12 ? rho : 1e-12;
  const double rc = sqrt(static_cast<double>(rc2));
  const int cw = 1 << w.log2_w;
  const int h = static_cast<int>(ceil((rc + 1.0) / cw));
  auto plain = [&]() {  // one column of cells per strip, every query walks global memory
    m.tw = 1;
    m.h = 0;
    m.th = max(1, min(min(w.G, kStripRows), static_cast<int>(lround(256.0 / rr))));
    m.ntx = w.G;
    m.nty = (w.G + m.th - 1) / m.th;
    m.stage = 0;
    return m;
  };
  if (h < 1 || 4 * h + 1 > kStripRows || 2 * h + 1 > w.G) return plain();
  // two columns once the halo is two wide (each particle staged fewer times)
  int tw = h >= 2 ? 2 : 1;
  while (tw < 16 && 2 * tw <= w.G && 256.0 / (tw * rr) > 1.1 * (kTwRows - 2 * h)) tw *= 2;
  if (tw + 2 * h > w.G) return plain();
  const int W = tw + 2 * h;
  const bool narrow = (static_cast<long long>(W) << w.log2_w) < 32768 &&
                      (static_cast<long long>(2 * h + 1) << w.log2_w) < 32768;
  const int cap = narrow ? kStripPts : kStripPts / 2;
  int th = static_cast<int>(ceil(256.0 / (tw * rr)));
  th = max(1, min(th, w.G));
  while (th > 1 && (th + 2 * h > kStripRows || (th + 2 * h) * W * rho > 0.75 * cap)) --th;
  m.tw = tw;
  m.th = th;
  m.h = h;
  m.ntx = w.G / tw;
  m.nty = (w.G + th - 1) / th;
  m.wide = narrow ? 0 : 1;
  m.stage = 1;
  return m;
}

constexpr int kHeavyRange = 768;  // staged candidates above which a wave takes the query
constexpr int kWaveKeys = 512;    // longest row a wave sorts in LDS
constexpr int kWaves = kBlock / 64;
constexpr int kChunkQ = 512;      // queries per chunk of a split strip
constexpr int kMaxChunks = 256;   // chunks one strip may be split into
constexpr int kChunkGrid = 1024;  // workgroups of the chunk kernels

// Wave-scope ordering of LDS accesses between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Append slot s to pass ph's deferred list (w.rank, free once the cells are
// built) when `defer`; one atomic per wave.  Every lane of the wave calls it.
__device__ __forceinline__ void defer_query(const DevWs& w, int ph, bool defer, int s) {
  const unsigned long long b = __ballot(defer);
  if (b == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(static_cast<long long>(b)) - 1;
  uint32_t base = 0u;
  if (lane == leader) base = atomicAdd(&w.hdr->ndefer[ph], static_cast<uint32_t>(__popcll(b)));
  base = __shfl(base, leader, 64);
  const uint32_t at = base + static_cast<uint32_t>(__popcll(b & ((1ull << lane) - 1ull)));
  if (defer && at < static_cast<uint32_t>(w.n)) w.rank[at] = s;  // each query at most once a pass
}

// A staged query: its LDS index, the LDS range [lo, hi) of the 2h + 1 halo
// rows around its own, and its staged position (packed, or x and y).
struct StagedQuery {
  int self, lo, hi, pq, pqy;
};

struct StripView {
  const int* lpos;
  const int2* lpos2;
  const int* lidx;
  bool wide;
  __device__ long long d2(int i, const StagedQuery& q) const {
    if (wide) {
      const int2 c = lpos2[i];
      const long long dx = c.x - q.pq, dy = c.y - q.pqy;
      return dx * dx + dy * dy;
    }
    return rel_d2(lpos[i], q.pq);
  }
};

// LDS of one strip pass.
struct StripShared {
  int2 lpos_store[kStripPts / 2 + kUnroll];
  int lidx[kStripPts + kUnroll];
  int rbase[kStripRows + 1];
  int ga0[kStripRows];
  int n0[kStripRows];
  int ga1[kStripRows];
  int qoff[kStripRows + 1];
  int tself[kStripRows];
  int wsum[kBlock / 64];
  uint8_t rowid[kStripPts];
  int4 chunk[kMaxChunks];  // this strip's chunks: {tile, r0 | r1 << 16 | unstaged << 30, qa, qb}
  int heavy[kChunkQ];      // queries of the current batch left to the waves
  int nchunk, nlocal, nheavy, nlane;
};

// Strip of tile `tile` as a strip geometry, rows [r0, r1) of it.
__device__ __forceinline__ StripGeo tile_geo(const DevWs& w, const MetricCfg& mc, int tile, int r0,
                                             int r1, bool stage) {
  const int tyi = tile / mc.ntx, txi = tile - tyi * mc.ntx;
  const int y0 = tyi * mc.th;
  return StripGeo{txi * mc.tw, y0 + r0, r1 - r0, mc.tw, stage ? mc.h : 0, mc.h, mc.wide != 0};
}

// Where Op::light leaves a row: done, to one wave (Op::heavy) or to one lane
// of a second sweep (Op::lane), so that rows of one kind share wavefronts.
enum RowPath { kRowDone = 0, kRowWave = 1, kRowLane = 2 };

// Queries [qa, qb) of the strip g just staged, in batches of kChunkQ: one
// lane each runs Op::light; the rows it passes on are then taken, from the
// same staged data, one lane each (Op::lane) or one wave each (Op::heavy);
// both lists share S.heavy, from either end.  Without staging (`staged`
// false) every query goes to the deferred list for the wave kernels.
template <class Op>
__device__ __forceinline__ void run_queries(const DevWs& w, const MetricCfg& mc, StripShared& S,
                                            const StripGeo& g, bool staged, int qa, int qb,
                                            const Op& op) {
  const StripView view{reinterpret_cast<const int*>(S.lpos_store), S.lpos_store, S.lidx, mc.wide != 0};
  auto row_of = [&](int qi) {
    int r = 0;
#pragma unroll
    for (int step = kRowStep; step > 0; step >>= 1)
      if (r + step < g.ty && S.qoff[r + step] <= qi) r += step;
    return r;
  };
  if (!staged) {
    const int pad = ((qb - qa) + 63) & ~63;  // whole waves, for defer_query
    for (int t = threadIdx.x; t < pad; t += kBlock) {
      const int qi = qa + t;
      int slot = 0;
      if (qi < qb) {
        const int r = row_of(qi);
        slot = w.start[static_cast<int64_t>(g.y0 + r) * w.G + g.x0] + (qi - S.qoff[r]);
      }
      defer_query(w, Op::kPass, qi < qb, slot);
    }
    return;
  }
  auto query = [&](int qi) {
    const int r = row_of(qi);
    const int self = S.tself[r] + (qi - S.qoff[r]);
    const int2 p2 = mc.wide ? S.lpos_store[self] : make_int2(view.lpos[self], 0);
    return StagedQuery{self, S.rbase[r], S.rbase[r + 2 * mc.h + 1], p2.x, p2.y};
  };
  for (int b0 = qa; b0 < qb; b0 += kChunkQ) {
    const int b1 = min(qb, b0 + kChunkQ);
    if (threadIdx.x == 0) {
      S.nheavy = 0;
      S.nlane = 0;
    }
    __syncthreads();
    for (int qi = b0 + threadIdx.x; qi < b1; qi += kBlock) {
      const int path = op.light(w, query(qi), view);
      if (path == kRowWave) S.heavy[atomicAdd(&S.nheavy, 1)] = qi;
      if (path == kRowLane) S.heavy[kChunkQ - 1 - atomicAdd(&S.nlane, 1)] = qi;
    }
    __syncthreads();
    const int nl = S.nlane;
    for (int d = threadIdx.x; d < nl; d += kBlock) op.lane(w, query(S.heavy[kChunkQ - 1 - d]), view);
    // Wave rows: wave v takes rows v, v + kWaves, ...; lane j first finds the
    // query and loads the row data of the wave's j-th next row, so that the
    // rows' latencies overlap, and the wave then takes them one by one.
    const int nh = S.nheavy;
    const int lane = threadIdx.x & 63;
    for (int d0 = threadIdx.x >> 6; d0 < nh; d0 += 64 * kWaves) {
      const int dj = d0 + kWaves * lane;
      StagedQuery qj{0, 0, 0, 0, 0};
      typename Op::Row rj{};
      if (dj < nh) {
        qj = query(S.heavy[dj]);
        rj = op.row(view, qj);
      }
      const int cnt = min(64, (nh - d0 + kWaves - 1) / kWaves);
      for (int j = 0; j < cnt; ++j) {
        const StagedQuery q{__shfl(qj.self, j, 64), __shfl(qj.lo, j, 64), __shfl(qj.hi, j, 64),
                            __shfl(qj.pq, j, 64), __shfl(qj.pqy, j, 64)};
        op.heavy(w, q, view, Op::row_at(rj, j));
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ StripLds strip_lds(StripShared& S) {
  return StripLds{S.lpos_store, S.lidx, S.rbase, S.ga0, S.n0, S.ga1, S.qoff, S.tself, S.wsum, S.rowid};
}

// One chunk {tile, rows, query range}: stage its rows and run its queries.
template <class Op>
__device__ __forceinline__ void run_chunk(const DevWs& w, const MetricCfg& mc, StripShared& S, int4 c,
                                          int total, const Op& op) {
  const bool unstaged = (c.y >> 30) & 1;
  const int r0 = c.y & 0x1FF, r1 = (c.y >> 16) & 0x1FF;
  const StripGeo g = tile_geo(w, mc, c.x, r0, r1, !unstaged);
  int npts, nq;
  // Staging (global reads and barriers) issues first; other strips' searches
  // fill its gaps.
  __builtin_amdgcn_s_setprio(3);
  const bool staged = strip_stage<true>(w, g, strip_lds(S), total, npts, nq);
  __builtin_amdgcn_s_setprio(0);
  run_queries(w, mc, S, g, staged, min(c.z, nq), min(c.w, nq), op);
  __syncthreads();  // LDS is restaged by the next chunk
}

// Chunks of a strip whose halo does not fit LDS or that holds more than
// kChunkQ queries (thread 0; rbase and qoff of the whole strip staged):
// runs of rows whose halo fits and whose queries number at most qmax, a row
// with more queries cut into ranges of qmax; a row whose own halo does not
// fit forms an unstaged chunk.  qmax doubles until at most kMaxChunks.
__device__ __forceinline__ int split_strip(const MetricCfg& mc, StripShared& S, int tile, int ty,
                                           int cap) {
  const int two_h = 2 * mc.h;
  for (int qmax = kChunkQ;; qmax *= 2) {
    int nc = 0;
    for (int r0 = 0; r0 < ty && nc <= kMaxChunks;) {
      const bool fits = S.rbase[r0 + two_h + 1] - S.rbase[r0] <= cap;
      int r1 = r0 + 1;
      if (fits)
        while (r1 < ty && S.rbase[r1 + two_h + 1] - S.rbase[r0] <= cap && S.qoff[r1 + 1] - S.qoff[r0] <= qmax)
          ++r1;
      const int nq = S.qoff[r1] - S.qoff[r0];
      const int word = r0 | (r1 << 16) | (fits ? 0 : 1 << 30);
      if (nq > 0) {
        const int step = fits ? qmax : nq;  // an unstaged row only defers its queries
        for (int qa = 0; qa < nq && nc <= kMaxChunks; qa += step) {
          if (nc < kMaxChunks) S.chunk[nc] = make_int4(tile, word, qa, min(qa + step, nq));
          ++nc;
        }
      }
      r0 = r1;
    }
    if (nc <= kMaxChunks) return nc;
  }
}

// Strip kernels' body: stage tile `tile`; a strip that fits LDS and holds at
// most kChunkQ queries is run here; otherwise its chunks go to the chunk
// list (those beyond the list's capacity are run here).
template <class Op>
__device__ __forceinline__ void strip_tile(const DevWs& w, const MetricCfg& mc, int tile, const Op& op) {
  __shared__ StripShared S;
  const int total = min(w.start[w.C], w.n);
  const int cap = mc.wide ? kStripPts / 2 : kStripPts;
  const int tyi = tile / mc.ntx;
  const int ty = min(mc.th, w.G - tyi * mc.th);
  const StripGeo geo = tile_geo(w, mc, tile, 0, ty, mc.stage != 0);
  int npts, nq;
  __builtin_amdgcn_s_setprio(3);
  const bool staged = strip_stage<true>(w, geo, strip_lds(S), total, npts, nq);
  __builtin_amdgcn_s_setprio(0);
  if (nq == 0) return;
  if (!mc.stage || (staged && nq <= kChunkQ)) {
    run_queries(w, mc, S, geo, staged, 0, nq, op);
    return;
  }
  if (threadIdx.x == 0) {
    const int nc = split_strip(mc, S, tile, ty, cap);
    const uint32_t base = atomicAdd(&w.hdr->nchunk[Op::kPass], static_cast<uint32_t>(nc));
    const int room = base >= static_cast<uint32_t>(w.chunk_cap)
                         ? 0 : min(nc, w.chunk_cap - static_cast<int>(base));
    for (int c = 0; c < room; ++c) w.chunks[base + c] = S.chunk[c];
    S.nchunk = nc;
    S.nlocal = room;  // chunks [room, nc) did not fit the list
  }
  __syncthreads();
  const int nc = S.nchunk;
  for (int c = S.nlocal; c < nc; ++c) run_chunk(w, mc, S, S.chunk[c], total, op);
}

// Chunk kernels' body: the workgroups take the listed chunks in turn.
template <class Op>
__device__ __forceinline__ void strip_chunks(const DevWs& w, const MetricCfg& mc, const Op& op) {
  __shared__ StripShared S;
  const int total = min(w.start[w.C], w.n);
  const int nc = static_cast<int>(min<uint32_t>(w.hdr->nchunk[Op::kPass], static_cast<uint32_t>(w.chunk_cap)));
  for (int c = blockIdx.x; c < nc; c += gridDim.x) run_chunk(w, mc, S, w.chunks[c], total, op);
}

// Wave kernels' driver: the waves of the grid take the deferred rows of
// pass ph in turn, f(slot) with the whole wave.
template <class F>
__device__ __forceinline__ void for_each_deferred(const DevWs& w, int ph, F&& f) {
  const int nd = static_cast<int>(min<uint32_t>(w.hdr->ndefer[ph], static_cast<uint32_t>(w.n)));
  const int nw = gridDim.x * kWaves;
  for (int d = blockIdx.x * kWaves + (threadIdx.x >> 6); d < nd; d += nw) f(w.rank[d]);
}

// Wave-parallel exact walk over the cells that can hold a point within rc2
// of the particle in slot s: f(hit, d2, index) once per round in every lane.
template <class F>
__device__ __forceinline__ void wave_within(const DevWs& w, int s, const int4& q, long long rc2,
                                            int total, F&& f) {
  const int lane = threadIdx.x & 63;
  for_each_cell_within(w, q.x, q.y, rc2, total, [&](int beg, int end) {
    for (int t0 = beg; t0 < end; t0 += 64) {
      const int t = t0 + lane;
      long long d2 = 0;
      int j = 0;
      bool hit = false;
      if (t < end && t != s) {
        d2 = slot_d2(w, t, q.x, q.y, j);
        hit = d2 <= rc2;
      }
      f(hit, d2, j);
    }
  });
}

// Empty both passes' lists and reset the row-length scan; first kernel of
// every metric-list call.
__global__ __launch_bounds__(kBlock) void k_metric_reset(DevWs w) {
  for (int t = threadIdx.x; t < w.nb_scan_m; t += blockDim.x) w.scan_m->flags[t] = 0ull;
  if (threadIdx.x == 0) {
    w.scan_m->ticket = 0u;
    for (int ph = 0; ph < 2; ++ph) {
      w.hdr->ndefer[ph] = 0u;
      w.hdr->nchunk[ph] = 0u;
    }
  }
}

// Count pass: row lengths |{j != i : d^2 <= rc2}| into offsets[i].
struct CountOp {
  static constexpr int kPass = 0;
  int32_t* offsets;
  unsigned long long rc2;
  __device__ __forceinline__ int light(const DevWs&, const StagedQuery& q, const StripView& v) const {
    if (q.hi - q.lo > kHeavyRange) return kRowWave;
    // The query itself (distance 0, inside its own range) is counted with the
    // others and taken off at the end.  Whole rounds run without an end check;
    // only the range's last round masks what lies beyond it (staging is
    // padded by kUnroll entries).
    int cnt = 0;
    const int full = q.lo + ((q.hi - q.lo) & ~(kUnroll - 1));
    if (v.wide) {
      auto round = [&](int i, bool tail) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          cnt += ((!tail || i + u < q.hi) && static_cast<unsigned long long>(v.d2(i + u, q)) <= rc2) ? 1 : 0;
      };
      for (int i = q.lo; i < full; i += kUnroll) round(i, false);
      if (full < q.hi) round(full, true);
    } else {
      const uint32_t r32 = static_cast<uint32_t>(min(rc2, 0xFFFFFFFFull));
      auto round = [&](int i, bool tail) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          cnt += ((!tail || i + u < q.hi) && rel_d2_u(v.lpos[i + u], q.pq) <= r32) ? 1 : 0;
      };
      for (int i = q.lo; i < full; i += kUnroll) round(i, false);
      if (full < q.hi) round(full, true);
    }
    offsets[v.lidx[q.self]] = cnt - 1;
    return kRowDone;
  }
  __device__ __forceinline__ void lane(const DevWs&, const StagedQuery&, const StripView&) const {}
  using Row = int;  // no row data
  __device__ __forceinline__ Row row(const StripView&, const StagedQuery&) const { return 0; }
  __device__ static __forceinline__ Row row_at(Row, int) { return 0; }
  // One wave: the same count over the staged range.
  __device__ __forceinline__ void heavy(const DevWs&, const StagedQuery& q, const StripView& v, Row) const {
    int cnt = 0;
    for (int i0 = q.lo; i0 < q.hi; i0 += 64) {
      const int i = i0 + static_cast<int>(threadIdx.x & 63);
      const bool hit = i < q.hi && i != q.self && static_cast<unsigned long long>(v.d2(i, q)) <= rc2;
      cnt += __popcll(__ballot(hit));
    }
    if ((threadIdx.x & 63) == 0) offsets[v.lidx[q.self]] = cnt;
  }
};

__global__ __launch_bounds__(kBlock) void k_metric_count(DevWs w, MetricCfg mc, long long rc2,
                                                         int32_t* __restrict__ offsets) {
  if (!ws_ready(w)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  strip_tile(w, mc, xcd_tile(blockIdx.x, gridDim.x), CountOp{offsets, static_cast<unsigned long long>(rc2)});
}

__global__ __launch_bounds__(kBlock) void k_metric_count_chunks(DevWs w, MetricCfg mc, long long rc2,
                                                                int32_t* __restrict__ offsets) {
  strip_chunks(w, mc, CountOp{offsets, static_cast<unsigned long long>(rc2)});
}

__global__ __launch_bounds__(kBlock) void k_metric_count_waves(DevWs w, long long rc2,
                                                               int32_t* __restrict__ offsets) {
  const int total = min(w.start[w.C], w.n);
  for_each_deferred(w, 0, [&](int s) {
    const int4 q = w.sorted[s];
    int cnt = 0;
    wave_within(w, s, q, rc2, total, [&](bool hit, long long, int) { cnt += __popcll(__ballot(hit)); });
    if ((threadIdx.x & 63) == 0) offsets[q.z] = cnt;
  });
}

// Rows of the fill: offset and length of a row from its two offsets, checked
// against nnz.
__device__ __forceinline__ bool row_bounds(const DevWs& w, const nm_int2u& o, long long nnz, long long& base,
                                           long long& m) {
  base = o.x;
  m = static_cast<long long>(o.y) - base;
  if (base < 0 || m < 0 || base + m > nnz) {
    set_err(w.hdr, NM_E_INVAL);
    return false;
  }
  return true;
}

// The same for row j, read from `offsets` (one 8-byte load).
__device__ __forceinline__ bool fill_row(const DevWs& w, const int32_t* offsets, long long nnz, int j,
                                         long long& base, long long& m) {
  return row_bounds(w, *reinterpret_cast<const nm_int2u*>(offsets + j), nnz, base, m);
}

// One thread: the m smallest exact (d^2, index) keys of a staged query, in
// chunks of kChunk; false if fewer than m were found.
__device__ __forceinline__ bool strip_fill(const StagedQuery& q, const StripView& v, long long rc2,
                                           long long m, int32_t* __restrict__ out) {
  long long written = 0;
  unsigned long long last = 0ull;  // every real key is >= 1
  while (written < m) {
    const int need = static_cast<int>(min<long long>(kChunk, m - written));
    TopK<kChunk, false> top;
    top.init(need);
    for (int i = q.lo; i < q.hi; i += kUnroll) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const long long d2 = v.d2(i + u, q);
        if (i + u < q.hi && i + u != q.self && d2 <= rc2) {
          const unsigned long long kk = pack_key(d2, v.lidx[i + u]);
          if (kk > last && kk < top.worst()) top.push(kk, 0);
        }
      }
    }
    if (top.worst() == ~0ull) return false;
#pragma unroll
    for (int t = 0; t < kChunk; ++t)
      if (t >= kChunk - need) out[written + t - (kChunk - need)] = key_index(top.key[t]);
    written += need;
    last = top.worst();
  }
  return true;
}

// One thread, 32-bit keys (d^2 >> sh) << 13 | LDS index through the
// insertion network, in chunks of KT; exact when no two entries written have
// the same distance field (then ordered by index, as the exact keys would
// be). Returns false on such a tie, or if fewer than m were found: the caller
// then runs the exact selection.
template <int KT, bool kWide>
__device__ __forceinline__ bool strip_fill32(const StagedQuery& q, const StripView& v, long long rc2,
                                             int sh, long long m, int32_t* __restrict__ out) {
  uint32_t last = 0u, prev_d = 0xFFFFFFFFu;
  long long written = 0;
  while (written < m) {
    const int need = static_cast<int>(min<long long>(KT, m - written));
    uint32_t key[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) key[t] = (t < KT - need) ? 0u : kKey32Inf;
    // whole rounds without an end check; only the range's last round masks
    // what lies beyond it
    auto round = [&](int i, bool tail) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        bool in;
        uint32_t dfield;
        if (kWide) {
          const long long d2 = v.d2(i + u, q);
          in = d2 <= rc2;
          dfield = static_cast<uint32_t>(d2 >> sh);
        } else {
          const uint32_t d2 = rel_d2_u(v.lpos[i + u], q.pq);
          in = d2 <= static_cast<uint32_t>(rc2);
          dfield = d2 >> sh;
        }
        const uint32_t kk = (dfield << 13) | static_cast<uint32_t>(i + u);
        net_insert(key, (in && (!tail || i + u < q.hi) && i + u != q.self && kk > last) ? kk : kKey32Inf);
      }
    };
    const int full = q.lo + ((q.hi - q.lo) & ~(kUnroll - 1));
    for (int i = q.lo; i < full; i += kUnroll) round(i, false);
    if (full < q.hi) round(full, true);
    if (key[KT - 1] == kKey32Inf) return false;
    bool good = key32_d(key[KT - need]) != prev_d;
#pragma unroll
    for (int t = 0; t < KT - 1; ++t)
      if (t >= KT - need) good = good && key32_d(key[t]) != key32_d(key[t + 1]);
    if (!good) return false;
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (t >= KT - need) out[written + t - (KT - need)] = v.lidx[key[t] & 0x1FFFu];
    written += need;
    last = key[KT - 1];
    prev_d = key32_d(last);
  }
  return true;
}

// One thread, chunked exact selection for a query in global memory (slot s).
__device__ __forceinline__ bool global_fill(const DevWs& w, int s, long long rc2, int total, long long m,
                                            int32_t* __restrict__ out) {
  const int4 e = w.sorted[s];
  long long written = 0;
  unsigned long long last = 0ull;
  while (written < m) {
    const int need = static_cast<int>(min<long long>(kChunk, m - written));
    TopK<kChunk, false> top;
    top.init(need);
    for_each_within(w, s, e.x, e.y, rc2, total, [&](long long d2, int j) {
      const unsigned long long kk = pack_key(d2, j);
      if (kk > last && kk < top.worst()) top.push(kk, 0);
    });
    if (top.worst() == ~0ull) return false;
#pragma unroll
    for (int t = 0; t < kChunk; ++t)
      if (t >= kChunk - need) out[written + t - (kChunk - need)] = key_index(top.key[t]);
    written += need;
    last = top.worst();
  }
  return true;
}

// This wave's key buffer in LDS (kernels of the fill pass); two spare
// entries keep each wave's buffer 16-byte aligned and pad odd rows.
__device__ __forceinline__ unsigned long long (&key_lds())[kWaves][kWaveKeys + 2] {
  __shared__ unsigned long long s_keys[kWaves][kWaveKeys + 2];
  return s_keys;
}
__device__ __forceinline__ unsigned long long* wave_keys() { return key_lds()[threadIdx.x >> 6]; }

// The same LDS as kSlots 16-bit slots per lane (LDS indices of a row's hits),
// column-major: slot c of lane t at c * kBlock + p(t), where p interleaves
// lanes t and t + 32 of a wavefront in one dword, so that a wavefront's
// appends touch each bank once per half.  The light rows of a batch use it,
// the waves' rows only after a barrier.
constexpr int kSlots = 32;
static_assert(kSlots * kBlock * 2 <= kWaves * (kWaveKeys + 2) * 8, "slot columns exceed the key buffer");
static_assert(kStripPts + kUnroll <= 0x2000, "LDS indices exceed the slots and the keys' index field");
__device__ __forceinline__ uint16_t* lane_slots() {
  const int t = threadIdx.x;
  const int p = (t & ~63) | ((t & 31) << 1) | ((t >> 5) & 1);
  return reinterpret_cast<uint16_t*>(&key_lds()[0][0]) + p;
}

// One wave: the m unique keys in buf written to out in ascending order.
// Lane l holds keys l, l + 64, ... (E per lane) and counts, over broadcast
// reads of the whole buffer, the keys below each: that count is its place.
template <int E>
__device__ __forceinline__ void rank_write_e(unsigned long long* buf, int m, int32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  if (lane == 0 && (m & 1)) buf[m] = ~0ull;  // pairs read past an odd row
  wave_sync();
  unsigned long long mine[E];
  int rank[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane + 64 * r;
    mine[r] = e < m ? buf[e] : ~0ull;
    rank[r] = 0;
  }
  // four pairs a round: their LDS reads are in flight together (a wave sorts
  // its rows one after another, so their latency is not hidden by others)
#pragma unroll 4
  for (int t = 0; t < m; t += 2) {
    const unsigned long long a = buf[t], b = buf[t + 1];
#pragma unroll
    for (int r = 0; r < E; ++r) rank[r] += (a < mine[r] ? 1 : 0) + (b < mine[r] ? 1 : 0);
  }
#pragma unroll
  for (int r = 0; r < E; ++r)
    if (lane + 64 * r < m) out[rank[r]] = key_index(mine[r]);
}

__device__ __forceinline__ void wave_sort_write(unsigned long long* buf, int m, int32_t* __restrict__ out) {
  if (m <= 64)
    rank_write_e<1>(buf, m, out);
  else if (m <= 128)
    rank_write_e<2>(buf, m, out);
  else if (m <= 256)
    rank_write_e<4>(buf, m, out);
  else
    rank_write_e<8>(buf, m, out);
}

// Ascending sort of NS keys in registers (bitonic network).
template <int NS>
__device__ __forceinline__ void bitonic_sort(uint32_t (&key)[NS]) {
#pragma unroll
  for (int size = 2; size <= NS; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          const uint32_t a = key[i], b = key[j];
          const bool up = (i & size) == 0;
          key[i] = up ? min(a, b) : max(a, b);
          key[j] = up ? max(a, b) : min(a, b);
        }
      }
    }
  }
}

// The c LDS indices of a slot column as 32-bit keys (d^2 >> sh) << 13 | index,
// sorted; the first must be the query itself (distance 0) and no two may share
// a distance field (then the order by index is the exact one).  The others go
// out as particle indices.  False otherwise: the caller runs the exact
// selection.
template <int NS>
__device__ __forceinline__ bool slots_sort_write(const StagedQuery& q, const StripView& v, const uint16_t* col,
                                                 int c, int sh, int32_t* __restrict__ out) {
  uint32_t key[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    key[t] = kKey32Inf;
    if (t < c) {
      const int j = col[t * kBlock];
      const uint32_t d2 = v.wide ? static_cast<uint32_t>(v.d2(j, q) >> sh) : rel_d2_u(v.lpos[j], q.pq) >> sh;
      key[t] = (d2 << 13) | static_cast<uint32_t>(j);
    }
  }
  bitonic_sort(key);
  bool good = key[0] == static_cast<uint32_t>(q.self);
#pragma unroll
  for (int t = 0; t + 1 < NS; ++t)
    if (t + 1 < c) good = good && key32_d(key[t]) != key32_d(key[t + 1]);
  if (!good) return false;
  // keys 1 .. c - 1 as 16-byte stores where four are left, the rest one by one
  auto at = [&](int t) { return v.lidx[key[t] & 0x1FFFu]; };
#pragma unroll
  for (int t = 1; t < NS; t += 4) {
    if (t + 3 < NS && t + 3 < c) {
      *reinterpret_cast<nm_int4u*>(out + t - 1) = nm_int4u{at(t), at(t + 1), at(t + 2), at(t + 3)};
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t + u < NS && t + u < c) out[t - 1 + u] = at(t + u);
    }
  }
  return true;
}

// One thread, a row of m entries with m + 2 <= kSlots: one pass over the
// range appends the LDS index of every hit (the query itself among them, at
// distance 0) to the lane's slot column, whose spare slot takes the
// candidates after the last hit; then the column is sorted and written.
// False when the hits are not m + 1 or on a tie of distance fields.
template <bool kWide>
__device__ __forceinline__ bool strip_fill_slots(const StagedQuery& q, const StripView& v, long long rc2,
                                                 int sh, long long m, int32_t* __restrict__ out) {
  uint16_t* col = lane_slots();
  const uint32_t r32 = static_cast<uint32_t>(min(rc2, 0xFFFFFFFFll));
  int c = 0;
  // whole rounds without an end check; only the range's last round masks
  // what lies beyond it
  auto round = [&](int i, bool tail) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool in = kWide ? v.d2(i + u, q) <= rc2 : rel_d2_u(v.lpos[i + u], q.pq) <= r32;
      col[min(c, kSlots - 1) * kBlock] = static_cast<uint16_t>(i + u);
      c += (in && (!tail || i + u < q.hi)) ? 1 : 0;
    }
  };
  const int full = q.lo + ((q.hi - q.lo) & ~(kUnroll - 1));
  for (int i = q.lo; i < full; i += kUnroll) round(i, false);
  if (full < q.hi) round(full, true);
  if (c != m + 1) return false;
  // one network width per wavefront (lanes taking two would run both)
  const unsigned long long w8 = __ballot(c > 8), w16 = __ballot(c > 16);
  if (w16) return slots_sort_write<kSlots>(q, v, col, c, sh, out);
  if (w8) return slots_sort_write<16>(q, v, col, c, sh, out);
  return slots_sort_write<8>(q, v, col, c, sh, out);
}

// Fill pass: row i of the CSR lists, ascending by (d^2, index).
struct FillOp {
  static constexpr int kPass = 1;
  const int32_t* offsets;
  int32_t* idx;
  long long rc2, nnz;
  int sh;  // distance field of the 32-bit keys: d^2 >> sh < 2^kDBits for d^2 <= rc2
  // Rows of up to kSlots - 2 entries: one pass into the lane's slot column.
  // Longer rows go to a wave (one lane would take several passes of the
  // kChunk-wide network, while the rest of the workgroup waits at the next
  // barrier); rows longer than a wave sorts, to the second sweep of lanes.
  __device__ __forceinline__ int light(const DevWs& w, const StagedQuery& q, const StripView& v) const {
    long long base, m;
    if (!fill_row(w, offsets, nnz, v.lidx[q.self], base, m) || m == 0) return kRowDone;
    const int range = q.hi - q.lo;
    if (m <= kWaveKeys && range > kHeavyRange) return kRowWave;
    if (m + 2 <= kSlots) {
      const bool done = v.wide ? strip_fill_slots<true>(q, v, rc2, sh, m, idx + base)
                               : strip_fill_slots<false>(q, v, rc2, sh, m, idx + base);
      if (!done && !strip_fill(q, v, rc2, m, idx + base)) set_err(w.hdr, NM_E_INVAL);
      return kRowDone;
    }
    return m <= kWaveKeys ? kRowWave : kRowLane;
  }
  __device__ __forceinline__ void lane(const DevWs& w, const StagedQuery& q, const StripView& v) const {
    long long base, m;
    if (!fill_row(w, offsets, nnz, v.lidx[q.self], base, m)) return;
    const bool done = v.wide ? strip_fill32<kChunk, true>(q, v, rc2, sh, m, idx + base)
                             : strip_fill32<kChunk, false>(q, v, rc2, sh, m, idx + base);
    if (!done && !strip_fill(q, v, rc2, m, idx + base)) set_err(w.hdr, NM_E_INVAL);
  }
  // One wave: the row's exact keys gathered from the staged range into LDS
  // (ballot compaction), placed by rank and written out (m <= kWaveKeys).
  using Row = nm_int2u;  // the row's offset and the next one
  __device__ __forceinline__ Row row(const StripView& v, const StagedQuery& q) const {
    return *reinterpret_cast<const nm_int2u*>(offsets + v.lidx[q.self]);
  }
  __device__ static __forceinline__ Row row_at(const Row& r, int j) {
    return Row{__shfl(r.x, j, 64), __shfl(r.y, j, 64)};
  }
  __device__ __forceinline__ void heavy(const DevWs& w, const StagedQuery& q, const StripView& v, Row o) const {
    long long base, m;
    if (!row_bounds(w, o, nnz, base, m) || m == 0) return;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long* buf = wave_keys();
    wave_sync();  // the previous row's reads of buf are done
    long long got = 0;
    for (int i0 = q.lo; i0 < q.hi; i0 += 64) {
      const int i = i0 + lane;
      long long d2 = 0;
      bool hit = false;
      if (i < q.hi && i != q.self) {
        d2 = v.d2(i, q);
        hit = d2 <= rc2;
      }
      const unsigned long long b = __ballot(hit);
      const long long pos = got + __popcll(b & below);
      if (hit && pos < m) buf[pos] = pack_key(d2, v.lidx[i]);
      got += __popcll(b);
    }
    if (got != m) {
      if (lane == 0) set_err(w.hdr, NM_E_INVAL);
      return;
    }
    wave_sort_write(buf, static_cast<int>(m), idx + base);
  }
};

__device__ __forceinline__ int key_shift(long long rc2) {
  int sh = 0;
  while ((rc2 >> sh) >= (1ll << kDBits) - 1) ++sh;
  return sh;
}

__global__ __launch_bounds__(kBlock) void k_metric_fill(DevWs w, MetricCfg mc, long long rc2,
                                                        const int32_t* __restrict__ offsets,
                                                        int32_t* __restrict__ idx, long long cap) {
  if (!ws_ready(w)) return;
  const long long nnz = offsets[w.n];
  if (nnz > cap || nnz < 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_err(w.hdr, NM_E_CAPACITY);
    return;
  }
  strip_tile(w, mc, xcd_tile(blockIdx.x, gridDim.x), FillOp{offsets, idx, rc2, nnz, key_shift(rc2)});
}

__global__ __launch_bounds__(kBlock) void k_metric_fill_chunks(DevWs w, MetricCfg mc, long long rc2,
                                                               const int32_t* __restrict__ offsets,
                                                               int32_t* __restrict__ idx, long long cap) {
  const long long nnz = offsets[w.n];
  if (nnz > cap || nnz < 0) return;  // reported by the strip kernel; the lists are empty
  strip_chunks(w, mc, FillOp{offsets, idx, rc2, nnz, key_shift(rc2)});
}

// One wave per deferred row: its keys gathered into LDS by ballot
// compaction, placed by rank and written out; rows longer than
// kWaveKeys take the chunked selection in the wave's first lane.
__global__ __launch_bounds__(kBlock) void k_metric_fill_waves(DevWs w, long long rc2,
                                                              const int32_t* __restrict__ offsets,
                                                              int32_t* __restrict__ idx, long long cap) {
  const long long nnz = offsets[w.n];
  const bool ok = nnz <= cap && nnz >= 0;  // otherwise the list is empty
  const int total = min(w.start[w.C], w.n);
  const int lane = threadIdx.x & 63;
  unsigned long long* buf = wave_keys();
  const unsigned long long below = (1ull << lane) - 1ull;
  for_each_deferred(w, 1, [&](int s) {
    const int4 q = w.sorted[s];
    long long base, m;
    if (!ok || !fill_row(w, offsets, nnz, q.z, base, m) || m == 0) return;
    int32_t* out = idx + base;
    if (m > kWaveKeys) {
      if (lane == 0 && !global_fill(w, s, rc2, total, m, out)) set_err(w.hdr, NM_E_INVAL);
      return;
    }
    long long got = 0;
    wave_sync();  // the previous row's reads of buf are done
    wave_within(w, s, q, rc2, total, [&](bool hit, long long d2, int j) {
      const unsigned long long b = __ballot(hit);
      const long long pos = got + __popcll(b & below);
      if (hit && pos < m) buf[pos] = pack_key(d2, j);
      got += __popcll(b);
    });
    if (got != m) {
      if (lane == 0) set_err(w.hdr, NM_E_INVAL);
      return;
    }
    wave_sort_write(buf, static_cast<int>(m), out);
  });
}

// Grid of the wave kernels: enough waves to spread a deferred list over
// every CU.
int wave_grid(const DevWs& w) { return max(1, min(1024, (w.n + kWaves - 1) / kWaves)); }

}  // namespace

hipError_t launch_metric_count(const DevWs& w, long long rc2, int32_t* offsets, hipStream_t s) {
  const MetricCfg mc = metric_cfg(w, rc2);
  hipLaunchKernelGGL(k_metric_reset, dim3(1), dim3(kBlock), 0, s, w);
  hipLaunchKernelGGL(k_metric_count, dim3(mc.ntx * mc.nty), dim3(kBlock), 0, s, w, mc, rc2, offsets);
  hipLaunchKernelGGL(k_metric_count_chunks, dim3(kChunkGrid), dim3(kBlock), 0, s, w, mc, rc2, offsets);
  hipLaunchKernelGGL(k_metric_count_waves, dim3(wave_grid(w)), dim3(kBlock), 0, s, w, rc2, offsets);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_rows(offsets, w.n, w.scan_m, w.nb_scan_m, w.hdr, s);
}

hipError_t launch_metric_fill(const DevWs& w, long long rc2, const int32_t* offsets, int32_t* idx,
                              long long cap, hipStream_t s) {
  const MetricCfg mc = metric_cfg(w, rc2);
  hipLaunchKernelGGL(k_metric_fill, dim3(mc.ntx * mc.nty), dim3(kBlock), 0, s, w, mc, rc2, offsets,
                     idx, cap);
  hipLaunchKernelGGL(k_metric_fill_chunks, dim3(kChunkGrid), dim3(kBlock), 0, s, w, mc, rc2, offsets,
                     idx, cap);
  hipLaunchKernelGGL(k_metric_fill_waves, dim3(wave_grid(w)), dim3(kBlock), 0, s, w, rc2, offsets, idx,
                     cap);
  return hipGetLastError();
}

}  // namespace nm
