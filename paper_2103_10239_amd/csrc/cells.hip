// cells.hip -- cell binning (Sec. I: partition the box into a grid of cells
// so that neighbour finding only looks at nearby cells).
//
// Counting sort in three kernels:
//   bin_count   per particle: cell id, rank inside the cell (atomic histogram)
//   scan        exclusive prefix sum of the histogram -> cell start table,
//               single pass with decoupled look-back; clears the histogram
//   bin_scatter per particle: write (x, y, index, noise word) to its slot in
//               cell order; the fused step also draws the Philox noise word
//               here (four consecutive particles share one Philox block) and
//               stores, in fp64, the unit vector of the heading and the
//               random unit vector of Eq. (2).
#include "nm_internal.h"

namespace nm {

namespace {

constexpr unsigned long long kFlagAgg = 1ull << 62;     // tile aggregate available
constexpr unsigned long long kFlagPrefix = 2ull << 62;  // inclusive prefix available
constexpr unsigned long long kValueMask = (1ull << 62) - 1ull;
constexpr int kSpinLimit = 1 << 22;

__device__ void reset_scan(ScanState* st, int nb) {
  for (int t = threadIdx.x; t < nb; t += blockDim.x) st->flags[t] = 0ull;
  if (threadIdx.x == 0) st->ticket = 0u;
}

// Zero the histogram and the deferral flags, reset the scan states and stamp
// the header; workgroup `b` of `nb` takes a strided share.
__device__ __forceinline__ void ws_init_body(const DevWs& w, int b, int nb) {
  const int64_t stride = static_cast<int64_t>(nb) * blockDim.x;
  for (int64_t c = static_cast<int64_t>(b) * blockDim.x + threadIdx.x; c < w.C; c += stride)
    w.count[c] = 0;
  for (int64_t i = static_cast<int64_t>(b) * blockDim.x + threadIdx.x; i < w.n; i += stride)
    w.dflag[i] = 0;
  if (b == 0) {
    reset_scan(w.scan_c, w.nb_scan_c);
    reset_scan(w.scan_m, w.nb_scan_m);
    if (threadIdx.x == 0) {
      w.hdr->magic = kMagic;
      w.hdr->err = 0;
      w.hdr->n = w.n;
      w.hdr->box = w.box;
      w.hdr->cell_w = w.cell_w;
      w.hdr->built = 0u;
      for (int ph = 0; ph < 2; ++ph) {
        w.hdr->ndefer[ph] = 0u;
        w.hdr->nchunk[ph] = 0u;
      }
      w.hdr->nvwide = 0u;
      w.hdr->nvdone = 0u;
      w.hdr->nvstale = 0u;
      w.hdr->nvfail = 0u;
      w.hdr->varea2 = 0ull;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ws_init(DevWs w) { ws_init_body(w, blockIdx.x, gridDim.x); }

// Cell and in-cell rank of the particles of workgroup `b`; workgroup 0 also
// resets the scan state for the following prefix sum.
__device__ __forceinline__ void bin_count_body(const int32_t* __restrict__ x,
                                               const int32_t* __restrict__ y, const DevWs& w,
                                               int b) {
  if (b == 0) {
    reset_scan(w.scan_c, w.nb_scan_c);
    if (threadIdx.x == 0) {
      if (w.hdr->magic != kMagic || w.hdr->n != w.n || w.hdr->box != w.box ||
          w.hdr->cell_w != w.cell_w)
        set_err(w.hdr, NM_E_INVAL);
      w.hdr->built = 0u;
    }
  }
  const int i = b * kBlock + threadIdx.x;
  if (i >= w.n) return;
  const int xi = x[i], yi = y[i];
  if (static_cast<uint32_t>(xi) >= static_cast<uint32_t>(w.box) ||
      static_cast<uint32_t>(yi) >= static_cast<uint32_t>(w.box)) {
    set_err(w.hdr, NM_E_RANGE);
    w.rank[i] = -1;
    return;
  }
  const int64_t c = static_cast<int64_t>(yi >> w.log2_w) * w.G + (xi >> w.log2_w);
  w.rank[i] = atomicAdd(&w.count[c], 1);
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const int32_t* __restrict__ x,
                                                      const int32_t* __restrict__ y, DevWs w) {
  bin_count_body(x, y, w, blockIdx.x);
}

// Exclusive prefix sum of in[0, m) into out[0, m], out[m] = total.  `in` may
// alias `out`.  With clear_in (and in != out) the input is zeroed after it
// is read.  Single pass with decoupled look-back: each tile publishes its
// aggregate, then the first wave of the tile inspects 64 predecessor tiles at
// a time, adding aggregates until it meets a published inclusive prefix.
// Tiles take increasing tickets, so every predecessor of a tile is already
// running when the tile waits on it: the look-back always ends (a bounded
// spin records NM_E_DEVICE instead of waiting forever).
__device__ __forceinline__ void scan_body(int32_t* in, int32_t* out, int64_t m, ScanState* st,
                                          WsHeader* hdr, int clear_in) {
  __shared__ uint32_t s_tile;
  __shared__ long long s_wave[kBlock / 64];
  __shared__ long long s_prefix;
  if (threadIdx.x == 0) s_tile = atomicAdd(&st->ticket, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t base = static_cast<int64_t>(tile) * kScanTile + threadIdx.x * kScanItems;

  int32_t v[kScanItems];
  long long sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t idx = base + j;
    v[j] = idx < m ? in[idx] : 0;
    sum += v[j];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  long long wave_off = 0, agg = 0;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) {
    if (q < wave) wave_off += s_wave[q];
    agg += s_wave[q];
  }
  if (wave == 0) {
    unsigned long long* flags = st->flags;
    long long prefix = 0;
    if (tile == 0) {
      if (lane == 0)
        __hip_atomic_store(&flags[0], kFlagPrefix | static_cast<unsigned long long>(agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&flags[tile], kFlagAgg | static_cast<unsigned long long>(agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int top = static_cast<int>(tile) - 1;  // predecessor seen by lane 0
      int spins = 0;
      while (true) {
        const int j = top - lane;
        // Tiles before tile 0 do not exist: read them as a prefix of 0.
        const unsigned long long f =
            j >= 0 ? __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : kFlagPrefix;
        const unsigned long long state = f & ~kValueMask;
        const unsigned long long pending = __ballot(state == 0ull);
        const unsigned long long done = __ballot(state == kFlagPrefix);
        const int p = done ? __ffsll(static_cast<long long>(done)) - 1 : 64;
        const unsigned long long upto = p >= 63 ? ~0ull : ((2ull << p) - 1ull);
        if (pending & upto) {
          if (++spins > kSpinLimit) {
            if (lane == 0) set_err(hdr, NM_E_DEVICE);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        long long part = lane <= p ? static_cast<long long>(f & kValueMask) : 0ll;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
        prefix += part;
        if (p < 64) break;
        top -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(&flags[tile], kFlagPrefix | static_cast<unsigned long long>(prefix + agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_prefix = prefix;
      if ((prefix + agg) > 0x7FFFFFFFll) set_err(hdr, NM_E_CAPACITY);
    }
  }
  __syncthreads();
  long long run = s_prefix + wave_off + (incl - sum);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t idx = base + j;
    if (idx < m) {
      out[idx] = static_cast<int32_t>(run);
      if (clear_in) in[idx] = 0;
    }
    run += v[j];
  }
  const int64_t ntiles = (m + kScanTile - 1) / kScanTile;
  if (threadIdx.x == 0 && static_cast<int64_t>(tile) == (ntiles > 0 ? ntiles - 1 : 0))
    out[m] = static_cast<int32_t>(s_prefix + agg);
}

__global__ __launch_bounds__(kBlock) void k_scan(int32_t* in, int32_t* out, int64_t m,
                                                 ScanState* st, WsHeader* hdr, int clear_in) {
  scan_body(in, out, m, st, hdr, clear_in);
}

template <bool kFused>
__device__ __forceinline__ void scatter_body(const int32_t* __restrict__ x,
                                             const int32_t* __restrict__ y,
                                             const float* __restrict__ theta, const DevWs& w,
                                             int b, uint32_t step_lo, uint32_t step_hi,
                                             uint32_t sys_id, uint32_t seed_lo, uint32_t seed_hi) {
  const WsHeader* h = w.hdr;
  if (h->magic != kMagic || h->n != w.n || h->box != w.box || h->cell_w != w.cell_w) return;
  const int t = b * kBlock + threadIdx.x;
  const int i0 = 4 * t;
  if (i0 >= w.n) return;
  uint4 noise = make_uint4(0u, 0u, 0u, 0u);
  if (kFused) noise = Philox::block(make_uint4(static_cast<uint32_t>(t), step_lo, step_hi, sys_id),
                                    seed_lo, seed_hi);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + q;
    if (i >= w.n) break;
    const int r = w.rank[i];
    if (r < 0) continue;
    const int xi = x[i], yi = y[i];
    const int64_t c = static_cast<int64_t>(yi >> w.log2_w) * w.G + (xi >> w.log2_w);
    const int pos = w.start[c] + r;
    if (static_cast<uint32_t>(pos) >= static_cast<uint32_t>(w.n)) {  // inconsistent table
      set_err(w.hdr, NM_E_INVAL);
      continue;
    }
    w.sorted[pos] = make_int4(xi, yi, i, static_cast<int>(uint4_word(noise, q)));
    if (kFused) {
      double sn, cs, xs, xc;
      sincos(static_cast<double>(theta[i]), &sn, &cs);
      sincos(noise_angle(uint4_word(noise, q)), &xs, &xc);
      w.cs[2 * pos] = make_double2(cs, sn);      // unit vector of the heading at time t
      w.cs[2 * pos + 1] = make_double2(xc, xs);  // the random unit vector xi of Eq. (2)
    }
  }
  if (t == 0) w.hdr->built = kBuilt;
}

template <bool kFused>
__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* __restrict__ x,
                                                        const int32_t* __restrict__ y,
                                                        const float* __restrict__ theta, DevWs w,
                                                        uint32_t step_lo, uint32_t step_hi,
                                                        uint32_t sys_id, uint32_t seed_lo,
                                                        uint32_t seed_hi) {
  scatter_body<kFused>(x, y, theta, w, blockIdx.x, step_lo, step_hi, sys_id, seed_lo, seed_hi);
}

// ---------------------------------------------------------------------------
// Two-level binning for one system per launch: no device-wide atomics, and
// the sorted copy is written bin by bin.
//   coarse_count    workgroup b takes particles [b P, (b+1) P) and counts
//                   them per coarse bin (2^sb consecutive cells) in LDS;
//                   hist[bin * nblk + b] = that count
//   scan            exclusive prefix sum of hist (bin-major order): the first
//                   coarse-order slot of each (bin, workgroup)
//   coarse_scatter  each particle, with its heading bits, to its
//                   (bin, workgroup) range (order inside by LDS atomics)
//   fine_sort       one workgroup per bin: counting sort of the bin's
//                   particles by cell in LDS, the bin's part of the cell
//                   start table, and the sorted copy (the fused step also
//                   draws the Philox noise word and stores the fp64 unit
//                   vectors here)
// The result is the same cell start table and the same cell-ordered copy as
// the one-level binning, up to the order inside each cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool ws_header_ok(const DevWs& w) {
  const WsHeader* h = w.hdr;
  return h->magic == kMagic && h->n == w.n && h->box == w.box && h->cell_w == w.cell_w;
}

__device__ __forceinline__ bool in_box(int xi, int yi, const DevWs& w) {
  return static_cast<uint32_t>(xi) < static_cast<uint32_t>(w.box) &&
         static_cast<uint32_t>(yi) < static_cast<uint32_t>(w.box);
}

// The two-level kernels take kCoarseP particles per workgroup of kT lanes,
// kCoarseP / kT per lane: every lane issues all its loads before its first
// LDS atomic, so that a workgroup has its whole share in flight at once.
// The single-system launches take kCoarseT lanes (four waves per SIMD on the
// one workgroup a CU holds); the batched stages, whose kernels also run the
// one-level bodies, take kBlock.  Consecutive blocks run on one XCD: the
// pieces that blocks b, b + 1, ... write into a bin's range (and into a row
// of the histogram) are adjacent, and meet in that XCD's L2 as whole lines.
constexpr int kCoarseT = 1024;

template <int kT>
__device__ __forceinline__ void coarse_count_body(const int32_t* __restrict__ x,
                                                  const int32_t* __restrict__ y, const DevWs& w, int b) {
  constexpr int kU = kCoarseP / kT;
  __shared__ int h[kCoarseBins];
  if (b == 0) {
    reset_scan(w.scan_h, w.nb_scan_h);
    if (threadIdx.x == 0) {
      if (!ws_header_ok(w)) set_err(w.hdr, NM_E_INVAL);
      w.hdr->built = 0u;
    }
  }
  const int i0 = b * kCoarseP + threadIdx.x, i1 = min((b + 1) * kCoarseP, w.n);
  int xv[kU], yv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int i = i0 + u * kT;
    xv[u] = i < i1 ? x[i] : 0;
    yv[u] = i < i1 ? y[i] : 0;
  }
  for (int t = threadIdx.x; t < w.nbins; t += kT) h[t] = 0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    if (i0 + u * kT >= i1) break;
    if (!in_box(xv[u], yv[u], w)) {
      set_err(w.hdr, NM_E_RANGE);
      continue;
    }
    const int64_t c = static_cast<int64_t>(yv[u] >> w.log2_w) * w.G + (xv[u] >> w.log2_w);
    atomicAdd(&h[static_cast<int>(c >> w.sb)], 1);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < w.nbins; t += kT)
    w.hist[static_cast<int64_t>(t) * w.nblk + b] = h[t];
}

__global__ __launch_bounds__(kCoarseT) void k_coarse_count(const int32_t* __restrict__ x,
                                                         const int32_t* __restrict__ y, DevWs w) {
  coarse_count_body<kCoarseT>(x, y, w, xcd_tile(blockIdx.x, gridDim.x));
}

template <bool kFused, int kT>
__device__ __forceinline__ void coarse_scatter_body(const int32_t* __restrict__ x,
                                                    const int32_t* __restrict__ y,
                                                    const float* __restrict__ theta, const DevWs& w,
                                                    int b) {
  constexpr int kU = kCoarseP / kT;
  __shared__ int cur[kCoarseBins];
  if (!ws_header_ok(w)) return;
  const int i0 = b * kCoarseP + threadIdx.x, i1 = min((b + 1) * kCoarseP, w.n);
  int xv[kU], yv[kU], tv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int i = i0 + u * kT;
    xv[u] = i < i1 ? x[i] : 0;
    yv[u] = i < i1 ? y[i] : 0;
    tv[u] = (kFused && i < i1) ? __float_as_int(theta[i]) : 0;
  }
  for (int t = threadIdx.x; t < w.nbins; t += kT) cur[t] = w.hist[static_cast<int64_t>(t) * w.nblk + b];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int i = i0 + u * kT;
    if (i >= i1) break;
    if (!in_box(xv[u], yv[u], w)) continue;
    const int64_t c = static_cast<int64_t>(yv[u] >> w.log2_w) * w.G + (xv[u] >> w.log2_w);
    const int pos = atomicAdd(&cur[static_cast<int>(c >> w.sb)], 1);
    if (static_cast<uint32_t>(pos) >= static_cast<uint32_t>(w.n)) {  // inconsistent table
      set_err(w.hdr, NM_E_INVAL);
      continue;
    }
    w.coarse[pos] = make_int4(xv[u], yv[u], i, tv[u]);
  }
}

template <bool kFused>
__global__ __launch_bounds__(kCoarseT) void k_coarse_scatter(const int32_t* __restrict__ x,
                                                           const int32_t* __restrict__ y,
                                                           const float* __restrict__ theta, DevWs w) {
  coarse_scatter_body<kFused, kCoarseT>(x, y, theta, w, xcd_tile(blockIdx.x, gridDim.x));
}

// Per bin: counting sort of its particles by cell in LDS.  The first
// kFineU entries of each lane stay in registers between the count and the
// scatter (a bin holds about kFineU * kBlock particles at the mean density
// the cell width is tuned for); entries beyond are read twice.  The sorted
// entries pass through an LDS stage of kFineStage ranks and are written out
// in order, lane t taking ranks t, t + kBlock, ...: the outputs then leave
// in whole lines instead of one scattered 16- and 32-byte piece per
// particle.
constexpr int kFineU = 8;
constexpr int kFineStage = 1280;

template <bool kFused>
__device__ __forceinline__ void fine_sort_body(const DevWs& w, int bin, uint32_t step_lo, uint32_t step_hi,
                                               uint32_t sys_id, uint32_t seed_lo, uint32_t seed_hi) {
  __shared__ __align__(16) int h[kFineCells];
  __shared__ __align__(16) int4 stage[kFineStage];
  __shared__ int s_wsum[kBlock / 64];
  if (!ws_header_ok(w)) return;
  const int64_t m = static_cast<int64_t>(w.nbins) * w.nblk;
  const int b0 = w.hist[static_cast<int64_t>(bin) * w.nblk];
  const int b1 = bin + 1 < w.nbins ? w.hist[static_cast<int64_t>(bin + 1) * w.nblk] : w.hist[m];
  const int64_t c0 = static_cast<int64_t>(bin) << w.sb;
  const int S = static_cast<int>(min(static_cast<int64_t>(1) << w.sb, w.C - c0));
  if (b0 < 0 || b1 < b0 || b1 > w.n) {  // inconsistent table
    if (threadIdx.x == 0) set_err(w.hdr, NM_E_INVAL);
    return;
  }
  auto cell_of = [&](const int4& e) {
    return static_cast<int>(static_cast<int64_t>(e.y >> w.log2_w) * w.G + (e.x >> w.log2_w) - c0);
  };
  const int p0 = b0 + threadIdx.x;
  int4 ev[kFineU];
#pragma unroll
  for (int u = 0; u < kFineU; ++u) {
    const int p = p0 + u * kBlock;
    ev[u] = p < b1 ? w.coarse[p] : make_int4(0, 0, 0, 0);
  }
  for (int t = threadIdx.x; t < S; t += kBlock) h[t] = 0;
  __syncthreads();
  auto count = [&](const int4& e) {
    const int cl = cell_of(e);
    if (static_cast<uint32_t>(cl) < static_cast<uint32_t>(S))
      atomicAdd(&h[cl], 1);
    else
      set_err(w.hdr, NM_E_INVAL);  // inconsistent table
  };
#pragma unroll
  for (int u = 0; u < kFineU; ++u)
    if (p0 + u * kBlock < b1) count(ev[u]);
  for (int p = p0 + kFineU * kBlock; p < b1; p += kBlock) count(w.coarse[p]);
  __syncthreads();
  // Exclusive prefix over the bin's S cells (a power of two): lane t takes
  // `per` consecutive cells, read and written as 16-byte vectors when per >= 4.
  const int per = S >= kBlock ? S / kBlock : 1;
  const int j0 = threadIdx.x * per;
  constexpr int kMaxPer = kFineCells / kBlock;
  int cnt[kMaxPer];
  int sum = 0;
#pragma unroll
  for (int j = 0; j < kMaxPer; j += 4) {
    if (j < per && j0 + j < S) {
      if (per >= 4) {
        const int4 v = *reinterpret_cast<const int4*>(&h[j0 + j]);
        cnt[j] = v.x; cnt[j + 1] = v.y; cnt[j + 2] = v.z; cnt[j + 3] = v.w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) cnt[j + q] = (q < per) ? h[j0 + q] : 0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) cnt[j + q] = 0;
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxPer; ++j) sum += cnt[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  int run = incl - sum;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q)
    if (q < wave) run += s_wsum[q];
  int ex[kMaxPer];
#pragma unroll
  for (int j = 0; j < kMaxPer; ++j) {
    ex[j] = run;
    run += cnt[j];
  }
  if (j0 < S) {
    if (per >= 4) {
#pragma unroll
      for (int j = 0; j < kMaxPer; j += 4) {
        if (j < per) {
          *reinterpret_cast<int4*>(&h[j0 + j]) = make_int4(ex[j], ex[j + 1], ex[j + 2], ex[j + 3]);
          *reinterpret_cast<nm_int4u*>(&w.start[c0 + j0 + j]) =
              nm_int4u{b0 + ex[j], b0 + ex[j + 1], b0 + ex[j + 2], b0 + ex[j + 3]};
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < per) {
          h[j0 + q] = ex[q];
          w.start[c0 + j0 + q] = b0 + ex[q];
        }
      }
    }
  }
  if (bin == w.nbins - 1 && threadIdx.x == 0) w.start[w.C] = b1;
  __syncthreads();
  // Particle e at sorted position pos: its entry, and with kFused the unit
  // vectors of its heading and of its noise draw.
  auto emit = [&](const int4& e, int pos) {
    uint32_t word = 0u;
    if (kFused) {
      const uint4 blk = Philox::block(make_uint4(static_cast<uint32_t>(e.z) >> 2, step_lo, step_hi, sys_id),
                                      seed_lo, seed_hi);
      word = uint4_word(blk, e.z & 3);
      double sn, cs, xs, xc;
      sincos(static_cast<double>(__int_as_float(e.w)), &sn, &cs);
      sincos(noise_angle(word), &xs, &xc);
      w.cs[2 * pos] = make_double2(cs, sn);      // unit vector of the heading at time t
      w.cs[2 * pos + 1] = make_double2(xc, xs);  // the random unit vector xi of Eq. (2)
    }
    w.sorted[pos] = make_int4(e.x, e.y, e.z, static_cast<int>(word));
  };
  // A bin whose entries all sit in registers is written in rounds of
  // kFineStage ranks: each round stages its ranks' entries in LDS and writes
  // them out in order.  Larger bins write each particle where it lands.
  const int nbin = b1 - b0;
  const bool staged = nbin <= kFineU * kBlock;
  int rv[kFineU];
#pragma unroll
  for (int u = 0; u < kFineU; ++u) {
    rv[u] = -1;
    if (p0 + u * kBlock < b1) {
      const int cl = cell_of(ev[u]);
      if (static_cast<uint32_t>(cl) < static_cast<uint32_t>(S)) {
        rv[u] = atomicAdd(&h[cl], 1);
        if (!staged) emit(ev[u], b0 + rv[u]);
      }
    }
  }
  for (int p = p0 + kFineU * kBlock; p < b1; p += kBlock) {  // only when !staged
    const int4 e = w.coarse[p];
    const int cl = cell_of(e);
    if (static_cast<uint32_t>(cl) < static_cast<uint32_t>(S)) emit(e, b0 + atomicAdd(&h[cl], 1));
  }
  if (staged) {
    for (int q0 = 0; q0 < nbin; q0 += kFineStage) {
      __syncthreads();  // the previous round has read the stage
#pragma unroll
      for (int u = 0; u < kFineU; ++u)
        if (static_cast<uint32_t>(rv[u] - q0) < static_cast<uint32_t>(kFineStage)) stage[rv[u] - q0] = ev[u];
      __syncthreads();
      const int nr = min(kFineStage, nbin - q0);
      for (int r = threadIdx.x; r < nr; r += kBlock) emit(stage[r], b0 + q0 + r);
    }
  }
  if (bin == 0 && threadIdx.x == 0) w.hdr->built = kBuilt;
}

template <bool kFused>
__global__ __launch_bounds__(kBlock) void k_fine_sort(DevWs w, uint32_t step_lo, uint32_t step_hi,
                                                      uint32_t sys_id, uint32_t seed_lo,
                                                      uint32_t seed_hi) {
  fine_sort_body<kFused>(w, blockIdx.x, step_lo, step_hi, sys_id, seed_lo, seed_hi);
}

// ---------------------------------------------------------------------------
// Batched stages.  Workgroup g takes the stage's items g, g + gridDim.x, ...;
// an item is one workgroup's share of one system.  The scan runs on a
// persistent grid (its tiles wait on tiles of running workgroups only); the
// other stages, whose items never wait on one another, launch one workgroup
// per item, so that the hardware hands items of uneven cost to whichever CU
// is free.
// ---------------------------------------------------------------------------
__device__ __forceinline__ const BatchSys& batch_item(const BatchRef& b, int stage, int it, int& li) {
  const BatchSys& d = b.sys[b.items[b.begin[stage] + it]];
  li = it - d.base[stage];
  return d;
}

__global__ __launch_bounds__(kBlock) void k_bb_init(BatchRef b) {
  const int ni = b.begin[kStInit + 1] - b.begin[kStInit];
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    int li;
    const BatchSys& d = batch_item(b, kStInit, it, li);
    ws_init_body(d.w, li, d.nitems[kStInit]);
  }
}

__global__ __launch_bounds__(kBlock) void k_bb_count(BatchRef b) {
  const int ni = b.begin[kStCount + 1] - b.begin[kStCount];
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    int li;
    const BatchSys& d = batch_item(b, kStCount, it, li);
    if (d.w.nbins > 0)
      coarse_count_body<kBlock>(d.x[d.parity], d.y[d.parity], d.w, li);
    else
      bin_count_body(d.x[d.parity], d.y[d.parity], d.w, li);
    __syncthreads();  // the next item's LDS histogram
  }
}

// Tiles of one system's scan are claimed by ticket inside scan_body, so a
// tile only ever waits on tiles already claimed by running workgroups.
__global__ __launch_bounds__(kBlock) void k_bb_scan(BatchRef b) {
  const int ni = b.begin[kStScan + 1] - b.begin[kStScan];
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    int li;
    const BatchSys& d = batch_item(b, kStScan, it, li);
    if (d.w.nbins > 0)
      scan_body(d.w.hist, d.w.hist, static_cast<int64_t>(d.w.nbins) * d.w.nblk, d.w.scan_h, d.w.hdr, 0);
    else
      scan_body(d.w.count, d.w.start, d.w.C, d.w.scan_c, d.w.hdr, 1);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_bb_scatter(BatchRef b) {
  const int ni = b.begin[kStScatter + 1] - b.begin[kStScatter];
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    int li;
    const BatchSys& d = batch_item(b, kStScatter, it, li);
    const int p = d.parity;
    if (d.w.nbins > 0)
      coarse_scatter_body<true, kBlock>(d.x[p], d.y[p], d.th[p], d.w, li);
    else
      scatter_body<true>(d.x[p], d.y[p], d.th[p], d.w, li, d.step_lo, d.step_hi, d.sys_id,
                         d.seed_lo, d.seed_hi);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_bb_fine(BatchRef b) {
  const int ni = b.begin[kStFine + 1] - b.begin[kStFine];
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    int li;
    const BatchSys& d = batch_item(b, kStFine, it, li);
    fine_sort_body<true>(d.w, li, d.step_lo, d.step_hi, d.sys_id, d.seed_lo, d.seed_hi);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_ws_init(const DevWs& w, hipStream_t s) {
  const int64_t want = (w.C + kBlock - 1) / kBlock;
  const int blocks = static_cast<int>(want < 4096 ? (want > 0 ? want : 1) : 4096);
  hipLaunchKernelGGL(k_ws_init, dim3(blocks), dim3(kBlock), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_build(const DevWs& w, const int32_t* x, const int32_t* y, const float* theta,
                        const nm_params* p, uint64_t step, hipStream_t s) {
  const bool fused = theta != nullptr && p != nullptr;
  if (w.nbins > 0 && w.n >= kCoarseMinN) {  // two-level
    hipLaunchKernelGGL(k_coarse_count, dim3(w.nblk), dim3(kCoarseT), 0, s, x, y, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t m = static_cast<int64_t>(w.nbins) * w.nblk;
    e = launch_scan_rows(w.hist, m, w.scan_h, static_cast<int>((m + kScanTile - 1) / kScanTile), w.hdr, s);
    if (e != hipSuccess) return e;
    if (fused) {
      hipLaunchKernelGGL(k_coarse_scatter<true>, dim3(w.nblk), dim3(kCoarseT), 0, s, x, y, theta, w);
      hipLaunchKernelGGL(k_fine_sort<true>, dim3(w.nbins), dim3(kBlock), 0, s, w,
                         static_cast<uint32_t>(step), static_cast<uint32_t>(step >> 32), p->sys_id,
                         static_cast<uint32_t>(p->seed), static_cast<uint32_t>(p->seed >> 32));
    } else {
      hipLaunchKernelGGL(k_coarse_scatter<false>, dim3(w.nblk), dim3(kCoarseT), 0, s, x, y, theta, w);
      hipLaunchKernelGGL(k_fine_sort<false>, dim3(w.nbins), dim3(kBlock), 0, s, w, 0u, 0u, 0u, 0u, 0u);
    }
    return hipGetLastError();
  }
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_bin_count, dim3(nb), dim3(kBlock), 0, s, x, y, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan, dim3(w.nb_scan_c), dim3(kBlock), 0, s, w.count, w.start, w.C, w.scan_c,
                     w.hdr, 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nq = (w.n + 4 * kBlock - 1) / (4 * kBlock);
  if (fused) {
    hipLaunchKernelGGL(k_bin_scatter<true>, dim3(nq), dim3(kBlock), 0, s, x, y, theta, w,
                       static_cast<uint32_t>(step), static_cast<uint32_t>(step >> 32), p->sys_id,
                       static_cast<uint32_t>(p->seed), static_cast<uint32_t>(p->seed >> 32));
  } else {
    hipLaunchKernelGGL(k_bin_scatter<false>, dim3(nq), dim3(kBlock), 0, s, x, y, theta, w, 0u, 0u,
                       0u, 0u, 0u);
  }
  return hipGetLastError();
}

int batch_grid(const void* kernel, int items) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return items < 1 ? 1 : (items < 256 ? items : 256);
    cus = prop.multiProcessorCount;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const long long cap = static_cast<long long>(per_cu) * cus;
  return static_cast<int>(items < 1 ? 1 : (items < cap ? items : cap));
}

hipError_t launch_batch_bin(const BatchRef& b, int stage, hipStream_t s) {
  const int items = b.begin[stage + 1] - b.begin[stage];
  if (items <= 0) return hipSuccess;
  const void* k = nullptr;
  switch (stage) {
    case kStInit: k = reinterpret_cast<const void*>(k_bb_init); break;
    case kStCount: k = reinterpret_cast<const void*>(k_bb_count); break;
    case kStScan: k = reinterpret_cast<const void*>(k_bb_scan); break;
    case kStScatter: k = reinterpret_cast<const void*>(k_bb_scatter); break;
    case kStFine: k = reinterpret_cast<const void*>(k_bb_fine); break;
    default: return hipErrorInvalidValue;
  }
  const int grid = stage == kStScan ? batch_grid(k, items) : items;
  switch (stage) {
    case kStInit: hipLaunchKernelGGL(k_bb_init, dim3(grid), dim3(kBlock), 0, s, b); break;
    case kStCount: hipLaunchKernelGGL(k_bb_count, dim3(grid), dim3(kBlock), 0, s, b); break;
    case kStScan: hipLaunchKernelGGL(k_bb_scan, dim3(grid), dim3(kBlock), 0, s, b); break;
    case kStScatter: hipLaunchKernelGGL(k_bb_scatter, dim3(grid), dim3(kBlock), 0, s, b); break;
    default: hipLaunchKernelGGL(k_bb_fine, dim3(grid), dim3(kBlock), 0, s, b); break;
  }
  return hipGetLastError();
}

// Shared with the metric list: prefix sum over the row lengths.
hipError_t launch_scan_rows(int32_t* data, int64_t m, ScanState* st, int nb, WsHeader* hdr,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(nb), dim3(kBlock), 0, s, data, data, m, st, hdr, 0);
  return hipGetLastError();
}

}  // namespace nm
