// strip.h -- LDS staging of a strip of cells with its halo, shared by the
// k-NN kernel (knn.hip) and the metric-list kernels (metric.hip).
//
// A strip is tw columns by ty rows of cells starting at (x0, y0); its halo
// adds hx columns either side and hy rows above and below (W = tw + 2 hx
// columns, R = ty + 2 hy rows, W <= G).  Staging writes, in LDS:
//   rbase[r]   offset of halo row r (r <= R); each row holds the particles of
//              its W cells in cell order, in one or two slot ranges (the
//              columns wrap around the box at most once)
//   lpos[p]    the particle's position in the strip's periodic image relative
//              to the halo corner: a packed pair of 16-bit offsets (narrow),
//              or an int32 pair (wide)
//   lslot[p]   its cell-ordered slot, or (kStoreIndex) its particle index
//   qoff[rq]   prefix of the strip's own queries over its rows (rq <= ty)
//   tself[rq]  LDS index of the first query of strip row rq
#pragma once

#include "nm_internal.h"

namespace nm {

constexpr int kStripPts = 2560;           // staged particles (wide strips: half)
constexpr int kStripRows = 128;           // R <= kStripRows (row tables small enough for 5 strips per CU)
constexpr int kRowStep = kStripRows / 2;  // binary search over <= kStripRows rows
constexpr int kTwRows = 256;              // strips widen while ~256 queries need more rows than this
constexpr int kUnroll = 4;                // candidates read per round of a block loop

// Exclusive prefix sum of v over the workgroup (thread order); *total gets
// the sum.  Uses s_wsum[kBlock / 64].
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) {
    if (q < wave) before += s_wsum[q];
    all += s_wsum[q];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

typedef short short2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int rel_d2(int packed_c, int packed_q) {
  const short2v d = __builtin_bit_cast(short2v, packed_c) - __builtin_bit_cast(short2v, packed_q);
  return __builtin_amdgcn_sdot2(d, d, 0, false);
}

// The same as an unsigned 32-bit value (below 2^31 + 1), the dot product
// taken with a zero accumulator operand, so that no register is cleared first.
__device__ __forceinline__ uint32_t rel_d2_u(int packed_c, int packed_q) {
  const short2v d = __builtin_bit_cast(short2v, packed_c) - __builtin_bit_cast(short2v, packed_q);
  uint32_t r;
  asm("v_dot2_i32_i16 %0, %1, %1, 0" : "=v"(r) : "v"(__builtin_bit_cast(int, d)));
  return r;
}

__device__ __forceinline__ int pack_rel(int rx, int ry) {
  return static_cast<int>((static_cast<uint32_t>(rx) & 0xFFFFu) | (static_cast<uint32_t>(ry) << 16));
}

struct StripGeo {
  int x0, y0, ty, tw, hx, hy;
  bool wide;
};

struct StripLds {
  int2* lpos_store;  // [kStripPts / 2 + kUnroll] (narrow: read as int[])
  int* lslot;        // [kStripPts]
  int* rbase;        // [kStripRows + 1]
  int* ga0;          // [kStripRows] first slot of the row's first piece
  int* n0;           // [kStripRows] particles in the row's first piece
  int* ga1;          // [kStripRows] first slot of its second piece
  int* qoff;         // [kStripRows + 1]
  int* tself;        // [kStripRows]
  int* wsum;         // [kBlock / 64]
  uint8_t* rowid;    // [kStripPts] halo row of each staged particle
  uint16_t* qmap;    // [kStripPts] LDS index of each query of the strip (may be null)
};

// Cell-ordered slot of staged particle i (the inverse of the staging copy).
__device__ __forceinline__ int strip_slot(const StripLds& s, int i) {
  const int r = s.rowid[i];
  const int inrow = i - s.rbase[r];
  const int n0 = s.n0[r];
  return inrow >= n0 ? s.ga1[r] + (inrow - n0) : s.ga0[r] + inrow;
}

// Row tables and (when the halo fits: hx > 0 and npts <= cap) the staged
// particles of strip g.  Every thread of the workgroup must call it; it ends
// with a barrier.  Returns whether the particles were staged; npts and nq
// get the halo's and the strip's particle counts.
template <bool kStoreIndex>
__device__ __forceinline__ bool strip_stage(const DevWs& w, const StripGeo& g, const StripLds& s,
                                            int total, int& npts, int& nq) {
  const int G = w.G, L = w.box, gm = G - 1, lw = w.log2_w;
  const int hx = g.hx, hy = g.hy, tw = g.tw;
  const int R = g.ty + 2 * hy;
  const int uL = g.x0 - hx, uR = g.x0 + tw + hx - 1;
  const int ox0 = uL << lw, oy0 = (g.y0 - hy) << lw;  // halo corner (strip image)
  int* lpos = reinterpret_cast<int*>(s.lpos_store);

  // Each halo row (one per thread): its one or two slot ranges and, for the
  // strip's own rows, the query range.
  int rlen = 0, qlen = 0, qrow_off = 0;
  const int rho = threadIdx.x;
  if (rho < R) {
    const int v = g.y0 - hy + rho;
    const int64_t prow = static_cast<int64_t>(v & gm) * G;
    if (hx > 0) {
      const int e0 = uL < 0 ? -1 : min(uR, G - 1);  // last column of the first piece
      const int ga0 = w.start[prow + (uL & gm)];
      const int n0 = w.start[prow + (e0 & gm) + 1] - ga0;
      int n1 = 0, ga1 = 0;
      if (e0 < uR) {
        ga1 = w.start[prow + ((e0 + 1) & gm)];
        n1 = w.start[prow + (uR & gm) + 1] - ga1;
      }
      s.ga0[rho] = ga0;
      s.n0[rho] = n0;
      s.ga1[rho] = ga1;
      rlen = n0 + n1;
      // the strip's own columns start at unwrapped column x0 (in [0, G)):
      // in the second piece when the first one is the wrapped left edge
      qrow_off = uL < 0 ? n0 + (w.start[prow + g.x0] - ga1) : w.start[prow + g.x0] - ga0;
    }
    const int rq = rho - hy;
    if (rq >= 0 && rq < g.ty) {
      const int a0 = w.start[prow + g.x0];
      qlen = max(min(w.start[prow + g.x0 + tw], total) - a0, 0);
    }
  }
  const int rb = block_exclusive_scan(rlen, s.wsum, &npts);
  if (rho < R) s.rbase[rho] = rb;
  const int rq = rho - hy;
  const bool qrow = rho < R && rq >= 0 && rq < g.ty;
  const int qo = block_exclusive_scan(qrow ? qlen : 0, s.wsum, &nq);
  if (qrow) {
    s.qoff[rq] = qo;
    s.tself[rq] = rb + qrow_off;
  }
  if (threadIdx.x == 0) {
    s.rbase[R] = npts;
    s.qoff[g.ty] = nq;
  }
  __syncthreads();
  const bool staged = nq > 0 && hx > 0 && npts <= (g.wide ? kStripPts / 2 : kStripPts);
  if (staged) {
    // Row of every staged particle (one thread per halo row), then the
    // particles as offsets from the halo corner, one per thread per round.
    if (rho < R)
      for (int p = rb; p < rb + rlen; ++p) s.rowid[p] = static_cast<uint8_t>(rho);
    if (s.qmap && qrow)
      for (int j = 0; j < qlen; ++j) s.qmap[qo + j] = static_cast<uint16_t>(rb + qrow_off + j);
    __syncthreads();
    constexpr int kCopyU = 4;  // particles per thread per round: their loads go out together
    for (int base = threadIdx.x; base < npts; base += kCopyU * kBlock) {
      int4 e[kCopyU];
      int ox[kCopyU], oy[kCopyU], sv[kCopyU];
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int pidx = base + u * kBlock;
        if (pidx < npts) {
          const int r = s.rowid[pidx];
          const int inrow = pidx - s.rbase[r];
          const int n0 = s.n0[r];
          const bool second = inrow >= n0;
          const int src = second ? s.ga1[r] + (inrow - n0) : s.ga0[r] + inrow;
          ox[u] = (second ? (uL < 0 ? 0 : L) : (uL < 0 ? -L : 0)) - ox0;
          const int v = g.y0 - hy + r;
          oy[u] = (v < 0 ? -L : (v >= G ? L : 0)) - oy0;
          sv[u] = src;
          e[u] = w.sorted[src];
        }
      }
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int pidx = base + u * kBlock;
        if (pidx < npts) {
          if (g.wide)
            s.lpos_store[pidx] = make_int2(e[u].x + ox[u], e[u].y + oy[u]);
          else
            lpos[pidx] = pack_rel(e[u].x + ox[u], e[u].y + oy[u]);
          s.lslot[pidx] = kStoreIndex ? e[u].z : sv[u];
        }
      }
    }
    __syncthreads();
  }
  return staged;
}

}  // namespace nm
