// nm_internal.h -- device-side building blocks shared by the HIP kernels.
//
// Layout of the caller-owned workspace (all offsets 256-byte aligned):
//   header      WsHeader: magic, error word, grid echo, build stamp
//   scan_cells  ScanState for the cell-histogram prefix sum
//   scan_metric ScanState for the metric-list row-length prefix sum
//   count       int32[C]     per-cell histogram (kept zero between builds)
//   start       int32[C + 1] first cell-ordered slot of each cell
//   rank        int32[n]     slot of each particle inside its cell
//   sorted      int4[n]      cell-ordered (x, y, particle index, noise word)
//   cs          double2[2n]  cell-ordered (cos theta, sin theta) and (cos phi, sin phi)
//                            of the noise, fused step only
//   dflag       uint8[n]     1 for a slot whose k-NN search is deferred (kept 0
//                            between launches)
//   chunks      int4[cap]    row chunks of dense metric strips, cap = n / 32 + 1024
//   vlist       int32[n]     slots of Voronoi cells handed to the 64-bit kernel
//   coarse      int4[n]      particles in coarse-bin order (two-level binning)
//   hist        int32[nbins * nblk + 1]  per-workgroup coarse-bin counts, then
//                            their exclusive prefix sum (bin-major)
//   scan_hist   ScanState for that prefix sum
// C = G^2 cells, G = L / w.  Cells are numbered row-major: c = cy * G + cx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/nm.h"

namespace nm {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;
// Two-level binning: coarse bins are runs of 2^sb consecutive cells, at most
// kCoarseBins of them; the first pass takes kCoarseP particles per workgroup.
constexpr int kCoarseBins = 1024;
constexpr int kCoarseP = 4096;
constexpr int kFineCells = 4096;  // cells per coarse bin the LDS sort takes (else one-level)
constexpr int kCoarseMinN = 1 << 17;  // smaller single systems: one-level binning (fewer launches)
constexpr int kCoarseMinBatch = 1024;  // the batched stages bin systems from this size in two levels
constexpr int kBinTarget = 1024;      // particles a coarse bin should hold at the mean density
constexpr uint32_t kMagic = 0x4E4D5753u;  // "NMWS"
constexpr uint32_t kBuilt = 0x42554C54u;  // "BULT"
constexpr int kKeyIndexBits = 24;         // particle index field of a search key
constexpr int kMaxParticles = 1 << kKeyIndexBits;

struct WsHeader {
  uint32_t magic;
  int32_t err;
  int32_t n, box, cell_w;
  uint32_t built;
  uint32_t ndefer[2];  // metric rows deferred to the wave kernels (count, fill pass)
  uint32_t nchunk[2];  // metric strip chunks pushed to the chunk kernels (count, fill pass)
  uint32_t nvwide;     // Voronoi cells listed for the 64-bit kernel (in vlist)
  uint32_t nvdone;     // workgroups of that kernel finished (the last one empties the list)
  uint32_t nvstale;    // Voronoi rows listed for recomputation (in rank)
  uint32_t nvfail;     // particles whose Voronoi row failed the last reuse test
  unsigned long long varea2;  // sum over Voronoi rows of a_t x a_{t+1} (six times the area covered)
  int32_t pad[48];
};
static_assert(sizeof(WsHeader) == 256, "header is one 256-byte block");

struct ScanState {
  uint32_t ticket;
  uint32_t pad[63];
  unsigned long long flags[1];  // one word per tile (flexible)
};

// Host-computed view of a workspace, passed to kernels by value.
struct DevWs {
  WsHeader* hdr;
  ScanState* scan_c;
  ScanState* scan_m;
  int32_t* count;
  int32_t* start;
  int32_t* rank;  // in-cell rank while binning; then the metric kernels' deferred list
  int4* sorted;
  double2* cs;
  uint8_t* dflag;
  int4* chunks;
  int32_t* vlist;
  int4* coarse;
  int32_t* hist;
  ScanState* scan_h;
  int32_t chunk_cap;
  int32_t sb, nbins, nblk, nb_scan_h;  // two-level binning (nbins == 0: one-level)
  int32_t n;
  int32_t box;
  int32_t cell_w;
  int32_t log2_box;
  int32_t log2_w;
  int32_t G;
  int32_t nb_scan_c;
  int32_t nb_scan_m;
  int64_t C;
};

struct Layout {
  int64_t off_scan_c, off_scan_m, off_count, off_start, off_rank, off_sorted, off_cs,
      off_dflag, off_chunks, off_vlist, off_coarse, off_hist, off_scan_h, total;
  int32_t log2_box, log2_w, G, nb_scan_c, nb_scan_m, chunk_cap, sb, nbins, nblk, nb_scan_h;
  int64_t C;
};

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void set_err(WsHeader* h, int code) {
  if (h) atomicCAS(&h->err, 0, code);
}

// Signed offset congruent to d modulo L = 2^(32 - sh), in [-L/2, L/2).
__device__ __forceinline__ int wrap_axis(int d, int sh) {
  return static_cast<int>(static_cast<uint32_t>(d) << sh) >> sh;
}

// Smallest |offset| (minimum image) from a query at offset o inside its own
// cell to any point of the cell `dc` columns away (cells of width w).
__device__ __forceinline__ int axis_gap(int dc, int o, int w, int sh) {
  if (dc == 0) return 0;
  const int a = dc * w - o;
  const int b = a + w - 1;
  return min(abs(wrap_axis(a, sh)), abs(wrap_axis(b, sh)));
}

// Map a hardware block id to a logical tile so that each of the 8 XCDs (which
// receive blocks round-robin) walks one contiguous stretch of the cell-ordered
// particles: neighbouring queries then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, t = b >> 3;
  return x * q + min(x, r) + t;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
// Ten rounds; each round multiplies words 0 and 2 by fixed odd constants,
// swaps the halves and folds in the round key; the key advances by a Weyl
// sequence between rounds.
// ---------------------------------------------------------------------------
struct Philox {
  static constexpr uint32_t kMulA = 0xD2511F53u;
  static constexpr uint32_t kMulB = 0xCD9E8D57u;
  static constexpr uint32_t kWeylA = 0x9E3779B9u;
  static constexpr uint32_t kWeylB = 0xBB67AE85u;

  __device__ static uint4 block(uint4 c, uint32_t ka, uint32_t kb) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      const uint32_t hA = __umulhi(kMulA, c.x), lA = kMulA * c.x;
      const uint32_t hB = __umulhi(kMulB, c.z), lB = kMulB * c.z;
      c = make_uint4(hB ^ c.y ^ ka, lB, hA ^ c.w ^ kb, lA);
      ka += kWeylA;
      kb += kWeylB;
    }
    return c;
  }
};

__device__ __forceinline__ uint32_t uint4_word(uint4 v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

// Noise angle phi = (u 2^-32) 2pi - pi, each fp64 operation rounded separately
// (the library is compiled with -ffp-contract=off, so no fused multiply-add).
__device__ __forceinline__ double noise_angle(uint32_t u) {
  const double unit = static_cast<double>(u) * 0x1p-32;  // exact
  const double turn = unit * 6.283185307179586;           // fp64(2 pi)
  return turn - 3.141592653589793;                        // fp64(pi)
}

// Direction of the alignment vector (vx, vy) as an fp32 angle: the vector is
// rescaled exactly by a power of two into [1/2, 1) and then rounded to fp32
// for atan2f, so the angle moves by under 2^-23 rad plus atan2f's own error.
// The zero vector keeps `keep` (the normaliser of Eq. (2) is undefined there).
__device__ __forceinline__ float vec_angle(double vx, double vy, float keep) {
  const double mx = fmax(fabs(vx), fabs(vy));
  if (mx == 0.0) return keep;
  int ex;
  frexp(mx, &ex);
  return atan2f(static_cast<float>(ldexp(vy, -ex)), static_cast<float>(ldexp(vx, -ex)));
}

constexpr uint32_t kVariantMask = NM_NOISE_SCALAR | NM_MOVE_NEW_HEADING;

// The two variants, out of line so that the default path keeps its
// register footprint in the kernels that inline it.
//   angular noise: arg(A) + eta phi in fp64 (th + eta phi when A = 0),
//                  wrapped into [-pi, pi) by t - 2pi floor((t + pi) / 2pi);
//   new-heading move: v0 (cos, sin) of the new heading, rounded half to even.
inline __device__ __noinline__ float scalar_noise_heading(double ax, double ay, double phi, float eta,
                                                         float th) {
  const double base = (ax == 0.0 && ay == 0.0) ? static_cast<double>(th) : atan2(ay, ax);
  const double t = base + static_cast<double>(eta) * phi;
  const double two_pi = 6.283185307179586;  // fp64(2 pi)
  return static_cast<float>(t - two_pi * floor((t + 3.141592653589793) / two_pi));
}

inline __device__ __noinline__ int2 new_heading_move(int v0, float thn) {
  double s, c;
  sincos(static_cast<double>(thn), &s, &c);
  return make_int2(static_cast<int>(rint(static_cast<double>(v0) * c)),
                   static_cast<int>(rint(static_cast<double>(v0) * s)));
}

// New heading of particle with heading *thp (read only when needed), from
// the average (ax, ay) of the unit vectors of Eq. (2) (zero when there are
// none) and its noise angle phi with unit vector (xc, xs): the direction of
// A + eta xi, the zero vector keeping the heading (Eq. (2)), or the angular
// noise variant.
__device__ __forceinline__ float heading_update(double ax, double ay, double xc, double xs, double phi,
                                                float eta, const float* thp, uint32_t variant) {
  if (variant & NM_NOISE_SCALAR) return scalar_noise_heading(ax, ay, phi, eta, *thp);
  const double e = static_cast<double>(eta);
  const double vx = ax + e * xc;
  const double vy = ay + e * xs;
  return (vx == 0.0 && vy == 0.0) ? *thp : vec_angle(vx, vy, 0.0f);
}

// Displacement of Eq. (1), rounded to the grid (half to even): v0 times the
// unit vector (own_c, own_s) of the heading at time t, or of the new heading
// thn with NM_MOVE_NEW_HEADING.
__device__ __forceinline__ void move_step(int v0, double own_c, double own_s, float thn, uint32_t variant,
                                          int& ddx, int& ddy) {
  if (variant & NM_MOVE_NEW_HEADING) {
    const int2 d = new_heading_move(v0, thn);
    ddx = d.x;
    ddy = d.y;
    return;
  }
  ddx = static_cast<int>(rint(static_cast<double>(v0) * own_c));
  ddy = static_cast<int>(rint(static_cast<double>(v0) * own_s));
}

// ---------------------------------------------------------------------------
// Register-resident sorted list of the KMAX smallest 64-bit keys.  The first
// KMAX - k entries hold the sentinel 0 (below every real key, which is >= 1),
// so the last k entries act as a sorted list of length k with its largest
// element at a fixed register, keys[KMAX - 1].
// ---------------------------------------------------------------------------
// With kSlots, each key carries the cell-ordered slot of its particle along.
template <int KMAX, bool kSlots = false>
struct TopK {
  unsigned long long key[KMAX];
  int32_t slot[kSlots ? KMAX : 1];

  __device__ void init(int k) {
#pragma unroll
    for (int t = 0; t < KMAX; ++t) key[t] = (t < KMAX - k) ? 0ull : ~0ull;
#pragma unroll
    for (int t = 0; t < (kSlots ? KMAX : 1); ++t) slot[t] = -1;
  }
  __device__ unsigned long long worst() const { return key[KMAX - 1]; }

  // Insert (kk, s) and drop the largest entry.  Caller ensures kk < worst().
  __device__ void push(unsigned long long kk, int32_t s) {
#pragma unroll
    for (int t = KMAX - 1; t > 0; --t) {
      const bool shift = kk < key[t - 1];
      const bool here = kk < key[t];
      const unsigned long long nk = shift ? key[t - 1] : (here ? kk : key[t]);
      if constexpr (kSlots) slot[t] = shift ? slot[t - 1] : (here ? s : slot[t]);
      key[t] = nk;
    }
    if (kk < key[0]) {
      key[0] = kk;
      if constexpr (kSlots) slot[0] = s;
    }
  }
};

// Search key of a candidate: (d^2, index) packed so that integer order is the
// lexicographic order; +1 keeps 0 free for the sentinel.  d^2 <= 2^39 for
// L <= 2^20, so the packed value stays below 2^64.
__device__ __forceinline__ unsigned long long pack_key(long long d2, int32_t j) {
  return ((static_cast<unsigned long long>(d2) << kKeyIndexBits) |
          static_cast<unsigned long long>(j)) + 1ull;
}
__device__ __forceinline__ int32_t key_index(unsigned long long kk) {
  return static_cast<int32_t>((kk - 1ull) & ((1ull << kKeyIndexBits) - 1ull));
}
__device__ __forceinline__ long long key_d2(unsigned long long kk) {
  return static_cast<long long>((kk - 1ull) >> kKeyIndexBits);
}
__device__ __forceinline__ long long key_bound_d2(unsigned long long kk) {
  // d^2 of the current worst key, or "infinite" while the list is not full.
  return kk == ~0ull ? (1ll << 62) : key_d2(kk);
}

// ---------------------------------------------------------------------------
// Ring walk over the cell grid.  Ring r holds the 8r cells at Chebyshev
// distance r from the home cell (one cell for r = 0), walked once around the
// perimeter from (-r, -r).  Offsets outside one window [lo, hi] of G
// consecutive values per axis are skipped, so that no cell is visited twice
// when rings wrap around the periodic box.  `visit(dx, dy)` has a single call
// site, which keeps one inlined copy of the candidate loop.
// ---------------------------------------------------------------------------
template <class Visit>
__device__ __forceinline__ void for_ring(int r, int lo, int hi, Visit&& visit) {
  const int ncell = r == 0 ? 1 : 8 * r;
  int dx = -r, dy = -r, sx = 1, sy = 0, left = 2 * r;
#pragma unroll 1
  for (int q = 0; q < ncell; ++q) {
    if (dx >= lo && dx <= hi && dy >= lo && dy <= hi) visit(dx, dy);
    dx += sx;
    dy += sy;
    if (--left == 0) {
      left = 2 * r;
      const int t = sx;
      sx = -sy;
      sy = t;
    }
  }
}

// Query geometry derived from its position.
struct QueryGeom {
  int hx, hy, ox, oy, edge, lo, hi, rmax;
  __device__ QueryGeom(int qx, int qy, const DevWs& w) {
    const int cw = 1 << w.log2_w;
    hx = qx >> w.log2_w;
    hy = qy >> w.log2_w;
    ox = qx & (cw - 1);
    oy = qy & (cw - 1);
    edge = min(min(ox, cw - 1 - ox), min(oy, cw - 1 - oy));
    lo = -(w.G >> 1);
    hi = w.G - 1 - (w.G >> 1);
    rmax = max(-lo, hi);
  }
  // Lower bound on d^2 of any particle outside rings 0..r.
  __device__ long long ring_bound(int r, int cw) const {
    const long long b = static_cast<long long>(r) * cw + edge + 1;
    return b * b;
  }
};

// ---------------------------------------------------------------------------
// Fast-path search block.  A B x B block of cells around the query: for odd
// B centred on its home cell, for even B shifted toward the half of the home
// cell that holds the query, so that the query is at least (B - 1) / 2 cell
// widths from every cell outside.  Each block row is one contiguous range of
// cell-ordered slots, or two where the row wraps around the box in x; range
// 2r + part covers part `part` of block row r.  Candidates get 32-bit keys
//   (min(d^2, bound) >> sh) << 13 | range << 8 | offset in the range,
// pushed through a branch-free insertion network; a neighbour's slot is
// start[first cell of its range] + offset.  The result is used only when
// certified exact: every range shorter than 256, the k+1 smallest keys with
// distinct distance fields, and the k-th squared distance strictly below the
// squared distance from the query to the nearest cell outside the block.
// ---------------------------------------------------------------------------
constexpr int kMaxB = 15;  // 2 * kMaxB ranges fit the 5-bit range field
constexpr uint32_t kKey32Inf = 0xFFFFFFFFu;
constexpr int kDBits = 19;  // distance field of a 32-bit key

struct FastCfg {
  int bmax;    // largest block side of 32-bit distances (0 disables the fast path)
  int bfix;    // fixed block side, or 0 to pick it per query from density
  float reach; // distance to the block edge, in mean k-th-neighbour radii
  int bmax_w;  // largest block side of the 64-bit-distance ("wide") tiles
  int split;   // strips whose halo overflows LDS run as staged sub-strips
};

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Branch-free insertion of kk into an ascending list of KT keys whose first
// entries may be the sentinel 0: key[t] <- med3(key[t-1], kk, key[t]).
template <int KT>
__device__ __forceinline__ void net_insert(uint32_t (&key)[KT], uint32_t kk) {
#pragma unroll
  for (int t = KT - 1; t > 0; --t) key[t] = umed3(key[t - 1], kk, key[t]);
  key[0] = min(key[0], kk);
}

__device__ __forceinline__ uint32_t key32_d(uint32_t kk) { return kk >> 13; }

// One list row of k entries, v[KMAX - k .. KMAX): a full row goes out as
// 16-byte and smaller vector stores (rows start on any 4-byte boundary), so
// that a wavefront's scattered rows cost a few stores per lane, not k.
typedef int nm_int4u __attribute__((ext_vector_type(4), aligned(4)));
typedef int nm_int3u __attribute__((ext_vector_type(3), aligned(4)));
typedef int nm_int2u __attribute__((ext_vector_type(2), aligned(4)));
// Only short rows are gathered for vector stores: holding a longer row in
// registers until its last entry raises the register count of the kernels
// with large KMAX past what the stores save.
template <int KMAX>
constexpr bool kRowVec = KMAX <= 8;

template <int KMAX>
__device__ __forceinline__ void store_row(int32_t* row, const int (&v)[KMAX], int k) {
  if (k == KMAX) {
#pragma unroll
    for (int t = 0; t + 4 <= KMAX; t += 4)
      *reinterpret_cast<nm_int4u*>(row + t) = nm_int4u{v[t], v[t + 1], v[t + 2], v[t + 3]};
    constexpr int b = KMAX & ~3, r = KMAX & 3;
    if constexpr (r == 3) *reinterpret_cast<nm_int3u*>(row + b) = nm_int3u{v[b], v[b + 1], v[b + 2]};
    if constexpr (r == 2) *reinterpret_cast<nm_int2u*>(row + b) = nm_int2u{v[b], v[b + 1]};
    if constexpr (r == 1) row[b] = v[b];
  } else {
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
      if (t >= KMAX - k) row[t - (KMAX - k)] = v[t];
  }
}

// Geometry of one query's block.
struct QBlock {
  int hx, hy, lo_x, lo_y, B, sh;
  long long bound;  // squared distance to the nearest cell outside the block
};

__device__ __forceinline__ QBlock make_qblock(const DevWs& w, int qx, int qy, int B) {
  QBlock b;
  const int cw = 1 << w.log2_w;
  b.hx = qx >> w.log2_w;
  b.hy = qy >> w.log2_w;
  const int ox = qx & (cw - 1), oy = qy & (cw - 1);
  const int half = B >> 1;
  b.lo_x = (B & 1) ? -half : -half + (ox >= (cw >> 1) ? 1 : 0);
  b.lo_y = (B & 1) ? -half : -half + (oy >= (cw >> 1) ? 1 : 0);
  b.B = B;
  const int hi_x = b.lo_x + B - 1, hi_y = b.lo_y + B - 1;
  const int gl = ox - b.lo_x * cw + 1, gr = (hi_x + 1) * cw - ox;
  const int gd = oy - b.lo_y * cw + 1, gu = (hi_y + 1) * cw - oy;
  const long long m = min(min(gl, gr), min(gd, gu));
  b.bound = m * m;
  const int bits = 64 - __clzll(b.bound);
  b.sh = bits > kDBits ? bits - kDBits : 0;
  return b;
}

// Cell range of part `part` (0 or 1) of block row r: first cell index, cell
// count (0 if the part is empty), and the query's x / y in that range's image.
struct RangeGeom {
  int64_t cell0;
  int ncell;
  int qx, qy;
};

__device__ __forceinline__ RangeGeom range_geom(const DevWs& w, const QBlock& b, int r, int part,
                                                int qx, int qy) {
  const int G = w.G, L = w.box;
  RangeGeom g;
  int cy = b.hy + b.lo_y + r;
  g.qy = qy;
  if (cy < 0) {
    cy += G;
    g.qy = qy + L;
  } else if (cy >= G) {
    cy -= G;
    g.qy = qy - L;
  }
  const int c0 = b.hx + b.lo_x, c1 = b.hx + b.lo_x + b.B - 1;
  int a, e;
  g.qx = qx;
  if (c0 < 0) {  // part 0: the wrapped cells on the right edge, part 1: from column 0
    if (part == 0) {
      a = c0 + G;
      e = G - 1;
      g.qx = qx + L;
    } else {
      a = 0;
      e = c1;
    }
  } else if (c1 >= G) {  // part 0: up to the right edge, part 1: wrapped from column 0
    if (part == 0) {
      a = c0;
      e = G - 1;
    } else {
      a = 0;
      e = c1 - G;
      g.qx = qx - L;
    }
  } else {
    a = c0;
    e = part == 0 ? c1 : c0 - 1;
  }
  g.cell0 = static_cast<int64_t>(cy) * G + a;
  g.ncell = e - a + 1;
  return g;
}

// Walk the block's candidates.  visit(x, y, qx_image, qy_image, tag, valid)
// gets tag = range << 8 | offset; pairs of candidates are loaded together
// (the second clamped into the range, arriving with valid = false when it is
// padding).  Returns false if a range is too long for the 8-bit offset.
template <class Visit>
__device__ __forceinline__ bool walk_block(const DevWs& w, const QBlock& b, int s, int qx, int qy,
                                           int total, Visit&& visit) {
  const int2* pos = reinterpret_cast<const int2*>(w.sorted);
  bool ok = true;
  for (int r = 0; r < b.B; ++r) {
    for (int part = 0; part < 2; ++part) {
      const RangeGeom g = range_geom(w, b, r, part, qx, qy);
      if (g.ncell <= 0) continue;
      const int a = w.start[g.cell0];
      const int e = min(w.start[g.cell0 + g.ncell], total);
      if (e - a > 256) ok = false;
      const int tag0 = ((2 * r + part) << 8) - a;  // tag of slot t is tag0 + t
      auto run = [&](int t0, int t1) {
        for (int t = t0; t < t1; t += 2) {
          const int u = min(t + 1, t1 - 1);
          const int2 p0 = pos[2 * t], p1 = pos[2 * u];
          visit(p0.x, p0.y, g.qx, g.qy, tag0 + t, true);
          visit(p1.x, p1.y, g.qx, g.qy, tag0 + u, t + 1 < t1);
        }
      };
      if (s >= a && s < e) {  // the query's own range: skip its slot
        run(a, s);
        run(s + 1, e);
      } else {
        run(a, e);
      }
    }
  }
  return ok;
}

// Slot of the candidate with tag `tag` in block b.
__device__ __forceinline__ int tag_slot(const DevWs& w, const QBlock& b, uint32_t tag, int qx, int qy) {
  const int rid = static_cast<int>((tag >> 8) & 31u);
  const RangeGeom g = range_geom(w, b, rid >> 1, rid & 1, qx, qy);
  return w.start[g.cell0] + static_cast<int>(tag & 255u);
}

// k-NN strip geometry (knn.hip): a workgroup owns a strip of tw x th cells
// and stages a halo of hx columns and hy rows around it.
struct TileCfg {
  int tw, th;  // strip width and height in cells
  int hx, hy;  // halo in cells (hx = 0: no staging)
  int ntx;     // strips across (G / tw)
  int nty;     // strips down
  int bmax;    // largest block height (rows) the halo supports
  int wide;    // 1: staged offsets are int32 pairs and distances 64-bit (a
               // block spans 2^15 units or more); 0: packed 16-bit offsets
};

// Parameters and outputs of the fused Eq. (2) / Eq. (1) epilogue.
struct AlignArgs {
  int32_t v0;
  float eta;
  int32_t include_self;
  uint32_t variant;  // NM_NOISE_SCALAR, NM_MOVE_NEW_HEADING
  const float* theta;
  int32_t* x_out;
  int32_t* y_out;
  float* theta_out;
  int32_t cone;  // field-of-view lists: cos(half angle) * 4096
};

// ---------------------------------------------------------------------------
// Batched form: many independent systems advanced by one launch per stage.
// Each stage is a persistent launch whose workgroups walk the stage's work
// items (items of one system are contiguous; `items` maps an item to its
// system).  The state of system s is double-buffered: step t reads buffer
// `parity` and writes buffer 1 - parity; the advance stage flips the parity
// and increments the step, so one captured step replays for any step.
// ---------------------------------------------------------------------------
// The k-NN stage is two: systems whose grid uses the sub-strip kernel
// (NM_BLOCK_SUBSTRIPS) have their tiles in kStKnnSplit, the others in kStKnn.
// Systems binned in two levels (workspace nbins > 0) run the coarse count,
// the scan of their bin x block table, the coarse scatter and the per-bin
// sort in kStCount, kStScan, kStScatter and kStFine; the others run the
// one-level count, scan and scatter and have no kStFine items.
enum BatchStage { kStInit = 0, kStCount, kStScan, kStScatter, kStFine, kStKnn, kStKnnSplit, kStages };

struct BatchSys {
  DevWs w;
  FastCfg f;
  TileCfg tc;
  int32_t* x[2];
  int32_t* y[2];
  float* th[2];
  int32_t* nbr;       // int32[n * k], this system's rows
  int32_t v0;
  float eta;
  int32_t include_self;
  uint32_t variant;
  uint32_t sys_id, seed_lo, seed_hi;
  uint32_t step_lo, step_hi;  // Philox step of the next step (device-updated)
  int32_t parity;             // buffer holding the current state (device-updated)
  int32_t ntiles;             // k-NN tiles
  int32_t base[kStages];      // first item of this system in each stage
  int32_t nitems[kStages];    // items of this system in each stage
};

// A workgroup-uniform copy of a descriptor read from global memory, held in
// scalar registers (the loads are vector loads because earlier stores of the
// kernel may alias them; each dword is then taken from the first lane).
template <class T>
__device__ __forceinline__ T uniform_load(const T* src) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized descriptor");
  T out;
  const int* s = reinterpret_cast<const int*>(src);
  int* o = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int i = 0; i < static_cast<int>(sizeof(T) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(s[i]);
  return out;
}

struct BatchRef {
  BatchSys* sys;        // device array [nsys]
  const int32_t* items; // device: stage item -> system, stages concatenated
  int32_t nsys;
  int32_t begin[kStages + 1];  // stage s owns items [begin[s], begin[s + 1])
};

// Host-side helpers (abi.hip).// Host-side helpers (abi.hip).
bool make_layout(const nm_grid* g, Layout* out);
DevWs dev_ws(const nm_grid* g, const Layout& lay, void* ws);

// Launchers implemented in the kernel files.
hipError_t launch_ws_init(const DevWs& w, hipStream_t s);
hipError_t launch_build(const DevWs& w, const int32_t* x, const int32_t* y, const float* theta,
                        const nm_params* p, uint64_t step, hipStream_t s);
FastCfg fast_cfg(const DevWs& w, int k, int block);
hipError_t launch_knn(const DevWs& w, int k, int block, int32_t* nbr, long long* d2, hipStream_t s);
hipError_t launch_knn_align(const DevWs& w, int k, int block, const nm_params* p,
                            const float* theta, int32_t* nbr, int32_t* x_out, int32_t* y_out,
                            float* theta_out, hipStream_t s);
hipError_t launch_metric_count(const DevWs& w, long long rc2, int32_t* offsets, hipStream_t s);
hipError_t launch_metric_fill(const DevWs& w, long long rc2, const int32_t* offsets, int32_t* idx,
                              long long cap, hipStream_t s);
hipError_t launch_scan_rows(int32_t* data, int64_t m, ScanState* st, int nb, WsHeader* hdr,
                            hipStream_t s);
TileCfg tile_cfg(const DevWs& w, const FastCfg& f, int k);
// Host-only description of the k-NN kernel a grid runs (nm_knn_layout).
void knn_layout(const DevWs& w, int k, int block, int32_t out[10]);
// Persistent grid for a batched stage: at most `items` workgroups, at most
// what stays resident on the device.
int batch_grid(const void* kernel, int items);
hipError_t launch_batch_bin(const BatchRef& b, int stage, hipStream_t s);
hipError_t launch_batch_knn(const BatchRef& b, int k, hipStream_t s);
hipError_t launch_batch_advance(const BatchRef& b, hipStream_t s);
hipError_t launch_knn_fov(const DevWs& w, int block, const float* theta, int k, int c, int32_t* nbr,
                          hipStream_t s);
hipError_t launch_knn_fov_strips(const DevWs& w, int block, const float* theta, int k, int c,
                                 int32_t* nbr, hipStream_t s);
hipError_t launch_polar_order(const float* theta, int32_t n, double* sums, hipStream_t s);
hipError_t launch_voronoi(const DevWs& w, int dmax, int32_t* ring, int32_t* deg, hipStream_t s);
hipError_t launch_voronoi_forces(const int32_t* x, const int32_t* y, int32_t n, int log2_box, int dmax,
                                 const int32_t* ring, const int32_t* deg, const nm_vm_params* p,
                                 double* area, double* perim, double* fx, double* fy, double* energy,
                                 double* vert, WsHeader* err, hipStream_t s);
hipError_t launch_voronoi_check(const DevWs& w, const int32_t* x, const int32_t* y, int dmax,
                                const int32_t* ring, const int32_t* deg, uint8_t* stale, int32_t* nfail,
                                hipStream_t s);
hipError_t launch_voronoi_update(const DevWs& w, const int32_t* x, const int32_t* y, int dmax,
                                 int32_t* ring, int32_t* deg, uint8_t* stale, int32_t* nfail, int rounds,
                                 hipStream_t s);
hipError_t launch_align(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                        const int32_t* nbr, const int32_t* offsets, int32_t k, long long nnz_cap,
                        const nm_params* p, uint64_t step, int32_t* x_out, int32_t* y_out,
                        float* theta_out, WsHeader* err_hdr, hipStream_t s);

}  // namespace nm
