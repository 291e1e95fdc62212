// vmodel.hip -- the Voronoi model of dense tissue (Sec. V): each particle
// owns its Voronoi cell, the energy is Eq. (3),
//   E = sum_i K_A (A_i - A_0)^2 + K_P (P_i - P_0)^2,
// and the force on particle i is -dE/dr_i (Eq. 9), by the chain rule through
// the cell vertices (Eqs. 10-19); the vertex forces -dE/dh of the vertex
// model (Eqs. 5-8) are a by-product.
//
// Input: the Voronoi rows of nm_voronoi (counter-clockwise; consecutive
// entries a_t, a_{t+1} of row i are the Delaunay triangle (i, a_t, a_{t+1})
// whose circumcentre h_t is vertex t of cell i).  One lane per particle, two
// passes:
//   1. the vertices h_t (relative to the particle), the area (shoelace) and
//      the perimeter of every cell;
//   2. for every vertex h_t of cell i, dE/dh_t summed over the three cells
//      that share it (cell i, cell a_t and cell a_{t+1}; each needs h_t's two
//      neighbours in its own polygon: h_{t-1}, h_{t+1} and the vertex across
//      the edge between a_t and a_{t+1}, found in a_t's row), then
//      F_i -= (dh_t/dr_i)^T dE/dh_t.
// Vectors r_ab point from a to b.  Readings of the printed formulas (they
// are the gradient of Eq. 3 only so; finite differences of the energy decide):
// Eq. (8) dP/dh = t_ij/|t_ij| - t_ik/|t_ik|; c = r_ij x r_jk in Eqs. (15) and
// (19); Eq. (18) ends in -|r_ij|^2 r_jk.
// Everything is fp64 from exact integer minimum-image offsets.
#include "nm_internal.h"

namespace nm {
namespace {

struct V2 {
  double x, y;
};
__device__ __forceinline__ V2 operator+(V2 a, V2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ V2 operator-(V2 a, V2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ V2 operator*(V2 a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ double dot(V2 a, V2 b) { return a.x * b.x + a.y * b.y; }
__device__ __forceinline__ double cross(V2 a, V2 b) { return a.x * b.y - a.y * b.x; }

struct VmArgs {
  double ka, kp, a0, p0;
};

// minimum-image offset from i to j, as an exact fp64 vector
__device__ __forceinline__ V2 offset(const int32_t* __restrict__ x, const int32_t* __restrict__ y, int sh,
                                     int i, int j) {
  return {static_cast<double>(wrap_axis(x[j] - x[i], sh)), static_cast<double>(wrap_axis(y[j] - y[i], sh))};
}

// Circumcentre of (i, j, k) relative to i from r_ij, r_ik (Eqs. 15-16).
__device__ __forceinline__ V2 circumcentre(V2 rij, V2 rik) {
  const V2 rjk = rik - rij;
  const double c = cross(rij, rjk);
  const double d = 2.0 * c * c;
  const double bd = -dot(rik, rik) * dot(rij, rjk);
  const double gd = dot(rij, rij) * dot(rik, rjk);
  const V2 z = rij * bd + rik * gd;
  return z * (1.0 / d);
}

// g^T (dh/dr_i) for the circumcentre h of (i, j, k) (Eqs. 16-19).
__device__ __forceinline__ V2 pull_back(V2 rij, V2 rik, V2 g) {
  const V2 rjk = rik - rij;
  const double c = cross(rij, rjk);
  const double d = 2.0 * c * c;
  const double bd = -dot(rik, rik) * dot(rij, rjk);
  const double gd = dot(rij, rij) * dot(rik, rjk);
  const V2 z = rij * bd + rik * gd;
  const V2 dbd = rik * (2.0 * dot(rij, rjk)) + rjk * dot(rik, rik);     // Eq. 17
  const V2 dgd = rij * (-2.0 * dot(rik, rjk)) - rjk * dot(rij, rij);    // Eq. 18
  const V2 dd = V2{-rjk.y, rjk.x} * (2.0 / c);                           // Eq. 19
  const double a[2] = {rij.x, rij.y}, b[2] = {rik.x, rik.y}, zz[2] = {z.x, z.y};
  const double gb[2] = {dbd.x, dbd.y}, gg[2] = {dgd.x, dgd.y}, gdd[2] = {dd.x, dd.y};
  const double gv[2] = {g.x, g.y};
  double out[2] = {0.0, 0.0};
#pragma unroll
  for (int la = 0; la < 2; ++la)
#pragma unroll
    for (int nu = 0; nu < 2; ++nu) {
      const double delta = nu == la ? 1.0 : 0.0;
      const double inner = a[nu] * gb[la] + b[nu] * gg[la] - (bd + gd) * delta - zz[nu] * gdd[la];
      out[la] += gv[nu] * (delta + inner / d);
    }
  return {out[0], out[1]};
}

// Eqs. (6)-(8): dE_c/dh for the vertex h of cell c between its
// counter-clockwise predecessor hp and successor hn.
__device__ __forceinline__ V2 cell_vertex_grad(V2 hp, V2 h, V2 hn, double A, double P, const VmArgs& a) {
  const V2 tij = h - hp;
  const V2 tik = hn - h;
  const double lij = sqrt(dot(tij, tij)), lik = sqrt(dot(tik, tik));
  const V2 ln_ij = {tij.y, -tij.x};
  const V2 ln_ik = {tik.y, -tik.x};
  const V2 dA = (ln_ij + ln_ik) * 0.5;
  const V2 dP = tij * (1.0 / lij) - tik * (1.0 / lik);
  return dA * (2.0 * a.ka * (A - a.a0)) + dP * (2.0 * a.kp * (P - a.p0));
}

// Rows of up to this many entries are read whole when checked or searched
// (one read of each kind in flight for the row, not one chain per entry).
constexpr int kRowRead = 8;

// Row i's m entries: bad (an index outside [0, n)) or coincident (a
// particle at i's own position).  Returns whether the row was read whole,
// with its entries' positions in px, py.
__device__ __forceinline__ bool row_faults(const int32_t* __restrict__ x, const int32_t* __restrict__ y, int n,
                                           int dmax, const int32_t* row, int m, int i, bool& bad,
                                           bool& coincident, int (&px)[kRowRead], int (&py)[kRowRead]) {
  bad = coincident = false;
  const int xi = x[i], yi = y[i];
  if (m <= kRowRead && dmax >= kRowRead) {
    int rw[kRowRead];
#pragma unroll
    for (int u = 0; u < kRowRead; ++u) rw[u] = row[u];  // (rows are dmax long)
#pragma unroll
    for (int u = 0; u < kRowRead; ++u) {
      const bool in = u < m && static_cast<unsigned>(rw[u]) < static_cast<unsigned>(n);
      bad = bad || (u < m && !in);
      px[u] = in ? x[rw[u]] : xi + 1;
      py[u] = in ? y[rw[u]] : yi;
    }
#pragma unroll
    for (int u = 0; u < kRowRead; ++u) coincident = coincident || (px[u] == xi && py[u] == yi);
    return true;
  }
  for (int t = 0; t < m && !bad; ++t) bad = static_cast<unsigned>(row[t]) >= static_cast<unsigned>(n);
  for (int t = 0; t < m && !bad && !coincident; ++t) coincident = x[row[t]] == xi && y[row[t]] == yi;
  return false;
}

// Pass 1: area and perimeter of every cell (and its vertices, if asked).
__global__ __launch_bounds__(kBlock) void k_vm_cells(const int32_t* __restrict__ x,
                                                     const int32_t* __restrict__ y, int n, int log2_box,
                                                     int dmax, const int32_t* __restrict__ ring,
                                                     const int32_t* __restrict__ deg, double* __restrict__ area,
                                                     double* __restrict__ perim, double* __restrict__ vert,
                                                     WsHeader* err) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int sh = 32 - log2_box;
  const int m = deg[i];
  const int32_t* row = ring + static_cast<long long>(i) * dmax;
  if (m < 3 || m > dmax) {
    set_err(err, NM_E_INVAL);
    area[i] = perim[i] = 0.0;
    return;
  }
  bool bad, coincident;
  int px[kRowRead], py[kRowRead];
  const bool whole = row_faults(x, y, n, dmax, row, m, i, bad, coincident, px, py);
  if (bad) {
    set_err(err, NM_E_INVAL);
    area[i] = perim[i] = 0.0;
    return;
  }
  // the model gives each particle its own cell: coincident particles have none
  if (coincident) {
    set_err(err, NM_E_RANGE);
    area[i] = perim[i] = 0.0;
    return;
  }
  const int xi = x[i], yi = y[i];
  // entry t's offset, from the positions read with the row when it was read whole
  auto off_t = [&](int t) -> V2 {
    if (whole) {
      int ox = 0, oy = 0;
#pragma unroll
      for (int u = 0; u < kRowRead; ++u)
        if (u == t) {
          ox = px[u];
          oy = py[u];
        }
      return {static_cast<double>(wrap_axis(ox - xi, sh)), static_cast<double>(wrap_axis(oy - yi, sh))};
    }
    return offset(x, y, sh, i, row[t]);
  };
  const V2 r0 = off_t(0);
  V2 ra = r0;
  V2 h0 = {0.0, 0.0}, hprev = {0.0, 0.0};
  double a2 = 0.0, per = 0.0;
  for (int t = 0; t < m; ++t) {
    const V2 rb = t + 1 < m ? off_t(t + 1) : r0;
    const V2 h = circumcentre(ra, rb);
    if (vert) {
      double* v = vert + (static_cast<long long>(i) * dmax + t) * 4;
      v[0] = h.x;
      v[1] = h.y;
    }
    if (t == 0) {
      h0 = h;
    } else {
      a2 += cross(hprev, h);
      per += sqrt(dot(h - hprev, h - hprev));
    }
    hprev = h;
    ra = rb;
  }
  a2 += cross(hprev, h0);
  per += sqrt(dot(h0 - hprev, h0 - hprev));
  area[i] = 0.5 * a2;
  perim[i] = per;
}

// Pass 2: the force on every particle, and the vertex forces if asked.
__global__ __launch_bounds__(kBlock) void k_vm_forces(const int32_t* __restrict__ x,
                                                      const int32_t* __restrict__ y, int n, int log2_box,
                                                      int dmax, const int32_t* __restrict__ ring,
                                                      const int32_t* __restrict__ deg,
                                                      const double* __restrict__ area,
                                                      const double* __restrict__ perim, VmArgs va,
                                                      double* __restrict__ fx, double* __restrict__ fy,
                                                      double* __restrict__ vert, WsHeader* err) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int sh = 32 - log2_box;
  const int m = deg[i];
  const int32_t* row = ring + static_cast<long long>(i) * dmax;
  V2 F = {0.0, 0.0};
  bool ok = m >= 3 && m <= dmax;
  int px[kRowRead], py[kRowRead];
  bool whole = false;
  if (ok) {
    bool bad, coincident;
    whole = row_faults(x, y, n, dmax, row, m, i, bad, coincident, px, py);
    ok = !bad && !coincident;
  }
  if (ok) {
    const int xi = x[i], yi = y[i];
    // entry t's offset, from the positions read with the row when it was read whole
    auto off_t = [&](int t) -> V2 {
      if (whole) {
        int ox = 0, oy = 0;
#pragma unroll
        for (int u = 0; u < kRowRead; ++u)
          if (u == t) {
            ox = px[u];
            oy = py[u];
          }
        return {static_cast<double>(wrap_axis(ox - xi, sh)), static_cast<double>(wrap_axis(oy - yi, sh))};
      }
      return offset(x, y, sh, i, row[t]);
    };
    // h_{t-1}, h_t, h_{t+1} rolled along the ring
    const V2 r0 = off_t(0);
    const V2 r1 = off_t(1 % m);
    const V2 rl = off_t(m - 1);
    const V2 h0 = circumcentre(r0, r1);
    V2 hprev = circumcentre(rl, r0);
    V2 h = h0;
    V2 rj = r0, rk = r1;
    const double Ai = area[i], Pi = perim[i];
    for (int t = 0; t < m; ++t) {
      const int j = row[t], k = row[t + 1 < m ? t + 1 : 0];
      const V2 rnext = off_t(t + 2 < m ? t + 2 : t + 2 - m);
      const V2 hnext = t + 1 < m ? circumcentre(rk, rnext) : h0;
      // the vertex across the edge between cells j and k: circumcentre of
      // (j, mm, k), mm the particle just before k in j's row (i follows k)
      const int mj = deg[j];
      const int32_t* rowj = ring + static_cast<long long>(j) * dmax;
      int sk = -1, after = -1, mm = -1;
      if (mj >= 3 && mj <= kRowRead && dmax >= kRowRead) {
        // the usual short row: its first kRowRead entries read together
        // (rows are dmax long), instead of one read per step of the search
        int rj8[kRowRead];
#pragma unroll
        for (int u = 0; u < kRowRead; ++u) rj8[u] = rowj[u];
#pragma unroll
        for (int u = 0; u < kRowRead; ++u)
          if (sk < 0 && u < mj && rj8[u] == k) sk = u;
#pragma unroll
        for (int u = 0; u < kRowRead; ++u) {
          if (u == (sk + 1 < mj ? sk + 1 : 0)) after = rj8[u];
          if (u == (sk > 0 ? sk - 1 : mj - 1)) mm = rj8[u];
        }
      } else if (mj >= 3 && mj <= dmax) {
        for (int u = 0; u < mj; ++u)
          if (rowj[u] == k) {
            sk = u;
            break;
          }
        if (sk >= 0) {
          after = rowj[sk + 1 < mj ? sk + 1 : 0];
          mm = rowj[sk > 0 ? sk - 1 : mj - 1];
        }
      }
      if (sk < 0 || after != i) {
        set_err(err, NM_E_INVAL);  // the rows are not one triangulation
        ok = false;
        break;
      }
      if (static_cast<unsigned>(mm) >= static_cast<unsigned>(n)) {
        set_err(err, NM_E_INVAL);
        ok = false;
        break;
      }
      const V2 rjm = offset(x, y, sh, j, mm);
      const V2 rjk = offset(x, y, sh, j, k);
      const V2 hacross = rj + circumcentre(rjm, rjk);
      V2 g = cell_vertex_grad(hprev, h, hnext, Ai, Pi, va);
      g = g + cell_vertex_grad(hacross, h, hprev, area[j], perim[j], va);
      g = g + cell_vertex_grad(hnext, h, hacross, area[k], perim[k], va);
      if (vert) {
        double* v = vert + (static_cast<long long>(i) * dmax + t) * 4;
        v[2] = -g.x;
        v[3] = -g.y;
      }
      F = F - pull_back(rj, rk, g);
      hprev = h;
      h = hnext;
      rj = rk;
      rk = rnext;
    }
  }
  fx[i] = ok ? F.x : 0.0;
  fy[i] = ok ? F.y : 0.0;
}

// Eq. (3) over many workgroups, still in a fixed order: workgroup g sums
// the cells of its contiguous share (lanes, then a fixed tree) into part[g];
// one workgroup then sums the parts in a fixed tree.  The parts go into the
// force array before the force pass overwrites it.
constexpr int kEParts = 256;
__global__ __launch_bounds__(kBlock) void k_vm_energy_part(const double* __restrict__ area,
                                                           const double* __restrict__ perim, int n, VmArgs va,
                                                           double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int b = blockIdx.x * chunk, e = min(n, b + chunk);
  double acc = 0.0;
  for (int i = b + threadIdx.x; i < e; i += kBlock) {
    const double da = area[i] - va.a0, dp = perim[i] - va.p0;
    acc += va.ka * da * da + va.kp * dp * dp;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kEParts) void k_vm_energy_sum(const double* __restrict__ part, int np,
                                                           double* __restrict__ energy) {
  __shared__ double red[kEParts];
  red[threadIdx.x] = static_cast<int>(threadIdx.x) < np ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int h = kEParts / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *energy = red[0];
}

}  // namespace

hipError_t launch_voronoi_forces(const int32_t* x, const int32_t* y, int32_t n, int log2_box, int dmax,
                                 const int32_t* ring, const int32_t* deg, const nm_vm_params* p,
                                 double* area, double* perim, double* fx, double* fy, double* energy,
                                 double* vert, WsHeader* err, hipStream_t s) {
  const VmArgs va{p->ka, p->kp, p->a0, p->p0};
  const int nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_vm_cells, dim3(nb), dim3(kBlock), 0, s, x, y, n, log2_box, dmax, ring, deg, area,
                     perim, vert, err);
  if (energy) {
    // (one workgroup alone read the cells at one CU's bandwidth: 0.25 ms at 2^20)
    const int np = n < kEParts ? n : kEParts;
    hipLaunchKernelGGL(k_vm_energy_part, dim3(np), dim3(kBlock), 0, s, area, perim, n, va, fx);
    hipLaunchKernelGGL(k_vm_energy_sum, dim3(1), dim3(kEParts), 0, s, fx, np, energy);
  }
  hipLaunchKernelGGL(k_vm_forces, dim3(nb), dim3(kBlock), 0, s, x, y, n, log2_box, dmax, ring, deg, area,
                     perim, va, fx, fy, vert, err);
  return hipGetLastError();
}

}  // namespace nm
