// fov.hip -- field-of-view topological lists: for every particle, the k
// nearest (by (d^2, index)) among the particles inside a cone around its
// heading (the topological rule of Sec. III restricted to what the particle
// faces).  The cone test and the exact per-query search are in fov.h.
//
// Two kernels: the strip kernel of the k-NN lists with the cone test as a
// candidate filter (knn.hip), and, for grids with block = -1, one lane per
// query in cell order running the exact ring search of fov.h.
#include "fov.h"

namespace nm {

namespace {

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
  fov_exact<KMAX>(w, s, q, fov_heading(theta[q.z], c), k, total, nbr);
}

template <int KMAX>
hipError_t launch_fov_t(const DevWs& w, const float* theta, int k, int c, int32_t* nbr, hipStream_t s) {
  const int nb = (w.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_knn_fov<KMAX>, dim3(nb), dim3(kBlock), 0, s, w, theta, k, c, nbr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_knn_fov(const DevWs& w, int block, const float* theta, int k, int c, int32_t* nbr,
                          hipStream_t s) {
  if (block >= 0) return launch_knn_fov_strips(w, block, theta, k, c, nbr, s);
  if (k <= 4) return launch_fov_t<4>(w, theta, k, c, nbr, s);
  if (k <= 8) return launch_fov_t<8>(w, theta, k, c, nbr, s);
  if (k <= 12) return launch_fov_t<12>(w, theta, k, c, nbr, s);
  if (k <= 16) return launch_fov_t<16>(w, theta, k, c, nbr, s);
  if (k <= 24) return launch_fov_t<24>(w, theta, k, c, nbr, s);
  return launch_fov_t<32>(w, theta, k, c, nbr, s);
}

}  // namespace nm
