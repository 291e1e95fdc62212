// align.hip -- the interaction and the integrator of one step, for any
// neighbour list (fixed k or CSR, e.g. the metric list):
//   Eq. (2): theta'_i = arg(eta xi_i + (1/m_i) sum_j n_j(t)), n = (cos, sin)
//   Eq. (1): r'_i = r_i + v0 n_i(t)   (grid units, rounded half to even)
// One lane per particle in the caller's order; the lanes of a wavefront read
// x, y, theta and the list rows contiguously and write the outputs
// contiguously.  Unit vectors are evaluated in fp64 from the fp32 headings.
#include "nm_internal.h"

namespace nm {

namespace {

struct StepArgs {
  int32_t box;
  int32_t v0;
  float eta;
  int32_t include_self;
  uint32_t variant;
  uint32_t seed_lo, seed_hi, sys_id, step_lo, step_hi;
};

__global__ __launch_bounds__(kBlock) void k_align(const int32_t* __restrict__ x,
                                                  const int32_t* __restrict__ y,
                                                  const float* __restrict__ theta, int32_t n,
                                                  const int32_t* __restrict__ nbr,
                                                  const int32_t* __restrict__ offsets, int32_t k,
                                                  long long nnz_cap, StepArgs a,
                                                  int32_t* __restrict__ x_out,
                                                  int32_t* __restrict__ y_out,
                                                  float* __restrict__ theta_out, WsHeader* err) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  long long begin, end;
  if (offsets) {
    begin = offsets[i];
    end = offsets[i + 1];
    if (begin < 0 || end < begin || end > nnz_cap) {
      set_err(err, NM_E_INVAL);
      begin = end = 0;
    }
  } else {
    begin = static_cast<long long>(i) * k;
    end = begin + k;
  }
  double sx = 0.0, sy = 0.0;
  long long m = 0;
  bool stop = false;
  // Neighbour j's unit vector, added in list order; a fixed-k row padded
  // after its last neighbour ends at the first -1.
  auto add = [&](int j, float thj) {
    if (stop) return;
    if (j == -1 && !offsets) {
      stop = true;
      return;
    }
    if (static_cast<uint32_t>(j) >= static_cast<uint32_t>(n)) {
      set_err(err, NM_E_INVAL);
      return;
    }
    double sn, cs;
    sincos(static_cast<double>(thj), &sn, &cs);
    sx += cs;
    sy += sn;
    ++m;
  };
  // Four neighbours a round: their index and heading reads are in flight
  // together instead of one chain of two dependent reads per neighbour.
  long long t = begin;
  for (; t + 4 <= end && !stop; t += 4) {
    int j4[4];
    float th4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) j4[u] = nbr[t + u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      th4[u] = static_cast<uint32_t>(j4[u]) < static_cast<uint32_t>(n) ? theta[j4[u]] : 0.0f;
#pragma unroll
    for (int u = 0; u < 4; ++u) add(j4[u], th4[u]);
  }
  for (; t < end && !stop; ++t) {
    const int j = nbr[t];
    add(j, static_cast<uint32_t>(j) < static_cast<uint32_t>(n) ? theta[j] : 0.0f);
  }
  const float th0 = theta[i];
  double own_s, own_c;
  sincos(static_cast<double>(th0), &own_s, &own_c);
  if (a.include_self) {
    sx += own_c;
    sy += own_s;
    ++m;
  }
  double ax = 0.0, ay = 0.0;
  if (m > 0) {
    ax = sx / static_cast<double>(m);
    ay = sy / static_cast<double>(m);
  }
  const uint4 blk = Philox::block(make_uint4(static_cast<uint32_t>(i >> 2), a.step_lo, a.step_hi,
                                             a.sys_id), a.seed_lo, a.seed_hi);
  const double phi = noise_angle(uint4_word(blk, i & 3));
  double sp, cp;
  sincos(phi, &sp, &cp);
  const float thn = heading_update(ax, ay, cp, sp, phi, a.eta, &th0, a.variant);
  theta_out[i] = thn;

  const int xi = x[i], yi = y[i];
  if (static_cast<uint32_t>(xi) >= static_cast<uint32_t>(a.box) ||
      static_cast<uint32_t>(yi) >= static_cast<uint32_t>(a.box))
    set_err(err, NM_E_RANGE);
  int ddx, ddy;
  move_step(a.v0, own_c, own_s, thn, a.variant, ddx, ddy);
  const int mask = a.box - 1;
  x_out[i] = (xi + ddx) & mask;
  y_out[i] = (yi + ddy) & mask;
}

// Polar order parameter: sums of cos and sin of the headings, fp64.  Each
// workgroup reduces a strided share in registers and LDS, then adds its two
// sums to the output with one atomic each (vector memory atomics); a last
// one-lane kernel forms |(sum cos, sum sin)| / n.
__global__ __launch_bounds__(64) void k_order_zero(double* sums) {
  if (threadIdx.x < 2) sums[threadIdx.x] = 0.0;
}

__global__ void k_order_norm(double* sums, int32_t n) {
  sums[2] = sqrt(sums[0] * sums[0] + sums[1] * sums[1]) / static_cast<double>(n);
}

__global__ __launch_bounds__(kBlock) void k_polar_order(const float* __restrict__ theta, int32_t n,
                                                        double* __restrict__ sums) {
  __shared__ double s_c[kBlock / 64], s_s[kBlock / 64];
  double c = 0.0, s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double sn, cs;
    sincos(static_cast<double>(theta[i]), &sn, &cs);
    c += cs;
    s += sn;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, 64);
    s += __shfl_xor(s, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_c[wave] = c;
    s_s[wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tc = 0.0, ts = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      tc += s_c[q];
      ts += s_s[q];
    }
    atomicAdd(&sums[0], tc);
    atomicAdd(&sums[1], ts);
  }
}

}  // namespace

hipError_t launch_polar_order(const float* theta, int32_t n, double* sums, hipStream_t s) {
  hipLaunchKernelGGL(k_order_zero, dim3(1), dim3(64), 0, s, sums);
  // one workgroup per CU at most: the two same-address atomics per workgroup
  // are serialised where the memory is (N = 2^20: 31 us per call on 1024
  // workgroups, 20 on 512, 16 on 256, 18 on 128)
  const int grid = max(1, min(256, (n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_polar_order, dim3(grid), dim3(kBlock), 0, s, theta, n, sums);
  hipLaunchKernelGGL(k_order_norm, dim3(1), dim3(1), 0, s, sums, n);
  return hipGetLastError();
}

hipError_t launch_align(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                        const int32_t* nbr, const int32_t* offsets, int32_t k, long long nnz_cap,
                        const nm_params* p, uint64_t step, int32_t* x_out, int32_t* y_out,
                        float* theta_out, WsHeader* err_hdr, hipStream_t s) {
  StepArgs a{p->box,
             p->v0,
             p->eta,
             p->include_self,
             p->variant,
             static_cast<uint32_t>(p->seed),
             static_cast<uint32_t>(p->seed >> 32),
             p->sys_id,
             static_cast<uint32_t>(step),
             static_cast<uint32_t>(step >> 32)};
  const int nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_align, dim3(nb), dim3(kBlock), 0, s, x, y, theta, n, nbr, offsets, k,
                     nnz_cap, a, x_out, y_out, theta_out, err_hdr);
  return hipGetLastError();
}

}  // namespace nm
