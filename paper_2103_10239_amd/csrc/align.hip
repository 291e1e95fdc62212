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
  for (long long t = begin; t < end; ++t) {
    const int j = nbr[t];
    if (static_cast<uint32_t>(j) >= static_cast<uint32_t>(n)) {
      set_err(err, NM_E_INVAL);
      continue;
    }
    double sn, cs;
    sincos(static_cast<double>(theta[j]), &sn, &cs);
    sx += cs;
    sy += sn;
    ++m;
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
  double sp, cp;
  sincos(noise_angle(uint4_word(blk, i & 3)), &sp, &cp);
  const double e = static_cast<double>(a.eta);
  const double vx = ax + e * cp;
  const double vy = ay + e * sp;
  theta_out[i] = vec_angle(vx, vy, th0);

  const int xi = x[i], yi = y[i];
  if (static_cast<uint32_t>(xi) >= static_cast<uint32_t>(a.box) ||
      static_cast<uint32_t>(yi) >= static_cast<uint32_t>(a.box))
    set_err(err, NM_E_RANGE);
  const int ddx = static_cast<int>(rint(static_cast<double>(a.v0) * own_c));
  const int ddy = static_cast<int>(rint(static_cast<double>(a.v0) * own_s));
  const int mask = a.box - 1;
  x_out[i] = (xi + ddx) & mask;
  y_out[i] = (yi + ddy) & mask;
}

}  // namespace

hipError_t launch_align(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                        const int32_t* nbr, const int32_t* offsets, int32_t k, long long nnz_cap,
                        const nm_params* p, uint64_t step, int32_t* x_out, int32_t* y_out,
                        float* theta_out, WsHeader* err_hdr, hipStream_t s) {
  StepArgs a{p->box,
             p->v0,
             p->eta,
             p->include_self,
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
