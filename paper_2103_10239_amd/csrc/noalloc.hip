// noalloc.hip -- nm_step_noalloc: the one-system step of nm_step (Alg. 1:
// cell binning, k-NN lists fused with Eq. (2) and Eq. (1)) for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  Its workspace is a file-scope device array instead of a caller
// buffer; every call on a device shares that device's array.
#include <mutex>

#include "nm_internal.h"

namespace nm {

// The workspace of nm_step_noalloc: at most kScratchBytes (nm_workspace_bytes
// of the grid), 256-byte aligned as every workspace.  Each device holds its
// own copy for the life of the process.  In host code `scratch` names a host
// stand-in: only the address from hipGetSymbolAddress reaches the kernels.
constexpr size_t kScratchBytes = size_t(32) << 20;
static_assert(static_cast<long long>(kScratchBytes) == NM_STEP_NOALLOC_MAX_BYTES, "documented limit");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

// The device address of this device's `scratch` (looked up once per device,
// with that device current).  nullptr on failure.
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

__global__ void k_report_err(const WsHeader* h, int32_t* out) { *out = h->err; }

}  // namespace
}  // namespace nm

using namespace nm;

extern "C" {

int nm_step_noalloc(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta, int32_t k,
                    const nm_params* p, uint64_t step, int32_t* nbr, int32_t* x_out, int32_t* y_out,
                    float* theta_out, int32_t* err, void* stream) {
  const int64_t need = nm_workspace_bytes(g);
  if (need < 0) return NM_E_INVAL;
  if (need > static_cast<int64_t>(kScratchBytes)) return NM_E_NOMEM;
  void* ws = scratch_on_current_device();
  if (ws == nullptr) return NM_E_DEVICE;
  // The array keeps the last call's contents (another grid's cells, its
  // error word and counters): prepare it for this grid first (a kernel, not
  // a memset, so that the call can be captured in a graph).
  int rc = nm_workspace_init(g, ws, kScratchBytes, stream);
  if (rc != NM_OK) return rc;
  rc = nm_step(g, x, y, theta, k, p, step, ws, kScratchBytes, nbr, x_out, y_out, theta_out, stream);
  if (rc != NM_OK || err == nullptr) return rc;
  hipLaunchKernelGGL(k_report_err, dim3(1), dim3(1), 0, reinterpret_cast<hipStream_t>(stream),
                     static_cast<const WsHeader*>(ws), err);
  return hipGetLastError() == hipSuccess ? NM_OK : NM_E_DEVICE;
}

}  // extern "C"
