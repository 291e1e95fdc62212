// abi.hip -- the extern "C" entry points declared in include/nm.h: argument
// validation on the host, workspace layout, and kernel launches on the
// caller's stream.  Nothing here allocates device memory.
#include <math.h>
#include <string.h>

#include "nm_internal.h"

namespace nm {

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kMaxCells = int64_t(1) << 28;

int64_t round_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int status_of(hipError_t e) { return e == hipSuccess ? NM_OK : NM_E_DEVICE; }

bool params_ok(const nm_params* p) {
  if (p == nullptr || (p->variant & ~kVariantMask) != 0) return false;
  if (!is_pow2(p->box) || p->box < 2 || p->box > (1 << 20)) return false;
  if (2ll * (p->v0 < 0 ? -static_cast<int64_t>(p->v0) : p->v0) >= p->box) return false;
  if (!(p->eta >= 0.0f) || !isfinite(p->eta)) return false;
  return p->include_self == 0 || p->include_self == 1;
}

}  // namespace

bool make_layout(const nm_grid* g, Layout* out) {
  if (g == nullptr) return false;
  const int side = g->block < 0 ? g->block : (g->block & ~NM_BLOCK_SUBSTRIPS);
  if (side < -1 || side > kMaxB || (side > 0 && side < 3)) return false;
  if (g->n < 2 || g->n > kMaxParticles) return false;
  if (!is_pow2(g->box) || g->box < 2 || g->box > (1 << 20)) return false;
  if (!is_pow2(g->cell_w) || g->cell_w > g->box) return false;
  Layout L{};
  L.log2_box = ilog2(g->box);
  L.log2_w = ilog2(g->cell_w);
  L.G = g->box >> L.log2_w;
  L.C = static_cast<int64_t>(L.G) * L.G;
  if (L.C > kMaxCells) return false;
  L.nb_scan_c = static_cast<int32_t>((L.C + kScanTile - 1) / kScanTile);
  L.nb_scan_m = static_cast<int32_t>((static_cast<int64_t>(g->n) + kScanTile - 1) / kScanTile);
  int64_t off = round_up(sizeof(WsHeader));
  L.off_scan_c = off;
  off += round_up(256 + 8 * static_cast<int64_t>(L.nb_scan_c));
  L.off_scan_m = off;
  off += round_up(256 + 8 * static_cast<int64_t>(L.nb_scan_m));
  L.off_count = off;
  off += round_up(4 * L.C);
  L.off_start = off;
  off += round_up(4 * (L.C + 1));
  L.off_rank = off;
  off += round_up(4 * static_cast<int64_t>(g->n));
  L.off_sorted = off;
  off += round_up(16 * static_cast<int64_t>(g->n));
  L.off_cs = off;
  off += round_up(32 * static_cast<int64_t>(g->n));
  L.off_dflag = off;
  off += round_up(static_cast<int64_t>(g->n));
  L.chunk_cap = g->n / 32 + 1024;
  L.off_chunks = off;
  off += round_up(16 * static_cast<int64_t>(L.chunk_cap));
  L.off_vlist = off;
  off += round_up(4 * static_cast<int64_t>(g->n));
  // Two-level binning when a coarse bin of at most kFineCells cells suffices:
  // at most kCoarseBins bins, each of about kBinTarget particles at the mean
  // density where the cells allow.  The space is there from kCoarseMinBatch
  // particles (the batched stages use it); a single system bins in two
  // levels from kCoarseMinN.
  L.sb = 0;
  while ((L.C >> L.sb) > kCoarseBins) ++L.sb;
  while ((int64_t(1) << L.sb) < kFineCells &&
         (static_cast<int64_t>(g->n) << L.sb) < static_cast<int64_t>(kBinTarget) * L.C)
    ++L.sb;
  if ((int64_t(1) << L.sb) <= kFineCells && g->n >= kCoarseMinBatch) {
    L.nbins = static_cast<int32_t>((L.C + (int64_t(1) << L.sb) - 1) >> L.sb);
    L.nblk = (g->n + kCoarseP - 1) / kCoarseP;
    const int64_t hsize = static_cast<int64_t>(L.nbins) * L.nblk + 1;
    L.nb_scan_h = static_cast<int32_t>((hsize + kScanTile - 1) / kScanTile);
    L.off_coarse = off;
    off += round_up(16 * static_cast<int64_t>(g->n));
    L.off_hist = off;
    off += round_up(4 * hsize);
    L.off_scan_h = off;
    off += round_up(256 + 8 * static_cast<int64_t>(L.nb_scan_h));
  }
  L.total = off;
  *out = L;
  return true;
}

DevWs dev_ws(const nm_grid* g, const Layout& lay, void* ws) {
  char* b = static_cast<char*>(ws);
  DevWs w{};
  w.hdr = reinterpret_cast<WsHeader*>(b);
  w.scan_c = reinterpret_cast<ScanState*>(b + lay.off_scan_c);
  w.scan_m = reinterpret_cast<ScanState*>(b + lay.off_scan_m);
  w.count = reinterpret_cast<int32_t*>(b + lay.off_count);
  w.start = reinterpret_cast<int32_t*>(b + lay.off_start);
  w.rank = reinterpret_cast<int32_t*>(b + lay.off_rank);
  w.sorted = reinterpret_cast<int4*>(b + lay.off_sorted);
  w.cs = reinterpret_cast<double2*>(b + lay.off_cs);
  w.dflag = reinterpret_cast<uint8_t*>(b + lay.off_dflag);
  w.chunks = reinterpret_cast<int4*>(b + lay.off_chunks);
  w.vlist = reinterpret_cast<int32_t*>(b + lay.off_vlist);
  w.chunk_cap = lay.chunk_cap;
  w.sb = lay.sb;
  w.nbins = lay.nbins;
  w.nblk = lay.nblk;
  w.nb_scan_h = lay.nb_scan_h;
  if (lay.nbins > 0) {
    w.coarse = reinterpret_cast<int4*>(b + lay.off_coarse);
    w.hist = reinterpret_cast<int32_t*>(b + lay.off_hist);
    w.scan_h = reinterpret_cast<ScanState*>(b + lay.off_scan_h);
  }
  w.n = g->n;
  w.box = g->box;
  w.cell_w = g->cell_w;
  w.log2_box = lay.log2_box;
  w.log2_w = lay.log2_w;
  w.G = lay.G;
  w.nb_scan_c = lay.nb_scan_c;
  w.nb_scan_m = lay.nb_scan_m;
  w.C = lay.C;
  return w;
}

}  // namespace nm

using namespace nm;

namespace {

bool ws_ok(const nm_grid* g, const void* ws, size_t ws_bytes, Layout* lay) {
  if (!make_layout(g, lay) || ws == nullptr) return false;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return false;
  return static_cast<int64_t>(ws_bytes) >= lay->total;
}

}  // namespace

extern "C" {

const char* nm_status_str(int status) {
  switch (status) {
    case NM_OK: return "ok";
    case NM_E_INVAL: return "invalid argument";
    case NM_E_RANGE: return "coordinate outside [0, L)";
    case NM_E_CAPACITY: return "metric list exceeds capacity";
    case NM_E_NOMEM: return "job can never fit the memory budget";
    case NM_E_DEVICE: return "HIP device or launch failure";
    default: return "unknown status";
  }
}

int64_t nm_workspace_bytes(const nm_grid* g) {
  Layout lay;
  if (!make_layout(g, &lay)) return NM_E_INVAL;
  return lay.total;
}

int32_t nm_suggest_cell_w(int32_t n, int32_t box, double per_cell) {
  if (n < 1 || !is_pow2(box) || !(per_cell > 0.0)) return 1;
  const double w = static_cast<double>(box) * sqrt(per_cell / static_cast<double>(n));
  int e = static_cast<int>(lround(log2(w > 1.0 ? w : 1.0)));
  const int lb = ilog2(box);
  if (e > lb) e = lb;
  if (e < 0) e = 0;
  while (2 * (lb - e) > 28) ++e;  // keep the cell table within its limit
  return static_cast<int32_t>(1) << e;
}

int nm_workspace_init(const nm_grid* g, void* ws, size_t ws_bytes, void* stream) {
  Layout lay;
  if (!ws_ok(g, ws, ws_bytes, &lay)) return NM_E_INVAL;
  return status_of(launch_ws_init(dev_ws(g, lay, ws), as_stream(stream)));
}

int nm_build_cells(const nm_grid* g, const int32_t* x, const int32_t* y, void* ws,
                   size_t ws_bytes, void* stream) {
  Layout lay;
  if (!ws_ok(g, ws, ws_bytes, &lay) || x == nullptr || y == nullptr) return NM_E_INVAL;
  return status_of(launch_build(dev_ws(g, lay, ws), x, y, nullptr, nullptr, 0, as_stream(stream)));
}

int nm_knn(const nm_grid* g, const void* ws, int32_t k, int32_t* nbr, int64_t* d2, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || nbr == nullptr) return NM_E_INVAL;
  if (k < 1 || k > NM_MAX_K || k > g->n - 1) return NM_E_INVAL;
  return status_of(launch_knn(dev_ws(g, lay, const_cast<void*>(ws)), k, g->block, nbr,
                              reinterpret_cast<long long*>(d2), as_stream(stream)));
}

int nm_knn_layout(const nm_grid* g, int32_t k, int32_t* out) {
  Layout lay;
  if (!make_layout(g, &lay) || out == nullptr) return NM_E_INVAL;
  if (k < 1 || k > NM_MAX_K || k > g->n - 1) return NM_E_INVAL;
  DevWs w{};  // geometry only: the layout reads no device memory
  w.n = g->n;
  w.box = g->box;
  w.cell_w = g->cell_w;
  w.log2_box = lay.log2_box;
  w.log2_w = lay.log2_w;
  w.G = lay.G;
  w.C = lay.C;
  knn_layout(w, k, g->block, out);
  return NM_OK;
}

int nm_knn_fov(const nm_grid* g, const void* ws, int32_t k, const float* theta, int32_t cos_q,
               int32_t* nbr, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || nbr == nullptr || theta == nullptr) return NM_E_INVAL;
  if (k < 1 || k > NM_MAX_K || k > g->n - 1 || cos_q < -4096 || cos_q > 4096) return NM_E_INVAL;
  return status_of(launch_knn_fov(dev_ws(g, lay, const_cast<void*>(ws)), g->block, theta, k, cos_q,
                                  nbr, as_stream(stream)));
}

int nm_metric_list(const nm_grid* g, void* ws, int64_t rc2, int32_t* offsets, int32_t* idx,
                   int64_t cap, int64_t* nnz_host, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || offsets == nullptr) return NM_E_INVAL;
  if (rc2 < 0 || rc2 >= (int64_t(1) << 40) || cap < 0) return NM_E_INVAL;
  const DevWs w = dev_ws(g, lay, ws);
  hipStream_t s = as_stream(stream);
  hipError_t e = launch_metric_count(w, rc2, offsets, s);
  if (e != hipSuccess) return NM_E_DEVICE;
  if (nnz_host != nullptr) {
    int32_t nnz = 0, err = 0;
    if (hipMemcpyAsync(&nnz, offsets + g->n, sizeof(nnz), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&err, &w.hdr->err, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return NM_E_DEVICE;
    if (err == NM_E_CAPACITY) return NM_E_CAPACITY;
    *nnz_host = nnz;
    if (idx != nullptr && nnz > cap) return NM_E_CAPACITY;
  }
  if (idx == nullptr) return NM_OK;
  return status_of(launch_metric_fill(w, rc2, offsets, idx, cap, s));
}

int nm_voronoi(const nm_grid* g, void* ws, int32_t dmax, int32_t* ring, int32_t* deg, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || ring == nullptr || deg == nullptr) return NM_E_INVAL;
  if (g->n < 3 || g->box < 8 || dmax < 3 || dmax > NM_VORONOI_MAX_DEG) return NM_E_INVAL;
  return status_of(launch_voronoi(dev_ws(g, lay, ws), dmax, ring, deg, as_stream(stream)));
}

int nm_voronoi_check(const nm_grid* g, void* ws, const int32_t* x, const int32_t* y, int32_t dmax,
                     const int32_t* ring, const int32_t* deg, uint8_t* stale, int32_t* nfail,
                     void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || x == nullptr || y == nullptr || ring == nullptr ||
      deg == nullptr || stale == nullptr)
    return NM_E_INVAL;
  if (g->n < 3 || g->box < 8 || dmax < 3 || dmax > NM_VORONOI_MAX_DEG) return NM_E_INVAL;
  return status_of(launch_voronoi_check(dev_ws(g, lay, ws), x, y, dmax, ring, deg, stale, nfail,
                                        as_stream(stream)));
}

int nm_voronoi_update(const nm_grid* g, void* ws, const int32_t* x, const int32_t* y, int32_t dmax,
                      int32_t* ring, int32_t* deg, uint8_t* stale, int32_t* nfail, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || x == nullptr || y == nullptr || ring == nullptr ||
      deg == nullptr || stale == nullptr)
    return NM_E_INVAL;
  if (g->n < 3 || g->box < 8 || dmax < 3 || dmax > NM_VORONOI_MAX_DEG) return NM_E_INVAL;
  return status_of(launch_voronoi_update(dev_ws(g, lay, ws), x, y, dmax, ring, deg, stale, nfail, 2,
                                         as_stream(stream)));
}

int nm_voronoi_forces(const int32_t* x, const int32_t* y, int32_t n, int32_t box, int32_t dmax,
                      const int32_t* ring, const int32_t* deg, const nm_vm_params* vp, double* area,
                      double* perim, double* fx, double* fy, double* energy, double* vertex,
                      void* ws_err, void* stream) {
  if (x == nullptr || y == nullptr || ring == nullptr || deg == nullptr || vp == nullptr ||
      area == nullptr || perim == nullptr || fx == nullptr || fy == nullptr)
    return NM_E_INVAL;
  if (n < 3 || n > kMaxParticles || !is_pow2(box) || box < 8 || box > (1 << 20)) return NM_E_INVAL;
  if (dmax < 3 || dmax > NM_VORONOI_MAX_DEG) return NM_E_INVAL;
  if (!isfinite(vp->ka) || !isfinite(vp->kp) || !isfinite(vp->a0) || !isfinite(vp->p0)) return NM_E_INVAL;
  return status_of(launch_voronoi_forces(x, y, n, ilog2(box), dmax, ring, deg, vp, area, perim, fx, fy,
                                         energy, vertex, static_cast<WsHeader*>(ws_err),
                                         as_stream(stream)));
}

int nm_polar_order(const float* theta, int32_t n, double* sums, void* stream) {
  if (theta == nullptr || sums == nullptr || n < 1) return NM_E_INVAL;
  return status_of(launch_polar_order(theta, n, sums, as_stream(stream)));
}

int nm_align_step(const int32_t* x, const int32_t* y, const float* theta, int32_t n,
                  const int32_t* nbr, const int32_t* offsets, int32_t k, int64_t nnz_cap,
                  const nm_params* p, uint64_t step, int32_t* x_out, int32_t* y_out,
                  float* theta_out, void* ws_err, void* stream) {
  if (!params_ok(p) || n < 1 || n > kMaxParticles) return NM_E_INVAL;
  if (x == nullptr || y == nullptr || theta == nullptr || x_out == nullptr || y_out == nullptr ||
      theta_out == nullptr)
    return NM_E_INVAL;
  if (offsets == nullptr && (k < 0 || (k > 0 && nbr == nullptr))) return NM_E_INVAL;
  if (offsets != nullptr && (nnz_cap < 0 || (nnz_cap > 0 && nbr == nullptr))) return NM_E_INVAL;
  const void* ins[3] = {x, y, theta};
  const void* outs[3] = {x_out, y_out, theta_out};
  for (const void* a : ins)
    for (const void* b : outs)
      if (a == b) return NM_E_INVAL;
  return status_of(launch_align(x, y, theta, n, nbr, offsets, k, nnz_cap, p, step, x_out, y_out,
                                theta_out, static_cast<WsHeader*>(ws_err), as_stream(stream)));
}

int nm_bin_step(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta,
                const nm_params* p, uint64_t step, void* ws, size_t ws_bytes, void* stream) {
  Layout lay;
  if (!ws_ok(g, ws, ws_bytes, &lay) || !params_ok(p) || p->box != g->box) return NM_E_INVAL;
  if (x == nullptr || y == nullptr || theta == nullptr) return NM_E_INVAL;
  return status_of(launch_build(dev_ws(g, lay, ws), x, y, theta, p, step, as_stream(stream)));
}

int nm_knn_align(const nm_grid* g, const void* ws, int32_t k, const nm_params* p,
                 const float* theta, int32_t* nbr, int32_t* x_out, int32_t* y_out,
                 float* theta_out, void* stream) {
  Layout lay;
  if (!make_layout(g, &lay) || ws == nullptr || !params_ok(p) || p->box != g->box)
    return NM_E_INVAL;
  if (theta == nullptr || nbr == nullptr || x_out == nullptr || y_out == nullptr ||
      theta_out == nullptr)
    return NM_E_INVAL;
  if (k < 1 || k > NM_MAX_K || k > g->n - 1) return NM_E_INVAL;
  const void* outs[3] = {x_out, y_out, theta_out};
  for (const void* b : outs)
    if (b == theta) return NM_E_INVAL;
  return status_of(launch_knn_align(dev_ws(g, lay, const_cast<void*>(ws)), k, g->block, p, theta,
                                    nbr, x_out, y_out, theta_out, as_stream(stream)));
}

int nm_step(const nm_grid* g, const int32_t* x, const int32_t* y, const float* theta, int32_t k,
            const nm_params* p, uint64_t step, void* ws, size_t ws_bytes, int32_t* nbr,
            int32_t* x_out, int32_t* y_out, float* theta_out, void* stream) {
  Layout lay;
  if (!ws_ok(g, ws, ws_bytes, &lay) || !params_ok(p) || p->box != g->box) return NM_E_INVAL;
  if (x == nullptr || y == nullptr || theta == nullptr || nbr == nullptr || x_out == nullptr ||
      y_out == nullptr || theta_out == nullptr)
    return NM_E_INVAL;
  if (k < 1 || k > NM_MAX_K || k > g->n - 1) return NM_E_INVAL;
  const void* ins[3] = {x, y, theta};
  const void* outs[3] = {x_out, y_out, theta_out};
  for (const void* a : ins)
    for (const void* b : outs)
      if (a == b) return NM_E_INVAL;
  const int rc = nm_bin_step(g, x, y, theta, p, step, ws, ws_bytes, stream);
  if (rc != NM_OK) return rc;
  return nm_knn_align(g, ws, k, p, theta, nbr, x_out, y_out, theta_out, stream);
}

int nm_tune_grid(const nm_grid* cand, int32_t ncand, const int32_t* x, const int32_t* y,
                 const float* theta, int32_t k, const nm_params* p, uint64_t step, void* ws,
                 size_t ws_bytes, int32_t* nbr, int32_t* x_out, int32_t* y_out, float* theta_out,
                 int32_t reps, int32_t* best, float* ms_out, void* stream) {
  if (cand == nullptr || ncand < 1 || reps < 1 || best == nullptr) return NM_E_INVAL;
  for (int c = 0; c < ncand; ++c) {
    Layout lay;
    if (!ws_ok(&cand[c], ws, ws_bytes, &lay) || cand[c].n != cand[0].n || cand[c].box != cand[0].box)
      return NM_E_INVAL;
  }
  hipStream_t s = as_stream(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return NM_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return NM_E_DEVICE;
  }
  int rc = NM_OK, arg = -1;
  float best_ms = 0.0f;
  for (int c = 0; c < ncand && rc == NM_OK; ++c) {
    rc = nm_workspace_init(&cand[c], ws, ws_bytes, stream);
    if (rc == NM_OK)
      rc = nm_step(&cand[c], x, y, theta, k, p, step, ws, ws_bytes, nbr, x_out, y_out, theta_out, stream);
    if (rc == NM_OK && hipEventRecord(e0, s) != hipSuccess) rc = NM_E_DEVICE;
    for (int t = 0; t < reps && rc == NM_OK; ++t)
      rc = nm_step(&cand[c], x, y, theta, k, p, step, ws, ws_bytes, nbr, x_out, y_out, theta_out, stream);
    float ms = 0.0f;
    if (rc == NM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = NM_E_DEVICE;
    if (rc == NM_OK) rc = nm_check(ws, stream);
    ms /= static_cast<float>(reps);
    if (ms_out) ms_out[c] = ms;
    if (rc == NM_OK && (arg < 0 || ms < best_ms)) {
      best_ms = ms;
      arg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NM_OK) return rc;
  *best = arg;
  return nm_workspace_init(&cand[arg], ws, ws_bytes, stream);
}

int nm_check(void* ws, void* stream) {
  if (ws == nullptr) return NM_E_INVAL;
  hipStream_t s = as_stream(stream);
  int32_t err = 0;
  const int32_t zero = 0;
  WsHeader* h = static_cast<WsHeader*>(ws);
  if (hipStreamSynchronize(s) != hipSuccess) return NM_E_DEVICE;
  if (hipMemcpy(&err, &h->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return NM_E_DEVICE;
  if (err != 0 && hipMemcpy(&h->err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
    return NM_E_DEVICE;
  return err;
}

}  // extern "C"
