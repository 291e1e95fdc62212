// batch.hip -- the batched form: many independent systems of uneven size
// advanced together, one launch per stage of the step (Alg. 1:
// cell binning, k-NN lists, Eq. (2) alignment and Eq. (1) move), with the
// whole step captured once into a HIP graph and replayed.
//
// Device memory (caller-owned, one buffer):
//   header    256 B: batch error word
//   sys       BatchSys[nsys]: per-system workspace view, tile geometry, state
//             pointers, Philox identity, step counter and buffer parity
//   items     int32[total items]: stage work item -> system
//   ws_s      per-system workspaces, each sized for the finest cell width the
//             tuner may choose, so a re-tune never moves memory
//
// Per-system results are those of the plain calls with the same parameters:
// the kernels are the same bodies, and the Philox counter of system s is
// (i / 4, step, sys_id_s) with the system's own step count.
#include <math.h>

#include <algorithm>
#include <map>
#include <vector>

#include "batch_host.h"

namespace nm {

namespace {

__global__ __launch_bounds__(kBlock) void k_bb_advance(BatchSys* sys, int nsys) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nsys) return;
  BatchSys& d = sys[s];
  d.parity ^= 1;
  const uint32_t lo = d.step_lo + 1u;
  d.step_lo = lo;
  if (lo == 0u) d.step_hi += 1u;
}

// First error recorded by any system (then cleared there) into the batch word.
__global__ __launch_bounds__(kBlock) void k_bb_errors(BatchSys* sys, int nsys, int32_t* err) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nsys) return;
  WsHeader* h = sys[s].w.hdr;
  const int e = h->err;
  if (e != 0) {
    atomicCAS(err, 0, e);
    h->err = 0;
  }
}

}  // namespace

hipError_t launch_batch_advance(const BatchRef& b, hipStream_t s) {
  hipLaunchKernelGGL(k_bb_advance, dim3((b.nsys + kBlock - 1) / kBlock), dim3(kBlock), 0, s, b.sys,
                     b.nsys);
  return hipGetLastError();
}

BatchSys make_batch_sys(const SysSpec& s, int k) {
  BatchSys d{};
  Layout lay;
  make_layout(&s.g, &lay);
  d.w = dev_ws(&s.g, lay, s.ws);
  d.f = fast_cfg(d.w, k, s.g.block);
  d.tc = tile_cfg(d.w, d.f, k);
  for (int t = 0; t < 2; ++t) {
    d.x[t] = s.x[t];
    d.y[t] = s.y[t];
    d.th[t] = s.th[t];
  }
  d.nbr = s.nbr;
  d.v0 = s.v0;
  d.eta = s.eta;
  d.include_self = s.include_self;
  d.variant = s.variant;
  d.sys_id = s.sys_id;
  d.seed_lo = static_cast<uint32_t>(s.seed);
  d.seed_hi = static_cast<uint32_t>(s.seed >> 32);
  d.step_lo = static_cast<uint32_t>(s.step);
  d.step_hi = static_cast<uint32_t>(s.step >> 32);
  d.parity = s.parity;
  d.ntiles = d.tc.ntx * d.tc.nty;
  const int64_t big = std::max<int64_t>(lay.C, s.g.n);
  d.nitems[kStInit] = static_cast<int32_t>(
      std::max<int64_t>(1, std::min<int64_t>(64, (big + 4 * kBlock - 1) / (4 * kBlock))));
  if (lay.nbins > 0) {  // two levels: coarse count, table scan, coarse scatter, per-bin sort
    d.nitems[kStCount] = lay.nblk;
    d.nitems[kStScan] = lay.nb_scan_h;
    d.nitems[kStScatter] = lay.nblk;
    d.nitems[kStFine] = lay.nbins;
  } else {
    d.nitems[kStCount] = (s.g.n + kBlock - 1) / kBlock;
    d.nitems[kStScan] = lay.nb_scan_c;
    d.nitems[kStScatter] = (s.g.n + 4 * kBlock - 1) / (4 * kBlock);
    d.nitems[kStFine] = 0;
  }
  d.nitems[kStKnn] = d.f.split ? 0 : d.ntiles;
  d.nitems[kStKnnSplit] = d.f.split ? d.ntiles : 0;
  return d;
}

void batch_items(std::vector<BatchSys>& sys, std::vector<int32_t>& items, int32_t begin[kStages + 1]) {
  items.clear();
  for (int st = 0; st < kStages; ++st) {
    begin[st] = static_cast<int32_t>(items.size());
    for (size_t q = 0; q < sys.size(); ++q) {
      sys[q].base[st] = static_cast<int32_t>(items.size()) - begin[st];
      items.insert(items.end(), sys[q].nitems[st], static_cast<int32_t>(q));
    }
  }
  begin[kStages] = static_cast<int32_t>(items.size());
}

hipError_t enqueue_batch_step(const BatchRef& r, int k, bool advance, hipStream_t s) {
  hipError_t e = launch_batch_bin(r, kStCount, s);
  if (e == hipSuccess) e = launch_batch_bin(r, kStScan, s);
  if (e == hipSuccess) e = launch_batch_bin(r, kStScatter, s);
  if (e == hipSuccess) e = launch_batch_bin(r, kStFine, s);
  if (e == hipSuccess) e = launch_batch_knn(r, k, s);
  if (e == hipSuccess && advance) e = launch_batch_advance(r, s);
  return e;
}

}  // namespace nm

using namespace nm;

// Host object behind the opaque nm_batch handle.
struct nm_batch {
  int32_t nsys = 0, box = 0, k = 0;
  nm_params p{};
  std::vector<int32_t> n, off;  // sizes and offsets into the concatenated arrays
  std::vector<uint32_t> sys_id;
  std::vector<int32_t> wlog;    // chosen log2 cell width per system
  std::vector<int32_t> block;   // chosen fast-path block side per system
  std::vector<int64_t> ws_off;  // per-system workspace offset inside the batch buffer
  std::vector<int64_t> ws_len;
  int64_t off_sys = 0, off_items = 0, items_cap = 0, total_bytes = 0;
  // bound state
  char* ws = nullptr;
  nm_batch_io io{};
  uint64_t step0 = 0;
  int64_t steps_done = 0;
  BatchRef ref{};
  std::vector<BatchSys> host_sys;
  std::vector<int32_t> host_items;
  hipGraphExec_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

constexpr int64_t kA = 256;
int64_t rup(int64_t v) { return (v + kA - 1) / kA * kA; }

int ilog2i(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

// Candidate cell occupancies of the tuner, finest first.
const double kPerCell[] = {0.5, 1.0, 2.0, 4.0};
constexpr int kNumPerCell = 4;
// Candidate k-NN block choices, weighed at the chosen cell width: the block
// side chosen per query, fixed sides 4 and 6 (which also set the strip's halo
// and width), and the sub-strip kernel with per-query sides.
const int32_t kBlockCand[] = {0, 4, 6, NM_BLOCK_SUBSTRIPS};
constexpr int kNumBlockCand = 4;

int32_t cell_w_for(int32_t n, int32_t box, double per_cell) {
  return nm_suggest_cell_w(n, box, per_cell);
}

nm_grid grid_of(const nm_batch* b, int s) {
  nm_grid g{};
  g.n = b->n[s];
  g.box = b->box;
  g.cell_w = 1 << b->wlog[s];
  g.block = b->block[s];
  return g;
}

// Descriptors and work items for the systems in `which` (in that order).
void build_tables(nm_batch* b, const std::vector<int>& which, std::vector<BatchSys>& sys,
                  std::vector<int32_t>& items, int32_t begin[kStages + 1]) {
  sys.clear();
  for (int s : which) {
    SysSpec sp{};
    sp.g = grid_of(b, s);
    sp.ws = b->ws + b->ws_off[s];
    const int64_t o = b->off[s];
    for (int t = 0; t < 2; ++t) {
      sp.x[t] = b->io.x[t] + o;
      sp.y[t] = b->io.y[t] + o;
      sp.th[t] = b->io.theta[t] + o;
    }
    sp.nbr = b->io.nbr + o * b->k;
    sp.v0 = b->p.v0;
    sp.eta = b->p.eta;
    sp.include_self = b->p.include_self;
    sp.variant = b->p.variant;
    sp.seed = b->p.seed;
    sp.sys_id = b->sys_id[s];
    sp.step = b->step0 + static_cast<uint64_t>(b->steps_done);
    sp.parity = static_cast<int32_t>(b->steps_done & 1);
    sys.push_back(make_batch_sys(sp, b->k));
  }
  batch_items(sys, items, begin);
}

// Largest item count of one system over every tuner candidate.
int64_t max_items(const nm_batch* b, int s) {
  int64_t best = 0;
  for (int c = 0; c < kNumPerCell; ++c) {
    for (int bc = 0; bc < kNumBlockCand; ++bc) {
      nm_grid g{b->n[s], b->box, cell_w_for(b->n[s], b->box, kPerCell[c]), kBlockCand[bc]};
      Layout lay;
      if (!make_layout(&g, &lay)) continue;
      const DevWs w = dev_ws(&g, lay, nullptr);  // geometry only
      const TileCfg tc = tile_cfg(w, fast_cfg(w, b->k, g.block), b->k);
      const int64_t tiles = static_cast<int64_t>(tc.ntx) * tc.nty;
      const int64_t bin_items = lay.nbins > 0
                                    ? 2 * static_cast<int64_t>(lay.nblk) + lay.nb_scan_h + lay.nbins
                                    : (g.n + kBlock - 1) / kBlock + lay.nb_scan_c +
                                          (g.n + 4 * kBlock - 1) / (4 * kBlock);
      best = std::max<int64_t>(best, 64 + bin_items + tiles);
    }
  }
  return best;
}

hipError_t upload(nm_batch* b, const std::vector<BatchSys>& sys, const std::vector<int32_t>& items,
                  const int32_t begin[kStages + 1], hipStream_t s) {
  if (static_cast<int64_t>(items.size()) > b->items_cap ||
      static_cast<int64_t>(sys.size()) > b->nsys)
    return hipErrorInvalidValue;
  BatchRef& r = b->ref;
  r.sys = reinterpret_cast<BatchSys*>(b->ws + b->off_sys);
  r.items = reinterpret_cast<const int32_t*>(b->ws + b->off_items);
  r.nsys = static_cast<int32_t>(sys.size());
  for (int st = 0; st <= kStages; ++st) r.begin[st] = begin[st];
  hipError_t e = hipMemcpyAsync(r.sys, sys.data(), sys.size() * sizeof(BatchSys),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpyAsync(const_cast<int32_t*>(r.items), items.data(), items.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
  // The host vectors are pageable: wait so that they may change afterwards.
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

void drop_graph(nm_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
}

// Tables for all systems with the current choices, uploaded, workspaces
// initialised (the cell width may have changed).
int rebuild_all(nm_batch* b, hipStream_t s) {
  std::vector<int> all(b->nsys);
  for (int q = 0; q < b->nsys; ++q) all[q] = q;
  int32_t begin[kStages + 1];
  build_tables(b, all, b->host_sys, b->host_items, begin);
  drop_graph(b);
  if (upload(b, b->host_sys, b->host_items, begin, s) != hipSuccess) return NM_E_DEVICE;
  if (launch_batch_bin(b->ref, kStInit, s) != hipSuccess) return NM_E_DEVICE;
  return NM_OK;
}

}  // namespace

extern "C" {

int nm_batch_plan(int32_t nsys, const int32_t* n, int32_t box, int32_t k, const nm_params* p,
                  const uint32_t* sys_ids, nm_batch** out, int64_t* ws_bytes) {
  if (out == nullptr || ws_bytes == nullptr || n == nullptr || p == nullptr) return NM_E_INVAL;
  *out = nullptr;
  if (nsys < 1 || nsys > NM_BATCH_MAX_SYS || k < 1 || k > NM_MAX_K) return NM_E_INVAL;
  if (p->box != box || (p->variant & ~kVariantMask) != 0 || (p->include_self != 0 && p->include_self != 1))
    return NM_E_INVAL;
  if (!(p->eta >= 0.0f) || !isfinite(p->eta) || 2ll * llabs(static_cast<long long>(p->v0)) >= box)
    return NM_E_INVAL;
  nm_batch* b = new nm_batch();
  b->nsys = nsys;
  b->box = box;
  b->k = k;
  b->p = *p;
  b->n.assign(n, n + nsys);
  b->off.resize(nsys);
  b->sys_id.resize(nsys);
  b->wlog.resize(nsys);
  b->block.assign(nsys, 0);
  b->ws_off.resize(nsys);
  b->ws_len.resize(nsys);
  int64_t total_n = 0, items = 0;
  for (int s = 0; s < nsys; ++s) {
    if (n[s] < k + 1 || n[s] > kMaxParticles) {
      delete b;
      return NM_E_INVAL;
    }
    b->off[s] = static_cast<int32_t>(total_n);
    total_n += n[s];
    if (total_n > INT32_MAX) {
      delete b;
      return NM_E_INVAL;
    }
    b->sys_id[s] = sys_ids ? sys_ids[s] : static_cast<uint32_t>(s);
    int64_t need = 0;
    for (int c = 0; c < kNumPerCell; ++c) {
      nm_grid g{n[s], box, cell_w_for(n[s], box, kPerCell[c]), 0};
      const int64_t bytes = nm_workspace_bytes(&g);
      if (bytes < 0) {
        delete b;
        return NM_E_INVAL;
      }
      need = std::max(need, bytes);
    }
    b->ws_len[s] = rup(need);
    b->wlog[s] = ilog2i(cell_w_for(n[s], box, 2.0));
    items += max_items(b, s);
  }
  int64_t off = rup(256);
  b->off_sys = off;
  off += rup(static_cast<int64_t>(sizeof(BatchSys)) * nsys);
  b->off_items = off;
  b->items_cap = items;
  off += rup(4 * items);
  for (int s = 0; s < nsys; ++s) {
    b->ws_off[s] = off;
    off += b->ws_len[s];
  }
  b->total_bytes = off;
  *ws_bytes = off;
  *out = b;
  return NM_OK;
}

int nm_batch_bind(nm_batch* b, void* ws, size_t ws_bytes, const nm_batch_io* io, uint64_t step0,
                  void* stream) {
  if (b == nullptr || ws == nullptr || io == nullptr) return NM_E_INVAL;
  if (static_cast<int64_t>(ws_bytes) < b->total_bytes || reinterpret_cast<uintptr_t>(ws) % kA != 0)
    return NM_E_INVAL;
  for (int t = 0; t < 2; ++t)
    if (io->x[t] == nullptr || io->y[t] == nullptr || io->theta[t] == nullptr) return NM_E_INVAL;
  if (io->nbr == nullptr || io->x[0] == io->x[1] || io->y[0] == io->y[1] ||
      io->theta[0] == io->theta[1])
    return NM_E_INVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  b->ws = static_cast<char*>(ws);
  b->io = *io;
  b->step0 = step0;
  b->steps_done = 0;
  if (hipMemsetAsync(b->ws, 0, 256, s) != hipSuccess) return NM_E_DEVICE;
  return rebuild_all(b, s);
}

int nm_batch_step(nm_batch* b, int32_t nsteps, int32_t use_graph, void* stream) {
  if (b == nullptr || b->ws == nullptr || nsteps < 0) return NM_E_INVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!use_graph) {
    for (int t = 0; t < nsteps; ++t)
      if (enqueue_batch_step(b->ref, b->k, true, s) != hipSuccess) return NM_E_DEVICE;
    b->steps_done += nsteps;
    return NM_OK;
  }
  if (b->graph == nullptr && nsteps > 0) {
    // Capture on a private stream (the null stream cannot be captured); the
    // graph is launched on the caller's stream.
    if (b->cap_stream == nullptr &&
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return NM_E_DEVICE;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
      return NM_E_DEVICE;
    const hipError_t e = enqueue_batch_step(b->ref, b->k, true, b->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || g == nullptr) {
      if (g) (void)hipGraphDestroy(g);
      return NM_E_DEVICE;
    }
    const hipError_t e3 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      b->graph = nullptr;
      return NM_E_DEVICE;
    }
  }
  for (int t = 0; t < nsteps; ++t)
    if (hipGraphLaunch(b->graph, s) != hipSuccess) return NM_E_DEVICE;
  b->steps_done += nsteps;
  return NM_OK;
}

int nm_batch_tune(nm_batch* b, int32_t reps, void* stream) {
  if (b == nullptr || b->ws == nullptr || reps < 1) return NM_E_INVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // Size classes: systems with the same floor(log2 n) share a choice.
  std::map<int, std::vector<int>> cls;
  for (int q = 0; q < b->nsys; ++q) cls[ilog2i(b->n[q] + 1) - 1].push_back(q);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return NM_E_DEVICE;
  const std::vector<int32_t> wlog0 = b->wlog, block0 = b->block;
  int rc = NM_OK;
  // Time `reps` steps of the class `mem` alone under the current choices
  // (after one untimed step on freshly initialised workspaces); < 0 on error.
  auto time_class = [&](const std::vector<int>& mem) -> float {
    std::vector<BatchSys> sys;
    std::vector<int32_t> items;
    int32_t begin[kStages + 1];
    build_tables(b, mem, sys, items, begin);
    if (upload(b, sys, items, begin, s) != hipSuccess || launch_batch_bin(b->ref, kStInit, s) != hipSuccess ||
        enqueue_batch_step(b->ref, b->k, false, s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess)
      return -1.0f;
    for (int t = 0; t < reps; ++t)
      if (enqueue_batch_step(b->ref, b->k, false, s) != hipSuccess) return -1.0f;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1.0f;
    return ms;
  };
  for (auto& kv : cls) {
    const std::vector<int>& mem = kv.second;
    // First the cell width (blocks chosen per query), then the block choice
    // at that width.
    float best_ms = 0.0f;
    int best_c = -1;
    for (int q : mem) b->block[q] = 0;
    for (int c = 0; c < kNumPerCell && rc == NM_OK; ++c) {
      for (int q : mem) b->wlog[q] = ilog2i(cell_w_for(b->n[q], b->box, kPerCell[c]));
      bool dup = false;  // same widths as an earlier candidate: nothing new to time
      for (int c2 = 0; c2 < c && !dup; ++c2) {
        dup = true;
        for (int q : mem) dup = dup && ilog2i(cell_w_for(b->n[q], b->box, kPerCell[c2])) == b->wlog[q];
      }
      if (dup) continue;
      const float ms = time_class(mem);
      if (ms < 0.0f) {
        rc = NM_E_DEVICE;
        break;
      }
      if (best_c < 0 || ms < best_ms) {
        best_ms = ms;
        best_c = c;
      }
    }
    if (rc != NM_OK) break;
    for (int q : mem) b->wlog[q] = ilog2i(cell_w_for(b->n[q], b->box, kPerCell[best_c]));
    int best_b = 0;  // kBlockCand[0] = 0, timed above at this width
    for (int bc = 1; bc < kNumBlockCand && rc == NM_OK; ++bc) {
      for (int q : mem) b->block[q] = kBlockCand[bc];
      const float ms = time_class(mem);
      if (ms < 0.0f) {
        rc = NM_E_DEVICE;
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_b = bc;
      }
    }
    if (rc != NM_OK) break;
    for (int q : mem) b->block[q] = kBlockCand[best_b];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NM_OK) {
    b->wlog = wlog0;
    b->block = block0;
    rebuild_all(b, s);
    return rc;
  }
  return rebuild_all(b, s);
}

int nm_batch_set_block(nm_batch* b, int32_t block, void* stream) {
  if (b == nullptr || b->ws == nullptr) return NM_E_INVAL;
  for (int q = 0; q < b->nsys; ++q) {
    nm_grid g = grid_of(b, q);
    g.block = block;
    Layout lay;
    if (!make_layout(&g, &lay)) return NM_E_INVAL;
  }
  b->block.assign(b->nsys, block);
  return rebuild_all(b, reinterpret_cast<hipStream_t>(stream));
}

int nm_batch_system(const nm_batch* b, int32_t s, nm_grid* g, int32_t* offset) {
  if (b == nullptr || s < 0 || s >= b->nsys) return NM_E_INVAL;
  if (g) *g = grid_of(b, s);
  if (offset) *offset = b->off[s];
  return NM_OK;
}

int64_t nm_batch_steps_done(const nm_batch* b) { return b ? b->steps_done : NM_E_INVAL; }

int nm_batch_check(nm_batch* b, void* stream) {
  if (b == nullptr || b->ws == nullptr) return NM_E_INVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t* err = reinterpret_cast<int32_t*>(b->ws);
  hipLaunchKernelGGL(k_bb_errors, dim3((b->nsys + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     b->ref.sys, b->nsys, err);
  int32_t host = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&host, err, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return NM_E_DEVICE;
  if (host != 0 && (hipMemsetAsync(err, 0, sizeof(int32_t), s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess))
    return NM_E_DEVICE;
  return host;
}

void nm_batch_destroy(nm_batch* b) {
  if (b == nullptr) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
