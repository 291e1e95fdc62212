// server.hip -- the served form: a request loop that keeps jobs' state on the
// device and advances every admitted job by one step of Alg. 1 (k-NN rule,
// Eq. (2), Eq. (1)) per engine iteration, with continuous batching.
//
//   submit      copies the job's host inputs, queues it (FIFO)
//   engine      admits queued jobs while the HBM ledger (bytes of the job's
//               workspace, double-buffered state and list) fits the budget
//               and a slot is free; device memory comes from a slab
//               allocator; jobs that arrive while others run join at the
//               next iteration.  Each iteration is one batched launch per
//               stage for all active jobs of the same k (the kernels of the
//               batched form), then every job's step count advances; a job
//               that reached its nsteps leaves the batch.
//   completer   waits for a finished job's last step, copies its state to
//               the host, releases its memory and ledger bytes.
//
// A job's results do not depend on what else is in the batch: the kernels
// compute each system independently, and its Philox stream is keyed by the
// job's own seed, sys_id and step count.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch_host.h"

namespace {

using nm::BatchRef;
using nm::BatchSys;
using nm::kStages;

constexpr int64_t kAlignB = 256;
int64_t rup(int64_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

// Device memory: slabs from hipMalloc on demand (1 GiB, or one job's size),
// first fit inside a slab, adjacent free ranges merged.  Slabs are kept
// until the server is destroyed.
class DevArena {
 public:
  ~DevArena() {
    for (auto& s : slabs_) (void)hipFree(s.base);
  }
  char* alloc(int64_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    bytes = rup(bytes);
    for (size_t i = 0; i < slabs_.size(); ++i) {
      char* p = carve(i, bytes);
      if (p) return p;
    }
    Slab s;
    s.size = std::max<int64_t>(kSlab, bytes);
    void* base = nullptr;
    if (hipMalloc(&base, static_cast<size_t>(s.size)) != hipSuccess) return nullptr;
    s.base = static_cast<char*>(base);
    s.free[0] = s.size;
    slabs_.push_back(std::move(s));
    reserved_ += slabs_.back().size;
    return carve(slabs_.size() - 1, bytes);
  }
  void release(char* p) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    Slab& s = slabs_[it->second.first];
    int64_t off = p - s.base, len = it->second.second;
    live_.erase(it);
    auto nx = s.free.lower_bound(off);
    if (nx != s.free.end() && off + len == nx->first) {
      len += nx->second;
      nx = s.free.erase(nx);
    }
    if (nx != s.free.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    s.free[off] = len;
  }
  int64_t reserved() const { return reserved_; }

 private:
  struct Slab {
    char* base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free;  // offset -> length
  };
  char* carve(size_t i, int64_t bytes) {
    Slab& s = slabs_[i];
    for (auto it = s.free.begin(); it != s.free.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, rest = it->second - bytes;
      s.free.erase(it);
      if (rest > 0) s.free[off + bytes] = rest;
      char* p = s.base + off;
      live_[p] = {static_cast<int>(i), bytes};
      return p;
    }
    return nullptr;
  }
  static constexpr int64_t kSlab = int64_t(1) << 30;
  std::mutex mu_;
  std::vector<Slab> slabs_;
  std::map<char*, std::pair<int, int64_t>> live_;
  int64_t reserved_ = 0;
};

enum JobState { kPending = 0, kActive, kFinishing, kDone };

struct Job {
  int64_t id = 0;
  int32_t n = 0, k = 0, nsteps = 0, want_nbr = 0;
  nm_params p{};
  std::vector<int32_t> hx, hy, hnbr;
  std::vector<float> ht;
  nm_grid g{};
  int64_t ws_bytes = 0, bytes = 0;
  char* dmem = nullptr;
  nm::SysSpec spec{};
  int64_t steps_done = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = kPending;
  int status = NM_OK;
  hipEvent_t last = nullptr;  // recorded after the job's last step
};

// Device tables of one k class (descriptors + work items), grown on demand.
struct KClass {
  std::vector<Job*> members;
  bool dirty = true;
  std::vector<BatchSys> sys;
  std::vector<int32_t> items;
  int32_t begin[kStages + 1] = {};
  char* dtab = nullptr;
  int64_t dtab_bytes = 0;
  char* pinned = nullptr;  // host staging of the tables
  int64_t pinned_bytes = 0;
  hipEvent_t uploaded = nullptr;
  BatchRef ref{};
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int64_t job_layout(int32_t n, int32_t k, int32_t box, nm_grid* g, int64_t* ws_bytes) {
  nm_grid gg{n, box, nm_suggest_cell_w(n, box, 2.0), 0};
  const int64_t wsb = nm_workspace_bytes(&gg);
  if (wsb < 0) return wsb;
  if (g) *g = gg;
  if (ws_bytes) *ws_bytes = rup(wsb);
  return rup(wsb) + 6 * rup(4 * static_cast<int64_t>(n)) + rup(4 * static_cast<int64_t>(n) * k);
}

}  // namespace

struct nm_server {
  int64_t budget = 0;
  int32_t max_slots = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_engine, cv_done, cv_complete;
  std::deque<Job*> pending;           // guarded by mu
  std::map<int64_t, Job*> jobs;       // guarded by mu
  std::deque<Job*> finishing;         // guarded by mu
  int64_t next_id = 1, used = 0, peak_used = 0, submitted = 0, completed = 0, iterations = 0;
  int32_t active_n = 0, peak_active = 0;
  bool stop = false, engine_exited = false;
  int engine_status = NM_OK;
  hipStream_t cs = nullptr, xs = nullptr;
  DevArena arena;
  std::map<int, KClass> classes;      // engine thread only
  std::vector<Job*> active;           // engine thread only
  std::deque<hipEvent_t> inflight;    // engine thread only
  std::thread engine, completer;
};

namespace {

void fail_job(nm_server* s, Job* j, int status) {
  std::lock_guard<std::mutex> g(s->mu);
  j->status = status;
  j->state = kDone;
  j->t_done = now_s(s->t0);
  if (j->dmem) {
    s->arena.release(j->dmem);
    j->dmem = nullptr;
    s->used -= j->bytes;
  }
  ++s->completed;
  s->cv_done.notify_all();
}

// Place an admitted job in device memory and enqueue its input upload and
// workspace initialisation.
bool start_job(nm_server* s, Job* j) {
  char* m = j->dmem;
  nm::SysSpec& sp = j->spec;
  sp.g = j->g;
  sp.ws = m;
  int64_t off = j->ws_bytes;
  const int64_t vec = rup(4 * static_cast<int64_t>(j->n));
  for (int t = 0; t < 2; ++t) {
    sp.x[t] = reinterpret_cast<int32_t*>(m + off);
    off += vec;
    sp.y[t] = reinterpret_cast<int32_t*>(m + off);
    off += vec;
    sp.th[t] = reinterpret_cast<float*>(m + off);
    off += vec;
  }
  sp.nbr = reinterpret_cast<int32_t*>(m + off);
  sp.v0 = j->p.v0;
  sp.eta = j->p.eta;
  sp.include_self = j->p.include_self;
  sp.variant = j->p.variant;
  sp.seed = j->p.seed;
  sp.sys_id = j->p.sys_id;
  sp.step = 0;
  sp.parity = 0;
  const size_t nb = 4 * static_cast<size_t>(j->n);
  if (hipMemcpyAsync(sp.x[0], j->hx.data(), nb, hipMemcpyHostToDevice, s->cs) != hipSuccess ||
      hipMemcpyAsync(sp.y[0], j->hy.data(), nb, hipMemcpyHostToDevice, s->cs) != hipSuccess ||
      hipMemcpyAsync(sp.th[0], j->ht.data(), nb, hipMemcpyHostToDevice, s->cs) != hipSuccess)
    return false;
  return nm_workspace_init(&j->g, m, static_cast<size_t>(j->ws_bytes), s->cs) == NM_OK;
}

bool upload_class(nm_server* s, KClass& c, int k) {
  c.sys.clear();
  for (Job* j : c.members) {
    nm::SysSpec sp = j->spec;
    sp.step = static_cast<uint64_t>(j->steps_done);
    sp.parity = static_cast<int32_t>(j->steps_done & 1);
    c.sys.push_back(nm::make_batch_sys(sp, k));
  }
  nm::batch_items(c.sys, c.items, c.begin);
  const int64_t sys_b = rup(static_cast<int64_t>(c.sys.size() * sizeof(BatchSys)));
  const int64_t need = sys_b + rup(static_cast<int64_t>(c.items.size() * sizeof(int32_t)));
  if (c.uploaded && hipEventSynchronize(c.uploaded) != hipSuccess) return false;  // staging free
  if (need > c.dtab_bytes) {
    // Tables grow rarely: wait for work that may still read the old ones.
    if (hipStreamSynchronize(s->cs) != hipSuccess) return false;
    if (c.dtab) (void)hipFree(c.dtab);
    if (c.pinned) (void)hipHostFree(c.pinned);
    c.dtab = nullptr;
    c.pinned = nullptr;
    c.dtab_bytes = std::max<int64_t>(need * 2, 1 << 20);
    void* d = nullptr;
    void* h = nullptr;
    if (hipMalloc(&d, static_cast<size_t>(c.dtab_bytes)) != hipSuccess) return false;
    if (hipHostMalloc(&h, static_cast<size_t>(c.dtab_bytes), hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(d);
      return false;
    }
    c.dtab = static_cast<char*>(d);
    c.pinned = static_cast<char*>(h);
  }
  std::memcpy(c.pinned, c.sys.data(), c.sys.size() * sizeof(BatchSys));
  std::memcpy(c.pinned + sys_b, c.items.data(), c.items.size() * sizeof(int32_t));
  if (hipMemcpyAsync(c.dtab, c.pinned, static_cast<size_t>(need), hipMemcpyHostToDevice, s->cs) != hipSuccess)
    return false;
  if (!c.uploaded && hipEventCreateWithFlags(&c.uploaded, hipEventDisableTiming) != hipSuccess)
    return false;
  if (hipEventRecord(c.uploaded, s->cs) != hipSuccess) return false;
  c.ref.sys = reinterpret_cast<BatchSys*>(c.dtab);
  c.ref.items = reinterpret_cast<const int32_t*>(c.dtab + sys_b);
  c.ref.nsys = static_cast<int32_t>(c.sys.size());
  for (int st = 0; st <= kStages; ++st) c.ref.begin[st] = c.begin[st];
  c.dirty = false;
  return true;
}

void engine_loop(nm_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    // Admission, FIFO, while the ledger and the slots allow.
    std::vector<Job*> admitted, refused;
    {
      std::unique_lock<std::mutex> g(s->mu);
      while (!s->pending.empty()) {
        Job* j = s->pending.front();
        if (s->used + j->bytes > s->budget ||
            static_cast<int32_t>(s->active.size() + admitted.size()) >= s->max_slots)
          break;
        j->dmem = s->arena.alloc(j->bytes);
        if (j->dmem == nullptr) {
          // Device memory exhausted: wait for running jobs to release theirs;
          // with none running, the job can never start.
          if (s->active.empty() && admitted.empty() && s->finishing.empty() && s->used == 0) {
            s->pending.pop_front();
            refused.push_back(j);
            continue;
          }
          break;
        }
        s->pending.pop_front();
        s->used += j->bytes;
        s->peak_used = std::max(s->peak_used, s->used);
        admitted.push_back(j);
      }
      if (s->active.empty() && admitted.empty() && refused.empty()) {
        if (s->stop && s->pending.empty()) break;
        s->cv_engine.wait_for(g, std::chrono::milliseconds(2));
        continue;
      }
    }
    for (Job* j : refused) fail_job(s, j, NM_E_NOMEM);
    for (Job* j : admitted) {
      if (!start_job(s, j)) {
        fail_job(s, j, NM_E_DEVICE);
        continue;
      }
      j->t_admit = now_s(s->t0);
      j->state = kActive;
      s->active.push_back(j);
      KClass& c = s->classes[j->k];
      c.members.push_back(j);
      c.dirty = true;
    }
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->active_n = static_cast<int32_t>(s->active.size());
      s->peak_active = std::max(s->peak_active, s->active_n);
    }
    if (s->active.empty()) continue;

    // One step for every active job: one batched launch per stage and k.
    bool ok = true;
    for (auto& kv : s->classes) {
      KClass& c = kv.second;
      if (c.members.empty()) continue;
      if (c.dirty && !upload_class(s, c, kv.first)) ok = false;
      if (ok && nm::enqueue_batch_step(c.ref, kv.first, true, s->cs) != hipSuccess) ok = false;
    }
    hipEvent_t ev = nullptr;
    if (ok && (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
               hipEventRecord(ev, s->cs) != hipSuccess))
      ok = false;
    std::vector<Job*> still;
    for (Job* j : s->active) {
      ++j->steps_done;
      if (j->steps_done < j->nsteps && ok) {
        still.push_back(j);
        continue;
      }
      KClass& c = s->classes[j->k];
      c.members.erase(std::find(c.members.begin(), c.members.end(), j));
      c.dirty = true;
      if (hipEventCreateWithFlags(&j->last, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(j->last, s->cs) != hipSuccess) {
        j->last = nullptr;
        fail_job(s, j, NM_E_DEVICE);
        continue;
      }
      std::lock_guard<std::mutex> g(s->mu);
      if (!ok) j->status = NM_E_DEVICE;
      j->state = kFinishing;
      s->finishing.push_back(j);
      s->cv_complete.notify_one();
    }
    s->active.swap(still);
    {
      std::lock_guard<std::mutex> g(s->mu);
      ++s->iterations;
      s->active_n = static_cast<int32_t>(s->active.size());
      if (!ok) s->engine_status = NM_E_DEVICE;
    }
    // Keep at most three iterations in flight.
    if (ev) s->inflight.push_back(ev);
    while (s->inflight.size() > 3) {
      (void)hipEventSynchronize(s->inflight.front());
      (void)hipEventDestroy(s->inflight.front());
      s->inflight.pop_front();
    }
  }
  for (hipEvent_t e : s->inflight) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  s->inflight.clear();
  std::lock_guard<std::mutex> g(s->mu);
  s->engine_exited = true;
  s->cv_complete.notify_all();
}

void completer_loop(nm_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> g(s->mu);
      s->cv_complete.wait(g, [&] { return !s->finishing.empty() || s->engine_exited; });
      if (s->finishing.empty()) break;
      j = s->finishing.front();
      s->finishing.pop_front();
    }
    int status = j->status;
    if (hipEventSynchronize(j->last) != hipSuccess) status = NM_E_DEVICE;
    (void)hipEventDestroy(j->last);
    j->last = nullptr;
    const int p = static_cast<int>(j->nsteps & 1);
    const size_t nb = 4 * static_cast<size_t>(j->n);
    int32_t err = 0;
    if (status == NM_OK) {
      if (j->want_nbr) j->hnbr.resize(static_cast<size_t>(j->n) * j->k);
      if (hipMemcpyAsync(j->hx.data(), j->spec.x[p], nb, hipMemcpyDeviceToHost, s->xs) != hipSuccess ||
          hipMemcpyAsync(j->hy.data(), j->spec.y[p], nb, hipMemcpyDeviceToHost, s->xs) != hipSuccess ||
          hipMemcpyAsync(j->ht.data(), j->spec.th[p], nb, hipMemcpyDeviceToHost, s->xs) != hipSuccess ||
          (j->want_nbr && hipMemcpyAsync(j->hnbr.data(), j->spec.nbr, nb * j->k, hipMemcpyDeviceToHost,
                                         s->xs) != hipSuccess) ||
          hipMemcpyAsync(&err, reinterpret_cast<char*>(j->dmem) + sizeof(uint32_t), sizeof(err),
                         hipMemcpyDeviceToHost, s->xs) != hipSuccess ||
          hipStreamSynchronize(s->xs) != hipSuccess)
        status = NM_E_DEVICE;
      else if (err != 0)
        status = err;
    }
    std::lock_guard<std::mutex> g(s->mu);
    s->arena.release(j->dmem);
    j->dmem = nullptr;
    s->used -= j->bytes;
    j->status = status;
    j->state = kDone;
    j->t_done = now_s(s->t0);
    ++s->completed;
    s->cv_done.notify_all();
    s->cv_engine.notify_one();
  }
}

}  // namespace

extern "C" {

int64_t nm_server_job_bytes(int32_t n, int32_t k, int32_t box) {
  if (n < 2 || k < 1 || k > NM_MAX_K || k > n - 1) return NM_E_INVAL;
  return job_layout(n, k, box, nullptr, nullptr);
}

int nm_server_create(int64_t budget_bytes, int32_t max_slots, nm_server** out) {
  if (out == nullptr || budget_bytes <= 0 || max_slots < 1 || max_slots > NM_BATCH_MAX_SYS)
    return NM_E_INVAL;
  *out = nullptr;
  nm_server* s = new nm_server();
  s->budget = budget_bytes;
  s->max_slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->cs, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->xs, hipStreamNonBlocking) != hipSuccess) {
    if (s->cs) (void)hipStreamDestroy(s->cs);
    delete s;
    return NM_E_DEVICE;
  }
  s->engine = std::thread(engine_loop, s);
  s->completer = std::thread(completer_loop, s);
  *out = s;
  return NM_OK;
}

int nm_server_submit(nm_server* s, const nm_job* job, int64_t* id) {
  if (s == nullptr || job == nullptr || id == nullptr) return NM_E_INVAL;
  const nm_params& p = job->p;
  if (job->n < 2 || job->k < 1 || job->k > NM_MAX_K || job->k > job->n - 1 || job->nsteps < 1)
    return NM_E_INVAL;
  if (job->x == nullptr || job->y == nullptr || job->theta == nullptr || (p.variant & ~nm::kVariantMask) != 0) return NM_E_INVAL;
  if (p.include_self != 0 && p.include_self != 1) return NM_E_INVAL;
  if (!(p.eta >= 0.0f) || !isfinite(p.eta) || 2ll * llabs(static_cast<long long>(p.v0)) >= p.box)
    return NM_E_INVAL;
  Job* j = new Job();
  j->bytes = job_layout(job->n, job->k, p.box, &j->g, &j->ws_bytes);
  if (j->bytes < 0) {
    delete j;
    return NM_E_INVAL;
  }
  if (j->bytes > s->budget) {
    delete j;
    return NM_E_NOMEM;
  }
  j->n = job->n;
  j->k = job->k;
  j->nsteps = job->nsteps;
  j->want_nbr = job->want_nbr ? 1 : 0;
  j->p = p;
  j->hx.assign(job->x, job->x + job->n);
  j->hy.assign(job->y, job->y + job->n);
  j->ht.assign(job->theta, job->theta + job->n);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) {
    delete j;
    return NM_E_INVAL;
  }
  j->id = s->next_id++;
  j->t_submit = now_s(s->t0);
  s->jobs[j->id] = j;
  s->pending.push_back(j);
  ++s->submitted;
  s->cv_engine.notify_one();
  *id = j->id;
  return NM_OK;
}

int nm_server_poll(nm_server* s, int64_t id) {
  if (s == nullptr) return NM_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return NM_E_INVAL;
  return it->second->state == kDone ? 1 : 0;
}

int nm_server_wait(nm_server* s, int64_t id, int32_t* x, int32_t* y, float* theta, int32_t* nbr,
                   nm_job_result* r) {
  if (s == nullptr) return NM_E_INVAL;
  Job* j = nullptr;
  {
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return NM_E_INVAL;
    j = it->second;
    s->cv_done.wait(g, [&] { return j->state == kDone; });
    s->jobs.erase(it);
  }
  const size_t n = static_cast<size_t>(j->n);
  if (j->status == NM_OK) {
    if (x) std::memcpy(x, j->hx.data(), 4 * n);
    if (y) std::memcpy(y, j->hy.data(), 4 * n);
    if (theta) std::memcpy(theta, j->ht.data(), 4 * n);
    if (nbr && j->want_nbr) std::memcpy(nbr, j->hnbr.data(), 4 * n * j->k);
  }
  if (r) {
    r->status = j->status;
    r->steps = static_cast<int32_t>(j->steps_done);
    r->submit_s = j->t_submit;
    r->admit_s = j->t_admit;
    r->done_s = j->t_done;
  }
  const int st = j->status;
  delete j;
  return st;
}

int nm_server_stats(nm_server* s, nm_server_info* out) {
  if (s == nullptr || out == nullptr) return NM_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->iterations = s->iterations;
  out->budget_bytes = s->budget;
  out->used_bytes = s->used;
  out->peak_used_bytes = s->peak_used;
  out->reserved_bytes = s->arena.reserved();
  out->active = s->active_n;
  out->peak_active = s->peak_active;
  out->queued = static_cast<int32_t>(s->pending.size());
  out->status = s->engine_status;
  out->now_s = now_s(s->t0);
  return NM_OK;
}

void nm_server_destroy(nm_server* s) {
  if (s == nullptr) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_engine.notify_all();
    s->cv_complete.notify_all();
  }
  s->engine.join();
  s->completer.join();
  for (auto& kv : s->classes) {
    KClass& c = kv.second;
    if (c.uploaded) (void)hipEventDestroy(c.uploaded);
    if (c.dtab) (void)hipFree(c.dtab);
    if (c.pinned) (void)hipHostFree(c.pinned);
  }
  for (auto& kv : s->jobs) delete kv.second;
  (void)hipStreamDestroy(s->cs);
  (void)hipStreamDestroy(s->xs);
  delete s;
}

}  // extern "C"
