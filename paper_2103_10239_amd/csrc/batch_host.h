// batch_host.h -- host-side construction of batched step descriptors, shared
// by the batched form (batch.hip) and the served form (server.hip).
#pragma once

#include <vector>

#include "nm_internal.h"

namespace nm {

// One system of a batch: grid, workspace, double-buffered state, list output,
// step parameters, Philox identity and its position in its own run.
struct SysSpec {
  nm_grid g;
  void* ws;  // initialised workspace of nm_workspace_bytes(&g) bytes
  int32_t* x[2];
  int32_t* y[2];
  float* th[2];
  int32_t* nbr;  // int32[n * k]
  int32_t v0;
  float eta;
  int32_t include_self;
  uint32_t variant;
  uint64_t seed;
  uint32_t sys_id;
  uint64_t step;   // Philox step of the system's next step
  int32_t parity;  // buffer holding its current state
};

// Device descriptor of one system for k nearest neighbours.
BatchSys make_batch_sys(const SysSpec& s, int k);

// Work items of every stage for the descriptors in order: fills each
// descriptor's item ranges and the concatenated stage tables.
void batch_items(std::vector<BatchSys>& sys, std::vector<int32_t>& items, int32_t begin[kStages + 1]);

// Enqueue one batched step (binning, k-NN + alignment; `advance`: then flip
// every system's parity and increment its step on the device).
hipError_t enqueue_batch_step(const BatchRef& r, int k, bool advance, hipStream_t s);

}  // namespace nm
