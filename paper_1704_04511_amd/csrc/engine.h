// Lock-step engine for many reconstructions (see engine.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "../../include/slrx.h"
#include "kernels.h"
#include "plan.h"

namespace slrx {

// Eigen-decomposition buffers for up to `cap` problems of size n, strided.
struct EigGroup {
  int n = 0, cap = 0;
  void* mem = nullptr;  // one allocation holding every buffer below
  EighBufs bufs;        // pointers into mem, strides for problem b
  int* tree = nullptr;  // divide-and-conquer tree for n (device)
  std::vector<int> level_start, node_sizes;
  ~EigGroup();
};

// Table of a grouped CG launch (kernels.h CgSlice): the device copy, a pinned
// staging copy, and the host copy it was made from (rewritten only when the
// problems of the group change).
struct CgTable {
  std::vector<CgSlice> host;
  CgSlice* dev = nullptr;
  CgSlice* pinned = nullptr;
  size_t cap = 0;                // entries of dev and pinned
  hipEvent_t copied = nullptr;   // the last upload from pinned has run
  bool pending = false;
  ~CgTable();
};

// Shared state of the batched eigen-decompositions and the grouped CG (own
// streams and events).
struct BatchEig {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;       // eigenpairs ready
  hipEvent_t ev_free = nullptr;  // every reader of the group buffers has run
  bool have_free = false;
  std::map<int, EigGroup> groups;
  hipStream_t cg_stream = nullptr;  // grouped CG passes
  hipEvent_t ev_cg = nullptr;       // a group's CG has run
  std::map<std::pair<int, int>, CgTable> cg_tables;  // by (M, n_cg)
  size_t allocated() const;  // device bytes held by the groups and tables
  ~BatchEig();
};

// Device bytes the shared eigen-decomposition buffers hold per problem of Gram
// size n (an upper bound of what one more problem of that size adds).
size_t engine_problem_bytes(int n);
// Shrink the groups to at most keep[n] problems of size n (absent: none), after
// the work that reads them has finished (synchronises the engine's stream).
slrx_status engine_trim(BatchEig& be, const std::map<int, int>& keep);

// Start a problem: masked data, initial iterate, start event, iteration 0.
slrx_status engine_begin(slrx_plan* pl);
// Enqueue one outer iteration for every given problem that has iterations
// left (no host synchronisation).
slrx_status engine_step(const std::vector<slrx_plan*>& plans, BatchEig& be);
// Record the completion event of a problem whose iterations are done.
slrx_status engine_end(slrx_plan* pl);

}  // namespace slrx
