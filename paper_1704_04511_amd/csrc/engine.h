// Lock-step engine for many reconstructions (see engine.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <vector>

#include "../../include/slrx.h"

namespace slrx {

// Workspace of the batched eigen-decomposition (own stream and handle).
struct BatchEig {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;       // eigenpairs ready
  hipEvent_t ev_free = nullptr;  // every consumer of the eigenpairs has run
  bool have_free = false;
  rocblas_handle handle = nullptr;
  int cap_nb = 0;                // capacity in matrices
  long cap_ss = 0;               // capacity in matrix elements (sum of s*s)
  long cap_s = 0;                // capacity in eigenvalues (sum of s)
  double2* A = nullptr;          // Gram matrices, then eigenvectors (column-major, one region per group)
  double* D = nullptr;           // eigenvalues, ascending
  double* E = nullptr;           // solver workspace
  rocblas_int* info = nullptr;
  ~BatchEig();
};

// Start a problem: masked data, initial iterate, start event, iteration 0.
slrx_status engine_begin(slrx_plan* pl);
// Enqueue one outer iteration for every given problem that has iterations
// left (no host synchronisation).
slrx_status engine_step(const std::vector<slrx_plan*>& plans, BatchEig& be);
// Record the completion event of a problem whose iterations are done.
slrx_status engine_end(slrx_plan* pl);

}  // namespace slrx
