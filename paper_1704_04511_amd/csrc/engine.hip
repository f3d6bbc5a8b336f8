// Lock-step execution of many reconstructions (batch and continuous serving).
//
// Every active problem advances by one outer IRLS iteration per engine step.
// Problems whose Gram matrices have the same size s <= kBatchEigMaxS share one
// batched FP64 eigen-decomposition (rocSOLVER zheevd, strided batched over a
// shared buffer); larger problems take the single-problem path (own Householder
// tridiagonalisation).  The choice depends on s only, and the batched solver
// treats every matrix independently, so each problem's result is the same
// whatever else is in the batch.  The Gram matrix, weights, masks and CG of each
// problem run on the problem's own stream, ordered against the shared
// eigen-decomposition by events.  Problems may join between steps (each keeps
// its own iteration index and epsilon schedule), which is what the server does.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <map>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "plan.h"

using namespace slrx;

// Largest Gram size solved in the batched eigen-decomposition.
constexpr int kBatchEigMaxS = 640;

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(SLRX_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                                 \
  } while (0)

#define STCHK(expr)               \
  do {                            \
    slrx_status _s = (expr);      \
    if (_s != SLRX_OK) return _s; \
  } while (0)

slrx::BatchEig::~BatchEig() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (handle) rocblas_destroy_handle(handle);
  if (A) (void)hipFree(A);
  if (D) (void)hipFree(D);
  if (E) (void)hipFree(E);
  if (info) (void)hipFree(info);
  if (ev) (void)hipEventDestroy(ev);
  if (ev_free) (void)hipEventDestroy(ev_free);
  if (stream) (void)hipStreamDestroy(stream);
}

// Room for nb matrices of total size ss_total (elements) and s_total eigenvalues.
static slrx_status be_reserve(BatchEig& be, int nb, long ss_total, long s_total) {
  if (!be.stream) {
    HIPCHK(hipStreamCreateWithFlags(&be.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&be.ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&be.ev_free, hipEventDisableTiming));
    if (rocblas_create_handle(&be.handle) != rocblas_status_success)
      return fail(SLRX_EDEVICE, "rocblas_create_handle failed");
    if (rocblas_set_stream(be.handle, be.stream) != rocblas_status_success)
      return fail(SLRX_EDEVICE, "rocblas_set_stream failed");
  }
  if (nb > be.cap_nb || ss_total > be.cap_ss || s_total > be.cap_s) {
    // every reader of the old buffers is ordered before be.stream's last work
    HIPCHK(hipStreamSynchronize(be.stream));
    if (be.A) (void)hipFree(be.A);
    if (be.D) (void)hipFree(be.D);
    if (be.E) (void)hipFree(be.E);
    if (be.info) (void)hipFree(be.info);
    be.A = nullptr; be.D = nullptr; be.E = nullptr; be.info = nullptr;
    be.cap_nb = nb > be.cap_nb ? nb : be.cap_nb;
    be.cap_ss = ss_total > be.cap_ss ? ss_total : be.cap_ss;
    be.cap_s = s_total > be.cap_s ? s_total : be.cap_s;
    if (hipMalloc(&be.A, (size_t)be.cap_ss * sizeof(double2)) != hipSuccess ||
        hipMalloc(&be.D, (size_t)be.cap_s * sizeof(double)) != hipSuccess ||
        hipMalloc(&be.E, (size_t)be.cap_s * sizeof(double)) != hipSuccess ||
        hipMalloc(&be.info, be.cap_nb * sizeof(rocblas_int)) != hipSuccess) {
      be.cap_nb = 0; be.cap_ss = 0; be.cap_s = 0;
      return fail(SLRX_ENOMEM, "batched eigen-decomposition workspace");
    }
  }
  return SLRX_OK;
}

slrx_status slrx::engine_begin(slrx_plan* pl) {
  STCHK(prepare(pl));
  pl->ktime = false;
  for (int c = 0; c < SLRX_K_NCLASS; ++c) pl->kused[c] = 0;
  HIPCHK(hipMemsetAsync(pl->info, 0, (SLRX_MAX_IRLS + 1) * sizeof(rocblas_int), pl->stream));
  HIPCHK(hipEventRecord(pl->ev_run[0], pl->stream));
  pl->it_next = 0;
  pl->running = true;
  pl->ran = false;
  pl->run_irls = pl->prm.n_irls;
  pl->run_timing = false;
  return SLRX_OK;
}

slrx_status slrx::engine_end(slrx_plan* pl) {
  HIPCHK(hipEventRecord(pl->ev_run[1], pl->stream));
  return SLRX_OK;
}

// One outer iteration of one problem on its own stream (the path of a plan run alone).
static slrx_status step_single(slrx_plan* pl) {
  const int it = pl->it_next;
  STCHK(step_gram(pl));
  STCHK(step_eigh(pl, it));
  STCHK(step_weights(pl, it, it == 0, pl->prm.gamma));
  STCHK(run_cg(pl, pl->prm.n_cg, it));
  pl->it_next = it + 1;
  return SLRX_OK;
}

slrx_status slrx::engine_step(const std::vector<slrx_plan*>& plans, BatchEig& be) {
  std::map<int, std::vector<slrx_plan*>> groups;
  for (slrx_plan* pl : plans)
    if (pl->it_next < pl->prm.n_irls) groups[pl->s()].push_back(pl);
  // every batched group gets its own region of the shared buffers
  int nb_total = 0;
  long ss_total = 0, s_total = 0;
  for (auto& kv : groups) {
    if (kv.first > kBatchEigMaxS) continue;
    nb_total += (int)kv.second.size();
    ss_total += (long)kv.second.size() * kv.first * kv.first;
    s_total += (long)kv.second.size() * kv.first;
  }
  if (nb_total > 0) STCHK(be_reserve(be, nb_total, ss_total, s_total));
  int ib = 0;
  long off_ss = 0, off_s = 0;
  for (auto& kv : groups) {
    const int s = kv.first;
    std::vector<slrx_plan*>& g = kv.second;
    const int nb = (int)g.size();
    if (s > kBatchEigMaxS) {
      for (slrx_plan* pl : g) STCHK(step_single(pl));
      continue;
    }
    const long ss = (long)s * s;
    double2* A = be.A + off_ss;
    double* D = be.D + off_s;
    double* E = be.E + off_s;
    rocblas_int* info = be.info + ib;
    // Gram matrices into the shared buffer once the previous step's readers are done
    for (int i = 0; i < nb; ++i) {
      slrx_plan* pl = g[i];
      if (be.have_free) HIPCHK(hipStreamWaitEvent(pl->stream, be.ev_free, 0));
      STCHK(step_gram(pl, true, A + (size_t)i * ss));
      HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
      HIPCHK(hipStreamWaitEvent(be.stream, pl->ev_step, 0));
    }
    rocblas_status rs = rocsolver_zheevd_strided_batched(
        be.handle, rocblas_evect_original, rocblas_fill_lower, s, (rocblas_double_complex*)A, s, ss, D, s, E, s,
        info, nb);
    if (rs != rocblas_status_success)
      return fail(SLRX_EDEVICE, "rocsolver_zheevd_strided_batched failed (status %d)", (int)rs);
    HIPCHK(hipEventRecord(be.ev, be.stream));
    for (int i = 0; i < nb; ++i) {
      slrx_plan* pl = g[i];
      const int it = pl->it_next;
      HIPCHK(hipStreamWaitEvent(pl->stream, be.ev, 0));
      HIPCHK(hipMemcpyAsync(pl->info + it, info + i, sizeof(rocblas_int), hipMemcpyDeviceToDevice, pl->stream));
      STCHK(step_weights(pl, it, it == 0, pl->prm.gamma, A + (size_t)i * ss, D + (size_t)i * s));
      HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
      HIPCHK(hipStreamWaitEvent(be.stream, pl->ev_step, 0));
      STCHK(run_cg(pl, pl->prm.n_cg, it));
      pl->it_next = it + 1;
    }
    ib += nb;
    off_ss += (long)nb * ss;
    off_s += (long)nb * s;
  }
  if (nb_total > 0) {
    HIPCHK(hipEventRecord(be.ev_free, be.stream));
    be.have_free = true;
  }
  return SLRX_OK;
}
