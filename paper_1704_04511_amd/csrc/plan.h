// Internal plan state of libslrx (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <string>
#include <vector>

#include "../../include/slrx.h"

namespace slrx {

constexpr int kMaxS = 3000;    // largest filter size s = N1 N2 M (own eigensolver chain)
constexpr int kMaxCg = 10000;  // largest CG iteration count
// info: eigensolver status per outer iteration, the single-step slot
// (SLRX_MAX_IRLS), and a flag raised by the Gram pass on a non-finite entry
constexpr int kInfoNonfinite = SLRX_MAX_IRLS + 1;
constexpr int kInfoEntries = SLRX_MAX_IRLS + 2;

enum Buf {
  B_B, B_BM, B_X0, B_IMG, B_X, B_R, B_P, B_Q, B_T, B_S, B_ET, B_ESTAGE,
  B_TWPF, B_TWQF, B_TWPD, B_TWQD,
  B_C1, B_G, B_RM, B_LAM, B_EWORK, B_VT, B_HRE, B_HIM, B_WSUM, B_S1,
  B_PARTA, B_PARTB, B_RRH, B_SCAL, B_STATS, B_INFO, B_FLAG,
  B_AW, B_UZ, B_TAU, B_TRIV, B_TRIP, B_BTS, B_DCTREE, B_DCWSI, B_DCWSD,
  kNumBuf
};

slrx_status fail(slrx_status st, const char* fmt, ...);
// Every device allocation of the library (fault injection for tests: slrx_fault_alloc).
hipError_t dev_malloc(void** p, size_t bytes);
// What a captured CG graph depends on beyond the plan's fixed buffers.
struct CgGraphKey {
  int P, Q, T, M, n_cg, circ, ncoils, pad;
  double lambda;
  void* coil_mem;
};
// Binds the failures of the calling thread to a plan while in scope (the plan's
// last error; the thread's last error is always set as well).
struct PlanScope {
  slrx_plan* prev;
  explicit PlanScope(slrx_plan* p);
  ~PlanScope();
};
// rocSOLVER handle and workspace of the library eigensolver (created once per plan).
slrx_status setup_libeigh(slrx_plan* pl);


}  // namespace slrx

struct slrx_plan {
  slrx_dims cap{};   // dims the buffers were sized for
  slrx_dims d{};     // current dims (filter may be smaller than cap)
  slrx_params prm{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  void* arena = nullptr;
  size_t arena_bytes = 0;
  float2 *b = nullptr, *bm = nullptr, *x0 = nullptr, *img = nullptr, *x = nullptr;
  float2 *r = nullptr, *p = nullptr, *q = nullptr, *t = nullptr;
  uint8_t* S = nullptr;
  float2* Et = nullptr;      // penalty masks, transposed planes [W][Q][P]
  float2* Estage = nullptr;  // masks in the ABI layout [W][P][Q]
  float2 *twPf = nullptr, *twQf = nullptr;
  double2 *twPd = nullptr, *twQd = nullptr;
  double2 *c1 = nullptr, *g = nullptr, *Rm = nullptr;
  double *lam = nullptr, *ework = nullptr, *VT = nullptr, *Hre = nullptr, *Him = nullptr;
  double2 *wsum = nullptr, *s1 = nullptr;
  double2 *Aw = nullptr, *UZ = nullptr, *tau = nullptr, *triv = nullptr, *trip = nullptr;
  double2* bts = nullptr;  // back-transformation scratch
  int* dc_tree = nullptr;  // divide-and-conquer tree (4 ints per internal node)
  int* dc_wsi = nullptr;
  double* dc_wsd = nullptr;
  int dc_tree_n = 0;       // size the tree was built for
  std::vector<int> dc_level_start, dc_node_sizes;
  double *partA = nullptr, *partB = nullptr, *rr_hist = nullptr, *scal = nullptr, *stats = nullptr;
  rocblas_int* info = nullptr;
  int* flag = nullptr;

  // multichannel data (slrx_set_coils): one allocation holding the coil maps
  // (transposed per coil), the coil k-space, the per-coil volumes of the
  // operator's forward half (complex64) and adjoint half (complex128), the
  // image rho_u and the coil combination's group sums (complex128)
  int ncoils = 0, ncoils_cap = 0;
  void* coil_mem = nullptr;
  float2 *Ct = nullptr, *Bc = nullptr, *Yc = nullptr, *rho = nullptr;
  double2 *Yc64 = nullptr, *dco = nullptr;

  // IRLS-direct (SLRX_FLAG_DIRECT): one allocation, made at the first direct run,
  // holding the lifted matrix of the iterate (complex128, for the Gram matrix), the
  // lifted matrix of the CG direction and its product with H (complex64), and H
  // (complex64); its own rocBLAS handle for the two plain GEMMs
  void* direct_mem = nullptr;
  size_t direct_bytes = 0;
  double2* X64 = nullptr;
  float2 *Xv = nullptr, *Yd = nullptr, *Hf = nullptr;
  rocblas_handle dblas = nullptr;

  // rocSOLVER handle and workspace of the library eigensolver, a test reference
  // selected by SLRX_FLAG_LIBEIGH; created at its first use
  rocblas_handle blas = nullptr;
  void* blas_ws = nullptr;
  size_t blas_ws_size = 0;
  std::string last_error;  // message of this plan's last failed call

  // the CG body of run_cg captured as a graph, and what it was captured for
  hipStream_t cap_stream = nullptr;
  hipGraph_t cg_graph = nullptr;
  hipGraphExec_t cg_exec = nullptr;
  slrx::CgGraphKey cg_key{};

  hipEvent_t ev_run[2] = {nullptr, nullptr};
  hipEvent_t ev_step = nullptr;  // ordering against a shared batched eigen-decomposition
  hipEvent_t ev_begin = nullptr; // start of a lock-step engine step (timing of the CG strategy)
  int it_next = 0;               // next outer iteration (lock-step engine)
  hipEvent_t ev_iter[2] = {nullptr, nullptr};  // end of the last two engine steps (server pacing)
  std::vector<hipEvent_t> ev_phase;
  // per-kernel-class launch timing (SLRX_FLAG_KTIME): event pairs, reused across runs
  std::vector<hipEvent_t> kev[SLRX_K_NCLASS];
  int kused[SLRX_K_NCLASS] = {};
  bool ktime = false;

  bool has_b = false, has_S = false, has_init = false;
  bool prepared = false, running = false, ran = false;
  int run_irls = 0;
  bool run_timing = false;

  size_t vol() const { return (size_t)d.T * d.P * d.Q; }
  int s() const { return d.N1 * d.N2 * d.M; }
  // the library eigensolver (test reference) instead of the own chain
  bool lib_eigh() const;
  // the pixel-wise prior (HLR-Voxel) instead of the multi-fold Toeplitz lifting
  bool voxel() const { return (prm.flags & SLRX_FLAG_HLR_VOXEL) != 0; }
  // IRLS-direct: the explicit linear lifting instead of the FFT-based approximations
  bool direct() const { return (prm.flags & SLRX_FLAG_DIRECT) != 0; }
};

namespace slrx {
// Records an event pair around the launches made during its lifetime.
struct KTimer {
  slrx_plan* pl;
  int cls;
  int idx = -1;
  KTimer(slrx_plan* p, int c);
  ~KTimer();
};
slrx_status fft2(slrx_plan* pl, const float2* src, float2* dst, int sign, const uint8_t* mask);
slrx_status prepare(slrx_plan* pl);
slrx_status images(slrx_plan* pl);
slrx_status penalty_pass(slrx_plan* pl);
slrx_status load_masks(slrx_plan* pl, const float2* E_dev);
slrx_status store_masks(slrx_plan* pl);
slrx_status step_gram(slrx_plan* pl, bool colmajor = false, double2* R_out = nullptr);
slrx_status step_eigh(slrx_plan* pl, int it);
// Device buffers of the own eigen-decomposition chain for nb problems of equal
// size n (problem b at the given strides; D, E, tau, triv, trip at stride n).
struct EighBufs {
  int n = 0, nb = 1;
  double2 *A = nullptr, *V = nullptr, *Z = nullptr, *tau = nullptr, *bts = nullptr;
  double2* triv[2] = {nullptr, nullptr};
  double2* trip[2] = {nullptr, nullptr};
  double *D = nullptr, *E = nullptr, *Q = nullptr, *Qs = nullptr, *U = nullptr, *wsd = nullptr;
  int* wsi = nullptr;
  const int* tree = nullptr;
  const std::vector<int>* level_start = nullptr;
  const std::vector<int>* node_sizes = nullptr;
  long sA = 0, sZ = 0, sQ = 0, s_wsi = 0, s_wsd = 0, s_bts = 0;
};
EighBufs plan_eigh_bufs(slrx_plan* pl);
hipError_t eigh_tri(const EighBufs& e, hipStream_t s);     // Gram in A (row-major) -> D, E, tau, V
hipError_t eigh_tdeig(const EighBufs& e, hipStream_t s);   // D, E -> eigenvalues D, vectors Z
hipError_t eigh_backtr(const EighBufs& e, hipStream_t s);  // Z <- Q Z (A used as workspace)
slrx_status dc_prepare(slrx_plan* pl);
slrx_status step_weights(slrx_plan* pl, int it, bool first, double gamma, const double2* U = nullptr,
                         const double* lamv = nullptr, bool want_H = false);
// Weight update of the pixel-wise prior (SLRX_FLAG_HLR_VOXEL), in place of
// step_gram, step_eigh and step_weights.
slrx_status step_voxel(slrx_plan* pl, int it, bool first, double gamma);
// IRLS-direct (SLRX_FLAG_DIRECT): the Gram matrix of the explicit lifting into Aw,
// H from the eigenpairs, and the CG on the explicit operator.
slrx_status direct_setup(slrx_plan* pl);
slrx_status step_direct_gram(slrx_plan* pl);
slrx_status step_direct_weights(slrx_plan* pl, int it, bool first, double gamma);
slrx_status run_cg_direct(slrx_plan* pl, int n_cg, int it);
slrx_status apply_op(slrx_plan* pl, const float2* v, float2* out, bool init, double* part);
slrx_status coil_pass(slrx_plan* pl);
// graph: replay the CG body from a captured graph where allowed (plans run
// alone); the lock-step engine launches one by one (graph launches on its many
// concurrent streams measured slower than the launches themselves)
slrx_status run_cg(slrx_plan* pl, int n_cg, int it, bool graph = true);
void cg_graph_reset(slrx_plan* pl);
slrx_status enqueue_run(slrx_plan* pl);
slrx_status finish(slrx_plan* pl);
}  // namespace slrx
