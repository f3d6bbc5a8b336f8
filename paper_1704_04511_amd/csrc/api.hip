// libslrx C ABI: plans, the IRLS loop of Algorithm 1 on one GPU, single-step
// entry points, batch execution.  Host orchestration only; every arithmetic
// step runs in the kernels of k_op.hip / k_gram.hip (and rocSOLVER's FP64
// Hermitian eigensolver).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <new>
#include <thread>
#include <string>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "plan.h"
#include "../../include/slrx.h"

using namespace slrx;

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;
static thread_local slrx_plan* g_cur_plan = nullptr;

slrx::PlanScope::PlanScope(slrx_plan* p) : prev(g_cur_plan) { g_cur_plan = p; }
slrx::PlanScope::~PlanScope() { g_cur_plan = prev; }

slrx_status slrx::fail(slrx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (g_cur_plan) g_cur_plan->last_error = buf;
  static const bool log = std::getenv("SLRX_LOG") != nullptr;  // every failure to stderr
  if (log) std::fprintf(stderr, "[slrx] %s: %s\n", slrx_status_str(st), buf);
  return st;
}

// ------------------------------------------------------------ allocation
// Every device allocation of the library goes through dev_malloc.  Fault
// injection for tests: SLRX_FAULT_ALLOC=n (read at the first allocation) or
// slrx_fault_alloc(n) makes the n-th allocation from then on (0 = the next one)
// fail as if the device were out of memory, without allocating.
static std::mutex g_alloc_mu;
static long g_alloc_fault = -2;  // -2: environment not read yet; -1: off

hipError_t slrx::dev_malloc(void** p, size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (g_alloc_fault == -2) {
      const char* e = std::getenv("SLRX_FAULT_ALLOC");
      g_alloc_fault = e ? std::atol(e) : -1;
    }
    if (g_alloc_fault >= 0 && g_alloc_fault-- == 0) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(p, bytes);
}

extern "C" void slrx_fault_alloc(int32_t n) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc_fault = n < 0 ? -1 : n;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(SLRX_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                                \
  } while (0)

#define STCHK(expr)                     \
  do {                                  \
    slrx_status _s = (expr);            \
    if (_s != SLRX_OK) return _s;       \
  } while (0)

slrx::KTimer::KTimer(slrx_plan* p, int c) : pl(p), cls(c) {
  if (!pl->ktime) return;
  const uint32_t mask = pl->prm.flags >> 16;
  if (mask != 0 && !((mask >> cls) & 1u)) return;
  auto& v = pl->kev[cls];
  const int i = pl->kused[cls];
  while ((int)v.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    v.push_back(e);
  }
  if (hipEventRecord(v[2 * i], pl->stream) != hipSuccess) return;
  idx = i;
  pl->kused[cls] = i + 1;
}

slrx::KTimer::~KTimer() {
  if (idx >= 0) (void)hipEventRecord(pl->kev[cls][2 * idx + 1], pl->stream);
}

bool slrx_plan::lib_eigh() const { return (prm.flags & SLRX_FLAG_LIBEIGH) != 0; }

extern "C" const char* slrx_status_str(slrx_status s) {
  switch (s) {
    case SLRX_OK: return "ok";
    case SLRX_EINVAL: return "invalid argument";
    case SLRX_ENOMEM: return "out of device memory";
    case SLRX_EDEVICE: return "device error";
    case SLRX_ESTATE: return "invalid state";
    case SLRX_ENUMERIC: return "numerical failure";
    case SLRX_EBUSY: return "busy";
    case SLRX_ENOTREADY: return "not ready";
    case SLRX_ECANCELED: return "canceled";
    case SLRX_ETIMEDOUT: return "timed out";
  }
  return "unknown status";
}

extern "C" const char* slrx_last_error(const slrx_plan* pl) {
  return pl ? pl->last_error.c_str() : g_last_error.c_str();
}

extern "C" void slrx_default_params(slrx_params* out) {
  if (!out) return;
  out->lambda = 1e-3;
  out->p = 0.6;
  out->gamma = 1.4;
  out->eps0_frac = 0.01;
  out->n_irls = 15;
  out->n_cg = 10;
  out->flags = 0;
}

// -------------------------------------------------------------- validation
static slrx_status validate_dims(const slrx_dims* d) {
  if (!d) return fail(SLRX_EINVAL, "dims is NULL");
  if (!fft_len_supported(d->P) || !fft_len_supported(d->Q))
    return fail(SLRX_EINVAL, "unsupported frame size %dx%d (supported: 8,16,32,64,96,128,160,192,256)", d->P, d->Q);
  if (d->T < 1 || d->T > max_frames()) return fail(SLRX_EINVAL, "T=%d out of range [1,%d]", d->T, max_frames());
  if (d->M < 1 || d->M > d->T || d->M > max_taps())
    return fail(SLRX_EINVAL, "M=%d out of range [1,min(T,%d)]", d->M, max_taps());
  if (d->N1 < 1 || d->N1 > d->P || d->N2 < 1 || d->N2 > d->Q)
    return fail(SLRX_EINVAL, "filter %dx%d does not fit the %dx%d frame", d->N1, d->N2, d->P, d->Q);
  const long s = (long)d->N1 * d->N2 * d->M;
  if (s > kMaxS) return fail(SLRX_EINVAL, "filter size s=%ld exceeds %d", s, kMaxS);
  return SLRX_OK;
}

static slrx_status validate_params(const slrx_params* p) {
  if (!p) return fail(SLRX_EINVAL, "params is NULL");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return fail(SLRX_EINVAL, "lambda must be finite and >= 0");
  if (!(p->p >= 0.0 && p->p <= 1.0)) return fail(SLRX_EINVAL, "p must be in [0,1]");
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return fail(SLRX_EINVAL, "gamma must be finite and > 1");
  if (!(p->eps0_frac > 0.0) || !std::isfinite(p->eps0_frac)) return fail(SLRX_EINVAL, "eps0_frac must be finite and > 0");
  if (p->n_irls < 1 || p->n_irls > SLRX_MAX_IRLS) return fail(SLRX_EINVAL, "n_irls must be in [1,%d]", SLRX_MAX_IRLS);
  if (p->n_cg < 0 || p->n_cg > kMaxCg) return fail(SLRX_EINVAL, "n_cg must be in [0,%d]", kMaxCg);
  return SLRX_OK;
}

// Flags that constrain the dims or each other.
static slrx_status validate_combo(const slrx_dims& d, const slrx_params& p) {
  if (p.flags & SLRX_FLAG_DIRECT) {
    if (p.flags & (SLRX_FLAG_GIRAF | SLRX_FLAG_HLR_VOXEL | SLRX_FLAG_LIBEIGH))
      return fail(SLRX_EINVAL,
                  "SLRX_FLAG_DIRECT does not combine with SLRX_FLAG_GIRAF, SLRX_FLAG_HLR_VOXEL or SLRX_FLAG_LIBEIGH");
  }
  if (p.flags & SLRX_FLAG_HLR_VOXEL) {
    if (d.N1 != 1 || d.N2 != 1)
      return fail(SLRX_EINVAL, "SLRX_FLAG_HLR_VOXEL needs N1 = N2 = 1 (got %dx%d)", d.N1, d.N2);
    if (p.flags & (SLRX_FLAG_GIRAF | SLRX_FLAG_LIBEIGH))
      return fail(SLRX_EINVAL, "SLRX_FLAG_HLR_VOXEL does not combine with SLRX_FLAG_GIRAF or SLRX_FLAG_LIBEIGH");
  }
  return SLRX_OK;
}

extern "C" slrx_status slrx_validate(const slrx_dims* dims, const slrx_params* params) {
  STCHK(validate_dims(dims));
  if (params) {
    STCHK(validate_params(params));
    STCHK(validate_combo(*dims, *params));
  }
  return SLRX_OK;
}

// ------------------------------------------------------------- footprint
static size_t align_up(size_t n) { return (n + 255) & ~(size_t)255; }

// Buffer layout of one plan; used both for the footprint and for allocation.
struct Layout {
  size_t off[kNumBuf];
  size_t total;
};

static Layout plan_layout(const slrx_dims& d) {
  const size_t V = (size_t)d.T * d.P * d.Q;
  const size_t s = (size_t)d.N1 * d.N2 * d.M;
  const size_t W = (size_t)d.M * (d.M + 1) / 2;
  const size_t L1 = 2 * d.N1 - 1, L2 = 2 * d.N2 - 1;
  size_t sz[kNumBuf] = {};
  sz[B_B] = V * 8;
  sz[B_BM] = V * 8;
  sz[B_X0] = V * 8;
  sz[B_IMG] = V * 8;
  sz[B_X] = V * 8;
  sz[B_R] = V * 8;
  sz[B_P] = V * 8;
  sz[B_Q] = V * 8;
  sz[B_T] = V * 8;
  sz[B_S] = V;
  sz[B_ET] = W * d.P * d.Q * 8;
  sz[B_ESTAGE] = W * d.P * d.Q * 8;
  sz[B_TWPF] = d.P * 8;
  sz[B_TWQF] = d.Q * 8;
  sz[B_TWPD] = d.P * 16;
  sz[B_TWQD] = d.Q * 16;
  sz[B_C1] = W * d.P * L2 * 16;
  sz[B_G] = W * L1 * L2 * 16;
  sz[B_RM] = s * s * 16;
  sz[B_LAM] = s * 8;
  sz[B_EWORK] = s * 8;
  sz[B_VT] = 2 * s * s * 8;
  sz[B_HRE] = s * s * 8;
  sz[B_HIM] = s * s * 8;
  sz[B_WSUM] = W * L1 * L2 * 16;
  sz[B_S1] = W * L1 * d.Q * 16;
  sz[B_PARTA] = 4096 * 8;
  sz[B_PARTB] = 4096 * 8;
  sz[B_RRH] = (kMaxCg + 2) * 8;
  sz[B_SCAL] = 64 * 8;
  sz[B_STATS] = 3 * SLRX_MAX_IRLS * 8;
  sz[B_INFO] = (kInfoEntries) * 4;
  sz[B_FLAG] = 64;
  sz[B_AW] = s * s * 16;
  sz[B_UZ] = s * s * 16;
  sz[B_TAU] = s * 16;
  sz[B_TRIV] = 2 * s * 16;
  sz[B_TRIP] = 2 * s * 16;
  sz[B_BTS] = bt_scratch_elems(s) * 16;
  sz[B_DCTREE] = (size_t)4 * s * sizeof(int);
  sz[B_DCWSI] = dc_ws_ints(s) * sizeof(int);
  sz[B_DCWSD] = dc_ws_doubles(s) * sizeof(double);
  Layout L;
  size_t o = 0;
  for (int i = 0; i < kNumBuf; ++i) {
    L.off[i] = o;
    o += align_up(sz[i]);
  }
  L.total = o;
  return L;
}

extern "C" size_t slrx_footprint(const slrx_dims* dims) {
  if (validate_dims(dims) != SLRX_OK) return 0;
  return plan_layout(*dims).total;
}

// ------------------------------------------------------------ plan create
static slrx_status make_twiddles(slrx_plan* pl) {
  const int P = pl->cap.P, Q = pl->cap.Q;
  std::vector<float2> fp(P), fq(Q);
  std::vector<double2> dp(P), dq(Q);
  const double two_pi = 6.283185307179586476925286766559;
  for (int t = 0; t < P; ++t) {
    const double a = -two_pi * (double)t / (double)P;
    dp[t] = make_double2(std::cos(a), std::sin(a));
    fp[t] = make_float2((float)dp[t].x, (float)dp[t].y);
  }
  for (int t = 0; t < Q; ++t) {
    const double a = -two_pi * (double)t / (double)Q;
    dq[t] = make_double2(std::cos(a), std::sin(a));
    fq[t] = make_float2((float)dq[t].x, (float)dq[t].y);
  }
  HIPCHK(hipMemcpy(pl->twPf, fp.data(), P * sizeof(float2), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->twQf, fq.data(), Q * sizeof(float2), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->twPd, dp.data(), P * sizeof(double2), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->twQd, dq.data(), Q * sizeof(double2), hipMemcpyHostToDevice));
  return SLRX_OK;
}

slrx_status slrx::setup_libeigh(slrx_plan* pl) {
  if (pl->blas) return SLRX_OK;
  if (rocblas_create_handle(&pl->blas) != rocblas_status_success)
    return fail(SLRX_EDEVICE, "rocblas_create_handle failed");
  if (rocblas_set_stream(pl->blas, pl->stream) != rocblas_status_success)
    return fail(SLRX_EDEVICE, "rocblas_set_stream failed");
  const int s = pl->cap.N1 * pl->cap.N2 * pl->cap.M;
  size_t ws = 0;
  rocblas_start_device_memory_size_query(pl->blas);
  // sizes for every s up to the capacity are bounded by the capacity's
  rocsolver_zheevd(pl->blas, rocblas_evect_original, rocblas_fill_lower, s,
                   (rocblas_double_complex*)pl->Rm, s, pl->lam, pl->ework, pl->info);
  rocblas_stop_device_memory_size_query(pl->blas, &ws);
  if (ws < 1024) ws = 1024;
  if (dev_malloc(&pl->blas_ws, ws) != hipSuccess) return fail(SLRX_ENOMEM, "eigensolver workspace (%zu bytes)", ws);
  pl->blas_ws_size = ws;
  if (rocblas_set_workspace(pl->blas, pl->blas_ws, ws) != rocblas_status_success)
    return fail(SLRX_EDEVICE, "rocblas_set_workspace failed");
  return SLRX_OK;
}

static void assign_buffers(slrx_plan* pl, const Layout& L) {
  char* b = (char*)pl->arena;
  auto at = [&](int i) { return (void*)(b + L.off[i]); };
  pl->b = (float2*)at(B_B);
  pl->bm = (float2*)at(B_BM);
  pl->x0 = (float2*)at(B_X0);
  pl->img = (float2*)at(B_IMG);
  pl->x = (float2*)at(B_X);
  pl->r = (float2*)at(B_R);
  pl->p = (float2*)at(B_P);
  pl->q = (float2*)at(B_Q);
  pl->t = (float2*)at(B_T);
  pl->S = (uint8_t*)at(B_S);
  pl->Et = (float2*)at(B_ET);
  pl->Estage = (float2*)at(B_ESTAGE);
  pl->twPf = (float2*)at(B_TWPF);
  pl->twQf = (float2*)at(B_TWQF);
  pl->twPd = (double2*)at(B_TWPD);
  pl->twQd = (double2*)at(B_TWQD);
  pl->c1 = (double2*)at(B_C1);
  pl->g = (double2*)at(B_G);
  pl->Rm = (double2*)at(B_RM);
  pl->lam = (double*)at(B_LAM);
  pl->ework = (double*)at(B_EWORK);
  pl->VT = (double*)at(B_VT);
  pl->Hre = (double*)at(B_HRE);
  pl->Him = (double*)at(B_HIM);
  pl->wsum = (double2*)at(B_WSUM);
  pl->s1 = (double2*)at(B_S1);
  pl->partA = (double*)at(B_PARTA);
  pl->partB = (double*)at(B_PARTB);
  pl->rr_hist = (double*)at(B_RRH);
  pl->scal = (double*)at(B_SCAL);
  pl->stats = (double*)at(B_STATS);
  pl->info = (rocblas_int*)at(B_INFO);
  pl->flag = (int*)at(B_FLAG);
  pl->Aw = (double2*)at(B_AW);
  pl->UZ = (double2*)at(B_UZ);
  pl->tau = (double2*)at(B_TAU);
  pl->triv = (double2*)at(B_TRIV);
  pl->trip = (double2*)at(B_TRIP);
  pl->bts = (double2*)at(B_BTS);
  pl->dc_tree = (int*)at(B_DCTREE);
  pl->dc_wsi = (int*)at(B_DCWSI);
  pl->dc_wsd = (double*)at(B_DCWSD);
}

extern "C" slrx_status slrx_plan_create(const slrx_dims* dims, const slrx_params* params, void* hip_stream,
                                        slrx_plan** out) {
  if (!out) return fail(SLRX_EINVAL, "out is NULL");
  *out = nullptr;
  STCHK(validate_dims(dims));
  slrx_params prm;
  if (params) {
    STCHK(validate_params(params));
    STCHK(validate_combo(*dims, *params));
    prm = *params;
  } else {
    slrx_default_params(&prm);
  }
  slrx_plan* pl = new (std::nothrow) slrx_plan();
  if (!pl) return fail(SLRX_ENOMEM, "host allocation failed");
  pl->cap = *dims;
  pl->d = *dims;
  pl->prm = prm;
  HIPCHK(hipGetDevice(&pl->device));
  if (hip_stream) {
    pl->stream = (hipStream_t)hip_stream;
    pl->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking) != hipSuccess) {
      delete pl;
      return fail(SLRX_EDEVICE, "hipStreamCreate failed");
    }
    pl->own_stream = true;
  }
  const Layout L = plan_layout(*dims);
  if (dev_malloc(&pl->arena, L.total) != hipSuccess) {
    (void)hipGetLastError();
    slrx_plan_destroy(pl);
    return fail(SLRX_ENOMEM, "device allocation of %zu bytes failed", L.total);
  }
  pl->arena_bytes = L.total;
  assign_buffers(pl, L);
  slrx_status st = SLRX_OK;
  if (hipMemset(pl->arena, 0, L.total) != hipSuccess) st = fail(SLRX_EDEVICE, "hipMemset failed");
  if (st == SLRX_OK) st = make_twiddles(pl);
  if (st == SLRX_OK) st = dc_prepare(pl);
  if (st == SLRX_OK) {
    for (int i = 0; i < 2; ++i)
      if (hipEventCreate(&pl->ev_run[i]) != hipSuccess) st = fail(SLRX_EDEVICE, "hipEventCreate failed");
    if (hipEventCreateWithFlags(&pl->ev_step, hipEventDisableTiming) != hipSuccess)
      st = fail(SLRX_EDEVICE, "hipEventCreate failed");
    if (hipEventCreateWithFlags(&pl->ev_begin, hipEventDisableTiming) != hipSuccess)
      st = fail(SLRX_EDEVICE, "hipEventCreate failed");
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&pl->ev_iter[i], hipEventDisableTiming) != hipSuccess)
        st = fail(SLRX_EDEVICE, "hipEventCreate failed");
  }
  if (st != SLRX_OK) {
    slrx_plan_destroy(pl);
    return st;
  }
  *out = pl;
  return SLRX_OK;
}

extern "C" void slrx_plan_destroy(slrx_plan* pl) {
  if (!pl) return;
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  for (auto& e : pl->ev_phase) (void)hipEventDestroy(e);
  for (auto& v : pl->kev)
    for (auto& e : v) (void)hipEventDestroy(e);
  for (int i = 0; i < 2; ++i)
    if (pl->ev_run[i]) (void)hipEventDestroy(pl->ev_run[i]);
  if (pl->ev_step) (void)hipEventDestroy(pl->ev_step);
  if (pl->ev_begin) (void)hipEventDestroy(pl->ev_begin);
  for (int i = 0; i < 2; ++i)
    if (pl->ev_iter[i]) (void)hipEventDestroy(pl->ev_iter[i]);
  cg_graph_reset(pl);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  if (pl->dblas) rocblas_destroy_handle(pl->dblas);
  if (pl->direct_mem) (void)hipFree(pl->direct_mem);
  if (pl->blas) rocblas_destroy_handle(pl->blas);
  if (pl->blas_ws) (void)hipFree(pl->blas_ws);
  if (pl->coil_mem) (void)hipFree(pl->coil_mem);
  if (pl->arena) (void)hipFree(pl->arena);
  if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
  delete pl;
}

// ------------------------------------------------------------- host copies
static slrx_status copy_in(slrx_plan* pl, void* dst, const void* src, size_t bytes, slrx_mem mem) {
  if (!src) return fail(SLRX_EINVAL, "input pointer is NULL");
  if (mem == SLRX_MEM_HOST) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
  } else if (mem == SLRX_MEM_DEVICE) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, pl->stream));
  } else {
    return fail(SLRX_EINVAL, "bad memory kind %d", (int)mem);
  }
  return SLRX_OK;
}

static slrx_status copy_out(slrx_plan* pl, void* dst, const void* src, size_t bytes, slrx_mem mem) {
  if (!dst) return fail(SLRX_EINVAL, "output pointer is NULL");
  if (mem == SLRX_MEM_HOST) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
  } else if (mem == SLRX_MEM_DEVICE) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, pl->stream));
  } else {
    return fail(SLRX_EINVAL, "bad memory kind %d", (int)mem);
  }
  return SLRX_OK;
}

static slrx_status check_idle(slrx_plan* pl) {
  if (!pl) return fail(SLRX_EINVAL, "plan is NULL");
  if (pl->running) {
    const hipError_t q = hipEventQuery(pl->ev_run[1]);
    if (q == hipErrorNotReady) return fail(SLRX_EBUSY, "plan is running");
  }
  return SLRX_OK;
}

extern "C" slrx_status slrx_set_kspace(slrx_plan* pl, const void* b, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  STCHK(copy_in(pl, pl->b, b, pl->vol() * sizeof(float2), mem));
  pl->has_b = true;
  pl->prepared = false;
  return SLRX_OK;
}

extern "C" slrx_status slrx_set_coils(slrx_plan* pl, int32_t ncoils, const void* C, const void* b, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  if (ncoils < 0 || ncoils > SLRX_MAX_COILS)
    return fail(SLRX_EINVAL, "ncoils=%d out of range [0,%d]", (int)ncoils, SLRX_MAX_COILS);
  if (mem != SLRX_MEM_HOST && mem != SLRX_MEM_DEVICE) return fail(SLRX_EINVAL, "bad memory kind %d", (int)mem);
  if (ncoils > 0 && (!C || !b)) return fail(SLRX_EINVAL, "coil maps or coil data pointer is NULL");
  if (ncoils > 0 && pl->direct()) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT is single-channel only");
  const slrx_dims& d = pl->d;
  const size_t V = pl->vol(), pq = (size_t)d.P * d.Q;
  if (ncoils != pl->ncoils_cap) {
    HIPCHK(hipStreamSynchronize(pl->stream));
    if (pl->coil_mem) HIPCHK(hipFree(pl->coil_mem));
    pl->coil_mem = nullptr;
    pl->ncoils_cap = 0;
    pl->Ct = pl->Bc = pl->Yc = pl->rho = nullptr;
    pl->Yc64 = pl->dco = nullptr;
    if (ncoils > 0) {
      // complex64 units: maps, coil k-space, forward-half volumes, image; then
      // complex128: adjoint-half volumes, group sums
      const size_t n32 = (size_t)ncoils * pq + 2 * (size_t)ncoils * V + V;
      const size_t n64 = (size_t)ncoils * V + (size_t)coil_groups(ncoils) * V;
      const size_t cb = n32 * sizeof(float2) + n64 * sizeof(double2);
      if (dev_malloc(&pl->coil_mem, cb) != hipSuccess) {
        (void)hipGetLastError();
        pl->coil_mem = nullptr;
        pl->ncoils = 0;  // the plan is left without coil data
        pl->prepared = false;
        return fail(SLRX_ENOMEM, "coil buffers (%zu bytes)", cb);
      }
      pl->ncoils_cap = ncoils;
      pl->Ct = (float2*)pl->coil_mem;
      pl->Bc = pl->Ct + (size_t)ncoils * pq;
      pl->Yc = pl->Bc + (size_t)ncoils * V;
      pl->rho = pl->Yc + (size_t)ncoils * V;
      pl->Yc64 = (double2*)(pl->rho + V);
      pl->dco = pl->Yc64 + (size_t)ncoils * V;
    }
  }
  pl->ncoils = 0;
  pl->prepared = false;
  if (ncoils == 0) return SLRX_OK;
  // maps [j][P][Q] staged in the per-coil volumes, stored transposed [j][Q][P]
  STCHK(copy_in(pl, pl->Yc, C, (size_t)ncoils * pq * sizeof(float2), mem));
  HIPCHK(launch_transpose_planes(ncoils, d.P, d.Q, pl->Yc, pl->Ct, pl->stream));
  STCHK(copy_in(pl, pl->Bc, b, (size_t)ncoils * V * sizeof(float2), mem));
  HIPCHK(hipStreamSynchronize(pl->stream));
  pl->ncoils = ncoils;
  return SLRX_OK;
}

extern "C" slrx_status slrx_set_mask(slrx_plan* pl, const uint8_t* S, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  STCHK(copy_in(pl, pl->S, S, pl->vol(), mem));
  pl->has_S = true;
  pl->prepared = false;
  return SLRX_OK;
}

extern "C" slrx_status slrx_set_init(slrx_plan* pl, const void* x0, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  STCHK(copy_in(pl, pl->x0, x0, pl->vol() * sizeof(float2), mem));
  pl->has_init = true;
  pl->prepared = false;
  return SLRX_OK;
}

extern "C" slrx_status slrx_clear_init(slrx_plan* pl) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  pl->has_init = false;
  pl->prepared = false;
  return SLRX_OK;
}

extern "C" slrx_status slrx_set_filter(slrx_plan* pl, int32_t N1, int32_t N2, int32_t M) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  slrx_dims d = pl->d;
  d.N1 = N1;
  d.N2 = N2;
  d.M = M;
  STCHK(validate_dims(&d));
  STCHK(validate_combo(d, pl->prm));
  if (N1 > pl->cap.N1 || N2 > pl->cap.N2 || M > pl->cap.M)
    return fail(SLRX_EINVAL, "filter %dx%dx%d exceeds the plan's capacity %dx%dx%d", N1, N2, M, pl->cap.N1,
                pl->cap.N2, pl->cap.M);
  pl->d = d;
  pl->ran = false;
  return dc_prepare(pl);
}

extern "C" slrx_status slrx_set_params(slrx_plan* pl, const slrx_params* prm) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  STCHK(validate_params(prm));
  STCHK(validate_combo(pl->d, *prm));
  pl->prm = *prm;
  return SLRX_OK;
}

slrx_status slrx::enqueue_run(slrx_plan* pl) {
  if (pl->direct() && pl->ncoils > 0) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT is single-channel only");
  STCHK(prepare(pl));
  if (pl->direct()) STCHK(direct_setup(pl));
  const bool timing = (pl->prm.flags & SLRX_FLAG_TIMING) != 0;
  const int nirls = pl->prm.n_irls;
  pl->ktime = (pl->prm.flags & SLRX_FLAG_KTIME) != 0;
  for (int c = 0; c < SLRX_K_NCLASS; ++c) pl->kused[c] = 0;
  if (timing) {
    const size_t need = (size_t)nirls * 4 + 1;
    while (pl->ev_phase.size() < need) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pl->ev_phase.push_back(e);
    }
  }
  HIPCHK(hipMemsetAsync(pl->info, 0, kInfoEntries * sizeof(rocblas_int), pl->stream));
  HIPCHK(hipEventRecord(pl->ev_run[0], pl->stream));
  // roctx ranges (host side: they bracket the enqueueing of each outer iteration)
  roctxRangePushA("slrx run");
  struct PopRange {
    ~PopRange() { roctxRangePop(); }
  } pop_run;
  for (int it = 0; it < nirls; ++it) {
    roctxRangePushA("slrx outer iteration");
    PopRange pop_it;
    if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it], pl->stream));
    if (pl->direct()) {
      STCHK(step_direct_gram(pl));
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 1], pl->stream));
      STCHK(step_eigh(pl, it));
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 2], pl->stream));
      STCHK(step_direct_weights(pl, it, it == 0, pl->prm.gamma));
    } else if (pl->voxel()) {  // the whole per-pixel weight update counts as the weights phase
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 1], pl->stream));
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 2], pl->stream));
      STCHK(step_voxel(pl, it, it == 0, pl->prm.gamma));
    } else {
      STCHK(step_gram(pl));
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 1], pl->stream));
      STCHK(step_eigh(pl, it));
      if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 2], pl->stream));
      STCHK(step_weights(pl, it, it == 0, pl->prm.gamma));
    }
    if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * it + 3], pl->stream));
    STCHK(pl->direct() ? run_cg_direct(pl, pl->prm.n_cg, it) : run_cg(pl, pl->prm.n_cg, it));
  }
  if (timing) HIPCHK(hipEventRecord(pl->ev_phase[4 * nirls], pl->stream));
  HIPCHK(hipEventRecord(pl->ev_run[1], pl->stream));
  pl->running = true;
  pl->ran = false;
  pl->run_irls = nirls;
  pl->run_timing = timing;
  return SLRX_OK;
}

extern "C" slrx_status slrx_run(slrx_plan* pl) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  return enqueue_run(pl);
}

slrx_status slrx::finish(slrx_plan* pl) {
  if (!pl->running) return SLRX_OK;
  HIPCHK(hipEventSynchronize(pl->ev_run[1]));
  pl->running = false;
  pl->ran = true;
  std::vector<rocblas_int> info(kInfoEntries);
  HIPCHK(hipMemcpy(info.data(), pl->info, kInfoEntries * sizeof(rocblas_int), hipMemcpyDeviceToHost));
  if (info[kInfoNonfinite] != 0) {
    pl->ran = false;
    return fail(SLRX_ENUMERIC, "non-finite Gram matrix (non-finite data, initial guess or iterate)");
  }
  std::vector<double> st(3 * SLRX_MAX_IRLS);
  HIPCHK(hipMemcpy(st.data(), pl->stats, st.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int it = 0; it < pl->run_irls; ++it) {
    if (info[it] != 0) {
      pl->ran = false;
      return fail(SLRX_ENUMERIC, "eigen-decomposition did not converge at outer iteration %d (info %d)", it,
                  (int)info[it]);
    }
    if (!std::isfinite(st[SLRX_MAX_IRLS + it]) || !std::isfinite(st[it])) {
      pl->ran = false;
      return fail(SLRX_ENUMERIC, "non-finite Gram eigenvalues at outer iteration %d", it);
    }
  }
  return SLRX_OK;
}

extern "C" slrx_status slrx_sync(slrx_plan* pl) {
  PlanScope scope(pl);
  if (!pl) return fail(SLRX_EINVAL, "plan is NULL");
  STCHK(finish(pl));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return SLRX_OK;
}

static slrx_status require_done(slrx_plan* pl) {
  if (!pl) return fail(SLRX_EINVAL, "plan is NULL");
  if (pl->running) {
    if (hipEventQuery(pl->ev_run[1]) == hipErrorNotReady) return fail(SLRX_EBUSY, "plan is running");
    STCHK(finish(pl));
  }
  if (!pl->ran) return fail(SLRX_ENOTREADY, "no completed run");
  return SLRX_OK;
}

extern "C" slrx_status slrx_get_images(slrx_plan* pl, void* out, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(require_done(pl));
  STCHK(images(pl));
  return copy_out(pl, out, pl->img, pl->vol() * sizeof(float2), mem);
}

extern "C" slrx_status slrx_fit_t2(slrx_plan* pl, const void* img, const double* te_ms, double* t2_out,
                                   double* amp_out, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  if (!te_ms || !t2_out) return fail(SLRX_EINVAL, "echo times or output pointer is NULL");
  if (mem != SLRX_MEM_HOST && mem != SLRX_MEM_DEVICE) return fail(SLRX_EINVAL, "bad memory kind %d", (int)mem);
  const slrx_dims& d = pl->d;
  if (d.T < 2) return fail(SLRX_EINVAL, "a line fit needs at least two frames (T=%d)", d.T);
  FitArgs fa{};
  fa.npix = (long)d.P * d.Q;
  fa.T = d.T;
  double tbar = 0.0;
  for (int t = 0; t < d.T; ++t) {
    if (!std::isfinite(te_ms[t])) return fail(SLRX_EINVAL, "echo time %d is not finite", t);
    fa.te[t] = te_ms[t];
    tbar += te_ms[t];
  }
  tbar /= d.T;
  double stt = 0.0;
  for (int t = 0; t < d.T; ++t) stt += (te_ms[t] - tbar) * (te_ms[t] - tbar);
  if (!(stt > 0.0)) return fail(SLRX_EINVAL, "echo times must not all be equal");
  fa.tbar = tbar;
  fa.stt = stt;
  if (img) {
    STCHK(copy_in(pl, pl->img, img, pl->vol() * sizeof(float2), mem));
  } else {
    STCHK(require_done(pl));
    STCHK(images(pl));
  }
  // outputs staged in the CG scratch q (T >= 2 frames of complex64 hold two FP64 maps)
  double* t2d = (double*)pl->q;
  double* ampd = t2d + fa.npix;
  fa.img = pl->img;
  fa.t2 = t2d;
  fa.amp = amp_out ? ampd : nullptr;
  HIPCHK(launch_fit_t2(fa, pl->stream));
  STCHK(copy_out(pl, t2_out, t2d, (size_t)fa.npix * sizeof(double), mem));
  if (amp_out) STCHK(copy_out(pl, amp_out, ampd, (size_t)fa.npix * sizeof(double), mem));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return SLRX_OK;
}

extern "C" slrx_status slrx_get_kspace(slrx_plan* pl, void* out, slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(require_done(pl));
  return copy_out(pl, out, pl->x, pl->vol() * sizeof(float2), mem);
}

extern "C" slrx_status slrx_get_stats(slrx_plan* pl, slrx_stats* out) {
  PlanScope scope(pl);
  if (!out) return fail(SLRX_EINVAL, "out is NULL");
  STCHK(require_done(pl));
  std::memset(out, 0, sizeof *out);
  std::vector<double> st(3 * SLRX_MAX_IRLS);
  HIPCHK(hipMemcpy(st.data(), pl->stats, st.size() * sizeof(double), hipMemcpyDeviceToHost));
  out->n_irls_done = pl->run_irls;
  for (int i = 0; i < pl->run_irls; ++i) {
    out->eps[i] = st[i];
    out->lambda_max[i] = st[SLRX_MAX_IRLS + i];
    out->cg_rr_final[i] = st[2 * SLRX_MAX_IRLS + i];
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, pl->ev_run[0], pl->ev_run[1]));
  out->ms_total = ms;
  if (pl->ktime) {
    for (int c = 0; c < SLRX_K_NCLASS; ++c) {
      double tot = 0.0;
      for (int i = 0; i < pl->kused[c]; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pl->kev[c][2 * i], pl->kev[c][2 * i + 1]));
        tot += ms;
      }
      out->kt_ms[c] = tot;
      out->kt_count[c] = pl->kused[c];
    }
  }
  if (pl->run_timing) {
    for (int it = 0; it < pl->run_irls; ++it) {
      float a = 0, b = 0, c = 0, e = 0;
      HIPCHK(hipEventElapsedTime(&a, pl->ev_phase[4 * it], pl->ev_phase[4 * it + 1]));
      HIPCHK(hipEventElapsedTime(&b, pl->ev_phase[4 * it + 1], pl->ev_phase[4 * it + 2]));
      HIPCHK(hipEventElapsedTime(&c, pl->ev_phase[4 * it + 2], pl->ev_phase[4 * it + 3]));
      HIPCHK(hipEventElapsedTime(&e, pl->ev_phase[4 * it + 3], pl->ev_phase[4 * it + 4]));
      out->ms_gram += a;
      out->ms_eigh += b;
      out->ms_weights += c;
      out->ms_cg += e;
    }
  }
  return SLRX_OK;
}

// Several independent problems.  With hip_stream NULL they run in lock step
// on the engine (one outer iteration of every problem per step, one launch
// sequence of the eigen-decomposition per Gram size, every other kernel on the
// problem's own stream); the call returns once all work is enqueued.  With a
// stream the plans run one after another on it, each as slrx_run would.
static std::mutex g_batch_mu;
static BatchEig* g_batch_eig = nullptr;  // kept for the life of the process

extern "C" slrx_status slrx_run_batch(slrx_plan* const* plans, int32_t n, void* hip_stream) {
  if (!plans || n < 0) return fail(SLRX_EINVAL, "bad plan list");
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(SLRX_EINVAL, "plan %d is NULL", i);
    STCHK(check_idle(plans[i]));
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(SLRX_EINVAL, "plan %d appears twice", i);
  }
  if (hip_stream) {
    for (int i = 0; i < n; ++i) {
      slrx_plan* pl = plans[i];
      hipStream_t own = pl->stream;
      pl->stream = (hipStream_t)hip_stream;
      if (pl->blas) rocblas_set_stream(pl->blas, pl->stream);
      slrx_status st = enqueue_run(pl);
      pl->stream = own;
      if (pl->blas) rocblas_set_stream(pl->blas, own);
      if (st != SLRX_OK) return st;
    }
    return SLRX_OK;
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (!g_batch_eig) g_batch_eig = new BatchEig();
  std::vector<slrx_plan*> v(plans, plans + n);
  slrx_status st = SLRX_OK;
  size_t begun = 0;
  for (; begun < v.size() && st == SLRX_OK; ++begun) st = engine_begin(v[begun]);
  int maxit = 0;
  for (slrx_plan* pl : v) maxit = pl->prm.n_irls > maxit ? pl->prm.n_irls : maxit;
  for (int step = 0; step < maxit && st == SLRX_OK; ++step) st = engine_step(v, *g_batch_eig);
  for (size_t i = 0; i < v.size() && st == SLRX_OK; ++i) st = engine_end(v[i]);
  if (st != SLRX_OK) {  // no result: every begun plan drains its stream and is idle again
    for (size_t i = 0; i < begun; ++i) {
      (void)hipStreamSynchronize(v[i]->stream);
      v[i]->running = false;
      v[i]->ran = false;
      v[i]->prepared = false;
    }
  }
  return st;
}

// ------------------------------------------------------------ single steps
static slrx_status ensure_prepared(slrx_plan* pl) {
  STCHK(check_idle(pl));
  if (pl->running) STCHK(finish(pl));
  if (!pl->prepared) STCHK(prepare(pl));
  return SLRX_OK;
}

extern "C" slrx_status slrx_step_gram(slrx_plan* pl, void* R_out, slrx_mem mem) {
  PlanScope scope(pl);
  if (pl && pl->voxel()) return fail(SLRX_EINVAL, "SLRX_FLAG_HLR_VOXEL has no global Gram matrix");
  if (pl && pl->direct()) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT plans run whole reconstructions only");
  STCHK(ensure_prepared(pl));
  STCHK(step_gram(pl, true));
  const size_t s = (size_t)pl->d.N1 * pl->d.N2 * pl->d.M;
  STCHK(copy_out(pl, R_out, pl->Rm, s * s * 16, mem));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return SLRX_OK;
}

// slrx_step_weights of the pixel-wise prior: the masks alone.
static slrx_status step_weights_voxel(slrx_plan* pl, double eps, double* lam_out, void* H_out, void* E_out,
                                      slrx_mem mem) {
  if (lam_out || H_out)
    return fail(SLRX_EINVAL, "SLRX_FLAG_HLR_VOXEL has per-pixel weights only: lam and H outputs must be NULL");
  STCHK(ensure_prepared(pl));
  HIPCHK(hipMemsetAsync(pl->info + kInfoNonfinite, 0, sizeof(rocblas_int), pl->stream));
  HIPCHK(hipMemcpyAsync(pl->scal, &eps, sizeof(double), hipMemcpyHostToDevice, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  STCHK(step_voxel(pl, -1, false, 1.0));
  if (E_out) {
    const slrx_dims& d = pl->d;
    const size_t W = (size_t)d.M * (d.M + 1) / 2;
    STCHK(store_masks(pl));
    STCHK(copy_out(pl, E_out, pl->Estage, W * d.P * d.Q * sizeof(float2), mem));
  }
  HIPCHK(hipStreamSynchronize(pl->stream));
  int bad = 0;
  HIPCHK(hipMemcpy(&bad, pl->info + kInfoNonfinite, sizeof(int), hipMemcpyDeviceToHost));
  if (bad) return fail(SLRX_ENUMERIC, "non-finite Gram matrix (non-finite data, initial guess or iterate)");
  return SLRX_OK;
}

extern "C" slrx_status slrx_step_weights(slrx_plan* pl, double eps, double* lam_out, void* H_out, void* E_out,
                                         slrx_mem mem) {
  PlanScope scope(pl);
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(SLRX_EINVAL, "eps must be finite and > 0");
  if (pl && pl->voxel()) return step_weights_voxel(pl, eps, lam_out, H_out, E_out, mem);
  if (pl && pl->direct()) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT plans run whole reconstructions only");
  STCHK(ensure_prepared(pl));
  STCHK(step_gram(pl));
  STCHK(step_eigh(pl, -1));
  HIPCHK(hipMemcpyAsync(pl->scal, &eps, sizeof(double), hipMemcpyHostToDevice, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  STCHK(step_weights(pl, -1, false, 1.0, nullptr, nullptr, H_out != nullptr));
  const slrx_dims& d = pl->d;
  const size_t s = (size_t)d.N1 * d.N2 * d.M;
  const size_t W = (size_t)d.M * (d.M + 1) / 2;
  if (lam_out) STCHK(copy_out(pl, lam_out, pl->lam, s * 8, mem));
  if (H_out) {
    if (mem == SLRX_MEM_DEVICE) {
      HIPCHK(launch_interleave((long)(s * s), pl->Hre, pl->Him, (double2*)H_out, pl->stream));
    } else {
      std::vector<double> re(s * s), im(s * s);
      HIPCHK(hipMemcpyAsync(re.data(), pl->Hre, s * s * 8, hipMemcpyDeviceToHost, pl->stream));
      HIPCHK(hipMemcpyAsync(im.data(), pl->Him, s * s * 8, hipMemcpyDeviceToHost, pl->stream));
      HIPCHK(hipStreamSynchronize(pl->stream));
      double* h = (double*)H_out;
      for (size_t i = 0; i < s * s; ++i) {
        h[2 * i] = re[i];
        h[2 * i + 1] = im[i];
      }
    }
  }
  if (E_out) {
    STCHK(store_masks(pl));
    STCHK(copy_out(pl, E_out, pl->Estage, W * d.P * d.Q * sizeof(float2), mem));
  }
  HIPCHK(hipStreamSynchronize(pl->stream));
  int info = 0;
  HIPCHK(hipMemcpy(&info, pl->info + SLRX_MAX_IRLS, sizeof(int), hipMemcpyDeviceToHost));
  if (info != 0) return fail(SLRX_ENUMERIC, "eigen-decomposition did not converge (info %d)", info);
  return SLRX_OK;
}

extern "C" slrx_status slrx_step_tdeig(slrx_plan* pl, const double* D, const double* E, double* lam_out, void* Z_out,
                                       slrx_mem mem) {
  PlanScope scope(pl);
  STCHK(check_idle(pl));
  if (!D || (!E && pl->s() > 1) || !lam_out || !Z_out) return fail(SLRX_EINVAL, "NULL argument");
  const int s = pl->s();
  if (s > dc_max_n()) return fail(SLRX_EINVAL, "s = %d exceeds the divide-and-conquer limit %d", s, dc_max_n());
  STCHK(copy_in(pl, pl->lam, D, (size_t)s * sizeof(double), mem));
  if (s > 1) STCHK(copy_in(pl, pl->ework, E, (size_t)(s - 1) * sizeof(double), mem));
  HIPCHK(eigh_tdeig(plan_eigh_bufs(pl), pl->stream));
  STCHK(copy_out(pl, lam_out, pl->lam, (size_t)s * sizeof(double), mem));
  STCHK(copy_out(pl, Z_out, pl->UZ, (size_t)s * s * sizeof(double2), mem));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return SLRX_OK;
}

extern "C" slrx_status slrx_step_apply(slrx_plan* pl, const void* E, const void* v, void* out, slrx_mem mem) {
  PlanScope scope(pl);
  if (pl && pl->direct()) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT plans run whole reconstructions only");
  STCHK(ensure_prepared(pl));
  const slrx_dims& d = pl->d;
  const size_t W = (size_t)d.M * (d.M + 1) / 2;
  STCHK(copy_in(pl, pl->Estage, E, W * d.P * d.Q * sizeof(float2), mem));
  STCHK(load_masks(pl, pl->Estage));
  STCHK(copy_in(pl, pl->r, v, pl->vol() * sizeof(float2), mem));
  STCHK(apply_op(pl, pl->r, pl->q, false, pl->partA));
  STCHK(copy_out(pl, out, pl->q, pl->vol() * sizeof(float2), mem));
  HIPCHK(hipStreamSynchronize(pl->stream));
  return SLRX_OK;
}

extern "C" slrx_status slrx_step_cg(slrx_plan* pl, const void* E, int32_t n_cg) {
  PlanScope scope(pl);
  if (n_cg < 0 || n_cg > kMaxCg) return fail(SLRX_EINVAL, "n_cg out of range");
  if (pl && pl->direct()) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT plans run whole reconstructions only");
  STCHK(ensure_prepared(pl));
  pl->ktime = false;
  const slrx_dims& d = pl->d;
  const size_t W = (size_t)d.M * (d.M + 1) / 2;
  STCHK(copy_in(pl, pl->Estage, E, W * d.P * d.Q * sizeof(float2), SLRX_MEM_HOST));
  STCHK(load_masks(pl, pl->Estage));
  STCHK(run_cg(pl, n_cg, -1));
  HIPCHK(hipEventRecord(pl->ev_run[0], pl->stream));
  HIPCHK(hipEventRecord(pl->ev_run[1], pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  pl->ran = true;
  pl->run_irls = 0;
  pl->run_timing = false;
  return SLRX_OK;
}
