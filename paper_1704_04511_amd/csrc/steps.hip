// Device steps of the IRLS loop (host orchestration of the kernels).
//
// State per plan: x is the k-space iterate (Algorithm 1's rho-hat), bm = S o b
// the masked data (the right-hand side A^H b of eq. "eq:grad_ls"), img the
// images F^-1 x used by the Gram matrix and the output, Et the penalty masks.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>

#include "kernels.h"
#include "plan.h"
#include "tune.h"

using namespace slrx;

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

// Unitary 2-D transforms per frame: dst = F src (sign -1) or F^-1 src (+1);
// uses the plan's transposed scratch volume t.
slrx_status slrx::fft2(slrx_plan* pl, const float2* src, float2* dst, int sign, const uint8_t* mask) {
  const slrx_dims& d = pl->d;
  RowArgs ra{};
  ra.P = d.P; ra.Q = d.Q; ra.T = d.T;
  ra.mode = mask ? ROW_MASKED : ROW_PLAIN;
  ra.sign = sign;
  ra.src = src;
  ra.S = mask;
  ra.dst = pl->t;
  ra.scale = 1.0f;
  ra.tw = pl->twQf;
  HIPCHK(launch_rows(ra, pl->stream));
  ColArgs ca{};
  ca.P = d.P; ca.Q = d.Q; ca.T = d.T;
  ca.sign = sign;
  ca.src = pl->t;
  ca.dst = dst;
  ca.scale = (float)(1.0 / std::sqrt((double)d.P * d.Q));
  ca.tw = pl->twPf;
  HIPCHK(launch_cols(ca, pl->stream));
  return SLRX_OK;
}

// Right-hand side bm = S o b and the initial iterate x = S o b (zero-filled
// k-space, Algorithm 1 initialisation) or the user's x0.  With coils the
// right-hand side is A^H b = F sum_j C_j^* F^-1 (S o b_j) (Sec. II.A), the
// adjoint half of the coil data term in complex128 (k_coil.hip), rounded once.
slrx_status slrx::prepare(slrx_plan* pl) {
  if (!(pl->has_b || pl->ncoils > 0) || !pl->has_S)
    return fail(SLRX_ESTATE, "k-space (or coil data) and mask must be set before running");
  const long V = (long)pl->vol();
  if (pl->ncoils > 0) {
    const slrx_dims& d = pl->d;
    CoilArgs ca{};
    ca.P = d.P; ca.Q = d.Q; ca.T = d.T; ca.nc = pl->ncoils;
    ca.Ct = pl->Ct;
    ca.Y64 = pl->Yc64;
    ca.vstride = V;
    ca.S = pl->S;
    ca.B = pl->Bc;
    ca.d64 = pl->dco;
    ca.groups = coil_groups(pl->ncoils);
    ca.out = pl->bm;
    ca.tw64 = pl->twQd;
    HIPCHK(launch_coil_rhs_rows(ca, pl->stream));
    ca.tw64 = pl->twPd;
    ca.cscale64 = 1.0 / ((double)d.P * d.Q);
    HIPCHK(launch_coil_combine(ca, pl->stream));
    ca.tw64 = pl->twQd;
    HIPCHK(launch_coil_rhs_fin(ca, pl->stream));
  } else {
    HIPCHK(launch_mask_data(V, pl->S, pl->b, pl->bm, pl->stream));
  }
  const float2* x0 = pl->has_init ? pl->x0 : pl->bm;
  HIPCHK(hipMemcpyAsync(pl->x, x0, V * sizeof(float2), hipMemcpyDeviceToDevice, pl->stream));
  pl->prepared = true;
  return SLRX_OK;
}

slrx_status slrx::images(slrx_plan* pl) { return fft2(pl, pl->x, pl->img, +1, nullptr); }

// Gram matrix of the current iterate: row-major into Aw for the own
// tridiagonalisation, column-major into Rm for rocSOLVER zheevd (or when
// colmajor is forced, for the single-step entry point).
slrx_status slrx::step_gram(slrx_plan* pl, bool colmajor, double2* R_out) {
  const slrx_dims& d = pl->d;
  KTimer kt(pl, SLRX_K_GRAM);
  STCHK(images(pl));
  GramArgs ga{};
  ga.P = d.P; ga.Q = d.Q; ga.T = d.T; ga.N1 = d.N1; ga.N2 = d.N2; ga.M = d.M;
  ga.rho = pl->img;
  ga.c1 = pl->c1;
  ga.g = pl->g;
  const bool lib = pl->lib_eigh() || colmajor;
  ga.R = R_out ? R_out : (lib ? pl->Rm : pl->Aw);
  ga.rowmajor = lib ? 0 : 1;
  ga.twP = pl->twPd;
  ga.twQ = pl->twQd;
  ga.circ = (pl->prm.flags & SLRX_FLAG_GIRAF) ? 1 : 0;
  ga.bad = (int*)(pl->info + kInfoNonfinite);
  HIPCHK(launch_gram(ga, pl->stream));
  return SLRX_OK;
}

// Eigen-decomposition of the Gram matrix: Householder tridiagonalisation,
// divide and conquer on the real tridiagonal, blocked back-transformation
// (eigenvectors into UZ); or, as a test reference only, rocSOLVER zheevd on Rm
// (SLRX_FLAG_LIBEIGH).
// Tree of the divide-and-conquer solver for the current s (host table copied
// to the device; called while the plan is idle).
slrx_status slrx::dc_prepare(slrx_plan* pl) {
  const int s = pl->s();
  if (s > dc_max_n() || s == pl->dc_tree_n) return SLRX_OK;
  std::vector<int> nodes;
  dc_build_tree(s, nodes, pl->dc_level_start);
  pl->dc_node_sizes.resize(nodes.size() / 4);
  for (size_t q = 0; q < nodes.size() / 4; ++q) pl->dc_node_sizes[q] = nodes[4 * q + 1];
  if (!nodes.empty()) HIPCHK(hipMemcpy(pl->dc_tree, nodes.data(), nodes.size() * sizeof(int), hipMemcpyHostToDevice));
  pl->dc_tree_n = s;
  return SLRX_OK;
}

EighBufs slrx::plan_eigh_bufs(slrx_plan* pl) {
  const int s = pl->s();
  EighBufs e;
  e.n = s;
  e.nb = 1;
  e.A = pl->Aw;
  e.V = pl->Rm;
  e.Z = pl->UZ;
  e.tau = pl->tau;
  e.triv[0] = pl->triv;
  e.triv[1] = pl->triv + s;
  e.trip[0] = pl->trip;
  e.trip[1] = pl->trip + s;
  e.bts = pl->bts;
  e.D = pl->lam;
  e.E = pl->ework;
  e.Q = pl->VT;  // VT and Hre are free until the weights are formed
  e.Qs = pl->VT + (size_t)s * s;
  e.U = pl->Hre;
  e.wsd = pl->dc_wsd;
  e.wsi = pl->dc_wsi;
  e.tree = pl->dc_tree;
  e.level_start = &pl->dc_level_start;
  e.node_sizes = &pl->dc_node_sizes;
  return e;
}

hipError_t slrx::eigh_tri(const EighBufs& e, hipStream_t st) {
  TriArgs ta{};
  ta.n = e.n;
  ta.Aw = e.A;
  ta.Vst = e.V;
  ta.strideA = e.sA;
  ta.D = e.D;
  ta.E = e.E;
  ta.tau = e.tau;
  ta.vbuf[0] = e.triv[0];
  ta.vbuf[1] = e.triv[1];
  ta.pbuf[0] = e.trip[0];
  ta.pbuf[1] = e.trip[1];
  // workgroups per launch: tuned per (n, problems) on the first decompositions;
  // then the row access policy for the chosen budget
  TuneTicket tk, tk_access;
  const int cand = tune_begin(TUNE_TRI, e.n, e.nb, 0, tri_budget_candidates(e.nb), st, tk);
  bool stream = false;
  if (tune_choice(TUNE_TRI, e.n, e.nb, 0) == cand)
    stream = tune_begin(TUNE_TRI_ACCESS, e.n, e.nb, cand, 2, st, tk_access) == 1;
  const hipError_t err = launch_tridiag(ta, e.nb, st, cand, stream);
  tune_end(tk, st);
  tune_end(tk_access, st);
  return err;
}

hipError_t slrx::eigh_tdeig(const EighBufs& e, hipStream_t st) {
  TdArgs td;
  td.n = e.n;
  td.D = e.D;
  td.E = e.E;
  td.Z = e.Z;
  td.Q = e.Q;
  td.Qs = e.Qs;
  td.U = e.U;
  td.nodes = e.tree;
  td.level_start = *e.level_start;
  td.node_sizes = *e.node_sizes;
  td.ws_i = e.wsi;
  td.ws_d = e.wsd;
  td.nb = e.nb;
  td.sQ = e.sQ;
  td.sZ = e.sZ;
  td.s_wsi = e.s_wsi;
  td.s_wsd = e.s_wsd;
  return launch_tdeig(td, st);
}

hipError_t slrx::eigh_backtr(const EighBufs& e, hipStream_t st) {
  BackTrArgs bt{};
  bt.n = e.n;
  bt.V = e.V;
  bt.Y = e.A;  // free once the reduction is done
  bt.Z = e.Z;
  bt.tau = e.tau;
  bt.scratch = e.bts;
  bt.nb = e.nb;
  bt.sV = e.sA;
  bt.sY = e.sA;
  bt.sZ = e.sZ;
  bt.s_scratch = e.s_bts;
  return launch_backtransform(bt, st);
}

slrx_status slrx::step_eigh(slrx_plan* pl, int it) {
  const int s = pl->s();
  rocblas_int* info = pl->info + (it < 0 ? SLRX_MAX_IRLS : it);
  if (pl->lib_eigh()) {
    STCHK(setup_libeigh(pl));
    KTimer kt(pl, SLRX_K_TDEIG);
    rocblas_status rs = rocsolver_zheevd(pl->blas, rocblas_evect_original, rocblas_fill_lower, s,
                                         (rocblas_double_complex*)pl->Rm, s, pl->lam, pl->ework, info);
    if (rs != rocblas_status_success) return fail(SLRX_EDEVICE, "rocsolver_zheevd failed (status %d)", (int)rs);
    return SLRX_OK;
  }
  if (pl->dc_tree_n != s) return fail(SLRX_ESTATE, "divide-and-conquer tree not built for s = %d", s);
  const EighBufs e = plan_eigh_bufs(pl);
  {
    KTimer kt(pl, SLRX_K_TRI);
    HIPCHK(eigh_tri(e, pl->stream));
  }
  {
    KTimer kt(pl, SLRX_K_TDEIG);
    HIPCHK(eigh_tdeig(e, pl->stream));
  }
  {
    KTimer kt(pl, SLRX_K_BACKTR);
    HIPCHK(eigh_backtr(e, pl->stream));
  }
  return SLRX_OK;
}

// Weights and masks from the eigenpairs in lam / Rm: the lag sums of
// H = U diag(alpha) U^H from the filter spectra where the shape allows
// (spec_supported), else from H itself (filter product on MFMA, then its
// diagonal sums). want_H also forms H (in Hre / Him) on the spectral path.
slrx_status slrx::step_weights(slrx_plan* pl, int it, bool first, double gamma, const double2* U,
                               const double* lamv, bool want_H) {
  const slrx_dims& d = pl->d;
  const int s = d.N1 * d.N2 * d.M;
  WeightArgs wa{};
  wa.s = s;
  wa.lamv = lamv ? lamv : pl->lam;
  wa.U = U ? U : (pl->lib_eigh() ? pl->Rm : pl->UZ);
  wa.VT = pl->VT;
  wa.eps = pl->scal;
  wa.lam_max_out = it >= 0 ? pl->stats + SLRX_MAX_IRLS + it : nullptr;
  wa.eps_out = it >= 0 ? pl->stats + it : nullptr;
  wa.first = first ? 1 : 0;
  wa.eps0_frac = pl->prm.eps0_frac;
  wa.gamma = gamma;
  wa.p = pl->prm.p;
  const int ng = spec_supported(d.N1, d.N2, d.M) ? spec_groups(d.N1, d.N2, d.M, (size_t)s * s) : 0;
  {
    KTimer kt(pl, SLRX_K_FILTER);
    if (ng > 0) {
      HIPCHK(launch_eps(wa, pl->stream));
      SpecArgs sa{};
      sa.N1 = d.N1; sa.N2 = d.N2; sa.M = d.M; sa.s = s;
      sa.ngroups = ng;
      sa.lamv = wa.lamv;
      sa.U = wa.U;
      sa.eps = pl->scal;
      sa.p = pl->prm.p;
      sa.part = (double2*)pl->VT;  // s^2 double2, unused by this path until H is formed
      sa.C = sa.part + (size_t)ng * (d.M * (d.M + 1) / 2) * (2 * d.N1 - 1) * (2 * d.N2 - 1);
      HIPCHK(launch_spec_masks(sa, pl->wsum, pl->stream));
      if (want_H) {
        HIPCHK(launch_weights(wa, pl->stream, false));
        HIPCHK(launch_filter_product(s, pl->VT, pl->Hre, pl->Him, pl->stream));
      }
    } else {
      HIPCHK(launch_weights(wa, pl->stream));
      HIPCHK(launch_filter_product(s, pl->VT, pl->Hre, pl->Him, pl->stream));
    }
  }
  MaskArgs ma{};
  ma.P = d.P; ma.Q = d.Q; ma.N1 = d.N1; ma.N2 = d.N2; ma.M = d.M;
  ma.Hre = ng > 0 ? nullptr : pl->Hre;  // null: wsum is already the lag sums
  ma.Him = pl->Him;
  ma.wsum = pl->wsum;
  ma.s1 = pl->s1;
  ma.Et = pl->Et;
  ma.twP = pl->twPd;
  ma.twQ = pl->twQd;
  KTimer kt(pl, SLRX_K_MASKS);
  HIPCHK(launch_masks(ma, pl->stream));
  return SLRX_OK;
}

// Weight update of the pixel-wise prior (HLR-Voxel, SLRX_FLAG_HLR_VOXEL): per
// pixel the Gram matrix of its own Toeplitz lifting, its eigen-decomposition and
// the masks conj((G_r + eps I)^(p/2-1)) (k_voxel.hip).  On the first outer
// iteration a pass over the eigenvalues alone gives eps^(0) from the largest
// eigenvalue over all pixels before the masks pass; later iterations take
// eps <- eps / gamma first and record the largest eigenvalue from the masks
// pass itself.  it < 0: the single-step entry point, eps already set.
slrx_status slrx::step_voxel(slrx_plan* pl, int it, bool first, double gamma) {
  const slrx_dims& d = pl->d;
  STCHK(images(pl));
  KTimer kt(pl, SLRX_K_VOXEL);
  VoxelArgs va{};
  va.P = d.P; va.Q = d.Q; va.T = d.T; va.M = d.M;
  va.img = pl->img;
  va.part = it >= 0 ? pl->partB : nullptr;
  va.eps = pl->scal;
  va.p = pl->prm.p;
  va.Et = pl->Et;
  va.bad = (int*)(pl->info + kInfoNonfinite);
  VoxelEpsArgs ea{};
  ea.part = pl->partB;
  ea.nparts = voxel_tiles(d.P, d.Q);
  ea.eps = pl->scal;
  ea.lam_max_out = it >= 0 ? pl->stats + SLRX_MAX_IRLS + it : nullptr;
  ea.eps_out = it >= 0 ? pl->stats + it : nullptr;
  ea.eps0_frac = pl->prm.eps0_frac;
  ea.gamma = gamma;
  if (it < 0) {
    HIPCHK(launch_voxel(va, true, pl->stream));
    return SLRX_OK;
  }
  if (first) {
    HIPCHK(launch_voxel(va, false, pl->stream));
    ea.mode = 0;
    HIPCHK(launch_voxel_eps(ea, pl->stream));
    HIPCHK(launch_voxel(va, true, pl->stream));
  } else {
    ea.mode = 1;
    HIPCHK(launch_voxel_eps(ea, pl->stream));
    HIPCHK(launch_voxel(va, true, pl->stream));
    ea.mode = 2;
    HIPCHK(launch_voxel_eps(ea, pl->stream));
  }
  return SLRX_OK;
}

// IRLS-direct buffers (k_direct.hip) for the current dims: allocated at the first
// direct run and grown when a later run needs more; a rocBLAS handle of its own.
slrx_status slrx::direct_setup(slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  const DirectArgs da = direct_args(d.P, d.Q, d.T, d.N1, d.N2, d.M, 0.0);
  const size_t s = (size_t)pl->s();
  auto up = [](size_t n) { return (n + 255) & ~(size_t)255; };
  const size_t b64 = up((size_t)da.rows * s * 16), b32 = up((size_t)da.rows * s * 8), bh = up(s * s * 8);
  const size_t need = b64 + 2 * b32 + bh;
  if (need > pl->direct_bytes) {
    if (pl->direct_mem) HIPCHK(hipFree(pl->direct_mem));
    pl->direct_mem = nullptr;
    pl->direct_bytes = 0;
    if (dev_malloc(&pl->direct_mem, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SLRX_ENOMEM, "IRLS-direct buffers (%zu bytes: lifted matrices of %ld x %zu)", need, da.rows, s);
    }
    pl->direct_bytes = need;
  }
  char* m = (char*)pl->direct_mem;
  pl->X64 = (double2*)m;
  pl->Xv = (float2*)(m + b64);
  pl->Yd = (float2*)(m + b64 + b32);
  pl->Hf = (float2*)(m + b64 + 2 * b32);
  if (!pl->dblas) {
    if (rocblas_create_handle(&pl->dblas) != rocblas_status_success)
      return fail(SLRX_EDEVICE, "rocblas_create_handle failed");
  }
  if (rocblas_set_stream(pl->dblas, pl->stream) != rocblas_status_success)
    return fail(SLRX_EDEVICE, "rocblas_set_stream failed");
  return SLRX_OK;
}

// R = X^H X of the explicit linear lifting X of the iterate (complex128), row-major
// into Aw for the eigen-decomposition chain: X is stored row-major (rows x s), i.e.
// column-major s x rows, and the column-major product X_c X_c^H is R^T, whose
// column-major layout is R's row-major one.
slrx_status slrx::step_direct_gram(slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  KTimer kt(pl, SLRX_K_GRAM);
  const DirectArgs da = direct_args(d.P, d.Q, d.T, d.N1, d.N2, d.M, 0.0);
  const int s = pl->s();
  HIPCHK(launch_dlift64(da, pl->x, pl->X64, pl->stream));
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  const rocblas_status st = rocblas_zgemm(pl->dblas, rocblas_operation_none, rocblas_operation_conjugate_transpose, s,
                                          s, (rocblas_int)da.rows, &one, (const rocblas_double_complex*)pl->X64, s,
                                          (const rocblas_double_complex*)pl->X64, s, &zero,
                                          (rocblas_double_complex*)pl->Aw, s);
  if (st != rocblas_status_success) return fail(SLRX_EDEVICE, "rocblas_zgemm failed (status %d)", (int)st);
  return SLRX_OK;
}

// H = U (Lambda + eps I)^(p/2-1) U^H from the eigenpairs (the eps schedule and the
// filter product of the main method), rounded to complex64 for the CG operator.
slrx_status slrx::step_direct_weights(slrx_plan* pl, int it, bool first, double gamma) {
  const int s = pl->s();
  KTimer kt(pl, SLRX_K_FILTER);
  WeightArgs wa{};
  wa.s = s;
  wa.lamv = pl->lam;
  wa.U = pl->UZ;
  wa.VT = pl->VT;
  wa.eps = pl->scal;
  wa.lam_max_out = it >= 0 ? pl->stats + SLRX_MAX_IRLS + it : nullptr;
  wa.eps_out = it >= 0 ? pl->stats + it : nullptr;
  wa.first = first ? 1 : 0;
  wa.eps0_frac = pl->prm.eps0_frac;
  wa.gamma = gamma;
  wa.p = pl->prm.p;
  HIPCHK(launch_weights(wa, pl->stream));
  HIPCHK(launch_filter_product(s, pl->VT, pl->Hre, pl->Him, pl->stream));
  HIPCHK(launch_hf((long)s * s, pl->Hre, pl->Him, pl->Hf, pl->stream));
  return SLRX_OK;
}

// A v = S o v + lam T^*(T(v) H) on the explicit lifting; init: out = bm - A v.
static slrx_status direct_apply(slrx_plan* pl, const float2* v, float2* out, bool init, double* part) {
  const slrx_dims& d = pl->d;
  const DirectArgs da = direct_args(d.P, d.Q, d.T, d.N1, d.N2, d.M, pl->prm.lambda);
  const int s = pl->s();
  HIPCHK(launch_dlift32(da, v, pl->Xv, pl->stream));
  // row-major Y = Xv H: column-major Y^T = H^T Xv^T, and the row-major layouts of H
  // and Xv are the column-major layouts of H^T and Xv^T
  const rocblas_float_complex one(1.f, 0.f), zero(0.f, 0.f);
  const rocblas_status st = rocblas_cgemm(pl->dblas, rocblas_operation_none, rocblas_operation_none, s,
                                          (rocblas_int)da.rows, s, &one, (const rocblas_float_complex*)pl->Hf, s,
                                          (const rocblas_float_complex*)pl->Xv, s, &zero,
                                          (rocblas_float_complex*)pl->Yd, s);
  if (st != rocblas_status_success) return fail(SLRX_EDEVICE, "rocblas_cgemm failed (status %d)", (int)st);
  HIPCHK(launch_dadj(da, pl->Yd, v, pl->S, pl->bm, out, init ? 1 : 0, part, pl->flag, pl->stream));
  return SLRX_OK;
}

// n_cg CG iterations on the explicit operator, warm-started at x (the arithmetic
// of the CG of run_cg: same scalars, same stop rule).
slrx_status slrx::run_cg_direct(slrx_plan* pl, int n_cg, int it) {
  const long V = (long)pl->vol();
  const int nadj = direct_blocks(V);
  const int nupd = update_blocks(V);
  KTimer kt(pl, SLRX_K_DIRECT);
  STCHK(direct_apply(pl, pl->x, pl->r, true, pl->partA));
  for (int k = 0; k < n_cg; ++k) {
    HIPCHK(launch_dpupdate(V, pl->r, pl->p, k == 0 ? pl->partA : pl->partB, k == 0 ? nadj : nupd, pl->rr_hist, k,
                           pl->stream));
    STCHK(direct_apply(pl, pl->p, pl->q, false, pl->partA));
    UpdArgs ua{};
    ua.n = V;
    ua.x = pl->x;
    ua.r = pl->r;
    ua.p = pl->p;
    ua.q = pl->q;
    ua.partA = pl->partA;
    ua.nA = nadj;
    ua.rr_hist = pl->rr_hist;
    ua.k = k;
    ua.partB = pl->partB;
    ua.flag = pl->flag;
    HIPCHK(launch_update(ua, pl->stream));
  }
  if (it >= 0)
    HIPCHK(launch_store_sum(n_cg == 0 ? pl->partA : pl->partB, n_cg == 0 ? nadj : nupd,
                            pl->stats + 2 * SLRX_MAX_IRLS + it, pl->stream));
  return SLRX_OK;
}

// The coil passes of the multichannel operator on the row pass output t:
// rho_u, per coil the masked round trip through k-space (complex128 after the
// mask), and their combination's group sums, column-transformed (added to the
// penalty by the finishing pass).
slrx_status slrx::coil_pass(slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  CoilArgs ca{};
  ca.P = d.P; ca.Q = d.Q; ca.T = d.T; ca.nc = pl->ncoils;
  ca.t = pl->t;
  ca.rho = pl->rho;
  ca.Ct = pl->Ct;
  ca.Y = pl->Yc;
  ca.Y64 = pl->Yc64;
  ca.vstride = (long)pl->vol();
  ca.S = pl->S;
  ca.tw = pl->twPf;
  HIPCHK(launch_coil_cols(ca, pl->stream));
  ca.tw = pl->twQf;
  ca.tw64 = pl->twQd;
  HIPCHK(launch_coil_rows(ca, pl->stream));
  const double pq = (double)d.P * d.Q;
  ca.tw64 = pl->twPd;
  ca.d64 = pl->dco;
  ca.cscale64 = 1.0 / (pq * pq);
  ca.groups = coil_groups(pl->ncoils);
  HIPCHK(launch_coil_combine(ca, pl->stream));
  return SLRX_OK;
}

// The multichannel fields of the finishing pass.
static void fin_coil(slrx_plan* pl, FinArgs& fa) {
  fa.coil = pl->ncoils > 0 ? 1 : 0;
  if (!fa.coil) return;
  fa.d64 = pl->dco;
  fa.dparts = coil_groups(pl->ncoils);
  fa.dstride = (long)pl->vol();
  fa.tw64 = pl->twQd;
}

// A v = S o v + lam F G F^-1 v in k-space (init: out = bm - A v); with coils
// the data term is F sum_j C_j^* F^-1 S F C_j F^-1 v.
slrx_status slrx::apply_op(slrx_plan* pl, const float2* v, float2* out, bool init, double* part) {
  const slrx_dims& d = pl->d;
  RowArgs ra{};
  ra.P = d.P; ra.Q = d.Q; ra.T = d.T;
  ra.mode = ROW_PLAIN;
  ra.sign = +1;
  ra.src = v;
  ra.dst = pl->t;
  ra.scale = 1.0f;
  ra.tw = pl->twQf;
  HIPCHK(launch_rows(ra, pl->stream));
  if (pl->ncoils > 0) STCHK(coil_pass(pl));
  STCHK(penalty_pass(pl));
  FinArgs fa{};
  fa.P = d.P; fa.Q = d.Q; fa.T = d.T;
  fa.init = init ? 1 : 0;
  fa.t = pl->t;
  fa.v = v;
  fa.S = pl->S;
  fa.y = pl->bm;
  fa.out = out;
  fa.part = part;
  fa.flag = pl->flag;
  fa.tw = pl->twQf;
  fin_coil(pl, fa);
  HIPCHK(launch_fin(fa, pl->stream));
  return SLRX_OK;
}

slrx_status slrx::penalty_pass(slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  PenArgs pa{};
  pa.P = d.P; pa.Q = d.Q; pa.T = d.T; pa.M = d.M;
  pa.buf = pl->t;
  pa.Et = pl->Et;
  pa.scale = (float)(pl->prm.lambda / ((double)d.P * d.Q));
  pa.tw = pl->twPf;
  pa.circ = (pl->prm.flags & SLRX_FLAG_GIRAF) ? 1 : 0;
  if (pl->ncoils > 0) {
    pa.nc = pl->ncoils;
    pa.rho = pl->rho;
  }
  HIPCHK(launch_pen(pa, pl->stream));
  return SLRX_OK;
}

// n_cg iterations of CG on (S + lam F G F^-1) x = S o b (with coils:
// (A^H A + lam F G F^-1) x = A^H b), warm-started at x: the initial residual
// and the iterations, enqueued on pl->stream.
static slrx_status cg_body(slrx_plan* pl, int n_cg) {
  const slrx_dims& d = pl->d;
  const long V = (long)pl->vol();
  const int nfin = fin_blocks(d.P, d.T);
  const int nupd = update_blocks(V);
  STCHK(apply_op(pl, pl->x, pl->r, true, pl->partA));
  for (int k = 0; k < n_cg; ++k) {
    RowArgs ra{};
    ra.P = d.P; ra.Q = d.Q; ra.T = d.T;
    ra.mode = ROW_PUPDATE;
    ra.sign = +1;
    ra.src = pl->r;
    ra.pvec = pl->p;
    ra.dst = pl->t;
    ra.scale = 1.0f;
    ra.tw = pl->twQf;
    ra.k = k;
    ra.part = k == 0 ? pl->partA : pl->partB;
    ra.npart = k == 0 ? nfin : nupd;
    ra.rr_hist = pl->rr_hist;
    {
      KTimer kt(pl, SLRX_K_ROWS);
      HIPCHK(launch_rows(ra, pl->stream));
    }
    if (pl->ncoils > 0) {
      KTimer kt(pl, SLRX_K_COIL);
      STCHK(coil_pass(pl));
    }
    {
      KTimer kt(pl, SLRX_K_COLS);
      STCHK(penalty_pass(pl));
    }
    FinArgs fa{};
    fa.P = d.P; fa.Q = d.Q; fa.T = d.T;
    fa.init = 0;
    fa.t = pl->t;
    fa.v = pl->p;
    fa.S = pl->S;
    fa.y = pl->bm;
    fa.out = pl->q;
    fa.part = pl->partA;
    fa.flag = pl->flag;
    fa.tw = pl->twQf;
    fin_coil(pl, fa);
    {
      KTimer kt(pl, SLRX_K_FIN);
      HIPCHK(launch_fin(fa, pl->stream));
    }
    UpdArgs ua{};
    ua.n = V;
    ua.x = pl->x;
    ua.r = pl->r;
    ua.p = pl->p;
    ua.q = pl->q;
    ua.partA = pl->partA;
    ua.nA = nfin;
    ua.rr_hist = pl->rr_hist;
    ua.k = k;
    ua.partB = pl->partB;
    ua.flag = pl->flag;
    {
      KTimer kt(pl, SLRX_K_UPDATE);
      HIPCHK(launch_update(ua, pl->stream));
    }
  }
  return SLRX_OK;
}

// Everything the CG body's launches depend on besides the plan's fixed buffers.
static CgGraphKey cg_key(const slrx_plan* pl, int n_cg) {
  CgGraphKey k{};
  k.P = pl->d.P; k.Q = pl->d.Q; k.T = pl->d.T; k.M = pl->d.M;
  k.n_cg = n_cg;
  k.lambda = pl->prm.lambda;
  k.circ = (pl->prm.flags & SLRX_FLAG_GIRAF) ? 1 : 0;
  k.ncoils = pl->ncoils;
  k.coil_mem = pl->coil_mem;
  return k;
}

// The CG body is replayed from a captured graph unless the caller asked for
// launches one by one or times any of its kernel classes.
static bool cg_graph_allowed(const slrx_plan* pl) {
  if (pl->prm.flags & SLRX_FLAG_NO_GRAPH) return false;
  if (!pl->ktime) return true;
  const uint32_t mask = pl->prm.flags >> 16;
  const uint32_t cg = (1u << SLRX_K_ROWS) | (1u << SLRX_K_COLS) | (1u << SLRX_K_FIN) | (1u << SLRX_K_UPDATE) |
                      (1u << SLRX_K_COIL);
  return mask != 0 && (mask & cg) == 0;
}

void slrx::cg_graph_reset(slrx_plan* pl) {
  if (pl->cg_exec) (void)hipGraphExecDestroy(pl->cg_exec);
  if (pl->cg_graph) (void)hipGraphDestroy(pl->cg_graph);
  pl->cg_exec = nullptr;
  pl->cg_graph = nullptr;
}

// Capture the CG body on the plan's capture stream (kernel launches only: no
// memory set or copy nodes) and instantiate it.
static slrx_status capture_cg(slrx_plan* pl, int n_cg, const CgGraphKey& key) {
  cg_graph_reset(pl);
  if (!pl->cap_stream) HIPCHK(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  hipStream_t own = pl->stream;
  pl->stream = pl->cap_stream;
  HIPCHK(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
  const slrx_status st = cg_body(pl, n_cg);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
  pl->stream = own;
  if (st != SLRX_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != SLRX_OK ? st : fail(SLRX_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(SLRX_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
  }
  pl->cg_graph = g;
  pl->cg_exec = x;
  pl->cg_key = key;
  return SLRX_OK;
}

slrx_status slrx::run_cg(slrx_plan* pl, int n_cg, int it, bool graph) {
  const slrx_dims& d = pl->d;
  const long V = (long)pl->vol();
  if (graph && cg_graph_allowed(pl)) {
    const CgGraphKey key = cg_key(pl, n_cg);
    if (pl->cg_exec && std::memcmp(&key, &pl->cg_key, sizeof key) == 0) {
      HIPCHK(hipGraphLaunch(pl->cg_exec, pl->stream));
    } else {
      // this time one by one (first launches set up kernel attributes outside any
      // capture), replayed from the next call on
      STCHK(cg_body(pl, n_cg));
      STCHK(capture_cg(pl, n_cg, key));
    }
  } else {
    STCHK(cg_body(pl, n_cg));
  }
  if (it >= 0) {
    const int nfin = fin_blocks(d.P, d.T);
    const int nupd = update_blocks(V);
    HIPCHK(launch_store_sum(n_cg == 0 ? pl->partA : pl->partB, n_cg == 0 ? nfin : nupd,
                            pl->stats + 2 * SLRX_MAX_IRLS + it, pl->stream));
  }
  return SLRX_OK;
}

// Masks given in the ABI layout [W][P][Q] -> the plan's transposed planes.
slrx_status slrx::load_masks(slrx_plan* pl, const float2* E_dev) {
  const slrx_dims& d = pl->d;
  const int W = d.M * (d.M + 1) / 2;
  HIPCHK(launch_transpose_planes(W, d.P, d.Q, E_dev, pl->Et, pl->stream));
  return SLRX_OK;
}

// The plan's transposed planes -> [W][P][Q] in the staging buffer.
slrx_status slrx::store_masks(slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  const int W = d.M * (d.M + 1) / 2;
  HIPCHK(launch_transpose_planes(W, d.Q, d.P, pl->Et, pl->Estage, pl->stream));
  return SLRX_OK;
}
