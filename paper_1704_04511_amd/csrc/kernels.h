// Launch wrappers of the libslrx kernels (host side).  All launches are
// asynchronous on the given stream and return hipGetLastError().
#pragma once
#include <vector>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slrx {

// Supported transform lengths along each image axis.
bool fft_len_supported(int n);
int max_frames();  // largest T handled by the column penalty pass
int max_taps();    // largest M

// ---------------------------------------------------------------- FFT passes
enum RowMode { ROW_PLAIN = 0, ROW_MASKED = 1, ROW_PUPDATE = 2 };

// Row DFT (length Q) of a row-major volume; output transposed per frame
// ([t][col][row]).  ROW_PUPDATE also forms p = r + beta p (beta from partials).
struct RowArgs {
  int P, Q, T;
  int mode;              // RowMode
  int sign;              // -1 forward, +1 inverse (unnormalised)
  const float2* src;     // input (r for ROW_PUPDATE)
  float2* pvec;          // ROW_PUPDATE: p (read p_old, write p)
  const uint8_t* S;      // ROW_MASKED: mask
  float2* dst;           // transposed output
  float scale;
  const float2* tw;      // e^{-2 pi i t / Q}, t < Q
  int k;                 // ROW_PUPDATE: CG iteration index
  const double* part;    // ROW_PUPDATE: partials holding rr_k
  int npart;
  double* rr_hist;       // rr_hist[k] written by block 0; rr_hist[k-1] read
};
hipError_t launch_rows(const RowArgs& a, hipStream_t s);

// Column DFT (length P) of a transposed volume; output row-major.
struct ColArgs {
  int P, Q, T;
  int sign;
  const float2* src;     // transposed
  float2* dst;           // row-major
  float scale;
  const float2* tw;      // e^{-2 pi i t / P}, t < P
};
hipError_t launch_cols(const ColArgs& a, hipStream_t s);

// Column pass of the operator on a transposed volume, in place: inverse column
// DFT, penalty G over all frames scaled by `scale`, forward column DFT.
struct PenArgs {
  int P, Q, T, M;
  float2* buf;           // transposed [t][c][r]
  const float2* Et;      // masks, transposed planes [w][c][r]
  float scale;           // lam / (P Q)
  const float2* tw;      // e^{-2 pi i t / P}
  // multichannel data term (nc > 0): input rho (the coil column pass's image)
  // instead of inverting the columns of buf
  int nc;
  const float2* rho;     // image rho_u, transposed
  int circ;              // G circulant along the frames (GIRAF)
};
hipError_t launch_pen(const PenArgs& a, hipStream_t s);

// Forward row DFT of the transposed penalty volume back to row-major, plus the
// data term S o v and the CG dot product (or the initial residual).
struct FinArgs {
  int P, Q, T;
  int init;              // 1: out = y - A v, partial <out,out>;  0: out = A v, partial <v,out>
  const float2* t;       // transposed penalty volume
  const float2* v;       // x (init) or p, row-major k-space
  const uint8_t* S;
  const float2* y;       // right-hand side S o b (init)
  float2* out;
  double* part;          // per-block partials
  int* flag;             // CG stop flag (cleared by block 0 when init)
  const float2* tw;      // e^{-2 pi i t / Q}
  // multichannel data term (coil = 1): no S o v; the complex128 forward row DFT
  // of the coil combination (d64: dparts group sums, column-transformed,
  // transposed, group g at g * dstride) is added to the penalty before rounding
  int coil;
  const double2* d64;
  int dparts;
  long dstride;
  const double2* tw64;   // e^{-2 pi i t / Q}, complex128
};
hipError_t launch_fin(const FinArgs& a, hipStream_t s);
int fin_blocks(int P, int T);

// CG vector update x += alpha p, r -= alpha q, partial <r,r>.
struct UpdArgs {
  long n;
  float2 *x, *r;
  const float2 *p, *q;
  const double* partA; int nA;   // <p,q> partials
  const double* rr_hist; int k;  // rr_k
  double* partB;                 // out partials
  int* flag;
};
hipError_t launch_update(const UpdArgs& a, hipStream_t s);
int update_blocks(long n);

// Grouped CG passes (batches): one launch covers every problem of a group (any
// frame sizes and counts, one tap count M, single-channel data); each problem's
// blocks do exactly what they do in the problem's own launches.
struct CgSlice {
  int P, Q, T, circ;
  float pen_scale;                      // lam / (P Q)
  float2 *x, *r, *p, *q, *t;
  const float2* bm;                     // right-hand side S o b
  const uint8_t* S;
  const float2* Et;                     // masks, transposed planes
  const float2 *twQ, *twP;              // complex64 twiddles of the row and column lengths
  double *partA, *partB, *rr_hist;
  int* flag;
  int nfin, nupd;                       // partial counts of the finishing and update passes
  int rows_gx, rows_gy, cols_gx, upd_gx;  // the problem's own grids
  int rows0, cols0, upd0;               // its first block in the grouped grids (multiples of 8)
};
struct CgGroup {
  const CgSlice* tab;                   // device copy of the table, ns entries
  int ns, M;
  int rows_blocks, cols_blocks, upd_blocks;
  size_t pen_lds;                       // dynamic LDS of the grouped column pass
};
void cg_slice_grids(CgSlice& c);        // fills the grids and partial counts from P, Q, T
size_t group_pen_lds(int P, int Q, int T);
// mode: ROW_PLAIN (initial residual, x) or ROW_PUPDATE (iteration k)
hipError_t launch_group_rows(const CgGroup& g, int mode, int k, hipStream_t s);
hipError_t launch_group_pen(const CgGroup& g, hipStream_t s);
hipError_t launch_group_fin(const CgGroup& g, int init, hipStream_t s);
hipError_t launch_group_update(const CgGroup& g, int k, hipStream_t s);

// Multichannel data term (k_coil.hip): complex64 forward half, complex128
// adjoint half after the sampling mask.
struct CoilArgs {
  int P, Q, T, nc;
  const float2* t;       // row pass output (transposed)
  float2* rho;           // out: image rho_u (transposed)
  const float2* Ct;      // coil maps, transposed per coil [j][c][r]
  float2* Y;             // per-coil volumes after the forward half (transposed), coil j at j * vstride
  double2* Y64;          // per-coil volumes after the inverse row DFT (transposed), complex128
  long vstride;
  const uint8_t* S;      // sampling mask, row-major [t][kr][kc]
  const float2* tw;      // twiddles of the pass's transform length (P: columns, Q: rows)
  const double2* tw64;   // the same in complex128
  double2* d64;          // combine pass out: per-group sums, column-transformed (transposed), group g at g * vstride
  double cscale64;       // (P Q)^-2 in the operator, (P Q)^-1 for the right-hand side
  int groups;            // coil groups of the combine pass (coil_groups(nc))
  const float2* B;       // right-hand side: coil k-space, row-major [j][t][kr][kc], coil j at j * vstride
  float2* out;           // right-hand side: A^H b, row-major k-space
};
// Coils are combined in up to kCoilGroups groups in parallel; the finishing
// pass adds their sums in group order.
constexpr int kCoilGroups = 4;
inline int coil_groups(int nc) { return nc < kCoilGroups ? nc : kCoilGroups; }
hipError_t launch_coil_cols(const CoilArgs& a, hipStream_t s);
hipError_t launch_coil_rows(const CoilArgs& a, hipStream_t s);
hipError_t launch_coil_combine(const CoilArgs& a, hipStream_t s);
hipError_t launch_coil_rhs_rows(const CoilArgs& a, hipStream_t s);
hipError_t launch_coil_rhs_fin(const CoilArgs& a, hipStream_t s);

// Mono-exponential fit per pixel (k_fit.hip); te holds the T echo times.
struct FitArgs {
  long npix;
  int T;
  const float2* img;     // [T][npix]
  double te[32];
  double tbar, stt;      // mean echo time, sum of squared centred times
  double* t2;            // [npix]
  double* amp;           // [npix] or null
};
hipError_t launch_fit_t2(const FitArgs& a, hipStream_t s);

hipError_t launch_mask_data(long n, const uint8_t* S, const float2* b, float2* out, hipStream_t s);
hipError_t launch_store_sum(const double* part, int n, double* dst, hipStream_t s);
hipError_t launch_interleave(long n, const double* re, const double* im, double2* out, hipStream_t s);
// out[w][j][i] = in[w][i][j] for W planes of A x B.
hipError_t launch_transpose_planes(int W, int A, int B, const float2* in, float2* out, hipStream_t s);

// ---------------------------------------------------------------- Gram etc.
struct GramArgs {
  int P, Q, T, N1, N2, M;
  const float2* rho;        // images [T][P][Q]
  double2* c1;              // [W][P][2N2-1]
  double2* g;               // [W][2N1-1][2N2-1]
  double2* R;               // s x s full Hermitian: column-major, or row-major if rowmajor
  int rowmajor;
  const double2* twP;       // e^{-2 pi i t/P}, t < P
  const double2* twQ;
  int circ;                 // lagged sums over all n with frame indices mod T (GIRAF)
  int* bad;                 // set to 1 if any entry is non-finite (then written as 0), or null
};
hipError_t launch_gram(const GramArgs& a, hipStream_t s);

// Pixel-wise weights (HLR-Voxel): per pixel the M x M Gram matrix of its
// Toeplitz lifting, its eigen-decomposition, and the masks conj((G + eps I)^(p/2-1)).
struct VoxelArgs {
  int P, Q, T, M;           // P, Q multiples of 8; M <= 8
  const float2* img;        // images [T][P][Q]
  double* part;             // largest eigenvalue per 8 x 8 tile (voxel_tiles entries), or null
  const double* eps;        // eps (device), masks pass only
  double p;
  float2* Et;               // masks, transposed planes [W][Q][P] (masks pass only)
  int* bad;                 // set to 1 on a non-finite Gram entry (then taken as 0), or null
};
int voxel_tiles(int P, int Q);
// vec = false: eigenvalues only (tile maxima); vec = true: the masks as well.
hipError_t launch_voxel(const VoxelArgs& a, bool vec, hipStream_t s);
struct VoxelEpsArgs {
  const double* part;
  int nparts;
  int mode;                 // 0: eps = eps0_frac * max; 1: eps = eps / gamma; 2: max record only
  double* eps;
  double* lam_max_out;      // may be null
  double* eps_out;          // may be null
  double eps0_frac, gamma;
};
hipError_t launch_voxel_eps(const VoxelEpsArgs& a, hipStream_t s);

// IRLS-direct (k_direct.hip): the explicit linear lifting, its adjoint and CG glue.
struct DirectArgs {
  int P, Q, T, N1, N2, M;
  int a1min, a2min, a1max, a2max;  // filter offsets: a in [amin, amax] per axis
  int nw1, nw2;                    // valid shifts per axis
  long rows;                       // (T-M+1) nw1 nw2 rows of the lifted matrix
  double lam;
};
DirectArgs direct_args(int P, int Q, int T, int N1, int N2, int M, double lam);
int direct_blocks(long V);  // blocks (and partials) of the adjoint pass for V samples
// X = T(x), row-major rows x s (complex128 or complex64)
hipError_t launch_dlift64(const DirectArgs& a, const float2* x, double2* X, hipStream_t s);
hipError_t launch_dlift32(const DirectArgs& a, const float2* x, float2* X, hipStream_t s);
// out = S o v + lam T^*(Y) (init: y - that, partials <out,out>, flag cleared); else partials <v,out>
hipError_t launch_dadj(const DirectArgs& a, const float2* Y, const float2* v, const uint8_t* S, const float2* y,
                       float2* out, int init, double* part, int* flag, hipStream_t s);
// p = r + beta p with beta from the partials of rr_k and rr_hist[k-1]; records rr_hist[k]
hipError_t launch_dpupdate(long n, const float2* r, float2* p, const double* part, int npart, double* rr_hist, int k,
                           hipStream_t s);
hipError_t launch_hf(long n, const double* re, const double* im, float2* out, hipStream_t s);

struct WeightArgs {
  int s;
  const double* lamv;       // eigenvalues, ascending
  const double2* U;         // eigenvectors, column-major s x s
  double* VT;               // [2s][s]: rows k' < s: Re(U[:,k']) sqrt(alpha), then Im
  double* eps;              // eps state (in/out)
  double* lam_max_out;      // per-iteration record (may be null)
  double* eps_out;          // per-iteration record (may be null)
  int first;                // 1 on the first IRLS iteration
  double eps0_frac, gamma, p;
};
hipError_t launch_eps(const WeightArgs& a, hipStream_t s);  // the eps update alone
hipError_t launch_weights(const WeightArgs& a, hipStream_t s, bool eps = true);

// Householder tridiagonalisation R = Q T Q^H of nbatch n x n Hermitian matrices
// (one launch per column).  Aw: row-major full matrices (overwritten); Vst:
// reflectors in LAPACK zhetrd lower layout (column-major); D, E: real
// tridiagonal; tau: reflector scalars; vbuf/pbuf: 2 x nbatch x n scratch each.
struct TriArgs {
  int n, k;
  double2* Aw;
  double2* Vst;
  long strideA;             // elements between matrices of the batch
  double* D;
  double* E;
  double2* tau;
  double2* vbuf[2];
  double2* pbuf[2];
};
// cand: the tuner's candidate launch shape (tri_budget: workgroups per column
// launch across the batch; for one problem candidate 2 also caps the rows per
// workgroup at those loaded at kernel entry); stream: nontemporal loads and
// stores of the trailing-block rows.  Results depend on neither.
hipError_t launch_tridiag(const TriArgs& a, int nbatch, hipStream_t s, int cand, bool stream);
int tri_budget_candidates(int nbatch);
int tri_budget(int nbatch, int cand);
int tri_max_n();

// U = Q Z from the reflectors of launch_tridiag (all column-major n x n).
struct BackTrArgs {
  int n;
  double2* V;           // reflectors as stored by launch_tridiag; made explicit in place
  double2* Y;           // workspace, n x n
  double2* Z;           // in: tridiagonal eigenvectors; out: eigenvectors of the Hermitian matrix
  const double2* tau;   // n
  double2* scratch;     // bt_scratch_elems(n)
  int nb = 1;           // problems of equal n: problem b uses V + b sV, Y + b sY, Z + b sZ,
  long sV = 0, sY = 0, sZ = 0, s_scratch = 0;  // tau + b n, scratch + b s_scratch
};
hipError_t launch_backtransform(const BackTrArgs& a, hipStream_t s);
size_t bt_scratch_elems(int n);

// Eigenpairs of the real symmetric tridiagonal (D, E) by divide and conquer:
// D gets the ascending eigenvalues, Z (column-major n x n complex) the
// eigenvectors with imaginary part 0.
struct TdArgs {
  int n;
  double* D;                     // n: diagonal in, eigenvalues out
  const double* E;               // n - 1 off-diagonal entries
  double2* Z;                    // n x n output
  double* Q;                     // n x n workspace
  double* Qs;                    // n x n workspace
  double* U;                     // n x n workspace
  const int* nodes;              // device copy of the tree from dc_build_tree
  std::vector<int> level_start;  // from dc_build_tree
  std::vector<int> node_sizes;   // size of every node, host copy
  int* ws_i;                     // dc_ws_ints(n)
  double* ws_d;                  // dc_ws_doubles(n)
  int nb = 1;                    // problems of equal n solved together; problem b uses
  long sQ = 0, sZ = 0;           // D + b n, E + b n, Q/Qs/U + b sQ, Z + b sZ,
  long s_wsi = 0, s_wsd = 0;     // ws_i + b s_wsi, ws_d + b s_wsd
};
void dc_build_tree(int n, std::vector<int>& nodes, std::vector<int>& level_start);
size_t dc_ws_ints(int n);
size_t dc_ws_doubles(int n);
int dc_max_n();
hipError_t launch_tdeig(const TdArgs& a, hipStream_t s);

// H = V V^H on FP64 MFMA: Hre, Him row-major s x s.
hipError_t launch_filter_product(int s, const double* VT, double* Hre, double* Him, hipStream_t st);

struct MaskArgs {
  int P, Q, N1, N2, M;
  const double* Hre; const double* Him;
  double2* wsum;            // [W][2N1-1][2N2-1]
  double2* s1;              // [W][2N1-1][Q]
  float2* Et;               // [W][Q][P] (transposed planes)
  const double2* twP; const double2* twQ;
};
hipError_t launch_masks(const MaskArgs& a, hipStream_t s);

// Lag sums wsum of H = U diag(alpha) U^H from the filter spectra, without H
// (M <= kSpecMaxM, 2 N1 - 1 <= 32, s <= kSpecMaxS, LDS bounds: spec_supported).
constexpr int kSpecMaxM = 5;
constexpr int kSpecMaxS = 2048;   // largest s = N1 N2 M
constexpr int kSpecSlices = 8;    // fixed-order slices of the group sums
struct SpecArgs {
  int N1, N2, M, s;
  int ngroups, kper;     // eigenvector groups (spec_groups) and eigenvectors per group
  const double* lamv;    // eigenvalues
  const double2* U;      // eigenvectors, column-major s x s
  const double* eps;     // eps of this iteration (device)
  double p;
  double2* part;         // [ngroups][W][L1 L2] partial sums
  double2* C;            // [kSpecSlices][W][L1 L2] slice sums
};
bool spec_supported(int N1, int N2, int M);
int spec_groups(int N1, int N2, int M, size_t cap);
hipError_t launch_spec_masks(const SpecArgs& a, double2* wsum, hipStream_t st);

}  // namespace slrx
