// Per-pixel weights of the pixel-wise Hankel low-rank prior (HLR-Voxel,
// Sec. II.E, eq. "eq: MORASA-objective"; solved by IRLS as the paper does for
// this comparison system in Sec. IV).
//
// Pixel r has its own Toeplitz matrix T_r of its series rho_t(r) (rows
// n = M-1..T-1, column m holding rho_{n-m}(r); the blocks of eq.
// "eq:Toeplitz_g") and its own M x M Gram matrix
//   G_r[m][m'] = sum_{n=M-1}^{T-1} conj(rho_{n-m}(r)) rho_{n-m'}(r).
// The IRLS weight of the pixel's Schatten-p term is H_r = (G_r + eps I)^(p/2-1)
// (eigenvalues clamped at zero), and sum_r ||T_r H_r^(1/2)||_F^2 is the
// windowed quadratic form that the CG column pass applies, with per-pixel masks
// E_r = conj(H_r): pairs m <= m', planes transposed [w][col][row] like the
// masks of the main method.
//
// One thread per pixel, one 64-thread workgroup per 8 x 8 pixel tile (64-byte
// row segments for both the frame reads and the transposed mask writes).  G_r
// is accumulated in FP64 from the complex64 images; its eigen-decomposition is
// the cyclic Jacobi method for Hermitian matrices in registers: a rotation on
// (p, q) first turns a_pq real with the phase of its conjugate on column q, then
// applies the real symmetric Jacobi rotation of that 2 x 2 block; sweeps stop
// once the off-diagonal part is below 1e-16 of the matrix norm (quadratic
// convergence: a handful of sweeps for M <= 8).  Each workgroup also writes the
// largest eigenvalue of its 64 pixels to a partial, so that eps^(0) (Sec. III.C,
// a fraction of the largest eigenvalue over every pixel) and the per-iteration
// record come from a deterministic reduction, not from atomics.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace slrx {
namespace {

constexpr int kVoxTile = 8;  // pixels per tile side; P and Q are multiples of 8

constexpr int off_id(int p, int q, int M) { return p * M - p * (p + 1) / 2 + (q - p - 1); }  // p < q

SLRX_DEV double2 dscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
SLRX_DEV double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Hermitian M x M matrix: real diagonal and the strict upper triangle.
template <int M>
struct Herm {
  double d[M];
  double2 o[M > 1 ? M * (M - 1) / 2 : 1];
  SLRX_DEV double2 get(int k, int p) const { return k < p ? o[off_id(k, p, M)] : dconj(o[off_id(p, k, M)]); }
  SLRX_DEV void put(int k, int p, double2 v) {
    if (k < p) o[off_id(k, p, M)] = v;
    else o[off_id(p, k, M)] = dconj(v);
  }
};

// Cyclic Jacobi on A (overwritten: eigenvalues on the diagonal); with VEC the
// rotations are accumulated into V (columns: eigenvectors, V = I on entry).
template <int M, bool VEC>
SLRX_DEV void jacobi(Herm<M>& A, double2 (&V)[VEC ? M * M : 1]) {
  constexpr int kMaxSweeps = 30;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    double off = 0.0, dd = 0.0;
#pragma unroll
    for (int i = 0; i < (M > 1 ? M * (M - 1) / 2 : 0); ++i) off += A.o[i].x * A.o[i].x + A.o[i].y * A.o[i].y;
#pragma unroll
    for (int i = 0; i < M; ++i) dd += A.d[i] * A.d[i];
    if (!(off > 1e-32 * dd)) break;  // also stops on a zero matrix
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
      for (int q = p + 1; q < M; ++q) {
        const double2 g = A.o[off_id(p, q, M)];
        const double r = sqrt(g.x * g.x + g.y * g.y);
        if (r > 0.0) {
          const double2 ec = make_double2(g.x / r, -g.y / r);  // conj(g) / |g|
          const double tau = (A.d[q] - A.d[p]) / (2.0 * r);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
          A.d[p] -= t * r;
          A.d[q] += t * r;
          A.o[off_id(p, q, M)] = make_double2(0.0, 0.0);
#pragma unroll
          for (int k = 0; k < M; ++k) {
            if (k == p || k == q) continue;
            const double2 akp = A.get(k, p), akq = dmul(ec, A.get(k, q));
            A.put(k, p, dsub(dscale(akp, c), dscale(akq, s)));
            A.put(k, q, dadd(dscale(akp, s), dscale(akq, c)));
          }
          if constexpr (VEC) {
#pragma unroll
            for (int k = 0; k < M; ++k) {
              const double2 vkp = V[k * M + p], vkq = dmul(ec, V[k * M + q]);
              V[k * M + p] = dsub(dscale(vkp, c), dscale(vkq, s));
              V[k * M + q] = dadd(dscale(vkp, s), dscale(vkq, c));
            }
          }
        }
      }
  }
}

// VEC = false: eigenvalues only, the tile maxima into part.  VEC = true: the
// masks E_r = conj(H_r) into Et (and the tile maxima into part when given).
template <int M, bool VEC>
__global__ __launch_bounds__(64) void k_voxel(VoxelArgs a) {
  const int P = a.P, Q = a.Q, T = a.T;
  const long fs = (long)P * Q;
  const int tilesQ = Q / kVoxTile;
  const int r = (int)(blockIdx.x / tilesQ) * kVoxTile + (int)(threadIdx.x >> 3);
  const int c = (int)(blockIdx.x % tilesQ) * kVoxTile + (int)(threadIdx.x & 7);
  const float2* src = a.img + (long)r * Q + c;

  // G_r from a sliding window z[m] = rho_{n-m}
  Herm<M> A;
#pragma unroll
  for (int i = 0; i < M; ++i) A.d[i] = 0.0;
#pragma unroll
  for (int i = 0; i < (M > 1 ? M * (M - 1) / 2 : 1); ++i) A.o[i] = make_double2(0.0, 0.0);
  double2 z[M];
#pragma unroll
  for (int m = 0; m < M; ++m) z[m] = make_double2(0.0, 0.0);
  for (int n = 0; n < T; ++n) {
#pragma unroll
    for (int m = M - 1; m > 0; --m) z[m] = z[m - 1];
    z[0] = f2d(src[(long)n * fs]);
    if (n >= M - 1) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        A.d[m] += z[m].x * z[m].x + z[m].y * z[m].y;
#pragma unroll
        for (int mp = m + 1; mp < M; ++mp) A.o[off_id(m, mp, M)] = dadd(A.o[off_id(m, mp, M)], dcmul(z[m], z[mp]));
      }
    }
  }
  bool finite = true;
#pragma unroll
  for (int i = 0; i < M; ++i) finite = finite && isfinite(A.d[i]);
#pragma unroll
  for (int i = 0; i < (M > 1 ? M * (M - 1) / 2 : 0); ++i) finite = finite && isfinite(A.o[i].x) && isfinite(A.o[i].y);
  if (!finite) {
    if (a.bad) *a.bad = 1;
#pragma unroll
    for (int i = 0; i < M; ++i) A.d[i] = 0.0;
#pragma unroll
    for (int i = 0; i < (M > 1 ? M * (M - 1) / 2 : 1); ++i) A.o[i] = make_double2(0.0, 0.0);
  }

  double2 V[VEC ? M * M : 1];
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < M * M; ++i) V[i] = make_double2(i % (M + 1) == 0 ? 1.0 : 0.0, 0.0);
  }
  jacobi<M, VEC>(A, V);

  if (a.part) {
    double top = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) top = fmax(top, A.d[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) top = fmax(top, __shfl_xor(top, off, 64));
    if (threadIdx.x == 0) a.part[blockIdx.x] = top;
  }
  if constexpr (VEC) {
    const double e = *a.eps, ex = 0.5 * a.p - 1.0;
    double al[M];
#pragma unroll
    for (int i = 0; i < M; ++i) al[i] = pow(fmax(A.d[i], 0.0) + e, ex);
    // E[m][m'] = sum_i alpha_i conj(V[m][i]) V[m'][i], m <= m'
    float2* dst = a.Et + (long)c * P + r;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int mp = m; mp < M; ++mp) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < M; ++i) acc = dadd(acc, dscale(dcmul(V[m * M + i], V[mp * M + i]), al[i]));
        dst[(long)pair_id(m, mp, M) * fs] = make_float2((float)acc.x, (float)acc.y);
      }
  }
}

// The eps schedule on the tile maxima (one workgroup): mode 0 (first outer
// iteration) eps = eps0_frac * max, with both records; mode 1 eps = eps / gamma
// and its record; mode 2 the lambda_max record alone.
__global__ __launch_bounds__(256) void k_voxel_eps(VoxelEpsArgs a) {
  __shared__ double red[256];
  double v = 0.0;
  if (a.mode != 1)
    for (int i = threadIdx.x; i < a.nparts; i += 256) v = fmax(v, a.part[i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double lmax = red[0];
  if (a.mode == 0) *a.eps = a.eps0_frac * lmax;
  if (a.mode == 1) *a.eps = *a.eps / a.gamma;
  if (a.mode != 1 && a.lam_max_out) *a.lam_max_out = lmax;
  if (a.mode != 2 && a.eps_out) *a.eps_out = *a.eps;
}

template <int M>
hipError_t launch_m(const VoxelArgs& a, bool vec, hipStream_t s) {
  const unsigned nb = (unsigned)(a.P / kVoxTile) * (unsigned)(a.Q / kVoxTile);
  if (vec) k_voxel<M, true><<<nb, 64, 0, s>>>(a);
  else k_voxel<M, false><<<nb, 64, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

int voxel_tiles(int P, int Q) { return (P / kVoxTile) * (Q / kVoxTile); }

hipError_t launch_voxel(const VoxelArgs& a, bool vec, hipStream_t s) {
  if (a.P % kVoxTile || a.Q % kVoxTile || (vec && (!a.Et || !a.eps))) return hipErrorInvalidValue;
  switch (a.M) {
    case 1: return launch_m<1>(a, vec, s);
    case 2: return launch_m<2>(a, vec, s);
    case 3: return launch_m<3>(a, vec, s);
    case 4: return launch_m<4>(a, vec, s);
    case 5: return launch_m<5>(a, vec, s);
    case 6: return launch_m<6>(a, vec, s);
    case 7: return launch_m<7>(a, vec, s);
    case 8: return launch_m<8>(a, vec, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_voxel_eps(const VoxelEpsArgs& a, hipStream_t s) {
  k_voxel_eps<<<1, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace slrx
