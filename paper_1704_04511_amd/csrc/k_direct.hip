// IRLS-direct (SLRX_FLAG_DIRECT): the method without the FFT-based
// approximations, which the paper compares with (Sec. IV, Fig. 2).  The lifting
// is linear in all three dimensions: k-space in centred order (DC at
// (P/2, Q/2)), rows (n, w) for n = M-1..T-1 and the valid shifts w (the
// N1 x N2 support w - a inside the grid, (P-N1+1)(Q-N2+1) of them), columns
// (m, a) with a the filter offsets in row-major order; entry xc[n-m][w-a].
// Both sub-problems run on the explicit matrix:
//   * R = X^H X with X the lifted matrix of the iterate in complex128 (a plain
//     library GEMM, then the library's own eigen-decomposition chain);
//   * the least-squares operator A v = S o v + lam T^*(T(v) H): T(v) gathered
//     in complex64, times H (a plain library GEMM), and the adjoint T^* as a
//     gather per k-space sample (every entry of T(v) H that was read from that
//     sample, in a fixed order, accumulated in FP64), fused with S o v and the CG
//     dot product.
// This file holds the gathers and the CG glue; the GEMMs are rocBLAS calls.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace slrx {
namespace {

constexpr int kDirNT = 256;

// Lifted-matrix entry (r, j) -> the k-space index it reads, in DFT order.
SLRX_DEV long lift_src(const DirectArgs& a, long r, int j) {
  const int NN = a.N1 * a.N2;
  const int m = j / NN, ia = j % NN;
  const int a1 = ia / a.N2 + a.a1min, a2 = ia % a.N2 + a.a2min;
  const int i2 = (int)(r % a.nw2);
  const long rq = r / a.nw2;
  const int i1 = (int)(rq % a.nw1);
  const int n = (int)(rq / a.nw1) + a.M - 1;
  const int c1 = i1 + a.a1max - a1, c2 = i2 + a.a2max - a2;  // centred coordinates of w - a
  const int k1 = (c1 + a.P / 2) % a.P, k2 = (c2 + a.Q / 2) % a.Q;
  return ((long)(n - m) * a.P + k1) * a.Q + k2;
}

template <typename OUT>
__global__ __launch_bounds__(kDirNT) void k_dlift(DirectArgs a, const float2* __restrict__ x, OUT* __restrict__ X) {
  const int s = a.N1 * a.N2 * a.M;
  const long n = a.rows * s;
  for (long e = (long)blockIdx.x * kDirNT + threadIdx.x; e < n; e += (long)gridDim.x * kDirNT) {
    const float2 v = x[lift_src(a, e / s, (int)(e % s))];
    if constexpr (sizeof(OUT) == sizeof(double2)) X[e] = OUT{(double)v.x, (double)v.y};
    else X[e] = OUT{v.x, v.y};
  }
}

// out = S o v + lam T^*(Y) (init: out = y - that), partial dot products per block.
__global__ __launch_bounds__(kDirNT) void k_dadj(DirectArgs a, const float2* __restrict__ Y,
                                                 const float2* __restrict__ v, const uint8_t* __restrict__ S,
                                                 const float2* __restrict__ y, float2* __restrict__ out, int init,
                                                 double* part, int* flag) {
  __shared__ double red[kDirNT / 64];
  const int P = a.P, Q = a.Q, NN = a.N1 * a.N2, s = NN * a.M;
  const long V = (long)a.T * P * Q;
  double dot = 0.0;
  for (long g = (long)blockIdx.x * kDirNT + threadIdx.x; g < V; g += (long)gridDim.x * kDirNT) {
    const int k2 = (int)(g % Q);
    const long gq = g / Q;
    const int k1 = (int)(gq % P), f = (int)(gq / P);
    const int c1 = (k1 + P / 2) % P, c2 = (k2 + Q / 2) % Q;  // centred coordinates
    double ax = 0.0, ay = 0.0;
    for (int m = 0; m < a.M; ++m) {
      const int n = f + m;
      if (n < a.M - 1 || n >= a.T) continue;
      for (int ia = 0; ia < NN; ++ia) {
        const int i1 = c1 + ia / a.N2 + a.a1min - a.a1max, i2 = c2 + ia % a.N2 + a.a2min - a.a2max;
        if (i1 < 0 || i1 >= a.nw1 || i2 < 0 || i2 >= a.nw2) continue;
        const long r = ((long)(n - a.M + 1) * a.nw1 + i1) * a.nw2 + i2;
        const float2 t = Y[r * s + m * NN + ia];
        ax += t.x;
        ay += t.y;
      }
    }
    const float2 vv = v[g];
    const float sv = S[g] ? 1.f : 0.f;
    float2 av = make_float2(sv * vv.x + (float)(a.lam * ax), sv * vv.y + (float)(a.lam * ay));
    if (init) {
      const float2 yv = y[g];
      av = make_float2(yv.x - av.x, yv.y - av.y);
      dot += (double)av.x * av.x + (double)av.y * av.y;
    } else {
      dot += (double)vv.x * av.x + (double)vv.y * av.y;
    }
    out[g] = av;
  }
  dot = block_sum<kDirNT>(dot, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = dot;
    if (init && blockIdx.x == 0) *flag = 0;
  }
}

// p = r + beta p, beta = rr_k / rr_{k-1} from the partials of rr_k (rr_hist[k] recorded).
__global__ __launch_bounds__(kDirNT) void k_dpupdate(long n, const float2* __restrict__ r, float2* __restrict__ p,
                                                     const double* part, int npart, double* rr_hist, int k) {
  __shared__ double red[kDirNT / 64];
  const double rr = reduce_partials<kDirNT>(part, npart, red);
  double beta = 0.0;
  if (k > 0) {
    const double prev = rr_hist[k - 1];
    beta = prev > 0.0 ? rr / prev : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rr_hist[k] = rr;
  const float fb = (float)beta;
  for (long i = (long)blockIdx.x * kDirNT + threadIdx.x; i < n; i += (long)gridDim.x * kDirNT) {
    const float2 rv = r[i];
    const float2 po = k > 0 ? p[i] : make_float2(0.f, 0.f);
    p[i] = make_float2(rv.x + fb * po.x, rv.y + fb * po.y);
  }
}

__global__ void k_hf(long n, const double* __restrict__ re, const double* __restrict__ im, float2* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)re[i], (float)im[i]);
}

unsigned grid_for(long n) {
  const long b = (n + kDirNT - 1) / kDirNT;
  return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace

DirectArgs direct_args(int P, int Q, int T, int N1, int N2, int M, double lam) {
  DirectArgs a{};
  a.P = P; a.Q = Q; a.T = T; a.N1 = N1; a.N2 = N2; a.M = M;
  a.a1min = -(N1 / 2);
  a.a2min = -(N2 / 2);
  a.a1max = N1 - 1 - N1 / 2;
  a.a2max = N2 - 1 - N2 / 2;
  a.nw1 = P - N1 + 1;
  a.nw2 = Q - N2 + 1;
  a.rows = (long)(T - M + 1) * a.nw1 * a.nw2;
  a.lam = lam;
  return a;
}

int direct_blocks(long V) { return (int)grid_for(V); }

hipError_t launch_dlift64(const DirectArgs& a, const float2* x, double2* X, hipStream_t s) {
  k_dlift<double2><<<grid_for(a.rows * a.N1 * a.N2 * a.M), kDirNT, 0, s>>>(a, x, X);
  return hipGetLastError();
}

hipError_t launch_dlift32(const DirectArgs& a, const float2* x, float2* X, hipStream_t s) {
  k_dlift<float2><<<grid_for(a.rows * a.N1 * a.N2 * a.M), kDirNT, 0, s>>>(a, x, X);
  return hipGetLastError();
}

hipError_t launch_dadj(const DirectArgs& a, const float2* Y, const float2* v, const uint8_t* S, const float2* y,
                       float2* out, int init, double* part, int* flag, hipStream_t s) {
  const long V = (long)a.T * a.P * a.Q;
  k_dadj<<<grid_for(V), kDirNT, 0, s>>>(a, Y, v, S, y, out, init, part, flag);
  return hipGetLastError();
}

hipError_t launch_dpupdate(long n, const float2* r, float2* p, const double* part, int npart, double* rr_hist, int k,
                           hipStream_t s) {
  k_dpupdate<<<grid_for(n), kDirNT, 0, s>>>(n, r, p, part, npart, rr_hist, k);
  return hipGetLastError();
}

hipError_t launch_hf(long n, const double* re, const double* im, float2* out, hipStream_t s) {
  k_hf<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, re, im, out);
  return hipGetLastError();
}

}  // namespace slrx
