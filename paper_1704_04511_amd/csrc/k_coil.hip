// Multichannel data term of the CG operator (Sec. II.A, eq. "measurement_ij").
//
// With coil sensitivities C_j the least-squares step applies
//   A^H A v = F sum_j C_j^* F^-1 (S o F (C_j F^-1 v))
// instead of S o v.  The forward half (up to the sampling mask) runs in
// complex64; the adjoint half after the mask runs in complex128 and is
// rounded once, element by element, when it is added to the penalty in
// k-space.  Round-off of a transform spreads over every output entry, and the
// adjoint half would otherwise spread O(eps32 |data|) into the k-space
// directions the data term leaves (nearly) unconstrained, where the operator
// is only lam G; errors of the forward half are confined to sampled entries
// by the mask and only reach the range of A^H.  The operator keeps its row
// pass (inverse row DFT of v, transposed output) and gains three passes:
//   1. k_coil_cols (per column tile, frame and coil): the inverse column DFT
//      gives the image rho_u = IDFT2(v) (kept for the penalty by coil 0), then
//      the forward column DFT of C_j rho_u;
//   2. k_coil_rows (per k-space row tile, frame and coil): forward row DFT, the
//      frame's sampling mask, then in complex128 the inverse row DFT;
//   3. k_coil_combine (per column tile, frame and group of coils, complex128):
//      d_g = cscale sum_{j in group g} conj(C_j) IDFT_col(Y_j), one coil after
//      another with the next coil's loads in flight during the current
//      transform, then the forward column DFT of d_g;
// the column pass (k_cols_pen, coil mode) forms the penalty alone, and the
// finishing row pass adds the complex128 forward row DFT of d_0 + d_1 + ...
// (in that order) to it.  All transforms here are unnormalised; cscale =
// (PQ)^-2 makes the composition the unitary operator.  The right-hand side
// A^H b uses the same adjoint half (k_coil_rhs_rows, k_coil_combine with
// cscale = (PQ)^-1, k_coil_rhs_fin).  Volumes use the transposed layout of the
// column pass ([t][c][r]); the coil maps are stored transposed per coil
// ([j][c][r]).
#include "common.h"
#include "fft.h"
#include "kernels.h"

namespace slrx {

constexpr int kCoilNT = 256;
constexpr int kCoilRB = 8;  // k-space rows per block of the row pass

// Columns per block of the coil column and combine passes: a power of two
// dividing Q with CB * N <= 1024 elements (four per thread).
template <int N> struct CoilCap { static constexpr int v = 1024 / N > 0 ? 1024 / N : 1; };
__host__ __device__ inline int coil_col_block(int cap, int Q) {
  int cb = 1;
  while (cb * 2 <= cap) cb *= 2;
  while (cb > 1 && (Q % cb) != 0) cb >>= 1;
  return cb;
}

// ---------------------------------------------------- pass 1: coil columns
// Block: CB columns of one frame for one coil.  In: the row pass output t
// (transposed).  Out: rho_u (transposed, coil 0 only) and DFT_col(C_j rho_u).
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_cols(CoilArgs a) {
  constexpr int CAP = CoilCap<N>::v;
  constexpr int BS = fft_stride(N);
  __shared__ float2 img[CAP * BS];
  __shared__ float2 twt[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int CB = coil_col_block(CAP, Q);
  const int c0 = blockIdx.x * CB, f = blockIdx.y, j = blockIdx.z;
  const long fs = (long)P * Q;
  const long base = (long)f * fs + (long)c0 * P;  // CB contiguous columns of frame f
  const int nel = CB * N;
  fft_twiddles<N, kCoilNT>(twt, a.tw);
  auto at = [&](int e) { return (e / N) * BS + fft_pidx(e % N); };
  const float2* C = a.Ct + (long)j * fs + (long)c0 * P;
  for (int e = threadIdx.x; e < nel; e += kCoilNT) img[at(e)] = a.t[base + e];
  __syncthreads();
  fft_lds<N, +1, CAP, kCoilNT>(img, twt, CB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT) {
    const float2 v = img[at(e)];
    if (j == 0) a.rho[base + e] = v;
    img[at(e)] = cmul(C[e], v);
  }
  __syncthreads();
  fft_lds<N, -1, CAP, kCoilNT>(img, twt, CB);
  float2* Y = a.Y + (long)j * a.vstride + base;
  for (int e = threadIdx.x; e < nel; e += kCoilNT) Y[e] = img[at(e)];
}

// ------------------------------------------------------- pass 2: coil rows
// Block: RB k-space rows of one frame and coil, gathered from the transposed
// layout; forward row DFT (complex64), sampling mask S (row-major
// [t][kr][kc]), inverse row DFT in complex128, stored to Y64 at the same
// (transposed) positions.
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_rows(CoilArgs a) {
  constexpr int BS = fft_stride(N);
  __shared__ float2 lds[kCoilRB * BS];
  __shared__ double2 lds64[kCoilRB * BS];
  __shared__ float2 twt[fft_tw_size<N>()];
  __shared__ double2 twt64[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int RB = P < kCoilRB ? P : kCoilRB;
  const int r0 = blockIdx.x * RB, f = blockIdx.y, j = blockIdx.z;
  const long fs = (long)P * Q;
  const float2* Y = a.Y + (long)j * a.vstride + (long)f * fs;
  double2* Y64 = a.Y64 + (long)j * a.vstride + (long)f * fs;
  const uint8_t* S = a.S + (long)f * fs;
  const int nel = RB * N;
  fft_twiddles<N, kCoilNT>(twt, a.tw);
  fft_twiddles<N, kCoilNT>(twt64, a.tw64);
  // element e: column c = e / RB, row r0 + e % RB (consecutive threads walk a column)
  for (int e = threadIdx.x; e < nel; e += kCoilNT)
    lds[(e % RB) * BS + fft_pidx(e / RB)] = Y[(long)(e / RB) * P + r0 + e % RB];
  __syncthreads();
  fft_lds<N, -1, kCoilRB, kCoilNT>(lds, twt, RB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT) {
    const int i = e / N, kc = e % N;
    const float2 v = lds[i * BS + fft_pidx(kc)];
    lds64[i * BS + fft_pidx(kc)] = S[(long)(r0 + i) * Q + kc] ? f2d(v) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_lds<N, +1, kCoilRB, kCoilNT>(lds64, twt64, RB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT)
    Y64[(long)(e / RB) * P + r0 + e % RB] = lds64[(e % RB) * BS + fft_pidx(e / RB)];
}

// Right-hand side, first half: the coil k-space b_j (row-major [j][t][kr][kc]),
// masked, inverse row DFT in complex128, stored to Y64 in the transposed layout.
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_rhs_rows(CoilArgs a) {
  constexpr int BS = fft_stride(N);
  __shared__ double2 lds64[kCoilRB * BS];
  __shared__ double2 twt64[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int RB = P < kCoilRB ? P : kCoilRB;
  const int r0 = blockIdx.x * RB, f = blockIdx.y, j = blockIdx.z;
  const long fs = (long)P * Q;
  const float2* B = a.B + (long)j * a.vstride + (long)f * fs;
  double2* Y64 = a.Y64 + (long)j * a.vstride + (long)f * fs;
  const uint8_t* S = a.S + (long)f * fs;
  const int nel = RB * N;
  fft_twiddles<N, kCoilNT>(twt64, a.tw64);
  for (int e = threadIdx.x; e < nel; e += kCoilNT) {  // row-major: consecutive threads walk a row
    const int i = e / N, kc = e % N;
    const long g = (long)(r0 + i) * Q + kc;
    lds64[i * BS + fft_pidx(kc)] = S[g] ? f2d(B[g]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_lds<N, +1, kCoilRB, kCoilNT>(lds64, twt64, RB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT)
    Y64[(long)(e / RB) * P + r0 + e % RB] = lds64[(e % RB) * BS + fft_pidx(e / RB)];
}

// Right-hand side, last step: the complex128 forward row DFT of d_0 + d_1 + ..
// (transposed layout), rounded to complex64, row-major out.
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_rhs_fin(CoilArgs a) {
  constexpr int BS = fft_stride(N);
  __shared__ double2 lds64[kCoilRB * BS];
  __shared__ double2 twt64[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int RB = P < kCoilRB ? P : kCoilRB;
  const int r0 = blockIdx.x * RB, f = blockIdx.y;
  const long fo = (long)f * P * Q;
  fft_twiddles<N, kCoilNT>(twt64, a.tw64);
  rows_sum_fwd<N, kCoilRB, kCoilNT>(lds64, twt64, a.d64, a.groups, a.vstride, fo, P, r0, RB);
  for (int e = threadIdx.x; e < RB * N; e += kCoilNT) {
    const int i = e / N, kc = e % N;
    const double2 v = lds64[i * BS + fft_pidx(kc)];
    a.out[fo + (long)(r0 + i) * Q + kc] = make_float2((float)v.x, (float)v.y);
  }
}

// ---------------------------------------------------- pass 3: coil combine
// Block: CB columns of one frame and one group g of coils (a balanced split of
// the coils into the groups of the grid's z dimension), complex128 throughout.
// d_g = cscale sum_{j in g} conj(C_j) IDFT_col(Y64_j), coils in order (a fixed
// summation order); each thread keeps the sums of its elements in registers
// and loads coil j+1 while coil j is transformed; then the forward column DFT
// of d_g, stored to d64 (transposed layout).
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_combine(CoilArgs a) {
  constexpr int CAP = CoilCap<N>::v;
  constexpr int BS = fft_stride(N);
  constexpr int EPT = (CAP * N + kCoilNT - 1) / kCoilNT;  // elements per thread
  __shared__ double2 lds[CAP * BS];
  __shared__ double2 twt[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int CB = coil_col_block(CAP, Q);
  const int c0 = blockIdx.x * CB, f = blockIdx.y, g = blockIdx.z;
  const int j0 = g * a.nc / a.groups, j1 = (g + 1) * a.nc / a.groups;  // coils of group g
  const long fs = (long)P * Q;
  const long base = (long)f * fs + (long)c0 * P;
  const int nel = CB * N;
  fft_twiddles<N, kCoilNT>(twt, a.tw64);
  auto at = [&](int e) { return (e / N) * BS + fft_pidx(e % N); };
  double2 acc[EPT], y[EPT];
  float2 cj[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kCoilNT;
    acc[u] = make_double2(0.0, 0.0);
    if (e < nel) {
      y[u] = a.Y64[(long)j0 * a.vstride + base + e];
      cj[u] = a.Ct[(long)j0 * fs + (long)c0 * P + e];
    }
  }
  for (int j = j0; j < j1; ++j) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kCoilNT;
      if (e < nel) lds[at(e)] = y[u];
    }
    float2 cur[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) cur[u] = cj[u];
    if (j + 1 < j1) {  // next coil in flight during this transform
      const double2* Yn = a.Y64 + (long)(j + 1) * a.vstride + base;
      const float2* Cn = a.Ct + (long)(j + 1) * fs + (long)c0 * P;
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = threadIdx.x + u * kCoilNT;
        if (e < nel) {
          y[u] = Yn[e];
          cj[u] = Cn[e];
        }
      }
    }
    __syncthreads();
    fft_lds<N, +1, CAP, kCoilNT>(lds, twt, CB);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * kCoilNT;
      if (e < nel) acc[u] = cadd(acc[u], cmul(cconj(f2d(cur[u])), lds[at(e)]));
    }
    // each thread reads back only its own elements, which it alone overwrites next
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kCoilNT;
    if (e < nel) lds[at(e)] = cscale(acc[u], a.cscale64);
  }
  __syncthreads();
  fft_lds<N, -1, CAP, kCoilNT>(lds, twt, CB);
  double2* dg = a.d64 + (long)g * a.vstride;
  for (int e = threadIdx.x; e < nel; e += kCoilNT) dg[base + e] = lds[at(e)];
}

// ---------------------------------------------------------------- launches
template <int N>
static hipError_t coil_cols_n(const CoilArgs& a, hipStream_t s) {
  const int cb = coil_col_block(CoilCap<N>::v, a.Q);
  k_coil_cols<N><<<dim3(a.Q / cb, a.T, a.nc), kCoilNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_coil_cols(const CoilArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.P, coil_cols_n, a, s) }

template <int N>
static hipError_t coil_combine_n(const CoilArgs& a, hipStream_t s) {
  const int cb = coil_col_block(CoilCap<N>::v, a.Q);
  k_coil_combine<N><<<dim3(a.Q / cb, a.T, a.groups), kCoilNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_coil_combine(const CoilArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.P, coil_combine_n, a, s) }

template <int N>
static hipError_t coil_rows_n(const CoilArgs& a, hipStream_t s) {
  const int rb = a.P < kCoilRB ? a.P : kCoilRB;
  k_coil_rows<N><<<dim3(a.P / rb, a.T, a.nc), kCoilNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_coil_rows(const CoilArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.Q, coil_rows_n, a, s) }

template <int N>
static hipError_t coil_rhs_rows_n(const CoilArgs& a, hipStream_t s) {
  const int rb = a.P < kCoilRB ? a.P : kCoilRB;
  k_coil_rhs_rows<N><<<dim3(a.P / rb, a.T, a.nc), kCoilNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_coil_rhs_rows(const CoilArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.Q, coil_rhs_rows_n, a, s) }

template <int N>
static hipError_t coil_rhs_fin_n(const CoilArgs& a, hipStream_t s) {
  const int rb = a.P < kCoilRB ? a.P : kCoilRB;
  k_coil_rhs_fin<N><<<dim3(a.P / rb, a.T), kCoilNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_coil_rhs_fin(const CoilArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.Q, coil_rhs_fin_n, a, s) }


}  // namespace slrx
