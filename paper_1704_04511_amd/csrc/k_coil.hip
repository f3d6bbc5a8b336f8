// Multichannel data term of the CG operator (Sec. II.A, eq. "measurement_ij").
//
// With coil sensitivities C_j the least-squares step applies
//   A^H A v = F sum_j C_j^* F^-1 (S o F (C_j F^-1 v))
// instead of S o v.  The operator keeps its row pass (inverse row DFT of v,
// transposed output) and gains three passes before its column pass:
//   1. k_coil_cols (per column tile, frame and coil): the inverse column DFT
//      gives the image rho_u = IDFT2(v) (kept for the penalty by coil 0), then
//      the forward column DFT of C_j rho_u;
//   2. k_coil_rows (per k-space row tile, frame and coil): forward row DFT, the
//      frame's sampling mask, inverse row DFT;
//   3. k_coil_combine (per column tile, frame and group of coils): the coil
//      combination d_g = (PQ)^-2 sum_{j in group g} conj(C_j) IDFT_col(Y_j),
//      one coil after another with the next coil's loads in flight during the
//      current transform;
// and the column pass (k_cols_pen, coil mode) adds d_0 + d_1 + ... (in that
// order) to the penalty before its forward column DFT.  All transforms here
// are unnormalised; the (PQ)^-2 makes the composition the unitary operator.
// Volumes use the transposed layout of the column pass ([t][c][r]); the coil
// maps are stored transposed per coil ([j][c][r]).
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
// layout; forward row DFT, sampling mask S (row-major [t][kr][kc]), inverse
// row DFT, stored back in place.
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_rows(CoilArgs a) {
  constexpr int BS = fft_stride(N);
  __shared__ float2 lds[kCoilRB * BS];
  __shared__ float2 twt[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int RB = P < kCoilRB ? P : kCoilRB;
  const int r0 = blockIdx.x * RB, f = blockIdx.y, j = blockIdx.z;
  const long fs = (long)P * Q;
  float2* Y = a.Y + (long)j * a.vstride + (long)f * fs;
  const uint8_t* S = a.S + (long)f * fs;
  const int nel = RB * N;
  fft_twiddles<N, kCoilNT>(twt, a.tw);
  // element e: column c = e / RB, row r0 + e % RB (consecutive threads walk a column)
  for (int e = threadIdx.x; e < nel; e += kCoilNT)
    lds[(e % RB) * BS + fft_pidx(e / RB)] = Y[(long)(e / RB) * P + r0 + e % RB];
  __syncthreads();
  fft_lds<N, -1, kCoilRB, kCoilNT>(lds, twt, RB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT) {
    const int i = e / N, kc = e % N;
    if (!S[(long)(r0 + i) * Q + kc]) lds[i * BS + fft_pidx(kc)] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<N, +1, kCoilRB, kCoilNT>(lds, twt, RB);
  for (int e = threadIdx.x; e < nel; e += kCoilNT)
    Y[(long)(e / RB) * P + r0 + e % RB] = lds[(e % RB) * BS + fft_pidx(e / RB)];
}

// ---------------------------------------------------- pass 3: coil combine
// Block: CB columns of one frame and one group g of coils (a balanced split of
// the coils into the groups of the grid's z dimension).
// d_g = cscale sum_{j in g} conj(C_j) IDFT_col(Y_j), coils in order (a fixed
// summation order); each thread keeps the sums of its elements in registers
// and loads coil j+1 while coil j is transformed.
template <int N>
__global__ __launch_bounds__(kCoilNT) void k_coil_combine(CoilArgs a) {
  constexpr int CAP = CoilCap<N>::v;
  constexpr int BS = fft_stride(N);
  constexpr int EPT = (CAP * N + kCoilNT - 1) / kCoilNT;  // elements per thread
  __shared__ float2 lds[CAP * BS];
  __shared__ float2 twt[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int CB = coil_col_block(CAP, Q);
  const int c0 = blockIdx.x * CB, f = blockIdx.y, g = blockIdx.z;
  const int j0 = g * a.nc / a.groups, j1 = (g + 1) * a.nc / a.groups;  // coils of group g
  const long fs = (long)P * Q;
  const long base = (long)f * fs + (long)c0 * P;
  const int nel = CB * N;
  fft_twiddles<N, kCoilNT>(twt, a.tw);
  auto at = [&](int e) { return (e / N) * BS + fft_pidx(e % N); };
  float2 acc[EPT], y[EPT], cj[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kCoilNT;
    acc[u] = make_float2(0.f, 0.f);
    if (e < nel) {
      y[u] = a.Y[(long)j0 * a.vstride + base + e];
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
      const float2* Yn = a.Y + (long)(j + 1) * a.vstride + base;
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
      if (e < nel) acc[u] = cadd(acc[u], cmul(cconj(cur[u]), lds[at(e)]));
    }
  }
  float2* dg = a.d + (long)g * a.vstride;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * kCoilNT;
    if (e < nel) dg[base + e] = cscale(acc[u], a.cscale);
  }
}

// acc (+)= conj(C_j) o w over a row-major volume; C_j stored transposed [c][r].
__global__ void k_coil_acc(long n, int P, int Q, const float2* Ct, const float2* w, float2* acc, int assign) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long pq = (long)P * Q;
  const long rc = i % pq;
  const int r = (int)(rc / Q), c = (int)(rc % Q);
  const float2 v = cmul(cconj(Ct[(long)c * P + r]), w[i]);
  acc[i] = assign ? v : cadd(acc[i], v);
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

hipError_t launch_coil_acc(long n, int P, int Q, const float2* Ct, const float2* w, float2* acc, bool assign,
                           hipStream_t s) {
  k_coil_acc<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, P, Q, Ct, w, acc, assign ? 1 : 0);
  return hipGetLastError();
}

}  // namespace slrx
