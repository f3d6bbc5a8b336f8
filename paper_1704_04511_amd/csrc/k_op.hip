// CG operator kernels in k-space (Sec. III.A, eq. "eq:grad_ls"):
//   A v = S o v + lam F G F^-1 v,
// F the unitary 2-D DFT per frame and G the per-pixel penalty that couples the
// T frames of a pixel through the M x M masks E_r (summed filter power spectra
// of the weight update).  Keeping the data term S o v exact in k-space means
// FFT round-off only enters through the lam-scaled penalty.
//
// One operator application is three passes over the volume:
//   1. rows:    inverse row DFT of v (fused CG direction update p = r + beta p),
//               written with each frame transposed ([t][col][row]);
//   2. columns: inverse column DFT, G over all T frames of each pixel (scaled
//               by lam / (P Q)), forward column DFT -- a block holds every
//               frame of its columns in LDS;
//   3. rows:    forward row DFT back to row-major, plus S o v and the partial
//               dot product <v, A v> (or r = b - A x for the initial residual).
// Plain unitary 2-D transforms (images for the Gram matrix, outputs) reuse
// pass 1 and a column pass that writes row-major.
#include "common.h"
#include "fft.h"
#include "kernels.h"

namespace slrx {

constexpr int kNT = 256;
constexpr int kTMax = 32;  // frames handled by the column penalty pass
constexpr int kMMax = 8;   // taps

bool fft_len_supported(int n) {
  switch (n) {
    case 8: case 16: case 32: case 64: case 96: case 128: case 160: case 192: case 256: return true;
    default: return false;
  }
}
int max_frames() { return kTMax; }
int max_taps() { return kMMax; }

// Rows per block of the row passes (a tile of RB rows x N columns).
__host__ __device__ inline int row_block(int P) { return P < 16 ? P : 16; }

// Columns per block of the column penalty pass: largest power of two with
// CB * N <= 256 that divides Q.
template <int N> struct ColCap { static constexpr int v = (256 / N) < 1 ? 1 : (256 / N > 32 ? 32 : 256 / N); };
__host__ __device__ inline int col_block(int cap, int Q) {
  int cb = 1;
  while (cb * 2 <= cap) cb *= 2;
  while (cb > 1 && (Q % cb) != 0) cb >>= 1;
  return cb;
}

// ------------------------------------------------------------ pass 1: rows
// Row DFT of RB rows of one frame; output transposed: dst[t][c][r].
template <int N, int SIGN>
__global__ __launch_bounds__(kNT) void k_rows_t(RowArgs a) {
  constexpr int RBMAX = 16;
  __shared__ float2 lds[RBMAX * N];
  __shared__ float2 tw[N];
  __shared__ double red[kNT / 64];
  const int P = a.P, Q = a.Q;
  const int RB = row_block(P);
  const int t = blockIdx.y;
  const int r0 = blockIdx.x * RB;
  const long fo = (long)t * P * Q;
  const long g0 = fo + (long)r0 * Q;
  const int nel = RB * N;
  for (int i = threadIdx.x; i < N; i += kNT) tw[i] = a.tw[i];

  if (a.mode == ROW_PUPDATE) {
    const double rr = reduce_partials<kNT>(a.part, a.npart, red);
    double beta = 0.0;
    if (a.k > 0) {
      const double prev = a.rr_hist[a.k - 1];
      beta = prev > 0.0 ? rr / prev : 0.0;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.rr_hist[a.k] = rr;
    const float fb = (float)beta;
    constexpr int U = 8;  // loads in flight per thread
    for (int e0 = threadIdx.x; e0 < nel; e0 += kNT * U) {
      float2 v[U], po[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT;
        if (e < nel) {
          v[u] = a.src[g0 + e];
          po[u] = a.k > 0 ? a.pvec[g0 + e] : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * kNT;
        if (e < nel) {
          const float2 pv = make_float2(v[u].x + fb * po[u].x, v[u].y + fb * po[u].y);
          a.pvec[g0 + e] = pv;
          lds[e] = pv;
        }
      }
    }
  } else if (a.mode == ROW_MASKED) {
    for (int e = threadIdx.x; e < nel; e += kNT) {
      const float2 v = a.src[g0 + e];
      lds[e] = a.S[g0 + e] ? v : make_float2(0.f, 0.f);
    }
  } else {
    for (int e = threadIdx.x; e < nel; e += kNT) lds[e] = a.src[g0 + e];
  }
  __syncthreads();
  fft_lds<N, SIGN, RBMAX, kNT, 1, N, false>(lds, tw, RB);
  const float sc = a.scale;
  // transposed store: consecutive threads take consecutive rows of one column
  for (int e = threadIdx.x; e < nel; e += kNT) {
    const int i = e % RB, c = e / RB;
    a.dst[fo + (long)c * P + r0 + i] = cscale(lds[i * N + c], sc);
  }
}

// -------------------------------------------------- pass 2: columns + penalty
// Block: CB columns of all T frames, each column a contiguous transform of
// length N = P in the transposed layout.  Inverse column DFT, G, forward DFT.
template <int N, int M>
__global__ __launch_bounds__(kNT) void k_cols_pen(PenArgs a) {
  constexpr int CAP = ColCap<N>::v;
  constexpr int MAXB = kTMax * CAP;
  constexpr int W = M * (M + 1) / 2;
  extern __shared__ float2 lds[];  // [T][CB][N]
  __shared__ float2 tw[N];
  const int T = a.T, P = a.P, Q = a.Q;
  const int CB = col_block(CAP, Q);
  const int c0 = blockIdx.x * CB;
  const long fs = (long)P * Q;
  for (int i = threadIdx.x; i < N; i += kNT) tw[i] = a.tw[i];
  const int per_t = CB * N;  // <= kNT: one pixel per thread
  const int pix = threadIdx.x;
  const bool has_pix = pix < per_t;
  const long po = (long)c0 * P + pix;  // pixel (row pix % N, column c0 + pix / N) in a frame
  {
    float2 v[kTMax];
#pragma unroll
    for (int t = 0; t < kTMax; ++t) v[t] = (has_pix && t < T) ? a.buf[(long)t * fs + po] : make_float2(0.f, 0.f);
    if (has_pix)
#pragma unroll
      for (int t = 0; t < kTMax; ++t)
        if (t < T) lds[t * per_t + pix] = v[t];
  }
  // this pixel's masks, stored [w][c][r]; loaded now so they arrive during the transform
  float2 e[W];
#pragma unroll
  for (int w = 0; w < W; ++w) e[w] = has_pix ? a.Et[(long)w * fs + po] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lds<N, +1, MAXB, kNT, 1, N, false>(lds, tw, T * CB);

  const float sc = a.scale;  // lam / (P Q)
  if (has_pix) {
    float2 z[M], acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      z[m] = lds[(M - 1 - m) * per_t + pix];  // z[m] = rho_{n-m}, n = M-1
      acc[m] = make_float2(0.f, 0.f);
    }
    for (int n = M - 1; n < T; ++n) {
      if (n > M - 1) {
#pragma unroll
        for (int m = M - 1; m > 0; --m) z[m] = z[m - 1];
        z[0] = lds[n * per_t + pix];
      }
      // acc[m] (output frame n - m) += sum_m' E[m][m'] z[m']
#pragma unroll
      for (int m = 0; m < M; ++m) {
        float2 s = acc[m];
#pragma unroll
        for (int mp = 0; mp < M; ++mp) {
          const float2 em = (m <= mp) ? e[pair_id(m, mp, M)] : cconj(e[pair_id(mp, m, M)]);
          s = make_float2(s.x + em.x * z[mp].x - em.y * z[mp].y, s.y + em.x * z[mp].y + em.y * z[mp].x);
        }
        acc[m] = s;
      }
      // frame n - M + 1 is complete; its input already sits in registers (z)
      lds[(n - M + 1) * per_t + pix] = cscale(acc[M - 1], sc);
#pragma unroll
      for (int m = M - 1; m > 0; --m) acc[m] = acc[m - 1];
      acc[0] = make_float2(0.f, 0.f);
    }
    // frames T-1-m, m = 0..M-2
#pragma unroll
    for (int m = 0; m < M - 1; ++m) lds[(T - 1 - m) * per_t + pix] = cscale(acc[m + 1], sc);
  }
  __syncthreads();
  fft_lds<N, -1, MAXB, kNT, 1, N, false>(lds, tw, T * CB);
  if (has_pix)
    for (int t = 0; t < T; ++t) a.buf[(long)t * fs + po] = lds[t * per_t + pix];
}

// Plain column DFT of up to 16 columns of one frame: transposed in, row-major out.
template <int N, int SIGN>
__global__ __launch_bounds__(kNT) void k_cols_plain(ColArgs a) {
  constexpr int CB = 16;
  __shared__ float2 lds[CB * N];
  __shared__ float2 tw[N];
  const int P = a.P, Q = a.Q;
  const int cb = Q < CB ? Q : CB;
  const int t = blockIdx.y;
  const int c0 = blockIdx.x * cb;
  const long fo = (long)t * P * Q;
  for (int i = threadIdx.x; i < N; i += kNT) tw[i] = a.tw[i];
  for (int e = threadIdx.x; e < cb * N; e += kNT) lds[e] = a.src[fo + (long)c0 * P + e];  // [cc][r]
  __syncthreads();
  fft_lds<N, SIGN, CB, kNT, 1, N, false>(lds, tw, cb);
  const float sc = a.scale;
  // row-major store: consecutive threads take consecutive columns of one row
  for (int e = threadIdx.x; e < cb * N; e += kNT) {
    const int cc = e % cb, r = e / cb;
    a.dst[fo + (long)r * Q + c0 + cc] = cscale(lds[cc * N + r], sc);
  }
}

// ----------------------------------------------- pass 3: rows + combine + dot
// Forward row DFT of RB rows of frame t read from the transposed layout, then
//   init: r = b - (S o x + pen), partial <r, r>;   else: q = S o p + pen, partial <p, q>.
template <int N>
__global__ __launch_bounds__(kNT) void k_rows_fin(FinArgs a) {
  constexpr int RBMAX = 16;
  __shared__ float2 lds[RBMAX * N];
  __shared__ float2 tw[N];
  __shared__ double red[kNT / 64];
  const int P = a.P, Q = a.Q;
  const int RB = row_block(P);
  const int t = blockIdx.y;
  const int r0 = blockIdx.x * RB;
  const long fo = (long)t * P * Q;
  const int nel = RB * N;
  for (int i = threadIdx.x; i < N; i += kNT) tw[i] = a.tw[i];
  constexpr int UR = RBMAX * N / kNT < 16 ? RBMAX * N / kNT : 16;
  constexpr int U = UR < 1 ? 1 : UR;  // elements per thread held in registers
  const long g0 = fo + (long)r0 * Q;
  {
    float2 tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kNT;
      if (e < nel) tv[u] = a.t[fo + (long)(e / RB) * P + r0 + e % RB];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kNT;
      if (e < nel) lds[(e % RB) * N + e / RB] = tv[u];
    }
    for (int e = threadIdx.x + U * kNT; e < nel; e += kNT) lds[(e % RB) * N + e / RB] = a.t[fo + (long)(e / RB) * P + r0 + e % RB];
  }
  // the operands of the combine step, loaded before the transform
  float2 vv[U], yv[U];
  uint8_t sv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * kNT;
    if (e < nel) {
      vv[u] = a.v[g0 + e];
      sv[u] = a.S[g0 + e];
      yv[u] = a.init ? a.y[g0 + e] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  fft_lds<N, -1, RBMAX, kNT, 1, N, false>(lds, tw, RB);
  double dot = 0.0;
  auto combine = [&](int e, float2 v, uint8_t sm, float2 bv) {
    const long g = g0 + e;
    const float2 pen = lds[e];
    const float2 av = sm ? make_float2(v.x + pen.x, v.y + pen.y) : pen;
    if (a.init) {
      const float2 rv = make_float2(bv.x - av.x, bv.y - av.y);
      a.out[g] = rv;
      dot += (double)rv.x * rv.x + (double)rv.y * rv.y;
    } else {
      a.out[g] = av;
      dot += (double)v.x * av.x + (double)v.y * av.y;
    }
  };
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * kNT;
    if (e < nel) combine(e, vv[u], sv[u], yv[u]);
  }
  for (int e = threadIdx.x + U * kNT; e < nel; e += kNT)
    combine(e, a.v[g0 + e], a.S[g0 + e], a.init ? a.y[g0 + e] : make_float2(0.f, 0.f));
  dot = block_sum<kNT>(dot, red);
  if (threadIdx.x == 0) {
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    a.part[bid] = dot;
    if (a.init && bid == 0) *a.flag = 0;
  }
}

// --------------------------------------------------------------- update
// Two complex elements per 16-byte access, kUpdU accesses per thread in flight.
constexpr int kUpdU = 4;
__global__ __launch_bounds__(kNT) void k_update(UpdArgs a) {
  __shared__ double red[kNT / 64];
  const double pq = reduce_partials<kNT>(a.partA, a.nA, red);
  const double rr = a.rr_hist[a.k];
  const bool stop = (*a.flag != 0) || !(rr > 0.0) || !(pq > 0.0);
  const float al = stop ? 0.f : (float)(rr / pq);
  const long n4 = a.n / 2;  // float4 count (the volume has an even element count)
  float4* x4 = (float4*)a.x;
  float4* r4 = (float4*)a.r;
  const float4* p4 = (const float4*)a.p;
  const float4* q4 = (const float4*)a.q;
  double acc = 0.0;
  const long stride = (long)gridDim.x * kNT;
  for (long b = (long)blockIdx.x * kNT + threadIdx.x; b < n4; b += stride * kUpdU) {
    float4 rv[kUpdU], xv[kUpdU], pv[kUpdU], qv[kUpdU];
#pragma unroll
    for (int u = 0; u < kUpdU; ++u) {
      const long i = b + u * stride;
      if (i < n4) {
        rv[u] = r4[i];
        if (!stop) {
          xv[u] = x4[i];
          pv[u] = p4[i];
          qv[u] = q4[i];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kUpdU; ++u) {
      const long i = b + u * stride;
      if (i >= n4) continue;
      float4 ri = rv[u];
      if (!stop) {
        const float4 xi = make_float4(xv[u].x + al * pv[u].x, xv[u].y + al * pv[u].y, xv[u].z + al * pv[u].z,
                                      xv[u].w + al * pv[u].w);
        ri = make_float4(ri.x - al * qv[u].x, ri.y - al * qv[u].y, ri.z - al * qv[u].z, ri.w - al * qv[u].w);
        x4[i] = xi;
        r4[i] = ri;
      }
      acc += (double)ri.x * ri.x + (double)ri.y * ri.y + (double)ri.z * ri.z + (double)ri.w * ri.w;
    }
  }
  acc = block_sum<kNT>(acc, red);
  if (threadIdx.x == 0) {
    a.partB[blockIdx.x] = acc;
    if (stop && blockIdx.x == 0) *a.flag = 1;
  }
}

__global__ void k_mask_data(long n, const uint8_t* S, const float2* b, float2* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = S[i] ? b[i] : make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(kNT) void k_store_sum(const double* part, int n, double* dst) {
  __shared__ double red[kNT / 64];
  const double v = reduce_partials<kNT>(part, n, red);
  if (threadIdx.x == 0) *dst = v;
}

__global__ void k_interleave(long n, const double* re, const double* im, double2* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2(re[i], im[i]);
}

// W planes: out[w][j][i] = in[w][i][j] for A x B input planes (complex64).
__global__ void k_transpose_planes(int W, int A, int B, const float2* in, float2* out) {
  const long n = (long)W * A * B;
  const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const long w = o / ((long)A * B);
  const int rem = (int)(o % ((long)A * B));
  const int j = rem / A, i = rem % A;  // output index [w][j][i]
  out[o] = in[(w * A + i) * B + j];
}

// --------------------------------------------------------------- launches
#define SLRX_DISPATCH_N(n, F, ...)            \
  switch (n) {                                \
    case 8: return F<8>(__VA_ARGS__);         \
    case 16: return F<16>(__VA_ARGS__);       \
    case 32: return F<32>(__VA_ARGS__);       \
    case 64: return F<64>(__VA_ARGS__);       \
    case 96: return F<96>(__VA_ARGS__);       \
    case 128: return F<128>(__VA_ARGS__);     \
    case 160: return F<160>(__VA_ARGS__);     \
    case 192: return F<192>(__VA_ARGS__);     \
    case 256: return F<256>(__VA_ARGS__);     \
  }                                           \
  return hipErrorInvalidValue;

template <int N>
static hipError_t rows_t_n(const RowArgs& a, hipStream_t s) {
  dim3 grid(a.P / row_block(a.P), a.T);
  if (a.sign < 0) k_rows_t<N, -1><<<grid, kNT, 0, s>>>(a);
  else k_rows_t<N, +1><<<grid, kNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_rows(const RowArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.Q, rows_t_n, a, s) }

template <int N>
static hipError_t cols_plain_n(const ColArgs& a, hipStream_t s) {
  const int cb = a.Q < 16 ? a.Q : 16;
  dim3 grid(a.Q / cb, a.T);
  if (a.sign < 0) k_cols_plain<N, -1><<<grid, kNT, 0, s>>>(a);
  else k_cols_plain<N, +1><<<grid, kNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_cols(const ColArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.P, cols_plain_n, a, s) }

template <int N, int M>
static hipError_t pen_nm(const PenArgs& a, hipStream_t s) {
  const int cb = col_block(ColCap<N>::v, a.Q);
  const size_t lds = (size_t)a.T * cb * N * sizeof(float2);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cols_pen<N, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((size_t)kTMax * ColCap<N>::v * N * sizeof(float2)));
    if (e != hipSuccess) return e;
    attr = true;
  }
  k_cols_pen<N, M><<<dim3(a.Q / cb), kNT, lds, s>>>(a);
  return hipGetLastError();
}

template <int N>
static hipError_t pen_n(const PenArgs& a, hipStream_t s) {
  switch (a.M) {
    case 1: return pen_nm<N, 1>(a, s);
    case 2: return pen_nm<N, 2>(a, s);
    case 3: return pen_nm<N, 3>(a, s);
    case 4: return pen_nm<N, 4>(a, s);
    case 5: return pen_nm<N, 5>(a, s);
    case 6: return pen_nm<N, 6>(a, s);
    case 7: return pen_nm<N, 7>(a, s);
    case 8: return pen_nm<N, 8>(a, s);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_pen(const PenArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.P, pen_n, a, s) }

template <int N>
static hipError_t fin_n(const FinArgs& a, hipStream_t s) {
  dim3 grid(a.P / row_block(a.P), a.T);
  k_rows_fin<N><<<grid, kNT, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_fin(const FinArgs& a, hipStream_t s) { SLRX_DISPATCH_N(a.Q, fin_n, a, s) }

int fin_blocks(int P, int T) { return (P / row_block(P)) * T; }

int update_blocks(long n) {
  long b = (n / 2 + (long)kNT * kUpdU - 1) / ((long)kNT * kUpdU);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_update(const UpdArgs& a, hipStream_t s) {
  k_update<<<update_blocks(a.n), kNT, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_mask_data(long n, const uint8_t* S, const float2* b, float2* out, hipStream_t s) {
  k_mask_data<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, S, b, out);
  return hipGetLastError();
}

hipError_t launch_store_sum(const double* part, int n, double* dst, hipStream_t s) {
  k_store_sum<<<1, kNT, 0, s>>>(part, n, dst);
  return hipGetLastError();
}

hipError_t launch_interleave(long n, const double* re, const double* im, double2* out, hipStream_t s) {
  k_interleave<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, re, im, out);
  return hipGetLastError();
}

hipError_t launch_transpose_planes(int W, int A, int B, const float2* in, float2* out, hipStream_t s) {
  const long n = (long)W * A * B;
  k_transpose_planes<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(W, A, B, in, out);
  return hipGetLastError();
}

}  // namespace slrx
