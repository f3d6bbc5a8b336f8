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
// With coil maps (k_coil.hip) the column pass takes the image from the coil
// passes instead of inverting the columns itself, and pass 3 adds the data
// term A^H A v (its complex128 last row transform) in place of S o v.  With the GIRAF option G is circulant along the
// frames.  Plain unitary 2-D transforms (images for the Gram matrix, outputs)
// reuse pass 1 and a column pass that writes row-major.
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

// Rows per block of the row passes (a tile of RB rows x N columns).  Eight
// rows keep the transposed stores at 64-byte pieces and give 2.5 blocks per CU
// at 256 x 256 x 20 rather than 1.25.
constexpr int kRowB = 8;
__host__ __device__ inline int row_block(int P) { return P < kRowB ? P : kRowB; }

// Block -> (row band, frame) of the row passes.  Blocks are dealt to the 8
// XCDs round-robin; consecutive work items are given to one XCD, so the two
// halves of a 128-byte line of the transposed output (neighbouring bands)
// meet in the same L2.
// A block's coordinates in the grid of its problem: the launch's own grid, or a
// slice of a grouped launch covering several problems (every problem's blocks
// then do exactly what they do in a launch of their own).
struct Blk {
  int bx, by, gx, gy;
};
SLRX_DEV Blk launch_blk() { return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y}; }

SLRX_DEV void row_tile(const Blk& b, int& band, int& frame) {
  const int gx = b.gx, nb = b.gx * b.gy;
  int id = b.by * gx + b.bx;
  if ((nb & 7) == 0) id = (id & 7) * (nb >> 3) + (id >> 3);
  band = id % gx;
  frame = id / gx;
}

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
SLRX_DEV void rows_t_body(const RowArgs& a, const Blk& b, float2* lds, float2* twt, double* red) {
  constexpr int RBMAX = kRowB;
  constexpr int BS = fft_stride(N);
  const int P = a.P, Q = a.Q;
  const int RB = row_block(P);
  int band, t;
  row_tile(b, band, t);
  const int r0 = band * RB;
  const long fo = (long)t * P * Q;
  const long g0 = fo + (long)r0 * Q;
  const int nel = RB * N;
  fft_twiddles<N, kNT>(twt, a.tw);
  auto at = [&](int e) { return (e / N) * BS + fft_pidx(e % N); };  // tile element (row, column) in LDS

  if (a.mode == ROW_PUPDATE) {
    const double rr = reduce_partials<kNT>(a.part, a.npart, red);
    double beta = 0.0;
    if (a.k > 0) {
      const double prev = a.rr_hist[a.k - 1];
      beta = prev > 0.0 ? rr / prev : 0.0;
    }
    if (b.bx == 0 && b.by == 0 && threadIdx.x == 0) a.rr_hist[a.k] = rr;
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
          lds[at(e)] = pv;
        }
      }
    }
  } else if (a.mode == ROW_MASKED) {
    for (int e = threadIdx.x; e < nel; e += kNT) {
      const float2 v = a.src[g0 + e];
      lds[at(e)] = a.S[g0 + e] ? v : make_float2(0.f, 0.f);
    }
  } else {
    for (int e = threadIdx.x; e < nel; e += kNT) lds[at(e)] = a.src[g0 + e];
  }
  __syncthreads();
  fft_lds<N, SIGN, RBMAX, kNT>(lds, twt, RB);
  const float sc = a.scale;
  // transposed store: consecutive threads take consecutive rows of one column
  for (int e = threadIdx.x; e < nel; e += kNT) {
    const int i = e % RB, c = e / RB;
    a.dst[fo + (long)c * P + r0 + i] = cscale(lds[i * BS + fft_pidx(c)], sc);
  }
}

template <int N, int SIGN>
__global__ __launch_bounds__(kNT) void k_rows_t(RowArgs a) {
  __shared__ float2 lds[kRowB * fft_stride(N)];
  __shared__ float2 twt[fft_tw_size<N>()];
  __shared__ double red[kNT / 64];
  rows_t_body<N, SIGN>(a, launch_blk(), lds, twt, red);
}

// -------------------------------------------------- pass 2: columns + penalty
// Block: CB columns of all T frames, each column a contiguous transform of
// length N = P in the transposed layout.  Inverse column DFT, G, forward DFT.
// Two threads per pixel (halves h = 0, 1): frame loads and stores are split
// by frame parity, every transform pass takes one butterfly per thread, and
// the penalty's outputs are split by frame parity.
constexpr int kPenNT = 512;

template <int N, int M>
SLRX_DEV void cols_pen_body(const PenArgs& a, const Blk& b, float2* lds, float2* twt) {
  constexpr int CAP = ColCap<N>::v;
  constexpr int MAXB = kTMax * CAP;
  constexpr int W = M * (M + 1) / 2;
  constexpr int BS = fft_stride(N);
  constexpr int ME = M > 1 ? 2 * M - 2 : 1;  // frames at each end with a partial window
  // lds: [T][CB] transforms of length N, padded
  const int T = a.T, P = a.P, Q = a.Q;
  const int CB = col_block(CAP, Q);
  const int c0 = b.bx * CB;
  const long fs = (long)P * Q;
  fft_twiddles<N, kPenNT>(twt, a.tw);
  const int per_t = CB * BS;  // LDS stride of a frame
  const int pix = threadIdx.x & 255, h = threadIdx.x >> 8;  // CB * N <= 256 pixels
  const bool has_pix = pix < CB * N;
  const int pl = (pix / N) * BS + fft_pidx(pix % N);  // the pixel's slot in a frame
  const long po = (long)c0 * P + pix;  // pixel (row pix % N, column c0 + pix / N) in a frame
  // this pixel's frames of parity h and all of its masks (stored [w][c][r]);
  // the masks are issued with the frames and first used after the transform.
  // With coils the input is the image rho_u itself (no inverse transform).
  const bool coil = a.nc > 0;
  const float2* src = coil ? a.rho : a.buf;
  float2 e[W];
  {
    float2 v[kTMax / 2];
#pragma unroll
    for (int i = 0; i < kTMax / 2; ++i) {
      const int t = 2 * i + h;
      v[i] = (has_pix && t < T) ? src[(long)t * fs + po] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) e[w] = has_pix ? a.Et[(long)w * fs + po] : make_float2(0.f, 0.f);
    if (has_pix)
#pragma unroll
      for (int i = 0; i < kTMax / 2; ++i)
        if (2 * i + h < T) lds[(2 * i + h) * per_t + pl] = v[i];
  }
  __syncthreads();
  if (!coil) fft_lds<N, +1, MAXB, kPenNT>(lds, twt, T * CB);

  // G on this pixel's frames:
  //   (G rho)_t = sum_{n = max(t, M-1)}^{min(t+M-1, T-1)} sum_m' E[n-t][m'] rho_{n-m'}.
  // For M-1 <= t <= T-M every n of the window is present and the sum is
  // Toeplitz in t: (G rho)_t = u_0 rho_t + sum_{d=1}^{M-1} (u_d rho_{t-d} + conj(u_d) rho_{t+d}),
  // u_d = sum_m E[m][m+d] the diagonal sums of E.  The first and last M-1
  // frames keep the windowed sum; when T < 2M-1 there is no Toeplitz part and
  // one thread per pixel runs the windowed sum over all frames.
  const float sc = a.scale;  // lam / (P Q)
  const bool circ = a.circ != 0;
  const bool split = !circ && T >= 2 * M - 1;
  auto mac = [](float2 acc, float2 c, float2 x) {
    return make_float2(acc.x + c.x * x.x - c.y * x.y, acc.y + c.x * x.y + c.y * x.x);
  };
  auto E = [&](int m, int mp) { return (m <= mp) ? e[pair_id(m, mp, M)] : cconj(e[pair_id(mp, m, M)]); };
  float2 rho[kTMax], rt[ME];  // rt[i] = rho_{T-1-i}
  // GIRAF: every window is complete and G is circulant along the frames,
  // (G rho)_t = sum_{d=-(M-1)}^{M-1} g_d rho_{(t+d) mod T}, g_{-d} = u_d, g_d = conj(u_d);
  // outputs of parity h kept in registers until every input is read
  float2 gout[kTMax / 2];
  if (circ && has_pix) {
    float2 u[M];
#pragma unroll
    for (int d = 0; d < M; ++d) {
      float2 s = e[pair_id(0, d, M)];
#pragma unroll
      for (int m = 1; m + d < M; ++m) s = cadd(s, e[pair_id(m, m + d, M)]);
      u[d] = s;
    }
#pragma unroll
    for (int i = 0; i < kTMax / 2; ++i) {
      const int t = 2 * i + h;
      float2 acc = make_float2(0.f, 0.f);
      if (t < T) {
        acc = mac(acc, u[0], lds[t * per_t + pl]);
#pragma unroll
        for (int d = 1; d < M; ++d) {
          const int lo = ((t - d) % T + T) % T, hi = (t + d) % T;
          acc = mac(acc, u[d], lds[lo * per_t + pl]);
          acc = mac(acc, cconj(u[d]), lds[hi * per_t + pl]);
        }
      }
      gout[i] = cscale(acc, sc);
    }
  }
  if (split && has_pix) {
#pragma unroll
    for (int t = 0; t < kTMax; ++t) rho[t] = t < T ? lds[t * per_t + pl] : make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < ME; ++i) rt[i] = lds[(T - 1 - i) * per_t + pl];
  }
  __syncthreads();  // every input read before any output is written in place
  if (circ && has_pix) {
#pragma unroll
    for (int i = 0; i < kTMax / 2; ++i)
      if (2 * i + h < T) lds[(2 * i + h) * per_t + pl] = gout[i];
  }
  if (split && has_pix) {
    float2 u[M];
#pragma unroll
    for (int d = 0; d < M; ++d) {
      float2 s = e[pair_id(0, d, M)];
#pragma unroll
      for (int m = 1; m + d < M; ++m) s = cadd(s, e[pair_id(m, m + d, M)]);
      u[d] = s;
    }
    // first frames t < M-1: n = t + m for m >= M-1-t
#pragma unroll
    for (int t = 0; t < M - 1; ++t) {
      if ((t & 1) != h) continue;
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int m = M - 1 - t; m < M; ++m)
#pragma unroll
        for (int mp = 0; mp < M; ++mp) acc = mac(acc, E(m, mp), rho[t + m - mp]);
      lds[t * per_t + pl] = cscale(acc, sc);
    }
    // Toeplitz part
#pragma unroll
    for (int t = M - 1; t < kTMax; ++t) {
      if (t > T - M || (t & 1) != h) continue;
      float2 acc = mac(make_float2(0.f, 0.f), u[0], rho[t]);
#pragma unroll
      for (int d = 1; d < M; ++d) {
        acc = mac(acc, u[d], rho[t - d]);
        acc = mac(acc, cconj(u[d]), rho[t + d < kTMax ? t + d : kTMax - 1]);
      }
      lds[t * per_t + pl] = cscale(acc, sc);
    }
    // last frames t = T-1-q, q < M-1: n = t + m for m <= q; rho_{t+m-m'} = rt[q-m+m']
#pragma unroll
    for (int q = 0; q < M - 1; ++q) {
      const int t = T - 1 - q;
      if ((t & 1) != h) continue;
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int m = 0; m <= q; ++m)
#pragma unroll
        for (int mp = 0; mp < M; ++mp) acc = mac(acc, E(m, mp), rt[q - m + mp]);
      lds[t * per_t + pl] = cscale(acc, sc);
    }
  } else if (!circ && !split && has_pix && h == 0) {
    // windowed sum over n with a sliding register window: z[m] = rho_{n-m};
    // acc[m] collects output frame n - m, written once complete
    float2 z[M], acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      z[m] = lds[(M - 1 - m) * per_t + pl];
      acc[m] = make_float2(0.f, 0.f);
    }
    for (int n = M - 1; n < T; ++n) {
      if (n > M - 1) {
#pragma unroll
        for (int m = M - 1; m > 0; --m) z[m] = z[m - 1];
        z[0] = lds[n * per_t + pl];
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
#pragma unroll
        for (int mp = 0; mp < M; ++mp) acc[m] = mac(acc[m], E(m, mp), z[mp]);
      }
      lds[(n - M + 1) * per_t + pl] = cscale(acc[M - 1], sc);
#pragma unroll
      for (int m = M - 1; m > 0; --m) acc[m] = acc[m - 1];
      acc[0] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < M - 1; ++m) lds[(T - 1 - m) * per_t + pl] = cscale(acc[m + 1], sc);
  }
  __syncthreads();
  fft_lds<N, -1, MAXB, kPenNT>(lds, twt, T * CB);
  if (has_pix)
    for (int t = h; t < T; t += 2) a.buf[(long)t * fs + po] = lds[t * per_t + pl];
}

template <int N, int M>
__global__ __launch_bounds__(kPenNT) void k_cols_pen(PenArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float2 twt[fft_tw_size<N>()];
  cols_pen_body<N, M>(a, launch_blk(), lds, twt);
}

// Plain column DFT of up to 16 columns of one frame: transposed in, row-major out.
template <int N, int SIGN>
__global__ __launch_bounds__(kNT) void k_cols_plain(ColArgs a) {
  constexpr int CB = 16;
  constexpr int BS = fft_stride(N);
  __shared__ float2 lds[CB * BS];
  __shared__ float2 twt[fft_tw_size<N>()];
  const int P = a.P, Q = a.Q;
  const int cb = Q < CB ? Q : CB;
  const int t = blockIdx.y;
  const int c0 = blockIdx.x * cb;
  const long fo = (long)t * P * Q;
  fft_twiddles<N, kNT>(twt, a.tw);
  for (int e = threadIdx.x; e < cb * N; e += kNT)  // [cc][r]
    lds[(e / N) * BS + fft_pidx(e % N)] = a.src[fo + (long)c0 * P + e];
  __syncthreads();
  fft_lds<N, SIGN, CB, kNT>(lds, twt, cb);
  const float sc = a.scale;
  // row-major store: consecutive threads take consecutive columns of one row
  for (int e = threadIdx.x; e < cb * N; e += kNT) {
    const int cc = e % cb, r = e / cb;
    a.dst[fo + (long)r * Q + c0 + cc] = cscale(lds[cc * BS + fft_pidx(r)], sc);
  }
}

// ----------------------------------------------- pass 3: rows + combine + dot
// Forward row DFT of RB rows of frame t read from the transposed layout, then
//   init: r = b - (S o x + pen), partial <r, r>;   else: q = S o p + pen, partial <p, q>.
// COIL (multichannel data term): no S o x; instead the complex128 forward row
// DFT of the coil combination's group sums is added to pen before rounding.
template <int N, bool COIL>
SLRX_DEV void rows_fin_body(const FinArgs& a, const Blk& b, float2* lds, float2* twt, double2* lds64,
                            double2* twt64, double* red) {
  constexpr int RBMAX = kRowB;
  constexpr int BS = fft_stride(N);
  const int P = a.P, Q = a.Q;
  const int RB = row_block(P);
  int band, t;
  row_tile(b, band, t);
  const int r0 = band * RB;
  const long fo = (long)t * P * Q;
  const int nel = RB * N;
  fft_twiddles<N, kNT>(twt, a.tw);
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
      if (e < nel) lds[(e % RB) * BS + fft_pidx(e / RB)] = tv[u];
    }
    for (int e = threadIdx.x + U * kNT; e < nel; e += kNT)
      lds[(e % RB) * BS + fft_pidx(e / RB)] = a.t[fo + (long)(e / RB) * P + r0 + e % RB];
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
  if constexpr (COIL) fft_twiddles<N, kNT>(twt64, a.tw64);
  __syncthreads();
  fft_lds<N, -1, RBMAX, kNT>(lds, twt, RB);
  if constexpr (COIL) rows_sum_fwd<N, RBMAX, kNT>(lds64, twt64, a.d64, a.dparts, a.dstride, fo, P, r0, RB);
  double dot = 0.0;
  auto combine = [&](int e, float2 v, uint8_t sm, float2 bv) {
    const long g = g0 + e;
    const float2 pen = lds[(e / N) * BS + fft_pidx(e % N)];
    if constexpr (COIL) {  // data term + penalty in complex128, rounded once
      const double2 av = cadd(f2d(pen), lds64[(e / N) * BS + fft_pidx(e % N)]);
      if (a.init) {
        const float2 rv = make_float2((float)((double)bv.x - av.x), (float)((double)bv.y - av.y));
        a.out[g] = rv;
        dot += (double)rv.x * rv.x + (double)rv.y * rv.y;
      } else {
        const float2 q = make_float2((float)av.x, (float)av.y);
        a.out[g] = q;
        dot += (double)v.x * q.x + (double)v.y * q.y;
      }
      return;
    }
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
    const int bid = b.by * b.gx + b.bx;
    a.part[bid] = dot;
    if (a.init && bid == 0) *a.flag = 0;
  }
}

template <int N, bool COIL>
__global__ __launch_bounds__(kNT) void k_rows_fin(FinArgs a) {
  __shared__ float2 lds[kRowB * fft_stride(N)];
  __shared__ float2 twt[fft_tw_size<N>()];
  __shared__ double2 lds64[COIL ? kRowB * fft_stride(N) : 1];
  __shared__ double2 twt64[COIL ? fft_tw_size<N>() : 1];
  __shared__ double red[kNT / 64];
  rows_fin_body<N, COIL>(a, launch_blk(), lds, twt, lds64, twt64, red);
}

// --------------------------------------------------------------- update
// Two complex elements per 16-byte access, kUpdU accesses per thread in flight.
constexpr int kUpdU = 4;
SLRX_DEV void update_body(const UpdArgs& a, const Blk& b, double* red) {
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
  const long stride = (long)b.gx * kNT;
  for (long i0 = (long)b.bx * kNT + threadIdx.x; i0 < n4; i0 += stride * kUpdU) {
    float4 rv[kUpdU], xv[kUpdU], pv[kUpdU], qv[kUpdU];
#pragma unroll
    for (int u = 0; u < kUpdU; ++u) {
      const long i = i0 + u * stride;
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
      const long i = i0 + u * stride;
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
    a.partB[b.bx] = acc;
    if (stop && b.bx == 0) *a.flag = 1;
  }
}

__global__ __launch_bounds__(kNT) void k_update(UpdArgs a) {
  __shared__ double red[kNT / 64];
  update_body(a, launch_blk(), red);
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

// ------------------------------------------------ grouped launches (batches)
// One launch of a CG pass for every problem of a group (problems of any frame
// size and count that share the tap count M).  The grid is the concatenation
// of the problems' own grids, each starting at a multiple of 8 blocks (so a
// block keeps its XCD); a block finds its problem in the group's table and
// runs exactly the work, with exactly the same arithmetic and partial-sum
// slots, that it runs in a launch for that problem alone.
constexpr int kTwMax = fft_tw_size<256>() > fft_tw_size<192>()
                           ? (fft_tw_size<256>() > fft_tw_size<160>() ? fft_tw_size<256>() : fft_tw_size<160>())
                           : (fft_tw_size<192>() > fft_tw_size<160>() ? fft_tw_size<192>() : fft_tw_size<160>());
static_assert(kTwMax >= fft_tw_size<128>() && kTwMax >= fft_tw_size<96>() && kTwMax >= fft_tw_size<64>(),
              "twiddle table of the grouped passes");

// Largest LDS row count of a column block over the transform lengths (CB * stride).
constexpr int pen_cols(int cap, int n) { return cap * fft_stride(n); }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kPenCols = cmax(cmax(cmax(pen_cols(ColCap<8>::v, 8), pen_cols(ColCap<16>::v, 16)),
                                   cmax(pen_cols(ColCap<32>::v, 32), pen_cols(ColCap<64>::v, 64))),
                              cmax(cmax(pen_cols(ColCap<96>::v, 96), pen_cols(ColCap<128>::v, 128)),
                                   cmax(cmax(pen_cols(ColCap<160>::v, 160), pen_cols(ColCap<192>::v, 192)),
                                        pen_cols(ColCap<256>::v, 256))));

SLRX_DEV int group_slice(const CgSlice* tab, int ns, int gb, int CgSlice::*start) {
  int i = 0;
  while (i + 1 < ns && gb >= tab[i + 1].*start) ++i;
  return i;
}

#define SLRX_SWITCH_N(n, ...)                                                 \
  switch (n) {                                                                \
    case 8: { constexpr int N_ = 8; __VA_ARGS__; } break;                     \
    case 16: { constexpr int N_ = 16; __VA_ARGS__; } break;                   \
    case 32: { constexpr int N_ = 32; __VA_ARGS__; } break;                   \
    case 64: { constexpr int N_ = 64; __VA_ARGS__; } break;                   \
    case 96: { constexpr int N_ = 96; __VA_ARGS__; } break;                   \
    case 128: { constexpr int N_ = 128; __VA_ARGS__; } break;                 \
    case 160: { constexpr int N_ = 160; __VA_ARGS__; } break;                 \
    case 192: { constexpr int N_ = 192; __VA_ARGS__; } break;                 \
    case 256: { constexpr int N_ = 256; __VA_ARGS__; } break;                 \
  }

// mode ROW_PLAIN: x into the row pass (initial residual); ROW_PUPDATE: p = r + beta p.
__global__ __launch_bounds__(kNT) void k_group_rows(const CgSlice* tab, int ns, int mode, int k) {
  __shared__ float2 lds[kRowB * fft_stride(256)];
  __shared__ float2 twt[kTwMax];
  __shared__ double red[kNT / 64];
  const int gb = (int)blockIdx.x;
  const CgSlice& c = tab[group_slice(tab, ns, gb, &CgSlice::rows0)];
  const int lb = gb - c.rows0;
  if (lb >= c.rows_gx * c.rows_gy) return;  // alignment padding
  const Blk b{lb % c.rows_gx, lb / c.rows_gx, c.rows_gx, c.rows_gy};
  RowArgs a{};
  a.P = c.P; a.Q = c.Q; a.T = c.T;
  a.mode = mode;
  a.sign = +1;
  a.src = mode == ROW_PUPDATE ? c.r : c.x;
  a.pvec = c.p;
  a.dst = c.t;
  a.scale = 1.0f;
  a.tw = c.twQ;
  a.k = k;
  a.part = k == 0 ? c.partA : c.partB;
  a.npart = k == 0 ? c.nfin : c.nupd;
  a.rr_hist = c.rr_hist;
  SLRX_SWITCH_N(c.Q, rows_t_body<N_, +1>(a, b, lds, twt, red))
}

template <int M>
__global__ __launch_bounds__(kPenNT) void k_group_pen(const CgSlice* tab, int ns) {
  extern __shared__ float2 lds[];
  __shared__ float2 twt[kTwMax];
  const int gb = (int)blockIdx.x;
  const CgSlice& c = tab[group_slice(tab, ns, gb, &CgSlice::cols0)];
  const int lb = gb - c.cols0;
  if (lb >= c.cols_gx) return;
  const Blk b{lb, 0, c.cols_gx, 1};
  PenArgs a{};
  a.P = c.P; a.Q = c.Q; a.T = c.T; a.M = M;
  a.buf = c.t;
  a.Et = c.Et;
  a.scale = c.pen_scale;
  a.tw = c.twP;
  a.circ = c.circ;
  SLRX_SWITCH_N(c.P, cols_pen_body<N_, M>(a, b, lds, twt))
}

__global__ __launch_bounds__(kNT) void k_group_fin(const CgSlice* tab, int ns, int init) {
  __shared__ float2 lds[kRowB * fft_stride(256)];
  __shared__ float2 twt[kTwMax];
  __shared__ double red[kNT / 64];
  const int gb = (int)blockIdx.x;
  const CgSlice& c = tab[group_slice(tab, ns, gb, &CgSlice::rows0)];
  const int lb = gb - c.rows0;
  if (lb >= c.rows_gx * c.rows_gy) return;
  const Blk b{lb % c.rows_gx, lb / c.rows_gx, c.rows_gx, c.rows_gy};
  FinArgs a{};
  a.P = c.P; a.Q = c.Q; a.T = c.T;
  a.init = init;
  a.t = c.t;
  a.v = init ? c.x : c.p;
  a.S = c.S;
  a.y = c.bm;
  a.out = init ? c.r : c.q;
  a.part = c.partA;
  a.flag = c.flag;
  a.tw = c.twQ;
  SLRX_SWITCH_N(c.Q, rows_fin_body<N_, false>(a, b, lds, twt, nullptr, nullptr, red))
}

__global__ __launch_bounds__(kNT) void k_group_update(const CgSlice* tab, int ns, int k) {
  __shared__ double red[kNT / 64];
  const int gb = (int)blockIdx.x;
  const CgSlice& c = tab[group_slice(tab, ns, gb, &CgSlice::upd0)];
  const int lb = gb - c.upd0;
  if (lb >= c.upd_gx) return;
  UpdArgs a{};
  a.n = (long)c.T * c.P * c.Q;
  a.x = c.x;
  a.r = c.r;
  a.p = c.p;
  a.q = c.q;
  a.partA = c.partA;
  a.nA = c.nfin;
  a.rr_hist = c.rr_hist;
  a.k = k;
  a.partB = c.partB;
  a.flag = c.flag;
  update_body(a, Blk{lb, 0, c.upd_gx, 1}, red);
}

// The problem's own grids and partial counts (what its single launches use).
void cg_slice_grids(CgSlice& c) {
  c.rows_gx = c.P / row_block(c.P);
  c.rows_gy = c.T;
  int cb = 1;
  SLRX_SWITCH_N(c.P, cb = col_block(ColCap<N_>::v, c.Q))
  c.cols_gx = c.Q / cb;
  c.upd_gx = update_blocks((long)c.T * c.P * c.Q);
  c.nfin = fin_blocks(c.P, c.T);
  c.nupd = c.upd_gx;
}

size_t group_pen_lds(int P, int Q, int T) {
  size_t lds = 0;
  SLRX_SWITCH_N(P, lds = (size_t)T * col_block(ColCap<N_>::v, Q) * fft_stride(N_) * sizeof(float2))
  return lds;
}

hipError_t launch_group_rows(const CgGroup& g, int mode, int k, hipStream_t s) {
  k_group_rows<<<g.rows_blocks, kNT, 0, s>>>(g.tab, g.ns, mode, k);
  return hipGetLastError();
}

template <int M>
static hipError_t group_pen_m(const CgGroup& g, hipStream_t s) {
  static LdsLimit lim;
  const hipError_t e = lim.ensure((const void*)k_group_pen<M>, (size_t)kTMax * kPenCols * sizeof(float2));
  if (e != hipSuccess) return e;
  k_group_pen<M><<<g.cols_blocks, kPenNT, g.pen_lds, s>>>(g.tab, g.ns);
  return hipGetLastError();
}

hipError_t launch_group_pen(const CgGroup& g, hipStream_t s) {
  switch (g.M) {
    case 1: return group_pen_m<1>(g, s);
    case 2: return group_pen_m<2>(g, s);
    case 3: return group_pen_m<3>(g, s);
    case 4: return group_pen_m<4>(g, s);
    case 5: return group_pen_m<5>(g, s);
    case 6: return group_pen_m<6>(g, s);
    case 7: return group_pen_m<7>(g, s);
    case 8: return group_pen_m<8>(g, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_group_fin(const CgGroup& g, int init, hipStream_t s) {
  k_group_fin<<<g.rows_blocks, kNT, 0, s>>>(g.tab, g.ns, init);
  return hipGetLastError();
}

hipError_t launch_group_update(const CgGroup& g, int k, hipStream_t s) {
  k_group_update<<<g.upd_blocks, kNT, 0, s>>>(g.tab, g.ns, k);
  return hipGetLastError();
}

// --------------------------------------------------------------- launches

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
  const size_t lds = (size_t)a.T * cb * fft_stride(N) * sizeof(float2);
  static LdsLimit lim;
  const hipError_t e = lim.ensure((const void*)k_cols_pen<N, M>,
                                  (size_t)kTMax * ColCap<N>::v * fft_stride(N) * sizeof(float2));
  if (e != hipSuccess) return e;
  k_cols_pen<N, M><<<dim3(a.Q / cb), kPenNT, lds, s>>>(a);
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
  if (a.coil) k_rows_fin<N, true><<<grid, kNT, 0, s>>>(a);
  else k_rows_fin<N, false><<<grid, kNT, 0, s>>>(a);
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
