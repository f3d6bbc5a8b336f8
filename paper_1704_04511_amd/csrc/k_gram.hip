// Weight update kernels (FP64): Gram matrix by Fourier autocorrelation,
// IRLS weights, the filter product H = U diag(alpha) U^H on FP64 MFMA, and the
// penalty masks E (summed power spectra of the weighted filters).
//
// Gram (Sec. III.B, eq. "eq:block-expression for R" and eq. "eq:P_ij modified"):
//   c_{m,m'}(r) = sum_{n=M-1}^{T-1} conj(rho_{n-m}(r)) rho_{n-m'}(r)
// (the GIRAF variant: n = 0..T-1, frame indices mod T),
//   R[(m,a),(m',a')] = F_u(c_{m,m'})[a - a'],
// where only the (2N1-1) x (2N2-1) lags of the sliding window are ever read,
// so F_u is evaluated at those lags only (a pruned DFT, two small passes).
//
// Masks (Sec. III.A, eq. "eq:circ_fft" and the G precompute after eq.
// "eq:grad_ls"): E_r[m,m'] = sum_i alpha_i conj(mu_m^(i)(r)) mu_m'^(i)(r)
//   = sum_Delta w_{m',m}[Delta] e^{+2 pi i Delta.r},
//   w_{m',m}[Delta] = sum_{a'-a = Delta} H[(m',a'),(m,a)].
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace slrx {

typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ Gram pass 1
// Block per image row r1: lagged products for every tap pair (FP64), then the
// pruned DFT along r2 at lags delta2 = -(N2-1)..(N2-1).
template <int M>
__global__ __launch_bounds__(256) void k_gram_rows(GramArgs a) {
  constexpr int W = M * (M + 1) / 2;
  extern __shared__ double2 sm[];  // cw[W][Q], tw[Q]
  const int P = a.P, Q = a.Q, T = a.T, N2 = a.N2;
  const int L2 = 2 * N2 - 1;
  double2* cw = sm;
  double2* tw = sm + (size_t)W * Q;
  const int r1 = blockIdx.x;
  const long fs = (long)P * Q;
  for (int i = threadIdx.x; i < Q; i += 256) tw[i] = a.twQ[i];
  for (int r2 = threadIdx.x; r2 < Q; r2 += 256) {
    const long off = (long)r1 * Q + r2;
    double2 acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = make_double2(0.0, 0.0);
    // z[m] = rho_{n-m}; with circ the sum starts at n = 0 and frame indices wrap
    const int n0 = a.circ ? 0 : M - 1;
    double2 z[M];
#pragma unroll
    for (int m = 0; m < M; ++m) z[m] = f2d(a.rho[(long)((n0 - m + T) % T) * fs + off]);
    for (int n = n0; n < T; ++n) {
      if (n > n0) {
#pragma unroll
        for (int m = M - 1; m > 0; --m) z[m] = z[m - 1];
        z[0] = f2d(a.rho[(long)n * fs + off]);
      }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int mp = m; mp < M; ++mp) {
          const int w = pair_id(m, mp, M);
          acc[w] = dadd(acc[w], dcmul(z[m], z[mp]));
        }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) cw[(size_t)w * Q + r2] = acc[w];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < W * L2; o += 256) {
    const int w = o / L2, j2 = o % L2;
    const int d2 = j2 - (N2 - 1);
    const int dq = ((d2 % Q) + Q) % Q;
    double sx = 0.0, sy = 0.0;
    int idx = 0;
    const double2* cr = cw + (size_t)w * Q;
    for (int r2 = 0; r2 < Q; ++r2) {
      const double2 c = cr[r2], t = tw[idx];
      sx += c.x * t.x - c.y * t.y;
      sy += c.x * t.y + c.y * t.x;
      idx += dq;
      if (idx >= Q) idx -= Q;
    }
    a.c1[((size_t)w * P + r1) * L2 + j2] = make_double2(sx, sy);
  }
}

// Pass 2: pruned DFT along r1 at lags delta1 = -(N1-1)..(N1-1).
__global__ __launch_bounds__(256) void k_gram_cols(GramArgs a, int W) {
  // four lanes per output, each over every fourth r1, combined in a fixed order
  const int L1 = 2 * a.N1 - 1, L2 = 2 * a.N2 - 1;
  const int gt = blockIdx.x * 256 + threadIdx.x;
  const int o = gt >> 2, q = gt & 3;
  const bool valid = o < W * L1 * L2;
  const int oo = valid ? o : 0;
  const int w = oo / (L1 * L2), j1 = (oo / L2) % L1, j2 = oo % L2;
  const int P = a.P;
  const int d1 = j1 - (a.N1 - 1);
  const int dp = ((d1 % P) + P) % P;
  double sx = 0.0, sy = 0.0;
  if (valid) {
    int idx = (int)(((long)q * dp) % P);
    const int step = (int)(((long)4 * dp) % P);
    for (int r1 = q; r1 < P; r1 += 4) {
      const double2 c = a.c1[((size_t)w * P + r1) * L2 + j2];
      const double2 t = a.twP[idx];
      sx += c.x * t.x - c.y * t.y;
      sy += c.x * t.y + c.y * t.x;
      idx += step;
      if (idx >= P) idx -= P;
    }
  }
  sx += __shfl_xor(sx, 1, 64);
  sy += __shfl_xor(sy, 1, 64);
  sx += __shfl_xor(sx, 2, 64);
  sy += __shfl_xor(sy, 2, 64);
  if (valid && q == 0) a.g[o] = make_double2(sx, sy);
}

// Pass 3: window extraction into R (column-major, full Hermitian matrix).
__global__ __launch_bounds__(256) void k_gram_assemble(GramArgs a) {
  const int N1 = a.N1, N2 = a.N2, M = a.M;
  const int NN = N1 * N2, s = NN * M;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)s * s) return;
  // element (i, j): column-major R[i + j s], or row-major R[i s + j]
  const int i = a.rowmajor ? (int)(idx / s) : (int)(idx % s);
  const int j = a.rowmajor ? (int)(idx % s) : (int)(idx / s);
  const int m = i / NN, ia = i % NN, mp = j / NN, ib = j % NN;
  const int a1 = ia / N2 - N1 / 2, a2 = ia % N2 - N2 / 2;
  const int b1 = ib / N2 - N1 / 2, b2 = ib % N2 - N2 / 2;
  const int L2 = 2 * N2 - 1, L1 = 2 * N1 - 1;
  double2 v;
  if (m <= mp) {
    const int w = pair_id(m, mp, M);
    v = a.g[((size_t)w * L1 + (a1 - b1 + N1 - 1)) * L2 + (a2 - b2 + N2 - 1)];
  } else {
    const int w = pair_id(mp, m, M);
    v = dconj(a.g[((size_t)w * L1 + (b1 - a1 + N1 - 1)) * L2 + (b2 - a2 + N2 - 1)]);
  }
  // a non-finite entry (non-finite data or iterate) is reported and replaced by
  // zero, so the eigen-decomposition only ever sees finite input
  if (!isfinite(v.x) || !isfinite(v.y)) {
    v = make_double2(0.0, 0.0);
    if (a.bad) *a.bad = 1;
  }
  a.R[idx] = v;
}

template <int M>
static hipError_t gram_m(const GramArgs& a, hipStream_t s) {
  constexpr int W = M * (M + 1) / 2;
  const size_t lds = ((size_t)W * a.Q + a.Q) * sizeof(double2);
  static LdsLimit lim;
  const hipError_t e = lim.ensure((const void*)k_gram_rows<M>, ((size_t)W * 256 + 256) * sizeof(double2));
  if (e != hipSuccess) return e;
  k_gram_rows<M><<<a.P, 256, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_gram(const GramArgs& a, hipStream_t s) {
  hipError_t e;
  switch (a.M) {
    case 1: e = gram_m<1>(a, s); break;
    case 2: e = gram_m<2>(a, s); break;
    case 3: e = gram_m<3>(a, s); break;
    case 4: e = gram_m<4>(a, s); break;
    case 5: e = gram_m<5>(a, s); break;
    case 6: e = gram_m<6>(a, s); break;
    case 7: e = gram_m<7>(a, s); break;
    case 8: e = gram_m<8>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int W = a.M * (a.M + 1) / 2;
  const int n2 = W * (2 * a.N1 - 1) * (2 * a.N2 - 1);
  k_gram_cols<<<(4 * n2 + 255) / 256, 256, 0, s>>>(a, W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long sN = (long)a.N1 * a.N2 * a.M;
  k_gram_assemble<<<(unsigned)((sN * sN + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- weights
// eps^(0) = eps0_frac * lambda_max on the first iteration, else eps <- eps / gamma.
__global__ void k_eps(WeightArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double lmax = a.lamv[a.s - 1];
  const double e = a.first ? a.eps0_frac * lmax : (*a.eps) / a.gamma;
  *a.eps = e;
  if (a.lam_max_out) *a.lam_max_out = lmax;
  if (a.eps_out) *a.eps_out = e;
}

// V = U diag(sqrt(alpha)), alpha_k = (max(lambda_k, 0) + eps)^(p/2 - 1), stored K-major.
__global__ __launch_bounds__(256) void k_weights(WeightArgs a) {
  const int s = a.s;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)s * s) return;
  const int i = (int)(idx % s), k = (int)(idx / s);
  const double lk = a.lamv[k];
  const double al = pow((lk > 0.0 ? lk : 0.0) + *a.eps, a.p * 0.5 - 1.0);
  const double sa = sqrt(al);
  const double2 u = a.U[idx];
  a.VT[(long)k * s + i] = u.x * sa;
  a.VT[(long)(s + k) * s + i] = u.y * sa;
}

hipError_t launch_eps(const WeightArgs& a, hipStream_t s) {
  k_eps<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_weights(const WeightArgs& a, hipStream_t s, bool eps) {
  hipError_t e;
  if (eps && (e = launch_eps(a, s)) != hipSuccess) return e;
  const long n = (long)a.s * a.s;
  k_weights<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

// ----------------------------------------------------- filter product (MFMA)
// Hre[i][j] = sum_{k'<2s} A[k'][i] A[k'][j],  A = VT = [Re V^T; Im V^T]
// Him[i][j] = sum_{k<s} (Im_k[i] Re_k[j] - Re_k[i] Im_k[j])
// i.e. [Hre; Him] = [A; B] A^T with B = [Im; -Re] (real form of V V^H).
// Block: 64 x 64 output tile, 4 waves in 2 x 2, each 32 x 32 = 2 x 2 MFMA
// 16x16x4 f64 tiles; K staged through LDS in chunks of 16.
// Only tiles on or above the diagonal are computed (Hre is symmetric, Him
// antisymmetric); an off-diagonal tile is also stored mirrored.  Workgroups are
// dispatched to the XCDs in turn, so consecutive tiles of the row-major tile
// order are given to the same XCD (its L2 then holds the shared row panel).
__global__ __launch_bounds__(256) void k_filter_product(int s, const double* __restrict__ VT,
                                                        double* __restrict__ Hre, double* __restrict__ Him) {
  constexpr int TB = 64, KC = 32, NXCD = 8;
  __shared__ double Lre[KC][TB];
  __shared__ double Lim[KC][TB];
  __shared__ double Rt[KC][TB];
  const int nt = (s + TB - 1) / TB;
  const int ntiles = nt * (nt + 1) / 2;
  const int per = (ntiles + NXCD - 1) / NXCD;
  const int lin = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (lin >= ntiles) return;
  int bi = 0, rem = lin;
  while (rem >= nt - bi) {
    rem -= nt - bi;
    ++bi;
  }
  const int bj = bi + rem;
  const int i0 = bi * TB, j0 = bj * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int K = 2 * s;
  v4d accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accR[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      accI[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  // the next K chunk is loaded into registers while the current one is multiplied
  constexpr int U = KC * TB / 256;
  double pr[U], pm[U], pl[U];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      const int kk = e / TB, c = e % TB;
      const int k = k0 + kk;
      double li = 0.0, lr = 0.0, lm = 0.0;
      if (k < K) {
        const int ii = i0 + c, jj = j0 + c;
        if (ii < s) {
          lr = VT[(long)k * s + ii];
          lm = (k < s) ? VT[(long)(s + k) * s + ii] : -VT[(long)(k - s) * s + ii];
        }
        if (jj < s) li = VT[(long)k * s + jj];
      }
      pr[u] = lr;
      pm[u] = lm;
      pl[u] = li;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      const int kk = e / TB, c = e % TB;
      Lre[kk][c] = pr[u];
      Lim[kk][c] = pm[u];
      Rt[kk][c] = pl[u];
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int kq = 0; kq < KC; kq += 4) {
      const int kl = kq + (lane >> 4);
      double ar[2], am[2], br[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Lre[kl][wi + a * 16 + (lane & 15)];
        am[a] = Lim[kl][wi + a * 16 + (lane & 15)];
        br[a] = Rt[kl][wj + a * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], accR[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a], br[b], accI[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // D layout of the f64 16x16x4 MFMA: item v of lane l is row l/16 + 4v, column l%16.
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = i0 + wi + a * 16 + (lane >> 4) + 4 * v;
        const int jj = j0 + wj + b * 16 + (lane & 15);
        if (ii < s && jj < s) {
          Hre[(long)ii * s + jj] = accR[a][b][v];
          Him[(long)ii * s + jj] = accI[a][b][v];
          if (bi != bj) {
            Hre[(long)jj * s + ii] = accR[a][b][v];
            Him[(long)jj * s + ii] = -accI[a][b][v];
          }
        }
      }
}

hipError_t launch_filter_product(int s, const double* VT, double* Hre, double* Him, hipStream_t st) {
  const int nt = (s + 63) / 64, ntiles = nt * (nt + 1) / 2;
  const int grid = (ntiles + 7) / 8 * 8;  // whole rounds over the 8 XCDs
  k_filter_product<<<grid, 256, 0, st>>>(s, VT, Hre, Him);
  return hipGetLastError();
}

// ----------------------------------------------- masks from filter spectra
// The diagonal sums of H = U diag(alpha) U^H are the weighted correlations of
// the filters: with u_k(m, a) the tap-m, offset-a entry of eigenvector k,
//   wsum_{m<=m'}[Delta] = sum_k alpha_k sum_{a' - a = Delta} u_k(m', a') conj(u_k(m, a)).
// On the L1 x L2 = (2N1 - 1) x (2N2 - 1) grid every lag Delta is distinct, so
// the correlation is the inverse DFT of C_w(f) = sum_k alpha_k X_{k,m'}(f)
// conj(X_{k,m}(f)), X_{k,m} the DFT of u_k(m, .) over its N1 x N2 offsets:
// about s (6 M N^3 + 2 M^2 N^2) flop against the s^3 of forming H.
// k_spec_accum: workgroup (group g of eigenvectors, block of up to 8 columns
// f2); per eigenvector the N2-point DFTs of its rows for those columns (stage
// 1, in LDS), then one thread per frequency (f1, f2) finishes its M spectra
// and accumulates the W pair products.  Partial sums per group go to
// part[g][w][f], added in a fixed order by k_spec_reduce; k_spec_inverse
// transforms back to the lags.
constexpr int kSpecF2 = 8;     // columns f2 per workgroup
constexpr int kSpecPf = kSpecMaxS / 256;  // prefetched eigenvector entries per thread
constexpr int kSpecMaxL1 = 32; // 256 threads = 32 rows f1 x 8 columns f2

template <int M>
__global__ __launch_bounds__(256) void k_spec_accum(SpecArgs a) {
  constexpr int W = M * (M + 1) / 2;
  extern __shared__ double2 spl[];
  const int N1 = a.N1, N2 = a.N2, s = a.s;
  const int L1 = 2 * N1 - 1, L2 = 2 * N2 - 1, F = L1 * L2;
  const int c0 = blockIdx.y * kSpecF2, nf2 = min(kSpecF2, L2 - c0);
  double2* v = spl;                    // eigenvector k, s entries
  double2* Y = v + s;                  // [M N1][nf2]
  double2* t1 = Y + M * N1 * kSpecF2;  // e^{-2 pi i j / L1}
  double2* t2 = t1 + L1;               // e^{-2 pi i j / L2}
  const int tid = threadIdx.x;
  for (int j = tid; j < L1; j += 256) {
    double sn, cs;
    sincospi(-2.0 * j / L1, &sn, &cs);
    t1[j] = make_double2(cs, sn);
  }
  for (int j = tid; j < L2; j += 256) {
    double sn, cs;
    sincospi(-2.0 * j / L2, &sn, &cs);
    t2[j] = make_double2(cs, sn);
  }
  const int f1 = tid / kSpecF2, fl = tid % kSpecF2;
  const bool act = f1 < L1 && fl < nf2;
  double2 acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = make_double2(0.0, 0.0);
  const int k0 = blockIdx.x * a.kper, k1 = min(s, k0 + a.kper);
  const double e = *a.eps, ex = a.p * 0.5 - 1.0;
  // eigenvector k + 1 is loaded into registers while k is transformed
  double2 nxt[kSpecPf];
#pragma unroll
  for (int r = 0; r < kSpecPf; ++r) {
    const int i = tid + 256 * r;
    nxt[r] = (k0 < k1 && i < s) ? a.U[(long)k0 * s + i] : make_double2(0.0, 0.0);
  }
  for (int k = k0; k < k1; ++k) {
    __syncthreads();  // the previous eigenvector's v and Y are no longer read
#pragma unroll
    for (int r = 0; r < kSpecPf; ++r) {
      const int i = tid + 256 * r;
      if (i < s) v[i] = nxt[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSpecPf; ++r) {
      const int i = tid + 256 * r;
      if (k + 1 < k1 && i < s) nxt[r] = a.U[(long)(k + 1) * s + i];
    }
    // stage 1: Y[m N1 + a1][c] = sum_{a2} v(m, a1, a2) e^{-2 pi i a2 (c0 + c) / L2},
    // a thread per (a1, c) and all M taps (one twiddle per M products)
    for (int o = tid; o < N1 * nf2; o += 256) {
      const int c = o % nf2, a1 = o / nf2;
      const int g2 = c0 + c;
      double sx[M], sy[M];
#pragma unroll
      for (int m = 0; m < M; ++m) sx[m] = sy[m] = 0.0;
      int t = 0;
      for (int a2 = 0; a2 < N2; ++a2) {
        const double2 w = t2[t];
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const double2 x = v[(m * N1 + a1) * N2 + a2];
          sx[m] += x.x * w.x - x.y * w.y;
          sy[m] += x.x * w.y + x.y * w.x;
        }
        t += g2;
        if (t >= L2) t -= L2;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) Y[(m * N1 + a1) * kSpecF2 + c] = make_double2(sx[m], sy[m]);
    }
    __syncthreads();
    if (act) {
      const double lk = a.lamv[k];
      const double al = pow((lk > 0.0 ? lk : 0.0) + e, ex);
      double2 X[M];
#pragma unroll
      for (int m = 0; m < M; ++m) X[m] = make_double2(0.0, 0.0);
      int t = 0;
      for (int a1 = 0; a1 < N1; ++a1) {  // stage 2 along a1
        const double2 w = t1[t];
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const double2 y = Y[(m * N1 + a1) * kSpecF2 + fl];
          X[m].x += y.x * w.x - y.y * w.y;
          X[m].y += y.x * w.y + y.y * w.x;
        }
        t += f1;
        if (t >= L1) t -= L1;
      }
      int w = 0;
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int mp = m; mp < M; ++mp, ++w) {  // alpha X_{m'} conj(X_m)
          const double re = X[mp].x * X[m].x + X[mp].y * X[m].y;
          const double im = X[mp].y * X[m].x - X[mp].x * X[m].y;
          acc[w].x += al * re;
          acc[w].y += al * im;
        }
    }
  }
  if (act) {
    const int f = f1 * L2 + c0 + fl;
#pragma unroll
    for (int w = 0; w < W; ++w) a.part[((long)blockIdx.x * W + w) * F + f] = acc[w];
  }
}

// Slice q of the groups: C[q][w][f] = sum over groups g = q, q + kSpecSlices, ..
// of part[g][w][f], in group order (the slices are added in order by the
// inverse transform).
__global__ __launch_bounds__(256) void k_spec_reduce(SpecArgs a, int W) {
  const int F = (2 * a.N1 - 1) * (2 * a.N2 - 1);
  const long WF = (long)W * F;
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= kSpecSlices * WF) return;
  const int q = (int)(o / WF);
  const long wf = o % WF;
  double sx = 0.0, sy = 0.0;
  for (int g = q; g < a.ngroups; g += kSpecSlices) {
    const double2 v = a.part[(long)g * WF + wf];
    sx += v.x;
    sy += v.y;
  }
  a.C[o] = make_double2(sx, sy);
}

// wsum[w][j1][j2] = (1 / F) sum_f C[w][f] e^{+2 pi i (Delta1 f1 / L1 + Delta2 f2 / L2)},
// Delta = j - (N - 1): one workgroup per pair, the two 1-D transforms in turn.
__global__ __launch_bounds__(1024) void k_spec_inverse(SpecArgs a, double2* wsum, int W) {
  extern __shared__ double2 spl[];
  const int N1 = a.N1, N2 = a.N2, L1 = 2 * N1 - 1, L2 = 2 * N2 - 1, F = L1 * L2;
  const int w = blockIdx.x, tid = threadIdx.x;
  double2* Cs = spl;       // C[w][f1][f2]
  double2* Ts = Cs + F;    // [f1][j2]
  double2* t1 = Ts + F;    // e^{+2 pi i j / L1}
  double2* t2 = t1 + L1;   // e^{+2 pi i j / L2}
  const long WF = (long)W * F;
  for (int f = tid; f < F; f += 1024) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int q = 0; q < kSpecSlices; ++q) {
      const double2 v = a.C[q * WF + (long)w * F + f];
      sx += v.x;
      sy += v.y;
    }
    Cs[f] = make_double2(sx, sy);
  }
  for (int j = tid; j < L1; j += 1024) {
    double sn, cs;
    sincospi(2.0 * j / L1, &sn, &cs);
    t1[j] = make_double2(cs, sn);
  }
  for (int j = tid; j < L2; j += 1024) {
    double sn, cs;
    sincospi(2.0 * j / L2, &sn, &cs);
    t2[j] = make_double2(cs, sn);
  }
  __syncthreads();
  for (int o = tid; o < F; o += 1024) {  // along f2
    const int f1 = o / L2, j2 = o % L2;
    const int d2 = (j2 - (N2 - 1) + L2) % L2;
    const double2* cr = Cs + f1 * L2;
    double sx = 0.0, sy = 0.0;
    int u = 0;
    for (int f2 = 0; f2 < L2; ++f2) {
      const double2 c = cr[f2], e = t2[u];
      sx += c.x * e.x - c.y * e.y;
      sy += c.x * e.y + c.y * e.x;
      u += d2;
      if (u >= L2) u -= L2;
    }
    Ts[o] = make_double2(sx, sy);
  }
  __syncthreads();
  const double sc = 1.0 / F;
  for (int o = tid; o < F; o += 1024) {  // along f1
    const int j1 = o / L2, j2 = o % L2;
    const int d1 = (j1 - (N1 - 1) + L1) % L1;
    double sx = 0.0, sy = 0.0;
    int u = 0;
    for (int f1 = 0; f1 < L1; ++f1) {
      const double2 c = Ts[f1 * L2 + j2], e = t1[u];
      sx += c.x * e.x - c.y * e.y;
      sy += c.x * e.y + c.y * e.x;
      u += d1;
      if (u >= L1) u -= L1;
    }
    wsum[(long)w * F + o] = make_double2(sx * sc, sy * sc);
  }
}

bool spec_supported(int N1, int N2, int M) {
  const int s = N1 * N2 * M, L1 = 2 * N1 - 1, L2 = 2 * N2 - 1;
  if (M > kSpecMaxM || L1 > kSpecMaxL1 || s > kSpecMaxS) return false;
  // LDS of the accumulation and of the inverse transform within 64 KB
  const size_t acc = ((size_t)s + (size_t)M * N1 * kSpecF2 + L1 + L2) * sizeof(double2);
  const size_t inv = (2 * (size_t)L1 * L2 + L1 + L2) * sizeof(double2);
  return acc <= 65536 && inv <= 65536;
}

// Groups of eigenvectors that fit the partial sums (and C) into cap double2.
int spec_groups(int N1, int N2, int M, size_t cap) {
  const int s = N1 * N2 * M, W = M * (M + 1) / 2;
  const size_t per = (size_t)W * (2 * N1 - 1) * (2 * N2 - 1);
  const long gmax = (long)(cap / per) - kSpecSlices;  // room for the slice sums C
  if (gmax < 1) return 0;
  const int g = (int)std::min<long>(std::min<long>(gmax, 128), s);
  const int kper = (s + g - 1) / g;
  return (s + kper - 1) / kper;
}

hipError_t launch_spec_masks(const SpecArgs& a0, double2* wsum, hipStream_t st) {
  SpecArgs a = a0;
  const int M = a.M, W = M * (M + 1) / 2;
  const int L1 = 2 * a.N1 - 1, L2 = 2 * a.N2 - 1, F = L1 * L2;
  a.kper = (a.s + a.ngroups - 1) / a.ngroups;
  const dim3 grid(a.ngroups, (L2 + kSpecF2 - 1) / kSpecF2);
  const size_t lds = ((size_t)a.s + (size_t)M * a.N1 * kSpecF2 + L1 + L2) * sizeof(double2);
  switch (M) {
    case 1: k_spec_accum<1><<<grid, 256, lds, st>>>(a); break;
    case 2: k_spec_accum<2><<<grid, 256, lds, st>>>(a); break;
    case 3: k_spec_accum<3><<<grid, 256, lds, st>>>(a); break;
    case 4: k_spec_accum<4><<<grid, 256, lds, st>>>(a); break;
    case 5: k_spec_accum<5><<<grid, 256, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_spec_reduce<<<(unsigned)(((long)kSpecSlices * W * F + 255) / 256), 256, 0, st>>>(a, W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_spec_inverse<<<W, 1024, (2 * (size_t)F + L1 + L2) * sizeof(double2), st>>>(a, wsum, W);
  return hipGetLastError();
}

// ------------------------------------------------------------------ masks
// w_{m',m}[Delta] for pairs (m <= m'), Delta = a' - a.
__global__ __launch_bounds__(256) void k_diagsum(MaskArgs a, int W, int s) {
  // four lanes per output (16 outputs per wave, lane = 16 q + output), each over
  // every fourth term, combined in a fixed order
  const int N1 = a.N1, N2 = a.N2, M = a.M, NN = N1 * N2;
  const int L1 = 2 * N1 - 1, L2 = 2 * N2 - 1;
  const int gt = blockIdx.x * 256 + threadIdx.x;
  const int q = (gt & 63) >> 4, o = (gt >> 6) * 16 + (gt & 15);
  const bool valid = o < W * L1 * L2;
  const int oo = valid ? o : 0;
  const int w = oo / (L1 * L2), j1 = (oo / L2) % L1, j2 = oo % L2;
  int m = 0, mp = 0;
  for (int mm = 0; mm < M; ++mm)
    for (int nn = mm; nn < M; ++nn)
      if (pair_id(mm, nn, M) == w) { m = mm; mp = nn; }
  const int d1 = j1 - (N1 - 1), d2 = j2 - (N2 - 1);
  double sx = 0.0, sy = 0.0;
  const int i1lo = d1 < 0 ? -d1 : 0, i1hi = d1 > 0 ? N1 - d1 : N1;
  const int i2lo = d2 < 0 ? -d2 : 0, i2hi = d2 > 0 ? N2 - d2 : N2;
  const int w2 = i2hi - i2lo, cnt = valid ? (i1hi - i1lo) * w2 : 0;
  // H(row, col) read as conj(H(col, row)) for coalesced access across d2
  for (int t = q; t < cnt; t += 4) {
    const int i1 = i1lo + t / w2, i2 = i2lo + t % w2;
    const long row = (long)mp * NN + (i1 + d1) * N2 + (i2 + d2);  // (m', a')
    const long col = (long)m * NN + i1 * N2 + i2;                  // (m, a)
    sx += a.Hre[col * s + row];
    sy -= a.Him[col * s + row];
  }
  sx += __shfl_xor(sx, 16, 64);
  sy += __shfl_xor(sy, 16, 64);
  sx += __shfl_xor(sx, 32, 64);
  sy += __shfl_xor(sy, 32, 64);
  if (valid && q == 0) a.wsum[o] = make_double2(sx, sy);
}

// s1[w][j1][r2] = sum_{j2} w[w][j1][j2] e^{+2 pi i Delta2 r2 / Q}
__global__ __launch_bounds__(256) void k_mask_rows(MaskArgs a, int W) {
  const int L1 = 2 * a.N1 - 1, L2 = 2 * a.N2 - 1, Q = a.Q;
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= (long)W * L1 * Q) return;
  const int r2 = (int)(o % Q);
  const long wj = o / Q;  // w * L1 + j1
  double sx = 0.0, sy = 0.0;
  // twiddle index (Delta2 r2) mod Q, stepped by r2 as Delta2 grows by one
  int t = (int)(((long)((Q - (a.N2 - 1) % Q) % Q) * r2) % Q);
  for (int j2 = 0; j2 < L2; ++j2) {
    const double2 c = a.wsum[wj * L2 + j2];
    const double2 tw = a.twQ[t];  // conj gives the + sign
    sx += c.x * tw.x + c.y * tw.y;
    sy += c.y * tw.x - c.x * tw.y;
    t += r2;
    if (t >= Q) t -= Q;
  }
  a.s1[o] = make_double2(sx, sy);
}

// E_w(r1, r2) = sum_{j1} s1[w][j1][r2] e^{+2 pi i Delta1 r1 / P}, rounded to FP32 and
// stored as transposed planes Et[w][r2][r1] (the layout of the column penalty pass).
__global__ __launch_bounds__(256) void k_mask_cols(MaskArgs a, int W) {
  const int L1 = 2 * a.N1 - 1, P = a.P, Q = a.Q;
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= (long)W * P * Q) return;
  const int r1 = (int)(o % P);
  const int r2 = (int)((o / P) % Q);
  const int w = (int)(o / ((long)P * Q));
  double sx = 0.0, sy = 0.0;
  // twiddle index (Delta1 r1) mod P, stepped by r1 as Delta1 grows by one
  int t = (int)(((long)((P - (a.N1 - 1) % P) % P) * r1) % P);
  for (int j1 = 0; j1 < L1; ++j1) {
    const double2 c = a.s1[((long)w * L1 + j1) * Q + r2];
    const double2 tw = a.twP[t];
    sx += c.x * tw.x + c.y * tw.y;
    sy += c.y * tw.x - c.x * tw.y;
    t += r1;
    if (t >= P) t -= P;
  }
  a.Et[o] = make_float2((float)sx, (float)sy);
}

hipError_t launch_masks(const MaskArgs& a, hipStream_t s) {
  const int W = a.M * (a.M + 1) / 2;
  const int sN = a.N1 * a.N2 * a.M;
  const int L1 = 2 * a.N1 - 1, L2 = 2 * a.N2 - 1;
  hipError_t e;
  if (a.Hre) {  // lag sums from H; otherwise wsum holds them already
    const int n1 = W * L1 * L2;
    k_diagsum<<<(4 * n1 + 255) / 256, 256, 0, s>>>(a, W, sN);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const long n2 = (long)W * L1 * a.Q;
  k_mask_rows<<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(a, W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long n3 = (long)W * a.P * a.Q;
  k_mask_cols<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(a, W);
  return hipGetLastError();
}

}  // namespace slrx
