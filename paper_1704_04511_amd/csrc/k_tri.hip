// Householder reduction of the Hermitian Gram matrix to real symmetric
// tridiagonal form, R = Q T Q^H (FP64), first stage of the eigen-decomposition
// in the weight update (Sec. III.B, Algorithm 1 step 1).
//
// Column k needs a global matrix-vector product with the trailing block, so
// every column is one launch (the launch boundary is the grid-wide sync).  A
// launch for column k:
//   * in every workgroup (redundantly, identical arithmetic): finishes the
//     previous reflector's w = tau p - |tau|^2/2 (p^H v) v from the previous
//     launch's p = A v, corrects row k with the pending rank-2 update
//     A <- A - v w^H - w v^H, and forms reflector k, H = I - tau v v^H with
//     H^H x = (beta, 0, ..)^T, beta real (the elementary reflector convention
//     of LAPACK's zlarfg);
//   * on its rows i > k: applies the pending rank-2 update and accumulates
//     p_i = sum_j A_ij v_j for the next launch.
// The last columns, once the trailing block fits in the LDS of one workgroup,
// are reduced in a single launch (k_tri_tail).
// The working matrix Aw is full (both triangles) and row-major; reflectors are
// stored as LAPACK's zhetrd (lower) stores them: v(k+2:n) in column k of the
// column-major matrix Vst below the subdiagonal, tau(k), diagonal D, real
// subdiagonal E.
#include "common.h"
#include "kernels.h"

namespace slrx {

constexpr int kTriNT = 256;
constexpr int kTriRows = 4;  // rows of the trailing block per workgroup: one per wave
constexpr int kTriUnroll = 4;  // row elements in flight per lane beyond the prefetched part
constexpr int kTriCrit = 5;    // elements of row k / v / p per thread loaded up front

SLRX_DEV double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
SLRX_DEV double2 dscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Deterministic block sum of a complex value (fixed shuffle/tree order).
SLRX_DEV double2 block_sum2(double2 v, double2* red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_down(v.x, off, 64);
    v.y += __shfl_down(v.y, off, 64);
  }
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double2 s = make_double2(0.0, 0.0);
    for (int w = 0; w < kTriNT / 64; ++w) s = dadd(s, red[w]);
    red[kTriNT / 64] = s;
  }
  __syncthreads();
  v = red[kTriNT / 64];
  __syncthreads();
  return v;
}

// NU: row elements per lane loaded at kernel entry (the whole row when the
// trailing block is at most 64 NU wide), so the row's load latency overlaps
// the reflector computation.
template <int NU>
__global__ __launch_bounds__(kTriNT) void k_tri_step(TriArgs a) {
  extern __shared__ double2 sm[];
  __shared__ double2 red[kTriNT / 64 + 1];
  __shared__ double2 at_k[2];  // raw p_{k-1}[k], v_{k-1}[k]
  const int n = a.n, k = a.k;
  const int b = blockIdx.y;  // problem in a batch
  double2* Aw = a.Aw + (size_t)b * a.strideA;
  double2* vp = sm;           // v_{k-1}, indices >= k
  double2* wp = sm + n;       // w_{k-1}
  double2* col = sm + 2 * n;  // column k of the current matrix, then v_k
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool pending = k > 0;

  // 0. issue every independent global load first: v_{k-1}, p_{k-1} and row k
  //    (needed at once), then this wave's row of the trailing block (needed last).
  const int my_row = k + 1 + blockIdx.x * kTriRows + wave;  // one row per wave
  const bool has_row = my_row < n;
  double2* row = Aw + (size_t)(has_row ? my_row : 0) * n;
  const double2 t = pending ? a.tau[(size_t)b * n + (k - 1)] : make_double2(0.0, 0.0);
  const double2* rowk = Aw + (size_t)k * n;
  const double2* vprev = a.vbuf[(k + 1) & 1] + (size_t)b * n;  // written by launch k-1
  const double2* pprev = a.pbuf[(k + 1) & 1] + (size_t)b * n;
  double2 kv[kTriCrit], rv[kTriCrit], pv[kTriCrit];
#pragma unroll
  for (int u = 0; u < kTriCrit; ++u) {
    const int j = k + tid + kTriNT * u;
    if (j < n) {
      kv[u] = rowk[j];
      if (pending) {
        rv[u] = vprev[j];
        pv[u] = pprev[j];
      }
    }
  }
  double2 xpre[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int j = k + 1 + lane + 64 * u;
    xpre[u] = (has_row && j < n) ? row[j] : make_double2(0.0, 0.0);
  }
  double2 d = make_double2(0.0, 0.0);
  auto stage = [&](int j, double2 kj, double2 rj, double2 pj) {
    col[j] = dconj(kj);  // A(j, k) = conj(A(k, j))
    if (pending) {
      vp[j] = rj;
      wp[j] = pj;
      d = dadd(d, dcmul(pj, rj));
      if (j == k) {
        at_k[0] = pj;
        at_k[1] = rj;
      }
    }
  };
#pragma unroll
  for (int u = 0; u < kTriCrit; ++u) {
    const int j = k + tid + kTriNT * u;
    if (j < n) stage(j, kv[u], rv[u], pv[u]);
  }
  for (int j = k + tid + kTriNT * kTriCrit; j < n; j += kTriNT)  // n - k > kTriCrit * kTriNT only
    stage(j, rowk[j], pending ? vprev[j] : make_double2(0.0, 0.0), pending ? pprev[j] : make_double2(0.0, 0.0));

  // 1. pending reflector k-1: w = tau p + c v, c = -|tau|^2/2 (p^H v); apply it to
  //    column k: A(j,k) - v_j conj(w_k) - w_j conj(v_k); partial norm for step 3.
  double xn = 0.0;
  if (pending) {
    d = block_sum2(d, red);  // also orders at_k and the LDS vectors
    const double c = -0.5 * (t.x * t.x + t.y * t.y);
    const double2 cd = dscale(d, c);
    const double2 vk0 = at_k[1];
    const double2 wk0 = dadd(dmul(t, at_k[0]), dmul(cd, vk0));
    for (int j = k + tid; j < n; j += kTriNT) {
      const double2 w = dadd(dmul(t, wp[j]), dmul(cd, vp[j]));
      wp[j] = w;
      const double2 x = dsub(col[j], dadd(dmul(vp[j], dconj(wk0)), dmul(w, dconj(vk0))));
      col[j] = x;
      if (j >= k + 2) xn += x.x * x.x + x.y * x.y;
    }
  } else {
    __syncthreads();
    for (int j = k + 2 + tid; j < n; j += kTriNT) xn += col[j].x * col[j].x + col[j].y * col[j].y;
  }
  const double2 xn2 = block_sum2(make_double2(xn, 0.0), red);  // also orders col / wp
  if (k == n - 1) {  // last diagonal entry, no reflector left
    if (blockIdx.x == 0 && tid == 0) a.D[(size_t)b * n + k] = col[k].x;
    return;
  }

  // 3. reflector k on x = col[k+1 .. n-1]
  const double2 alpha = col[k + 1];
  double beta;
  double2 tau, scale;
  if (xn2.x == 0.0 && alpha.y == 0.0) {
    tau = make_double2(0.0, 0.0);
    beta = alpha.x;
    scale = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2.x);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    // scale = 1 / (alpha - beta)
    const double2 den = make_double2(alpha.x - beta, alpha.y);
    const double dd = den.x * den.x + den.y * den.y;
    scale = make_double2(den.x / dd, -den.y / dd);
  }
  const double dk = col[k].x;
  __syncthreads();
  for (int i = k + 1 + tid; i < n; i += kTriNT) col[i] = (i == k + 1) ? make_double2(1.0, 0.0) : dmul(col[i], scale);
  __syncthreads();
  if (blockIdx.x == 0) {
    double2* vout = a.vbuf[k & 1] + (size_t)b * n;
    double2* Vst = a.Vst + (size_t)b * a.strideA;
    for (int i = k + 1 + tid; i < n; i += kTriNT) {
      vout[i] = col[i];
      Vst[(size_t)k * n + i] = (i == k + 1) ? make_double2(beta, 0.0) : col[i];
    }
    if (tid == 0) {
      a.D[(size_t)b * n + k] = dk;
      a.E[(size_t)b * n + k] = beta;
      a.tau[(size_t)b * n + k] = tau;
    }
  }

  // 4. this wave's row of the trailing block: pending update, then
  //    p_i = sum_j A_ij v_j (the first elements are already in registers)
  if (!has_row) return;
  double2* pout = a.pbuf[k & 1] + (size_t)b * n;
  const double2 vpi = pending ? vp[my_row] : make_double2(0.0, 0.0);
  const double2 wpi = pending ? wp[my_row] : make_double2(0.0, 0.0);
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int j = k + 1 + lane + 64 * u;
    if (j < n) {
      double2 x = xpre[u];
      if (pending) {
        x = dsub(x, dadd(dmul(vpi, dconj(wp[j])), dmul(wpi, dconj(vp[j]))));
        row[j] = x;
      }
      acc = dadd(acc, dmul(x, col[j]));
    }
  }
  for (int j0 = k + 1 + lane + 64 * NU; j0 < n; j0 += 64 * kTriUnroll) {
    double2 x[kTriUnroll];
#pragma unroll
    for (int u = 0; u < kTriUnroll; ++u) {
      const int j = j0 + 64 * u;
      x[u] = j < n ? row[j] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kTriUnroll; ++u) {
      const int j = j0 + 64 * u;
      if (j < n) {
        if (pending) {
          x[u] = dsub(x[u], dadd(dmul(vpi, dconj(wp[j])), dmul(wpi, dconj(vp[j]))));
          row[j] = x[u];
        }
        acc = dadd(acc, dmul(x[u], col[j]));
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) pout[my_row] = acc;
}

// The last kTriTail columns in one launch: the trailing block (rows and columns
// k0..n-1) is small enough for the LDS of one workgroup, so its columns need
// only block barriers instead of launches.  First the pending update of
// reflector k0-1 is applied to the block, then each column is reduced as in
// k_tri_step (same reflector convention, same outputs), the rank-2 update
// applied to the whole block.  The outputs are kept in LDS and written at the
// end: a barrier waits for the wave's outstanding stores.
constexpr int kTriTail = 64;
constexpr int kTailNT = 256;

// Sum over the 64 lanes of a wave, every lane gets the total (fixed order).
SLRX_DEV double2 wave_sum2(double2 v) {
  for (int off = 1; off < 64; off <<= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

__global__ __launch_bounds__(kTailNT) void k_tri_tail(TriArgs a, int k0) {
  extern __shared__ double2 sm[];
  __shared__ double2 sc[4];  // tau, scale, d; beta in sc[3].x
  const int n = a.n, L = n - k0;
  const int b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double2* B = sm;           // L x L block, row-major, B[i][j] = A(k0 + i, k0 + j)
  double2* vv = B + L * L;   // reflector
  double2* pw = vv + L;      // A v
  double2* Vl = pw + L;      // reflectors of the block, column kk at Vl[kk * L]
  double2* tl = Vl + L * L;  // tau
  double* Dl = (double*)(tl + L);
  double* El = Dl + L;
  const double2* Aw = a.Aw + (size_t)b * a.strideA;
  double2* Vst = a.Vst + (size_t)b * a.strideA;
  double* D = a.D + (size_t)b * n;
  double* E = a.E + (size_t)b * n;
  double2* taus = a.tau + (size_t)b * n;
  const double2 zero = make_double2(0.0, 0.0);
  for (int e = tid; e < L * L; e += kTailNT) B[e] = Aw[(size_t)(k0 + e / L) * n + k0 + e % L];
  if (k0 > 0) {  // pending update of reflector k0-1: w = tau p + c (p^H v) v
    const double2* vprev = a.vbuf[(k0 + 1) & 1] + (size_t)b * n + k0;
    const double2* pprev = a.pbuf[(k0 + 1) & 1] + (size_t)b * n + k0;
    const double2 t = taus[k0 - 1];
    if (tid < L) {
      vv[tid] = vprev[tid];
      pw[tid] = pprev[tid];
    }
    if (wave == 0) {
      const double2 d = wave_sum2(lane < L ? dcmul(pprev[lane], vprev[lane]) : zero);
      if (lane == 0) sc[2] = d;
    }
    __syncthreads();
    const double c = -0.5 * (t.x * t.x + t.y * t.y);
    const double2 cd = dscale(sc[2], c);
    for (int e = tid; e < L * L; e += kTailNT) {
      const int i = e / L, j = e % L;
      const double2 wi = dadd(dmul(t, pw[i]), dmul(cd, vv[i]));
      const double2 wj = dadd(dmul(t, pw[j]), dmul(cd, vv[j]));
      B[e] = dsub(B[e], dadd(dmul(vv[i], dconj(wj)), dmul(wi, dconj(vv[j]))));
    }
  }
  __syncthreads();
  for (int kk = 0; kk < L - 1; ++kk) {
    // 1. reflector from x = column kk below the diagonal (B Hermitian: x_i = conj(B[kk][i]))
    if (wave == 0) {
      const int i = kk + 2 + lane;
      double2 x = i < L ? B[kk * L + i] : zero;
      const double xn2 = wave_sum2(make_double2(x.x * x.x + x.y * x.y, 0.0)).x;
      if (lane == 0) {
        const double2 alpha = dconj(B[kk * L + kk + 1]);
        double beta;
        double2 tau, scale;
        if (xn2 == 0.0 && alpha.y == 0.0) {
          tau = zero;
          beta = alpha.x;
          scale = zero;
        } else {
          const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
          beta = alpha.x >= 0.0 ? -nrm : nrm;
          tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
          const double2 den = make_double2(alpha.x - beta, alpha.y);
          const double dd = den.x * den.x + den.y * den.y;
          scale = make_double2(den.x / dd, -den.y / dd);
        }
        sc[0] = tau;
        sc[1] = scale;
        sc[3] = make_double2(beta, 0.0);
        Dl[kk] = B[kk * L + kk].x;
        El[kk] = beta;
        tl[kk] = tau;
      }
    }
    __syncthreads();
    const double2 tau = sc[0], scale = sc[1];
    for (int i = kk + 1 + tid; i < L; i += kTailNT) {
      const double2 v = (i == kk + 1) ? make_double2(1.0, 0.0) : dmul(dconj(B[kk * L + i]), scale);
      vv[i] = v;
      Vl[kk * L + i] = (i == kk + 1) ? sc[3] : v;
    }
    __syncthreads();
    // 2. p = B v on the trailing rows: four threads per row, p_i = sum_j conj(B[j][i]) v_j
    {
      const int i = kk + 1 + (tid >> 2), q = tid & 3;
      double2 acc = zero;
      if (i < L)
        for (int j = kk + 1 + q; j < L; j += 4) acc = dadd(acc, dmul(dconj(B[j * L + i]), vv[j]));
      acc.x += __shfl_xor(acc.x, 1, 64);
      acc.y += __shfl_xor(acc.y, 1, 64);
      acc.x += __shfl_xor(acc.x, 2, 64);
      acc.y += __shfl_xor(acc.y, 2, 64);
      if (i < L && q == 0) pw[i] = acc;
    }
    __syncthreads();
    // 3. d = p^H v, then the rank-2 update with w = tau p + c d v formed on the fly
    if (wave == 0) {
      const int i = kk + 1 + lane;
      const double2 d = wave_sum2(i < L ? dcmul(pw[i], vv[i]) : zero);
      if (lane == 0) sc[2] = d;
    }
    __syncthreads();
    const double c = -0.5 * (tau.x * tau.x + tau.y * tau.y);
    const double2 cd = dscale(sc[2], c);
    const int T = L - kk - 1;
    for (int e = tid; e < T * T; e += kTailNT) {
      const int i = kk + 1 + e / T, j = kk + 1 + e % T;
      const double2 wi = dadd(dmul(tau, pw[i]), dmul(cd, vv[i]));
      const double2 wj = dadd(dmul(tau, pw[j]), dmul(cd, vv[j]));
      B[i * L + j] = dsub(B[i * L + j], dadd(dmul(vv[i], dconj(wj)), dmul(wi, dconj(vv[j]))));
    }
    __syncthreads();
  }
  if (tid == 0) Dl[L - 1] = B[(L - 1) * L + L - 1].x;
  __syncthreads();
  for (int e = tid; e < (L - 1) * L; e += kTailNT) {
    const int kk = e / L, i = e % L;
    if (i > kk) Vst[(size_t)(k0 + kk) * n + k0 + i] = Vl[kk * L + i];
  }
  for (int kk = tid; kk < L; kk += kTailNT) {
    D[k0 + kk] = Dl[kk];
    if (kk < L - 1) {
      E[k0 + kk] = El[kk];
      taus[k0 + kk] = tl[kk];
    }
  }
}

int tri_max_n() { return 3000; }

static size_t tail_lds(int L) { return (size_t)(2 * L * L + 3 * L) * sizeof(double2) + 2 * (size_t)L * sizeof(double); }

template <int NU>
static hipError_t tri_attr() {
  return hipFuncSetAttribute((const void*)k_tri_step<NU>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)((size_t)3 * tri_max_n() * sizeof(double2)));
}

hipError_t launch_tridiag(const TriArgs& base, int nbatch, hipStream_t s) {
  const int n = base.n;
  const size_t lds = (size_t)3 * n * sizeof(double2);
  static bool attr = false;
  if (!attr) {
    hipError_t e = tri_attr<1>();
    if (e == hipSuccess) e = tri_attr<2>();
    if (e == hipSuccess) e = tri_attr<4>();
    if (e == hipSuccess) e = tri_attr<8>();
    if (e == hipSuccess) e = tri_attr<12>();
    if (e == hipSuccess) e = tri_attr<16>();
    if (e != hipSuccess) return e;
    attr = true;
  }
  static bool tail_attr = false;
  if (!tail_attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_tri_tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)tail_lds(kTriTail));
    if (e != hipSuccess) return e;
    tail_attr = true;
  }
  const int k0 = n > kTriTail ? n - kTriTail : 0;  // columns k0.. in one launch
  TriArgs a = base;
  for (int k = 0; k < k0; ++k) {
    a.k = k;
    const int rows = n - k - 1;
    const int gx = rows > 0 ? (rows + kTriRows - 1) / kTriRows : 1;
    const dim3 grid(gx, nbatch);
    const int chunks = (rows + 63) / 64;  // row elements per lane
    if (chunks <= 1) k_tri_step<1><<<grid, kTriNT, lds, s>>>(a);
    else if (chunks <= 2) k_tri_step<2><<<grid, kTriNT, lds, s>>>(a);
    else if (chunks <= 4) k_tri_step<4><<<grid, kTriNT, lds, s>>>(a);
    else if (chunks <= 8) k_tri_step<8><<<grid, kTriNT, lds, s>>>(a);
    else if (chunks <= 12) k_tri_step<12><<<grid, kTriNT, lds, s>>>(a);
    else k_tri_step<16><<<grid, kTriNT, lds, s>>>(a);
  }
  const int L = n - k0;
  k_tri_tail<<<dim3(1, nbatch), kTailNT, tail_lds(L), s>>>(a, k0);
  return hipGetLastError();
}

}  // namespace slrx
