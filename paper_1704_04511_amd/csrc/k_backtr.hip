// Back-transformation of the tridiagonal eigenvectors, U = Q Z (FP64), last
// stage of the Gram eigen-decomposition in the weight update (Sec. III.B,
// Algorithm 1 step 1).
//
// The Householder reduction leaves Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k
// v_k^H, v_k zero above row k+1 and one at row k+1.  Reflectors are grouped in
// blocks of kBtNb; a block is I - V T V^H with V (n x kBtNb) its reflectors and
// T upper triangular (the forward, column-wise compact WY form, T(i,i) = tau_i,
// T(0:i, i) = -tau_i T(0:i, 0:i) V(:, 0:i)^H v_i).  With Y = V T the block acts
// on Z as Z <- Z - Y (V^H Z), and Q Z applies the blocks from the last to the
// first.  Every product is a complex FP64 matrix product on the f64 16x16x4
// MFMA: output tiles of 64 x 16 (one 16 x 16 tile per wave), K staged through
// LDS in chunks of 16; long reductions are split over workgroups into partial
// results that the consumer sums in a fixed order (results are reproducible
// bit for bit).
#include "common.h"
#include "kernels.h"

namespace slrx {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBtNb = 64;  // reflectors per block
constexpr int kTM = 64, kTN = 16, kKC = 16;
constexpr int kBtSplitG = 4;  // split-K of the block Gram matrices
constexpr int kBtSplitW = 8;  // split-K of V^H Z

enum BtKind { BT_GRAM = 0, BT_YMAT = 1, BT_APPLY_W = 2, BT_APPLY_Z = 3 };

// One product of the back-transformation for reflector block g.  For
//   r0 = nb g + 1 (first row the block touches), m = n - r0, nr = reflectors in the block,
//   GRAM:    G_g = V_g^H V_g        (nr x nr, K = m), partial z -> Gp[(z * ng + g) nb^2]
//   YMAT:    Y_g = V_g T_g          (m x nr, K = nr)  -> Yx, column-major n x n, rows r0..
//   APPLY_W: W   = V_g^H Z(r0:, :)  (nr x n, K = m),  partial z -> Wp[z nb n]
//   APPLY_Z: Z(r0:, :) -= Y_g W     (m x n, K = nr),  W = the partials summed (k_bt_wsum).
struct BtArgs {
  int n, ng, nsplit, g;
  const double2* Vx;  // reflectors, column-major n x n, explicit zeros and unit entries
  double2* Yx;        // Y blocks, column-major n x n
  double2* Z;         // eigenvectors, column-major n x n
  double2* Gp;        // Gram partials of the blocks
  double2* Tb;        // T of the blocks, column-major nb x nb each
  double2* Wp;        // V^H Z partials, column-major nb x n each
  const double2* tau; // reflector scalars, n
  long sV, sY, sZ, sW;  // strides between the problems of a batch (sW: scratch)
};

// The arguments of problem b of a batch.
SLRX_DEV BtArgs bt_at(BtArgs a, int b) {
  a.Vx += b * a.sV;
  a.Yx += b * a.sY;
  a.Z += b * a.sZ;
  a.Gp += b * a.sW;
  a.Tb += b * a.sW;
  a.Wp += b * a.sW;
  a.tau += (long)b * a.n;
  return a;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_bt_gemm(BtArgs a0, int zper) {
  // blockIdx.z = problem * zper + (split / block index within the problem)
  const BtArgs a = bt_at(a0, blockIdx.z / zper);
  const int bz = blockIdx.z % zper;
  __shared__ double Lar[kKC][kTM + 1], Lai[kKC][kTM + 1];  // padded against bank conflicts
  __shared__ double Lbr[kKC][kTN + 1], Lbi[kKC][kTN + 1];
  const int n = a.n;
  int g, z;
  if (KIND == BT_GRAM) {
    g = bz / a.nsplit;
    z = bz % a.nsplit;
  } else if (KIND == BT_YMAT) {
    g = bz;
    z = 0;
  } else {
    g = a.g;
    z = bz;
  }
  const int k0 = kBtNb * g, r0 = k0 + 1, m = n - r0;
  const int nr = min(kBtNb, n - 1 - k0);
  int M, N, K;
  if (KIND == BT_GRAM) { M = nr; N = nr; K = m; }
  else if (KIND == BT_YMAT) { M = m; N = nr; K = nr; }
  else if (KIND == BT_APPLY_W) { M = nr; N = n; K = m; }
  else { M = m; N = n; K = nr; }
  const int i0 = blockIdx.y * kTM, j0 = blockIdx.x * kTN;
  if (i0 >= M || j0 >= N) return;
  // split-K range of this workgroup (whole chunks)
  int kb = 0, ke = K;
  if (KIND == BT_GRAM || KIND == BT_APPLY_W) {
    const int per = ((K + a.nsplit - 1) / a.nsplit + kKC - 1) / kKC * kKC;
    kb = z * per;
    ke = min(K, kb + per);
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  v4d accR = v4d{0.0, 0.0, 0.0, 0.0}, accI = v4d{0.0, 0.0, 0.0, 0.0};
  // global loads of one K chunk into registers (4 A elements and 1 B element per thread)
  constexpr int kAE = kTM * kKC / 256;
  double2 ra[kAE], rb;
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kAE; ++u) {
      const int e = tid + 256 * u;
      double2 v = make_double2(0.0, 0.0);
      if (KIND == BT_GRAM || KIND == BT_APPLY_W) {  // A(i, r) = conj(V(r0 + r, k0 + i))
        const int i = e / kKC, r = kc + e % kKC;
        if (i0 + i < M && r < ke) {
          v = a.Vx[(long)(r0 + r) + (long)(k0 + i0 + i) * n];
          v.y = -v.y;
        }
      } else {  // A(r, l) column-major: V for YMAT, Y for APPLY_Z
        const int i = e % kTM, l = kc + e / kTM;
        if (i0 + i < M && l < ke) {
          const double2* src = KIND == BT_YMAT ? a.Vx : a.Yx;
          v = src[(long)(r0 + i0 + i) + (long)(k0 + l) * n];
        }
      }
      ra[u] = v;
    }
    const int j = tid / kKC, k = kc + tid % kKC, c = j0 + j;
    rb = make_double2(0.0, 0.0);
    if (k < ke && c < N) {
      if (KIND == BT_GRAM) rb = a.Vx[(long)(r0 + k) + (long)(k0 + c) * n];
      else if (KIND == BT_YMAT) rb = a.Tb[(long)g * kBtNb * kBtNb + k + (long)c * kBtNb];
      else if (KIND == BT_APPLY_W) rb = a.Z[(long)(r0 + k) + (long)c * n];
      else rb = a.Wp[(long)a.nsplit * kBtNb * n + k + (long)c * kBtNb];  // summed W
    }
  };
  // APPLY_Z: this lane's Z elements, loaded before the product
  double2 zold[4];
  if (KIND == BT_APPLY_Z) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wave * 16 + (lane >> 4) + 4 * v;
      const int c = j0 + (lane & 15);
      zold[v] = (i < M && c < N) ? a.Z[(long)(r0 + i) + (long)c * n] : make_double2(0.0, 0.0);
    }
  }
  if (kb < ke) load_chunk(kb);
  for (int kc = kb; kc < ke; kc += kKC) {
#pragma unroll
    for (int u = 0; u < kAE; ++u) {
      const int e = tid + 256 * u;
      int i, kk;
      if (KIND == BT_GRAM || KIND == BT_APPLY_W) {
        i = e / kKC;
        kk = e % kKC;
      } else {
        kk = e / kTM;
        i = e % kTM;
      }
      Lar[kk][i] = ra[u].x;
      Lai[kk][i] = ra[u].y;
    }
    Lbr[tid % kKC][tid / kKC] = rb.x;
    Lbi[tid % kKC][tid / kKC] = rb.y;
    __syncthreads();
    if (kc + kKC < ke) load_chunk(kc + kKC);  // next chunk in flight during the products
#pragma unroll
    for (int kq = 0; kq < kKC; kq += 4) {
      const int kl = kq + (lane >> 4);
      const double ar = Lar[kl][wave * 16 + (lane & 15)];
      const double ai = Lai[kl][wave * 16 + (lane & 15)];
      const double br = Lbr[kl][lane & 15];
      const double bi = Lbi[kl][lane & 15];
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accR, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, accI, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, accI, 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the f64 16x16x4 MFMA: item v of lane l is row l/16 + 4v, column l%16.
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + wave * 16 + (lane >> 4) + 4 * v;
    const int c = j0 + (lane & 15);
    if (i >= M || c >= N) continue;
    const double2 r = make_double2(accR[v], accI[v]);
    if (KIND == BT_GRAM) {
      a.Gp[((long)z * a.ng + g) * kBtNb * kBtNb + i + (long)c * kBtNb] = r;
    } else if (KIND == BT_YMAT) {
      a.Yx[(long)(r0 + i) + (long)(k0 + c) * n] = r;
    } else if (KIND == BT_APPLY_W) {
      a.Wp[(long)z * kBtNb * n + i + (long)c * kBtNb] = r;
    } else {
      a.Z[(long)(r0 + i) + (long)c * n] = make_double2(zold[v].x - r.x, zold[v].y - r.y);
    }
  }
}

// W = sum of the split-K partials of V^H Z, in a fixed order, into the slot
// after the partials.
__global__ void k_bt_wsum(BtArgs a0) {
  const BtArgs a = bt_at(a0, blockIdx.y);
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  const long len = (long)kBtNb * a.n;
  if (o >= len) return;
  double2 v = make_double2(0.0, 0.0);
  for (int p = 0; p < a.nsplit; ++p) {
    const double2 w = a.Wp[(long)p * len + o];
    v.x += w.x;
    v.y += w.y;
  }
  a.Wp[(long)a.nsplit * len + o] = v;
}

// Reflectors in explicit form, in place: column k of the n x n column-major
// matrix becomes v_k (zero above row k+1, one at row k+1; the last column is zero).
__global__ void k_bt_explicit(int n, double2* V0, long sV) {
  double2* V = V0 + blockIdx.y * sV;
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= (long)n * n) return;
  const int R = (int)(o % n), k = (int)(o / n);
  if (R < k + 1) V[o] = make_double2(0.0, 0.0);
  else if (R == k + 1) V[o] = make_double2(1.0, 0.0);
}

// T of each block by recursive doubling: for adjacent index blocks A, B (B after
// A), the product of their block reflectors has T = [T_A, -T_A G_AB T_B; 0, T_B]
// with G_AB = V_A^H V_B; blocks of 1, 2, 4, .., 32 are joined level by level,
// every entry of a level in parallel.  T is packed by columns (T(l, q) at
// q(q+1)/2 + l, l <= q); G's strict upper triangle likewise (l < i at
// i(i-1)/2 + l) and is overwritten level by level with X = G_AB T_B.  Indices
// beyond the block's reflectors get tau = 0 and G = 0, so their rows and
// columns of T are zero.
__global__ __launch_bounds__(256) void k_bt_tmat(BtArgs a0) {
  const BtArgs a = bt_at(a0, blockIdx.y);
  const double2* tau = a.tau;
  __shared__ double2 T[kBtNb * (kBtNb + 1) / 2];
  __shared__ double2 G[kBtNb * (kBtNb - 1) / 2];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int k0 = kBtNb * g, nr = min(kBtNb, a.n - 1 - k0);
  auto tix = [](int l, int q) { return q * (q + 1) / 2 + l; };
  auto gix = [](int l, int i) { return i * (i - 1) / 2 + l; };
  for (int e = tid; e < kBtNb * (kBtNb - 1) / 2; e += 256) {
    int i = 1;
    while ((i + 1) * i / 2 <= e) ++i;  // e = i(i-1)/2 + l, l < i
    const int l = e - i * (i - 1) / 2;
    double2 gsum = make_double2(0.0, 0.0);
    if (i < nr)
      for (int p = 0; p < a.nsplit; ++p) {
        const double2 gv = a.Gp[((long)p * a.ng + g) * kBtNb * kBtNb + l + (long)i * kBtNb];
        gsum.x += gv.x;
        gsum.y += gv.y;
      }
    G[e] = gsum;
  }
  for (int e = tid; e < kBtNb * (kBtNb + 1) / 2; e += 256) T[e] = make_double2(0.0, 0.0);
  __syncthreads();
  if (tid < nr) T[tix(tid, tid)] = tau[k0 + tid];
  __syncthreads();
  for (int bs = 1; bs < kBtNb; bs *= 2) {
    const int per_pair = bs * bs, total = (kBtNb / (2 * bs)) * per_pair;  // = 32 bs <= 1024
    double2 x[4];
    // X(p, c) = sum_{q in B, q <= c} G(p, q) T(q, c), p in A, c in B
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      x[u] = make_double2(0.0, 0.0);
      if (e < total) {
        const int pr = e / per_pair, r = e % per_pair;
        const int a0 = 2 * bs * pr, b0 = a0 + bs;
        const int p = a0 + r / bs, c = b0 + r % bs;
        for (int q = b0; q <= c; ++q) x[u] = dadd(x[u], dmul(G[gix(p, q)], T[tix(q, c)]));
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      if (e < total) {
        const int pr = e / per_pair, r = e % per_pair;
        const int a0 = 2 * bs * pr, b0 = a0 + bs;
        G[gix(a0 + r / bs, b0 + r % bs)] = x[u];
      }
    }
    __syncthreads();
    // T(r, c) = -sum_{p in A, p >= r} T(r, p) X(p, c), r in A, c in B
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      if (e < total) {
        const int pr = e / per_pair, rr = e % per_pair;
        const int a0 = 2 * bs * pr, b0 = a0 + bs;
        const int r = a0 + rr / bs, c = b0 + rr % bs;
        double2 acc = make_double2(0.0, 0.0);
        for (int p = r; p < b0; ++p) acc = dadd(acc, dmul(T[tix(r, p)], G[gix(p, c)]));
        T[tix(r, c)] = make_double2(-acc.x, -acc.y);
      }
    }
    __syncthreads();
  }
  double2* out = a.Tb + (long)g * kBtNb * kBtNb;
  for (int e = tid; e < kBtNb * kBtNb; e += 256) {
    const int r = e % kBtNb, c = e / kBtNb;
    out[e] = r <= c ? T[tix(r, c)] : make_double2(0.0, 0.0);
  }
}

}  // namespace

static int bt_nblocks(int n) { return n > 1 ? (n - 2) / kBtNb + 1 : 0; }

size_t bt_scratch_elems(int n) {
  const int ng = bt_nblocks(n);
  return (size_t)ng * kBtNb * kBtNb * (1 + kBtSplitG) + (size_t)(kBtSplitW + 1) * kBtNb * n;
}

hipError_t launch_backtransform(const BackTrArgs& b, hipStream_t s) {
  const int n = b.n, nb = b.nb;
  if (n < 2) return hipSuccess;  // Q = I
  const int ng = bt_nblocks(n);
  BtArgs a{};
  a.n = n;
  a.ng = ng;
  a.Vx = b.V;
  a.Yx = b.Y;
  a.Z = b.Z;
  a.tau = b.tau;
  a.Tb = b.scratch;
  a.Gp = b.scratch + (size_t)ng * kBtNb * kBtNb;
  a.Wp = a.Gp + (size_t)ng * kBtNb * kBtNb * kBtSplitG;
  a.sV = b.sV;
  a.sY = b.sY;
  a.sZ = b.sZ;
  a.sW = b.s_scratch;
  k_bt_explicit<<<dim3((unsigned)(((long)n * n + 255) / 256), nb), 256, 0, s>>>(n, b.V, b.sV);
  const int mt = (n - 1 + kTM - 1) / kTM;  // row tiles of the largest block (m = n - 1)
  a.nsplit = kBtSplitG;
  k_bt_gemm<BT_GRAM><<<dim3(kBtNb / kTN, 1, nb * ng * kBtSplitG), 256, 0, s>>>(a, ng * kBtSplitG);
  k_bt_tmat<<<dim3(ng, nb), 256, 0, s>>>(a);
  a.nsplit = 1;
  k_bt_gemm<BT_YMAT><<<dim3(kBtNb / kTN, mt, nb * ng), 256, 0, s>>>(a, ng);
  const int nt = (n + kTN - 1) / kTN;
  a.nsplit = kBtSplitW;
  for (int g = ng - 1; g >= 0; --g) {
    a.g = g;
    const int m = n - (kBtNb * g + 1);
    k_bt_gemm<BT_APPLY_W><<<dim3(nt, 1, nb * kBtSplitW), 256, 0, s>>>(a, kBtSplitW);
    k_bt_wsum<<<dim3((unsigned)(((long)kBtNb * n + 255) / 256), nb), 256, 0, s>>>(a);
    k_bt_gemm<BT_APPLY_Z><<<dim3(nt, (m + kTM - 1) / kTM, nb), 256, 0, s>>>(a, 1);
  }
  return hipGetLastError();
}

}  // namespace slrx
