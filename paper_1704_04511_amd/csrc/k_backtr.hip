// Back-transformation of the tridiagonal eigenvectors, U = Q Z (FP64), last
// stage of the Gram eigen-decomposition in the weight update (Sec. III.C,
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
//   APPLY_Z: Z(r0:, :) -= Y_g W     (m x n, K = nr),  W summed over the partials.
struct BtArgs {
  int n, ng, nsplit, g;
  const double2* Vx;  // reflectors, column-major n x n, explicit zeros and unit entries
  double2* Yx;        // Y blocks, column-major n x n
  double2* Z;         // eigenvectors, column-major n x n
  double2* Gp;        // Gram partials of the blocks
  double2* Tb;        // T of the blocks, column-major nb x nb each
  double2* Wp;        // V^H Z partials, column-major nb x n each
};

template <int KIND>
__global__ __launch_bounds__(256) void k_bt_gemm(BtArgs a) {
  __shared__ double Lar[kKC][kTM + 1], Lai[kKC][kTM + 1];  // padded against bank conflicts
  __shared__ double Lbr[kKC][kTN + 1], Lbi[kKC][kTN + 1];
  const int n = a.n;
  int g, z;
  if (KIND == BT_GRAM) {
    g = blockIdx.z / a.nsplit;
    z = blockIdx.z % a.nsplit;
  } else if (KIND == BT_YMAT) {
    g = blockIdx.z;
    z = 0;
  } else {
    g = a.g;
    z = blockIdx.z;
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
  for (int kc = kb; kc < ke; kc += kKC) {
    // A tile: rows i0.., k kc..
    for (int e = tid; e < kTM * kKC; e += 256) {
      int i, kk;
      double2 v = make_double2(0.0, 0.0);
      if (KIND == BT_GRAM || KIND == BT_APPLY_W) {  // A(i, r) = conj(V(r0 + r, k0 + i))
        i = e / kKC;
        kk = e % kKC;
        const int r = kc + kk;
        if (i0 + i < M && r < ke) {
          v = a.Vx[(long)(r0 + r) + (long)(k0 + i0 + i) * n];
          v.y = -v.y;
        }
      } else {  // A(r, l) column-major: V for YMAT, Y for APPLY_Z
        kk = e / kTM;
        i = e % kTM;
        const int l = kc + kk;
        if (i0 + i < M && l < ke) {
          const double2* src = KIND == BT_YMAT ? a.Vx : a.Yx;
          v = src[(long)(r0 + i0 + i) + (long)(k0 + l) * n];
        }
      }
      Lar[kk][i] = v.x;
      Lai[kk][i] = v.y;
    }
    // B tile: k kc.., columns j0..
    {
      const int j = tid / kKC, kk = tid % kKC;
      const int k = kc + kk, c = j0 + j;
      double2 v = make_double2(0.0, 0.0);
      if (k < ke && c < N) {
        if (KIND == BT_GRAM) v = a.Vx[(long)(r0 + k) + (long)(k0 + c) * n];
        else if (KIND == BT_YMAT) v = a.Tb[(long)g * kBtNb * kBtNb + k + (long)c * kBtNb];
        else if (KIND == BT_APPLY_W) v = a.Z[(long)(r0 + k) + (long)c * n];
        else {
          for (int p = 0; p < a.nsplit; ++p) {
            const double2 w = a.Wp[(long)p * kBtNb * n + k + (long)c * kBtNb];
            v.x += w.x;
            v.y += w.y;
          }
        }
      }
      Lbr[kk][j] = v.x;
      Lbi[kk][j] = v.y;
    }
    __syncthreads();
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
      double2* dst = a.Z + (long)(r0 + i) + (long)c * n;
      *dst = make_double2(dst->x - r.x, dst->y - r.y);
    }
  }
}

// Reflectors in explicit form, in place: column k of the n x n column-major
// matrix becomes v_k (zero above row k+1, one at row k+1; the last column is zero).
__global__ void k_bt_explicit(int n, double2* V) {
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= (long)n * n) return;
  const int R = (int)(o % n), k = (int)(o / n);
  if (R < k + 1) V[o] = make_double2(0.0, 0.0);
  else if (R == k + 1) V[o] = make_double2(1.0, 0.0);
}

// T of each block from its Gram matrix (summed over the partials) and tau.
// T is upper triangular, kept packed by columns in LDS: T(l, q) at q(q+1)/2 + l.
__global__ __launch_bounds__(64) void k_bt_tmat(BtArgs a, const double2* tau) {
  __shared__ double2 T[kBtNb * (kBtNb + 1) / 2];
  __shared__ double2 t[kBtNb];
  const int g = blockIdx.x, l = threadIdx.x;
  const int k0 = kBtNb * g, nr = min(kBtNb, a.n - 1 - k0);
  for (int i = 0; i < nr; ++i) {
    const double2 ti = tau[k0 + i];
    if (l < i) {
      double2 gsum = make_double2(0.0, 0.0);
      for (int p = 0; p < a.nsplit; ++p) {
        const double2 gv = a.Gp[((long)p * a.ng + g) * kBtNb * kBtNb + l + (long)i * kBtNb];
        gsum.x += gv.x;
        gsum.y += gv.y;
      }
      // t_l = -tau_i (v_l^H v_i)
      t[l] = make_double2(-(ti.x * gsum.x - ti.y * gsum.y), -(ti.x * gsum.y + ti.y * gsum.x));
    }
    __syncthreads();
    if (l < i) {
      double2 acc = make_double2(0.0, 0.0);
      for (int q = l; q < i; ++q) acc = dadd(acc, dmul(T[q * (q + 1) / 2 + l], t[q]));
      T[i * (i + 1) / 2 + l] = acc;
    }
    if (l == i) T[i * (i + 1) / 2 + i] = ti;
    __syncthreads();
  }
  double2* out = a.Tb + (long)g * kBtNb * kBtNb;
  for (int c = 0; c < kBtNb; ++c)
    out[l + (long)c * kBtNb] = (l <= c && c < nr) ? T[c * (c + 1) / 2 + l] : make_double2(0.0, 0.0);
}

}  // namespace

static int bt_nblocks(int n) { return n > 1 ? (n - 2) / kBtNb + 1 : 0; }

size_t bt_scratch_elems(int n) {
  const int ng = bt_nblocks(n);
  return (size_t)ng * kBtNb * kBtNb * (1 + kBtSplitG) + (size_t)kBtSplitW * kBtNb * n;
}

hipError_t launch_backtransform(const BackTrArgs& b, hipStream_t s) {
  const int n = b.n;
  if (n < 2) return hipSuccess;  // Q = I
  const int ng = bt_nblocks(n);
  BtArgs a{};
  a.n = n;
  a.ng = ng;
  a.Vx = b.V;
  a.Yx = b.Y;
  a.Z = b.Z;
  a.Tb = b.scratch;
  a.Gp = b.scratch + (size_t)ng * kBtNb * kBtNb;
  a.Wp = a.Gp + (size_t)ng * kBtNb * kBtNb * kBtSplitG;
  k_bt_explicit<<<(unsigned)(((long)n * n + 255) / 256), 256, 0, s>>>(n, b.V);
  const int mt = (n - 1 + kTM - 1) / kTM;  // row tiles of the largest block (m = n - 1)
  a.nsplit = kBtSplitG;
  k_bt_gemm<BT_GRAM><<<dim3(kBtNb / kTN, 1, ng * kBtSplitG), 256, 0, s>>>(a);
  k_bt_tmat<<<ng, 64, 0, s>>>(a, b.tau);
  a.nsplit = 1;
  k_bt_gemm<BT_YMAT><<<dim3(kBtNb / kTN, mt, ng), 256, 0, s>>>(a);
  const int nt = (n + kTN - 1) / kTN;
  a.nsplit = kBtSplitW;
  for (int g = ng - 1; g >= 0; --g) {
    a.g = g;
    const int m = n - (kBtNb * g + 1);
    k_bt_gemm<BT_APPLY_W><<<dim3(nt, 1, kBtSplitW), 256, 0, s>>>(a);
    k_bt_gemm<BT_APPLY_Z><<<dim3(nt, (m + kTM - 1) / kTM, 1), 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace slrx
