// Eigenpairs of the real symmetric tridiagonal matrix left by the Householder
// reduction (FP64), middle stage of the Gram eigen-decomposition in the weight
// update (Sec. III.B, Algorithm 1 step 1): divide and conquer.
//
// The index range is halved recursively down to single entries; every
// coupling E[c-1] between the halves at a split c is torn off as a rank-one
// term |E[c-1]| v v^T, v = (e_{c-1}, sign(E[c-1]) e_c), so each diagonal entry
// first loses |E[i-1]| + |E[i]|.  The tree is then merged bottom-up, one launch
// sequence per tree level with every node of the level in parallel.  A merge of
// children with eigenpairs (D1, Q1), (D2, Q2) solves
//   diag(D1, D2) + rho z z^T,  z = (last row of Q1, sign * first row of Q2) / sqrt(2),
//   rho = 2 |E[c-1]|:
//   1. deflate (one thread, in sorted order): entries with rho |z_i| <= tol keep
//      (d_i, e_i); nearly equal d_i, d_j are rotated so that one z entry vanishes
//      (tol = 8 eps max(max |d|, max |z|), the usual criterion);
//   2. every remaining root lambda_j of 1 + rho sum z_i^2 / (d_i - lambda) lies in
//      (d_j, d_{j+1}) (the last in (d_k, d_k + rho |z|^2)); it is found by
//      bisection on the bit pattern of its offset tau from the nearer pole, so
//      differences d_i - lambda_j = (d_i - d_origin) - tau keep full relative
//      accuracy;
//   3. z is recomputed from the roots (Loewner's formula, Gu and Eisenstat),
//      which makes the vectors u_j = (D - lambda_j)^{-1} z_hat orthogonal to
//      working precision;
//   4. the merged eigenvectors are the sorted, rotated columns of
//      diag(Q1, Q2) times U (an FP64 MFMA product); deflated columns are copied.
// Eigenvector matrices are kept row-major, one n x n array with every node's
// block on the diagonal; the final eigenvalues are sorted ascending and the
// eigenvectors are written column-major as complex numbers (imaginary part 0)
// for the back-transformation.  All reductions have a fixed order.
#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace slrx {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kDcMaxN = 3000;

struct DcArgs {
  int n;
  double* D;          // diagonal in, eigenvalues out
  const double* E;    // off-diagonal
  double* Q;          // eigenvector state, row-major n x n
  double* Qs;         // gathered / rotated columns of a merge, row-major n x n
  double* U;          // merge eigenvectors, column-major blocks, n x n
  const int4* nodes;  // (start, size, size of the first child, unused) per internal node
  int node0;          // first node of the level being merged
  int* ws_i;          // 4 n ints: perm, order, rot_p, rot_q
  double* ws_d;       // 7 n doubles: dl, zl, rot_c, rot_s, tau, zhat, deflation records
  int* ws_node;       // 4 ints per node: k, nrot, 0, 0
  int* ws_orig;       // n ints: pole each root is measured from
  double2* Z;         // output eigenvectors, complex column-major n x n
  int count;          // nodes in the level being merged
  long sQ, sZ, s_wsi, s_wsd;  // strides between the problems of a batch
};

// The arguments of problem b of a batch (D, E have stride n).
SLRX_DEV DcArgs dc_at(DcArgs a, int b) {
  a.D += (long)b * a.n;
  a.E += (long)b * a.n;
  a.Q += b * a.sQ;
  a.Qs += b * a.sQ;
  a.U += b * a.sQ;
  a.ws_i += b * a.s_wsi;
  a.ws_node += b * a.s_wsi;
  a.ws_orig += b * a.s_wsi;
  a.ws_d += b * a.s_wsd;
  a.Z += b * a.sZ;
  return a;
}

SLRX_DEV double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
SLRX_DEV double wave_prod(double v) {
  for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off, 64);
  return v;
}
SLRX_DEV double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Tear every coupling off the diagonal; leaves (single entries) start with Q = 1.
__global__ void k_dc_init(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.y);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  double d = a.D[i];
  if (i >= 1) d -= fabs(a.E[i - 1]);
  if (i <= a.n - 2) d -= fabs(a.E[i]);
  a.D[i] = d;
  a.Q[(long)i * a.n + i] = 1.0;
}

// Sort, z, deflation of one merge (one workgroup per node, its size a multiple
// of 64 that covers the largest node of the level, at most kDefNT).
constexpr int kDefNT = 1024;
constexpr int kDefRank = 256;  // largest node sorted by rank counting
inline size_t dc_deflate_lds(int m) { return (size_t)m * (4 * sizeof(double) + 4 * sizeof(int)); }

// Inclusive block scan of chunk[0, nt) (sum, or max when MAX).
template <bool MAX>
SLRX_DEV void block_scan(int* chunk, int tid, int nt) {
  for (int off = 1; off < nt; off <<= 1) {
    const int v = tid >= off ? chunk[tid - off] : (MAX ? -1 : 0);
    __syncthreads();
    chunk[tid] = MAX ? max(chunk[tid], v) : chunk[tid] + v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kDefNT) void k_dc_deflate(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.y);
  extern __shared__ double lds[];
  const int4 nd = a.nodes[a.node0 + blockIdx.x];
  const int s = nd.x, m = nd.y, n1 = nd.z, n = a.n;
  const int node = a.node0 + blockIdx.x;
  const int nt = blockDim.x;
  double* dv = lds;     // node entries; after the sort, the kept entries' poles
  double* zv = dv + m;  // node couplings; after the sort, the kept entries' couplings
  double* ds = zv + m;  // sorted poles
  double* zs = ds + m;  // sorted couplings
  int* perm = (int*)(zs + m);  // sorted position -> node column
  int* order = perm + m;       // final column order -> sorted position
  int* flag = order + m;       // per sorted entry, see below
  int* ki = flag + m;          // kept entry i -> sorted position
  __shared__ int chunk[kDefNT];
  __shared__ double red[2][kDefNT / 64];
  __shared__ int kout, nkept, nrout;
  __shared__ unsigned long long cbits[(kDcMaxN + 63) / 64];  // candidate pairs, by kept index
  const int tid = threadIdx.x, lane = tid & 63;
  const double beta = a.E[s + n1 - 1];
  const double rho = 2.0 * fabs(beta);
  const double sgn = beta >= 0.0 ? 1.0 : -1.0;
  const double r2 = 0.70710678118654752440;
  for (int i = tid; i < m; i += nt) {
    dv[i] = a.D[s + i];
    zv[i] = i < n1 ? a.Q[(long)(s + n1 - 1) * n + s + i] * r2 : sgn * a.Q[(long)(s + n1) * n + s + i] * r2;
  }
  __syncthreads();
  // Sort by (pole, node column), the stable order. Up to kDefRank entries by
  // rank (each thread counts the entries before its own); above, a bitonic
  // network over the next power of two, keys staged in ds/zs and columns in
  // order/flag/ki (free until the sort is done; P2 doubles < 2m, P2 ints < 3m).
  double dmax = 0.0, zmax = 0.0;
  if (m <= kDefRank) {
    for (int i = tid; i < m; i += nt) {
      const double di = dv[i];
      int r = 0;
      int j = 0;
      for (; j + 8 <= m; j += 8) {  // eight independent LDS reads in flight
        double dj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) dj[u] = dv[j + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) r += (dj[u] < di) || (dj[u] == di && j + u < i);
      }
      for (; j < m; ++j) r += (dv[j] < di) || (dv[j] == di && j < i);
      perm[r] = i;
      dmax = fmax(dmax, fabs(di));
      zmax = fmax(zmax, fabs(zv[i]));
    }
  } else {
    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    double* sk = ds;
    int* si = order;
    for (int i = tid; i < P2; i += nt) {
      sk[i] = i < m ? dv[i] : __builtin_huge_val();
      si[i] = i;
      if (i < m) {
        dmax = fmax(dmax, fabs(dv[i]));
        zmax = fmax(zmax, fabs(zv[i]));
      }
    }
    __syncthreads();
    for (int kb = 2; kb <= P2; kb <<= 1) {
      for (int j = kb >> 1; j > 0; j >>= 1) {
        for (int q = tid; q < P2 / 2; q += nt) {
          const int lo = 2 * j * (q / j) + (q % j), hi = lo + j;
          const double a = sk[lo], b = sk[hi];
          const int ia = si[lo], ib = si[hi];
          const bool gt = a > b || (a == b && ia > ib);
          if (gt == ((lo & kb) == 0)) {
            sk[lo] = b;
            sk[hi] = a;
            si[lo] = ib;
            si[hi] = ia;
          }
        }
        __syncthreads();
      }
    }
    for (int r = tid; r < m; r += nt) perm[r] = si[r];
  }
  dmax = wave_max(dmax);
  zmax = wave_max(zmax);
  if (lane == 0) {
    red[0][tid >> 6] = dmax;
    red[1][tid >> 6] = zmax;
  }
  __syncthreads();
  for (int t = tid; t < m; t += nt) {
    ds[t] = dv[perm[t]];
    zs[t] = zv[perm[t]];
  }
  double mx = 0.0;
  for (int w = 0; w < nt / 64; ++w) mx = fmax(mx, fmax(red[0][w], red[1][w]));
  const double tol = 8.0 * __DBL_EPSILON__ * mx;
  __syncthreads();
  // Deflation with LAPACK's criteria, in sorted order. An entry whose coupling
  // is negligible (rho |z| <= tol) is an eigenpair as it stands. Of two
  // consecutive kept entries p < t, with c = z_t / r, s = -z_p / r, r^2 = z_p^2
  // + z_t^2, the rotation that moves z_p into z_t deflates p when
  // |(d_t - d_p) c s| <= tol; t then carries the coupling r and the pole
  // d_p s^2 + d_t c^2, and the test of the next pair uses them. Along a chain of
  // rotations these are running sums: r^2 = Z2 = sum z^2 and the pole is
  // N / Z2 with N = sum d z^2, and the test reads
  //   (d_t Z2 - N)^2 z_t^2 <= tol^2 Z2 (Z2 + z_t^2)^2,
  // products only. One thread walks the kept entries with that test (poles
  // scaled by 1/mx, so that tol becomes 8 eps); c, s and the deflated poles of
  // the rotations it records follow in parallel.
  //   flag bit 0: kept; bit 1: rotated into (bits 3.. hold the entry rotated
  //   away into it); bit 2: rotated away.
  const int per = (m + nt - 1) / nt;
  const int u0 = tid * per, u1 = min(m, u0 + per);
  int cnt = 0;
  for (int u = u0; u < u1; ++u) {
    const int f = rho * fabs(zs[u]) > tol;
    flag[u] = f;
    cnt += f;
  }
  chunk[tid] = cnt;
  __syncthreads();
  block_scan<false>(chunk, tid, nt);
  {
    int i = chunk[tid] - cnt;
    for (int u = u0; u < u1; ++u) {
      if (!flag[u]) continue;
      dv[i] = ds[u];
      zv[i] = zs[u];
      ki[i] = u;
      ++i;
    }
  }
  if (tid == 0) nkept = chunk[nt - 1];
  __syncthreads();
  const int nk = nkept;
  double* rc = a.ws_d + 2 * n + s;   // rotation c; Z2 before it while walking
  double* rsn = a.ws_d + 3 * n + s;  // rotation s; N / mx before it while walking
  double* rec = a.ws_d + 6 * n + s;  // kept index of the entry rotated away, ~index at a chain start
  int* rp = a.ws_i + 2 * n + s;
  int* rq = a.ws_i + 3 * n + s;
  const double inv = 1.0 / mx;
  const double tol2 = 64.0 * __DBL_EPSILON__ * __DBL_EPSILON__;
  // Pairs (i-1, i) whose entry values pass the test with twice its tolerance:
  // a pair outside these, reached with the values of i-1 unchanged, does not
  // rotate, and the walk skips it.
  for (int i0 = tid & ~63; i0 < nk; i0 += nt) {
    const int i = i0 + lane;
    bool cand = false;
    if (i >= 1 && i < nk) {
      const double zp = zv[i - 1], zt = zv[i];
      const double Z2 = zp * zp, zt2 = zt * zt, r2 = Z2 + zt2;
      const double x = (dv[i] * inv) * Z2 - (dv[i - 1] * inv) * Z2;
      cand = x * x * zt2 <= 2.0 * tol2 * Z2 * r2 * r2 || !(2.0 * tol2 * Z2 * r2 * r2 >= 1e-290);
    }
    const unsigned long long b = __ballot(cand);
    if (lane == 0) cbits[i0 >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (nk + 63) >> 6;
    auto next = [&](int f) {  // smallest candidate i >= f, or -1
      for (int w = f >> 6; w < nw; ++w) {
        unsigned long long b = cbits[w];
        if (w == (f >> 6)) b &= ~0ull << (f & 63);
        if (b) return (w << 6) + __builtin_ctzll(b);
      }
      return -1;
    };
    int nrot = 0;
    int i = nk >= 2 ? next(1) : -1;
    while (i >= 0) {
      // a chain from the pair (i-1, i): Z2, N of the entry carrying the coupling
      const double zp = zv[i - 1];
      double Z2 = zp * zp, N = (dv[i - 1] * inv) * Z2;
      bool start = true;
      double zt = zv[i], dt = dv[i] * inv;
      for (;;) {
        const int in = min(i + 1, nk - 1);  // next entry's values in flight
        const double zn = zv[in], dn = dv[in];
        const double zt2 = zt * zt;
        const double r2 = Z2 + zt2;
        const double x = dt * Z2 - N;
        const double rhs = tol2 * Z2 * r2 * r2;
        bool rot;
        if (rhs >= 1e-290) {
          rot = x * x * zt2 <= rhs;
        } else {  // products near underflow: the test in its direct form
          const double r = sqrt(r2);
          rot = fabs((dt - N / Z2) * (zt / r) * (sqrt(Z2) / r)) <= 8.0 * __DBL_EPSILON__;
        }
        if (!rot) break;
        rec[nrot] = start ? (double)~(i - 1) : (double)(i - 1);
        rc[nrot] = Z2;
        rsn[nrot] = N;
        ++nrot;
        Z2 = r2;
        N = N + dt * zt2;
        start = false;
        if (++i >= nk) break;
        zt = zn;
        dt = dn * inv;
      }
      i = i < nk ? next(i + 1) : -1;
    }
    nrout = nrot;
  }
  __syncthreads();
  const int nrot = nrout;
  for (int j = tid; j < nrot; j += nt) {
    const int e = (int)rec[j];
    const bool start = e < 0;
    const int ip = start ? ~e : e, it = ip + 1;
    const bool end = j == nrot - 1 || (int)rec[j + 1] < 0;  // the next rotation starts a new chain
    const int p = ki[ip], t = ki[it];
    const double zt = zv[it], dt = dv[it];
    const double Z2 = rc[j];
    const double zp = start ? zv[ip] : sqrt(Z2);
    const double dp = start ? dv[ip] : (rsn[j] / Z2) * mx;
    const double r = hypot(zt, zp);
    const double c = zt / r, sv = -zp / r;
    rp[j] = p;
    rq[j] = t;
    rc[j] = c;
    rsn[j] = sv;
    ds[p] = dp * c * c + dt * sv * sv;
    zs[p] = 0.0;
    if (end) {
      ds[t] = dp * sv * sv + dt * c * c;
      zs[t] = r;
    }
    flag[t] = 3 | (end ? 0 : 4) | (p << 3);
    if (start) flag[p] = 5;
  }
  __syncthreads();
  // Final order: the kept entries that were not rotated away, in sorted order,
  // then the deflated ones from the back in the order of deflation (an entry
  // with a negligible coupling at its own position, a rotated-away entry at the
  // position of the entry it was rotated into). Both counts by one block scan,
  // packed into one int (m < 65536).
  cnt = 0;
  for (int u = u0; u < u1; ++u) {
    const int f = flag[u];
    if (!(f & 1) || (f & 2)) cnt += 1;
    if ((f & 1) && !(f & 4)) cnt += 0x10000;
  }
  chunk[tid] = cnt;
  __syncthreads();
  block_scan<false>(chunk, tid, nt);
  int be = (chunk[tid] - cnt) & 0xffff, bk = (chunk[tid] - cnt) >> 16;
  for (int u = u0; u < u1; ++u) {
    const int f = flag[u];
    if (!(f & 1) || (f & 2)) order[m - 1 - be++] = (f & 2) ? (f >> 3) : u;
    if ((f & 1) && !(f & 4)) order[bk++] = u;
  }
  if (tid == 0) {
    kout = chunk[nt - 1] >> 16;
    a.ws_node[4 * node] = kout;
    a.ws_node[4 * node + 1] = nrot;
  }
  __syncthreads();
  const int k = kout;
  double* dl = a.ws_d + s;
  double* zl = a.ws_d + n + s;
  for (int c = tid; c < m; c += nt) {
    const int t = order[c];
    a.ws_i[n + s + c] = t;
    a.ws_i[s + t] = perm[t];
    if (c < k) {
      dl[c] = ds[t];
      zl[c] = zs[t];
    } else {
      a.D[s + c] = ds[t];  // deflated eigenvalue
    }
  }
}

// Columns of diag(Q1, Q2) in sorted order, deflation rotations, then the final
// column order (non-deflated first); one wave per row of the node.
__global__ __launch_bounds__(256) void k_dc_gather(DcArgs a0, int mmax) {
  const DcArgs a = dc_at(a0, blockIdx.z);
  extern __shared__ double lds[];
  const int node = a.node0 + blockIdx.y;
  const int4 nd = a.nodes[node];
  const int s = nd.x, m = nd.y, n1 = nd.z, n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = blockIdx.x * 4 + wave;
  double* row = lds + wave * mmax;
  const bool active = r < m;
  const int* perm = a.ws_i + s;
  const int* order = a.ws_i + n + s;
  if (active) {
    const bool top = r < n1;
    const double* qrow = a.Q + (long)(s + r) * n + s;
    for (int t = lane; t < m; t += 64) {
      const int col = perm[t];
      row[t] = (top == (col < n1)) ? qrow[col] : 0.0;
    }
  }
  __syncthreads();
  if (active && lane == 0) {
    const int nrot = a.ws_node[4 * node + 1];
    const int* rp = a.ws_i + 2 * n + s;
    const int* rq = a.ws_i + 3 * n + s;
    const double* rc = a.ws_d + 2 * n + s;
    const double* rsn = a.ws_d + 3 * n + s;
    for (int q = 0; q < nrot; ++q) {
      const int p0 = rp[q], p1 = rq[q];
      const double c = rc[q], sv = rsn[q];
      const double x = row[p0], y = row[p1];
      row[p0] = c * x + sv * y;
      row[p1] = c * y - sv * x;
    }
  }
  __syncthreads();
  if (active) {
    double* out = a.Qs + (long)(s + r) * n + s;
    for (int c = lane; c < m; c += 64) out[c] = row[order[c]];
  }
}

// Terms of f = 1 + psi + phi at offset tau from the origin pole, over one
// wave: psi sums the poles at or left of d_j, phi the poles right of it
// (values and derivatives), fa the magnitudes (rounding bound of f).
struct SecTerms {
  double psi, dpsi, phi, dphi, fa;
};
SLRX_DEV SecTerms secular(const double* dl, const double* z2, int k, int j, double dor, double rho, double tau) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x & 63; i < k; i += 64) {
    const double r = 1.0 / ((dl[i] - dor) - tau);
    const double w = z2[i] * r;
    if (i <= j) {
      v[0] += w;
      v[1] += w * r;
    } else {
      v[2] += w;
      v[3] += w * r;
    }
    v[4] += fabs(w);
  }
  SecTerms t;
  t.psi = rho * wave_sum(v[0]);
  t.dpsi = rho * wave_sum(v[1]);
  t.phi = rho * wave_sum(v[2]);
  t.dphi = rho * wave_sum(v[3]);
  t.fa = rho * wave_sum(v[4]);
  return t;
}

// Midpoint of the bit patterns of two offsets of the same sign (one may be 0):
// halves the number of doubles between them, whatever their magnitudes.
SLRX_DEV double bit_mid(double x0, double x1, double sign) {
  const long long a = __double_as_longlong(fabs(x0)), b = __double_as_longlong(fabs(x1));
  return sign * __longlong_as_double(a + (b - a) / 2);
}

// One wave per root.  The root's offset tau from the nearer pole stays in a
// bracket [lo, hi] (f(lo) < 0 <= f(hi), f increasing).  Each step fits
// f ~ c + S / (a - tau) + T / (b - tau) at the current tau (a, b the offsets of
// the two poles around the root; S, T from the derivatives of psi and phi) and
// takes the model's root; a step that leaves the bracket or does not halve the
// previous step is replaced by bisection of the bit patterns, so the iteration
// always ends.  It stops when |f| is within the rounding of its terms.
__global__ __launch_bounds__(256) void k_dc_secular(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.z);
  extern __shared__ double sec_lds[];
  const int node = a.node0 + blockIdx.y;
  const int4 nd = a.nodes[node];
  const int s = nd.x, n = a.n;
  const int k = a.ws_node[4 * node];
  // the node's poles and squared couplings, read by every step of the four roots
  double* dl = sec_lds;
  double* z2 = sec_lds + k;
  if (blockIdx.x * 4 >= k) return;
  for (int i = threadIdx.x; i < k; i += 256) {
    dl[i] = a.ws_d[s + i];
    const double z = a.ws_d[n + s + i];
    z2[i] = z * z;
  }
  __syncthreads();
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= k) return;
  const double rho = 2.0 * fabs(a.E[s + nd.z - 1]);
  const bool last = j == k - 1;
  int o;
  double sign, hiv;
  if (!last) {
    const double gap = dl[j + 1] - dl[j];
    const SecTerms t = secular(dl, z2, k, j, dl[j], rho, 0.5 * gap);
    if (1.0 + t.psi + t.phi >= 0.0) {
      o = j;
      sign = 1.0;
    } else {
      o = j + 1;
      sign = -1.0;
    }
    hiv = 0.5 * gap;
  } else {
    double zz = 0.0;
    for (int i = threadIdx.x & 63; i < k; i += 64) zz += z2[i];
    o = j;
    sign = 1.0;
    hiv = rho * wave_sum(zz);
  }
  const double dor = dl[o];
  const double pa = dl[j] - dor;                     // left pole
  const double pb = last ? 0.0 : dl[j + 1] - dor;    // right pole (unused for the last root)
  double lo = sign > 0.0 ? 0.0 : -hiv, hi = sign > 0.0 ? hiv : 0.0;
  double x = sign * hiv;  // the midpoint (the far end for the last root)
  double prev_step = 1e300, fprev = 0.0;
  for (int it = 0; it < 200; ++it) {
    const SecTerms t = secular(dl, z2, k, j, dor, rho, x);
    const double f = 1.0 + t.psi + t.phi;
    if (fabs(f) <= 4.0 * __DBL_EPSILON__ * (1.0 + t.fa)) break;
    if (f < 0.0) lo = x;
    else hi = x;
    const long long nb =
        __double_as_longlong(fmax(fabs(lo), fabs(hi))) - __double_as_longlong(fmin(fabs(lo), fabs(hi)));
    if (nb <= 1) break;
    double xn = 0.0;
    bool ok = false;
    const double S = t.dpsi * (pa - x) * (pa - x);
    if (last) {
      const double c = f - S / (pa - x);
      if (c > 0.0) {
        xn = pa + S / c;
        ok = true;
      }
    } else {
      // When the last step cut |f| by less than 10x (a root close to a pole whose
      // coupling is tiny: the curvature of the other poles is then fitted onto it),
      // the nearer pole keeps its exact weight and the rest of f' goes to the other.
      double Sm = S, T = t.dphi * (pb - x) * (pb - x);
      if (it > 0 && fabs(f) > 0.1 * fabs(fprev)) {
        const double fp = t.dpsi + t.dphi;
        if (o == j) {
          Sm = rho * z2[j];
          T = (fp - Sm / ((pa - x) * (pa - x))) * (pb - x) * (pb - x);
        } else {
          T = rho * z2[j + 1];
          Sm = (fp - T / ((pb - x) * (pb - x))) * (pa - x) * (pa - x);
        }
      }
      const double c = f - Sm / (pa - x) - T / (pb - x);
      // c (pa - y)(pb - y) + S (pb - y) + T (pa - y) = 0
      const double qa = c, qb = -(c * (pa + pb) + Sm + T), qc = c * pa * pb + Sm * pb + T * pa;
      const double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        const double q = -0.5 * (qb + copysign(sqrt(disc), qb));
        if (qa != 0.0) {
          const double y = q / qa;
          if (y > lo && y < hi) {
            xn = y;
            ok = true;
          }
        }
        if (q != 0.0) {
          const double y = qc / q;
          if (y > lo && y < hi) {
            xn = y;
            ok = true;
          }
        }
      }
    }
    ok = ok && xn > lo && xn < hi && xn != 0.0;
    double step = ok ? fabs(xn - x) : 1e300;
    if (!ok || (it >= 2 && step > 0.5 * prev_step)) {
      xn = bit_mid(sign > 0.0 ? lo : hi, sign > 0.0 ? hi : lo, sign);
      step = fabs(xn - x);
    }
    prev_step = step;
    fprev = f;
    x = xn;
  }
  if ((threadIdx.x & 63) == 0) {
    a.D[s + j] = dor + x;
    a.ws_orig[s + j] = o;
    a.ws_d[4 * n + s + j] = x;
  }
}

// z_hat_i^2 = (lambda_i - d_i) / rho * prod_{j != i} (lambda_j - d_i) / (d_j - d_i); one wave per i.
__global__ __launch_bounds__(256) void k_dc_zhat(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.z);
  const int node = a.node0 + blockIdx.y;
  const int4 nd = a.nodes[node];
  const int s = nd.x, n = a.n;
  const int k = a.ws_node[4 * node];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= k) return;
  const double rho = 2.0 * fabs(a.E[s + nd.z - 1]);
  const double* dl = a.ws_d + s;
  const double* zl = a.ws_d + n + s;
  const double* taus = a.ws_d + 4 * n + s;
  const int* orig = a.ws_orig + s;
  const double di = dl[i];
  double p = 1.0;
  for (int j = threadIdx.x & 63; j < k; j += 64) {
    const double lj_di = (dl[orig[j]] - di) + taus[j];
    p *= (j == i) ? lj_di / rho : lj_di / (dl[j] - di);
  }
  p = wave_prod(p);
  if ((threadIdx.x & 63) == 0) a.ws_d[5 * n + s + i] = copysign(sqrt(fmax(p, 0.0)), zl[i]);
}

// u_j = z_hat / (d - lambda_j), normalised; one wave per column j (column-major U block).
__global__ __launch_bounds__(256) void k_dc_vectors(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.z);
  const int node = a.node0 + blockIdx.y;
  const int4 nd = a.nodes[node];
  const int s = nd.x, n = a.n;
  const int k = a.ws_node[4 * node];
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= k) return;
  const double* dl = a.ws_d + s;
  const double* zh = a.ws_d + 5 * n + s;
  const double dor = dl[a.ws_orig[s + j]];
  const double tau = a.ws_d[4 * n + s + j];
  double* u = a.U + (long)(s + j) * n + s;
  double ss = 0.0;
  for (int i = threadIdx.x & 63; i < k; i += 64) {
    const double v = zh[i] / ((dl[i] - dor) - tau);
    u[i] = v;
    ss += v * v;
  }
  const double sc = 1.0 / sqrt(wave_sum(ss));
  for (int i = threadIdx.x & 63; i < k; i += 64) u[i] *= sc;
}

// Q_node(:, 0:k) = Qs(:, 0:k) U, Q_node(:, k:m) = Qs(:, k:m): 64 x 64 tiles,
// four waves of 32 x 32, f64 16x16x4 MFMA, K staged through LDS in chunks of 16.
__global__ __launch_bounds__(256) void k_dc_gemm(DcArgs a0) {
  constexpr int TB = 64, KC = 32;
  __shared__ double La[KC][TB + 1];
  __shared__ double Lb[KC][TB + 1];
  const DcArgs a = dc_at(a0, blockIdx.z / a0.count);
  const int node = a.node0 + blockIdx.z % a0.count;
  const int4 nd = a.nodes[node];
  const int s = nd.x, m = nd.y, n = a.n;
  const int k = a.ws_node[4 * node];
  const int i0 = blockIdx.y * TB, j0 = blockIdx.x * TB;
  if (i0 >= m || j0 >= m) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Qs = a.Qs + (long)s * n + s;
  double* Q = a.Q + (long)s * n + s;
  if (j0 >= k) {  // deflated columns only: copy
    for (int e = tid; e < TB * TB; e += 256) {
      const int r = i0 + e / TB, c = j0 + e % TB;
      if (r < m && c < m) Q[(long)r * n + c] = Qs[(long)r * n + c];
    }
    return;
  }
  const double* Um = a.U + (long)s * n + s;  // U(i, c) at Um[c * n + i]
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) acc[ta][tb] = v4d{0.0, 0.0, 0.0, 0.0};
  // the next K chunk is loaded into registers while the current one is multiplied
  constexpr int U = TB * KC / 256;
  double ra[U], rb[U];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      const int rr = e / KC, kidx = kc + e % KC;
      const int r = i0 + rr, c = j0 + rr;
      ra[u] = (r < m && kidx < k) ? Qs[(long)r * n + kidx] : 0.0;
      rb[u] = (c < k && kidx < k) ? Um[(long)c * n + kidx] : 0.0;
    }
  };
  load(0);
  for (int kc = 0; kc < k; kc += KC) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      La[e % KC][e / KC] = ra[u];
      Lb[e % KC][e / KC] = rb[u];
    }
    __syncthreads();
    if (kc + KC < k) load(kc + KC);
#pragma unroll
    for (int kq = 0; kq < KC; kq += 4) {
      const int kl = kq + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = La[kl][wi + 16 * t + (lane & 15)];
        bv[t] = Lb[kl][wj + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta], bv[tb], acc[ta][tb], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the f64 16x16x4 MFMA: item v of lane l is row l/16 + 4v, column l%16.
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i0 + wi + 16 * ta + (lane >> 4) + 4 * v;
        const int c = j0 + wj + 16 * tb + (lane & 15);
        if (r >= m || c >= m) continue;
        Q[(long)r * n + c] = c < k ? acc[ta][tb][v] : Qs[(long)r * n + c];
      }
}

// Ascending eigenvalues and their permutation (one workgroup): bitonic sort of
// (value, index) pairs in LDS, padded to a power of two; ties keep index order.
__global__ __launch_bounds__(1024) void k_dc_sort(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.x);
  extern __shared__ double lds[];
  const int n = a.n;
  int N = 1;
  while (N < n) N <<= 1;
  double* key = lds;
  int* idx = (int*)(key + N);
  for (int i = threadIdx.x; i < N; i += 1024) {
    key[i] = i < n ? a.D[i] : __builtin_inf();
    idx[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N / 2; t += 1024) {
        const int i = 2 * t - (t & (stride - 1));  // i has bit `stride` clear
        const int j = i + stride;
        const bool up = (i & size) == 0;
        const double ki = key[i], kj = key[j];
        const int ii = idx[i], ij = idx[j];
        const bool gt = ki > kj || (ki == kj && ii > ij);
        if (gt == up) {
          key[i] = kj;
          key[j] = ki;
          idx[i] = ij;
          idx[j] = ii;
        }
      }
      __syncthreads();
    }
  }
  for (int r = threadIdx.x; r < n; r += 1024) {
    a.ws_i[r] = idx[r];
    a.D[r] = key[r];
  }
}

// Z(r, c) = Q(r, perm(c)) as complex, column-major; 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_dc_convert(DcArgs a0) {
  const DcArgs a = dc_at(a0, blockIdx.z);
  double2* Z = a.Z;
  __shared__ double tile[64][65];
  const int n = a.n;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int rr = e / 64, cc = e % 64;
    const int r = r0 + rr, c = c0 + cc;
    tile[cc][rr] = (r < n && c < n) ? a.Q[(long)r * n + a.ws_i[c]] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int cc = e / 64, rr = e % 64;
    const int r = r0 + rr, c = c0 + cc;
    if (r < n && c < n) Z[(long)c * n + r] = make_double2(tile[cc][rr], 0.0);
  }
}

}  // namespace

// Internal nodes of the halving tree, deepest level first.
void dc_build_tree(int n, std::vector<int>& nodes, std::vector<int>& level_start) {
  std::vector<std::vector<int>> by_depth;
  struct Item { int s, m, depth; };
  std::vector<Item> stack{{0, n, 0}};
  while (!stack.empty()) {
    const Item it = stack.back();
    stack.pop_back();
    if (it.m <= 1) continue;
    const int n1 = it.m / 2;
    if ((int)by_depth.size() <= it.depth) by_depth.resize(it.depth + 1);
    by_depth[it.depth].insert(by_depth[it.depth].end(), {it.s, it.m, n1, 0});
    stack.push_back({it.s, n1, it.depth + 1});
    stack.push_back({it.s + n1, it.m - n1, it.depth + 1});
  }
  nodes.clear();
  level_start.clear();
  for (int d = (int)by_depth.size() - 1; d >= 0; --d) {
    level_start.push_back((int)nodes.size() / 4);
    nodes.insert(nodes.end(), by_depth[d].begin(), by_depth[d].end());
  }
  level_start.push_back((int)nodes.size() / 4);
}

size_t dc_ws_ints(int n) { return (size_t)4 * n + 4 * (size_t)n + n; }  // ws_i, ws_node, ws_orig
size_t dc_ws_doubles(int n) { return (size_t)7 * n; }
int dc_max_n() { return kDcMaxN; }

hipError_t launch_tdeig(const TdArgs& t, hipStream_t st) {
  const int n = t.n;
  if (n < 1 || n > kDcMaxN) return hipErrorInvalidValue;
  static LdsLimit lim_deflate, lim_gather, lim_sort;
  hipError_t e = lim_deflate.ensure((const void*)k_dc_deflate, dc_deflate_lds(kDcMaxN));
  if (e == hipSuccess) e = lim_gather.ensure((const void*)k_dc_gather, (size_t)4 * kDcMaxN * sizeof(double));
  if (e == hipSuccess) e = lim_sort.ensure((const void*)k_dc_sort, (size_t)4096 * (sizeof(double) + sizeof(int)));
  if (e != hipSuccess) return e;
  DcArgs a{};
  a.n = n;
  a.D = t.D;
  a.E = t.E;
  a.Q = t.Q;
  a.Qs = t.Qs;
  a.U = t.U;
  a.Z = t.Z;
  a.nodes = (const int4*)t.nodes;
  a.ws_i = t.ws_i;
  a.ws_node = t.ws_i + 4 * n;
  a.ws_orig = t.ws_i + 8 * n;
  a.ws_d = t.ws_d;
  a.sQ = t.sQ;
  a.sZ = t.sZ;
  a.s_wsi = t.s_wsi;
  a.s_wsd = t.s_wsd;
  const int nb = t.nb;
  k_dc_init<<<dim3((n + 255) / 256, nb), 256, 0, st>>>(a);
  const int nlev = (int)t.level_start.size() - 1;
  for (int L = 0; L < nlev; ++L) {
    const int first = t.level_start[L], count = t.level_start[L + 1] - first;
    if (count <= 0) continue;
    int mmax = 0;
    for (int q = first; q < first + count; ++q) mmax = std::max(mmax, t.node_sizes[q]);
    a.node0 = first;
    a.count = count;
    const int dnt = std::min(kDefNT, (mmax + 63) / 64 * 64);
    k_dc_deflate<<<dim3(count, nb), dnt, dc_deflate_lds(mmax), st>>>(a);
    k_dc_gather<<<dim3((mmax + 3) / 4, count, nb), 256, (size_t)4 * mmax * sizeof(double), st>>>(a, mmax);
    k_dc_secular<<<dim3((mmax + 3) / 4, count, nb), 256, (size_t)2 * mmax * sizeof(double), st>>>(a);
    k_dc_zhat<<<dim3((mmax + 3) / 4, count, nb), 256, 0, st>>>(a);
    k_dc_vectors<<<dim3((mmax + 3) / 4, count, nb), 256, 0, st>>>(a);
    k_dc_gemm<<<dim3((mmax + 63) / 64, (mmax + 63) / 64, count * nb), 256, 0, st>>>(a);
  }
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  k_dc_sort<<<nb, 1024, (size_t)np2 * (sizeof(double) + sizeof(int)), st>>>(a);
  k_dc_convert<<<dim3((n + 63) / 64, (n + 63) / 64, nb), 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace slrx
