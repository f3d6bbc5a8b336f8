// Householder reduction of the Hermitian Gram matrix to real symmetric
// tridiagonal form, R = Q T Q^H (FP64), first stage of the eigen-decomposition
// in the weight update (Sec. III.B, Algorithm 1 step 1).
//
// Column k needs a global matrix-vector product with the trailing block, so
// every column is one launch (the launch boundary is the grid-wide sync; a
// software barrier between persistent workgroups costs as much or more on this
// part).  A launch for column k:
//   * in every workgroup (redundantly, identical arithmetic): finishes the
//     previous reflector's w = tau p - |tau|^2/2 (p^H v) v from the previous
//     launch's p = A v, corrects row k with the pending rank-2 update
//     A <- A - v w^H - w v^H, and forms reflector k, H = I - tau v v^H with
//     H^H x = (beta, 0, ..)^T, beta real (the elementary reflector convention
//     of LAPACK's zlarfg);
//   * on its rows i > k: applies the pending rank-2 update and accumulates
//     p_i = sum_j A_ij v_j for the next launch.
// The time of a launch is the serial chain of the reflector, not the traffic
// of the trailing block, so the chain is kept short: thread t holds the
// entries j = k + t + 256 u of every vector in registers (the same entries of
// every row it updates), and a launch makes exactly three block reductions
// (p^H v, the norm of the column, the row products), each a fixed DPP tree in
// every wave plus the four wave sums added in order, with the scalars other
// threads need (p_k, v_k, the subdiagonal entry, the rows' own coefficients)
// passed through the same exchange.  Results are bit-reproducible and do not
// depend on how many workgroups run or which rows a workgroup takes.
// The last 96 columns, whose trailing block fits in the registers of one
// workgroup, are reduced in a single launch (k_tri_tail).
// The working matrix Aw is full (both triangles) and row-major; reflectors are
// stored as LAPACK's zhetrd (lower) stores them: v(k+2:n) in column k of the
// column-major matrix Vst below the subdiagonal, tau(k), diagonal D, real
// subdiagonal E.
#include "common.h"
#include "kernels.h"

namespace slrx {

constexpr int kTriNT = 256;
constexpr int kTriRB = 4;      // rows of a workgroup whose elements are loaded at kernel entry
// Rows held in registers at a time for U vector entries per thread: fewer for the
// long columns of Gram matrices above 2048 (their register arrays otherwise need
// about 500 registers per lane, and the U = 12 instance holding four rows gave wrong
// eigenvalues for n > 2560 while U = 9 and 10 were exact).
template <int U> constexpr int tri_rb() { return U > 10 ? 1 : (U > 8 ? 2 : kTriRB); }
constexpr int kTriRMax = 32;   // rows per workgroup at most

SLRX_DEV double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// Trailing-block rows are read and written once per column launch.  STREAM
// marks those accesses nontemporal (the nt cache-policy bit of the load and
// store instructions); the values are the same either way.
typedef double d2v __attribute__((ext_vector_type(2)));
template <bool STREAM> SLRX_DEV double2 row_load(const double2* p) {
  if constexpr (STREAM) {
    const d2v v = __builtin_nontemporal_load((const d2v*)p);
    return make_double2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool STREAM> SLRX_DEV void row_store(double2* p, double2 e) {
  if constexpr (STREAM) {
    const d2v v = {e.x, e.y};
    __builtin_nontemporal_store(v, (d2v*)p);
  } else {
    *p = e;
  }
}
SLRX_DEV double2 dscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Copy of v from the lane selected by a DPP control (rows masked by RM keep 0).
template <int CTRL, int RM>
SLRX_DEV double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed tree (pairs, quads, half rows,
// rows, then rows 0+1 and 2+3 and the two halves); every lane gets the total.
// Call with all 64 lanes active.
SLRX_DEV double wave_total(double v) {
  v += dpp_mov<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_mov<0x140, 0xf>(v);  // row_mirror
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
SLRX_DEV double2 wave_total2(double2 v) { return make_double2(wave_total(v.x), wave_total(v.y)); }
// The four wave sums of an exchange slot, added in wave order.
SLRX_DEV double2 sum4(const double2* s, int stride) {
  double2 r = s[0];
  r = dadd(r, s[stride]);
  r = dadd(r, s[2 * stride]);
  return dadd(r, s[3 * stride]);
}

// One column of the reduction.  U: vector entries per thread (n - k <= 256 U);
// rows: rows of the trailing block per workgroup (blockIdx.x * rows + k + 1 ..);
// STREAM: nontemporal row accesses.
template <int U, bool STREAM>
__global__ __launch_bounds__(kTriNT) void k_tri_col(TriArgs a, int rows) {
  // exchange slots: [wave][item] for the three reductions
  __shared__ double2 xa[4][3];
  __shared__ double2 xb[4][3];
  __shared__ double2 xc[4][kTriRMax];
  __shared__ double2 coef[kTriRMax][2];  // v_{k-1}(i), w_{k-1}(i) of the workgroup's rows
  const int n = a.n, k = a.k;
  const int b = blockIdx.y;  // problem in a batch
  double2* Aw = a.Aw + (size_t)b * a.strideA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool pending = k > 0;
  const double2 zero = make_double2(0.0, 0.0);
  const int row0 = k + 1 + blockIdx.x * rows;
  const int nrow = min(rows, n - row0);  // >= 1 by the grid size

  // 0. every independent load first: row k, v_{k-1}, p_{k-1}, the first rows of the block
  const double2 t = pending ? a.tau[(size_t)b * n + (k - 1)] : zero;
  const double2* rowk = Aw + (size_t)k * n;
  const double2* vprev = a.vbuf[(k + 1) & 1] + (size_t)b * n;  // written by launch k-1
  const double2* pprev = a.pbuf[(k + 1) & 1] + (size_t)b * n;
  double2 rk[U], vp[U], pp[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = k + tid + kTriNT * u;
    rk[u] = vp[u] = pp[u] = zero;
    if (j < n) {
      rk[u] = rowk[j];
      if (pending) {
        vp[u] = vprev[j];
        pp[u] = pprev[j];
      }
    }
  }
  constexpr int RB = tri_rb<U>();
  double2 xr[RB][U];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = k + tid + kTriNT * u;
      xr[r][u] = (r < nrow && j > k && j < n) ? row_load<STREAM>(&Aw[(size_t)(row0 + r) * n + j]) : zero;
    }

  // 1. d = p^H v of the pending reflector; p_{k-1}(k), v_{k-1}(k) ride along
  double2 d = zero;
#pragma unroll
  for (int u = 0; u < U; ++u) d = dadd(d, dcmul(pp[u], vp[u]));
  d = wave_total2(d);
  if (lane == 0) xa[wave][0] = d;
  if (tid == 0) {
    xa[0][1] = pp[0];  // entry j = k
    xa[0][2] = vp[0];
  }
  __syncthreads();
  d = sum4(&xa[0][0], 3);
  const double2 pk = xa[0][1], vk = xa[0][2];

  // 2. w = tau p + c d v, c = -|tau|^2 / 2; column k with the pending update; its norm below k+1
  const double c = -0.5 * (t.x * t.x + t.y * t.y);
  const double2 cd = dscale(d, c);
  const double2 wk = dadd(dmul(t, pk), dmul(cd, vk));
  double2 w[U], col[U];
  double xn = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = k + tid + kTriNT * u;
    w[u] = dadd(dmul(t, pp[u]), dmul(cd, vp[u]));
    double2 x = dconj(rk[u]);  // A(j, k) = conj(A(k, j))
    if (pending) x = dsub(x, dadd(dmul(vp[u], dconj(wk)), dmul(w[u], dconj(vk))));
    col[u] = x;
    if (j >= k + 2 && j < n) xn += x.x * x.x + x.y * x.y;
  }
  xn = wave_total(xn);
  if (lane == 0) xb[wave][0] = make_double2(xn, 0.0);
  if (tid == 1) xb[0][1] = col[0];  // alpha = column entry k + 1
  if (tid == 0) xb[0][2] = col[0];  // diagonal entry k
  // coefficients of the workgroup's rows i: held by the thread with i = k + t + 256 u
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = k + tid + kTriNT * u;
    const int r = j - row0;
    if (r >= 0 && r < nrow) {
      coef[r][0] = vp[u];
      coef[r][1] = w[u];
    }
  }
  __syncthreads();
  const double xn2 = sum4(&xb[0][0], 3).x;
  const double2 alpha = xb[0][1];
  const double dk = xb[0][2].x;

  // 3. reflector k on x = column k rows k+1 .. n-1
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
    const double2 den = make_double2(alpha.x - beta, alpha.y);  // scale = 1 / (alpha - beta)
    const double dd = den.x * den.x + den.y * den.y;
    scale = make_double2(den.x / dd, -den.y / dd);
  }
  double2 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = k + tid + kTriNT * u;
    v[u] = j == k + 1 ? make_double2(1.0, 0.0) : (j >= k + 2 && j < n ? dmul(col[u], scale) : zero);
  }
  if (blockIdx.x == 0) {
    double2* vout = a.vbuf[k & 1] + (size_t)b * n;
    double2* Vst = a.Vst + (size_t)b * a.strideA;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = k + tid + kTriNT * u;
      if (j > k && j < n) {
        vout[j] = v[u];
        Vst[(size_t)k * n + j] = j == k + 1 ? make_double2(beta, 0.0) : v[u];
      }
    }
    if (tid == 0) {
      a.D[(size_t)b * n + k] = dk;
      a.E[(size_t)b * n + k] = beta;
      a.tau[(size_t)b * n + k] = tau;
    }
  }

  // 4. the workgroup's rows: pending update (written back), p_i = sum_j A_ij v_j,
  //    each row's partials summed over the wave at once (nrow is uniform)
  double2* pout = a.pbuf[k & 1] + (size_t)b * n;
  auto row_work = [&](int r, const double2 (&x)[U]) {
    const int i = row0 + r;
    const double2 vi = coef[r][0], wi = coef[r][1];
    double2 acc = zero;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = k + tid + kTriNT * u;
      if (j > k && j < n) {
        double2 e = x[u];
        if (pending) {
          e = dsub(e, dadd(dmul(vi, dconj(w[u])), dmul(wi, dconj(vp[u]))));
          row_store<STREAM>(&Aw[(size_t)i * n + j], e);
        }
        acc = dadd(acc, dmul(e, v[u]));
      }
    }
    acc = wave_total2(acc);
    if (lane == 0) xc[wave][r] = acc;
  };
#pragma unroll
  for (int r = 0; r < RB; ++r)
    if (r < nrow) row_work(r, xr[r]);
  for (int r0 = RB; r0 < nrow; r0 += RB) {  // rows beyond the prefetched ones
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = k + tid + kTriNT * u;
        xr[r][u] = (r0 + r < nrow && j > k && j < n) ? row_load<STREAM>(&Aw[(size_t)(row0 + r0 + r) * n + j])
                                                     : zero;
      }
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r0 + r < nrow) row_work(r0 + r, xr[r]);
  }
  __syncthreads();
  if (tid < nrow) pout[row0 + tid] = sum4(&xc[0][tid], kTriRMax);
}

// The last kTriTail columns in one launch, one workgroup of kTailNT threads per
// problem with the trailing block (rows and columns k0..n-1, at most
// kTriTail x kTriTail) in registers: thread t holds row i = t / 4 at the columns
// j = t % 4 + 4 c, c < kTriTail / 4, zero beyond the block.  First the pending update of reflector
// k0-1 is applied, then each column is reduced as in k_tri_col (same reflector
// convention, same outputs): the wave holding row k forms reflector k from it
// (the block is Hermitian, so column k below the diagonal is the conjugate of
// row k) and publishes v; every row forms its entry of p = A v (four lanes, a
// fixed DPP tree) and p^H v is summed over the waves in order; then the rank-2
// update runs on the registers, written as
//   A - v w^H - w v^H = A - conj(tau) v p^H - (tau p + 2 Re(c d) v) v^H
// for w = tau p + c d v, c = -|tau|^2 / 2, d = p^H v (real for a Hermitian A).
// v and p are zero outside rows k+1.., so the update leaves the finished rows
// and columns unchanged without masks (slots are skipped in chunks of eight,
// whose loads the compiler can then issue together); v and p are
// double-buffered by column parity, which leaves two barriers per column.  The
// outputs stay in LDS until the end (a barrier would otherwise wait for each
// column's global stores).
constexpr int kTriTail = 96;
constexpr int kTailNT = 384;
constexpr int kTailLanes = 4;                   // lanes per row
constexpr int kTailC = kTriTail / kTailLanes;   // columns per thread
constexpr int kTailRowsW = 64 / kTailLanes;     // rows per wave
constexpr int kTailChunk = 8;                   // column slots skipped or processed together
static_assert(kTailLanes == 4, "row sums are quad sums (sum_quad)");
static_assert(kTailNT / kTailLanes == kTriTail, "one row of the block per kTailLanes threads");
static_assert(kTailC % kTailChunk == 0 && kTailNT % 64 == 0, "whole chunks and waves");
// packed reflectors of the block: column kk's entries kk+1..L-1 at voff(kk)
__host__ __device__ inline int tail_voff(int L, int kk) { return kk * (2 * L - kk - 1) / 2; }
inline size_t tail_lds(int L) { return (size_t)tail_voff(L, L - 1) * sizeof(double2); }

// Sum over each aligned quad of lanes (fixed order); every lane of the quad
// gets its total.  Call with all 64 lanes active.
SLRX_DEV double sum_quad(double v) {
  v += dpp_mov<0xB1, 0xf>(v);  // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xf>(v);  // quad_perm [2,3,0,1]
  return v;
}
SLRX_DEV double2 sum_quad2(double2 v) { return make_double2(sum_quad(v.x), sum_quad(v.y)); }
// LDS writes of a wave made visible to its other lanes (a wave executes its LDS
// accesses in order; the fences keep the compiler from moving them across).
SLRX_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
SLRX_DEV double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(kTailNT) void k_tri_tail(TriArgs a, int k0) {
  extern __shared__ double2 vl[];  // reflectors, packed (tail_voff)
  __shared__ double2 vs[2][kTriTail], ps[2][kTriTail];
  __shared__ double2 xrow[kTriTail];  // row k, exchanged within the wave holding it
  __shared__ double2 tl[kTriTail];
  __shared__ double Dl[kTriTail], El[kTriTail];
  __shared__ double2 red[kTailNT / 64];
  __shared__ double2 tau_s[2];
  const int n = a.n, L = n - k0;
  const int b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = tid / kTailLanes, q = tid % kTailLanes;
  const double2* Aw = a.Aw + (size_t)b * a.strideA;
  const double2 zero = make_double2(0.0, 0.0);
  double2 A[kTailC];
#pragma unroll
  for (int c = 0; c < kTailC; ++c) {
    const int j = q + kTailLanes * c;
    A[c] = (i < L && j < L) ? Aw[(size_t)(k0 + i) * n + k0 + j] : zero;
  }
  // the rank-2 update of one reflector from v and p in LDS slot s; columns from slot c0
  auto rank2 = [&](int s, double2 t, double2 d, double2 vi, double2 pi, int c0) __attribute__((always_inline)) {
    const double2 al = dmul(dconj(t), vi);                                    // conj(tau) v_i
    const double2 be = dadd(dmul(t, pi), dscale(vi, -(t.x * t.x + t.y * t.y) * d.x));  // tau p_i + 2 Re(c d) v_i
#pragma unroll
    for (int h = 0; h < kTailC / kTailChunk; ++h) {
      if (kTailChunk * h + kTailChunk - 1 < c0) continue;  // chunks of slots left of the block
#pragma unroll
      for (int u = 0; u < kTailChunk; ++u) {
        const int c = kTailChunk * h + u, j = q + kTailLanes * c;
        const double2 pj = ps[s][j], vj = vs[s][j];
        A[c] = dsub(A[c], dadd(dmul(al, dconj(pj)), dmul(be, dconj(vj))));
      }
    }
  };
  // p^H v from the rows' terms: per wave in a fixed tree, then the waves in order
  auto wave_sums = [&](double2 part) __attribute__((always_inline)) {
    part = wave_total2(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double2 d = red[0];
#pragma unroll
    for (int w = 1; w < kTailNT / 64; ++w) d = dadd(d, red[w]);
    return d;
  };
  if (k0 > 0) {  // pending update of reflector k0-1 (v, p from the last column launch)
    const double2* vprev = a.vbuf[(k0 + 1) & 1] + (size_t)b * n + k0;
    const double2* pprev = a.pbuf[(k0 + 1) & 1] + (size_t)b * n + k0;
    if (tid < kTriTail) {
      vs[1][tid] = tid < L ? vprev[tid] : zero;
      ps[1][tid] = tid < L ? pprev[tid] : zero;
    }
    const double2 vi = i < L ? vprev[i] : zero, pi = i < L ? pprev[i] : zero;
    const double2 d = wave_sums(q == 0 ? dcmul(pi, vi) : zero);  // its barrier also publishes vs, ps
    rank2(1, a.tau[(size_t)b * n + k0 - 1], d, vi, pi, 0);
    __syncthreads();
  }
  for (int kk = 0; kk < L - 1; ++kk) {
    const int s = kk & 1;
    const int c1 = (kk + 1) / kTailLanes;  // first column slot that can be in the trailing block
    // 1. reflector kk from row kk (x_j = conj A(kk, j), j >= kk + 2; alpha = conj A(kk, kk + 1))
    if (wave == kk / kTailRowsW) {
      const bool mine = i == kk;
      double xn = 0.0;
      if (mine) {
#pragma unroll
        for (int c = 0; c < kTailC; ++c) {
          const int j = q + kTailLanes * c;
          if (j >= kk + 2) xn += A[c].x * A[c].x + A[c].y * A[c].y;
          xrow[j] = A[c];
        }
      }
      xn = sum_quad(xn);
      wave_sync();  // row kk in xrow for the whole wave
      const double xn2 = readlane_d(xn, (kk % kTailRowsW) * kTailLanes);
      const double2 alpha = dconj(xrow[kk + 1]);
      const double dk = xrow[kk].x;
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
        const double2 den = make_double2(alpha.x - beta, alpha.y);  // scale = 1 / (alpha - beta)
        const double dd = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dd, -den.y / dd);
      }
      // v from the row in xrow: lane l writes entries l, l + 64, .. (every slot)
      const int vo = tail_voff(L, kk) - kk - 1;
#pragma unroll
      for (int h = 0; h < (kTriTail + 63) / 64; ++h) {
        const int j = lane + 64 * h;
        if (j >= kTriTail) continue;
        const double2 v = j == kk + 1 ? make_double2(1.0, 0.0)
                                      : (j >= kk + 2 && j < L ? dmul(dconj(xrow[j]), scale) : zero);
        vs[s][j] = v;
        if (j > kk && j < L) vl[vo + j] = j == kk + 1 ? make_double2(beta, 0.0) : v;
      }
      if (lane == 0) {
        tau_s[s] = tau;
        Dl[kk] = dk;
        El[kk] = beta;
        tl[kk] = tau;
      }
    }
    __syncthreads();
    // 2. p_i = sum_j A_ij v_j for the rows of the trailing block, p^H v
    const double2 vi = vs[s][i];
    double2 pi = zero;
    const bool live = wave * kTailRowsW + kTailRowsW - 1 >= kk + 1;  // the wave holds trailing rows
    if (live) {
      double2 acc[4] = {zero, zero, zero, zero};  // four chains, added in order
#pragma unroll
      for (int h = 0; h < kTailC / kTailChunk; ++h) {
        if (kTailChunk * h + kTailChunk - 1 < c1) continue;
#pragma unroll
        for (int u = 0; u < kTailChunk; ++u) {
          const int c = kTailChunk * h + u;
          acc[u & 3] = dadd(acc[u & 3], dmul(A[c], vs[s][q + kTailLanes * c]));
        }
      }
      pi = sum_quad2(dadd(dadd(acc[0], acc[1]), dadd(acc[2], acc[3])));
      if (i <= kk || i >= L) pi = zero;
    }
    if (q == 0) ps[s][i] = pi;
    const double2 d = wave_sums(q == 0 ? dcmul(pi, vi) : zero);
    // 3. the rank-2 update of the trailing block
    if (live) rank2(s, tau_s[s], d, vi, pi, c1);
  }
  if (wave == (L - 1) / kTailRowsW) {  // the last diagonal entry
    if (i == L - 1) {
#pragma unroll
      for (int c = 0; c < kTailC; ++c) xrow[q + kTailLanes * c] = A[c];
    }
    wave_sync();
    if (lane == 0) Dl[L - 1] = xrow[L - 1].x;
  }
  __syncthreads();
  double2* Vst = a.Vst + (size_t)b * a.strideA;
  for (int kk = 0; kk < L - 1; ++kk) {
    const int vo = tail_voff(L, kk) - kk - 1;
    for (int j = kk + 1 + tid; j < L; j += kTailNT) Vst[(size_t)(k0 + kk) * n + k0 + j] = vl[vo + j];
  }
  for (int kk = tid; kk < L; kk += kTailNT) {
    a.D[(size_t)b * n + k0 + kk] = Dl[kk];
    if (kk < L - 1) {
      a.E[(size_t)b * n + k0 + kk] = El[kk];
      a.tau[(size_t)b * n + k0 + kk] = tl[kk];
    }
  }
}

int tri_max_n() { return 3000; }

template <int U>
static void launch_col(const TriArgs& a, int nbatch, int rows, bool stream, hipStream_t s) {
  const int nr = a.n - a.k - 1;
  const dim3 grid((nr + rows - 1) / rows, nbatch);
  if (stream) k_tri_col<U, true><<<grid, kTriNT, 0, s>>>(a, rows);
  else k_tri_col<U, false><<<grid, kTriNT, 0, s>>>(a, rows);
}

// Workgroup budgets per column launch (all problems of a batch together) the
// tuner chooses from: each workgroup recomputes the reflector, so many small
// problems want more rows per workgroup than one large one.
// One problem also tries 256 with long columns split so that every row of a
// workgroup is loaded at kernel entry (kTriRB rows each, up to 320 workgroups):
// 8.03 against 8.13 ms per 1125 x 1125 decomposition when measured.  The row
// access policy is tuned afterwards for the chosen budget: nontemporal rows took
// 7.15 against 8.04 ms for one 1125 x 1125 problem, but made a batch of 32
// problems of 405 about 6% slower.
static const int kTriBudget1[] = {128, 256, 256};
static const int kTriBudgetN[] = {256, 512, 1024, 2048, 4096};
int tri_budget_candidates(int nbatch) { return nbatch > 1 ? 5 : 3; }
int tri_budget(int nbatch, int cand) { return nbatch > 1 ? kTriBudgetN[cand] : kTriBudget1[cand]; }

hipError_t launch_tridiag(const TriArgs& base, int nbatch, hipStream_t s, int cand, bool stream) {
  const int budget = tri_budget(nbatch, cand);
  const bool fit = nbatch == 1 && cand == 2;
  const int n = base.n;
  if (n > tri_max_n()) return hipErrorInvalidValue;
  const int k0 = n > kTriTail ? n - kTriTail : 0;  // columns k0.. in one launch
  TriArgs a = base;
  for (int k = 0; k < k0; ++k) {
    a.k = k;
    const int nr = n - k - 1;                        // trailing rows
    // rows per workgroup: at most 256 workgroups per problem and about `budget` in all
    int rows = (nr + kTriNT - 1) / kTriNT;
    const int rb = (int)(((long)nr * nbatch + budget - 1) / budget);
    if (rb > rows) rows = rb < kTriRMax ? rb : kTriRMax;
    const int u = (n - k + kTriNT - 1) / kTriNT;      // vector entries per thread
    const int rbu = u > 10 ? 1 : (u > 8 ? 2 : kTriRB); // rows loaded at entry (tri_rb<U>)
    if (fit && rows > rbu && (nr + rbu - 1) / rbu <= 320) rows = rbu;
    if (u <= 1) launch_col<1>(a, nbatch, rows, stream, s);
    else if (u <= 2) launch_col<2>(a, nbatch, rows, stream, s);
    else if (u <= 3) launch_col<3>(a, nbatch, rows, stream, s);
    else if (u <= 4) launch_col<4>(a, nbatch, rows, stream, s);
    else if (u <= 5) launch_col<5>(a, nbatch, rows, stream, s);
    else if (u <= 6) launch_col<6>(a, nbatch, rows, stream, s);
    else if (u <= 8) launch_col<8>(a, nbatch, rows, stream, s);
    else if (u <= 9) launch_col<9>(a, nbatch, rows, stream, s);
    else if (u <= 10) launch_col<10>(a, nbatch, rows, stream, s);
    else launch_col<12>(a, nbatch, rows, stream, s);
  }
  static LdsLimit lim;
  const hipError_t e = lim.ensure((const void*)k_tri_tail, tail_lds(kTriTail));
  if (e != hipSuccess) return e;
  const int L = n - k0;
  k_tri_tail<<<dim3(1, nbatch), kTailNT, tail_lds(L), s>>>(a, k0);
  return hipGetLastError();
}

}  // namespace slrx
