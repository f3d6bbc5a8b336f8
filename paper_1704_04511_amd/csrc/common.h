// Shared device/host helpers for libslrx (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#define SLRX_DEV __device__ __forceinline__

// ---------------------------------------------------------------- complex
SLRX_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
SLRX_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
SLRX_DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
SLRX_DEV float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
SLRX_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// a * (i * sign): multiply by +i (sign > 0) or -i (sign < 0)
template <int SIGN> SLRX_DEV float2 cmul_i(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

SLRX_DEV double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
SLRX_DEV double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
SLRX_DEV double2 dcmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
SLRX_DEV double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
SLRX_DEV double2 f2d(float2 a) { return make_double2((double)a.x, (double)a.y); }

// Index of tap pair (m, m'), m <= m', in the row-major upper triangle of an M x M matrix.
__host__ __device__ inline int pair_id(int m, int mp, int M) { return m * M - (m * (m - 1)) / 2 + (mp - m); }

// Deterministic block reduction of one double (fixed tree order).
template <int NT>
SLRX_DEV double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  // wave-level reduction first (64 lanes), fixed shuffle order
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    red[0] = s;
  }
  __syncthreads();
  s = red[0];
  __syncthreads();
  return s;
}

// Sum of n partials in a fixed order, computed redundantly by every block (deterministic).
template <int NT>
SLRX_DEV double reduce_partials(const double* part, int n, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) v += part[i];
  return block_sum<NT>(v, red);
}

// Raises a kernel's dynamic-LDS limit once per device: the first launches on a
// device set it (concurrent first launches may both set it, which is harmless);
// the flag bits are atomic, so host threads can launch concurrently.
struct LdsLimit {
  std::atomic<uint32_t> set_on{0};  // bit d: device d
  hipError_t ensure(const void* kernel, size_t bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint32_t bit = dev >= 0 && dev < 32 ? 1u << dev : 0u;
    if (bit && (set_on.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess && bit) set_on.fetch_or(bit, std::memory_order_release);
    return e;
  }
};
