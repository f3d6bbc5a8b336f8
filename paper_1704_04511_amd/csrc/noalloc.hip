// The normal operator of the least-squares step (Sec. III.A, eq. "eq:grad_ls"),
// A v = S o v + lam F G F^-1 v, for callers that cannot allocate device memory:
// no plan, every device buffer beyond the caller's inputs and outputs lives in
// one file-scope device array (the transposed row-pass volume, the transposed
// penalty masks, the twiddles and the per-block partials of the finishing
// pass).  Same kernels as slrx_step_apply (k_op.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "kernels.h"
#include "plan.h"
#include "../../include/slrx.h"

using namespace slrx;

namespace {

constexpr size_t kDataBytes = (size_t)24 << 20;  // transposed volume + transposed masks
constexpr size_t kTailBytes = (size_t)128 << 10;  // twiddles, partials
constexpr size_t kTwOff = kDataBytes;              // P float2 twiddles, then Q
constexpr size_t kPartOff = kDataBytes + 4096;     // per-block partials of the finishing pass
constexpr size_t kPartBytes = kTailBytes - 4096;
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kDataBytes + kTailBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// e^{-2 pi i t / N} for t < N, rounded to complex64 (the FFT passes' table).
__global__ void k_twiddles(float2* tw, int N) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)N, &s, &c);
  tw[t] = make_float2((float)c, (float)s);
}

// Device address of the scratch array on the current device (looked up once per device).
slrx_status scratch_on_device(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SLRX_EDEVICE, "no HIP device");
  if (dev < 0 || dev >= kMaxDevices) return fail(SLRX_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLRX_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return SLRX_OK;
}

}  // namespace

extern "C" size_t slrx_apply_noalloc_limit(void) { return kDataBytes; }

extern "C" slrx_status slrx_apply_noalloc(const slrx_dims* dims, double lambda, uint32_t flags, const uint8_t* S,
                                          const void* E, const void* v, void* out, void* hip_stream) {
  if (!dims || !S || !E || !v || !out) return fail(SLRX_EINVAL, "NULL argument");
  const slrx_dims& d = *dims;
  if (!fft_len_supported(d.P) || !fft_len_supported(d.Q))
    return fail(SLRX_EINVAL, "unsupported frame size %dx%d (supported: 8,16,32,64,96,128,160,192,256)", d.P, d.Q);
  if (d.T < 1 || d.T > max_frames()) return fail(SLRX_EINVAL, "T=%d out of range [1,%d]", d.T, max_frames());
  if (d.M < 1 || d.M > d.T || d.M > max_taps())
    return fail(SLRX_EINVAL, "M=%d out of range [1,min(T,%d)]", d.M, max_taps());
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(SLRX_EINVAL, "lambda must be finite and >= 0");
  if (flags & ~(uint32_t)SLRX_FLAG_GIRAF) return fail(SLRX_EINVAL, "flags other than SLRX_FLAG_GIRAF");
  const size_t V = (size_t)d.T * d.P * d.Q;
  const int W = d.M * (d.M + 1) / 2;
  const size_t vol_bytes = align256(V * sizeof(float2));
  const size_t mask_bytes = align256((size_t)W * d.P * d.Q * sizeof(float2));
  if (vol_bytes + mask_bytes > kDataBytes)
    return fail(SLRX_EINVAL, "T P Q + W P Q = %zu complex64 values need %zu bytes of scratch; the limit is %zu",
                V + (size_t)W * d.P * d.Q, vol_bytes + mask_bytes, kDataBytes);
  if ((size_t)fin_blocks(d.P, d.T) * sizeof(double) > kPartBytes)
    return fail(SLRX_EINVAL, "too many partial sums for the scratch (P=%d, T=%d)", d.P, d.T);
  unsigned char* base = nullptr;
  const slrx_status st = scratch_on_device(&base);
  if (st != SLRX_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  float2* t = (float2*)base;
  float2* Et = (float2*)(base + vol_bytes);
  float2* twP = (float2*)(base + kTwOff);
  float2* twQ = twP + 256;
  double* part = (double*)(base + kPartOff);
  auto chk = [](hipError_t e) { return e == hipSuccess ? SLRX_OK : fail(SLRX_EDEVICE, "launch failed: %s", hipGetErrorString(e)); };
  k_twiddles<<<1, 256, 0, s>>>(twP, d.P);
  k_twiddles<<<1, 256, 0, s>>>(twQ, d.Q);
  slrx_status r = chk(hipGetLastError());
  if (r != SLRX_OK) return r;
  // masks [W][P][Q] -> transposed planes [W][Q][P]
  r = chk(launch_transpose_planes(W, d.P, d.Q, (const float2*)E, Et, s));
  if (r != SLRX_OK) return r;
  RowArgs ra{};
  ra.P = d.P; ra.Q = d.Q; ra.T = d.T;
  ra.mode = ROW_PLAIN;
  ra.sign = +1;
  ra.src = (const float2*)v;
  ra.dst = t;
  ra.scale = 1.0f;
  ra.tw = twQ;
  r = chk(launch_rows(ra, s));
  if (r != SLRX_OK) return r;
  PenArgs pa{};
  pa.P = d.P; pa.Q = d.Q; pa.T = d.T; pa.M = d.M;
  pa.buf = t;
  pa.Et = Et;
  pa.scale = (float)(lambda / ((double)d.P * d.Q));
  pa.tw = twP;
  pa.circ = (flags & SLRX_FLAG_GIRAF) ? 1 : 0;
  r = chk(launch_pen(pa, s));
  if (r != SLRX_OK) return r;
  FinArgs fa{};
  fa.P = d.P; fa.Q = d.Q; fa.T = d.T;
  fa.init = 0;  // out = A v; block partials of <v, A v> into the scratch, the stop flag untouched
  fa.t = t;
  fa.v = (const float2*)v;
  fa.S = S;
  fa.out = (float2*)out;
  fa.part = part;
  fa.flag = nullptr;
  fa.tw = twQ;
  fa.coil = 0;
  return chk(launch_fin(fa, s));
}
