// Mono-exponential fit per pixel (Sec. IV: T2 maps of the reconstructed
// series): least-squares line through y_t = log|rho_t| against the echo times,
// in FP64.  T2 = -1/slope where the slope is negative (+inf otherwise); the
// amplitude is exp(intercept at TE = 0).  One thread per pixel, the frames of a
// pixel read at stride P Q (coalesced across threads).
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace slrx {

constexpr int kFitTMax = 32;  // frames (the echo-time array of FitArgs)

__global__ __launch_bounds__(256) void k_fit_t2(FitArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.npix) return;
  // centred form sum_t (te_t - tbar)(y_t - ybar): a series with equal logs
  // (a pixel without signal) gets a slope of exactly zero
  double y[kFitTMax];
  double sy = 0.0;
#pragma unroll
  for (int t = 0; t < kFitTMax; ++t) {
    y[t] = 0.0;
    if (t < a.T) {
      const float2 v = a.img[(long)t * a.npix + i];
      const double m = sqrt((double)v.x * v.x + (double)v.y * v.y);
      y[t] = log(fmax(m, 1e-30));
      sy += y[t];
    }
  }
  const double ybar = sy / a.T;
  double sty = 0.0;
#pragma unroll
  for (int t = 0; t < kFitTMax; ++t)
    if (t < a.T) sty += (a.te[t] - a.tbar) * (y[t] - ybar);
  const double slope = sty / a.stt;
  a.t2[i] = slope < 0.0 ? -1.0 / slope : INFINITY;
  if (a.amp) a.amp[i] = exp(ybar - slope * a.tbar);
}

hipError_t launch_fit_t2(const FitArgs& a, hipStream_t s) {
  k_fit_t2<<<(unsigned)((a.npix + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace slrx
