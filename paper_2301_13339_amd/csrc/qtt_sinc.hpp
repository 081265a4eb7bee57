// Samples of the sinc kernel (3.1) with bandwidth B = 1/Delta_x, sinc(t) =
// sin(pi t)/(pi t), on the kernel grid of the signal: for 2^nk samples,
// x_m = -1/2 + m/2^nk.  The Toeplitz generator of the discrete convolution
// (2.2) has 2^(nk+1) entries: s_u = sinc(B x_{u - 2^(nk-1)}) for
// 2^(nk-1) <= u < 3*2^(nk-1) and 0 elsewhere (before normalisation (7.2)
// by the discrete sum).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace qtt {

__device__ __forceinline__ double sinc_gen(long long u, double B, int nk) {
  const long long nn = 1LL << nk;
  const long long m = u - (nn >> 1);
  if (m < 0 || m >= nn) return 0.0;
  const double x = -0.5 + (double)m / (double)nn;
  const double t = B * x;
  if (t == 0.0) return 1.0;
  return sinpi(t) / (M_PI * t);
}

// s_u and its bandwidth derivative ds_u/dB = (cos(pi B x) - sinc(B x)) / B
// (0 at x = 0), both 0 outside the kernel window.
__device__ __forceinline__ void sinc_gen_pair(long long u, double B, int nk, double* s,
                                              double* ds) {
  const long long nn = 1LL << nk;
  const long long m = u - (nn >> 1);
  if (m < 0 || m >= nn) {
    *s = 0.0;
    *ds = 0.0;
    return;
  }
  const double x = -0.5 + (double)m / (double)nn;
  const double t = B * x;
  if (t == 0.0) {
    *s = 1.0;
    *ds = 0.0;
    return;
  }
  const double sv = sinpi(t) / (M_PI * t);
  *s = sv;
  *ds = (cospi(t) - sv) / B;
}

}  // namespace qtt
