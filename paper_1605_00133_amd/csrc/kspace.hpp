// Small shared helpers of the propagator kernels: ceiling division and the
// k-space correction sinc(c0 dt |k| / 2), evaluated from its squared argument.
#pragma once

#include <hip/hip_runtime.h>

namespace pat {

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// sinc(sqrt(s)) = sin(h)/h at h^2 = s
__device__ __forceinline__ float sinc_of_sq(float s) {
  const float h = sqrtf(s);
  return h > 0.f ? sinf(h) / h : 1.f;
}
// sin(h)/h for s = h^2 >= 2.5 (outside the stable range of the scheme's
// time steps): kept out of line so that callers do not carry the inlined sine.
__device__ __noinline__ double sinc_of_sq_large(double s) {
  const double h = sqrt(s);
  return sin(h) / h;
}
__device__ __forceinline__ double sinc_of_sq(double s) {
  if (s < 2.5) {
    // Taylor series sum_k (-s)^k / (2k+1)!, truncated after k = 12 (< 4e-21 at s = 2.5)
    double r = 1.0 / 15511210043330985984000000.0;
    r = r * -s + 1.0 / 25852016738884976640000.0;
    r = r * -s + 1.0 / 51090942171709440000.0;
    r = r * -s + 1.0 / 121645100408832000.0;
    r = r * -s + 1.0 / 355687428096000.0;
    r = r * -s + 1.0 / 1307674368000.0;
    r = r * -s + 1.0 / 6227020800.0;
    r = r * -s + 1.0 / 39916800.0;
    r = r * -s + 1.0 / 362880.0;
    r = r * -s + 1.0 / 5040.0;
    r = r * -s + 1.0 / 120.0;
    r = r * -s + 1.0 / 6.0;
    return r * -s + 1.0;
  }
  return sinc_of_sq_large(s);
}

}  // namespace pat
