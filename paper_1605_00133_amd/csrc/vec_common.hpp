// Launchers of the TV-prox, reduction and vector kernels (vec_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace pat {

constexpr int kRedBlocks = 1024;   // partial sums per reduction (FP64 each)

hipError_t launch_pdhg_init(const float* v, float* q, float* qbar, long n, hipStream_t st);
hipError_t launch_pdhg_iter(const float* v, float* q, float* qbar, float* dual, int nx, int ny, int nz, int bc,
                            float sigma, float tau, float theta, float alpha, hipStream_t st);
// kind: 0 sum a^2, 1 sum a*b, 2 sum (a+b)^2; out: one double on the device
hipError_t launch_reduce_vec(const float* a, const float* b, long n, int kind, double* partial, double* out,
                             hipStream_t st);
hipError_t launch_reduce_tv(const float* q, int nx, int ny, int nz, int bc, double* partial, double* out,
                            hipStream_t st);
// maxima: 2 doubles of device scratch; out: MSE numerator (sum of squared differences)
hipError_t launch_psnr(const float* a, const float* b, int nx, int ny, int nz, int x0, int x1, int y0, int y1,
                       int z0, int z1, double* partial, double* maxima, double* out, hipStream_t st);
hipError_t launch_extrapolate(const float* x, const float* xp, float* out, float beta, long n, hipStream_t st);
hipError_t launch_axpy(const float* a, const float* b, float* out, float s, long n, hipStream_t st);
hipError_t launch_scale(const float* a, float* out, float s, long n, hipStream_t st);
// out[i] = a[i] + a[i + stride], i < n
hipError_t launch_sum2(const float* a, long stride, float* out, long n, hipStream_t st);
hipError_t launch_fill(float* out, float v, long n, hipStream_t st);
// dst = src, n16 words of 16 bytes (both 16-byte aligned, no overlap)
hipError_t launch_copy_probe(const void* src, void* dst, long n16, hipStream_t st);
// out[t][i] = w[i] a[t][i], t < nt, i < npix (may be in place)
hipError_t launch_scale_pixels(const float* a, const float* w, float* out, int nt, int npix, hipStream_t st);

}  // namespace pat
