// Sub-sampling operator C and its transpose on the detection-plane time series
// (eq. GenScan; Sec. 3.1 and 4.3), gfx950.
//
//  rSP (random single points): f[n][j] = s[n][idx[j]]; transpose writes
//    s[n][p] = f[n][inv[p]] or 0 through the inverse index map, so every
//    output element is written exactly once with coalesced stores.
//  sHd (scrambled Hadamard patterns): per time row, permute the plane by the
//    column scramble, apply the Sylvester-Walsh-Hadamard transform in LDS, keep
//    the selected rows and scale by 1/sqrt(n_pix) so that C C^T = I. The
//    transpose scatters the rows, transforms (W is symmetric) and un-permutes.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sample_common.hpp"

namespace pat {

constexpr int kThreadsShd = 1024;
constexpr int kMaxPixShd = 16384;                       // 64 KB of floats in LDS
constexpr int kPermPerThread = kMaxPixShd / kThreadsShd;

__global__ __launch_bounds__(256) void k_rsp_gather(const float* __restrict__ s, const int* __restrict__ idx,
                                                    float* __restrict__ f, int npix, int mc, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i / mc;
  const int j = (int)(i - n * mc);
  f[i] = s[n * npix + idx[j]];
}

__global__ __launch_bounds__(256) void k_rsp_scatter(const float* __restrict__ f, const int* __restrict__ inv,
                                                     float* __restrict__ s, int npix, int mc, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i / npix;
  const int p = (int)(i - n * npix);
  const int j = inv[p];
  s[i] = j >= 0 ? f[n * mc + j] : 0.f;
}

// In-place unnormalised Walsh-Hadamard transform of A[0..n) in LDS, Sylvester
// order, in groups of up to 16 elements per thread (log2 n / 4 LDS passes).
__device__ __forceinline__ void fwht_lds(float* A, int n, int tid) {
  for (int h = 1; h < n; ) {
    const int r = (n / h) < 16 ? (n / h) : 16;
    const int groups = n / r;
    for (int g = tid; g < groups; g += kThreadsShd) {
      const int lo = g % h, hi = g / h;
      const int base = hi * h * r + lo;
      float a[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) a[m] = m < r ? A[base + m * h] : 0.f;
#pragma unroll
      for (int len = 1; len < 16; len *= 2) {
        if (len < r) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (!(i & len) && (i + len) < 16) {
              const float x = a[i], y = a[i + len];
              a[i] = x + y;
              a[i + len] = x - y;
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 16; ++m)
        if (m < r) A[base + m * h] = a[m];
    }
    __syncthreads();
    h *= r;
  }
}

__global__ __launch_bounds__(kThreadsShd) void k_shd_forward(const float* __restrict__ s, const int* __restrict__ perm,
                                                             const int* __restrict__ rows, float* __restrict__ f,
                                                             int npix, int mc, float scale) {
  extern __shared__ float A[];
  const int tid = threadIdx.x;
  const long n = blockIdx.x;
  const float* src = s + n * npix;
  for (int i = tid; i < npix; i += kThreadsShd) A[i] = src[i];
  __syncthreads();
  float t[kPermPerThread];
#pragma unroll
  for (int k = 0; k < kPermPerThread; ++k) {
    const int q = tid + k * kThreadsShd;
    if (q < npix) t[k] = A[perm[q]];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPermPerThread; ++k) {
    const int q = tid + k * kThreadsShd;
    if (q < npix) A[q] = t[k];
  }
  __syncthreads();
  fwht_lds(A, npix, tid);
  float* dst = f + n * mc;
  for (int j = tid; j < mc; j += kThreadsShd) dst[j] = A[rows[j]] * scale;
}

__global__ __launch_bounds__(kThreadsShd) void k_shd_adjoint(const float* __restrict__ f, const int* __restrict__ invperm,
                                                             const int* __restrict__ rows, float* __restrict__ s,
                                                             int npix, int mc, float scale) {
  extern __shared__ float A[];
  const int tid = threadIdx.x;
  const long n = blockIdx.x;
  for (int i = tid; i < npix; i += kThreadsShd) A[i] = 0.f;
  __syncthreads();
  const float* src = f + n * mc;
  for (int j = tid; j < mc; j += kThreadsShd) A[rows[j]] = src[j];
  __syncthreads();
  fwht_lds(A, npix, tid);
  float* dst = s + n * npix;
  for (int i = tid; i < npix; i += kThreadsShd) dst[i] = A[invperm[i]] * scale;
}

hipError_t launch_rsp_gather(const float* s, const int* idx, float* f, int npix, int mc, int nt, hipStream_t st) {
  const long total = (long)nt * mc;
  if (total == 0) return hipSuccess;
  k_rsp_gather<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(s, idx, f, npix, mc, total);
  return hipGetLastError();
}

hipError_t launch_rsp_scatter(const float* f, const int* inv, float* s, int npix, int mc, int nt, hipStream_t st) {
  const long total = (long)nt * npix;
  if (total == 0) return hipSuccess;
  k_rsp_scatter<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(f, inv, s, npix, mc, total);
  return hipGetLastError();
}

hipError_t launch_shd_forward(const float* s, const int* perm, const int* rows, float* f, int npix, int mc, int nt,
                              hipStream_t st) {
  if (npix > kMaxPixShd) return hipErrorInvalidValue;
  const float scale = (float)(1.0 / std::sqrt((double)npix));
  k_shd_forward<<<nt, kThreadsShd, npix * sizeof(float), st>>>(s, perm, rows, f, npix, mc, scale);
  return hipGetLastError();
}

hipError_t launch_shd_adjoint(const float* f, const int* invperm, const int* rows, float* s, int npix, int mc, int nt,
                              hipStream_t st) {
  if (npix > kMaxPixShd) return hipErrorInvalidValue;
  const float scale = (float)(1.0 / std::sqrt((double)npix));
  k_shd_adjoint<<<nt, kThreadsShd, npix * sizeof(float), st>>>(f, invperm, rows, s, npix, mc, scale);
  return hipGetLastError();
}

int shd_max_pixels() { return kMaxPixShd; }

}  // namespace pat
