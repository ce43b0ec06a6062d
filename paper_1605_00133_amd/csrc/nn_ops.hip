// Resampling and elementwise layers of the learned update network (outside the
// paper's method): 2x2x2 average pooling and nearest-neighbour x2 upsampling
// with their backward passes, add (+ ReLU), axpby with an optional clamp at
// zero, and the squared-error loss with its gradient. All are streaming
// kernels bound by HBM bandwidth: each reads and writes every element once,
// with consecutive threads on consecutive x.
//
// Layout: [channels][nz][ny][nx], x fastest, where "channels" is the product
// of batch and channel counts. Fine grid (nz, ny, nx) even; the coarse voxel
// (z, y, x) covers fine voxels (2z + a, 2y + b, 2x + c), a, b, c in {0, 1}.
// The eight children are summed in a fixed order, and the loss is an FP64 sum
// over a fixed grid of block partials: results do not depend on scheduling.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pat_nn.h"
#include "pat_internal.hpp"

namespace {

constexpr int kT = 256;
constexpr int kLossBlocks = 1024;

// coarse[c][z][y][x] = scale * sum of the eight fine children
__global__ __launch_bounds__(kT) void k_sum8(const float* __restrict__ fine, float* __restrict__ coarse, long ncoarse,
                                             int nz2, int ny2, int nx2, float scale) {
  const long i = (long)blockIdx.x * kT + threadIdx.x;
  if (i >= ncoarse) return;
  const int x = (int)(i % nx2);
  long t = i / nx2;
  const int y = (int)(t % ny2);
  t /= ny2;
  const int z = (int)(t % nz2);
  const long c = t / nz2;
  const long nx = 2L * nx2, ny = 2L * ny2;
  const float* b = fine + ((c * 2 * nz2 + 2 * z) * ny + 2 * y) * nx + 2 * x;
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const float2 v = *reinterpret_cast<const float2*>(b + (a * ny + r) * nx);
      s += v.x + v.y;
    }
  coarse[i] = s * scale;
}

// fine[c][z][y][x] = scale * coarse[c][z/2][y/2][x/2]
__global__ __launch_bounds__(kT) void k_spread8(const float* __restrict__ coarse, float* __restrict__ fine, long nfine,
                                                int nz2, int ny2, int nx2, float scale) {
  const long i = (long)blockIdx.x * kT + threadIdx.x;
  if (i >= nfine) return;
  const long nx = 2L * nx2, ny = 2L * ny2, nz = 2L * nz2;
  const int x = (int)(i % nx);
  long t = i / nx;
  const int y = (int)(t % ny);
  t /= ny;
  const int z = (int)(t % nz);
  const long c = t / nz;
  fine[i] = scale * coarse[((c * nz2 + z / 2) * ny2 + y / 2) * nx2 + x / 2];
}

// y may alias a or b (one element per thread, read before written): no __restrict__
__global__ __launch_bounds__(kT) void k_add_act(const float* a, const float* b, float* y, long n, int relu) {
  const long i = (long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  float v = a[i];
  if (b) v += b[i];
  y[i] = relu ? fmaxf(v, 0.f) : v;
}

// out may alias x or yv, as above
__global__ __launch_bounds__(kT) void k_axpby(const float* x, const float* yv, float* out, long n, float alpha,
                                              float beta, int clamp0) {
  const long i = (long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  float v = alpha * x[i];
  if (yv) v += beta * yv[i];
  out[i] = clamp0 ? fmaxf(v, 0.f) : v;
}

// grad = 2 (a - t) / n (0 where a <= 0 if mask0), partial[block] = sum of (a - t)^2 in FP64
__global__ __launch_bounds__(kT) void k_mse(const float* __restrict__ a, const float* __restrict__ t,
                                            float* __restrict__ grad, long n, int mask0, double* __restrict__ partial) {
  __shared__ double red[kT];
  double s = 0.0;
  const float g = (float)(2.0 / (double)n);
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < n; i += (long)gridDim.x * kT) {
    const float ai = a[i];
    const float d = ai - t[i];
    s += (double)d * (double)d;
    if (grad) grad[i] = (mask0 && !(ai > 0.f)) ? 0.f : g * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kT) void k_mse_final(const double* __restrict__ partial, int nb, long n,
                                                  double* __restrict__ loss) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)n;
}

unsigned nblocks(long n) { return (unsigned)((n + kT - 1) / kT); }

pat_status launched(const char* who) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PAT_OK : pat::set_error(PAT_ERR_HIP, "%s: %s", who, hipGetErrorString(e));
}

// fine_sizes: (nz, ny, nx) is the fine grid; pairs_in: `in` is the fine tensor, read in pairs along x
pat_status resample_args(const char* who, const void* in, const void* out, int64_t channels, int32_t nz, int32_t ny,
                         int32_t nx, bool fine_sizes, bool pairs_in) {
  if (channels < 0 || nz < 1 || ny < 1 || nx < 1)
    return pat::set_error(PAT_ERR_INVALID, "%s: sizes must be positive (channels >= 0)", who);
  if (fine_sizes && ((nz | ny | nx) & 1))
    return pat::set_error(PAT_ERR_INVALID, "%s: the fine grid must have even sizes", who);
  const long nfine = (long)channels * nz * ny * nx * (fine_sizes ? 1 : 8);
  if (nfine > (1L << 36) || nfine / kT > 0x7fffffffL) return pat::set_error(PAT_ERR_INVALID, "%s: tensor too large", who);
  if (channels > 0 && (!in || !out)) return pat::set_error(PAT_ERR_INVALID, "%s: null pointer", who);
  if (pairs_in && channels > 0 && (reinterpret_cast<uintptr_t>(in) & 7u))
    return pat::set_error(PAT_ERR_INVALID, "%s: the fine tensor must be 8-byte aligned", who);
  return PAT_OK;
}

}  // namespace

extern "C" {

pat_status pat_pool2_forward(const float* x, float* y, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                             void* stream) {
  const pat_status st = resample_args("pat_pool2_forward", x, y, channels, nz, ny, nx, true, true);
  if (st != PAT_OK || channels == 0) return st;
  const long nc = (long)channels * (nz / 2) * (ny / 2) * (nx / 2);
  hipLaunchKernelGGL(k_sum8, dim3(nblocks(nc)), dim3(kT), 0, (hipStream_t)stream, x, y, nc, nz / 2, ny / 2, nx / 2,
                     0.125f);
  return launched("pat_pool2_forward");
}

pat_status pat_pool2_backward(const float* dy, float* dx, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                              void* stream) {
  const pat_status st = resample_args("pat_pool2_backward", dy, dx, channels, nz, ny, nx, true, false);
  if (st != PAT_OK || channels == 0) return st;
  const long nf = (long)channels * nz * ny * nx;
  hipLaunchKernelGGL(k_spread8, dim3(nblocks(nf)), dim3(kT), 0, (hipStream_t)stream, dy, dx, nf, nz / 2, ny / 2,
                     nx / 2, 0.125f);
  return launched("pat_pool2_backward");
}

pat_status pat_upsample2_forward(const float* x, float* y, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                                 void* stream) {
  const pat_status st = resample_args("pat_upsample2_forward", x, y, channels, nz, ny, nx, false, false);
  if (st != PAT_OK || channels == 0) return st;
  const long nf = (long)channels * 8 * nz * ny * nx;
  hipLaunchKernelGGL(k_spread8, dim3(nblocks(nf)), dim3(kT), 0, (hipStream_t)stream, x, y, nf, nz, ny, nx, 1.0f);
  return launched("pat_upsample2_forward");
}

pat_status pat_upsample2_backward(const float* dy, float* dx, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                                  void* stream) {
  const pat_status st = resample_args("pat_upsample2_backward", dy, dx, channels, nz, ny, nx, false, true);
  if (st != PAT_OK || channels == 0) return st;
  const long nc = (long)channels * nz * ny * nx;
  hipLaunchKernelGGL(k_sum8, dim3(nblocks(nc)), dim3(kT), 0, (hipStream_t)stream, dy, dx, nc, nz, ny, nx, 1.0f);
  return launched("pat_upsample2_backward");
}

pat_status pat_add_act(const float* a, const float* b, float* y, int64_t n, int32_t relu, void* stream) {
  if (n < 0) return pat::set_error(PAT_ERR_INVALID, "pat_add_act: n must be >= 0");
  if (n == 0) return PAT_OK;
  if (!a || !y) return pat::set_error(PAT_ERR_INVALID, "pat_add_act: null pointer");
  if (n / kT > 0x7fffffffL) return pat::set_error(PAT_ERR_INVALID, "pat_add_act: tensor too large");
  hipLaunchKernelGGL(k_add_act, dim3(nblocks(n)), dim3(kT), 0, (hipStream_t)stream, a, b, y, (long)n, relu ? 1 : 0);
  return launched("pat_add_act");
}

pat_status pat_axpby(const float* x, const float* y, float* out, int64_t n, float alpha, float beta, int32_t clamp0,
                     void* stream) {
  if (n < 0) return pat::set_error(PAT_ERR_INVALID, "pat_axpby: n must be >= 0");
  if (n == 0) return PAT_OK;
  if (!x || !out) return pat::set_error(PAT_ERR_INVALID, "pat_axpby: null pointer");
  if (n / kT > 0x7fffffffL) return pat::set_error(PAT_ERR_INVALID, "pat_axpby: tensor too large");
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, (hipStream_t)stream, x, y, out, (long)n, alpha, beta,
                     clamp0 ? 1 : 0);
  return launched("pat_axpby");
}

size_t pat_mse_workspace_bytes(void) { return kLossBlocks * sizeof(double); }

pat_status pat_mse(const float* a, const float* t, float* grad, int64_t n, int32_t mask0, double* loss,
                   void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1 || n > (1L << 40)) return pat::set_error(PAT_ERR_INVALID, "pat_mse: n must be in [1, 2^40]");
  if (!a || !t || !loss) return pat::set_error(PAT_ERR_INVALID, "pat_mse: null pointer");
  if (!workspace || workspace_bytes < pat_mse_workspace_bytes())
    return pat::set_error(PAT_ERR_NOMEM, "pat_mse: workspace of %zu bytes needed", pat_mse_workspace_bytes());
  if ((reinterpret_cast<uintptr_t>(workspace) | reinterpret_cast<uintptr_t>(loss)) & 7u)
    return pat::set_error(PAT_ERR_INVALID, "pat_mse: workspace and loss must be 8-byte aligned");
  const long nb0 = (n + kT - 1) / kT;
  const int nb = (int)(nb0 < kLossBlocks ? nb0 : kLossBlocks);
  double* part = static_cast<double*>(workspace);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kT), 0, (hipStream_t)stream, a, t, grad, (long)n, mask0 ? 1 : 0, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(kT), 0, (hipStream_t)stream, part, nb, (long)n, loss);
  return launched("pat_mse");
}

}  // extern "C"
