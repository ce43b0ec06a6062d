// Positivity-constrained TV prox (PDHG), deterministic FP64 reductions, PSNR
// and the FISTA/Bregman vector updates, gfx950.
//
// TV (App. A): isotropic forward differences. Neumann: the difference past the
// last voxel of a line is zero. Dirichlet: the volume is viewed as zero-padded
// by one voxel on every face; the dual then lives on the padded points
// 0..n of each axis (points at n+1 only ever see zero differences).
//
// PDHG (App. B, accelerated primal-dual method for the 1-strongly convex data
// term): per iteration one dual kernel (ascent on grad qbar, projection onto
// the ball of radius alpha) and one primal kernel (descent on -div y, clamp at
// zero, over-relaxation). Step sizes are computed on the host in FP64.
//
// Reductions: each block accumulates a fixed strided subset in FP64 and reduces
// it with a fixed tree in LDS; a single block then sums the partials in a fixed
// order. Results are bit-identical run to run.
#include <hip/hip_runtime.h>

#include "vec_common.hpp"

namespace pat {

constexpr int kThreadsVec = 256;

// ---------------------------------------------------------------- TV geometry
struct TvGeom {
  int nx, ny, nz;      // primal volume
  int dx, dy, dz;      // dual grid extents (n or n+1)
  int dirichlet;
  long ndual;          // dx*dy*dz
};

// value of the (possibly zero-padded) primal at dual-grid point (x, y, z)
__device__ __forceinline__ float tv_val(const float* __restrict__ q, const TvGeom& g, int x, int y, int z) {
  if (g.dirichlet) {
    if (x < 1 || y < 1 || z < 1 || x > g.nx || y > g.ny || z > g.nz) return 0.f;
    return q[((long)(z - 1) * g.ny + (y - 1)) * g.nx + (x - 1)];
  }
  return q[((long)z * g.ny + y) * g.nx + x];
}

// forward differences at dual point (x, y, z)
__device__ __forceinline__ float3 tv_grad(const float* __restrict__ q, const TvGeom& g, int x, int y, int z) {
  const float c = tv_val(q, g, x, y, z);
  float3 d;
  if (g.dirichlet) {
    d.x = tv_val(q, g, x + 1, y, z) - c;
    d.y = tv_val(q, g, x, y + 1, z) - c;
    d.z = tv_val(q, g, x, y, z + 1) - c;
  } else {
    d.x = x < g.nx - 1 ? tv_val(q, g, x + 1, y, z) - c : 0.f;
    d.y = y < g.ny - 1 ? tv_val(q, g, x, y + 1, z) - c : 0.f;
    d.z = z < g.nz - 1 ? tv_val(q, g, x, y, z + 1) - c : 0.f;
  }
  return d;
}

__global__ __launch_bounds__(kThreadsVec) void k_pdhg_dual(const float* __restrict__ qbar, float* __restrict__ ydual,
                                                           TvGeom g, float sigma, float alpha) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.ndual) return;
  const int x = (int)(i % g.dx);
  const int y = (int)((i / g.dx) % g.dy);
  const int z = (int)(i / ((long)g.dx * g.dy));
  const float3 d = tv_grad(qbar, g, x, y, z);
  float* yx = ydual;
  float* yy = ydual + g.ndual;
  float* yz = ydual + 2 * g.ndual;
  float vx = yx[i] + sigma * d.x;
  float vy = yy[i] + sigma * d.y;
  float vz = yz[i] + sigma * d.z;
  if (alpha > 0.f) {
    const float nrm = sqrtf(vx * vx + vy * vy + vz * vz);
    const float s = fmaxf(1.f, nrm / alpha);
    vx /= s; vy /= s; vz /= s;
  } else {
    vx = vy = vz = 0.f;
  }
  yx[i] = vx;
  yy[i] = vy;
  yz[i] = vz;
}

// divergence (negative adjoint of the forward difference) at primal voxel (x, y, z)
__device__ __forceinline__ float tv_div(const float* __restrict__ ydual, const TvGeom& g, int x, int y, int z) {
  const float* yx = ydual;
  const float* yy = ydual + g.ndual;
  const float* yz = ydual + 2 * g.ndual;
  if (g.dirichlet) {
    const int px = x + 1, py = y + 1, pz = z + 1;
    const long c = ((long)pz * g.dy + py) * g.dx + px;
    return (yx[c] - yx[c - 1]) + (yy[c] - yy[c - g.dx]) + (yz[c] - yz[c - (long)g.dx * g.dy]);
  }
  const long c = ((long)z * g.dy + y) * g.dx + x;
  float d = 0.f;
  if (x < g.nx - 1) d += yx[c];
  if (x >= 1) d -= yx[c - 1];
  if (y < g.ny - 1) d += yy[c];
  if (y >= 1) d -= yy[c - g.dx];
  if (z < g.nz - 1) d += yz[c];
  if (z >= 1) d -= yz[c - (long)g.dx * g.dy];
  return d;
}

__global__ __launch_bounds__(kThreadsVec) void k_pdhg_primal(const float* __restrict__ v, float* __restrict__ q,
                                                             float* __restrict__ qbar, const float* __restrict__ ydual,
                                                             TvGeom g, float tau, float theta) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % g.nx);
  const int y = (int)((i / g.nx) % g.ny);
  const int z = (int)(i / ((long)g.nx * g.ny));
  const float dv = tv_div(ydual, g, x, y, z);
  const float qo = q[i];
  const float qn = fmaxf(0.f, (qo + tau * dv + tau * v[i]) / (1.f + tau));
  q[i] = qn;
  qbar[i] = qn + theta * (qn - qo);
}

__global__ __launch_bounds__(kThreadsVec) void k_clip_copy(const float* __restrict__ v, float* __restrict__ q,
                                                           float* __restrict__ qbar, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = fmaxf(0.f, v[i]);
  q[i] = a;
  qbar[i] = a;
}

// ---------------------------------------------------------------- reductions
// Fixed launch shape: kRedBlocks blocks x kThreadsVec threads, element i handled
// by thread (i mod (kRedBlocks*kThreadsVec)) in increasing i.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kThreadsVec / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kThreadsVec / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  return sh[0];
}

// kind: 0 sum a^2, 1 sum a*b, 2 sum (a+b)^2
__global__ __launch_bounds__(kThreadsVec) void k_red_vec(const float* __restrict__ a, const float* __restrict__ b,
                                                         long n, int kind, double* __restrict__ partial) {
  __shared__ double sh[kThreadsVec];
  const long stride = (long)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = a[i];
    if (kind == 0) acc += x * x;
    else if (kind == 1) acc += x * (double)b[i];
    else { const double s = x + (double)b[i]; acc += s * s; }
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kThreadsVec) void k_red_tv(const float* __restrict__ q, TvGeom g,
                                                        double* __restrict__ partial) {
  __shared__ double sh[kThreadsVec];
  const long stride = (long)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < g.ndual; i += stride) {
    const int x = (int)(i % g.dx);
    const int y = (int)((i / g.dx) % g.dy);
    const int z = (int)(i / ((long)g.dx * g.dy));
    const float3 d = tv_grad(q, g, x, y, z);
    acc += sqrt((double)d.x * d.x + (double)d.y * d.y + (double)d.z * d.z);
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

struct Region {
  int nx, ny, nz;
  int x0, x1, y0, y1, z0, z1;   // half-open box
  __host__ __device__ long count() const { return (long)(x1 - x0) * (y1 - y0) * (z1 - z0); }
};

__device__ __forceinline__ long region_index(const Region& r, long k) {
  const int w = r.x1 - r.x0, h = r.y1 - r.y0;
  const int x = r.x0 + (int)(k % w);
  const int y = r.y0 + (int)((k / w) % h);
  const int z = r.z0 + (int)(k / ((long)w * h));
  return ((long)z * r.ny + y) * r.nx + x;
}

// max over the region of max(a, 0)
__global__ __launch_bounds__(kThreadsVec) void k_red_regmax(const float* __restrict__ a, Region reg,
                                                            double* __restrict__ partial) {
  __shared__ double sh[kThreadsVec];
  const long n = reg.count();
  const long stride = (long)gridDim.x * blockDim.x;
  double m = 0.0;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    m = fmax(m, (double)a[region_index(reg, k)]);
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__device__ __forceinline__ double psnr_norm(float v, double mx) {
  if (mx <= 0.0) return 0.0;
  const double t = fmax((double)v, 0.0) / mx;
  return t >= 0.1 ? t : 0.0;
}

// sum over the region of (thres(max(a,0)/ma) - thres(max(b,0)/mb))^2; maxima read from device
__global__ __launch_bounds__(kThreadsVec) void k_red_psnr(const float* __restrict__ a, const float* __restrict__ b,
                                                          Region reg, const double* __restrict__ maxima,
                                                          double* __restrict__ partial) {
  __shared__ double sh[kThreadsVec];
  const long n = reg.count();
  const long stride = (long)gridDim.x * blockDim.x;
  const double ma = maxima[0], mb = maxima[1];
  double acc = 0.0;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const long i = region_index(reg, k);
    const double d = psnr_norm(a[i], ma) - psnr_norm(b[i], mb);
    acc += d * d;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// out[slot] = sum (or max) of partial[0..nb) in a fixed order
__global__ __launch_bounds__(kThreadsVec) void k_red_final(const double* __restrict__ partial, int nb, int is_max,
                                                           double* __restrict__ out) {
  __shared__ double sh[kThreadsVec];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreadsVec) acc = is_max ? fmax(acc, partial[i]) : acc + partial[i];
  const double r = is_max ? block_max(acc, sh) : block_sum(acc, sh);
  if (threadIdx.x == 0) *out = r;
}

// ---------------------------------------------------------------- vector updates
// out = x + beta (x - xp)
__global__ __launch_bounds__(kThreadsVec) void k_extrapolate(const float* __restrict__ x, const float* __restrict__ xp,
                                                             float* __restrict__ out, float beta, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] + beta * (x[i] - xp[i]);
}

// out = a + s * b
__global__ __launch_bounds__(kThreadsVec) void k_axpy(const float* __restrict__ a, const float* __restrict__ b,
                                                      float* __restrict__ out, float s, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + s * b[i];
}

// out = s * a
__global__ __launch_bounds__(kThreadsVec) void k_scale(const float* __restrict__ a, float* __restrict__ out, float s,
                                                       long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = s * a[i];
}

// out = a + a[stride] (two plane series)
__global__ __launch_bounds__(kThreadsVec) void k_sum2(const float* __restrict__ a, long stride,
                                                      float* __restrict__ out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + a[i + stride];
}

// out[t][i] = w[i] * a[t][i] for the plane series [nt][npix] (sensor sensitivity, eq. FwdSenVar);
// out may be a (in place: one element per thread, read before written), so a and out are not __restrict__
__global__ __launch_bounds__(kThreadsVec) void k_scale_pixels(const float* a, const float* __restrict__ w, float* out,
                                                             long n, int npix) {
  const long i = (long)blockIdx.x * kThreadsVec + threadIdx.x;
  if (i < n) out[i] = w[i % npix] * a[i];
}

__global__ __launch_bounds__(kThreadsVec) void k_fill(float* __restrict__ out, float v, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

// ---------------------------------------------------------------- copy probe
// dst = src in 16-byte words: block b copies the kCopyUnroll * 256 consecutive words from
// b * kCopyUnroll * 256, all loads of a thread issued before its stores. This was the fastest of
// the copy forms measured (5.4-5.8 TB/s against 4.3-5.3 for grid-stride loops with or without
// non-temporal hints, and 5.0-5.3 for torch's copy): the device's practical HBM copy rate,
// against which the propagator's bandwidth is compared.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(kThreadsVec) void k_copy_probe(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                            long n16) {
  const long base = (long)blockIdx.x * (kCopyUnroll * kThreadsVec) + threadIdx.x;
  f32x4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long i = base + (long)u * kThreadsVec;
    if (i < n16) v[u] = src[i];
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long i = base + (long)u * kThreadsVec;
    if (i < n16) dst[i] = v[u];
  }
}

// ---------------------------------------------------------------- launchers
static unsigned nblocks(long n) { return (unsigned)((n + kThreadsVec - 1) / kThreadsVec); }

static TvGeom make_geom(int nx, int ny, int nz, int bc) {
  TvGeom g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.dirichlet = bc == 1;
  g.dx = nx + (bc == 1); g.dy = ny + (bc == 1); g.dz = nz + (bc == 1);
  g.ndual = (long)g.dx * g.dy * g.dz;
  return g;
}

hipError_t launch_pdhg_init(const float* v, float* q, float* qbar, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_clip_copy<<<nblocks(n), kThreadsVec, 0, st>>>(v, q, qbar, n);
  return hipGetLastError();
}

hipError_t launch_pdhg_iter(const float* v, float* q, float* qbar, float* dual, int nx, int ny, int nz, int bc,
                            float sigma, float tau, float theta, float alpha, hipStream_t st) {
  const TvGeom g = make_geom(nx, ny, nz, bc);
  k_pdhg_dual<<<nblocks(g.ndual), kThreadsVec, 0, st>>>(qbar, dual, g, sigma, alpha);
  k_pdhg_primal<<<nblocks((long)nx * ny * nz), kThreadsVec, 0, st>>>(v, q, qbar, dual, g, tau, theta);
  return hipGetLastError();
}

static int red_blocks(long n) {
  long b = (n + kThreadsVec - 1) / kThreadsVec;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_reduce_vec(const float* a, const float* b, long n, int kind, double* partial, double* out,
                             hipStream_t st) {
  const int nb = red_blocks(n);
  k_red_vec<<<nb, kThreadsVec, 0, st>>>(a, b, n, kind, partial);
  k_red_final<<<1, kThreadsVec, 0, st>>>(partial, nb, 0, out);
  return hipGetLastError();
}

hipError_t launch_reduce_tv(const float* q, int nx, int ny, int nz, int bc, double* partial, double* out,
                            hipStream_t st) {
  const TvGeom g = make_geom(nx, ny, nz, bc);
  const int nb = red_blocks(g.ndual);
  k_red_tv<<<nb, kThreadsVec, 0, st>>>(q, g, partial);
  k_red_final<<<1, kThreadsVec, 0, st>>>(partial, nb, 0, out);
  return hipGetLastError();
}

hipError_t launch_psnr(const float* a, const float* b, int nx, int ny, int nz, int x0, int x1, int y0, int y1,
                       int z0, int z1, double* partial, double* maxima, double* out, hipStream_t st) {
  Region r{nx, ny, nz, x0, x1, y0, y1, z0, z1};
  const long n = r.count();
  const int nb = red_blocks(n);
  k_red_regmax<<<nb, kThreadsVec, 0, st>>>(a, r, partial);
  k_red_final<<<1, kThreadsVec, 0, st>>>(partial, nb, 1, maxima);
  k_red_regmax<<<nb, kThreadsVec, 0, st>>>(b, r, partial);
  k_red_final<<<1, kThreadsVec, 0, st>>>(partial, nb, 1, maxima + 1);
  k_red_psnr<<<nb, kThreadsVec, 0, st>>>(a, b, r, maxima, partial);
  k_red_final<<<1, kThreadsVec, 0, st>>>(partial, nb, 0, out);
  return hipGetLastError();
}

hipError_t launch_extrapolate(const float* x, const float* xp, float* out, float beta, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_extrapolate<<<nblocks(n), kThreadsVec, 0, st>>>(x, xp, out, beta, n);
  return hipGetLastError();
}

hipError_t launch_axpy(const float* a, const float* b, float* out, float s, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_axpy<<<nblocks(n), kThreadsVec, 0, st>>>(a, b, out, s, n);
  return hipGetLastError();
}

hipError_t launch_scale(const float* a, float* out, float s, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_scale<<<nblocks(n), kThreadsVec, 0, st>>>(a, out, s, n);
  return hipGetLastError();
}

hipError_t launch_sum2(const float* a, long stride, float* out, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_sum2<<<nblocks(n), kThreadsVec, 0, st>>>(a, stride, out, n);
  return hipGetLastError();
}

hipError_t launch_scale_pixels(const float* a, const float* w, float* out, int nt, int npix, hipStream_t st) {
  const long n = (long)nt * npix;
  if (n == 0) return hipSuccess;
  k_scale_pixels<<<nblocks(n), kThreadsVec, 0, st>>>(a, w, out, n, npix);
  return hipGetLastError();
}

hipError_t launch_fill(float* out, float v, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_fill<<<nblocks(n), kThreadsVec, 0, st>>>(out, v, n);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, long n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const long per_block = (long)kThreadsVec * kCopyUnroll;
  const long grid = (n16 + per_block - 1) / per_block;   // <= 2^26 for the 2^40-byte limit
  k_copy_probe<<<(unsigned)grid, kThreadsVec, 0, st>>>(static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace pat
