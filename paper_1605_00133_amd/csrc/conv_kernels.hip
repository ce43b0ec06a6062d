// 3x3x3 convolution layers for a learned update step (outside the paper's
// method: a network mapping the iterate and the gradient A^T C^T (C A p - f)
// of eq. BP to the next iterate). BF16 operands on the matrix cores, FP32
// accumulation, FP32 tensors in HBM.
//
// Layout: activations [B][C][nz][ny][nx] (x fastest), weights [Co][Ci][3][3][3],
// zero padding of one voxel ("same" size). Every entry point is a GEMM over the
// taps and input channels:
//   forward       y[b][co][v]  = sum_{ci,tap} w[co][ci][tap] x[b][ci][v + d(tap)] (+ bias, ReLU)
//   input grad    dx[b][ci][v] = sum_{co,tap} w[co][ci][tap] dy[b][co][v - d(tap)]
//                 (the forward with w transposed over channels and the taps mirrored)
//   weight grad   dw[co][ci][tap] = sum_{b,v} dy[b][co][v] x[b][ci][v + d(tap)], db[co] = sum dy
// with tap = 9 (dz+1) + 3 (dy+1) + (dx+1).
//
// Matrix-core layouts (64 lanes, lane l, r = l & 15, q = l >> 4), result rows
// 4q..4q+3 (one per accumulator register), column r in both:
//   v_mfma_f32_16x16x16_bf16: A row r, K entries 4q..4q+3; B K entries 4q..4q+3, column r
//   v_mfma_f32_16x16x32_bf16: A row r, K entries 8q..8q+7; B K entries 8q..8q+7, column r
// Each operand value is rounded to BF16 (nearest even) when it is loaded or
// staged; sums stay FP32. The weight gradient writes one 16x16 partial per
// (chunk of rows, tile) and sums the chunks in a fixed order in FP64: results
// do not depend on scheduling.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/pat_nn.h"
#include "pat_internal.hpp"

#define PAT_NN_CHECK(expr)          \
  do {                              \
    const pat_status s_ = (expr);   \
    if (s_ != PAT_OK) return s_;    \
  } while (0)

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));   // bit patterns of 8 bfloat16
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTaps = 27;
constexpr int kWavesPerBlock = 4;
constexpr int kChunks = 256;   // row chunks of the weight gradient

__device__ __forceinline__ short bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u)   // Inf stays Inf, NaN stays a (quiet) NaN
    return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ void tap_offset(int tap, int& dz, int& dy, int& dx) {
  dz = tap / 9 - 1;
  dy = (tap / 3) % 3 - 1;
  dx = tap % 3 - 1;
}

// One wave: a 16 (x positions of one row) x 16 (output channels) tile.
// TW: the input-gradient form (weights [cin][cout][27] read transposed and mirrored).
template <bool TW>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_conv3d(
    const float* __restrict__ x, const float* __restrict__ w, const float* __restrict__ bias,
    float* __restrict__ y, int nb, int cin, int cout, int nz, int ny, int nx, int relu, int xtiles, int ctiles) {
  const int lane = threadIdx.x & 63;
  long t = (long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int xt = (int)(t % xtiles);
  t /= xtiles;
  const int ct = (int)(t % ctiles);
  t /= ctiles;
  const int yy = (int)(t % ny);
  t /= ny;
  const int zz = (int)(t % nz);
  t /= nz;
  const int b = (int)t;
  if (b >= nb) return;   // wave-uniform: the grid is rounded up to whole blocks
  const int r = lane & 15, q = lane >> 4;
  const int x0 = xt * 16;
  const int K = cin * kTaps;
  const long vol = (long)nz * ny * nx;
  const float* xb = x + (long)b * cin * vol;
  const int co_b = ct * 16 + r;   // this lane's B column
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, bw;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + 4 * q + i;
      float av = 0.f, bv = 0.f;
      if (k < K) {
        const int ci = k / kTaps, tap = k - ci * kTaps;
        int dz, dy, dx;
        tap_offset(tap, dz, dy, dx);
        const int z2 = zz + dz, y2 = yy + dy, x2 = x0 + r + dx;
        if (z2 >= 0 && z2 < nz && y2 >= 0 && y2 < ny && x2 >= 0 && x2 < nx)
          av = xb[ci * vol + ((long)z2 * ny + y2) * nx + x2];
        if (co_b < cout)
          bv = TW ? w[((long)ci * cout + co_b) * kTaps + (kTaps - 1 - tap)] : w[((long)co_b * cin + ci) * kTaps + tap];
      }
      a[i] = bf16_rne(av);
      bw[i] = bf16_rne(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc, 0, 0, 0);
  }
  if (co_b >= cout) return;
  const float bb = bias ? bias[co_b] : 0.f;
  float* yrow = y + ((long)b * cout + co_b) * vol + ((long)zz * ny + yy) * nx;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int xo = x0 + 4 * q + i;
    if (xo < nx) {
      float v = acc[i] + bb;
      yrow[xo] = relu ? fmaxf(v, 0.f) : v;
    }
  }
}

// Packed weights: the B operand of every 32-wide K chunk of v_mfma_f32_16x16x32_bf16
// in lane order, wb[((ct * nch + ch) * 64 + lane) * 8 + i] = B[k = 32 ch + 8 q + i][n = 16 ct + r],
// K ordered tap-major over a channel count padded to a multiple of 8
// (k = tap * cpad + c), zero outside the layer. TW: the input-gradient form.
template <bool TW>
__global__ __launch_bounds__(256) void k_conv3d_pack_weights(const float* __restrict__ w, short* __restrict__ wb,
                                                             int cin, int cout, int cpad, int nch, int ctiles) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)ctiles * nch * 512) return;
  const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
  const long cc = i >> 9;
  const int ch = (int)(cc % nch), ct = (int)(cc / nch);
  const int k = ch * 32 + 8 * (lane >> 4) + e, n = ct * 16 + (lane & 15);
  float v = 0.f;
  if (k < kTaps * cpad && n < cout) {
    const int tap = k / cpad, c = k - tap * cpad;
    if (c < cin)
      v = TW ? w[((long)c * cout + n) * kTaps + (kTaps - 1 - tap)] : w[((long)n * cin + c) * kTaps + tap];
  }
  wb[i] = bf16_rne(v);
}

constexpr int kTileX = 16, kTileY = 4;                     // output tile of one block: one row per wave
constexpr int kHaloX = kTileX + 2, kHaloY = kTileY + 2;
constexpr int kMaxCpadLds = 64;                            // larger layers use k_conv3d
constexpr int kMaxCt = 4;                                  // output-channel tiles per block
constexpr int kConvPlanes = 2;                             // output z-planes per block

// The input halo of a 16 x 4 x ZB output tile sits in LDS as bfloat16, channels
// innermost ([dz][y][x][cpad], ZB + 2 planes): the A operand of a lane (8
// channels at one tap of its voxel, v_mfma_f32_16x16x32_bf16: lane l holds row
// l & 15, K entries 8 (l >> 4) .. + 7) is one 16-byte LDS read. The packed B
// operand is one 16-byte global read per lane, the same for every block
// (cache-resident), and serves the ZB output planes of the block. Staging the
// halo (global loads, conversion, LDS stores) is a large share of the block's
// time: ZB planes per block stage (ZB + 2) / ZB planes per output plane, and
// each thread stages 8 channels of a voxel with one 16-byte LDS store.
template <int ZB>
__global__ __launch_bounds__(256) void k_conv3d_lds(const float* __restrict__ x, const short* __restrict__ wb,
                                                    const float* __restrict__ bias, float* __restrict__ y, int nb,
                                                    int cin, int cout, int nz, int ny, int nx, int relu, int cpad,
                                                    int nch, int ctiles, int xtiles, int ytiles, int cgroups,
                                                    int ztiles) {
  constexpr int kPlanes = ZB + 2;
  extern __shared__ __align__(16) unsigned char smem[];
  short* xs = reinterpret_cast<short*>(smem);
  const int plane = kHaloY * kHaloX * cpad;
  const int halo = kPlanes * plane;
  int* qoff = reinterpret_cast<int*>(xs + halo);           // halo is a multiple of 8 elements
  const int nq = kTaps * cpad / 8;
  long t = blockIdx.x;
  const int xt = (int)(t % xtiles);
  t /= xtiles;
  const int yt = (int)(t % ytiles);
  t /= ytiles;
  const int cg = (int)(t % cgroups);
  t /= cgroups;
  const int z0 = (int)(t % ztiles) * ZB;
  const int b = (int)(t / ztiles);
  const int x0 = xt * kTileX, y0 = yt * kTileY;
  const int tid = threadIdx.x;
  for (int j = tid; j < nq; j += 256) {
    const int tap = j / (cpad / 8), cq = j - tap * (cpad / 8);
    qoff[j] = (((tap / 9) * kHaloY + (tap / 3) % 3) * kHaloX + tap % 3) * cpad + 8 * cq;
  }
  const long vol = (long)nz * ny * nx;
  const float* xb = x + (long)b * cin * vol;
  // one item = 8 channels of one halo voxel, channel group fastest: consecutive lanes write
  // consecutive 16-byte LDS slots (one conflict-free store per item), and each of the 8 global
  // loads of an item reads consecutive x across the lanes of a channel group
  const int cq8 = cpad / 8;
  const int nitems = kPlanes * kHaloY * kHaloX * cq8;
  for (int i = tid; i < nitems; i += 256) {
    const int cq = i % cq8, vx = i / cq8;
    const int hx = vx % kHaloX;
    const int rest = vx / kHaloX;
    const int hy = rest % kHaloY, hz = rest / kHaloY;
    const int gz = z0 + hz - 1, gy = y0 + hy - 1, gx = x0 + hx - 1;
    bf16x8 pk = {0, 0, 0, 0, 0, 0, 0, 0};
    if (gz >= 0 && gz < nz && gy >= 0 && gy < ny && gx >= 0 && gx < nx) {
      const float* src = xb + (long)(8 * cq) * vol + ((long)gz * ny + gy) * nx + gx;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (8 * cq + k < cin) pk[k] = bf16_rne(src[(long)k * vol]);
    }
    *reinterpret_cast<bf16x8*>(xs + vx * cpad + 8 * cq) = pk;
  }
  __syncthreads();
  const int lane = tid & 63, wy = tid >> 6, r = lane & 15, q = lane >> 4;
  const int ct0 = cg * kMaxCt, nct = min(kMaxCt, ctiles - ct0);
  const short* arow = xs + (wy * kHaloX + r) * cpad;
  f32x4 acc[kMaxCt][ZB];
#pragma unroll
  for (int c = 0; c < kMaxCt; ++c)
#pragma unroll
    for (int p = 0; p < ZB; ++p) acc[c][p] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int ch = 0; ch < nch; ++ch) {
    const int j = ch * 4 + q;
    bf16x8 a[ZB];
#pragma unroll
    for (int p = 0; p < ZB; ++p) a[p] = j < nq ? *reinterpret_cast<const bf16x8*>(arow + p * plane + qoff[j]) : zero;
#pragma unroll
    for (int c = 0; c < kMaxCt; ++c) {
      if (c < nct) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(wb + (((long)(ct0 + c) * nch + ch) * 64 + lane) * 8);
#pragma unroll
        for (int p = 0; p < ZB; ++p)
          acc[c][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a[p]),
                                                              __builtin_bit_cast(bf16v8, bv), acc[c][p], 0, 0, 0);
      }
    }
  }
  const int yo = y0 + wy;
  if (yo >= ny) return;
#pragma unroll
  for (int c = 0; c < kMaxCt; ++c) {
    const int co = (ct0 + c) * 16 + r;
    if (c < nct && co < cout) {
      const float bb = bias ? bias[co] : 0.f;
#pragma unroll
      for (int p = 0; p < ZB; ++p) {
        if (z0 + p < nz) {
          float* yrow = y + ((long)b * cout + co) * vol + ((long)(z0 + p) * ny + yo) * nx;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int xo = x0 + 4 * q + i;
            if (xo < nx) {
              const float v = acc[c][p][i] + bb;
              yrow[xo] = relu ? fmaxf(v, 0.f) : v;
            }
          }
        }
      }
    }
  }
}

constexpr int kWgCols = 4;   // most column tiles per wave of the weight gradient (they share the dy operand)

// Weight (and bias) gradient partials: GEMM with M = co, N = k (27 cin taps, then one
// column of ones for the bias), K = voxels. Wave (chunk, mt, column group) sums the
// rows chunk, chunk + nchunk, ... of the B * nz * ny rows, 16 x positions at a time,
// into ncw <= kWgCols column tiles that share one A operand (dy).
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_conv3d_wgrad_partial(
    const float* __restrict__ x, const float* __restrict__ gy, float* __restrict__ part, int nb, int cin,
    int cout, int nz, int ny, int nx, int nchunk, int mtiles, int ngroups, int ncw) {
  const int lane = threadIdx.x & 63;
  long t = (long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int ng = (int)(t % ngroups);
  t /= ngroups;
  const int mt = (int)(t % mtiles);
  t /= mtiles;
  const int chunk = (int)t;
  if (chunk >= nchunk) return;   // wave-uniform
  const int r = lane & 15, q = lane >> 4;
  const int ncol = cin * kTaps + 1;
  const long vol = (long)nz * ny * nx;
  const long rows = (long)nb * nz * ny;
  const int co_a = mt * 16 + r;   // A row of this lane
  int ci[kWgCols], dz[kWgCols], dyo[kWgCols], dx[kWgCols];
  bool wcol[kWgCols], bcol[kWgCols];
#pragma unroll
  for (int j = 0; j < kWgCols; ++j) {
    const int kb = j < ncw ? (ng * ncw + j) * 16 + r : ncol;   // B column of this lane in tile j
    wcol[j] = kb < ncol - 1;
    bcol[j] = kb == ncol - 1;
    ci[j] = wcol[j] ? kb / kTaps : 0;
    tap_offset(wcol[j] ? kb - ci[j] * kTaps : 13, dz[j], dyo[j], dx[j]);
  }
  f32x4 acc[kWgCols];
#pragma unroll
  for (int j = 0; j < kWgCols; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long row = chunk; row < rows; row += nchunk) {
    const int yy = (int)(row % ny);
    const int zz = (int)((row / ny) % nz);
    const int b = (int)(row / ((long)ny * nz));
    const float* dyrow = gy + ((long)b * cout + co_a) * vol + ((long)zz * ny + yy) * nx;
    const float* xrow[kWgCols];
    bool rowin[kWgCols];
#pragma unroll
    for (int j = 0; j < kWgCols; ++j) {
      const int z2 = zz + dz[j], y2 = yy + dyo[j];
      rowin[j] = wcol[j] && z2 >= 0 && z2 < nz && y2 >= 0 && y2 < ny;
      xrow[j] = x + ((long)b * cin + ci[j]) * vol + ((long)(rowin[j] ? z2 : 0) * ny + (rowin[j] ? y2 : 0)) * nx;
    }
    for (int x0 = 0; x0 < nx; x0 += 16) {
      bf16x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int xv = x0 + 4 * q + i;
        a[i] = bf16_rne(xv < nx && co_a < cout ? dyrow[xv] : 0.f);
      }
#pragma unroll
      for (int j = 0; j < kWgCols; ++j) {
        bf16x4 bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int xv = x0 + 4 * q + i;
          float bx = 0.f;
          if (xv < nx) {
            if (rowin[j]) {
              const int x2 = xv + dx[j];
              if (x2 >= 0 && x2 < nx) bx = xrow[j][x2];
            } else if (bcol[j]) {
              bx = 1.f;
            }
          }
          bv[i] = bf16_rne(bx);
        }
        if (j < ncw) acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[j], 0, 0, 0);   // uniform
      }
    }
  }
  float* p = part + (long)chunk * cout * ncol;
#pragma unroll
  for (int j = 0; j < kWgCols; ++j) {
    const int kb = (ng * ncw + j) * 16 + r;
    if (j >= ncw || kb >= ncol) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * q + i;
      if (co < cout) p[(long)co * ncol + kb] = acc[j][i];
    }
  }
}

constexpr int kWgTiles = 8;   // (co tile, column tile) accumulators per wave of the LDS weight gradient
constexpr int kMaxChLds = 64;  // channel limit of the LDS weight gradient

// Weight-gradient partials with the operands in LDS. Block (chunk, tile group) sums the
// row groups chunk, chunk + nchunk, ... (4 rows of one (b, z) plane each), 16 x
// positions at a time: it stages that 4 x 16 tile of dy ([co][row][x], bfloat16) and
// the tile's input halo ([ci][dz][y][x], bfloat16) in LDS, then each wave adds its up
// to 8 tiles of the [co][ci * 27 + tap | bias] GEMM over the 64 voxels, one row (one
// K chunk) at a time. The row loop stays rolled so that only one row's operands are
// live (unrolled, the kernel needs 380 registers: one wave per SIMD). Partials as in
// k_conv3d_wgrad_partial.
__global__ __launch_bounds__(256) void k_conv3d_wgrad_lds(const float* __restrict__ x, const float* __restrict__ gy,
                                                          float* __restrict__ part, int nb, int cin, int cout, int nz,
                                                          int ny, int nx, int nchunk, int mtiles, int ntiles,
                                                          int tgroups, int ytiles, int xtiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int cpo = mtiles * 16;
  short* ds = reinterpret_cast<short*>(smem);                 // [cpo][kTileY][kTileX]
  short* xh = ds + cpo * kTileY * kTileX;                     // [cin][3][kHaloY][kHaloX]
  const int tg = (int)(blockIdx.x % tgroups), chunk = (int)(blockIdx.x / tgroups);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, q = lane >> 4;
  const int ncol = cin * kTaps + 1, T = mtiles * ntiles;
  const int tbase = (tg * 4 + wv) * kWgTiles;
  int aoff[kWgTiles], boff[kWgTiles], kind[kWgTiles];
#pragma unroll
  for (int s = 0; s < kWgTiles; ++s) {
    const int t = tbase + s;
    const int mt = t / ntiles, nt = t - mt * ntiles, n = nt * 16 + r;
    aoff[s] = (mt * 16 + r) * kTileY * kTileX;
    kind[s] = 2;   // zero column
    boff[s] = 0;
    if (t < T && n < ncol - 1) {
      const int ci = n / kTaps, tap = n - ci * kTaps;
      boff[s] = ((ci * 3 + tap / 9) * kHaloY + (tap / 3) % 3) * kHaloX + tap % 3;
      kind[s] = 0;
    } else if (t < T && n == ncol - 1) {
      kind[s] = 1;   // bias column: ones
    }
  }
  f32x4 acc[kWgTiles];
#pragma unroll
  for (int s = 0; s < kWgTiles; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long vol = (long)nz * ny * nx;
  const long groups = (long)nb * nz * ytiles;
  const int nds = cpo * kTileY * kTileX, nxh = cin * 3 * kHaloY * kHaloX;
  const short one = 0x3f80;   // 1.0 in bfloat16
  for (long g = chunk; g < groups; g += nchunk) {
    const int yt = (int)(g % ytiles);
    const int zz = (int)((g / ytiles) % nz);
    const int b = (int)(g / ((long)ytiles * nz));
    const int y0 = yt * kTileY;
    for (int xt = 0; xt < xtiles; ++xt) {
      const int x0 = xt * kTileX;
      __syncthreads();   // the previous tile's reads are done
      for (int i = tid; i < nds; i += 256) {
        const int xx = i % kTileX, rest = i / kTileX;
        const int ry = rest % kTileY, co = rest / kTileY;
        float v = 0.f;
        if (co < cout && y0 + ry < ny && x0 + xx < nx)
          v = gy[((long)b * cout + co) * vol + ((long)zz * ny + y0 + ry) * nx + x0 + xx];
        ds[i] = bf16_rne(v);
      }
      for (int i = tid; i < nxh; i += 256) {
        const int hx = i % kHaloX;
        int rest = i / kHaloX;
        const int hy = rest % kHaloY;
        rest /= kHaloY;
        const int hz = rest % 3, c = rest / 3;
        const int gz = zz + hz - 1, gyy = y0 + hy - 1, gx = x0 + hx - 1;
        float v = 0.f;
        if (gz >= 0 && gz < nz && gyy >= 0 && gyy < ny && gx >= 0 && gx < nx)
          v = x[((long)b * cin + c) * vol + ((long)gz * ny + gyy) * nx + gx];
        xh[i] = bf16_rne(v);
      }
      __syncthreads();
#pragma unroll 1
      for (int ry = 0; ry < kTileY; ++ry) {
#pragma unroll
        for (int s = 0; s < kWgTiles; ++s) {
          if (tbase + s < T) {   // wave-uniform
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(ds + aoff[s] + ry * kTileX + 4 * q);
            bf16x4 bv = {0, 0, 0, 0};
            if (kind[s] == 0) {
              const short* src = xh + boff[s] + ry * kHaloX + 4 * q;
              bv[0] = src[0];
              bv[1] = src[1];
              bv[2] = src[2];
              bv[3] = src[3];
            } else if (kind[s] == 1) {
              bv[0] = one;
              bv[1] = one;
              bv[2] = one;
              bv[3] = one;
            }
            acc[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[s], 0, 0, 0);
          }
        }
      }
    }
  }
  float* p = part + (long)chunk * cout * ncol;
#pragma unroll
  for (int s = 0; s < kWgTiles; ++s) {
    const int t = tbase + s;
    if (t >= T) continue;
    const int mt = t / ntiles, nt = t - mt * ntiles, n = nt * 16 + r;
    if (n >= ncol) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * q + i;
      if (co < cout) p[(long)co * ncol + n] = acc[s][i];
    }
  }
}

// dw[co][k] = sum over the chunks (FP64, fixed order: 16 interleaved partial sums per
// column, then those 16 in order); the last column goes to db. Block: 16 columns x 16.
__global__ __launch_bounds__(256) void k_conv3d_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dw,
                                                             float* __restrict__ db, int cin, int cout, int nchunk) {
  __shared__ double red[16][17];
  const int ncol = cin * kTaps + 1;
  const long total = (long)cout * ncol;
  const int lc = threadIdx.x & 15, lk = threadIdx.x >> 4;
  const long i = (long)blockIdx.x * 16 + lc;
  double s = 0.0;
  if (i < total)
    for (int c = lk; c < nchunk; c += 16) s += part[(long)c * total + i];
  red[lk][lc] = s;
  __syncthreads();
  if (lk != 0 || i >= total) return;
  double t = 0.0;
  for (int j = 0; j < 16; ++j) t += red[j][lc];
  const int co = (int)(i / ncol), k = (int)(i % ncol);
  if (k < ncol - 1)
    dw[(long)co * (ncol - 1) + k] = (float)t;
  else if (db)
    db[co] = (float)t;
}

__global__ __launch_bounds__(256) void k_relu_grad(const float* __restrict__ y, float* __restrict__ g, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}

// Adam: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2; w -= lr mhat / (sqrt(vhat) + eps)
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int nchunks(long rows) { return (int)(rows < kChunks ? rows : kChunks); }

// The LDS weight gradient runs (chunk, tile group) blocks. With one tile group (narrow
// layers: at most 32 output tiles) kChunks chunks leave one block per CU, too few to hide
// its staging latency: such layers take kChunksNarrow chunks, four blocks per CU (16 -> 16
// channels at 128^3: 1.86 -> 1.14 ms). Wider layers keep kChunks (with three tile groups,
// 342 chunks were 30 % slower than 256: more partials to write and sum). Never more chunks
// than row groups.
constexpr long kChunksNarrow = 1024;

bool wgrad_uses_lds(long rows, int cin, int cout) { return rows > 0 && cin <= kMaxChLds && cout <= kMaxChLds; }

int wgrad_lds_tgroups(int cin, int cout) {
  const int mtiles = (cout + 15) / 16, ntiles = (cin * kTaps + 1 + 15) / 16;
  return (mtiles * ntiles + 4 * kWgTiles - 1) / (4 * kWgTiles);
}

int wgrad_lds_chunks(int batch, int cin, int cout, int nz, int ny) {
  const long groups = (long)batch * nz * ((ny + kTileY - 1) / kTileY);
  long nc = wgrad_lds_tgroups(cin, cout) == 1 ? kChunksNarrow : kChunks;
  if (nc > groups) nc = groups;
  return (int)(nc < 1 ? 1 : nc);
}

pat_status conv_args(const char* who, int nb, int cin, int cout, int nz, int ny, int nx) {
  if (nb < 0 || cin < 1 || cout < 1 || nz < 1 || ny < 1 || nx < 1)
    return pat::set_error(PAT_ERR_INVALID, "%s: sizes must be positive (batch >= 0)", who);
  if ((long)cin * kTaps > (1L << 20) || (long)cout > (1L << 16))
    return pat::set_error(PAT_ERR_INVALID, "%s: too many channels", who);
  if ((long)nb * cin * nz * ny * nx > (1L << 34) || (long)nb * cout * nz * ny * nx > (1L << 34))
    return pat::set_error(PAT_ERR_INVALID, "%s: tensor too large", who);
  return PAT_OK;
}

pat_status launched(const char* who) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PAT_OK : pat::set_error(PAT_ERR_HIP, "%s: %s", who, hipGetErrorString(e));
}

int conv_cpad(int cin) { return (cin + 7) / 8 * 8; }
int conv_nch(int cin) { return (kTaps * conv_cpad(cin) + 31) / 32; }
bool conv_uses_lds(int cin) { return conv_cpad(cin) <= kMaxCpadLds; }
size_t conv_pack_bytes(int cin, int cout) {
  return conv_uses_lds(cin) ? (size_t)((cout + 15) / 16) * conv_nch(cin) * 512 * sizeof(short) : 0;
}

template <bool TW>
pat_status launch_conv(const char* who, const float* x, const float* w, const float* bias, float* y, int nb, int cin,
                       int cout, int nz, int ny, int nx, int relu, void* workspace, size_t workspace_bytes,
                       void* stream) {
  if (nb == 0) return PAT_OK;
  hipStream_t st = (hipStream_t)stream;
  if (conv_uses_lds(cin)) {
    const size_t need = conv_pack_bytes(cin, cout);
    if (!workspace || workspace_bytes < need)
      return pat::set_error(PAT_ERR_NOMEM, "%s: workspace of %zu bytes needed", who, need);
    const int cpad = conv_cpad(cin), nch = conv_nch(cin), ctiles = (cout + 15) / 16;
    const int xtiles = (nx + kTileX - 1) / kTileX, ytiles = (ny + kTileY - 1) / kTileY;
    const int cgroups = (ctiles + kMaxCt - 1) / kMaxCt;
    // two output planes per block (four staged planes, at most 55 KB of LDS): 92 VGPRs. Four
    // planes per block need 168 (three waves per SIMD) and ran 20-35 % slower; one plane per
    // block stages three planes per output plane instead of two.
    constexpr int zb = kConvPlanes;
    const int ztiles = (nz + zb - 1) / zb;
    const long blocks = (long)nb * ztiles * cgroups * ytiles * xtiles;
    if (blocks > 0x7fffffffL) return pat::set_error(PAT_ERR_INVALID, "%s: grid too large", who);
    short* wb = (short*)workspace;
    const long npack = (long)ctiles * nch * 512;
    hipLaunchKernelGGL(k_conv3d_pack_weights<TW>, dim3((unsigned)((npack + 255) / 256)), dim3(256), 0, st, w, wb, cin,
                       cout, cpad, nch, ctiles);
    const size_t lds = (size_t)(zb + 2) * kHaloY * kHaloX * cpad * sizeof(short) +
                       (size_t)(kTaps * cpad / 8) * sizeof(int);
    hipLaunchKernelGGL(k_conv3d_lds<zb>, dim3((unsigned)blocks), dim3(256), lds, st, x, wb, bias, y, nb, cin, cout, nz,
                       ny, nx, relu, cpad, nch, ctiles, xtiles, ytiles, cgroups, ztiles);
    return launched(who);
  }
  const int xtiles = (nx + 15) / 16, ctiles = (cout + 15) / 16;
  const long waves = (long)nb * nz * ny * ctiles * xtiles;
  const long blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 0x7fffffffL) return pat::set_error(PAT_ERR_INVALID, "%s: grid too large", who);
  hipLaunchKernelGGL(k_conv3d<TW>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, st, x, w, bias, y, nb, cin,
                     cout, nz, ny, nx, relu, xtiles, ctiles);
  return launched(who);
}

// Packed weights of pat_conv3d_forward_static: a file-scope device array, one
// copy per GPU, held until the process ends. Host code never passes its name to
// a kernel (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) unsigned char scratch[PAT_CONV_STATIC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the device of `st` (the current device for the
// null stream); found with that device current, then kept.
pat_status static_scratch(hipStream_t st, void** out) {
  int dev = -1;
  if (st) {
    hipDevice_t d = -1;
    const hipError_t e = hipStreamGetDevice(st, &d);
    if (e != hipSuccess) return pat::set_error(PAT_ERR_HIP, "hipStreamGetDevice: %s", hipGetErrorString(e));
    dev = d;
  } else {
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pat::set_error(PAT_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  if (dev < 0 || dev >= kMaxScratchDevices)
    return pat::set_error(PAT_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d", dev,
                          kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return pat::set_error(PAT_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PAT_OK;
}

}  // namespace

extern "C" {

size_t pat_conv3d_workspace_bytes(int32_t c_in, int32_t c_out) {
  if (c_in < 1 || c_out < 1 || (long)c_in * kTaps > (1L << 20) || (long)c_out > (1L << 16)) return 0;
  // forward packs (c_in -> c_out), the input gradient (c_out -> c_in): room for either
  const size_t a = conv_pack_bytes(c_in, c_out), b = conv_pack_bytes(c_out, c_in);
  const size_t m = a > b ? a : b;
  return m > 0 ? m : 256;
}

pat_status pat_conv3d_forward(const float* x, const float* w, const float* bias, float* y, int32_t batch,
                              int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx, int32_t relu,
                              void* workspace, size_t workspace_bytes, void* stream) {
  PAT_NN_CHECK(conv_args("pat_conv3d_forward", batch, c_in, c_out, nz, ny, nx));
  if (batch > 0 && (!x || !w || !y)) return pat::set_error(PAT_ERR_INVALID, "pat_conv3d_forward: null pointer");
  return launch_conv<false>("pat_conv3d_forward", x, w, bias, y, batch, c_in, c_out, nz, ny, nx, relu ? 1 : 0,
                            workspace, workspace_bytes, stream);
}

pat_status pat_conv3d_forward_static(const float* x, const float* w, const float* bias, float* y, int32_t batch,
                                     int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx, int32_t relu,
                                     void* stream) {
  static const char* who = "pat_conv3d_forward_static";
  PAT_NN_CHECK(conv_args(who, batch, c_in, c_out, nz, ny, nx));
  if (batch > 0 && (!x || !w || !y)) return pat::set_error(PAT_ERR_INVALID, "%s: null pointer", who);
  const size_t need = conv_pack_bytes(c_in, c_out);
  if (need > PAT_CONV_STATIC_SCRATCH_BYTES)
    return pat::set_error(PAT_ERR_INVALID, "%s: the layer's packed weights need %zu bytes, the static scratch holds %zu",
                          who, need, (size_t)PAT_CONV_STATIC_SCRATCH_BYTES);
  if (batch == 0) return PAT_OK;
  void* ws = nullptr;
  PAT_NN_CHECK(static_scratch((hipStream_t)stream, &ws));
  return launch_conv<false>(who, x, w, bias, y, batch, c_in, c_out, nz, ny, nx, relu ? 1 : 0, ws,
                            PAT_CONV_STATIC_SCRATCH_BYTES, stream);
}

pat_status pat_conv3d_backward_input(const float* dy, const float* w, float* dx, int32_t batch, int32_t c_in,
                                     int32_t c_out, int32_t nz, int32_t ny, int32_t nx, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  PAT_NN_CHECK(conv_args("pat_conv3d_backward_input", batch, c_in, c_out, nz, ny, nx));
  if (batch > 0 && (!dy || !w || !dx))
    return pat::set_error(PAT_ERR_INVALID, "pat_conv3d_backward_input: null pointer");
  // the forward over c_out input channels producing c_in, weights read transposed
  return launch_conv<true>("pat_conv3d_backward_input", dy, w, nullptr, dx, batch, c_out, c_in, nz, ny, nx, 0,
                           workspace, workspace_bytes, stream);
}

size_t pat_conv3d_backward_weight_workspace_bytes(int32_t batch, int32_t c_in, int32_t c_out, int32_t nz, int32_t ny,
                                                  int32_t nx) {
  if (conv_args("pat_conv3d_backward_weight_workspace_bytes", batch, c_in, c_out, nz, ny, nx) != PAT_OK) return 0;
  const long rows = (long)batch * nz * ny;
  const int nc = wgrad_uses_lds(rows, c_in, c_out) ? wgrad_lds_chunks(batch, c_in, c_out, nz, ny)
                                                    : nchunks(rows < 1 ? 1 : rows);
  return (size_t)nc * c_out * (c_in * kTaps + 1) * sizeof(float);
}

pat_status pat_conv3d_backward_weight(const float* x, const float* dy, float* dw, float* dbias, int32_t batch,
                                      int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx,
                                      void* workspace, size_t workspace_bytes, void* stream) {
  PAT_NN_CHECK(conv_args("pat_conv3d_backward_weight", batch, c_in, c_out, nz, ny, nx));
  if (!dw || (batch > 0 && (!x || !dy)))
    return pat::set_error(PAT_ERR_INVALID, "pat_conv3d_backward_weight: null pointer");
  const size_t need = pat_conv3d_backward_weight_workspace_bytes(batch, c_in, c_out, nz, ny, nx);
  if (!workspace || workspace_bytes < need)
    return pat::set_error(PAT_ERR_NOMEM, "pat_conv3d_backward_weight: workspace of %zu bytes needed", need);
  const long rows = (long)batch * nz * ny;
  int nc = nchunks(rows < 1 ? 1 : rows);
  const int mtiles = (c_out + 15) / 16, ntiles = (c_in * kTaps + 1 + 15) / 16;
  // sharing dy pays when there are many column tiles; with few, one tile per wave keeps more waves
  const int ncw = ntiles >= 16 ? kWgCols : 1;
  const int ngroups = (ntiles + ncw - 1) / ncw;
  float* part = (float*)workspace;
  if (wgrad_uses_lds(rows, c_in, c_out)) {
    const int ytiles = (ny + kTileY - 1) / kTileY, xtiles = (nx + kTileX - 1) / kTileX;
    nc = wgrad_lds_chunks(batch, c_in, c_out, nz, ny);   // the count the workspace was sized for
    const int tgroups = wgrad_lds_tgroups(c_in, c_out);
    const size_t lds = ((size_t)mtiles * 16 * kTileY * kTileX + (size_t)c_in * 3 * kHaloY * kHaloX) * sizeof(short);
    hipLaunchKernelGGL(k_conv3d_wgrad_lds, dim3((unsigned)((long)nc * tgroups)), dim3(256), lds, (hipStream_t)stream, x,
                       dy, part, batch, c_in, c_out, nz, ny, nx, nc, mtiles, ntiles, tgroups, ytiles, xtiles);
    PAT_NN_CHECK(launched("pat_conv3d_backward_weight"));
  } else if (rows > 0) {
    const long waves = (long)nc * mtiles * ngroups;
    hipLaunchKernelGGL(k_conv3d_wgrad_partial, dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)),
                       dim3(64 * kWavesPerBlock), 0, (hipStream_t)stream, x, dy, part, batch, c_in, c_out, nz, ny, nx,
                       nc, mtiles, ngroups, ncw);
    PAT_NN_CHECK(launched("pat_conv3d_backward_weight"));
  }
  const long n = (long)c_out * (c_in * kTaps + 1);
  // with no rows every partial is zero: reduce over zero chunks
  hipLaunchKernelGGL(k_conv3d_wgrad_reduce, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, (hipStream_t)stream,
                     part, dw, dbias, c_in, c_out, rows > 0 ? nc : 0);
  return launched("pat_conv3d_backward_weight");
}

pat_status pat_relu_backward(const float* y, float* grad, int64_t n, void* stream) {
  if (n < 0) return pat::set_error(PAT_ERR_INVALID, "pat_relu_backward: n must be >= 0");
  if (n == 0) return PAT_OK;
  if (!y || !grad) return pat::set_error(PAT_ERR_INVALID, "pat_relu_backward: null pointer");
  hipLaunchKernelGGL(k_relu_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, grad, n);
  return launched("pat_relu_backward");
}

pat_status pat_adam_step(float* w, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* stream) {
  if (n < 0 || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return pat::set_error(PAT_ERR_INVALID, "pat_adam_step: argument out of range");
  if (n == 0) return PAT_OK;
  if (!w || !grad || !m || !v) return pat::set_error(PAT_ERR_INVALID, "pat_adam_step: null pointer");
  const double c1 = 1.0 - std::pow((double)beta1, step), c2 = 1.0 - std::pow((double)beta2, step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w, grad, m, v, n,
                     lr, beta1, beta2, eps, (float)c1, (float)c2);
  return launched("pat_adam_step");
}

}  // extern "C"
