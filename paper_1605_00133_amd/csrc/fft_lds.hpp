// In-place radix-R FFT stages on complex float data held in LDS, for gfx950.
//
// The wave propagator needs many small power-of-two transforms (lengths
// 8..128) along each axis of a 3D grid. A length-L transform is split into at
// most two radix stages (8, 16, 8x4, 8x8, 16x8); every thread loads R elements
// of one butterfly from LDS, runs the R-point DFT in registers and writes the R
// results back to the same LDS slots. Because each butterfly reads and writes
// its own slots, a stage needs no second buffer, only a barrier before the next.
//
//  * forward: decimation in frequency, natural-order input, output X[k] at
//    position pos(k) (digit-reversed), unnormalised, sign -1;
//  * inverse: the exact reverse of the forward stages (conjugate twiddles, then
//    the conjugate DFT), digit-reversed input, natural-order output,
//    unnormalised, sign +1; inverse(forward(x)) = L x.
//
// Pointwise spectral work between a forward and an inverse transform therefore
// never permutes data: it only needs freq(p), the frequency held at position p.
#pragma once

#include <hip/hip_runtime.h>

namespace pat {

__host__ __device__ constexpr int fft_nstages(int L) { return L <= 16 ? 1 : 2; }

__host__ __device__ constexpr int fft_radix(int L, int s) {
  return L == 4 ? 4 : L == 8 ? 8 : L == 16 ? 16 :
         L == 32 ? (s == 0 ? 8 : 4) : L == 64 ? 8 : L == 128 ? (s == 0 ? 16 : 8) : 16;
}

// Sub-transform length entering stage s.
__host__ __device__ constexpr int fft_sublen(int L, int s) { return s == 0 ? L : L / fft_radix(L, 0); }

// Position of frequency k after the forward transform.
__host__ __device__ constexpr int fft_pos(int L, int k) {
  return fft_nstages(L) == 1 ? k : (L / fft_radix(L, 0)) * (k % fft_radix(L, 0)) + k / fft_radix(L, 0);
}

// Frequency held at position p after the forward transform.
__host__ __device__ constexpr int fft_freq(int L, int p) {
  return fft_nstages(L) == 1 ? p : p / (L / fft_radix(L, 0)) + fft_radix(L, 0) * (p % (L / fft_radix(L, 0)));
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---- small DFTs in registers ------------------------------------------------
template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kCos8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kSin8 = 0.38268343236508977173f;   // sin(pi/8)

// multiply by w8^j = exp(-+ 2 pi i j / 8)
template <bool INV, int J>
__device__ __forceinline__ float2 tw8(float2 a) {
  if constexpr (J == 0) return a;
  if constexpr (J == 2) return mul_mi<INV>(a);
  if constexpr (J == 1) {
    // (1 -+ i)/sqrt2
    return INV ? make_float2((a.x - a.y) * kSqrtHalf, (a.x + a.y) * kSqrtHalf)
               : make_float2((a.x + a.y) * kSqrtHalf, (a.y - a.x) * kSqrtHalf);
  }
  if constexpr (J == 3) {
    // (-1 -+ i)/sqrt2
    return INV ? make_float2((-a.x - a.y) * kSqrtHalf, (a.x - a.y) * kSqrtHalf)
               : make_float2((a.y - a.x) * kSqrtHalf, (-a.x - a.y) * kSqrtHalf);
  }
  return a;
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
  // even/odd split: E = DFT4(a0,a2,a4,a6), O = DFT4(a1,a3,a5,a7)
  dft4<INV>(a[0], a[2], a[4], a[6]);
  dft4<INV>(a[1], a[3], a[5], a[7]);
  float2 o1 = tw8<INV, 1>(a[3]);
  float2 o2 = tw8<INV, 2>(a[5]);
  float2 o3 = tw8<INV, 3>(a[7]);
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// w16^j for j = 0..9 (the products n2*k1 needed below), sign chosen by INV
template <bool INV>
__device__ __forceinline__ float2 tw16(float2 a, int j) {
  float c, s;
  switch (j) {
    case 1: c = kCos8; s = kSin8; break;
    case 2: c = kSqrtHalf; s = kSqrtHalf; break;
    case 3: c = kSin8; s = kCos8; break;
    case 4: c = 0.f; s = 1.f; break;
    case 6: c = -kSqrtHalf; s = kSqrtHalf; break;
    case 9: c = -kCos8; s = -kSin8; break;
    default: return a;
  }
  // exp(-+ i theta) = c -+ i s
  float sg = INV ? s : -s;
  return make_float2(a.x * c - a.y * sg, a.x * sg + a.y * c);
}

template <bool INV>
__device__ __forceinline__ void dft16(float2* a) {
  // n = 4 n1 + n2, k = k1 + 4 k2:  X = sum_n2 w4^{n2 k2} [ w16^{n2 k1} sum_n1 a[4n1+n2] w4^{n1 k1} ]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  // now a[4*k1 + n2] holds B[n2][k1]
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) a[4 * k1 + n2] = tw16<INV>(a[4 * k1 + n2], n2 * k1);
  float2 b[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 c0 = a[4 * k1 + 0], c1 = a[4 * k1 + 1], c2 = a[4 * k1 + 2], c3 = a[4 * k1 + 3];
    dft4<INV>(c0, c1, c2, c3);
    b[k1] = c0; b[k1 + 4] = c1; b[k1 + 8] = c2; b[k1 + 12] = c3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = b[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2* a) {
  if constexpr (R == 2) dft2<INV>(a[0], a[1]);
  else if constexpr (R == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<INV>(a);
  else if constexpr (R == 16) dft16<INV>(a);
}

// ---- one radix stage over nseq sequences ------------------------------------
// Element n of sequence q lives at buf[q*seq_stride + n*elem_stride].
// SEQ_FAST: consecutive threads take consecutive sequences (use when sequences
// are adjacent in LDS, i.e. seq_stride == 1); otherwise consecutive butterflies
// of one sequence (use when elem_stride == 1).
template <int L, int S, bool INV, bool SEQ_FAST>
__device__ __forceinline__ void fft_stage(float2* buf, int nseq, int seq_stride, int elem_stride,
                                          const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int R = fft_radix(L, S);
  constexpr int LS = fft_sublen(L, S);
  constexpr int M = LS / R;
  constexpr int NB = L / R;
  constexpr int TWS = L / LS;
  const int total = nseq * NB;
  for (int w = tid; w < total; w += nthr) {
    int q, j;
    if (SEQ_FAST) { q = w % nseq; j = w / nseq; }
    else { j = w % NB; q = w / NB; }
    const int blk = j / M, n1 = j % M;
    float2* base = buf + q * seq_stride + (blk * LS + n1) * elem_stride;
    float2 a[R];
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = base[m * M * elem_stride];
    if constexpr (!INV) {
      dft_r<R, false>(a);
      if constexpr (M > 1) {
#pragma unroll
        for (int k = 1; k < R; ++k) a[k] = cmul(a[k], tw[TWS * n1 * k]);
      }
    } else {
      if constexpr (M > 1) {
#pragma unroll
        for (int k = 1; k < R; ++k) a[k] = cmulconj(a[k], tw[TWS * n1 * k]);
      }
      dft_r<R, true>(a);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) base[m * M * elem_stride] = a[m];
  }
}

// Forward transform (natural in, digit-reversed out). Caller syncs before; ends synced.
template <int L, bool SEQ_FAST>
__device__ __forceinline__ void fft_forward(float2* buf, int nseq, int seq_stride, int elem_stride,
                                            const float2* __restrict__ tw, int tid, int nthr) {
  fft_stage<L, 0, false, SEQ_FAST>(buf, nseq, seq_stride, elem_stride, tw, tid, nthr);
  __syncthreads();
  if constexpr (fft_nstages(L) > 1) {
    fft_stage<L, 1, false, SEQ_FAST>(buf, nseq, seq_stride, elem_stride, tw, tid, nthr);
    __syncthreads();
  }
}

// Inverse transform (digit-reversed in, natural out). Caller syncs before; ends synced.
template <int L, bool SEQ_FAST>
__device__ __forceinline__ void fft_inverse(float2* buf, int nseq, int seq_stride, int elem_stride,
                                            const float2* __restrict__ tw, int tid, int nthr) {
  if constexpr (fft_nstages(L) > 1) {
    fft_stage<L, 1, true, SEQ_FAST>(buf, nseq, seq_stride, elem_stride, tw, tid, nthr);
    __syncthreads();
  }
  fft_stage<L, 0, true, SEQ_FAST>(buf, nseq, seq_stride, elem_stride, tw, tid, nthr);
  __syncthreads();
}

}  // namespace pat
