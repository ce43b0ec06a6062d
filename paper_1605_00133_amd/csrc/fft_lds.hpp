// In-place radix-R FFT stages on complex data held in LDS, for gfx950.
//
// The wave propagator needs many small power-of-two transforms (lengths
// 4..128) along each axis of a 3D grid. A length-L transform is split into at
// most two radix stages (4, 8, 16, 8x4, 8x8, 16x8); every thread loads R
// elements of one butterfly from LDS, runs the R-point DFT in registers and
// writes the R results back to the same LDS slots. Because each butterfly reads
// and writes its own slots, a stage needs no second buffer, only a barrier
// before the next.
//
//  * forward: decimation in frequency, natural-order input, output X[k] at
//    position pos(k) (digit-reversed), unnormalised, sign -1;
//  * inverse: the exact reverse of the forward stages (conjugate twiddles, then
//    the conjugate DFT), digit-reversed input, natural-order output,
//    unnormalised, sign +1; inverse(forward(x)) = L x.
//
// Pointwise spectral work between a forward and an inverse transform therefore
// never permutes data: it only needs freq(p), the frequency held at position p.
//
// The arithmetic type V is float2 or double2. Data in HBM is always float2;
// with V = double2 a transform keeps FP64 values in registers and LDS and
// rounds to FP32 only when its result leaves the kernel.
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

template <typename V> struct ScalarOf;
template <> struct ScalarOf<float2> { using T = float; };
template <> struct ScalarOf<double2> { using T = double; };

template <typename V>
__device__ __forceinline__ V mkc(typename ScalarOf<V>::T x, typename ScalarOf<V>::T y) {
  V r;
  r.x = x;
  r.y = y;
  return r;
}

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mkc<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mkc<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mkc<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cmulconj(V a, V b) {  // a * conj(b)
  return mkc<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return mkc<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, typename ScalarOf<V>::T s) {
  return mkc<V>(a.x * s, a.y * s);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V>
__device__ __forceinline__ V mul_mi(V a) {
  return INV ? mkc<V>(-a.y, a.x) : mkc<V>(a.y, -a.x);
}

// float2 <-> arithmetic type
template <typename V> __device__ __forceinline__ V widen(float2 a) { return mkc<V>(a.x, a.y); }
template <typename V> __device__ __forceinline__ float2 narrow(V a) { return make_float2((float)a.x, (float)a.y); }

// ---- small DFTs in registers ------------------------------------------------
template <bool INV, typename V>
__device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3) {
  V t0 = cadd(a0, a2), t1 = csub(a0, a2);
  V t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kCos8 = 0.92387953251128675613;   // cos(pi/8)
constexpr double kSin8 = 0.38268343236508977173;   // sin(pi/8)

// multiply by w8^J = exp(-+ 2 pi i J / 8)
template <bool INV, int J, typename V>
__device__ __forceinline__ V tw8(V a) {
  using S = typename ScalarOf<V>::T;
  const S h = (S)kSqrtHalf;
  if constexpr (J == 0) return a;
  else if constexpr (J == 2) return mul_mi<INV>(a);
  else if constexpr (J == 1)   // (1 -+ i)/sqrt2
    return INV ? mkc<V>((a.x - a.y) * h, (a.x + a.y) * h) : mkc<V>((a.x + a.y) * h, (a.y - a.x) * h);
  else                         // J == 3: (-1 -+ i)/sqrt2
    return INV ? mkc<V>((-a.x - a.y) * h, (a.x - a.y) * h) : mkc<V>((a.y - a.x) * h, (-a.x - a.y) * h);
}

template <bool INV, typename V>
__device__ __forceinline__ void dft8(V* a) {
  // even/odd split: E = DFT4(a0,a2,a4,a6), O = DFT4(a1,a3,a5,a7)
  dft4<INV>(a[0], a[2], a[4], a[6]);
  dft4<INV>(a[1], a[3], a[5], a[7]);
  V o1 = tw8<INV, 1>(a[3]);
  V o2 = tw8<INV, 2>(a[5]);
  V o3 = tw8<INV, 3>(a[7]);
  V e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// multiply by w16^j for the products j = n2*k1 that occur below, sign chosen by INV
template <bool INV, typename V>
__device__ __forceinline__ V tw16(V a, int j) {
  using S = typename ScalarOf<V>::T;
  S c, s;
  switch (j) {
    case 1: c = (S)kCos8; s = (S)kSin8; break;
    case 2: c = (S)kSqrtHalf; s = (S)kSqrtHalf; break;
    case 3: c = (S)kSin8; s = (S)kCos8; break;
    case 4: c = (S)0; s = (S)1; break;
    case 6: c = -(S)kSqrtHalf; s = (S)kSqrtHalf; break;
    case 9: c = -(S)kCos8; s = -(S)kSin8; break;
    default: return a;
  }
  // exp(-+ i theta) = c -+ i s
  const S sg = INV ? s : -s;
  return mkc<V>(a.x * c - a.y * sg, a.x * sg + a.y * c);
}

template <bool INV, typename V>
__device__ __forceinline__ void dft16(V* a) {
  // n = 4 n1 + n2, k = k1 + 4 k2:  X = sum_n2 w4^{n2 k2} [ w16^{n2 k1} sum_n1 a[4n1+n2] w4^{n1 k1} ]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  // now a[4*k1 + n2] holds B[n2][k1]
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) a[4 * k1 + n2] = tw16<INV>(a[4 * k1 + n2], n2 * k1);
  V b[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    V c0 = a[4 * k1 + 0], c1 = a[4 * k1 + 1], c2 = a[4 * k1 + 2], c3 = a[4 * k1 + 3];
    dft4<INV>(c0, c1, c2, c3);
    b[k1] = c0; b[k1 + 4] = c1; b[k1 + 8] = c2; b[k1 + 12] = c3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = b[i];
}

template <int R, bool INV, typename V>
__device__ __forceinline__ void dft_r(V* a) {
  if constexpr (R == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<INV>(a);
  else if constexpr (R == 16) dft16<INV>(a);
}

// ---- one radix stage over NSEQ sequences ------------------------------------
// Element n of sequence q lives at buf[q*SS + n*ES]. All geometry is compile
// time, so the butterfly loop is fully unrolled and the LDS reads of every
// butterfly a thread owns are issued together. SEQ_FAST: consecutive threads
// take consecutive sequences (use when SS == 1); otherwise consecutive
// butterflies of one sequence (use when ES == 1). tw: the L-point twiddle
// table exp(-2 pi i j / L), j < L, in the arithmetic type (an LDS copy).
template <int L, int S, bool INV, bool SEQ_FAST, int NSEQ, int SS, int ES, int NT, typename V>
__device__ __forceinline__ void fft_stage(V* buf, const V* tw, int tid) {
  constexpr int R = fft_radix(L, S);
  constexpr int LS = fft_sublen(L, S);
  constexpr int M = LS / R;
  constexpr int NB = L / R;
  constexpr int TWS = L / LS;
  constexpr int TOTAL = NSEQ * NB;
  constexpr int IT = (TOTAL + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = tid + i * NT;
    if (TOTAL % NT == 0 || w < TOTAL) {
      int q, j;
      if (SEQ_FAST) { q = w % NSEQ; j = w / NSEQ; }
      else { j = w % NB; q = w / NB; }
      const int blk = j / M, n1 = j % M;
      V* base = buf + q * SS + (blk * LS + n1) * ES;
      V a[R];
#pragma unroll
      for (int m = 0; m < R; ++m) a[m] = base[m * M * ES];
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
      for (int m = 0; m < R; ++m) base[m * M * ES] = a[m];
    }
  }
}

// Forward transform (natural in, digit-reversed out). Caller syncs before; ends synced.
template <int L, bool SEQ_FAST, int NSEQ, int SS, int ES, int NT, typename V>
__device__ __forceinline__ void fft_forward(V* buf, const V* tw, int tid) {
  fft_stage<L, 0, false, SEQ_FAST, NSEQ, SS, ES, NT>(buf, tw, tid);
  __syncthreads();
  if constexpr (fft_nstages(L) > 1) {
    fft_stage<L, 1, false, SEQ_FAST, NSEQ, SS, ES, NT>(buf, tw, tid);
    __syncthreads();
  }
}

// Inverse transform (digit-reversed in, natural out). Caller syncs before; ends synced.
template <int L, bool SEQ_FAST, int NSEQ, int SS, int ES, int NT, typename V>
__device__ __forceinline__ void fft_inverse(V* buf, const V* tw, int tid) {
  if constexpr (fft_nstages(L) > 1) {
    fft_stage<L, 1, true, SEQ_FAST, NSEQ, SS, ES, NT>(buf, tw, tid);
    __syncthreads();
  }
  fft_stage<L, 0, true, SEQ_FAST, NSEQ, SS, ES, NT>(buf, tw, tid);
  __syncthreads();
}

}  // namespace pat
