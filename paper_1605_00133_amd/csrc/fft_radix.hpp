// Small DFTs in registers and the two-stage split of the propagator's FFTs, for gfx950.
//
// The wave propagator needs transforms of lengths 8..128 along each axis of a
// 3D grid (powers of two, and 48 = 12 * 4, 96 = 12 * 8 for 96^3 grids). A
// length-L transform is split as L = R0 * M (R0 = 16 for L = 16, 128; 12 for
// L = 48, 96; 8 for L = 8, 32, 64; M = L / R0, M = 1 for L <= 16):
//
//  * forward stage 0 (decimation in frequency): for every n1 < M the R0 values
//    x[n1 + M m], m < R0, go through an R0-point DFT and are multiplied by
//    w_L^(n1 k); result k is kept at index n1 + M k;
//  * forward stage 1: every block b < R0 (indices M b + j, j < M) goes through
//    an M-point DFT; frequency b + R0 k1 ends at position M b + k1.
//
// A thread owns one butterfly of a stage with all its values in registers;
// stages exchange data through LDS once. The inverse runs the same two stages
// backwards (conjugate DFTs and twiddles), reading positions and producing
// natural order, unnormalised, so inverse(forward(x)) = L x. Pointwise
// spectral work between a forward and an inverse transform never permutes
// data: it only needs freq(p), the frequency held at position p.
//
// The arithmetic type V is float2 or double2. Data in HBM is always float2;
// with V = double2 the values stay FP64 in registers and LDS and are rounded to
// FP32 only when they leave the kernel.
#pragma once

#include <hip/hip_runtime.h>


namespace pat {

__host__ __device__ constexpr int fft_nstages(int L) { return L <= 16 ? 1 : 2; }

__host__ __device__ constexpr int fft_radix(int L, int s) {
  return L == 4 ? 4 : L == 8 ? 8 : L == 16 ? 16 :
         L == 32 ? (s == 0 ? 8 : 4) : L == 64 ? 8 : L == 128 ? (s == 0 ? 16 : 8) :
         L == 48 ? (s == 0 ? 12 : 4) : L == 96 ? (s == 0 ? 12 : 8) : 16;
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

// 3-point DFT: X0 = a0 + t, X1,2 = (a0 - t/2) -+ i (sqrt3/2) (a1 - a2) (forward; inverse: +-), t = a1 + a2
constexpr double kSqrt3Half = 0.86602540378443864676;   // sin(pi/3)

template <bool INV, typename V>
__device__ __forceinline__ void dft3(V& a0, V& a1, V& a2) {
  using S = typename ScalarOf<V>::T;
  const V t = cadd(a1, a2);
  const V m = mkc<V>(a0.x - (S)0.5 * t.x, a0.y - (S)0.5 * t.y);
  const V d = csub(a1, a2);
  const V r = mul_mi<INV>(cscale(d, (S)kSqrt3Half));   // -i (sqrt3/2) d forward, +i inverse
  a0 = cadd(a0, t);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

// multiply by w12^j = exp(-+ 2 pi i j / 12) for the products j = n2 k1 of dft12
template <bool INV, typename V>
__device__ __forceinline__ V tw12(V a, int j) {
  using S = typename ScalarOf<V>::T;
  S c, s;
  switch (j) {
    case 1: c = (S)kSqrt3Half; s = (S)0.5; break;
    case 2: c = (S)0.5; s = (S)kSqrt3Half; break;
    case 3: c = (S)0; s = (S)1; break;
    case 4: c = -(S)0.5; s = (S)kSqrt3Half; break;
    case 6: c = -(S)1; s = (S)0; break;
    default: return a;
  }
  const S sg = INV ? s : -s;   // exp(-+ i theta) = c -+ i s
  return mkc<V>(a.x * c - a.y * sg, a.x * sg + a.y * c);
}

template <bool INV, typename V>
__device__ __forceinline__ void dft12(V* a) {
  // n = 4 n1 + n2 (n1 < 3, n2 < 4), k = k1 + 3 k2:
  // X = sum_n2 w4^{n2 k2} [ w12^{n2 k1} sum_n1 a[4n1+n2] w3^{n1 k1} ]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft3<INV>(a[n2], a[4 + n2], a[8 + n2]);
  // now a[4*k1 + n2] holds B[n2][k1]
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 3; ++k1) a[4 * k1 + n2] = tw12<INV>(a[4 * k1 + n2], n2 * k1);
  V b[12];
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    V c0 = a[4 * k1 + 0], c1 = a[4 * k1 + 1], c2 = a[4 * k1 + 2], c3 = a[4 * k1 + 3];
    dft4<INV>(c0, c1, c2, c3);
    b[k1] = c0; b[k1 + 3] = c1; b[k1 + 6] = c2; b[k1 + 9] = c3;
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) a[i] = b[i];
}

template <int R, bool INV, typename V>
__device__ __forceinline__ void dft_r(V* a) {
  if constexpr (R == 1) (void)a;
  else if constexpr (R == 3) dft3<INV>(a[0], a[1], a[2]);
  else if constexpr (R == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<INV>(a);
  else if constexpr (R == 12) dft12<INV>(a);
  else if constexpr (R == 16) dft16<INV>(a);
  else static_assert(R == 1 || R == 3 || R == 4 || R == 8 || R == 12 || R == 16, "radix not built");
}

// Stage-0 twiddles of butterfly n1 (< M): a[k] *= w^k (forward) or conj(w)^k
// (inverse) for k = 1..R-1, w = exp(-2 pi i n1 / L), read from the transposed
// table twT[k M + n1] = exp(-2 pi i n1 k / L) (L = R M entries). Threads with
// consecutive n1 read consecutive slots, threads with equal n1 the same slot.
template <int R, int M, bool INV, typename V>
__device__ __forceinline__ void stage_twiddle(V* a, const V* twT, int n1) {
#pragma unroll
  for (int k = 1; k < R; ++k) a[k] = INV ? cmulconj(a[k], twT[k * M + n1]) : cmul(a[k], twT[k * M + n1]);
}

// As stage_twiddle, with the powers of w = twT[M + n1] built by repeated
// multiplication in registers (one table read; a relative error of a few
// 1e-16 in FP64): for FP64 butterflies whose table reads would otherwise all
// be held in registers at once.
template <int R, int M, bool INV, typename V>
__device__ __forceinline__ void stage_twiddle_pow(V* a, const V* twT, int n1) {
  const V w = twT[M + n1];
  V wk = w;
#pragma unroll
  for (int k = 1; k < R; ++k) {
    a[k] = INV ? cmulconj(a[k], wk) : cmul(a[k], wk);
    if (k + 1 < R) wk = cmul(wk, w);
  }
}

// Fill twT[k M + n1] = tw[n1 k] from the natural L-point table tw (k < R, n1 < M).
template <int R, int M, typename V, int NT>
__device__ __forceinline__ void fill_stage_table(V* twT, const V* tw, int tid) {
  for (int i = tid; i < R * M; i += NT) twT[i] = tw[(i % M) * (i / M)];
}

}  // namespace pat
