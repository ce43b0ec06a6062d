// Line propagator for gfx950: one kernel launch per time step runs every line
// of all three field components (see line_common.hpp for the scheme of
// Sec. 4.3 in mixed spaces, the layouts and the hub).
//
// A block of 128 threads (two waves) owns a tile of 16 lines of one axis. Each
// 1D transform of length N = R0 M is the two-stage split of fft_radix.hpp; a
// thread owns one stage-0 butterfly (R0 values at points n1 + M m of one line)
// or two stage-1 butterflies (M values at positions M mb + k1, frequency
// mb + R0 k1), with all values FP64 in registers, and the tile T in LDS is the
// exchange between the stages ([point][line], 16 lines per row). The time step
// of a component is inverse - update - forward - multiply - inverse - update -
// forward: four transforms and four LDS crossings; the updates run in the
// stage-0 layout, where a thread holds natural points, and the multipliers in
// the stage-1 layout, where it holds frequencies. HBM traffic per component and
// step: the hub (three component spectra, summed in FP64), both states in and
// out, and the output spectrum, each 8 (N/2+1) N^2 bytes.
#include "fft_radix.hpp"
#include "kspace.hpp"
#include "line_common.hpp"

namespace pat {

constexpr int kLT = 16;          // lines per tile
constexpr int kThreadsL = 128;   // threads per tile block

template <int N>
struct LD {
  static constexpr int H = N / 2, NK = H + 1;
  static constexpr int R0 = fft_radix(N, 0), M = N / R0;
  static constexpr int NL = NK * N;                                // lines per axis
  static constexpr int NTILE = NL / kLT;
  static constexpr int N0 = kLT * M, I0 = cdiv(N0, kThreadsL);    // stage-0 butterflies per tile
  static constexpr int N1 = kLT * R0, I1 = cdiv(N1, kThreadsL);   // stage-1 butterflies per tile
  static_assert(N % kLT == 0 && NL % kLT == 0, "a tile is 16 lines");
};

template <int N>
struct LineLds {
  double2 T[N * kLT];   // value of tile line l at point (or position) j: T[j * 16 + l]
};

// hub index of (kz, kx, ky_pos)
template <int N>
__device__ __forceinline__ int hidx(int kz, int kx, int kyp) {
  return (kz * LD<N>::NK + kx) * N + kyp;
}

// The fixed coordinates of a line and the part of the squared sinc argument
// that they contribute.
//   x lines (AX 0): lg = kz N + ky_pos, kz <= N/2 (the Hermitian half)
//   y lines (AX 1): lg = kz (N/2+1) + kx
//   z lines (AX 2): lg = kx N + ky_pos
template <int N, int AX>
struct LineGeo {
  int lg, kx, kyp, kz, kyn;   // kyn: ky_pos of -ky
  double s0;
  __device__ __forceinline__ LineGeo(int tile, int l, const LineTables& T) {
    using D = LD<N>;
    lg = tile * kLT + l;
    if (AX == 0) { kyp = lg % N; kz = lg / N; kx = 0; }
    else if (AX == 1) { kx = lg % D::NK; kz = lg / D::NK; kyp = 0; }
    else { kyp = lg % N; kx = lg / N; kz = 0; }
    const int kyf = fft_freq(N, kyp);
    kyn = fft_pos(N, (N - kyf) % N);
    double ha, hb;
    if (AX == 0) { ha = T.h[kyf]; hb = T.h[kz]; }
    else if (AX == 1) { ha = T.h[kx]; hb = T.h[kz]; }
    else { ha = T.h[kx]; hb = T.h[kyf]; }
    s0 = ha * ha + hb * hb;
  }
  // k-space correction at frequency f along the line
  __device__ __forceinline__ double kappa(const LineTables& T, int f) const {
    const double hf = T.h[f];
    return sinc_of_sq(s0 + hf * hf);
  }
};

// Sum of nh component spectra at frequency f (natural) / position p along the
// line. x lines read kx > N/2 as the conjugate at (-kx, -ky, -kz).
template <int N, int AX>
__device__ __forceinline__ double2 hub_sum(const float2* const* h, int nh, const LineGeo<N, AX>& g, int f, int p) {
  using D = LD<N>;
  int idx;
  bool cj = false;
  if (AX == 0) {
    if (f <= D::H) {
      idx = hidx<N>(g.kz, f, g.kyp);
    } else {
      idx = hidx<N>((N - g.kz) % N, N - f, g.kyn);
      cj = true;
    }
  } else if (AX == 1) {
    idx = hidx<N>(g.kz, g.kx, p);
  } else {
    idx = hidx<N>(f, g.kx, g.kyp);
  }
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < nh) {
      const float2 v = h[c][idx];
      s.x += v.x;
      s.y += v.y;
    }
  }
  if (cj) s.y = -s.y;
  return s;
}

// Adjoint source: the plane spectrum S[kx][ky_pos] of c0^2 y^n, the same for every kz.
template <int N, int AX>
__device__ __forceinline__ double2 src_val(const float2* S, const LineGeo<N, AX>& g, int f, int p) {
  using D = LD<N>;
  if (AX == 0) {
    if (f <= D::H) return widen<double2>(S[f * N + g.kyp]);
    const float2 v = S[(N - f) * N + g.kyn];
    return make_double2(v.x, -v.y);
  }
  if (AX == 1) return widen<double2>(S[g.kx * N + p]);
  return widen<double2>(S[g.kx * N + g.kyp]);
}

// Store the value of frequency f / position p of the line into a component
// spectrum. x lines with 0 < kz < N/2 also write the conjugate at
// (-kx, -ky, -kz) for kx = 0 or kx >= N/2, the half of the spectrum no x line owns.
template <int N, int AX>
__device__ __forceinline__ void hub_store(float2* out, const LineGeo<N, AX>& g, int f, int p, double2 v) {
  using D = LD<N>;
  if (AX == 0) {
    if (f <= D::H) out[hidx<N>(g.kz, f, g.kyp)] = narrow(v);
    if (g.kz >= 1 && g.kz < D::H && (f == 0 || f >= D::H))
      out[hidx<N>(N - g.kz, (N - f) % N, g.kyn)] = make_float2((float)v.x, (float)-v.y);
  } else if (AX == 1) {
    out[hidx<N>(g.kz, g.kx, p)] = narrow(v);
  } else {
    out[hidx<N>(f, g.kx, g.kyp)] = narrow(v);
  }
}

// Stage-0 twiddles w^(n1 k), k = 1..R-1, from w = tw[n1] by repeated multiplication.
template <int R, bool INV>
__device__ __forceinline__ void twiddle_pow(double2* a, double2 w) {
  double2 wk = w;
#pragma unroll
  for (int k = 1; k < R; ++k) {
    a[k] = INV ? cmulconj(a[k], wk) : cmul(a[k], wk);
    if (k + 1 < R) wk = cmul(wk, w);
  }
}

// Item decomposition of a tile: stage-0 item b -> line b % 16, butterfly n1 = b / 16;
// stage-1 item b -> line b % 16, block mb = b / 16.
template <int N>
struct S0Reg {
  double2 a[LD<N>::I0][LD<N>::R0];
};
template <int N>
struct S1Reg {
  double2 v[LD<N>::I1][LD<N>::M];
};

// stage-1 registers (after an inverse stage-1 DFT) -> T
template <int N>
__device__ __forceinline__ void s1_to_T(LineLds<N>& L, S1Reg<N>& r, int i, int l, int mb) {
  using D = LD<N>;
#pragma unroll
  for (int n1 = 0; n1 < D::M; ++n1) L.T[(D::M * mb + n1) * kLT + l] = r.v[i][n1];
}

// T -> stage-1 registers, forward stage-1 DFT
template <int N>
__device__ __forceinline__ void T_to_s1_fwd(const LineLds<N>& L, S1Reg<N>& r, int i, int l, int mb) {
  using D = LD<N>;
#pragma unroll
  for (int k1 = 0; k1 < D::M; ++k1) r.v[i][k1] = L.T[(D::M * mb + k1) * kLT + l];
  dft_r<D::M, false>(r.v[i]);
}

// T -> stage-0 registers, inverse stage 0 (natural points n1 + M m)
template <int N>
__device__ __forceinline__ void T_to_s0_inv(const LineLds<N>& L, S0Reg<N>& r, int i, int l, int n1,
                                            const LineTables& T) {
  using D = LD<N>;
#pragma unroll
  for (int m = 0; m < D::R0; ++m) r.a[i][m] = L.T[(n1 + D::M * m) * kLT + l];
  if constexpr (D::M > 1) twiddle_pow<D::R0, true>(r.a[i], T.tw[n1]);
  dft_r<D::R0, true>(r.a[i]);
}

// stage-0 registers (natural points) -> forward stage 0 -> T (the slots the
// same thread read in T_to_s0_inv, so no barrier is needed before it)
template <int N>
__device__ __forceinline__ void s0_fwd_to_T(LineLds<N>& L, S0Reg<N>& r, int i, int l, int n1, const LineTables& T) {
  using D = LD<N>;
  dft_r<D::R0, false>(r.a[i]);
  if constexpr (D::M > 1) twiddle_pow<D::R0, false>(r.a[i], T.tw[n1]);
#pragma unroll
  for (int k = 0; k < D::R0; ++k) L.T[(n1 + D::M * k) * kLT + l] = r.a[i][k];
}

enum LineMode { LM_FWD_INIT = 0, LM_FWD_STEP = 1, LM_ADJ_STEP = 2, LM_ADJ_FINAL = 3 };

struct LineStepArgs {
  const float2* hin[3];   // component spectra read and summed
  int nh;                 // how many of them (the others are zero)
  double hscale;          // factor of their sum
  const float2* src;      // adjoint: source plane spectrum added to the hub
  float2* hout[3];        // output component spectra
  float2* plane;          // forward step: plane spectrum of the hub read (z lines), or null
  int first;              // adjoint: states of the previous step are zero
};

// One tile of lines of axis AX.
template <int N, int AX, int MODE>
__device__ __forceinline__ void line_tile(LineLds<N>& L, const LineTables& T, const LineScalars& sc,
                                          const LineBuffers& B, const LineStepArgs& A, int tile, int tid) {
  using D = LD<N>;
  constexpr int R0 = D::R0, M = D::M;
  constexpr bool ADJ = MODE == LM_ADJ_STEP || MODE == LM_ADJ_FINAL;
  float2* su = B.su[AX];
  float2* sr = B.sr[AX];
  const float* pa = T.a[AX];
  const float* pb = T.b[AX];
  const bool want_plane = !ADJ && AX == 2 && A.plane != nullptr;
  S1Reg<N> s1;
  S0Reg<N> s0;
  double2 psum = make_double2(0.0, 0.0);

  // (A) the hub at the line's frequencies, times the first multiplier, inverse stage 1
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, AX> g(tile, l, T);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1, p = M * mb + k1;
        double2 P = hub_sum<N, AX>(A.hin, A.nh, g, f, p);
        P = cscale(P, A.hscale);
        if (ADJ) P = cadd(P, src_val<N, AX>(A.src, g, f, p));
        if (want_plane) psum = cadd(psum, P);
        if (MODE == LM_FWD_STEP) P = cscale(cmul(P, T.mp[f]), g.kappa(T, f) * sc.inv_n);
        else if (MODE == LM_FWD_INIT) P = cscale(P, sc.inv_n * sc.inv_3c2);
        else P = cscale(P, sc.inv_n);
        s1.v[i][k1] = P;
      }
      dft_r<M, true>(s1.v[i]);
      s1_to_T<N>(L, s1, i, l, mb);
    }
  }
  __syncthreads();

  if constexpr (MODE == LM_FWD_INIT) {
    // rho = F^-1 P / (3 c0^2), u = dt/(2 rho0) F^-1 [m+ P]
#pragma unroll
    for (int i = 0; i < D::I0; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N0) {
        const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
        T_to_s0_inv<N>(L, s0, i, l, n1, T);
#pragma unroll
        for (int m = 0; m < R0; ++m) sr[(n1 + M * m) * D::NL + lg] = narrow(s0.a[i][m]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N1) {
        const int l = b % kLT, mb = b / kLT;
        const LineGeo<N, AX> g(tile, l, T);
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          const int f = mb + R0 * k1, p = M * mb + k1;
          const double2 P = cscale(hub_sum<N, AX>(A.hin, A.nh, g, f, p), A.hscale);
          s1.v[i][k1] = cscale(cmul(P, T.mp[f]), g.kappa(T, f) * sc.inv_n * sc.half_dt_over_rho0);
        }
        dft_r<M, true>(s1.v[i]);
        s1_to_T<N>(L, s1, i, l, mb);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D::I0; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N0) {
        const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
        T_to_s0_inv<N>(L, s0, i, l, n1, T);
#pragma unroll
        for (int m = 0; m < R0; ++m) su[(n1 + M * m) * D::NL + lg] = narrow(s0.a[i][m]);
      }
    }
    return;
  }

  // (B) first update in the natural layout, forward stage 0
  //   forward: u <- a (a u - dt/rho0 g), transform u
  //   adjoint: rho^ <- b^2 rho^ + q, transform b rho^
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
      T_to_s0_inv<N>(L, s0, i, l, n1, T);
      if (!ADJ) {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int x = n1 + M * m, idx = x * D::NL + lg;
          const double af = pa[x];
          const double2 uo = widen<double2>(su[idx]);
          const double2 un = make_double2(af * (af * uo.x - sc.dt_over_rho0 * s0.a[i][m].x),
                                          af * (af * uo.y - sc.dt_over_rho0 * s0.a[i][m].y));
          su[idx] = narrow(un);
          s0.a[i][m] = un;
        }
      } else {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int x = n1 + M * m, idx = x * D::NL + lg;
          const double bf = pb[x];
          double2 rh = s0.a[i][m];
          if (!A.first) {
            const double2 ro = widen<double2>(sr[idx]);
            rh = make_double2(bf * bf * ro.x + rh.x, bf * bf * ro.y + rh.y);
          }
          if (MODE == LM_ADJ_STEP) {
            sr[idx] = narrow(rh);
            s0.a[i][m] = cscale(rh, bf);
          } else {
            s0.a[i][m] = cscale(rh, sc.inv_3c2);
          }
        }
      }
      s0_fwd_to_T<N>(L, s0, i, l, n1, T);
    }
  }
  __syncthreads();

  if constexpr (MODE == LM_ADJ_FINAL) {
    // out = F(rho^) / (3 c0^2) - dt/(2 rho0) m- F(v)
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N1) {
        const int l = b % kLT, mb = b / kLT;
        T_to_s1_fwd<N>(L, s1, i, l, mb);
      }
    }
    if (!A.first) {
      S1Reg<N> w;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < D::I0; ++i) {
        const int b = tid + i * kThreadsL;
        if (b < D::N0) {
          const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
#pragma unroll
          for (int m = 0; m < R0; ++m) s0.a[i][m] = widen<double2>(su[(n1 + M * m) * D::NL + lg]);
          s0_fwd_to_T<N>(L, s0, i, l, n1, T);
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < D::I1; ++i) {
        const int b = tid + i * kThreadsL;
        if (b < D::N1) {
          const int l = b % kLT, mb = b / kLT;
          const LineGeo<N, AX> g(tile, l, T);
          T_to_s1_fwd<N>(L, w, i, l, mb);
#pragma unroll
          for (int k1 = 0; k1 < M; ++k1) {
            const int f = mb + R0 * k1;
            const double2 t = cscale(cmul(w.v[i][k1], T.mm[f]), g.kappa(T, f) * sc.half_dt_over_rho0);
            s1.v[i][k1] = csub(s1.v[i][k1], t);
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N1) {
        const int l = b % kLT, mb = b / kLT;
        const LineGeo<N, AX> g(tile, l, T);
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) hub_store<N, AX>(A.hout[AX], g, mb + R0 * k1, M * mb + k1, s1.v[i][k1]);
      }
    }
    return;
  }

  // (C) forward stage 1, middle multiplier (forward m-, adjoint m+), inverse stage 1
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, AX> g(tile, l, T);
      T_to_s1_fwd<N>(L, s1, i, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1;
        s1.v[i][k1] = cscale(cmul(s1.v[i][k1], ADJ ? T.mp[f] : T.mm[f]), g.kappa(T, f) * sc.inv_n);
      }
      dft_r<M, true>(s1.v[i]);
      s1_to_T<N>(L, s1, i, l, mb);
    }
  }
  __syncthreads();

  // (D) second update, forward stage 0
  //   forward: rho <- b (b rho - dt rho0 h), transform rho
  //   adjoint: uh = v + dt rho0 t, v <- a^2 uh, transform a uh
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
      T_to_s0_inv<N>(L, s0, i, l, n1, T);
      if (!ADJ) {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int x = n1 + M * m, idx = x * D::NL + lg;
          const double bf = pb[x];
          const double2 ro = widen<double2>(sr[idx]);
          const double2 rn = make_double2(bf * (bf * ro.x - sc.dt_rho0 * s0.a[i][m].x),
                                          bf * (bf * ro.y - sc.dt_rho0 * s0.a[i][m].y));
          sr[idx] = narrow(rn);
          s0.a[i][m] = rn;
        }
      } else {
#pragma unroll
        for (int m = 0; m < R0; ++m) {
          const int x = n1 + M * m, idx = x * D::NL + lg;
          const double af = pa[x];
          double2 uh = cscale(s0.a[i][m], sc.dt_rho0);
          if (!A.first) uh = cadd(uh, widen<double2>(su[idx]));
          su[idx] = narrow(cscale(uh, af * af));
          s0.a[i][m] = cscale(uh, af);
        }
      }
      s0_fwd_to_T<N>(L, s0, i, l, n1, T);
    }
  }
  __syncthreads();

  // (E) forward stage 1 and the output spectrum (adjoint: times m-)
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, AX> g(tile, l, T);
      T_to_s1_fwd<N>(L, s1, i, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1, p = M * mb + k1;
        double2 o = s1.v[i][k1];
        if (ADJ) o = cscale(cmul(o, T.mm[f]), g.kappa(T, f));
        hub_store<N, AX>(A.hout[AX], g, f, p, o);
      }
    }
  }

  if (want_plane) {   // sum over kz of the hub read: the plane z = 0 of the pressure, / N^3
    __syncthreads();
    L.T[tid] = psum;
    __syncthreads();
    if (tid < kLT) {
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < kThreadsL / kLT; ++j) s = cadd(s, L.T[tid + kLT * j]);
      A.plane[tile * kLT + tid] = narrow(cscale(s, sc.inv_ntot));
    }
  }
}

template <int N, int MODE>
__global__ __launch_bounds__(kThreadsL) void k_line(LineTables T, LineScalars sc, LineBuffers B, LineStepArgs A) {
  __shared__ LineLds<N> L;
  const int tile = blockIdx.x, tid = threadIdx.x;
  if (blockIdx.y == 0) line_tile<N, 0, MODE>(L, T, sc, B, A, tile, tid);
  else if (blockIdx.y == 1) line_tile<N, 1, MODE>(L, T, sc, B, A, tile, tid);
  else line_tile<N, 2, MODE>(L, T, sc, B, A, tile, tid);
}

// Slab spectrum [z][kx][ky_pos] (z lines: [point][line]) -> z transform ->
// component spectrum hub[kz][kx][ky_pos], times scale.
template <int N>
__global__ __launch_bounds__(kThreadsL) void k_line_zfwd(LineTables T, const float2* __restrict__ spec, float2* hub,
                                                         double scale) {
  using D = LD<N>;
  __shared__ LineLds<N> L;
  const int tile = blockIdx.x, tid = threadIdx.x;
  S0Reg<N> s0;
  S1Reg<N> s1;
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
#pragma unroll
      for (int m = 0; m < D::R0; ++m) s0.a[i][m] = widen<double2>(spec[(n1 + D::M * m) * D::NL + lg]);
      s0_fwd_to_T<N>(L, s0, i, l, n1, T);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, 2> g(tile, l, T);
      T_to_s1_fwd<N>(L, s1, i, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < D::M; ++k1)
        hub_store<N, 2>(hub, g, mb + D::R0 * k1, D::M * mb + k1, cscale(s1.v[i][k1], scale));
    }
  }
}

// Sum of three component spectra -> inverse z transform times scale -> slab
// spectrum [z][kx][ky_pos].
template <int N>
__global__ __launch_bounds__(kThreadsL) void k_line_zinv(LineTables T, const float2* h0, const float2* h1,
                                                         const float2* h2, float2* spec, double scale) {
  using D = LD<N>;
  __shared__ LineLds<N> L;
  const int tile = blockIdx.x, tid = threadIdx.x;
  const float2* hs[3] = {h0, h1, h2};
  S0Reg<N> s0;
  S1Reg<N> s1;
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, 2> g(tile, l, T);
#pragma unroll
      for (int k1 = 0; k1 < D::M; ++k1)
        s1.v[i][k1] = cscale(hub_sum<N, 2>(hs, 3, g, mb + D::R0 * k1, D::M * mb + k1), scale);
      dft_r<D::M, true>(s1.v[i]);
      s1_to_T<N>(L, s1, i, l, mb);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
      T_to_s0_inv<N>(L, s0, i, l, n1, T);
#pragma unroll
      for (int m = 0; m < D::R0; ++m) spec[(n1 + D::M * m) * D::NL + lg] = narrow(s0.a[i][m]);
    }
  }
}

// Plane spectrum of the hub: plane[kx][ky_pos] = scale * sum_kz sum_c h_c.
template <int N>
__global__ __launch_bounds__(kThreadsL) void k_line_plane(const float2* h0, const float2* h1, const float2* h2,
                                                          int nh, float2* plane, double scale) {
  using D = LD<N>;
  const int lg = blockIdx.x * kThreadsL + threadIdx.x;   // kx N + ky_pos
  if (lg >= D::NL) return;
  double2 s = make_double2(0.0, 0.0);
  for (int kz = 0; kz < N; ++kz) {
    const size_t idx = (size_t)kz * D::NL + lg;
    const float2 a = h0[idx];
    s.x += a.x;
    s.y += a.y;
    if (nh > 1) {
      const float2 b = h1[idx], c = h2[idx];
      s.x += b.x + c.x;
      s.y += b.y + c.y;
    }
  }
  plane[lg] = narrow(cscale(s, scale));
}

// ---- launch sequences ------------------------------------------------------------

template <int N>
hipError_t line_forward(const LineTables& T, const LineScalars& sc, const LineBuffers& B, const WaveTables& wt,
                        const float* p0, float* planes_real, int nt, hipStream_t st, KernelTimer* kt) {
  using D = LD<N>;
  hipError_t e = launch_slab_r2c(N, p0, B.spec, N, 1.0f, wt, st);
  if (e != hipSuccess) return e;
  k_line_zfwd<N><<<D::NTILE, kThreadsL, 0, st>>>(T, B.spec, B.hub[0][0], 1.0 / sc.c2);
  LineStepArgs A{};
  A.hin[0] = B.hub[0][0];
  A.nh = 1;
  A.hscale = sc.c2;
  if (nt > 1) k_line<N, LM_FWD_INIT><<<dim3(D::NTILE, 3), kThreadsL, 0, st>>>(T, sc, B, A);
  for (int n = 0; n + 1 < nt; ++n) {
    const int cur = n & 1;
    for (int c = 0; c < 3; ++c) {
      A.hin[c] = B.hub[cur][c];
      A.hout[c] = B.hub[cur ^ 1][c];
    }
    A.nh = n == 0 ? 1 : 3;
    A.plane = B.planes + (size_t)n * D::NL;
    timed(kt, K_LINE_FWD, st, [&] {
      k_line<N, LM_FWD_STEP><<<dim3(D::NTILE, 3), kThreadsL, 0, st>>>(T, sc, B, A);
    });
  }
  const int last = (nt - 1) & 1;
  k_line_plane<N><<<cdiv(D::NL, kThreadsL), kThreadsL, 0, st>>>(B.hub[last][0], B.hub[last][1], B.hub[last][2],
                                                                nt == 1 ? 1 : 3,
                                                                B.planes + (size_t)(nt - 1) * D::NL,
                                                                sc.c2 * sc.inv_ntot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_slab_c2r(N, B.planes, planes_real, nt, 1.0f, wt, st);
}

template <int N>
hipError_t line_adjoint(const LineTables& T, const LineScalars& sc, const LineBuffers& B, const WaveTables& wt,
                        const float* planes_real, float* p, int nt, hipStream_t st, KernelTimer* kt) {
  using D = LD<N>;
  hipError_t e = launch_slab_r2c(N, planes_real, B.planes, nt, (float)sc.c2, wt, st);
  if (e != hipSuccess) return e;
  LineStepArgs A{};
  A.hscale = sc.adj_scale;
  int cur = 0;
  for (int j = 0; j + 1 < nt; ++j) {   // iteration of time index n = nt - 2 - j
    const int n = nt - 2 - j;
    cur = j & 1;
    for (int c = 0; c < 3; ++c) {
      A.hin[c] = B.hub[cur][c];
      A.hout[c] = B.hub[cur ^ 1][c];
    }
    A.nh = j == 0 ? 0 : 3;
    A.first = j == 0;
    A.src = B.planes + (size_t)(n + 1) * D::NL;
    timed(kt, K_LINE_ADJ, st, [&] {
      k_line<N, LM_ADJ_STEP><<<dim3(D::NTILE, 3), kThreadsL, 0, st>>>(T, sc, B, A);
    });
  }
  cur = (nt - 1) & 1;
  for (int c = 0; c < 3; ++c) {
    A.hin[c] = B.hub[cur][c];
    A.hout[c] = B.hub[cur ^ 1][c];
  }
  A.nh = nt == 1 ? 0 : 3;
  A.first = nt == 1;
  A.src = B.planes;
  k_line<N, LM_ADJ_FINAL><<<dim3(D::NTILE, 3), kThreadsL, 0, st>>>(T, sc, B, A);
  k_line_zinv<N><<<D::NTILE, kThreadsL, 0, st>>>(T, B.hub[cur ^ 1][0], B.hub[cur ^ 1][1], B.hub[cur ^ 1][2], B.spec,
                                                 sc.inv_ntot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_slab_c2r(N, B.spec, p, N, 1.0f, wt, st);
}

#define PAT_LINE_IMPL(N) {N, &line_forward<N>, &line_adjoint<N>}

static const LineImpl kLineImpls[] = {
    PAT_LINE_IMPL(16),
    PAT_LINE_IMPL(32),
    PAT_LINE_IMPL(64),
    PAT_LINE_IMPL(128),
};

const LineImpl* find_line_impl(int nx, int ny, int nz) {
  if (nx != ny || ny != nz) return nullptr;
  for (const auto& w : kLineImpls)
    if (w.n == nx) return &w;
  return nullptr;
}

}  // namespace pat
