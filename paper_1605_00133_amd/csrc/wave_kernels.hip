// k-space pseudospectral propagation of the acoustic initial-value problem
// (eq. PATfwd) and its exact transpose, on gfx950.
//
// Scheme (Sec. 4.3; the k-space PSTD method the paper cites), per time step:
//   u_xi   <- a_xi (a_xi u_xi   - dt/rho0 Dplus_xi p)         xi = x, y, z
//   rho_xi <- b_xi (b_xi rho_xi - dt rho0 Dminus_xi u_xi)
//   p       = c0^2 (rho_x + rho_y + rho_z);  record p on the plane z = 0
// with Dplus/Dminus_xi = IFFT[ i k_xi exp(+-i k_xi dx/2) sinc(c0 dt |k|/2) FFT[.] ]
// and PML factors a (staggered), b (collocated).
//
// Every 3D FFT is done in two global passes:
//   slab kernels (one workgroup per z-slab, 256 threads): 2D real<->complex
//     transform of the slab in LDS (x: packed half-length complex FFT plus
//     real-FFT post-processing; y: column FFT), fused with the real-space
//     update of the state fields;
//   pencil kernels (one workgroup per 16 ky columns of one kx, all z): z
//     transform in LDS, the k-space multipliers, inverse z transform.
// Slab spectra live in HBM as [z][kx][ky_pos] (kx = 0..nx/2 natural, ky in
// digit-reversed position order), so pencil tiles read 128-byte rows and no
// kernel ever permutes data.
//
// Forward step = pencil(grad: 1 in, 2 out) -> slab(u: per component) ->
// pencil(div: per component) -> slab(rho, p, sensor plane, R2C of p).
// Adjoint step = pencil(grad of b*rho^: per component) -> slab(u^, R2C of a*u^)
// -> pencil(sum of the three divergences: 3 in, 1 out) -> slab(rho^ + source).
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "wave_common.hpp"

namespace pat {

constexpr int kThreadsXY = 256;
constexpr int kThreadsZ = 128;

template <int NX, int NY, int NZ>
struct Dims {
  static constexpr int MX = NX / 2;          // complex length of a packed real row
  static constexpr int NKX = MX + 1;         // half-spectrum length
  static constexpr int PITCH = NKX;          // LDS row pitch (complex), odd
  static constexpr int SLAB_C = NKX * NY;    // complex values per slab spectrum
  static constexpr int SLAB_P = NY * MX;     // float2 pairs per real slab
  static constexpr int TY = NY >= 16 ? 16 : NY;
  static constexpr int NTILE = NKX * (NY / TY);
  static constexpr int EPT = (SLAB_P + kThreadsXY - 1) / kThreadsXY;
};

// ---- slab transforms -------------------------------------------------------

// R2C post-processing of rows already transformed by a forward MX-point FFT:
// row y holds Z[k] (Z = FFT of x[2n] + i x[2n+1]) at digit-reversed positions;
// on exit it holds X[k], k = 0..MX, in natural order (X = real FFT of x).
template <int NX, int NY, int NZ>
__device__ __forceinline__ void r2c_post(float2* S, const float2* __restrict__ tw_nx, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int MX = D::MX, NP = MX / 2 + 1, TOTAL = NY * NP;
  constexpr int IT = (TOTAL + kThreadsXY - 1) / kThreadsXY;
  float2 o1[IT], o2[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = tid + i * kThreadsXY;
    if (w < TOTAL) {
      const int y = w / NP, k = w % NP;
      const float2* row = S + y * D::PITCH;
      if (k == 0) {
        const float2 z0 = row[0];
        o1[i] = make_float2(z0.x + z0.y, 0.f);
        o2[i] = make_float2(z0.x - z0.y, 0.f);
      } else {
        const float2 A = row[fft_pos(MX, k)];
        const float2 B = cconj(row[fft_pos(MX, MX - k)]);
        const float2 E = cscale(cadd(A, B), 0.5f);
        const float2 Dd = csub(A, B);
        const float2 O = make_float2(0.5f * Dd.y, -0.5f * Dd.x);   // (A - B) / (2i)
        const float2 WO = cmul(tw_nx[k], O);
        o1[i] = cadd(E, WO);
        o2[i] = cconj(csub(E, WO));
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = tid + i * kThreadsXY;
    if (w < TOTAL) {
      const int y = w / NP, k = w % NP;
      float2* row = S + y * D::PITCH;
      row[k] = o1[i];
      row[MX - k] = o2[i];   // k == 0 writes X[MX]; k == MX/2 rewrites the same value
    }
  }
  __syncthreads();
}

// C2R pre-processing: row y holds X[k], k = 0..MX natural; on exit it holds
// Z'[k] = (X[k] + conj X[MX-k]) + i exp(+2 pi i k/NX) (X[k] - conj X[MX-k]) at
// digit-reversed positions, so that an inverse MX-point FFT yields
// x[2n] + i x[2n+1] (unnormalised real inverse transform).
template <int NX, int NY, int NZ>
__device__ __forceinline__ void c2r_pre(float2* S, const float2* __restrict__ tw_nx, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int MX = D::MX, NP = MX / 2 + 1, TOTAL = NY * NP;
  constexpr int IT = (TOTAL + kThreadsXY - 1) / kThreadsXY;
  float2 o1[IT], o2[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = tid + i * kThreadsXY;
    if (w < TOTAL) {
      const int y = w / NP, k = w % NP;
      const float2* row = S + y * D::PITCH;
      const float2 Xk = row[k], Xm = row[MX - k];
      {
        const float2 s = cadd(Xk, cconj(Xm)), d = csub(Xk, cconj(Xm));
        const float2 wd = cmulconj(d, tw_nx[k]);
        o1[i] = make_float2(s.x - wd.y, s.y + wd.x);
      }
      {
        const float2 s = cadd(Xm, cconj(Xk)), d = csub(Xm, cconj(Xk));
        const float2 wd = cmulconj(d, tw_nx[MX - k]);
        o2[i] = make_float2(s.x - wd.y, s.y + wd.x);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int w = tid + i * kThreadsXY;
    if (w < TOTAL) {
      const int y = w / NP, k = w % NP;
      float2* row = S + y * D::PITCH;
      row[fft_pos(MX, k)] = o1[i];
      if (k != 0 && 2 * k != MX) row[fft_pos(MX, MX - k)] = o2[i];
    }
  }
  __syncthreads();
}

// Real slab (packed pairs at S[y*PITCH + n]) -> slab spectrum (kx natural,
// ky digit-reversed) in place. Caller syncs before.
template <int NX, int NY, int NZ>
__device__ __forceinline__ void slab_r2c(float2* S, const WaveTables& t, int tid) {
  using D = Dims<NX, NY, NZ>;
  fft_forward<D::MX, false>(S, NY, D::PITCH, 1, t.tw_mx, tid, kThreadsXY);
  r2c_post<NX, NY, NZ>(S, t.tw_nx, tid);
  fft_forward<NY, true>(S, D::NKX, 1, D::PITCH, t.tw_y, tid, kThreadsXY);
}

// Slab spectrum -> real slab (packed pairs), unnormalised. Caller syncs before.
template <int NX, int NY, int NZ>
__device__ __forceinline__ void slab_c2r(float2* S, const WaveTables& t, int tid) {
  using D = Dims<NX, NY, NZ>;
  fft_inverse<NY, true>(S, D::NKX, 1, D::PITCH, t.tw_y, tid, kThreadsXY);
  c2r_pre<NX, NY, NZ>(S, t.tw_nx, tid);
  fft_inverse<D::MX, false>(S, NY, D::PITCH, 1, t.tw_mx, tid, kThreadsXY);
}

// Global slab spectrum [kx][ky_pos] -> LDS [ky_pos][kx], times mult (0: none,
// 1: per-kx table, 2: per-ky_pos table).
template <int NX, int NY, int NZ>
__device__ __forceinline__ void load_spec(float2* S, const float2* __restrict__ g, int mode,
                                          const float2* __restrict__ mult, int tid) {
  using D = Dims<NX, NY, NZ>;
  for (int e = tid; e < D::SLAB_C; e += kThreadsXY) {
    const int kx = e / NY, p = e % NY;
    float2 v = g[e];
    if (mode == 1) v = cmul(v, mult[kx]);
    else if (mode == 2) v = cmul(v, mult[p]);
    S[p * D::PITCH + kx] = v;
  }
}

template <int NX, int NY, int NZ>
__device__ __forceinline__ void store_spec(const float2* S, float2* __restrict__ g, int tid) {
  using D = Dims<NX, NY, NZ>;
  for (int e = tid; e < D::SLAB_C; e += kThreadsXY) {
    const int kx = e / NY, p = e % NY;
    g[e] = S[p * D::PITCH + kx];
  }
}

// blockIdx -> (slab z, component xi) so the three components of one slab run on
// the same XCD (block ids congruent mod 8), sharing that XCD's L2.
template <int NZ>
__device__ __forceinline__ void slab_field_of_block(int b, int& z, int& xi) {
  const int grp = b / 24, r = b % 24;
  xi = r / 8;
  z = grp * 8 + (r % 8);
}

// ---- forward kernels ---------------------------------------------------------

// rho_xi = p0 / (3 c0^2); plane 0 = p0[z = 0]; spec0 = slab R2C of p0.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_fwd_init(const float* __restrict__ p0, WaveBuffers B,
                                                         float* __restrict__ plane0, WaveTables t,
                                                         WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t off = (size_t)z * D::SLAB_P;
  const float2* src = reinterpret_cast<const float2*>(p0) + off;
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int y = e / D::MX, n = e % D::MX;
    const float2 v = src[e];
    S[y * D::PITCH + n] = v;
    const float2 r = cscale(v, sc.inv_3c2);
#pragma unroll
    for (int xi = 0; xi < 3; ++xi) reinterpret_cast<float2*>(B.rho[xi])[off + e] = r;
    if (z == 0) reinterpret_cast<float2*>(plane0)[e] = v;
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  store_spec<NX, NY, NZ>(S, B.spec[0] + (size_t)z * D::SLAB_C, tid);
}

// Pencil pass of the gradient: in = FFT_xy(p) (overwritten by Q), out2 = Gz, with
// Q = IFFT_z[kappa FFT_z(in)] / N and Gz = IFFT_z[kappa i kz e^{i kz dx/2} FFT_z(in)] / N.
// The x and y derivative factors are applied later in the slab kernel (they
// depend only on kx or ky_pos), so one input yields two outputs instead of three.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsZ) void k_zgrad(float2* __restrict__ P, float2* __restrict__ Gz,
                                                     WaveTables t, float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  constexpr int TY = D::TY, W = 2 * TY;
  __shared__ float2 T[NZ * W];
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int z = e / TY, j = e % TY;
    T[z * W + j] = P[((size_t)z * D::NKX + kx) * NY + p0 + j];
  }
  __syncthreads();
  fft_forward<NZ, true>(T, TY, 1, W, t.tw_z, tid, kThreadsZ);
  const float hx = t.hx[kx];
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int q = e / TY, j = e % TY;
    const float hy = t.hy[p0 + j], hz = t.hz[q];
    const float h = sqrtf(hx * hx + hy * hy + hz * hz);
    const float kap = (h > 0.f ? sinf(h) / h : 1.f) * inv_ntot;
    const float2 v = cscale(T[q * W + j], kap);
    T[q * W + j] = v;
    T[q * W + TY + j] = cmul(v, t.mpz[q]);
  }
  __syncthreads();
  fft_inverse<NZ, true>(T, W, 1, W, t.tw_z, tid, kThreadsZ);
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int z = e / TY, j = e % TY;
    const size_t gi = ((size_t)z * D::NKX + kx) * NY + p0 + j;
    P[gi] = T[z * W + j];
    Gz[gi] = T[z * W + TY + j];
  }
}

// Pencil pass applying kappa/N times i k_xi exp(s i k_xi dx/2) (PLUS: s = +1,
// else -1) to component xi = blockIdx.y, in place.
template <int NX, int NY, int NZ, bool PLUS>
__global__ __launch_bounds__(kThreadsZ) void k_zmul(float2* H0, float2* H1, float2* H2, WaveTables t,
                                                    float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  constexpr int TY = D::TY;
  __shared__ float2 T[NZ * TY];
  const int tid = threadIdx.x, xi = blockIdx.y;
  float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int z = e / TY, j = e % TY;
    T[e] = H[((size_t)z * D::NKX + kx) * NY + p0 + j];
  }
  __syncthreads();
  fft_forward<NZ, true>(T, TY, 1, TY, t.tw_z, tid, kThreadsZ);
  const float hx = t.hx[kx];
  const float2* mx = PLUS ? t.mpx : t.mmx;
  const float2* my = PLUS ? t.mpy : t.mmy;
  const float2* mz = PLUS ? t.mpz : t.mmz;
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int q = e / TY, j = e % TY;
    const float hy = t.hy[p0 + j], hz = t.hz[q];
    const float h = sqrtf(hx * hx + hy * hy + hz * hz);
    const float kap = (h > 0.f ? sinf(h) / h : 1.f) * inv_ntot;
    const float2 m = xi == 0 ? mx[kx] : (xi == 1 ? my[p0 + j] : mz[q]);
    T[e] = cmul(cscale(T[e], kap), m);
  }
  __syncthreads();
  fft_inverse<NZ, true>(T, TY, 1, TY, t.tw_z, tid, kThreadsZ);
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int z = e / TY, j = e % TY;
    H[((size_t)z * D::NKX + kx) * NY + p0 + j] = T[e];
  }
}

// Velocity update of component xi for slab z, then R2C of the new u_xi.
// Q, Gz: outputs of k_zgrad; U0, U1, U2: spectra of the new u components
// (U2 aliases Gz: only this block reads Gz[z] and it does so before writing).
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_fwd_u(const float2* __restrict__ Q, const float2* Gz,
                                                      float2* U0, float2* U1, float2* U2, WaveBuffers B,
                                                      WaveTables t, WaveScalars sc, int init) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block<NZ>(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C;
  if (xi == 0) load_spec<NX, NY, NZ>(S, Q + cz, 1, t.mpx, tid);
  else if (xi == 1) load_spec<NX, NY, NZ>(S, Q + cz, 2, t.mpy, tid);
  else load_spec<NX, NY, NZ>(S, Gz + cz, 0, nullptr, tid);
  __syncthreads();
  slab_c2r<NX, NY, NZ>(S, t, tid);
  float2* u = reinterpret_cast<float2*>(B.u[xi]) + (size_t)z * D::SLAB_P;
  const float azz = t.az[z];
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int y = e / D::MX, n = e % D::MX;
    const float2 g = S[y * D::PITCH + n];
    float a0, a1;
    if (xi == 0) { a0 = t.ax[2 * n]; a1 = t.ax[2 * n + 1]; }
    else if (xi == 1) { a0 = a1 = t.ay[y]; }
    else { a0 = a1 = azz; }
    const float2 uo = init ? cscale(g, sc.half_dt_over_rho0) : u[e];
    const float2 un = make_float2(a0 * (a0 * uo.x - sc.dt_over_rho0 * g.x),
                                  a1 * (a1 * uo.y - sc.dt_over_rho0 * g.y));
    u[e] = un;
    S[y * D::PITCH + n] = un;
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  float2* U = xi == 0 ? U0 : (xi == 1 ? U1 : U2);
  store_spec<NX, NY, NZ>(S, U + cz, tid);
}

// Density update of all three components of slab z, p = c0^2 sum rho, sensor
// plane, and R2C of p into Pout.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_fwd_rho(const float2* __restrict__ H0,
                                                        const float2* __restrict__ H1,
                                                        const float2* __restrict__ H2, WaveBuffers B,
                                                        float2* __restrict__ Pout, float* __restrict__ plane,
                                                        WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  float2 pacc[D::EPT];
#pragma unroll
  for (int i = 0; i < D::EPT; ++i) pacc[i] = make_float2(0.f, 0.f);
  for (int xi = 0; xi < 3; ++xi) {
    const float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
    load_spec<NX, NY, NZ>(S, H + cz, 0, nullptr, tid);
    __syncthreads();
    slab_c2r<NX, NY, NZ>(S, t, tid);
    float2* r = reinterpret_cast<float2*>(B.rho[xi]) + rz;
    const float bzz = t.bz[z];
#pragma unroll
    for (int i = 0; i < D::EPT; ++i) {
      const int e = tid + i * kThreadsXY;
      if (e < D::SLAB_P) {
        const int y = e / D::MX, n = e % D::MX;
        const float2 h = S[y * D::PITCH + n];
        float b0, b1;
        if (xi == 0) { b0 = t.bx[2 * n]; b1 = t.bx[2 * n + 1]; }
        else if (xi == 1) { b0 = b1 = t.by[y]; }
        else { b0 = b1 = bzz; }
        const float2 ro = r[e];
        const float2 rn = make_float2(b0 * (b0 * ro.x - sc.dt_rho0 * h.x), b1 * (b1 * ro.y - sc.dt_rho0 * h.y));
        r[e] = rn;
        pacc[i] = cadd(pacc[i], rn);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < D::EPT; ++i) {
    const int e = tid + i * kThreadsXY;
    if (e < D::SLAB_P) {
      const int y = e / D::MX, n = e % D::MX;
      const float2 p = cscale(pacc[i], sc.c2);
      S[y * D::PITCH + n] = p;
      if (z == 0) reinterpret_cast<float2*>(plane)[e] = p;
    }
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  store_spec<NX, NY, NZ>(S, Pout + cz, tid);
}

// ---- adjoint kernels ---------------------------------------------------------

// rho^_xi = c0^2 S^T y^{nt-1}, u^_xi = 0, W_xi = R2C(b_xi rho^_xi).
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_adj_init(const float* __restrict__ ylast, WaveBuffers B,
                                                         WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block<NZ>(blockIdx.x, z, xi);
  const size_t rz = (size_t)z * D::SLAB_P, cz = (size_t)z * D::SLAB_C;
  float2* rb = reinterpret_cast<float2*>(B.rho[xi]) + rz;
  float2* ub = reinterpret_cast<float2*>(B.u[xi]) + rz;
  const float2 zero = make_float2(0.f, 0.f);
  if (z != 0) {
    for (int e = tid; e < D::SLAB_P; e += kThreadsXY) { rb[e] = zero; ub[e] = zero; }
    for (int e = tid; e < D::SLAB_C; e += kThreadsXY) B.spec[xi][cz + e] = zero;
    return;
  }
  const float2* y = reinterpret_cast<const float2*>(ylast);
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int yy = e / D::MX, n = e % D::MX;
    const float2 r = cscale(y[e], sc.c2);
    rb[e] = r;
    ub[e] = zero;
    float b0, b1;
    if (xi == 0) { b0 = t.bx[2 * n]; b1 = t.bx[2 * n + 1]; }
    else if (xi == 1) { b0 = b1 = t.by[yy]; }
    else { b0 = b1 = t.bz[0]; }
    S[yy * D::PITCH + n] = make_float2(b0 * r.x, b1 * r.y);
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  store_spec<NX, NY, NZ>(S, B.spec[xi] + cz, tid);
}

// u^_xi: uh = u^ + dt rho0 Dplus_xi(b rho^) (the pencil pass already applied the
// multiplier), u^ <- a^2 uh, W_xi = R2C(a uh) in place.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_adj_u(WaveBuffers B, WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block<NZ>(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C;
  load_spec<NX, NY, NZ>(S, B.spec[xi] + cz, 0, nullptr, tid);
  __syncthreads();
  slab_c2r<NX, NY, NZ>(S, t, tid);
  float2* ub = reinterpret_cast<float2*>(B.u[xi]) + (size_t)z * D::SLAB_P;
  const float azz = t.az[z];
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int y = e / D::MX, n = e % D::MX;
    const float2 g = S[y * D::PITCH + n];
    float a0, a1;
    if (xi == 0) { a0 = t.ax[2 * n]; a1 = t.ax[2 * n + 1]; }
    else if (xi == 1) { a0 = a1 = t.ay[y]; }
    else { a0 = a1 = azz; }
    const float2 uo = ub[e];
    const float2 uh = make_float2(uo.x + sc.dt_rho0 * g.x, uo.y + sc.dt_rho0 * g.y);
    ub[e] = make_float2(a0 * a0 * uh.x, a1 * a1 * uh.y);
    S[y * D::PITCH + n] = make_float2(a0 * uh.x, a1 * uh.y);
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  store_spec<NX, NY, NZ>(S, B.spec[xi] + cz, tid);
}

// Pencil pass of the summed divergence: out = IFFT_z[ sum_xi kappa/N i k_xi
// e^{-i k_xi dx/2} FFT_z(W_xi) ].
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsZ) void k_zdiv_sum(const float2* __restrict__ W0,
                                                        const float2* __restrict__ W1,
                                                        const float2* __restrict__ W2,
                                                        float2* __restrict__ out, WaveTables t,
                                                        float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  constexpr int TY = D::TY, W = 2 * TY;
  __shared__ float2 T[NZ * W];
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  const float hx = t.hx[kx];
  for (int xi = 0; xi < 3; ++xi) {
    const float2* H = xi == 0 ? W0 : (xi == 1 ? W1 : W2);
    for (int e = tid; e < NZ * TY; e += kThreadsZ) {
      const int z = e / TY, j = e % TY;
      T[z * W + j] = H[((size_t)z * D::NKX + kx) * NY + p0 + j];
    }
    __syncthreads();
    fft_forward<NZ, true>(T, TY, 1, W, t.tw_z, tid, kThreadsZ);
    for (int e = tid; e < NZ * TY; e += kThreadsZ) {
      const int q = e / TY, j = e % TY;
      const float hy = t.hy[p0 + j], hz = t.hz[q];
      const float h = sqrtf(hx * hx + hy * hy + hz * hz);
      const float kap = (h > 0.f ? sinf(h) / h : 1.f) * inv_ntot;
      const float2 m = xi == 0 ? t.mmx[kx] : (xi == 1 ? t.mmy[p0 + j] : t.mmz[q]);
      const float2 v = cmul(cscale(T[q * W + j], kap), m);
      T[q * W + TY + j] = xi == 0 ? v : cadd(T[q * W + TY + j], v);
    }
    __syncthreads();
  }
  fft_inverse<NZ, true>(T + TY, TY, 1, W, t.tw_z, tid, kThreadsZ);
  for (int e = tid; e < NZ * TY; e += kThreadsZ) {
    const int z = e / TY, j = e % TY;
    out[((size_t)z * D::NKX + kx) * NY + p0 + j] = T[z * W + TY + j];
  }
}

// rho^_xi <- b^2 rho^_xi + c0^2 dt/rho0 q + c0^2 S^T y^n; then W_xi = R2C(b rho^_xi),
// or on the last (final != 0) step W_xi = R2C(u^_xi) for the initial-condition transpose.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_adj_rho(const float2* __restrict__ Qs, WaveBuffers B,
                                                        const float* __restrict__ yplane, WaveTables t,
                                                        WaveScalars sc, int final_step) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block<NZ>(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  load_spec<NX, NY, NZ>(S, Qs + cz, 0, nullptr, tid);
  __syncthreads();
  slab_c2r<NX, NY, NZ>(S, t, tid);
  float2* rb = reinterpret_cast<float2*>(B.rho[xi]) + rz;
  const float2* ub = reinterpret_cast<const float2*>(B.u[xi]) + rz;
  const float2* y = reinterpret_cast<const float2*>(yplane);
  const float qs = sc.c2 * sc.dt_over_rho0;
  const float bzz = t.bz[z];
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int yy = e / D::MX, n = e % D::MX;
    const float2 q = S[yy * D::PITCH + n];
    float b0, b1;
    if (xi == 0) { b0 = t.bx[2 * n]; b1 = t.bx[2 * n + 1]; }
    else if (xi == 1) { b0 = b1 = t.by[yy]; }
    else { b0 = b1 = bzz; }
    const float2 ro = rb[e];
    float2 rn = make_float2(b0 * b0 * ro.x + qs * q.x, b1 * b1 * ro.y + qs * q.y);
    if (z == 0) {
      const float2 s = y[e];
      rn.x += sc.c2 * s.x;
      rn.y += sc.c2 * s.y;
    }
    rb[e] = rn;
    S[yy * D::PITCH + n] = final_step ? ub[e] : make_float2(b0 * rn.x, b1 * rn.y);
  }
  __syncthreads();
  slab_r2c<NX, NY, NZ>(S, t, tid);
  store_spec<NX, NY, NZ>(S, B.spec[xi] + cz, tid);
}

// p = (rho^_x + rho^_y + rho^_z)/(3 c0^2) - dt/(2 rho0) sum_xi Dminus_xi u^_xi.
template <int NX, int NY, int NZ>
__global__ __launch_bounds__(kThreadsXY) void k_adj_final(const float2* __restrict__ Qs, WaveBuffers B,
                                                          float* __restrict__ pout, WaveTables t,
                                                          WaveScalars sc, int with_velocity) {
  using D = Dims<NX, NY, NZ>;
  __shared__ float2 S[NY * D::PITCH];
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  if (with_velocity) {
    load_spec<NX, NY, NZ>(S, Qs + cz, 0, nullptr, tid);
    __syncthreads();
    slab_c2r<NX, NY, NZ>(S, t, tid);
  }
  const float2* r0 = reinterpret_cast<const float2*>(B.rho[0]) + rz;
  const float2* r1 = reinterpret_cast<const float2*>(B.rho[1]) + rz;
  const float2* r2 = reinterpret_cast<const float2*>(B.rho[2]) + rz;
  float2* p = reinterpret_cast<float2*>(pout) + rz;
  for (int e = tid; e < D::SLAB_P; e += kThreadsXY) {
    const int y = e / D::MX, n = e % D::MX;
    const float2 a = r0[e], b = r1[e], c = r2[e];
    float2 v = make_float2((a.x + b.x + c.x) * sc.inv_3c2, (a.y + b.y + c.y) * sc.inv_3c2);
    if (with_velocity) {
      const float2 g = S[y * D::PITCH + n];
      v.x -= sc.half_dt_over_rho0 * g.x;
      v.y -= sc.half_dt_over_rho0 * g.y;
    }
    p[e] = v;
  }
}

// ---- launch sequences ----------------------------------------------------------

template <typename F>
inline void timed(KernelTimer* kt, int id, hipStream_t st, F&& launch) {
  const bool on = kt && (kt->which == id || kt->which == -2) && kt->count < kt->cap;
  if (on) (void)hipEventRecord(kt->ev[2 * kt->count], st);
  launch();
  if (on) {
    (void)hipEventRecord(kt->ev[2 * kt->count + 1], st);
    kt->ids[kt->count] = id;
    kt->count++;
  }
}

template <int NX, int NY, int NZ>
hipError_t wave_forward(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* p0, float* planes, int nt, hipStream_t st, KernelTimer* kt) {
  using D = Dims<NX, NY, NZ>;
  const size_t npix = (size_t)NX * NY;
  k_fwd_init<NX, NY, NZ><<<NZ, kThreadsXY, 0, st>>>(p0, B, planes, t, sc);
  for (int n = 0; n < nt - 1; ++n) {
    timed(kt, K_ZGRAD, st, [&] {
      k_zgrad<NX, NY, NZ><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], t, sc.inv_ntot);
    });
    timed(kt, K_FWD_U, st, [&] {
      k_fwd_u<NX, NY, NZ><<<3 * NZ, kThreadsXY, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], B.spec[1], B,
                                                          t, sc, n == 0 ? 1 : 0);
    });
    timed(kt, K_ZDIV, st, [&] {
      k_zmul<NX, NY, NZ, false><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], t,
                                                                          sc.inv_ntot);
    });
    timed(kt, K_FWD_RHO, st, [&] {
      k_fwd_rho<NX, NY, NZ><<<NZ, kThreadsXY, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], B, B.spec[0],
                                                        planes + (size_t)(n + 1) * npix, t, sc);
    });
  }
  return hipGetLastError();
}

template <int NX, int NY, int NZ>
hipError_t wave_adjoint(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* planes, float* p, int nt, hipStream_t st, KernelTimer* kt) {
  using D = Dims<NX, NY, NZ>;
  const size_t npix = (size_t)NX * NY;
  k_adj_init<NX, NY, NZ><<<3 * NZ, kThreadsXY, 0, st>>>(planes + (size_t)(nt - 1) * npix, B, t, sc);
  if (nt == 1) {
    k_adj_final<NX, NY, NZ><<<NZ, kThreadsXY, 0, st>>>(B.spec[3], B, p, t, sc, 0);
    return hipGetLastError();
  }
  for (int n = nt - 2; n >= 0; --n) {
    timed(kt, K_ZGRAD_ADJ, st, [&] {
      k_zmul<NX, NY, NZ, true><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], t,
                                                                         sc.inv_ntot);
    });
    timed(kt, K_ADJ_U, st, [&] { k_adj_u<NX, NY, NZ><<<3 * NZ, kThreadsXY, 0, st>>>(B, t, sc); });
    timed(kt, K_ZDIV_SUM, st, [&] {
      k_zdiv_sum<NX, NY, NZ><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                             sc.inv_ntot);
    });
    timed(kt, K_ADJ_RHO, st, [&] {
      k_adj_rho<NX, NY, NZ><<<3 * NZ, kThreadsXY, 0, st>>>(B.spec[3], B, planes + (size_t)n * npix, t, sc,
                                                           n == 0 ? 1 : 0);
    });
  }
  k_zdiv_sum<NX, NY, NZ><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                         sc.inv_ntot);
  k_adj_final<NX, NY, NZ><<<NZ, kThreadsXY, 0, st>>>(B.spec[3], B, p, t, sc, 1);
  return hipGetLastError();
}

#define PAT_WAVE_IMPL(N) {N, N, N, &wave_forward<N, N, N>, &wave_adjoint<N, N, N>}

static const WaveImpl kWaveImpls[] = {
    PAT_WAVE_IMPL(16),
    PAT_WAVE_IMPL(32),
    PAT_WAVE_IMPL(64),
    PAT_WAVE_IMPL(128),
};

const WaveImpl* find_wave_impl(int nx, int ny, int nz) {
  for (const auto& w : kWaveImpls)
    if (w.nx == nx && w.ny == ny && w.nz == nz) return &w;
  return nullptr;
}

}  // namespace pat
