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
//   slab kernels (one workgroup per z-slab): 2D real<->complex transform of the
//     slab in LDS (x: packed half-length complex FFT plus real-FFT
//     post-processing; y: column FFT), fused with the real-space update of the
//     state fields;
//   pencil kernels (one workgroup per 16 ky columns of one kx, all z): z
//     transform in LDS, the k-space multipliers, inverse z transform.
// Slab spectra live in HBM as float2 [z][kx][ky_pos] (kx = 0..nx/2 natural, ky
// in digit-reversed position order), so pencil tiles read 128-byte rows and no
// kernel ever permutes data. The state fields are float in HBM and updated in
// FP32; the transforms run in the arithmetic type V (float2, or double2 for
// FP64 butterflies with a single FP32 rounding per pass).
//
// Latency: every loop has a compile-time trip count and is unrolled, global
// loads of a thread are issued together, and the small tables a kernel needs
// (twiddles, PML profiles, wavenumbers, derivative factors) are copied to LDS
// at kernel start, so no butterfly or pointwise step waits on a global load.
//
// Forward step = pencil(grad: 1 in, 2 out) -> slab(u: per component) ->
// pencil(div: per component) -> slab(rho, p, sensor plane, R2C of p).
// Adjoint step = pencil(grad of b*rho^: per component) -> slab(u^, R2C of a*u^)
// -> pencil(sum of the three divergences: 3 in, 1 out) -> slab(rho^ + source).
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "wave_common.hpp"

namespace pat {

constexpr int kThreadsZ = 128;

// threads per slab workgroup (8 waves): FP32 slabs of 128^2 take 66.5 KB of LDS
// (two workgroups per CU), FP64 slabs 133 KB (one per CU, up to 256 VGPRs).
template <typename V> struct SlabThreads { static constexpr int value = 512; };

template <int NX, int NY, int NZ>
struct Dims {
  static constexpr int MX = NX / 2;          // complex length of a packed real row
  static constexpr int NKX = MX + 1;         // half-spectrum length
  static constexpr int PITCH = NKX;          // LDS row pitch (complex), odd
  static constexpr int SLAB_C = NKX * NY;    // complex values per slab spectrum
  static constexpr int SLAB_P = NY * MX;     // float2 pairs per real slab
  static constexpr int TY = NY >= 16 ? 16 : NY;
  static constexpr int NTILE = NKX * (NY / TY);
  static constexpr int ZIT = (NZ * TY + kThreadsZ - 1) / kThreadsZ;   // tile elements per z thread
  static constexpr int TWN = MX + NKX + NY;  // slab twiddles: MX-point, real-FFT, NY-point
  // rows per chunk of the real-FFT pre/post-processing (bounds its registers)
  static constexpr int NP = MX / 2 + 1;
  static constexpr int RC0 = 1024 / NP >= NY ? NY : (1024 / NP >= 64 ? 64 : 1024 / NP >= 32 ? 32 : 1024 / NP >= 16 ? 16 : 8);
  static constexpr int RC = RC0 > NY ? NY : RC0;
};

template <typename V> struct TabSel;
template <> struct TabSel<float2> {
  static __device__ __forceinline__ const SpecTables<float2, float>& get(const WaveTables& t) { return t.f; }
};
template <> struct TabSel<double2> {
  static __device__ __forceinline__ const SpecTables<double2, double>& get(const WaveTables& t) { return t.d; }
};

// sinc(sqrt(s)) = sin(h)/h at h^2 = s
__device__ __forceinline__ float sinc_of_sq(float s) {
  const float h = sqrtf(s);
  return h > 0.f ? sinf(h) / h : 1.f;
}
__device__ __forceinline__ double sinc_of_sq(double s) {
  if (s < 2.5) {
    // Taylor series sum_k (-s)^k / (2k+1)!, truncated after k = 12 (< 4e-21 at s = 2.5)
    double r = 1.0 / 15511210043330985984000000.0;
    r = r * -s + 1.0 / 25852016738884976640000.0;
    r = r * -s + 1.0 / 51090942171709440000.0;
    r = r * -s + 1.0 / 121645100408832000.0;
    r = r * -s + 1.0 / 355687428096000.0;
    r = r * -s + 1.0 / 1307674368000.0;
    r = r * -s + 1.0 / 6227020800.0;
    r = r * -s + 1.0 / 39916800.0;
    r = r * -s + 1.0 / 362880.0;
    r = r * -s + 1.0 / 5040.0;
    r = r * -s + 1.0 / 120.0;
    r = r * -s + 1.0 / 6.0;
    return r * -s + 1.0;
  }
  const double h = sqrt(s);
  return sin(h) / h;
}

// ---- LDS workspace of a slab workgroup ---------------------------------------
template <int NX, int NY, int NZ, typename V>
struct SlabLds {
  using D = Dims<NX, NY, NZ>;
  V S[NY * D::PITCH];     // the slab
  V tw[D::TWN];           // [0, MX): MX-point, [MX, MX+NKX): exp(-2 pi i k/NX), then NY-point
  float px[NX];           // PML profile along x of the component handled
  float py[NY];           // PML profile along y
};

// Copy the slab twiddles and up to two PML profiles into LDS (caller syncs).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void load_slab_tables(SlabLds<NX, NY, NZ, V>& L, const WaveTables& t,
                                                 const float* pml_x, const float* pml_y, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  const auto& T = TabSel<V>::get(t);
  for (int i = tid; i < D::TWN; i += NT) {
    V w;
    if (i < D::MX) w = T.tw_mx[i];
    else if (i < D::MX + D::NKX) w = T.tw_nx[i - D::MX];
    else w = T.tw_y[i - D::MX - D::NKX];
    L.tw[i] = w;
  }
  if (pml_x)
    for (int i = tid; i < NX; i += NT) L.px[i] = pml_x[i];
  if (pml_y)
    for (int i = tid; i < NY; i += NT) L.py[i] = pml_y[i];
}

// ---- slab transforms -------------------------------------------------------

// R2C post-processing of rows already transformed by a forward MX-point FFT:
// row y holds Z[k] (Z = FFT of x[2n] + i x[2n+1]) at digit-reversed positions;
// on exit it holds X[k], k = 0..MX, in natural order (X = real FFT of x).
// Rows are processed in chunks of RC: read all pairs of the chunk, barrier, write.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void r2c_post(V* S, const V* tw_nx, int tid) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int MX = D::MX, NP = D::NP, TOTAL = D::RC * NP;
  constexpr int IT = (TOTAL + NT - 1) / NT;
#pragma unroll
  for (int r0 = 0; r0 < NY; r0 += D::RC) {
    V o1[IT], o2[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (w < TOTAL) {
        const int y = r0 + w / NP, k = w % NP;
        const V* row = S + y * D::PITCH;
        if (k == 0) {
          const V z0 = row[0];
          o1[i] = mkc<V>(z0.x + z0.y, (Sc)0);
          o2[i] = mkc<V>(z0.x - z0.y, (Sc)0);
        } else {
          const V A = row[fft_pos(MX, k)];
          const V B = cconj(row[fft_pos(MX, MX - k)]);
          const V E = cscale(cadd(A, B), (Sc)0.5);
          const V Dd = csub(A, B);
          const V O = mkc<V>((Sc)0.5 * Dd.y, (Sc)-0.5 * Dd.x);   // (A - B) / (2i)
          const V WO = cmul(tw_nx[k], O);
          o1[i] = cadd(E, WO);
          o2[i] = cconj(csub(E, WO));
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (w < TOTAL) {
        const int y = r0 + w / NP, k = w % NP;
        V* row = S + y * D::PITCH;
        row[k] = o1[i];
        row[MX - k] = o2[i];   // k == 0 writes X[MX]; k == MX/2 rewrites the same value
      }
    }
    __syncthreads();
  }
}

// C2R pre-processing: row y holds X[k], k = 0..MX natural; on exit it holds
// Z'[k] = (X[k] + conj X[MX-k]) + i exp(+2 pi i k/NX) (X[k] - conj X[MX-k]) at
// digit-reversed positions, so that an inverse MX-point FFT yields
// x[2n] + i x[2n+1] (unnormalised real inverse transform).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void c2r_pre(V* S, const V* tw_nx, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int MX = D::MX, NP = D::NP, TOTAL = D::RC * NP;
  constexpr int IT = (TOTAL + NT - 1) / NT;
#pragma unroll
  for (int r0 = 0; r0 < NY; r0 += D::RC) {
    V o1[IT], o2[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (w < TOTAL) {
        const int y = r0 + w / NP, k = w % NP;
        const V* row = S + y * D::PITCH;
        const V Xk = row[k], Xm = row[MX - k];
        {
          const V s = cadd(Xk, cconj(Xm)), d = csub(Xk, cconj(Xm));
          const V wd = cmulconj(d, tw_nx[k]);
          o1[i] = mkc<V>(s.x - wd.y, s.y + wd.x);
        }
        {
          const V s = cadd(Xm, cconj(Xk)), d = csub(Xm, cconj(Xk));
          const V wd = cmulconj(d, tw_nx[MX - k]);
          o2[i] = mkc<V>(s.x - wd.y, s.y + wd.x);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (w < TOTAL) {
        const int y = r0 + w / NP, k = w % NP;
        V* row = S + y * D::PITCH;
        row[fft_pos(MX, k)] = o1[i];
        if (k != 0 && 2 * k != MX) row[fft_pos(MX, MX - k)] = o2[i];
      }
    }
    __syncthreads();
  }
}

// Real slab (packed pairs at S[y*PITCH + n]) -> slab spectrum (kx natural,
// ky digit-reversed) in place. Caller syncs before.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void slab_r2c(SlabLds<NX, NY, NZ, V>& L, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  fft_forward<D::MX, false, NY, D::PITCH, 1, NT>(L.S, L.tw, tid);
  r2c_post<NX, NY, NZ>(L.S, L.tw + D::MX, tid);
  fft_forward<NY, true, D::NKX, 1, D::PITCH, NT>(L.S, L.tw + D::MX + D::NKX, tid);
}

// Slab spectrum -> real slab (packed pairs), unnormalised. Caller syncs before.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void slab_c2r(SlabLds<NX, NY, NZ, V>& L, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  fft_inverse<NY, true, D::NKX, 1, D::PITCH, NT>(L.S, L.tw + D::MX + D::NKX, tid);
  c2r_pre<NX, NY, NZ>(L.S, L.tw + D::MX, tid);
  fft_inverse<D::MX, false, NY, D::PITCH, 1, NT>(L.S, L.tw, tid);
}

// Global slab spectrum [kx][ky_pos] -> LDS [ky_pos][kx], times mult (0: none,
// 1: per-kx table, 2: per-ky_pos table; mult is global and read in the same
// batch as the data).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void load_spec(V* S, const float2* __restrict__ g, int mode,
                                          const V* __restrict__ mult, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int IT = (D::SLAB_C + NT - 1) / NT;
  float2 r[IT];
  V m[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {     // all global loads in flight before any LDS write
    const int e = tid + i * NT;
    if (e < D::SLAB_C) {
      r[i] = g[e];
      if (mode == 1) m[i] = mult[e / NY];
      else if (mode == 2) m[i] = mult[e % NY];
    }
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_C) {
      const int kx = e / NY, p = e % NY;
      V v = widen<V>(r[i]);
      if (mode != 0) v = cmul(v, m[i]);
      S[p * D::PITCH + kx] = v;
    }
  }
}

template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void store_spec(const V* S, float2* __restrict__ g, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int IT = (D::SLAB_C + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_C) {
      const int kx = e / NY, p = e % NY;
      g[e] = narrow(S[p * D::PITCH + kx]);
    }
  }
}

// Batched read of a z-pencil tile (fixed kx, TY consecutive ky_pos, all z) into
// LDS columns [col0, col0 + TY) of a row pitch W.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void load_tile(V* T, int W, int col0, const float2* __restrict__ H, int kx, int p0,
                                          int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int TY = D::TY;
  float2 r[D::ZIT];
#pragma unroll
  for (int i = 0; i < D::ZIT; ++i) {
    const int e = tid + i * kThreadsZ;
    if (e < NZ * TY) r[i] = H[((size_t)(e / TY) * D::NKX + kx) * NY + p0 + e % TY];
  }
#pragma unroll
  for (int i = 0; i < D::ZIT; ++i) {
    const int e = tid + i * kThreadsZ;
    if (e < NZ * TY) T[(e / TY) * W + col0 + e % TY] = widen<V>(r[i]);
  }
}

template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void store_tile(const V* T, int W, int col0, float2* __restrict__ H, int kx, int p0,
                                           int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int TY = D::TY;
#pragma unroll
  for (int i = 0; i < D::ZIT; ++i) {
    const int e = tid + i * kThreadsZ;
    if (e < NZ * TY) H[((size_t)(e / TY) * D::NKX + kx) * NY + p0 + e % TY] = narrow(T[(e / TY) * W + col0 + e % TY]);
  }
}

// ---- LDS workspace of a pencil workgroup ---------------------------------------
// Per-tile spectral tables: the z twiddles, the sinc arguments along z and y,
// and the derivative factor of the multiplier along z (by kz_pos) or y (by
// ky_pos); the x factor is one value per tile.
template <int NX, int NY, int NZ, typename V, int W>
struct PencilLds {
  using Sc = typename ScalarOf<V>::T;
  V T[NZ * W];
  V twz[NZ];
  Sc hz[NZ];
  V mz[NZ];
  Sc hy[16];
  V my[16];
};

// Load the tile's tables; caller syncs. mz / my may be null when unused.
template <int NX, int NY, int NZ, typename V, int W>
__device__ __forceinline__ void load_pencil_tables(PencilLds<NX, NY, NZ, V, W>& L, const WaveTables& t, int p0,
                                                   const V* mz, const V* my, int tid) {
  using D = Dims<NX, NY, NZ>;
  const auto& T = TabSel<V>::get(t);
  for (int i = tid; i < NZ; i += kThreadsZ) {
    L.twz[i] = T.tw_z[i];
    L.hz[i] = T.hz[i];
    if (mz) L.mz[i] = mz[i];
  }
  if (tid < D::TY) {
    L.hy[tid] = T.hy[p0 + tid];
    if (my) L.my[tid] = my[p0 + tid];
  }
}

// blockIdx -> (slab z, component xi) so the three components of one slab run on
// the same XCD (block ids congruent mod 8), sharing that XCD's L2.
__device__ __forceinline__ void slab_field_of_block(int b, int& z, int& xi) {
  const int grp = b / 24, r = b % 24;
  xi = r / 8;
  z = grp * 8 + (r % 8);
}

// ---- forward kernels ---------------------------------------------------------

// rho_xi = p0 / (3 c0^2); plane 0 = p0[z = 0]; spec0 = slab R2C of p0.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_fwd_init(const float* __restrict__ p0, WaveBuffers B,
                                                                    float* __restrict__ plane0, WaveTables t,
                                                                    WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t off = (size_t)z * D::SLAB_P;
  const float2* src = reinterpret_cast<const float2*>(p0) + off;
  load_slab_tables(L, t, nullptr, nullptr, tid);
  float2 v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (tid + i * NT < D::SLAB_P) v[i] = src[tid + i * NT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      L.S[(e / D::MX) * D::PITCH + e % D::MX] = widen<V>(v[i]);
      const float2 r = make_float2(v[i].x * sc.inv_3c2, v[i].y * sc.inv_3c2);
#pragma unroll
      for (int xi = 0; xi < 3; ++xi) reinterpret_cast<float2*>(B.rho[xi])[off + e] = r;
      if (z == 0) reinterpret_cast<float2*>(plane0)[e] = v[i];
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  store_spec<NX, NY, NZ>(L.S, B.spec[0] + (size_t)z * D::SLAB_C, tid);
}

// Pencil pass of the gradient: in = FFT_xy(p) (overwritten by Q), out2 = Gz, with
// Q = IFFT_z[kappa FFT_z(in)] / N and Gz = IFFT_z[kappa i kz e^{i kz dx/2} FFT_z(in)] / N.
// The x and y derivative factors are applied later in the slab kernel (they
// depend only on kx or ky_pos), so one input yields two outputs instead of three.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsZ) void k_zgrad(float2* __restrict__ P, float2* __restrict__ Gz,
                                                     WaveTables t, float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  constexpr int TY = D::TY, W = 2 * TY;
  __shared__ PencilLds<NX, NY, NZ, V, W> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  load_pencil_tables(L, t, p0, tab.mpz, (const V*)nullptr, tid);
  const Sc hx = tab.hx[kx];
  load_tile<NX, NY, NZ>(L.T, W, 0, P, kx, p0, tid);
  __syncthreads();
  fft_forward<NZ, true, TY, 1, W, kThreadsZ>(L.T, L.twz, tid);
#pragma unroll
  for (int i = 0; i < D::ZIT; ++i) {
    const int e = tid + i * kThreadsZ;
    if (e < NZ * TY) {
      const int q = e / TY, j = e % TY;
      const Sc kap = sinc_of_sq(hx * hx + L.hy[j] * L.hy[j] + L.hz[q] * L.hz[q]) * (Sc)inv_ntot;
      const V v = cscale(L.T[q * W + j], kap);
      L.T[q * W + j] = v;
      L.T[q * W + TY + j] = cmul(v, L.mz[q]);
    }
  }
  __syncthreads();
  fft_inverse<NZ, true, W, 1, W, kThreadsZ>(L.T, L.twz, tid);
  store_tile<NX, NY, NZ>(L.T, W, 0, P, kx, p0, tid);
  store_tile<NX, NY, NZ>(L.T, W, TY, Gz, kx, p0, tid);
}

// Pencil pass applying kappa/N times i k_xi exp(s i k_xi dx/2) (PLUS: s = +1,
// else -1) to component xi = blockIdx.y, in place.
template <int NX, int NY, int NZ, typename V, bool PLUS>
__global__ __launch_bounds__(kThreadsZ) void k_zmul(float2* H0, float2* H1, float2* H2, WaveTables t,
                                                    float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  constexpr int TY = D::TY;
  __shared__ PencilLds<NX, NY, NZ, V, TY> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x, xi = blockIdx.y;
  float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  load_pencil_tables(L, t, p0, xi == 2 ? (PLUS ? tab.mpz : tab.mmz) : (const V*)nullptr,
                     xi == 1 ? (PLUS ? tab.mpy : tab.mmy) : (const V*)nullptr, tid);
  const Sc hx = tab.hx[kx];
  const V mxk = (PLUS ? tab.mpx : tab.mmx)[kx];
  load_tile<NX, NY, NZ>(L.T, TY, 0, H, kx, p0, tid);
  __syncthreads();
  fft_forward<NZ, true, TY, 1, TY, kThreadsZ>(L.T, L.twz, tid);
#pragma unroll
  for (int i = 0; i < D::ZIT; ++i) {
    const int e = tid + i * kThreadsZ;
    if (e < NZ * TY) {
      const int q = e / TY, j = e % TY;
      const Sc kap = sinc_of_sq(hx * hx + L.hy[j] * L.hy[j] + L.hz[q] * L.hz[q]) * (Sc)inv_ntot;
      const V m = xi == 0 ? mxk : (xi == 1 ? L.my[j] : L.mz[q]);
      L.T[e] = cmul(cscale(L.T[e], kap), m);
    }
  }
  __syncthreads();
  fft_inverse<NZ, true, TY, 1, TY, kThreadsZ>(L.T, L.twz, tid);
  store_tile<NX, NY, NZ>(L.T, TY, 0, H, kx, p0, tid);
}

// Velocity update of component xi for slab z, then R2C of the new u_xi.
// Q, Gz: outputs of k_zgrad; U0, U1, U2: spectra of the new u components
// (U2 aliases Gz: only this block reads Gz[z] and it does so before writing).
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_fwd_u(const float2* __restrict__ Q, const float2* Gz,
                                                                 float2* U0, float2* U1, float2* U2, WaveBuffers B,
                                                                 WaveTables t, WaveScalars sc, int init) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C;
  load_slab_tables(L, t, xi == 0 ? t.ax : nullptr, xi == 1 ? t.ay : nullptr, tid);
  if (xi == 0) load_spec<NX, NY, NZ>(L.S, Q + cz, 1, tab.mpx, tid);
  else if (xi == 1) load_spec<NX, NY, NZ>(L.S, Q + cz, 2, tab.mpy, tid);
  else load_spec<NX, NY, NZ>(L.S, Gz + cz, 0, (const V*)nullptr, tid);
  // prefetch the velocity component: its loads overlap the transform
  float2* u = reinterpret_cast<float2*>(B.u[xi]) + (size_t)z * D::SLAB_P;
  float2 uo[EPT];
  if (!init) {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (tid + i * NT < D::SLAB_P) uo[i] = u[tid + i * NT];
  }
  const float azz = t.az[z];
  __syncthreads();
  slab_c2r(L, tid);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const int y = e / D::MX, n = e % D::MX;
      const float2 g = narrow(L.S[y * D::PITCH + n]);
      float a0, a1;
      if (xi == 0) { a0 = L.px[2 * n]; a1 = L.px[2 * n + 1]; }
      else if (xi == 1) { a0 = a1 = L.py[y]; }
      else { a0 = a1 = azz; }
      const float2 o = init ? make_float2(g.x * sc.half_dt_over_rho0, g.y * sc.half_dt_over_rho0) : uo[i];
      const float2 un = make_float2(a0 * (a0 * o.x - sc.dt_over_rho0 * g.x),
                                    a1 * (a1 * o.y - sc.dt_over_rho0 * g.y));
      u[e] = un;
      L.S[y * D::PITCH + n] = widen<V>(un);
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  float2* U = xi == 0 ? U0 : (xi == 1 ? U1 : U2);
  store_spec<NX, NY, NZ>(L.S, U + cz, tid);
}

// Density update of all three components of slab z, p = c0^2 sum rho, sensor
// plane, and R2C of p into Pout.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_fwd_rho(const float2* __restrict__ H0,
                                                                   const float2* __restrict__ H1,
                                                                   const float2* __restrict__ H2, WaveBuffers B,
                                                                   float2* __restrict__ Pout,
                                                                   float* __restrict__ plane, WaveTables t,
                                                                   WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  load_slab_tables(L, t, t.bx, t.by, tid);
  const float bzz = t.bz[z];
  float2 pacc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) pacc[i] = make_float2(0.f, 0.f);
#pragma unroll 1
  for (int xi = 0; xi < 3; ++xi) {
    const float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
    load_spec<NX, NY, NZ>(L.S, H + cz, 0, (const V*)nullptr, tid);
    __syncthreads();
    slab_c2r(L, tid);
    float2* r = reinterpret_cast<float2*>(B.rho[xi]) + rz;
    float2 rold[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (tid + i * NT < D::SLAB_P) rold[i] = r[tid + i * NT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      if (e < D::SLAB_P) {
        const int y = e / D::MX, n = e % D::MX;
        const float2 h = narrow(L.S[y * D::PITCH + n]);
        float b0, b1;
        if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
        else if (xi == 1) { b0 = b1 = L.py[y]; }
        else { b0 = b1 = bzz; }
        const float2 ro = rold[i];
        const float2 rn = make_float2(b0 * (b0 * ro.x - sc.dt_rho0 * h.x), b1 * (b1 * ro.y - sc.dt_rho0 * h.y));
        r[e] = rn;
        pacc[i] = make_float2(pacc[i].x + rn.x, pacc[i].y + rn.y);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const float2 p = make_float2(pacc[i].x * sc.c2, pacc[i].y * sc.c2);
      L.S[(e / D::MX) * D::PITCH + e % D::MX] = widen<V>(p);
      if (z == 0) reinterpret_cast<float2*>(plane)[e] = p;
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  store_spec<NX, NY, NZ>(L.S, Pout + cz, tid);
}

// ---- adjoint kernels ---------------------------------------------------------

// rho^_xi = c0^2 S^T y^{nt-1}, u^_xi = 0, W_xi = R2C(b_xi rho^_xi).
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_adj_init(const float* __restrict__ ylast, WaveBuffers B,
                                                                    WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block(blockIdx.x, z, xi);
  const size_t rz = (size_t)z * D::SLAB_P, cz = (size_t)z * D::SLAB_C;
  float2* rb = reinterpret_cast<float2*>(B.rho[xi]) + rz;
  float2* ub = reinterpret_cast<float2*>(B.u[xi]) + rz;
  const float2 zero = make_float2(0.f, 0.f);
  if (z != 0) {
    for (int e = tid; e < D::SLAB_P; e += NT) { rb[e] = zero; ub[e] = zero; }
    for (int e = tid; e < D::SLAB_C; e += NT) B.spec[xi][cz + e] = zero;
    return;
  }
  load_slab_tables(L, t, xi == 0 ? t.bx : nullptr, xi == 1 ? t.by : nullptr, tid);
  const float bzz = t.bz[0];
  const float2* y = reinterpret_cast<const float2*>(ylast);
  float2 v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (tid + i * NT < D::SLAB_P) v[i] = y[tid + i * NT];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const int yy = e / D::MX, n = e % D::MX;
      const float2 r = make_float2(v[i].x * sc.c2, v[i].y * sc.c2);
      rb[e] = r;
      ub[e] = zero;
      float b0, b1;
      if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
      else if (xi == 1) { b0 = b1 = L.py[yy]; }
      else { b0 = b1 = bzz; }
      L.S[yy * D::PITCH + n] = widen<V>(make_float2(b0 * r.x, b1 * r.y));
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  store_spec<NX, NY, NZ>(L.S, B.spec[xi] + cz, tid);
}

// u^_xi: uh = u^ + dt rho0 Dplus_xi(b rho^) (the pencil pass already applied the
// multiplier), u^ <- a^2 uh, W_xi = R2C(a uh) in place.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_adj_u(WaveBuffers B, WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C;
  load_slab_tables(L, t, xi == 0 ? t.ax : nullptr, xi == 1 ? t.ay : nullptr, tid);
  load_spec<NX, NY, NZ>(L.S, B.spec[xi] + cz, 0, (const V*)nullptr, tid);
  float2* ub = reinterpret_cast<float2*>(B.u[xi]) + (size_t)z * D::SLAB_P;
  float2 uold[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (tid + i * NT < D::SLAB_P) uold[i] = ub[tid + i * NT];
  const float azz = t.az[z];
  __syncthreads();
  slab_c2r(L, tid);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const int y = e / D::MX, n = e % D::MX;
      const float2 g = narrow(L.S[y * D::PITCH + n]);
      float a0, a1;
      if (xi == 0) { a0 = L.px[2 * n]; a1 = L.px[2 * n + 1]; }
      else if (xi == 1) { a0 = a1 = L.py[y]; }
      else { a0 = a1 = azz; }
      const float2 uo = uold[i];
      const float2 uh = make_float2(uo.x + sc.dt_rho0 * g.x, uo.y + sc.dt_rho0 * g.y);
      ub[e] = make_float2(a0 * a0 * uh.x, a1 * a1 * uh.y);
      L.S[y * D::PITCH + n] = widen<V>(make_float2(a0 * uh.x, a1 * uh.y));
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  store_spec<NX, NY, NZ>(L.S, B.spec[xi] + cz, tid);
}

// Pencil pass of the summed divergence: out = IFFT_z[ sum_xi kappa/N i k_xi
// e^{-i k_xi dx/2} FFT_z(W_xi) ].
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsZ) void k_zdiv_sum(const float2* __restrict__ W0,
                                                        const float2* __restrict__ W1,
                                                        const float2* __restrict__ W2,
                                                        float2* __restrict__ out, WaveTables t,
                                                        float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  constexpr int TY = D::TY, W = 2 * TY;
  __shared__ PencilLds<NX, NY, NZ, V, W> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / TY), p0 = (blockIdx.x % (NY / TY)) * TY;
  load_pencil_tables(L, t, p0, tab.mmz, tab.mmy, tid);
  const Sc hx = tab.hx[kx];
  const V mxk = tab.mmx[kx];
  Sc kap[D::ZIT];
#pragma unroll 1
  for (int xi = 0; xi < 3; ++xi) {
    const float2* H = xi == 0 ? W0 : (xi == 1 ? W1 : W2);
    load_tile<NX, NY, NZ>(L.T, W, 0, H, kx, p0, tid);
    __syncthreads();
    if (xi == 0) {
#pragma unroll
      for (int i = 0; i < D::ZIT; ++i) {
        const int e = tid + i * kThreadsZ;
        const int q = (e / TY) % NZ, j = e % TY;
        kap[i] = sinc_of_sq(hx * hx + L.hy[j] * L.hy[j] + L.hz[q] * L.hz[q]) * (Sc)inv_ntot;
      }
    }
    fft_forward<NZ, true, TY, 1, W, kThreadsZ>(L.T, L.twz, tid);
#pragma unroll
    for (int i = 0; i < D::ZIT; ++i) {
      const int e = tid + i * kThreadsZ;
      if (e < NZ * TY) {
        const int q = e / TY, j = e % TY;
        const V m = xi == 0 ? mxk : (xi == 1 ? L.my[j] : L.mz[q]);
        const V v = cmul(cscale(L.T[q * W + j], kap[i]), m);
        L.T[q * W + TY + j] = xi == 0 ? v : cadd(L.T[q * W + TY + j], v);
      }
    }
    __syncthreads();
  }
  fft_inverse<NZ, true, TY, 1, W, kThreadsZ>(L.T + TY, L.twz, tid);
  store_tile<NX, NY, NZ>(L.T, W, TY, out, kx, p0, tid);
}

// rho^_xi <- b^2 rho^_xi + c0^2 dt/rho0 q + c0^2 S^T y^n; then W_xi = R2C(b rho^_xi),
// or on the last (final != 0) step W_xi = R2C(u^_xi) for the initial-condition transpose.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_adj_rho(const float2* __restrict__ Qs, WaveBuffers B,
                                                                   const float* __restrict__ yplane, WaveTables t,
                                                                   WaveScalars sc, int final_step) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int tid = threadIdx.x;
  int z, xi;
  slab_field_of_block(blockIdx.x, z, xi);
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  load_slab_tables(L, t, xi == 0 ? t.bx : nullptr, xi == 1 ? t.by : nullptr, tid);
  load_spec<NX, NY, NZ>(L.S, Qs + cz, 0, (const V*)nullptr, tid);
  float2* rb = reinterpret_cast<float2*>(B.rho[xi]) + rz;
  const float2* ub = reinterpret_cast<const float2*>(B.u[xi]) + rz;
  const float2* y = reinterpret_cast<const float2*>(yplane);
  float2 rold[EPT], src[EPT], uf[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      rold[i] = rb[e];
      src[i] = z == 0 ? y[e] : make_float2(0.f, 0.f);
      uf[i] = final_step ? ub[e] : make_float2(0.f, 0.f);
    }
  }
  const float bzz = t.bz[z];
  __syncthreads();
  slab_c2r(L, tid);
  const float qs = sc.c2 * sc.dt_over_rho0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const int yy = e / D::MX, n = e % D::MX;
      const float2 q = narrow(L.S[yy * D::PITCH + n]);
      float b0, b1;
      if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
      else if (xi == 1) { b0 = b1 = L.py[yy]; }
      else { b0 = b1 = bzz; }
      const float2 ro = rold[i];
      const float2 rn = make_float2(b0 * b0 * ro.x + qs * q.x + sc.c2 * src[i].x,
                                    b1 * b1 * ro.y + qs * q.y + sc.c2 * src[i].y);
      rb[e] = rn;
      L.S[yy * D::PITCH + n] = widen<V>(final_step ? uf[i] : make_float2(b0 * rn.x, b1 * rn.y));
    }
  }
  __syncthreads();
  slab_r2c(L, tid);
  store_spec<NX, NY, NZ>(L.S, B.spec[xi] + cz, tid);
}

// p = (rho^_x + rho^_y + rho^_z)/(3 c0^2) - dt/(2 rho0) sum_xi Dminus_xi u^_xi.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(SlabThreads<V>::value) void k_adj_final(const float2* __restrict__ Qs, WaveBuffers B,
                                                                     float* __restrict__ pout, WaveTables t,
                                                                     WaveScalars sc, int with_velocity) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  constexpr int EPT = (D::SLAB_P + NT - 1) / NT;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  const float2* r0 = reinterpret_cast<const float2*>(B.rho[0]) + rz;
  const float2* r1 = reinterpret_cast<const float2*>(B.rho[1]) + rz;
  const float2* r2 = reinterpret_cast<const float2*>(B.rho[2]) + rz;
  float2 rs[EPT];
  if (with_velocity) {
    load_slab_tables(L, t, nullptr, nullptr, tid);
    load_spec<NX, NY, NZ>(L.S, Qs + cz, 0, (const V*)nullptr, tid);
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      const float2 a = r0[e], b = r1[e], c = r2[e];
      rs[i] = make_float2((a.x + b.x + c.x) * sc.inv_3c2, (a.y + b.y + c.y) * sc.inv_3c2);
    }
  }
  if (with_velocity) {
    __syncthreads();
    slab_c2r(L, tid);
  }
  float2* p = reinterpret_cast<float2*>(pout) + rz;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    if (e < D::SLAB_P) {
      float2 v = rs[i];
      if (with_velocity) {
        const float2 g = narrow(L.S[(e / D::MX) * D::PITCH + e % D::MX]);
        v.x -= sc.half_dt_over_rho0 * g.x;
        v.y -= sc.half_dt_over_rho0 * g.y;
      }
      p[e] = v;
    }
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

template <int NX, int NY, int NZ, typename V>
hipError_t wave_forward(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* p0, float* planes, int nt, hipStream_t st, KernelTimer* kt) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  const size_t npix = (size_t)NX * NY;
  k_fwd_init<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(p0, B, planes, t, sc);
  for (int n = 0; n < nt - 1; ++n) {
    timed(kt, K_ZGRAD, st, [&] {
      k_zgrad<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], t, sc.inv_ntot);
    });
    timed(kt, K_FWD_U, st, [&] {
      k_fwd_u<NX, NY, NZ, V><<<3 * NZ, NT, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], B.spec[1], B, t,
                                                     sc, n == 0 ? 1 : 0);
    });
    timed(kt, K_ZDIV, st, [&] {
      k_zmul<NX, NY, NZ, V, false><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], t,
                                                                             sc.inv_ntot);
    });
    timed(kt, K_FWD_RHO, st, [&] {
      k_fwd_rho<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], B, B.spec[0],
                                                   planes + (size_t)(n + 1) * npix, t, sc);
    });
  }
  return hipGetLastError();
}

template <int NX, int NY, int NZ, typename V>
hipError_t wave_adjoint(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* planes, float* p, int nt, hipStream_t st, KernelTimer* kt) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = SlabThreads<V>::value;
  const size_t npix = (size_t)NX * NY;
  k_adj_init<NX, NY, NZ, V><<<3 * NZ, NT, 0, st>>>(planes + (size_t)(nt - 1) * npix, B, t, sc);
  if (nt == 1) {
    k_adj_final<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(B.spec[3], B, p, t, sc, 0);
    return hipGetLastError();
  }
  for (int n = nt - 2; n >= 0; --n) {
    timed(kt, K_ZGRAD_ADJ, st, [&] {
      k_zmul<NX, NY, NZ, V, true><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], t,
                                                                            sc.inv_ntot);
    });
    timed(kt, K_ADJ_U, st, [&] { k_adj_u<NX, NY, NZ, V><<<3 * NZ, NT, 0, st>>>(B, t, sc); });
    timed(kt, K_ZDIV_SUM, st, [&] {
      k_zdiv_sum<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                                sc.inv_ntot);
    });
    timed(kt, K_ADJ_RHO, st, [&] {
      k_adj_rho<NX, NY, NZ, V><<<3 * NZ, NT, 0, st>>>(B.spec[3], B, planes + (size_t)n * npix, t, sc,
                                                      n == 0 ? 1 : 0);
    });
  }
  k_zdiv_sum<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                            sc.inv_ntot);
  k_adj_final<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(B.spec[3], B, p, t, sc, 1);
  return hipGetLastError();
}

#define PAT_WAVE_IMPL(N)                                                            \
  {N, N, N, {&wave_forward<N, N, N, float2>, &wave_forward<N, N, N, double2>},     \
   {&wave_adjoint<N, N, N, float2>, &wave_adjoint<N, N, N, double2>}}

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
