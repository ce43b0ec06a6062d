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
//     slab, fused with the real-space update of the state fields;
//   pencil kernels (one workgroup per 16 ky columns of one kx, all z): z
//     transform, the k-space multipliers, inverse z transform.
// Slab spectra live in HBM as float2 [z][kx][ky_pos] (kx = 0..nx/2 natural, ky
// in digit-reversed position order), so pencil tiles read 128-byte rows and no
// kernel ever permutes data.
//
// Every butterfly runs in registers: a thread loads all values of its
// butterfly (from HBM or LDS), transforms them and passes them on; LDS is only
// the exchange between the two radix stages of a dimension and between the x
// and y passes. A slab round trip C2R -> update -> R2C therefore crosses LDS
// six times, a pencil round trip twice, and the real-space update works on the
// registers the inverse x stage left behind. Access patterns are chosen so
// that consecutive lanes touch consecutive LDS slots (odd row pitch), which
// keeps every exchange free of bank conflicts.
//
// The state fields are float in HBM and updated in FP32; the transforms run in
// the arithmetic type V (float2, or double2 for FP64 butterflies with a single
// FP32 rounding per pass).
//
// Forward step = pencil(grad: 1 in, 2 out) -> slab(u: per component) ->
// pencil(div: per component) -> slab(rho, p, sensor plane, R2C of p).
// Adjoint step = pencil(grad of b*rho^: per component) -> slab(u^, R2C of a*u^)
// -> pencil(sum of the three divergences: 3 in, 1 out) -> slab(rho^ + source).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_radix.hpp"
#include "wave_common.hpp"
#include "kspace.hpp"
#include "line_common.hpp"

namespace pat {

constexpr int kThreadsZ = 256;
constexpr int kThreadsSlab = 512;

// Slot of row index idx in an LDS slab row: one pad slot after every 8. With
// a row pitch = 1 mod 8, 8 lanes that touch 8 consecutive indices of one row,
// indices 8 apart, or the same index of rows 4 apart hit 8 distinct 16-byte
// slots, so every exchange below is free of bank conflicts; and for
// idx = j + 8 k (j < 8) the slot j + 9 k is a constant offset from a per-lane base.
__host__ __device__ constexpr int slot_of(int idx) { return idx + (idx >> 3); }
__host__ __device__ constexpr int slab_pitch(int mx) {   // smallest pitch > slot_of(mx), = 1 mod 8
  return slot_of(mx) + 1 + ((1 - (slot_of(mx) + 1) % 8) + 8) % 8;
}

template <int NX, int NY, int NZ>
struct Dims {
  static constexpr int MX = NX / 2;          // complex length of a packed real row
  static constexpr int NKX = MX + 1;         // half-spectrum length
  static constexpr int PITCH = slab_pitch(MX);   // LDS row pitch (complex), = 1 mod 8
  static constexpr int SLAB_C = NKX * NY;    // complex values per slab spectrum
  static constexpr int SLAB_P = NY * MX;     // float2 pairs per real slab
  // two-stage splits L = R0 * M of the x (packed), y and z transforms
  static constexpr int RX0 = fft_radix(MX, 0), MXB = MX / RX0;
  static constexpr int RY0 = fft_radix(NY, 0), MYB = NY / RY0;
  static constexpr int RZ0 = fft_radix(NZ, 0), MZB = NZ / RZ0;
  // x phases: every wave owns RPW whole rows, so exchanges inside a row never
  // leave the wave; per lane IX0 stage-0 butterflies and IXP pair items
  static constexpr int NWAVES = kThreadsSlab / 64;
  static constexpr int PPR = RX0 / 2;        // pair items (real-FFT split) per row
  static constexpr int RPW = NY / NWAVES > 0 ? NY / NWAVES : 1;
  static constexpr int IX0 = cdiv(RPW * MXB, 64), IXP = cdiv(RPW * PPR, 64);
  // pencil tiles
  static constexpr int TY = NY >= 16 ? 16 : NY;
  static constexpr int NTILE = NKX * (NY / TY);
  static constexpr int NZ0 = TY * MZB;       // z stage-0 butterflies per tile
  static constexpr int NZ1 = TY * RZ0;       // z stage-1 butterflies per tile
  static constexpr int IZ0 = cdiv(NZ0, kThreadsZ), IZ1 = cdiv(NZ1, kThreadsZ);
  static_assert(RX0 >= 4 && RX0 % 2 == 0, "x split needs an even first radix");
  static_assert(NY % NWAVES == 0 || NY < NWAVES, "rows must split evenly over the waves");
  static_assert(PITCH >= slot_of(MX) + 1 && PITCH % 8 == 1, "slab pitch");
};

// Register arrays of the real-space layout (per slot i, value m) and of a pencil tile.
template <int NX, int NY, int NZ>
using RealRegs = float2[Dims<NX, NY, NZ>::IX0][Dims<NX, NY, NZ>::RX0];
template <int NX, int NY, int NZ>
using ZRegs = float2[Dims<NX, NY, NZ>::IZ0][Dims<NX, NY, NZ>::RZ0];
template <int NX, int NY, int NZ, typename V>
using ZVals = V[Dims<NX, NY, NZ>::IZ1][Dims<NX, NY, NZ>::MZB];

template <typename V> struct TabSel;
template <> struct TabSel<float2> {
  static __device__ __forceinline__ const SpecTables<float2, float>& get(const WaveTables& t) { return t.f; }
};
template <> struct TabSel<double2> {
  static __device__ __forceinline__ const SpecTables<double2, double>& get(const WaveTables& t) { return t.d; }
};

// ---- LDS workspace of a slab workgroup ---------------------------------------
// S holds the slab as rows y (0..NY-1) of PITCH complex slots; index idx of a
// row (column kx of the spectrum, or an intermediate index of the x
// transform) lives in slot slot_of(idx), see sidx().
template <int NX, int NY, int NZ, typename V>
struct SlabLds {
  using D = Dims<NX, NY, NZ>;
  V S[NY * D::PITCH];
  V twx[D::MX];                        // x stage-0 twiddles, transposed table (MX points)
  V twn[D::NKX];                       // exp(-2 pi i k / NX), k <= MX (real-FFT split)
  V twy[NY];                           // y stage-0 twiddles, transposed table (NY points)
  V mul[NY > D::NKX ? NY : D::NKX];    // optional derivative factor by kx or by ky_pos
  float px[NX];                        // PML profile along x of the component handled
  float py[NY];                        // PML profile along y
};

// Tables into LDS (caller syncs). mult_mode: 0 none, 1 per kx (NKX entries),
// 2 per ky_pos (NY entries).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void load_slab_tables(SlabLds<NX, NY, NZ, V>& L, const WaveTables& t,
                                                 const float* pml_x, const float* pml_y, const V* mult,
                                                 int mult_mode, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = kThreadsSlab;
  const auto& T = TabSel<V>::get(t);
  fill_stage_table<D::RX0, D::MXB, V, NT>(L.twx, T.tw_mx, tid);
  for (int i = tid; i < D::NKX; i += NT) L.twn[i] = T.tw_nx[i];
  fill_stage_table<D::RY0, D::MYB, V, NT>(L.twy, T.tw_y, tid);
  if (mult_mode == 1)
    for (int i = tid; i < D::NKX; i += NT) L.mul[i] = mult[i];
  else if (mult_mode == 2)
    for (int i = tid; i < NY; i += NT) L.mul[i] = mult[i];
  if (pml_x)
    for (int i = tid; i < NX; i += NT) L.px[i] = pml_x[i];
  if (pml_y)
    for (int i = tid; i < NY; i += NT) L.py[i] = pml_y[i];
}

__device__ __forceinline__ int sidx(int row, int idx, int pitch) { return row * pitch + slot_of(idx); }

// Orders LDS traffic between the lanes of one wave (an exchange inside rows the
// wave owns needs no workgroup barrier: LDS runs a wave's operations in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Real-space register layout shared by every slab kernel: wave w owns rows
// [w RPW, (w+1) RPW); slot i of lane l is item e = l + 64 i of the wave (valid
// while e < RPW MXB), offset n1 = e % MXB, row y = w RPW + e / MXB; value m
// (< RX0) is the packed pair n = n1 + MXB m of row y, i.e. x = 2n, 2n + 1, at
// float2 index y * MX + n of the slab.
template <int NX, int NY, int NZ>
struct RowItem {
  using D = Dims<NX, NY, NZ>;
  int y, n1;
  bool ok;
  __device__ __forceinline__ RowItem(int tid, int i) {
    const int e = (tid & 63) + 64 * i;
    ok = e < D::RPW * D::MXB && (tid >> 6) * D::RPW < NY;
    y = (tid >> 6) * D::RPW + e / D::MXB;
    n1 = e % D::MXB;
  }
  __device__ __forceinline__ int pair(int m) const { return y * D::MX + n1 + D::MXB * m; }
  __device__ __forceinline__ int n(int m) const { return n1 + D::MXB * m; }
};

// Load one real slab (float2 pairs) in the register layout.
template <int NX, int NY, int NZ>
__device__ __forceinline__ void load_real(RealRegs<NX, NY, NZ>& r, const float2* __restrict__ src, int tid) {
  using D = Dims<NX, NY, NZ>;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) r[i][m] = src[it.pair(m)];
    }
  }
}

// ---- slab transforms -------------------------------------------------------

// Work items of the y stages. After the x transform the columns kx = 0 and
// kx = MX of a slab both hold transforms of real sequences along y (X[0] and
// X[MX] of a real row are real), so the slab keeps them packed as one complex
// column X[0] + i X[MX] at kx = 0 and the y stages run over MX columns only;
// the pair is split again where the column meets the spectrum in HBM. A wave
// of 64 lanes holds 64 consecutive columns of one butterfly (for MX a multiple
// of 64 the butterfly index, and hence its twiddles, is wave-uniform).
//   stage 1: item b -> kx = b % MX and the pair of M-point blocks c = b / MX and
//            mate(c) (frequencies f and -f lie in blocks c and R0 - c, blocks 0
//            and R0/2 hold their own negatives), so the thread that owns the
//            packed column's pair can split it in registers
//   stage 0 (R0-point butterflies n1 < M): item b -> kx = b % MX, n1 = b / MX
template <int NX, int NY, int NZ>
struct YItems {
  using D = Dims<NX, NY, NZ>;
  static constexpr int CY = D::RY0 / 2;                                     // block pairs
  static constexpr int N1 = D::MX * CY, I1 = cdiv(N1, kThreadsSlab);        // stage 1
  static constexpr int N0 = D::MX * D::MYB, I0 = cdiv(N0, kThreadsSlab);    // stage 0
  static constexpr bool UNIFORM = D::MX % 64 == 0;
  static_assert(D::RY0 >= 4 && D::RY0 % 2 == 0, "y block pairs need an even first radix");
  static __device__ __forceinline__ int mate(int c) { return c == 0 ? D::RY0 / 2 : D::RY0 - c; }
  static __device__ __forceinline__ bool s1(int tid, int i, int& kx, int& c) {
    const int b = tid + i * kThreadsSlab;
    kx = b % D::MX;
    c = b / D::MX;
    return b < N1;
  }
  static __device__ __forceinline__ bool s0(int tid, int i, int& kx, int& n1) {
    const int b = tid + i * kThreadsSlab;
    kx = b % D::MX;
    n1 = b / D::MX;
    return b < N0;
  }
};

template <typename V> using ConstTab = __attribute__((address_space(4))) const V;

// y stage-0 twiddles of butterfly n1: with a wave-uniform n1 they come through
// the scalar cache from the natural table tw_y (global, read-only); otherwise
// from the transposed LDS table.
template <int NX, int NY, int NZ, bool INV, typename V>
__device__ __forceinline__ void y_twiddle(V* a, const SlabLds<NX, NY, NZ, V>& L, const V* __restrict__ twg,
                                          int n1) {
  using D = Dims<NX, NY, NZ>;
  constexpr int M = D::MYB, R0 = D::RY0;
  if constexpr (M > 1) {
    if constexpr (YItems<NX, NY, NZ>::UNIFORM) {
      using Sc = typename ScalarOf<V>::T;
      const int n1u = __builtin_amdgcn_readfirstlane(n1);
      ConstTab<Sc>* t = (ConstTab<Sc>*)twg;   // (re, im) pairs
#pragma unroll
      for (int k = 1; k < R0; ++k) {
        const V w = mkc<V>(t[2 * n1u * k], t[2 * n1u * k + 1]);
        a[k] = INV ? cmulconj(a[k], w) : cmul(a[k], w);
      }
    } else {
      stage_twiddle<R0, M, INV>(a, L.twy, n1);
    }
  }
}

// n consecutive complex values from g (16-byte aligned for even offsets) as
// 16-byte loads where n is even.
template <int n>
__device__ __forceinline__ void load_run(float2 (&r)[n], const float2* __restrict__ g) {
  if constexpr (n % 2 == 0) {
#pragma unroll
    for (int k = 0; k < n; k += 2) {
      const float4 u = reinterpret_cast<const float4*>(g)[k / 2];
      r[k] = make_float2(u.x, u.y);
      r[k + 1] = make_float2(u.z, u.w);
    }
  } else {
#pragma unroll
    for (int k = 0; k < n; ++k) r[k] = g[k];
  }
}

// Registers of the y stage-1 global loads: the two blocks (c, mate(c)) of the
// item's column, and for kx = 0 the same blocks of column MX.
template <int NX, int NY, int NZ>
struct YRegs {
  float2 v[YItems<NX, NY, NZ>::I1][2][Dims<NX, NY, NZ>::MYB];
  float2 n[YItems<NX, NY, NZ>::I1][2][Dims<NX, NY, NZ>::MYB];
};

// Global loads of the slab spectrum g[kx][ky_pos] in the stage-1 layout; issued
// before anything else a kernel waits on, so their latency overlaps the table
// loads and the barrier that follows.
template <int NX, int NY, int NZ>
__device__ __forceinline__ void y_load(YRegs<NX, NY, NZ>& r, const float2* __restrict__ g, int tid) {
  using D = Dims<NX, NY, NZ>;
  using Y = YItems<NX, NY, NZ>;
  constexpr int M = D::MYB;
#pragma unroll
  for (int i = 0; i < Y::I1; ++i) {
    int kx, c;
    if (Y::s1(tid, i, kx, c)) {
      const int mc = Y::mate(c);
      load_run<M>(r.v[i][0], g + kx * NY + M * c);
      load_run<M>(r.v[i][1], g + kx * NY + M * mc);
      if (kx == 0) {
        load_run<M>(r.n[i][0], g + D::MX * NY + M * c);
        load_run<M>(r.n[i][1], g + D::MX * NY + M * mc);
      }
    }
  }
}

// y inverse transform of the loaded slab spectrum (times an optional derivative
// factor L.mul by kx (mode 1) or ky_pos (mode 2)); leaves the rows in natural
// y order (index kx, column 0 = X[0] + i X[MX]). Caller syncs before (tables);
// ends synced.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void y_inverse(SlabLds<NX, NY, NZ, V>& L, const YRegs<NX, NY, NZ>& r, int mode,
                                          const V* __restrict__ twg, int tid) {
  using D = Dims<NX, NY, NZ>;
  using Y = YItems<NX, NY, NZ>;
  constexpr int M = D::MYB, R0 = D::RY0, P = D::PITCH;
#pragma unroll
  for (int i = 0; i < Y::I1; ++i) {
    int kx, c;
    if (Y::s1(tid, i, kx, c)) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int mb = h == 0 ? c : Y::mate(c);
        V a[M];
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          a[k1] = widen<V>(r.v[i][h][k1]);
          if (mode == 1) a[k1] = cmul(a[k1], L.mul[kx]);
        }
        if (kx == 0) {   // pack column MX in as the imaginary part
#pragma unroll
          for (int k1 = 0; k1 < M; ++k1) {
            V u = widen<V>(r.n[i][h][k1]);
            if (mode == 1) u = cmul(u, L.mul[D::MX]);
            a[k1] = mkc<V>(a[k1].x - u.y, a[k1].y + u.x);
          }
        }
        if (mode == 2) {
#pragma unroll
          for (int k1 = 0; k1 < M; ++k1) a[k1] = cmul(a[k1], L.mul[M * mb + k1]);
        }
        dft_r<M, true>(a);
#pragma unroll
        for (int n1 = 0; n1 < M; ++n1) L.S[sidx(M * mb + n1, kx, P)] = a[n1];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Y::I0; ++i) {
    int kx, n1;
    if (Y::s0(tid, i, kx, n1)) {
      V a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = L.S[sidx(n1 + M * m, kx, P)];
      y_twiddle<NX, NY, NZ, true>(a, L, twg, n1);
      dft_r<R0, true>(a);
#pragma unroll
      for (int m = 0; m < R0; ++m) L.S[sidx(n1 + M * m, kx, P)] = a[m];
    }
  }
  __syncthreads();
}

// The float2 view of LDS slab slot (row, idx): the spectrum, narrowed to its
// storage precision, is staged in the slots it was computed in.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ float2* slot_f2(SlabLds<NX, NY, NZ, V>& L, int row, int idx) {
  return reinterpret_cast<float2*>(&L.S[sidx(row, idx, Dims<NX, NY, NZ>::PITCH)]);
}

// Split of the packed column's spectrum Z = Y0 + i YN (Y0, YN Hermitian) at
// ky_pos p from Z[f] and Z[-f]: Y0 = (Z[f] + conj Z[-f]) / 2,
// YN = (Z[f] - conj Z[-f]) / (2i); staged in slots (p, 0) and (p, MX).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void y_split_stage(SlabLds<NX, NY, NZ, V>& L, int p, V zf, V zm) {
  using Sc = typename ScalarOf<V>::T;
  *slot_f2(L, p, 0) = narrow(mkc<V>((Sc)0.5 * (zf.x + zm.x), (Sc)0.5 * (zf.y - zm.y)));
  *slot_f2(L, p, Dims<NX, NY, NZ>::MX) = narrow(mkc<V>((Sc)0.5 * (zf.y + zm.y), (Sc)0.5 * (zm.x - zf.x)));
}

// y forward transform of the rows (natural y, index kx, column 0 packed) into
// the slab spectrum g[kx][ky_pos]. Stage 0 runs in LDS; stage 1 leaves its
// outputs (float2) in the slots it read, every slot being read by exactly one
// thread, so no barrier is needed before those writes; after a barrier the
// slab is stored column by column, consecutive lanes on consecutive ky_pos
// (512 contiguous bytes per wave instruction instead of one 64-byte run per
// lane 1 KB apart, which the memory pipeline handles several times slower).
// Caller syncs before; the caller syncs again before S is written.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void y_forward_to_global(SlabLds<NX, NY, NZ, V>& L, float2* __restrict__ g,
                                                    const V* __restrict__ twg, int tid) {
  using D = Dims<NX, NY, NZ>;
  using Y = YItems<NX, NY, NZ>;
  constexpr int M = D::MYB, R0 = D::RY0, P = D::PITCH;
#pragma unroll
  for (int i = 0; i < Y::I0; ++i) {
    int kx, n1;
    if (Y::s0(tid, i, kx, n1)) {
      V a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = L.S[sidx(n1 + M * m, kx, P)];
      dft_r<R0, false>(a);
      y_twiddle<NX, NY, NZ, false>(a, L, twg, n1);
#pragma unroll
      for (int k = 0; k < R0; ++k) L.S[sidx(n1 + M * k, kx, P)] = a[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Y::I1; ++i) {
    int kx, c;
    if (Y::s1(tid, i, kx, c)) {
      const int mc = Y::mate(c);
      V za[M], zb[M];
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        za[k1] = L.S[sidx(M * c + k1, kx, P)];
        zb[k1] = L.S[sidx(M * mc + k1, kx, P)];
      }
      dft_r<M, false>(za);
      dft_r<M, false>(zb);
      if (kx != 0) {
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          *slot_f2(L, M * c + k1, kx) = narrow(za[k1]);
          *slot_f2(L, M * mc + k1, kx) = narrow(zb[k1]);
        }
      } else if (c == 0) {   // blocks 0 and R0/2: -f in the same block
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          y_split_stage(L, k1, za[k1], za[(M - k1) % M]);
          y_split_stage(L, M * mc + k1, zb[k1], zb[M - 1 - k1]);
        }
      } else {               // f in block c, -f in block R0 - c
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          y_split_stage(L, M * c + k1, za[k1], zb[M - 1 - k1]);
          y_split_stage(L, M * mc + k1, zb[k1], za[M - 1 - k1]);
        }
      }
    }
  }
  __syncthreads();
  // element e = kx * NY + ky_pos of the slab spectrum, kx = 0..MX
#pragma unroll
  for (int i = 0; i < cdiv(D::SLAB_C, kThreadsSlab); ++i) {
    const int e = tid + i * kThreadsSlab;
    if (e < D::SLAB_C) g[e] = *slot_f2(L, e % NY, e / NY);
  }
}

// The x transform of a real row of NX values runs as an MX-point complex FFT
// of the packed pairs z[n] = x[2n] + i x[2n+1] plus the split
//   X[k] = E_k + w^k O_k,  E_k = (Z[k] + conj Z[MX-k]) / 2,
//   O_k = (Z[k] - conj Z[MX-k]) / (2i),  w = exp(-2 pi i / NX),
// (and its inverse before the inverse transform). Frequencies k and MX - k
// meet in stage-1 blocks b and R0 - b (mod R0), so one thread takes both
// blocks of a pair {g, R0 - g} (g = 1..R0/2-1) or {0, R0/2} (g = 0, which also
// owns X[MX]) and the split runs in its registers.
template <typename V>
__device__ __forceinline__ V split_fwd(V zk, V zp, V w) {   // X[k] from Z[k], Z[MX-k]
  using Sc = typename ScalarOf<V>::T;
  const V e = cscale(cadd(zk, cconj(zp)), (Sc)0.5);
  const V d = csub(zk, cconj(zp));
  const V o = mkc<V>((Sc)0.5 * d.y, (Sc)-0.5 * d.x);
  return cadd(e, cmul(w, o));
}
template <typename V>
__device__ __forceinline__ V split_inv(V xk, V xp, V w) {   // 2 Z[k] from X[k], X[MX-k]
  const V s = cadd(xk, cconj(xp)), d = csub(xk, cconj(xp));
  const V wd = cmulconj(d, w);
  return mkc<V>(s.x - wd.y, s.y + wd.x);
}

// Pair item of the x phases: slot i of lane l is item e = l + 64 i of its wave
// (valid while e < RPW PPR): g = e % PPR, row y = w RPW + e / PPR.
template <int NX, int NY, int NZ>
struct PairItem {
  using D = Dims<NX, NY, NZ>;
  int y, g, ma, mb;
  bool ok;
  __device__ __forceinline__ PairItem(int tid, int i) {
    const int e = (tid & 63) + 64 * i;
    ok = e < D::RPW * D::PPR && (tid >> 6) * D::RPW < NY;
    // with 4 pair items per row, the two 4-lane halves of an 8-lane group take
    // rows 4 apart (r = 2j + h -> row j % 4 + 4 h + 8 (j / 4)), see slot_of()
    const int r = e / D::PPR;
    const int rr = (D::PPR == 4 && D::RPW % 8 == 0) ? ((r >> 1) & 3) + 4 * (r & 1) + 8 * (r >> 3) : r;
    y = (tid >> 6) * D::RPW + rr;
    g = e % D::PPR;
    ma = g;
    mb = g == 0 ? D::RX0 / 2 : D::RX0 - g;
  }
};

// Rows (natural kx, X[0..MX-1], slot 0 holding X[0] + i X[MX]) -> inverse x
// transform -> packed real pairs (unnormalised), handed to out(i, m, value) in
// the register layout (slot i, value m) as they come out. Caller syncs before.
// Every exchange stays inside the rows of one wave.
template <int NX, int NY, int NZ, typename V, typename F>
__device__ __forceinline__ void x_inverse_apply(SlabLds<NX, NY, NZ, V>& L, int tid, F&& out) {
  using D = Dims<NX, NY, NZ>;
  constexpr int R0 = D::RX0, M = D::MXB, P = D::PITCH;
  V za[D::IXP][M], zb[D::IXP][M];
#pragma unroll
  for (int i = 0; i < D::IXP; ++i) {
    const PairItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
      V xa[M], xb[M];
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        xa[k1] = L.S[sidx(it.y, it.ma + R0 * k1, P)];
        xb[k1] = L.S[sidx(it.y, it.mb + R0 * k1, P)];
      }
      const V* wa = L.twn + it.ma;   // w^k for k = ma + R0 k1 at wa[R0 k1]
      const V* wb = L.twn + it.mb;
      // Partners are taken two at a time so each input dies as its outputs are
      // formed (branches rather than selects keep xa, xb in registers).
      if (it.g != 0) {   // k = ma + R0 k1 pairs with mb + R0 (M-1-k1)
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          const V a = xa[k1], b = xb[M - 1 - k1];
          za[i][k1] = split_inv(a, b, wa[R0 * k1]);
          zb[i][M - 1 - k1] = split_inv(b, a, wb[R0 * (M - 1 - k1)]);
        }
      } else {           // block 0 pairs with itself, block R0/2 with itself
        // slot 0 holds X[0] + i X[MX] (both real): 2 Z[0] = X[0] + X[MX] + i (X[0] - X[MX])
        za[i][0] = mkc<V>(xa[0].x + xa[0].y, xa[0].x - xa[0].y);
#pragma unroll
        for (int k1 = 1; k1 <= M / 2; ++k1) {
          const int k2 = M - k1;
          const V a = xa[k1], b = xa[k2];
          za[i][k1] = split_inv(a, b, wa[R0 * k1]);
          if (k2 != k1) za[i][k2] = split_inv(b, a, wa[R0 * k2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < (M + 1) / 2; ++k1) {
          const int k2 = M - 1 - k1;
          const V a = xb[k1], b = xb[k2];
          zb[i][k1] = split_inv(a, b, wb[R0 * k1]);
          if (k2 != k1) zb[i][k2] = split_inv(b, a, wb[R0 * k2]);
        }
      }
      dft_r<M, true>(za[i]);
      dft_r<M, true>(zb[i]);
    }
  }
  wave_sync();   // every lane of the wave has read its row slots
#pragma unroll
  for (int i = 0; i < D::IXP; ++i) {
    const PairItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int n1 = 0; n1 < M; ++n1) {
        L.S[sidx(it.y, M * it.ma + n1, P)] = za[i][n1];
        L.S[sidx(it.y, M * it.mb + n1, P)] = zb[i][n1];
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
      V a[R0];
#pragma unroll
      for (int k = 0; k < R0; ++k) a[k] = L.S[sidx(it.y, it.n1 + M * k, P)];
      if constexpr (M > 1) stage_twiddle<R0, M, true>(a, L.twx, it.n1);
      dft_r<R0, true>(a);
#pragma unroll
      for (int m = 0; m < R0; ++m) out(i, m, narrow(a[m]));
    }
  }
}

template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void x_inverse_to_regs(SlabLds<NX, NY, NZ, V>& L, RealRegs<NX, NY, NZ>& out, int tid) {
  x_inverse_apply(L, tid, [&](int i, int m, float2 v) { out[i][m] = v; });
}

// Packed real pairs in the register layout -> forward x transform -> rows
// (natural kx, X[0..MX-1], slot 0 holding X[0] + i X[MX]); ends with a workgroup barrier (the y pass reads
// columns). The first stage writes the LDS slots the same thread read in
// x_inverse_to_regs, so no barrier is needed before it; otherwise the caller syncs.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void x_forward_from_regs(SlabLds<NX, NY, NZ, V>& L, const RealRegs<NX, NY, NZ>& in,
                                                    int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int R0 = D::RX0, M = D::MXB, P = D::PITCH;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
      V a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = widen<V>(in[i][m]);
      dft_r<R0, false>(a);
      if constexpr (M > 1) stage_twiddle<R0, M, false>(a, L.twx, it.n1);
#pragma unroll
      for (int k = 0; k < R0; ++k) L.S[sidx(it.y, it.n1 + M * k, P)] = a[k];
    }
  }
  wave_sync();
  V xa[D::IXP][M], xb[D::IXP][M];
#pragma unroll
  for (int i = 0; i < D::IXP; ++i) {
    const PairItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
      V za[M], zb[M];
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        za[k1] = L.S[sidx(it.y, M * it.ma + k1, P)];
        zb[k1] = L.S[sidx(it.y, M * it.mb + k1, P)];
      }
      dft_r<M, false>(za);
      dft_r<M, false>(zb);
      const V* wa = L.twn + it.ma;   // w^k for k = ma + R0 k1 at wa[R0 k1]
      const V* wb = L.twn + it.mb;
      // partner Z[MX - k], two at a time as above
      if (it.g != 0) {
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
          const V a = za[k1], b = zb[M - 1 - k1];
          xa[i][k1] = split_fwd(a, b, wa[R0 * k1]);
          xb[i][M - 1 - k1] = split_fwd(b, a, wb[R0 * (M - 1 - k1)]);
        }
      } else {
        // X[0] = Re Z[0] + Im Z[0] and X[MX] = Re Z[0] - Im Z[0], packed into slot 0
        xa[i][0] = mkc<V>(za[0].x + za[0].y, za[0].x - za[0].y);
#pragma unroll
        for (int k1 = 1; k1 <= M / 2; ++k1) {
          const int k2 = M - k1;
          const V a = za[k1], b = za[k2];
          xa[i][k1] = split_fwd(a, b, wa[R0 * k1]);
          if (k2 != k1) xa[i][k2] = split_fwd(b, a, wa[R0 * k2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < (M + 1) / 2; ++k1) {
          const int k2 = M - 1 - k1;
          const V a = zb[k1], b = zb[k2];
          xb[i][k1] = split_fwd(a, b, wb[R0 * k1]);
          if (k2 != k1) xb[i][k2] = split_fwd(b, a, wb[R0 * k2]);
        }
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < D::IXP; ++i) {
    const PairItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        L.S[sidx(it.y, it.ma + R0 * k1, P)] = xa[i][k1];
        L.S[sidx(it.y, it.mb + R0 * k1, P)] = xb[i][k1];
      }
    }
  }
  __syncthreads();
}

// ---- z pencils ---------------------------------------------------------------
// A tile is TY consecutive ky_pos columns (p0..p0+TY-1) of one kx over all z,
// held in LDS as T[z_index * TY + col]. Per-tile tables: the z twiddles, the
// sinc arguments along z and y, and the derivative factor along z (by kz_pos)
// or y (by ky_pos); the x factor is one value per tile.
template <int NX, int NY, int NZ, typename V, int NB>
struct PencilLds {
  using Sc = typename ScalarOf<V>::T;
  using D = Dims<NX, NY, NZ>;
  V T[NB][NZ * D::TY];
  V twz[NZ];   // z stage-0 twiddles, transposed table
  Sc hz[NZ];
  V mz[NZ];
  Sc hy[D::TY];
  V my[D::TY];
};

// Load the tile's tables; caller syncs. The derivative factor of a pass is kept
// separable, m = my[col] * mz[q]: my = mx (one value per tile) times the y
// factor (if any) by column, mz the z factor (if any) by kz position; absent
// factors are 1, so a product with them is exact.
template <int NX, int NY, int NZ, typename V, int NB>
__device__ __forceinline__ void load_pencil_tables(PencilLds<NX, NY, NZ, V, NB>& L, const WaveTables& t, int p0,
                                                   V mx, const V* my, const V* mz, int tid) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  const auto& T = TabSel<V>::get(t);
  fill_stage_table<D::RZ0, D::MZB, V, kThreadsZ>(L.twz, T.tw_z, tid);
  for (int i = tid; i < NZ; i += kThreadsZ) L.hz[i] = T.hz[i];
  if (mz) {
    for (int i = tid; i < NZ; i += kThreadsZ) L.mz[i] = mz[i];
  } else {
    for (int i = tid; i < NZ; i += kThreadsZ) L.mz[i] = mkc<V>((Sc)1, (Sc)0);
  }
  if (tid < D::TY) {
    L.hy[tid] = T.hy[p0 + tid];
    if (my) L.my[tid] = cmul(mx, my[p0 + tid]);
    else L.my[tid] = mx;
  }
}

// z stage-0 twiddles: FP64 builds the powers in registers (a table read per
// power would keep 15 complex doubles live next to the butterfly), FP32 reads them.
template <int R, int M, bool INV, typename V>
__device__ __forceinline__ void pencil_twiddle(V* a, const V* twT, int n1) {
  if constexpr (std::is_same<V, double2>::value) stage_twiddle_pow<R, M, INV>(a, twT, n1);
  else stage_twiddle<R, M, INV>(a, twT, n1);
}

// Global loads of a tile in the stage-0 butterfly layout: slot i of a thread is
// item b = tid + i * kThreadsZ, column b % TY, offset n1 = b / TY; value m is z = n1 + MZB m.
template <int NX, int NY, int NZ>
__device__ __forceinline__ void z_load(ZRegs<NX, NY, NZ>& r,
                                       const float2* __restrict__ H, int kx, int p0, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr unsigned ZS = D::NKX * NY;   // float2 stride between z planes
#pragma unroll
  for (int i = 0; i < D::IZ0; ++i) {
    const int b = tid + i * kThreadsZ;
    if (b < D::NZ0) {
      const int col = b % D::TY, n1 = b / D::TY;
      // wave-uniform base per value (scalar registers) plus one 32-bit lane byte offset
      const unsigned boff = ((unsigned)n1 * ZS + (unsigned)(kx * NY + p0 + col)) * 8u;
#pragma unroll
      for (int m = 0; m < D::RZ0; ++m)
        r[i][m] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(H + (size_t)(D::MZB * m) * ZS) + boff);
    }
  }
}

// Forward stage 0 of the loaded tile into T (values loaded as float2, or
// already in the arithmetic type).
template <typename V> __device__ __forceinline__ V as_arith(float2 v) { return widen<V>(v); }
template <typename V> __device__ __forceinline__ V as_arith(V v) { return v; }

template <int NX, int NY, int NZ, typename V, typename In>
__device__ __forceinline__ void z_fwd0(V* T, const In (&r)[Dims<NX, NY, NZ>::IZ0][Dims<NX, NY, NZ>::RZ0],
                                       const V* twz, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int R0 = D::RZ0, M = D::MZB;
#pragma unroll
  for (int i = 0; i < D::IZ0; ++i) {
    const int b = tid + i * kThreadsZ;
    if (b < D::NZ0) {
      const int col = b % D::TY, n1 = b / D::TY;
      V a[R0];
#pragma unroll
      for (int m = 0; m < R0; ++m) a[m] = as_arith<V>(r[i][m]);
      dft_r<R0, false>(a);
      if constexpr (M > 1) pencil_twiddle<R0, M, false>(a, twz, n1);
#pragma unroll
      for (int k = 0; k < R0; ++k) T[(n1 + M * k) * D::TY + col] = a[k];
    }
  }
}

// Forward stage 1 from T into registers: slot i is item b = tid + i * kThreadsZ,
// column b % TY, block mb = b / TY; value k1 is at kz position MZB mb + k1.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void z_fwd1(const V* T, ZVals<NX, NY, NZ, V>& v, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int M = D::MZB;
#pragma unroll
  for (int i = 0; i < D::IZ1; ++i) {
    const int b = tid + i * kThreadsZ;
    if (b < D::NZ1) {
      const int col = b % D::TY, mb = b / D::TY;
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) v[i][k1] = T[(M * mb + k1) * D::TY + col];
      dft_r<M, false>(v[i]);
    }
  }
}

// Inverse stage 1 of register values back into T (the slots z_fwd1 read).
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void z_inv1(V* T, ZVals<NX, NY, NZ, V>& v, int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int M = D::MZB;
#pragma unroll
  for (int i = 0; i < D::IZ1; ++i) {
    const int b = tid + i * kThreadsZ;
    if (b < D::NZ1) {
      const int col = b % D::TY, mb = b / D::TY;
      dft_r<M, true>(v[i]);
#pragma unroll
      for (int n1 = 0; n1 < M; ++n1) T[(M * mb + n1) * D::TY + col] = v[i][n1];
    }
  }
}

// Inverse stage 0 from T straight to HBM.
template <int NX, int NY, int NZ, typename V>
__device__ __forceinline__ void z_inv0_store(const V* T, float2* __restrict__ H, int kx, int p0, const V* twz,
                                             int tid) {
  using D = Dims<NX, NY, NZ>;
  constexpr int R0 = D::RZ0, M = D::MZB;
#pragma unroll
  for (int i = 0; i < D::IZ0; ++i) {
    const int b = tid + i * kThreadsZ;
    if (b < D::NZ0) {
      const int col = b % D::TY, n1 = b / D::TY;
      V a[R0];
#pragma unroll
      for (int k = 0; k < R0; ++k) a[k] = T[(n1 + M * k) * D::TY + col];
      if constexpr (M > 1) pencil_twiddle<R0, M, true>(a, twz, n1);
      dft_r<R0, true>(a);
      constexpr unsigned ZS = D::NKX * NY;
      const unsigned boff = ((unsigned)n1 * ZS + (unsigned)(kx * NY + p0 + col)) * 8u;
#pragma unroll
      for (int m = 0; m < R0; ++m)
        *reinterpret_cast<float2*>(reinterpret_cast<char*>(H + (size_t)(M * m) * ZS) + boff) = narrow(a[m]);
    }
  }
}

// kappa / N at column col, kz position q of the tile.
template <typename Sc>
__device__ __forceinline__ Sc kappa_n(Sc hx, Sc hy, Sc hz, float inv_ntot) {
  return sinc_of_sq(hx * hx + hy * hy + hz * hz) * (Sc)inv_ntot;
}

// blockIdx -> (slab z, component xi) so the three components of one slab run on
// the same XCD (block ids congruent mod 8), sharing that XCD's L2.
__device__ __forceinline__ void slab_field_of_block(int b, int& z, int& xi) {
  const int grp = b / 24, r = b % 24;
  xi = r / 8;
  z = grp * 8 + (r % 8);
}

// ---- forward kernels ---------------------------------------------------------

// rho_xi = p0 / (3 c0^2); sensor plane 0 = p0[z = 0] in the first of the two
// plane series (plane_b, the second, starts at 0); spec0 = slab R2C of p0.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_fwd_init(const float* __restrict__ p0, WaveBuffers B,
                                                           float* __restrict__ plane0, float* __restrict__ plane_b,
                                                           WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t off = (size_t)z * D::SLAB_P;
  load_slab_tables(L, t, nullptr, nullptr, (const V*)nullptr, 0, tid);
  float2 v[D::IX0][D::RX0];
  load_real<NX, NY, NZ>(v, reinterpret_cast<const float2*>(p0) + off, tid);
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) {
        float2 r = make_float2(v[i][m].x * sc.inv_3c2, v[i][m].y * sc.inv_3c2);
        if (B.c2f) {   // heterogeneous medium: rho_xi = p0 / (3 c(x)^2)
          const float2 cc = reinterpret_cast<const float2*>(B.c2f)[off + it.pair(m)];
          r = make_float2(v[i][m].x / (3.0f * cc.x), v[i][m].y / (3.0f * cc.y));
        }
#pragma unroll
        for (int xi = 0; xi < 3; ++xi) reinterpret_cast<float2*>(B.rho[xi])[off + it.pair(m)] = r;
        if (z == 0) {
          reinterpret_cast<float2*>(plane0)[it.pair(m)] = v[i][m];
          reinterpret_cast<float2*>(plane_b)[it.pair(m)] = make_float2(0.f, 0.f);
        }
      }
    }
  }
  __syncthreads();
  x_forward_from_regs(L, v, tid);
  y_forward_to_global(L, B.spec[0] + (size_t)z * D::SLAB_C, TabSel<V>::get(t).tw_y, tid);
}

// Pencil pass of the gradient: in = FFT_xy(p) = P0 (+ P1 when nin = 2; the two
// halves of the density pass), out Q and Gz with
// Q = IFFT_z[kappa FFT_z(in)] / N and Gz = IFFT_z[kappa i kz e^{i kz dx/2} FFT_z(in)] / N.
// The x and y derivative factors are applied later in the slab kernel (they
// depend only on kx or ky_pos), so one input yields two outputs instead of three.
// Qo may alias P0 and Gz P1: a tile reads all its inputs before it writes.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsZ) void k_zgrad(const float2* P0, const float2* P1, int nin, float2* Qo,
                                                     float2* Gz, WaveTables t, float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  __shared__ PencilLds<NX, NY, NZ, V, 1> L;   // one tile buffer: Q and Gz leave one after the other
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / D::TY), p0 = (blockIdx.x % (NY / D::TY)) * D::TY;
  float2 r[D::IZ0][D::RZ0], r1[D::IZ0][D::RZ0];
  z_load<NX, NY, NZ>(r, P0, kx, p0, tid);
  if (nin > 1) z_load<NX, NY, NZ>(r1, P1, kx, p0, tid);
  load_pencil_tables(L, t, p0, mkc<V>((Sc)1, (Sc)0), (const V*)nullptr, tab.mpz, tid);
  const Sc hx = tab.hx[kx];
  __syncthreads();
  if (nin > 1) {   // the sum is formed in FP32, like the stored spectra it adds up
#pragma unroll
    for (int i = 0; i < D::IZ0; ++i)
#pragma unroll
      for (int m = 0; m < D::RZ0; ++m) r[i][m] = make_float2(r[i][m].x + r1[i][m].x, r[i][m].y + r1[i][m].y);
  }
  z_fwd0<NX, NY, NZ>(L.T[0], r, L.twz, tid);
  __syncthreads();
  V v[D::IZ1][D::MZB], w[D::IZ1][D::MZB];
  z_fwd1<NX, NY, NZ>(L.T[0], v, tid);
#pragma unroll
  for (int i = 0; i < D::IZ1; ++i) {
    const int b = tid + i * kThreadsZ;
    const int col = b % D::TY, mb = b / D::TY;
#pragma unroll
    for (int k1 = 0; k1 < D::MZB; ++k1) {
      const int q = D::MZB * mb + k1;
      if (b < D::NZ1) {
        v[i][k1] = cscale(v[i][k1], kappa_n(hx, L.hy[col], L.hz[q], inv_ntot));
        w[i][k1] = cmul(v[i][k1], L.mz[q]);
      }
    }
  }
  z_inv1<NX, NY, NZ>(L.T[0], v, tid);
  __syncthreads();
  z_inv0_store<NX, NY, NZ>(L.T[0], Qo, kx, p0, L.twz, tid);
  __syncthreads();
  z_inv1<NX, NY, NZ>(L.T[0], w, tid);
  __syncthreads();
  z_inv0_store<NX, NY, NZ>(L.T[0], Gz, kx, p0, L.twz, tid);
}

// Pencil pass applying kappa/N times i k_xi exp(s i k_xi dx/2) (PLUS: s = +1,
// else -1) to component xi = blockIdx.y, in place.
template <int NX, int NY, int NZ, typename V, bool PLUS>
__global__ __launch_bounds__(kThreadsZ) void k_zmul(float2* H0, float2* H1, float2* H2, WaveTables t,
                                                    float inv_ntot) {
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  __shared__ PencilLds<NX, NY, NZ, V, 1> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x, xi = blockIdx.y;
  float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
  const int kx = blockIdx.x / (NY / D::TY), p0 = (blockIdx.x % (NY / D::TY)) * D::TY;
  float2 r[D::IZ0][D::RZ0];
  z_load<NX, NY, NZ>(r, H, kx, p0, tid);
  load_pencil_tables(L, t, p0, xi == 0 ? (PLUS ? tab.mpx : tab.mmx)[kx] : mkc<V>((Sc)1, (Sc)0),
                     xi == 1 ? (PLUS ? tab.mpy : tab.mmy) : (const V*)nullptr,
                     xi == 2 ? (PLUS ? tab.mpz : tab.mmz) : (const V*)nullptr, tid);
  const Sc hx = tab.hx[kx];
  __syncthreads();
  z_fwd0<NX, NY, NZ>(L.T[0], r, L.twz, tid);
  __syncthreads();
  V v[D::IZ1][D::MZB];
  z_fwd1<NX, NY, NZ>(L.T[0], v, tid);
#pragma unroll
  for (int i = 0; i < D::IZ1; ++i) {
    const int b = tid + i * kThreadsZ;
    const int col = b % D::TY, mb = b / D::TY;
#pragma unroll
    for (int k1 = 0; k1 < D::MZB; ++k1) {
      const int q = D::MZB * mb + k1;
      if (b < D::NZ1) {
        v[i][k1] = cmul(cscale(v[i][k1], kappa_n(hx, L.hy[col], L.hz[q], inv_ntot)), cmul(L.my[col], L.mz[q]));
      }
    }
  }
  z_inv1<NX, NY, NZ>(L.T[0], v, tid);
  __syncthreads();
  z_inv0_store<NX, NY, NZ>(L.T[0], H, kx, p0, L.twz, tid);
}

// ---- slab pairs -----------------------------------------------------------------
// The velocity passes have three components per slab, six 2D transforms. With
// one workgroup per CU (the FP64 slab fills the LDS), 3 nz workgroups of two
// transforms would take two rounds on 256 CUs; instead 2 nz workgroups take
// three transforms each: half 0 of slab z does the C2R and update of the z
// component and the whole x component, half 1 the whole y component and then
// the R2C of the z component, from the field half 0 handed over through
// global memory (flag per slab, tagged with the launch's epoch). The two
// halves of a slab are block ids 8 apart (same XCD). All 2 nz <= 256
// workgroups of a launch fit on the chip at once; and should fewer fit (other
// work holding CUs), the producer of a slab has the lower block id, so it was
// dispatched before its consumer and, never waiting itself, finishes: the wait
// ends either way. It is bounded anyway, and on a time-out the half writes NaN
// (caught downstream) instead of hanging.
constexpr int kHandoffSpin = 1 << 18;   // x ~128 cycles: ~14 ms

__device__ __forceinline__ void slab_pair_of_block(int b, int& z, int& half) {
  z = (b >> 4) * 8 + (b & 7);
  half = (b >> 3) & 1;
}

// The handed-over slab is written and read with system-coherent accesses
// (write-through to the point of coherence, no cache on the way back), so the
// hand-off needs no cache write-back or invalidation: the producer waits for its
// stores to complete, then raises the flag; the consumer polls the flag and
// reads the slab the same way.
__device__ __forceinline__ void st_coherent(float2* p, float2 v) {
  unsigned long long x;
  __builtin_memcpy(&x, &v, sizeof(x));
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ float2 ld_coherent(const float2* p) {
  const unsigned long long x =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  float2 v;
  __builtin_memcpy(&v, &x, sizeof(v));
  return v;
}

__device__ __forceinline__ void handoff_publish(unsigned* flag, unsigned epoch) {
  __builtin_amdgcn_s_waitcnt(0);   // this thread's coherent stores have completed
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Returns false on a time-out. Ends with a workgroup barrier.
__device__ __forceinline__ bool handoff_wait(const unsigned* flag, unsigned epoch) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int it = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != epoch && ++it < kHandoffSpin)
      __builtin_amdgcn_s_sleep(2);
    s_ok = it < kHandoffSpin;
  }
  __syncthreads();
  return s_ok != 0;
}

// Coherent read of a real slab in the register layout (the consumer side).
template <int NX, int NY, int NZ>
__device__ __forceinline__ void load_real_coherent(RealRegs<NX, NY, NZ>& r, const float2* src, int tid) {
  using D = Dims<NX, NY, NZ>;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) r[i][m] = ld_coherent(src + it.pair(m));
    }
  }
}

// C2R of component xi's spectrum slab, the velocity update, and the R2C input
// in w (register layout). ADJ = false (forward): src = Q (x, y: times the kx or
// ky_pos derivative factor) or Gz; u <- a (a u - dt/rho0 g), w = new u.
// ADJ = true: src = W_xi; uh = u^ + dt rho0 g, u^ <- a^2 uh, w = a uh.
// Starts with the table loads (caller makes sure LDS is free); no barrier at the end.
template <int NX, int NY, int NZ, typename V, bool ADJ, bool COH = false>
__device__ __forceinline__ void u_c2r_update(SlabLds<NX, NY, NZ, V>& L, const float2* src, int xi, int z,
                                             const WaveBuffers& B, const WaveTables& t, const WaveScalars& sc,
                                             int init, RealRegs<NX, NY, NZ>& w, int tid) {
  using D = Dims<NX, NY, NZ>;
  const auto& tab = TabSel<V>::get(t);
  const int mode = ADJ || xi == 2 ? 0 : xi + 1;
  float2* u = reinterpret_cast<float2*>(B.u[xi]) + (size_t)z * D::SLAB_P;
  YRegs<NX, NY, NZ> ry;
  y_load<NX, NY, NZ>(ry, src + (size_t)z * D::SLAB_C, tid);
  float2 uo[D::IX0][D::RX0];
  if (ADJ || !init) load_real<NX, NY, NZ>(uo, u, tid);   // in flight during the transform
  load_slab_tables(L, t, xi == 0 ? t.ax : nullptr, xi == 1 ? t.ay : nullptr,
                   mode == 1 ? tab.mpx : (mode == 2 ? tab.mpy : (const V*)nullptr), mode, tid);
  const float azz = t.az[z];
  __syncthreads();
  y_inverse(L, ry, mode, tab.tw_y, tid);
  x_inverse_to_regs(L, w, tid);
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) {
        const int n = it.n(m);
        float a0, a1;
        if (xi == 0) { a0 = L.px[2 * n]; a1 = L.px[2 * n + 1]; }
        else if (xi == 1) { a0 = a1 = L.py[it.y]; }
        else { a0 = a1 = azz; }
        const float2 g = w[i][m];
        if (!ADJ) {
          const float2 o = init ? make_float2(g.x * sc.half_dt_over_rho0, g.y * sc.half_dt_over_rho0) : uo[i][m];
          const float2 un = make_float2(a0 * (a0 * o.x - sc.dt_over_rho0 * g.x), a1 * (a1 * o.y - sc.dt_over_rho0 * g.y));
          if (COH) st_coherent(u + it.pair(m), un);   // handed over to the partner block
          else u[it.pair(m)] = un;
          w[i][m] = un;
        } else {
          const float2 uh = make_float2(uo[i][m].x + sc.dt_rho0 * g.x, uo[i][m].y + sc.dt_rho0 * g.y);
          u[it.pair(m)] = make_float2(a0 * a0 * uh.x, a1 * a1 * uh.y);
          w[i][m] = make_float2(a0 * uh.x, a1 * uh.y);
        }
      }
    }
  }
}

// Velocity pass of the forward step (see "slab pairs"): U_x, U_y and, in place
// of Gz, U_z = R2C of the new velocity components.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_fwd_u(const float2* __restrict__ Q, float2* Gz, float2* Ux,
                                                        float2* Uy, WaveBuffers B, WaveTables t, WaveScalars sc,
                                                        int init, unsigned* flags, unsigned epoch) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const auto& twy = TabSel<V>::get(t).tw_y;
  const int tid = threadIdx.x;
  int z, half;
  slab_pair_of_block(blockIdx.x, z, half);
  const size_t cz = (size_t)z * D::SLAB_C;
  float2 w[D::IX0][D::RX0];
  if (half == 0) {
    u_c2r_update<NX, NY, NZ, V, false, true>(L, Gz, 2, z, B, t, sc, init, w, tid);
    handoff_publish(flags + z, epoch);
    u_c2r_update<NX, NY, NZ, V, false>(L, Q, 0, z, B, t, sc, init, w, tid);
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, Ux + cz, twy, tid);
  } else {
    u_c2r_update<NX, NY, NZ, V, false>(L, Q, 1, z, B, t, sc, init, w, tid);
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, Uy + cz, twy, tid);
    const bool ok = handoff_wait(flags + z, epoch);
    load_real_coherent<NX, NY, NZ>(w, reinterpret_cast<const float2*>(B.u[2]) + (size_t)z * D::SLAB_P, tid);
    if (!ok) {
#pragma unroll
      for (int i = 0; i < D::IX0; ++i)
#pragma unroll
        for (int m = 0; m < D::RX0; ++m) w[i][m] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, Gz + cz, twy, tid);
  }
}

// Density update of slab z = blockIdx.x / 2. The slab's work is split over two
// blocks so that 2 nz blocks of at most three 2D transforms replace nz blocks
// of four: block half 0 updates rho_x, rho_y and writes Pa = R2C(c0^2 (rho_x +
// rho_y)); half 1 updates rho_z and writes Pb = R2C(c0^2 rho_z). The pencil pass
// of the gradient sums Pa + Pb = FFT_xy(p), p = c0^2 sum rho; the sensor plane
// contributions go to plane_a / plane_b (summed after the run). The sums are
// formed from the new components as stored (each thread re-reads its own
// values), which keeps the transforms free of a live accumulator.
// TR: time reversal (eq. TRnum): on the slab z = 0 the density components are set to
// dir / (3 c0^2) (the datum imposed on the detection plane, a Dirichlet condition)
// instead of being updated, and, if p_a / p_b are given, each half stores its part of
// the real pressure (half 0: c0^2 (rho_x + rho_y), half 1: c0^2 rho_z).
template <int NX, int NY, int NZ, typename V, bool TR = false>
__global__ __launch_bounds__(kThreadsSlab) void k_fwd_rho(const float2* H0, const float2* H1, const float2* H2,
                                                          WaveBuffers B, float2* Pa, float2* Pb,
                                                          float* __restrict__ plane_a, float* __restrict__ plane_b,
                                                          WaveTables t, WaveScalars sc, const float* __restrict__ dir,
                                                          float* __restrict__ p_a, float* __restrict__ p_b) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x >> 1, half = blockIdx.x & 1, tid = threadIdx.x;
  const int xi0 = half == 0 ? 0 : 2, nxi = half == 0 ? 2 : 1;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  load_slab_tables(L, t, half == 0 ? t.bx : nullptr, half == 0 ? t.by : nullptr, (const V*)nullptr, 0, tid);
  const float bzz = t.bz[z];
#pragma unroll 1
  for (int c = 0; c < nxi; ++c) {
    const int xi = xi0 + c;
    const float2* H = xi == 0 ? H0 : (xi == 1 ? H1 : H2);
    float2* r = reinterpret_cast<float2*>(B.rho[xi]) + rz;
    // an opaque copy of the thread index: the LDS and global addresses of the
    // passes are recomputed per component instead of being kept live across the loop
    int tl = tid;
    asm volatile("" : "+v"(tl));
    YRegs<NX, NY, NZ> ry;
    y_load<NX, NY, NZ>(ry, H + cz, tl);
    __syncthreads();   // tables (first pass) / previous pass done with S
    y_inverse(L, ry, 0, TabSel<V>::get(t).tw_y, tl);
    float2 ro[D::IX0][D::RX0];
    load_real<NX, NY, NZ>(ro, r, tl);   // in flight during the x pass
    // rho update as the inverse transform's values come out (no array of them)
    x_inverse_apply(L, tl, [&](int i, int m, float2 h) {
      const RowItem<NX, NY, NZ> it(tl, i);
      const int n = it.n(m);
      float b0, b1;
      if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
      else if (xi == 1) { b0 = b1 = L.py[it.y]; }
      else { b0 = b1 = bzz; }
      float2 rn = make_float2(b0 * (b0 * ro[i][m].x - sc.dt_rho0 * h.x), b1 * (b1 * ro[i][m].y - sc.dt_rho0 * h.y));
      if constexpr (TR) {
        if (z == 0) {
          const float2 d = reinterpret_cast<const float2*>(dir)[it.pair(m)];
          rn = make_float2(d.x * sc.inv_3c2, d.y * sc.inv_3c2);
        }
      }
      r[it.pair(m)] = rn;
    });
  }
  float2 p[D::IX0][D::RX0], r1[D::IX0][D::RX0];
  load_real<NX, NY, NZ>(p, reinterpret_cast<const float2*>(B.rho[xi0]) + rz, tid);
  if (nxi == 2) load_real<NX, NY, NZ>(r1, reinterpret_cast<const float2*>(B.rho[1]) + rz, tid);
  float* plane = half == 0 ? plane_a : plane_b;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) {
        float2 v = p[i][m];
        if (nxi == 2) v = make_float2(v.x + r1[i][m].x, v.y + r1[i][m].y);
        if (B.c2f) {   // heterogeneous medium: p = c(x)^2 sum rho
          const float2 cc = reinterpret_cast<const float2*>(B.c2f)[rz + it.pair(m)];
          p[i][m] = make_float2(v.x * cc.x, v.y * cc.y);
        } else {
          p[i][m] = make_float2(v.x * sc.c2, v.y * sc.c2);
        }
        if (z == 0) reinterpret_cast<float2*>(plane)[it.pair(m)] = p[i][m];
        if constexpr (TR) {
          float* po = half == 0 ? p_a : p_b;
          if (po) reinterpret_cast<float2*>(po)[rz + it.pair(m)] = p[i][m];
        }
      }
    }
  }
  x_forward_from_regs(L, p, tid);
  y_forward_to_global(L, (half == 0 ? Pa : Pb) + cz, TabSel<V>::get(t).tw_y, tid);
}

// ---- adjoint kernels ---------------------------------------------------------

// rho^_xi = c0^2 S^T y^{nt-1}, u^_xi = 0, W_xi = R2C(b_xi rho^_xi).
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_adj_init(const float* __restrict__ ylast, WaveBuffers B,
                                                           WaveTables t, WaveScalars sc) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = kThreadsSlab;
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
  load_slab_tables(L, t, xi == 0 ? t.bx : nullptr, xi == 1 ? t.by : nullptr, (const V*)nullptr, 0, tid);
  const float bzz = t.bz[0];
  float2 v[D::IX0][D::RX0];
  load_real<NX, NY, NZ>(v, reinterpret_cast<const float2*>(ylast), tid);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) {
        const int n = it.n(m);
        const float2 r = make_float2(v[i][m].x * sc.c2, v[i][m].y * sc.c2);
        rb[it.pair(m)] = r;
        ub[it.pair(m)] = zero;
        float b0, b1;
        if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
        else if (xi == 1) { b0 = b1 = L.py[it.y]; }
        else { b0 = b1 = bzz; }
        v[i][m] = make_float2(b0 * r.x, b1 * r.y);
      }
    }
  }
  x_forward_from_regs(L, v, tid);
  y_forward_to_global(L, B.spec[xi] + cz, TabSel<V>::get(t).tw_y, tid);
}

// u^_xi: uh = u^ + dt rho0 Dplus_xi(b rho^) (the pencil pass already applied the
// multiplier), u^ <- a^2 uh, W_xi = R2C(a uh) in place, as slab pairs (see
// "slab pairs"; the z component's a uh is handed over in its own spectrum slab,
// which is free once half 0 has read it).
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_adj_u(WaveBuffers B, WaveTables t, WaveScalars sc,
                                                        unsigned* flags, unsigned epoch) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const auto& twy = TabSel<V>::get(t).tw_y;
  const int tid = threadIdx.x;
  int z, half;
  slab_pair_of_block(blockIdx.x, z, half);
  const size_t cz = (size_t)z * D::SLAB_C;
  float2* hand = reinterpret_cast<float2*>(B.spec[2] + cz);   // SLAB_P float2 fit in a SLAB_C slab
  float2 w[D::IX0][D::RX0];
  if (half == 0) {
    u_c2r_update<NX, NY, NZ, V, true>(L, B.spec[2], 2, z, B, t, sc, 0, w, tid);
#pragma unroll
    for (int i = 0; i < D::IX0; ++i) {
      const RowItem<NX, NY, NZ> it(tid, i);
      if (it.ok) {
#pragma unroll
        for (int m = 0; m < D::RX0; ++m) st_coherent(hand + it.pair(m), w[i][m]);
      }
    }
    handoff_publish(flags + z, epoch);
    u_c2r_update<NX, NY, NZ, V, true>(L, B.spec[0], 0, z, B, t, sc, 0, w, tid);
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, B.spec[0] + cz, twy, tid);
  } else {
    u_c2r_update<NX, NY, NZ, V, true>(L, B.spec[1], 1, z, B, t, sc, 0, w, tid);
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, B.spec[1] + cz, twy, tid);
    const bool ok = handoff_wait(flags + z, epoch);
    load_real_coherent<NX, NY, NZ>(w, hand, tid);
    if (!ok) {
#pragma unroll
      for (int i = 0; i < D::IX0; ++i)
#pragma unroll
        for (int m = 0; m < D::RX0; ++m) w[i][m] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
    __syncthreads();   // every lane has its a uh before the slab is overwritten
    x_forward_from_regs(L, w, tid);
    y_forward_to_global(L, B.spec[2] + cz, twy, tid);
  }
}

// Pencil pass of the summed divergence: out = IFFT_z[ sum_xi kappa/N i k_xi
// e^{-i k_xi dx/2} FFT_z(W_xi) ].
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsZ) void k_zdiv_sum(const float2* __restrict__ W0,
                                                        const float2* __restrict__ W1,
                                                        const float2* __restrict__ W2,
                                                        float2* __restrict__ out, WaveTables t,
                                                        float inv_ntot) {
  // The x and y factors do not depend on kz, so they are applied before the z
  // transform: out = IFFT_z[ kappa/N ( FFT_z(mx W0 + my W1) + mz FFT_z(W2) ) ],
  // two forward transforms instead of three.
  using D = Dims<NX, NY, NZ>;
  using Sc = typename ScalarOf<V>::T;
  __shared__ PencilLds<NX, NY, NZ, V, 1> L;
  const auto& tab = TabSel<V>::get(t);
  const int tid = threadIdx.x;
  const int kx = blockIdx.x / (NY / D::TY), p0 = (blockIdx.x % (NY / D::TY)) * D::TY;
  float2 r0[D::IZ0][D::RZ0], r1[D::IZ0][D::RZ0];
  z_load<NX, NY, NZ>(r0, W0, kx, p0, tid);
  z_load<NX, NY, NZ>(r1, W1, kx, p0, tid);
  load_pencil_tables(L, t, p0, mkc<V>((Sc)1, (Sc)0), tab.mmy, tab.mmz, tid);
  const Sc hx = tab.hx[kx];
  const V mxk = tab.mmx[kx];
  __syncthreads();
  {
    V a[D::IZ0][D::RZ0];
#pragma unroll
    for (int i = 0; i < D::IZ0; ++i) {
      const int b = tid + i * kThreadsZ;
      const V myc = L.my[b % D::TY];
#pragma unroll
      for (int m = 0; m < D::RZ0; ++m)
        a[i][m] = cadd(cmul(mxk, widen<V>(r0[i][m])), cmul(myc, widen<V>(r1[i][m])));
    }
    z_fwd0<NX, NY, NZ>(L.T[0], a, L.twz, tid);
  }
  // W2 in flight during the first transform's second stage (the memory clobber
  // keeps the loads after the first stage, whose registers they reuse)
  int tn = tid;
  asm volatile("" : "+v"(tn)::"memory");
  z_load<NX, NY, NZ>(r0, W2, kx, p0, tn);
  __syncthreads();
  V acc[D::IZ1][D::MZB];
  z_fwd1<NX, NY, NZ>(L.T[0], acc, tid);
  __syncthreads();
  z_fwd0<NX, NY, NZ>(L.T[0], r0, L.twz, tid);
  __syncthreads();
  V v[D::IZ1][D::MZB];
  z_fwd1<NX, NY, NZ>(L.T[0], v, tid);
#pragma unroll
  for (int i = 0; i < D::IZ1; ++i) {
    const int b = tid + i * kThreadsZ;
    const int col = b % D::TY, mb = (b / D::TY) % D::RZ0;
#pragma unroll
    for (int k1 = 0; k1 < D::MZB; ++k1) {
      const int q = D::MZB * mb + k1;
      acc[i][k1] = cscale(cadd(acc[i][k1], cmul(v[i][k1], L.mz[q])),
                          kappa_n(hx, L.hy[col], L.hz[q], inv_ntot));
    }
  }
  z_inv1<NX, NY, NZ>(L.T[0], acc, tid);
  __syncthreads();
  z_inv0_store<NX, NY, NZ>(L.T[0], out, kx, p0, L.twz, tid);
}

// rho^_xi <- b^2 rho^_xi + (c0^2 dt/rho0 q + c0^2 S^T y^n), q = C2R of the summed
// divergence Qs; then W_xi = R2C(b rho^_xi), or on the last (final != 0) step
// W_xi = R2C(u^_xi) for the initial-condition transpose. Slab z = blockIdx.x / 2
// is split over two blocks sharing the one C2R: half 0 does rho_x and rho_y
// (one C2R, two R2C), half 1 rho_z (one C2R, one R2C).
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_adj_rho(const float2* __restrict__ Qs, WaveBuffers B,
                                                          const float* __restrict__ yplane, WaveTables t,
                                                          WaveScalars sc, int final_step) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x >> 1, half = blockIdx.x & 1, tid = threadIdx.x;
  const int xi0 = half == 0 ? 0 : 2, nxi = half == 0 ? 2 : 1;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  YRegs<NX, NY, NZ> ry;
  y_load<NX, NY, NZ>(ry, Qs + cz, tid);
  float2 src[D::IX0][D::RX0];
  if (z == 0) load_real<NX, NY, NZ>(src, reinterpret_cast<const float2*>(yplane), tid);   // data source
  load_slab_tables(L, t, half == 0 ? t.bx : nullptr, half == 0 ? t.by : nullptr, (const V*)nullptr, 0, tid);
  const float bzz = t.bz[z];
  __syncthreads();
  y_inverse(L, ry, 0, TabSel<V>::get(t).tw_y, tid);
  float2 q[D::IX0][D::RX0];
  x_inverse_to_regs(L, q, tid);
  const float qs = sc.c2 * sc.dt_over_rho0;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i)
#pragma unroll
    for (int m = 0; m < D::RX0; ++m) {
      q[i][m] = make_float2(qs * q[i][m].x, qs * q[i][m].y);
      if (z == 0) q[i][m] = make_float2(q[i][m].x + sc.c2 * src[i][m].x, q[i][m].y + sc.c2 * src[i][m].y);
    }
#pragma unroll 1
  for (int c = 0; c < nxi; ++c) {
    const int xi = xi0 + c;
    int tl = tid;   // opaque copy: addresses are recomputed per component, not kept live
    asm volatile("" : "+v"(tl));
    float2* rb = reinterpret_cast<float2*>(B.rho[xi]) + rz;
    float2 ro[D::IX0][D::RX0], w[D::IX0][D::RX0];
    load_real<NX, NY, NZ>(ro, rb, tl);
    if (c > 0) __syncthreads();   // the previous component's y pass is done with S
#pragma unroll
    for (int i = 0; i < D::IX0; ++i) {
      const RowItem<NX, NY, NZ> it(tl, i);
      if (it.ok) {
#pragma unroll
        for (int m = 0; m < D::RX0; ++m) {
          const int n = it.n(m);
          float b0, b1;
          if (xi == 0) { b0 = L.px[2 * n]; b1 = L.px[2 * n + 1]; }
          else if (xi == 1) { b0 = b1 = L.py[it.y]; }
          else { b0 = b1 = bzz; }
          const float2 rn = make_float2(b0 * b0 * ro[i][m].x + q[i][m].x, b1 * b1 * ro[i][m].y + q[i][m].y);
          rb[it.pair(m)] = rn;
          w[i][m] = make_float2(b0 * rn.x, b1 * rn.y);
        }
      }
    }
    // last step: the initial-condition transpose needs R2C(u^) instead (read once per adjoint)
    if (final_step) load_real<NX, NY, NZ>(w, reinterpret_cast<const float2*>(B.u[xi]) + rz, tl);
    x_forward_from_regs(L, w, tl);
    y_forward_to_global(L, B.spec[xi] + cz, TabSel<V>::get(t).tw_y, tl);
  }
}

// p = (rho^_x + rho^_y + rho^_z)/(3 c0^2) - dt/(2 rho0) sum_xi Dminus_xi u^_xi.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_adj_final(const float2* __restrict__ Qs, WaveBuffers B,
                                                            float* __restrict__ pout, WaveTables t,
                                                            WaveScalars sc, int with_velocity) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int z = blockIdx.x, tid = threadIdx.x;
  const size_t cz = (size_t)z * D::SLAB_C, rz = (size_t)z * D::SLAB_P;
  float2 g[D::IX0][D::RX0];
  if (with_velocity) {
    YRegs<NX, NY, NZ> ry;
    y_load<NX, NY, NZ>(ry, Qs + cz, tid);
    load_slab_tables(L, t, nullptr, nullptr, (const V*)nullptr, 0, tid);
    __syncthreads();
    y_inverse(L, ry, 0, TabSel<V>::get(t).tw_y, tid);
    x_inverse_to_regs(L, g, tid);
  }
  float2 r0[D::IX0][D::RX0], r1[D::IX0][D::RX0], r2[D::IX0][D::RX0];
  load_real<NX, NY, NZ>(r0, reinterpret_cast<const float2*>(B.rho[0]) + rz, tid);
  load_real<NX, NY, NZ>(r1, reinterpret_cast<const float2*>(B.rho[1]) + rz, tid);
  load_real<NX, NY, NZ>(r2, reinterpret_cast<const float2*>(B.rho[2]) + rz, tid);
  float2* p = reinterpret_cast<float2*>(pout) + rz;
#pragma unroll
  for (int i = 0; i < D::IX0; ++i) {
    const RowItem<NX, NY, NZ> it(tid, i);
    if (it.ok) {
#pragma unroll
      for (int m = 0; m < D::RX0; ++m) {
        float2 v = make_float2((r0[i][m].x + r1[i][m].x + r2[i][m].x) * sc.inv_3c2,
                               (r0[i][m].y + r1[i][m].y + r2[i][m].y) * sc.inv_3c2);
        if (with_velocity) {
          v.x -= sc.half_dt_over_rho0 * g[i][m].x;
          v.y -= sc.half_dt_over_rho0 * g[i][m].y;
        }
        p[it.pair(m)] = v;
      }
    }
  }
}

// ---- plain batched slab transforms (used by the line propagator) -----------------

// out[b] = scale * R2C_xy(in[b]) for slab b = blockIdx.x: real [NY][NX] -> [NX/2+1][ky_pos].
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_slab_r2c(const float* __restrict__ in, float2* out, float scale,
                                                           WaveTables t) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int tid = threadIdx.x;
  const size_t b = blockIdx.x;
  load_slab_tables(L, t, nullptr, nullptr, (const V*)nullptr, 0, tid);
  float2 v[D::IX0][D::RX0];
  load_real<NX, NY, NZ>(v, reinterpret_cast<const float2*>(in) + b * D::SLAB_P, tid);
#pragma unroll
  for (int i = 0; i < D::IX0; ++i)
#pragma unroll
    for (int m = 0; m < D::RX0; ++m) v[i][m] = make_float2(v[i][m].x * scale, v[i][m].y * scale);
  __syncthreads();
  x_forward_from_regs(L, v, tid);
  y_forward_to_global(L, out + b * D::SLAB_C, TabSel<V>::get(t).tw_y, tid);
}

// out[b] = scale * C2R_xy(in[b]) (unnormalised inverse) for slab b = blockIdx.x.
template <int NX, int NY, int NZ, typename V>
__global__ __launch_bounds__(kThreadsSlab) void k_slab_c2r(const float2* __restrict__ in, float* out, float scale,
                                                           WaveTables t) {
  using D = Dims<NX, NY, NZ>;
  __shared__ SlabLds<NX, NY, NZ, V> L;
  const int tid = threadIdx.x;
  const size_t b = blockIdx.x;
  YRegs<NX, NY, NZ> ry;
  y_load<NX, NY, NZ>(ry, in + b * D::SLAB_C, tid);
  load_slab_tables(L, t, nullptr, nullptr, (const V*)nullptr, 0, tid);
  __syncthreads();
  y_inverse(L, ry, 0, TabSel<V>::get(t).tw_y, tid);
  float2* o = reinterpret_cast<float2*>(out) + b * D::SLAB_P;
  x_inverse_apply(L, tid, [&](int i, int m, float2 v) {
    const RowItem<NX, NY, NZ> it(tid, i);
    o[it.pair(m)] = make_float2(v.x * scale, v.y * scale);
  });
}

template <int N>
hipError_t slab_r2c_n(const float* in, float2* out, int nb, float scale, const WaveTables& t, hipStream_t st) {
  k_slab_r2c<N, N, N, double2><<<nb, kThreadsSlab, 0, st>>>(in, out, scale, t);
  return hipGetLastError();
}
template <int N>
hipError_t slab_c2r_n(const float2* in, float* out, int nb, float scale, const WaveTables& t, hipStream_t st) {
  k_slab_c2r<N, N, N, double2><<<nb, kThreadsSlab, 0, st>>>(in, out, scale, t);
  return hipGetLastError();
}

hipError_t launch_slab_r2c(int n, const float* in, float2* out, int nb, float scale, const WaveTables& t,
                           hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  switch (n) {
    case 16: return slab_r2c_n<16>(in, out, nb, scale, t, st);
    case 32: return slab_r2c_n<32>(in, out, nb, scale, t, st);
    case 64: return slab_r2c_n<64>(in, out, nb, scale, t, st);
    case 96: return slab_r2c_n<96>(in, out, nb, scale, t, st);
    case 128: return slab_r2c_n<128>(in, out, nb, scale, t, st);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_slab_c2r(int n, const float2* in, float* out, int nb, float scale, const WaveTables& t,
                           hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  switch (n) {
    case 16: return slab_c2r_n<16>(in, out, nb, scale, t, st);
    case 32: return slab_c2r_n<32>(in, out, nb, scale, t, st);
    case 64: return slab_c2r_n<64>(in, out, nb, scale, t, st);
    case 96: return slab_c2r_n<96>(in, out, nb, scale, t, st);
    case 128: return slab_c2r_n<128>(in, out, nb, scale, t, st);
    default: return hipErrorInvalidValue;
  }
}

// ---- launch sequences ----------------------------------------------------------

inline unsigned next_epoch(HandOff& ho) {   // never 0, the value of a cleared flag
  if (++ho.epoch == 0) ho.epoch = 1;
  return ho.epoch;
}

template <int NX, int NY, int NZ, typename V>
hipError_t wave_forward(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* p0, float* planes, int nt, hipStream_t st, KernelTimer* kt, HandOff& ho) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = kThreadsSlab;
  const size_t npix = (size_t)NX * NY;
  k_fwd_init<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(p0, B, planes, planes + (size_t)nt * npix, t, sc);
  for (int n = 0; n < nt - 1; ++n) {
    timed(kt, K_ZGRAD, st, [&] {
      k_zgrad<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], n == 0 ? 1 : 2, B.spec[0],
                                                             B.spec[1], t, sc.inv_ntot);
    });
    timed(kt, K_FWD_U, st, [&] {
      k_fwd_u<NX, NY, NZ, V><<<2 * NZ, NT, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], B, t, sc,
                                                     n == 0 ? 1 : 0, ho.flags, next_epoch(ho));
    });
    timed(kt, K_ZDIV, st, [&] {
      k_zmul<NX, NY, NZ, V, false><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], t,
                                                                             sc.inv_ntot);
    });
    timed(kt, K_FWD_RHO, st, [&] {
      k_fwd_rho<NX, NY, NZ, V><<<2 * NZ, NT, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], B, B.spec[0], B.spec[1],
                                                       planes + (size_t)(n + 1) * npix,
                                                       planes + (size_t)(nt + n + 1) * npix, t, sc, nullptr, nullptr,
                                                       nullptr);
    });
  }
  return hipGetLastError();
}

template <int NX, int NY, int NZ, typename V>
hipError_t wave_adjoint(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B,
                        const float* planes, float* p, int nt, hipStream_t st, KernelTimer* kt, HandOff& ho) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = kThreadsSlab;
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
    timed(kt, K_ADJ_U, st, [&] {
      k_adj_u<NX, NY, NZ, V><<<2 * NZ, NT, 0, st>>>(B, t, sc, ho.flags, next_epoch(ho));
    });
    timed(kt, K_ZDIV_SUM, st, [&] {
      k_zdiv_sum<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                                sc.inv_ntot);
    });
    timed(kt, K_ADJ_RHO, st, [&] {
      k_adj_rho<NX, NY, NZ, V><<<2 * NZ, NT, 0, st>>>(B.spec[3], B, planes + (size_t)n * npix, t, sc,
                                                      n == 0 ? 1 : 0);
    });
  }
  k_zdiv_sum<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], t,
                                                            sc.inv_ntot);
  k_adj_final<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(B.spec[3], B, p, t, sc, 1);
  return hipGetLastError();
}

// Time reversal (eq. TRnum): the forward recurrence from zero fields with the reversed
// plane series imposed on z = 0 (k_fwd_rho<TR>). planes: [nt][ny][nx] (y^0 .. y^(nt-1));
// vol: a scratch volume; p_a, p_b: the two halves of the final pressure (p = p_a + p_b;
// for nt = 1 the pressure is vol itself); tplanes: 2 scratch planes.
template <int NX, int NY, int NZ, typename V>
hipError_t wave_time_reversal(const WaveTables& t, const WaveScalars& sc, const WaveBuffers& B, const float* planes,
                              float* vol, float* p_a, float* p_b, float* tplanes, int nt, hipStream_t st,
                              HandOff& ho) {
  using D = Dims<NX, NY, NZ>;
  constexpr int NT = kThreadsSlab;
  const size_t npix = (size_t)NX * NY, nvox = npix * NZ;
  hipError_t e = hipSuccess;
  for (int xi = 0; xi < 3 && e == hipSuccess; ++xi) e = hipMemsetAsync(B.u[xi], 0, nvox * sizeof(float), st);
  if (e == hipSuccess) e = hipMemsetAsync(vol, 0, nvox * sizeof(float), st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(vol, planes + (size_t)(nt - 1) * npix, npix * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  // fields zero except rho_xi = y^(nt-1) / (3 c0^2) on the plane; P^ = FFT of that pressure
  k_fwd_init<NX, NY, NZ, V><<<NZ, NT, 0, st>>>(vol, B, tplanes, tplanes + npix, t, sc);
  for (int n = 0; n < nt - 1; ++n) {
    const bool last = n + 1 == nt - 1;
    k_zgrad<NX, NY, NZ, V><<<D::NTILE, kThreadsZ, 0, st>>>(B.spec[0], B.spec[1], n == 0 ? 1 : 2, B.spec[0],
                                                           B.spec[1], t, sc.inv_ntot);
    k_fwd_u<NX, NY, NZ, V><<<2 * NZ, NT, 0, st>>>(B.spec[0], B.spec[1], B.spec[2], B.spec[3], B, t, sc, 0, ho.flags,
                                                   next_epoch(ho));
    k_zmul<NX, NY, NZ, V, false><<<dim3(D::NTILE, 3), kThreadsZ, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], t,
                                                                           sc.inv_ntot);
    k_fwd_rho<NX, NY, NZ, V, true><<<2 * NZ, NT, 0, st>>>(B.spec[2], B.spec[3], B.spec[1], B, B.spec[0], B.spec[1],
                                                           tplanes, tplanes + npix, t, sc,
                                                           planes + (size_t)(nt - 2 - n) * npix,
                                                           last ? p_a : nullptr, last ? p_b : nullptr);
  }
  return hipGetLastError();
}

#define PAT_WAVE_IMPL(N)                                                            \
  {N, N, N, {&wave_forward<N, N, N, float2>, &wave_forward<N, N, N, double2>},     \
   {&wave_adjoint<N, N, N, float2>, &wave_adjoint<N, N, N, double2>},              \
   {&wave_time_reversal<N, N, N, float2>, &wave_time_reversal<N, N, N, double2>}}

static const WaveImpl kWaveImpls[] = {
    PAT_WAVE_IMPL(16),
    PAT_WAVE_IMPL(32),
    PAT_WAVE_IMPL(64),
    PAT_WAVE_IMPL(96),
    PAT_WAVE_IMPL(128),
};

const WaveImpl* find_wave_impl(int nx, int ny, int nz) {
  for (const auto& w : kWaveImpls)
    if (w.nx == nx && w.ny == ny && w.nz == nz) return &w;
  return nullptr;
}

}  // namespace pat
