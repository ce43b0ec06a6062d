// Line propagator for gfx950: one kernel launch per time step runs every line
// of all three field components (see line_common.hpp for the scheme of
// Sec. 4.3 in mixed spaces, the layouts and the hub).
//
// A block of 128 threads (two waves) owns a tile of 16 lines of one axis. Each
// 1D transform of length N = R0 M is the two-stage split of fft_radix.hpp; a
// thread owns one stage-0 butterfly (R0 values at points n1 + M m of one line)
// or two stage-1 butterflies (M values at positions M mb + k1, frequency
// mb + R0 k1), with all arithmetic FP64 in registers, and the tile T in LDS is
// the exchange between the stages ([point][line], 16 lines per row), stored
// as FP32 pairs by default (the rounding is of the same size as that of the
// FP32 states in HBM; FP64 storage doubles the LDS and costs occupancy). The time step
// of a component is inverse - update - forward - multiply - inverse - update -
// forward: four transforms and four LDS crossings; the updates run in the
// stage-0 layout, where a thread holds natural points, and the multipliers in
// the stage-1 layout, where it holds frequencies. HBM traffic per component and
// step: its lines of the three component spectra of the hub (summed in FP64),
// both states in and out (each N^3/2 complex values), and its output spectrum
// (8 (N/2+1) N^2 bytes, conjugate partners included).
#include <type_traits>

#include "fft_radix.hpp"
#include "kspace.hpp"
#include "line_common.hpp"

namespace pat {

constexpr int kLT = 16;          // lines per tile
constexpr int kThreadsL = 128;   // threads per tile block

// First position of a run of N/2 - 1 consecutive positions (order of the
// forward transform) that holds one frequency of every pair (q, -q) with
// q != 0, N/2; -1 if there is none.
__host__ __device__ constexpr int kept_run_start(int n) {
  for (int ks = 0; ks + n / 2 - 1 <= n; ++ks) {
    bool ok = true;
    for (int i = 0; i < n / 2 - 1 && ok; ++i) {
      const int q = fft_freq(n, ks + i);
      if (q == 0 || q == n / 2) ok = false;
      for (int j = 0; j < i && ok; ++j)
        if (fft_freq(n, ks + j) == (n - q) % n) ok = false;
    }
    if (ok) return ks;
  }
  return -1;
}

template <int N>
struct LD {
  static constexpr int H = N / 2, NK = H + 1;
  static constexpr int R0 = fft_radix(N, 0), M = N / R0;
  static constexpr int NL = NK * N;          // z lines (kx <= N/2, ky) of the z transform kernels
  static constexpr int NTILE = NL / kLT;     // their tiles
  // Line slots of a step (per axis): the planes P = 1..N/2-1 of the half
  // coordinate in full, the two self-conjugate planes P = 0, N/2 by half (the
  // other half is conjugate), and their four real lines in pairs: N^2/2 slots.
  static constexpr int NS = N * N / 2;
  static constexpr int NREG = (H - 1) * N;   // slots of the regular planes
  static constexpr int NT = NS / kLT;        // step tiles per axis
  static constexpr int KS = kept_run_start(N);
  static constexpr int N0 = kLT * M, I0 = cdiv(N0, kThreadsL);    // stage-0 butterflies per tile
  static constexpr int N1 = kLT * R0, I1 = cdiv(N1, kThreadsL);   // stage-1 butterflies per tile
  static_assert(N % kLT == 0 && NL % kLT == 0 && NS % kLT == 0, "a tile is 16 lines");
  static_assert(KS >= 0, "a contiguous run of kept positions");
};

// PAT_LINE_LDS_F32: tile stored as FP32 (1) or FP64 (0) pairs.
// PAT_LINE_WAVES: minimum waves per SIMD asked of the register allocator (the
// step kernels need about 136 VGPRs, which gives three).
#ifndef PAT_LINE_LDS_F32
#define PAT_LINE_LDS_F32 1
#endif
constexpr bool kTF32 = PAT_LINE_LDS_F32 != 0;
#ifndef PAT_LINE_WAVES
#define PAT_LINE_WAVES 3
#endif
using TStore = std::conditional_t<kTF32, float2, double2>;

// Per-block copy of the small tables (LDS), so the phases after the first
// read them without a global round trip.
struct LTab {
  const double* h;     // (c0 dt / 2) k by natural index
  const double2* mp;   // i k exp(+i k dx/2)
  const double2* mm;   // i k exp(-i k dx/2)
  const double2* tw;   // exp(-2 pi i j / N)
  const float* a;      // PML factors of this block's axis
  const float* b;
};

template <int N>
struct LineLds {
  TStore T[N * kLT];   // value of tile line l at point (or position) j: T[j * 16 + l]
  double h[N];
  double2 mp[N], mm[N], tw[N];
  float a[N], b[N];
  float2 X[2][N];      // spectra of the two packed slots (last tile), natural frequency order
};

__device__ __forceinline__ void tput(float2& d, double2 v) { d = narrow(v); }
__device__ __forceinline__ void tput(double2& d, double2 v) { d = v; }
__device__ __forceinline__ double2 tget(const float2& d) { return widen<double2>(d); }
__device__ __forceinline__ double2 tget(const double2& d) { return d; }

// hub index of (kz, kx, ky_pos)
template <int N>
__device__ __forceinline__ int hidx(int kz, int kx, int kyp) {
  return (kz * LD<N>::NK + kx) * N + kyp;
}

// The fixed coordinates of the line in state slot lg. Each axis has a half
// coordinate P <= N/2 (x lines: kz; y and z lines: kx) and a full one Q (x and
// z lines: ky_pos; y lines: kz).
//   regular slots (P = 1..N/2-1): x, z: lg = (P-1) N + ky_pos; y: lg = kz (N/2-1) + P-1
//   P = 0 and P = N/2: only one line of each conjugate pair (Q, -Q), Q in the run
//     KS.. of positions (x, z) or kz = 1..N/2-1 (y); the line also writes the
//     outputs of its partner (kind 1)
//   last two slots: the real lines (P, 0) and (P, N/2) of P = 0 and P = N/2,
//     packed as line + i * second line (kind 2)
// An x line that is not real also writes the conjugates of its kx = 0 and
// kx >= N/2 outputs at (-kx, -ky, -kz) (the hub holds kx <= N/2 only).
template <int N, int AX>
struct LineGeo {
  int lg, kx, kyp, kz, kyf, kyn;   // kyf: natural ky of ky_pos, kyn: ky_pos of -ky
  int kind;                        // 0 regular, 1 one of a conjugate pair, 2 packed real pair
  __device__ __forceinline__ void set(int P, int Q) {
    if (AX == 0) { kz = P; kyp = Q; kx = 0; }
    else if (AX == 1) { kx = P; kz = Q; kyp = 0; }
    else { kx = P; kyp = Q; kz = 0; }
    kyf = fft_freq(N, kyp);
    kyn = fft_pos(N, (N - kyf) % N);
  }
  __device__ __forceinline__ explicit LineGeo(int slot) {
    using D = LD<N>;
    lg = slot;
    int P, Q;
    if (slot < D::NREG) {
      kind = 0;
      if (AX == 1) { P = 1 + slot % (D::H - 1); Q = slot / (D::H - 1); }
      else { P = 1 + slot / N; Q = slot % N; }
    } else if (slot < D::NS - 2) {
      kind = 1;
      const int j = slot - D::NREG, i = j % (D::H - 1);
      P = j < D::H - 1 ? 0 : D::H;
      Q = AX == 1 ? 1 + i : D::KS + i;
    } else {
      kind = 2;
      P = slot == D::NS - 2 ? 0 : D::H;
      Q = 0;
    }
    set(P, Q);
  }
  // a z line of the z transform kernels: lg = kx N + ky_pos
  __device__ __forceinline__ static LineGeo zline(int lg) {
    LineGeo g;
    g.lg = lg;
    g.kind = 0;
    g.set(lg / N, lg % N);
    return g;
  }
  // the second line of a packed slot: the same P, natural Q = N/2
  __device__ __forceinline__ LineGeo second() const {
    LineGeo g = *this;
    g.set(AX == 0 ? kz : kx, AX == 1 ? N / 2 : fft_pos(N, N / 2));
    return g;
  }
  LineGeo() = default;
  // the part of the squared sinc argument that the fixed coordinates contribute
  __device__ __forceinline__ double s0(const double* h) const {
    double ha, hb;
    if (AX == 0) { ha = h[kyf]; hb = h[kz]; }
    else if (AX == 1) { ha = h[kx]; hb = h[kz]; }
    else { ha = h[kx]; hb = h[kyf]; }
    return ha * ha + hb * hb;
  }
};

__device__ __forceinline__ double kappa_at(const double* h, double s0, int f) {
  const double hf = h[f];
  return sinc_of_sq(s0 + hf * hf);
}

// Hub index of frequency f (natural) / position p along the line; x lines read
// kx > N/2 as the conjugate at (-kx, -ky, -kz) (cj set).
template <int N, int AX>
__device__ __forceinline__ int hub_addr(const LineGeo<N, AX>& g, int f, int p, bool& cj) {
  using D = LD<N>;
  cj = false;
  if (AX == 0) {
    if (f <= D::H) return hidx<N>(g.kz, f, g.kyp);
    cj = true;
    return hidx<N>((N - g.kz) % N, N - f, g.kyn);
  }
  if (AX == 1) return hidx<N>(g.kz, g.kx, p);
  return hidx<N>(f, g.kx, g.kyp);
}

// Index into the plane spectrum S[kx][ky_pos] (adjoint source, the same for every kz).
template <int N, int AX>
__device__ __forceinline__ int src_addr(const LineGeo<N, AX>& g, int f, int p, bool& cj) {
  using D = LD<N>;
  cj = false;
  if (AX == 0) {
    if (f <= D::H) return f * N + g.kyp;
    cj = true;
    return (N - f) * N + g.kyn;
  }
  if (AX == 1) return g.kx * N + p;
  return g.kx * N + g.kyp;
}

// Sum of nh component spectra at frequency f / position p along the line.
template <int N, int AX>
__device__ __forceinline__ double2 hub_sum(const float2* const* h, int nh, const LineGeo<N, AX>& g, int f, int p) {
  bool cj;
  const int idx = hub_addr<N, AX>(g, f, p, cj);
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

// Store the value of frequency f / position p of the line into a component
// spectrum. The partner line (-Q at -P) of an x line that is not real owns no
// slot: its outputs are the conjugates at (-kx, -ky, -kz), written for kx = 0
// or kx >= N/2 (the x lines hold kx <= N/2). y and z lines of kind 1 write
// their partner's line, the conjugate at (-ky or -kz reversed) too.
template <int N, int AX>
__device__ __forceinline__ void hub_store(float2* out, const LineGeo<N, AX>& g, int f, int p, double2 v) {
  using D = LD<N>;
  const float2 vc = make_float2((float)v.x, (float)-v.y);
  if (AX == 0) {
    if (f <= D::H) out[hidx<N>(g.kz, f, g.kyp)] = narrow(v);
    if (g.kind != 2 && (f == 0 || f >= D::H)) out[hidx<N>((N - g.kz) % N, (N - f) % N, g.kyn)] = vc;
  } else if (AX == 1) {
    out[hidx<N>(g.kz, g.kx, p)] = narrow(v);
    if (g.kind == 1) out[hidx<N>((N - g.kz) % N, g.kx, fft_pos(N, (N - f) % N))] = vc;
  } else {
    out[hidx<N>(f, g.kx, g.kyp)] = narrow(v);
    if (g.kind == 1) out[hidx<N>((N - f) % N, g.kx, g.kyn)] = vc;
  }
}

// Element (point n1 + M m, line lg) of a [point][line] state as a wave-uniform
// base per m plus one 32-bit lane offset, so the 16 points of a stage-0
// butterfly share one address register.
template <int N>
struct StateAt {
  unsigned off;
  __device__ __forceinline__ StateAt(int n1, int lg) : off((unsigned)(n1 * LD<N>::NS + lg) * 8u) {}
  template <typename P>
  __device__ __forceinline__ P* operator()(P* base, int m) const {
    return reinterpret_cast<P*>(reinterpret_cast<char*>(base + (size_t)(LD<N>::M * m) * LD<N>::NS) + off);
  }
};

// Stage-0 twiddles w^(n1 k), k = 1..R-1, from w = tw[n1] by repeated multiplication.
template <int R, bool INV>
__device__ __forceinline__ void twiddle_pow(double2* a, double2 w) {
  double2 wk = w;
#pragma unroll
  for (int k = 1; k < R; ++k) {
    a[k] = INV ? cmulconj(a[k], wk) : cmul(a[k], wk);
    if (k + 1 < R) wk = cmul(wk, w);
    // in order: otherwise all R - 1 powers are formed first and held in registers
    __builtin_amdgcn_sched_barrier(0);
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

// stage-1 values (after an inverse stage-1 DFT) -> T
template <int N>
__device__ __forceinline__ void s1_to_T(LineLds<N>& L, const double2* v, int l, int mb) {
  using D = LD<N>;
#pragma unroll
  for (int n1 = 0; n1 < D::M; ++n1) tput(L.T[(D::M * mb + n1) * kLT + l], v[n1]);
}

// T -> stage-1 values, forward stage-1 DFT
template <int N>
__device__ __forceinline__ void T_to_s1_fwd(const LineLds<N>& L, double2* v, int l, int mb) {
  using D = LD<N>;
#pragma unroll
  for (int k1 = 0; k1 < D::M; ++k1) v[k1] = tget(L.T[(D::M * mb + k1) * kLT + l]);
  dft_r<D::M, false>(v);
}

// T -> stage-0 registers, inverse stage 0 (natural points n1 + M m)
template <int N>
__device__ __forceinline__ void T_to_s0_inv(const LineLds<N>& L, double2* a, int l, int n1, const double2* tw) {
  using D = LD<N>;
#pragma unroll
  for (int m = 0; m < D::R0; ++m) a[m] = tget(L.T[(n1 + D::M * m) * kLT + l]);
  if constexpr (D::M > 1) twiddle_pow<D::R0, true>(a, tw[n1]);
  dft_r<D::R0, true>(a);
}

// stage-0 registers (natural points) -> forward stage 0 -> T (the slots the
// same thread read in T_to_s0_inv, so no barrier is needed before it)
template <int N>
__device__ __forceinline__ void s0_fwd_to_T(LineLds<N>& L, double2* a, int l, int n1, const double2* tw) {
  using D = LD<N>;
  dft_r<D::R0, false>(a);
  if constexpr (D::M > 1) twiddle_pow<D::R0, false>(a, tw[n1]);
#pragma unroll
  for (int k = 0; k < D::R0; ++k) tput(L.T[(n1 + D::M * k) * kLT + l], a[k]);
}

// Packed real pairs (last tile, lines 14 and 15): the slot holds z = r1 + i r2
// with r1, r2 real along the line, so its spectrum Z splits into the Hermitian
// spectra Z1 = (Z(f) + conj Z(-f)) / 2 and Z2 = (Z(f) - conj Z(-f)) / (2i).
// packed_spectra writes Z of both slots, from T after a stage-0 pass, to X in
// natural order (threads 0..2 R0-1, one stage-1 block each); every thread can
// then split any frequency.
template <int N>
__device__ __forceinline__ void packed_spectra(LineLds<N>& L, int tid) {
  using D = LD<N>;
  if (tid < 2 * D::R0) {
    const int r = tid / D::R0, mb = tid % D::R0;
    double2 v[D::M];
    T_to_s1_fwd<N>(L, v, kLT - 2 + r, mb);
#pragma unroll
    for (int k1 = 0; k1 < D::M; ++k1) L.X[r][mb + D::R0 * k1] = narrow(v[k1]);
  }
}
template <int N>
__device__ __forceinline__ void packed_split(const LineLds<N>& L, int r, int f, double2& z1, double2& z2) {
  const double2 z = widen<double2>(L.X[r][f]), zm = widen<double2>(L.X[r][(N - f) % N]);
  z1 = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
  z2 = make_double2(0.5 * (z.y + zm.y), 0.5 * (zm.x - z.x));
}

enum LineMode { LM_FWD_INIT = 0, LM_FWD_STEP = 1, LM_ADJ_STEP = 2, LM_ADJ_FINAL = 3 };

struct LineStepArgs {
  const float2* hin[3];   // component spectra read and summed (the kernel's NH of them)
  double hscale;          // factor of their sum
  const float2* src;      // adjoint: source plane spectrum added to the hub
  float2* hout[3];        // output component spectra
  float2* plane;          // forward step: plane spectrum of the hub read (z lines), or null
};

// The two packed real pairs of the last tile (lines 14 and 15), handled apart
// from the item loops (which skip them) by threads 0..2 R0-1, one pair r and
// stage-1 block mb each, in code that stays small: the sinc on a real line is
// read from the table kr (kr_line gives its row), not evaluated.
//
// Pair r holds the lines (P, 0) and (P, N/2), P = r N/2; row of (P, Q): (P != 0) + (Q != 0).
__device__ __forceinline__ int kr_row(int r, int w) { return r + w; }

// packed_a: phase A of both lines, z = term(line 1) + i term(line 2), inverse
// stage 1 into T. kind 0: forward step (m+ sinc P / N), 1: forward init
// (P / (3 c0^2 N)), 2: the init's second transform (m+ sinc P dt/(2 rho0 N)),
// 3: adjoint (P / N, P including the source). ps1, ps2: the thread's parts of
// the plane sums of the two lines (z lines).
template <int N, int AX, int NH>
__device__ __forceinline__ void packed_a(LineLds<N>& L, const double* kr, const LineStepArgs& A, double scale,
                                         int kind, int tid, double2& ps1, double2& ps2) {
  using D = LD<N>;
  if (tid < 2 * D::R0) {
    const int r = tid / D::R0, mb = tid % D::R0;
    const LineGeo<N, AX> g1(D::NS - 2 + r);
    double2 v[D::M];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const LineGeo<N, AX> g = w == 0 ? g1 : g1.second();
      const double* kap = kr + kr_row(r, w) * N;
      double2 ps = make_double2(0.0, 0.0);
#pragma unroll
      for (int k1 = 0; k1 < D::M; ++k1) {
        const int f = mb + D::R0 * k1, p = D::M * mb + k1;
        bool cj;
        const int idx = hub_addr<N, AX>(g, f, p, cj);
        double2 P = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NH; ++c) P = cadd(P, widen<double2>(A.hin[c][idx]));
        if (cj) P.y = -P.y;
        P = cscale(P, kind == 3 && NH > 0 ? kap[f] * A.hscale : A.hscale);
        if (kind == 3) {
          double2 S = widen<double2>(A.src[src_addr<N, AX>(g, f, p, cj)]);
          if (cj) S.y = -S.y;
          P = cadd(P, S);
        }
        ps = cadd(ps, P);
        const double2 t = (kind == 0 || kind == 2) ? cscale(cmul(P, L.mp[f]), kap[f] * scale) : cscale(P, scale);
        v[k1] = w == 0 ? t : cadd(v[k1], mul_mi<true>(t));
      }
      if (w == 0) ps1 = ps;
      else ps2 = ps;
    }
    dft_r<D::M, true>(v);
    s1_to_T<N>(L, v, kLT - 2 + r, mb);
  }
}

// packed_c: phase C of both lines (T holds the stage-0 output of phase B):
// split the spectrum, each line times its own sinc, times m (m- forward, m+
// adjoint) / N, inverse stage 1 into T. Every thread of the block calls it.
template <int N>
__device__ __forceinline__ void packed_c(LineLds<N>& L, const double* kr, bool adj, double inv_n, int tid) {
  using D = LD<N>;
  // the sinc values first: their loads are in flight across the exchange
  const int r = tid / D::R0 % 2, mb = tid % D::R0;
  double ka[D::M], kb[D::M];
#pragma unroll
  for (int k1 = 0; k1 < D::M; ++k1) {
    ka[k1] = kr[kr_row(r, 0) * N + mb + D::R0 * k1];
    kb[k1] = kr[kr_row(r, 1) * N + mb + D::R0 * k1];
  }
  packed_spectra<N>(L, tid);
  __syncthreads();
  if (tid < 2 * D::R0) {
    double2 v[D::M];
#pragma unroll
    for (int k1 = 0; k1 < D::M; ++k1) {
      const int f = mb + D::R0 * k1;
      double2 z1, z2;
      packed_split<N>(L, r, f, z1, z2);
      const double2 z = cadd(cscale(z1, ka[k1]), mul_mi<true>(cscale(z2, kb[k1])));
      v[k1] = cscale(cmul(z, adj ? L.mp[f] : L.mm[f]), inv_n);
    }
    dft_r<D::M, true>(v);
    s1_to_T<N>(L, v, kLT - 2 + r, mb);
  }
}

// packed_e: the output spectra of both lines (adjoint: times m-). Every thread
// of the block calls it.
template <int N, int AX>
__device__ __forceinline__ void packed_e(LineLds<N>& L, bool adj, float2* out, int tid) {
  using D = LD<N>;
  const int r = tid / D::R0 % 2, mb = tid % D::R0;
  packed_spectra<N>(L, tid);
  __syncthreads();
  if (tid < 2 * D::R0) {
    const LineGeo<N, AX> g(D::NS - 2 + r);
    const LineGeo<N, AX> g2 = g.second();
#pragma unroll
    for (int k1 = 0; k1 < D::M; ++k1) {
      const int f = mb + D::R0 * k1, p = D::M * mb + k1;
      double2 z1, z2;
      packed_split<N>(L, r, f, z1, z2);
      if (adj) {
        z1 = cmul(z1, L.mm[f]);
        z2 = cmul(z2, L.mm[f]);
      }
      hub_store<N, AX>(out, g, f, p, z1);
      hub_store<N, AX>(out, g2, f, p, z2);
    }
  }
}

// One tile of lines of axis AX. The hub loads of a stage-1 item are issued
// together; the states are read where they are updated (a load issued a phase
// earlier costs more in registers, and occupancy, than it hides).
template <int N, int AX, int MODE, int NH>
__device__ __forceinline__ void line_tile(LineLds<N>& L, const LineTables& Tg, const LineScalars& sc,
                                          const LineBuffers& B, const LineStepArgs& A, int tile, int tid) {
  using D = LD<N>;
  constexpr int R0 = D::R0, M = D::M;
  constexpr bool ADJ = MODE == LM_ADJ_STEP || MODE == LM_ADJ_FINAL;
  // NH component spectra are summed (compile time, so the loads carry no
  // branches); an adjoint step that reads none is the first, with zero states
  constexpr bool reads = !(ADJ && NH == 0);
  static_assert(N <= kThreadsL, "one table entry per thread");
  float2* su = B.su[AX];
  float2* sr = B.sr[AX];
  const bool want_plane = !ADJ && AX == 2 && A.plane != nullptr;
  const LTab T{L.h, L.mp, L.mm, L.tw, L.a, L.b};
  const bool packed_tile = tile == D::NT - 1;   // holds the two packed real pairs

  // tables: one entry of each per thread
  double th = 0.0;
  double2 tmp = make_double2(0.0, 0.0), tmm = tmp, ttw = tmp;
  float ta = 0.f, tb = 0.f;
  if (tid < N) {
    th = Tg.h[tid];
    tmp = Tg.mp[tid];
    tmm = Tg.mm[tid];
    ttw = Tg.tw[tid];
    ta = Tg.a[AX][tid];
    tb = Tg.b[AX][tid];
  }

  if (tid < N) {
    L.h[tid] = th;
    L.mp[tid] = tmp;
    L.mm[tid] = tmm;
    L.tw[tid] = ttw;
    L.a[tid] = ta;
    L.b[tid] = tb;
  }
  __syncthreads();

  // (A) per stage-1 item: the hub (and the adjoint source) at its frequencies,
  // loads issued together; sum, first multiplier, inverse stage 1
  double2 psum = make_double2(0.0, 0.0), ps1 = psum, ps2 = psum;   // plane sums (ps1, ps2: packed pairs)
  S1Reg<N> keep;   // forward init: kappa times the hub values, for the second transform
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    const int l = b % kLT, mb = b / kLT;
    if (b < D::N1 && !(packed_tile && l >= kLT - 2)) {
      const LineGeo<N, AX> g(tile * kLT + l);
      float2 hv[M][NH > 0 ? NH : 1], sv[M];
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1, p = M * mb + k1;
        bool cj;
        const int idx = hub_addr<N, AX>(g, f, p, cj);
#pragma unroll
        for (int c = 0; c < NH; ++c) hv[k1][c] = A.hin[c][idx];
        if (ADJ) sv[k1] = A.src[src_addr<N, AX>(g, f, p, cj)];
      }
      const double s0 = g.s0(T.h);
      double2 v[M];
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1;
        double2 P = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NH; ++c) P = cadd(P, widen<double2>(hv[k1][c]));
        const bool cj = AX == 0 && f > D::H;
        if (cj) P.y = -P.y;
        // adjoint: the stored outputs are m-_c W_c; their sum takes the sinc here
        P = cscale(P, ADJ && NH > 0 ? kappa_at(T.h, s0, f) * A.hscale : A.hscale);
        if (ADJ) {
          double2 S = widen<double2>(sv[k1]);
          if (cj) S.y = -S.y;
          P = cadd(P, S);
        }
        if (want_plane) psum = cadd(psum, P);
        if (MODE == LM_FWD_INIT) keep.v[i][k1] = cscale(P, kappa_at(T.h, s0, f));
        if (MODE == LM_FWD_STEP) P = cscale(cmul(P, T.mp[f]), kappa_at(T.h, s0, f) * sc.inv_n);
        else if (MODE == LM_FWD_INIT) P = cscale(P, sc.inv_n * sc.inv_3c2);
        else P = cscale(P, sc.inv_n);
        v[k1] = P;
      }
      dft_r<M, true>(v);
      s1_to_T<N>(L, v, l, mb);
    }
    __builtin_amdgcn_sched_barrier(0);   // one item at a time: bounds the live registers
  }
  if (__builtin_expect(packed_tile, 0)) {
    const int kind = MODE == LM_FWD_STEP ? 0 : MODE == LM_FWD_INIT ? 1 : 3;
    const double scale = MODE == LM_FWD_INIT ? sc.inv_n * sc.inv_3c2 : sc.inv_n;
    packed_a<N, AX, NH>(L, Tg.kr, A, scale, kind, tid, ps1, ps2);
  }
  __syncthreads();

  S0Reg<N> s0r;
  if constexpr (MODE == LM_FWD_INIT) {
    // rho = F^-1 P / (3 c0^2), u = dt/(2 rho0) F^-1 [m+ P]
#pragma unroll
    for (int i = 0; i < D::I0; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N0) {
        const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
        T_to_s0_inv<N>(L, s0r.a[i], l, n1, T.tw);
#pragma unroll
        for (int m = 0; m < R0; ++m) sr[(n1 + M * m) * D::NS + lg] = narrow(s0r.a[i][m]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      const int l = b % kLT, mb = b / kLT;
      if (b < D::N1 && !(packed_tile && l >= kLT - 2)) {
        double2 v[M];
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1)
          v[k1] = cscale(cmul(keep.v[i][k1], T.mp[mb + R0 * k1]), sc.inv_n * sc.half_dt_over_rho0);
        dft_r<M, true>(v);
        s1_to_T<N>(L, v, l, mb);
      }
    }
    if (packed_tile) packed_a<N, AX, NH>(L, Tg.kr, A, sc.inv_n * sc.half_dt_over_rho0, 2, tid, ps1, ps2);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D::I0; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N0) {
        const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
        T_to_s0_inv<N>(L, s0r.a[i], l, n1, T.tw);
#pragma unroll
        for (int m = 0; m < R0; ++m) su[(n1 + M * m) * D::NS + lg] = narrow(s0r.a[i][m]);
      }
    }
    return;
  }

  // (B) first update in the natural layout, forward stage 0
  //   forward: u <- a (a u - dt/rho0 g), transform u
  //   adjoint: rho^ <- b^2 rho^ + q, transform b rho^ (final: rho^ / (3 c0^2))
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT;
      const StateAt<N> at(n1, tile * kLT + l);
      double2* a = s0r.a[i];
      T_to_s0_inv<N>(L, a, l, n1, T.tw);
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int x = n1 + M * m;
        if (!ADJ) {
          const double af = T.a[x];
          const double2 uo = widen<double2>(*at(su, m));
          const double2 un = make_double2(af * (af * uo.x - sc.dt_over_rho0 * a[m].x),
                                          af * (af * uo.y - sc.dt_over_rho0 * a[m].y));
          *at(su, m) = narrow(un);
          a[m] = un;
        } else {
          const double bf = T.b[x];
          double2 rh = a[m];
          if (reads) {
            const double2 ro = widen<double2>(*at(sr, m));
            rh = make_double2(bf * bf * ro.x + rh.x, bf * bf * ro.y + rh.y);
          }
          if (MODE == LM_ADJ_STEP) {
            *at(sr, m) = narrow(rh);
            a[m] = cscale(rh, bf);
          } else {
            a[m] = cscale(rh, sc.inv_3c2);
          }
        }
      }
      s0_fwd_to_T<N>(L, a, l, n1, T.tw);
    }
  }
  __syncthreads();

  if constexpr (MODE == LM_ADJ_FINAL) {
    // out = F(rho^) / (3 c0^2) - dt/(2 rho0) m- F(v); s2: the second line of a packed slot
    S1Reg<N> s1, s2;
    if (packed_tile) {
      packed_spectra<N>(L, tid);
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N1) {
        const int l = b % kLT, mb = b / kLT;
        T_to_s1_fwd<N>(L, s1.v[i], l, mb);
        if (packed_tile && l >= kLT - 2) {
#pragma unroll
          for (int k1 = 0; k1 < M; ++k1) packed_split<N>(L, l - (kLT - 2), mb + R0 * k1, s1.v[i][k1], s2.v[i][k1]);
        }
      }
    }
    if (reads) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < D::I0; ++i) {
        const int b = tid + i * kThreadsL;
        if (b < D::N0) {
          const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
#pragma unroll
          for (int m = 0; m < R0; ++m) s0r.a[i][m] = widen<double2>(su[(n1 + M * m) * D::NS + lg]);
          s0_fwd_to_T<N>(L, s0r.a[i], l, n1, T.tw);
        }
      }
      __syncthreads();
      if (packed_tile) {
        packed_spectra<N>(L, tid);
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < D::I1; ++i) {
        const int b = tid + i * kThreadsL;
        if (b < D::N1) {
          const int l = b % kLT, mb = b / kLT;
          const LineGeo<N, AX> g(tile * kLT + l);
          const double s0 = g.s0(T.h);
          double2 w[M];
          T_to_s1_fwd<N>(L, w, l, mb);
          if (g.kind == 2) {
            const int r = l - (kLT - 2);
            const double *k1r = Tg.kr + kr_row(r, 0) * N, *k2r = Tg.kr + kr_row(r, 1) * N;
#pragma unroll
            for (int k1 = 0; k1 < M; ++k1) {
              const int f = mb + R0 * k1;
              double2 w1, w2;
              packed_split<N>(L, r, f, w1, w2);
              s1.v[i][k1] = csub(s1.v[i][k1], cscale(cmul(w1, T.mm[f]), k1r[f] * sc.half_dt_over_rho0));
              s2.v[i][k1] = csub(s2.v[i][k1], cscale(cmul(w2, T.mm[f]), k2r[f] * sc.half_dt_over_rho0));
            }
          } else {
#pragma unroll
            for (int k1 = 0; k1 < M; ++k1) {
              const int f = mb + R0 * k1;
              const double2 t = cscale(cmul(w[k1], T.mm[f]), kappa_at(T.h, s0, f) * sc.half_dt_over_rho0);
              s1.v[i][k1] = csub(s1.v[i][k1], t);
            }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < D::I1; ++i) {
      const int b = tid + i * kThreadsL;
      if (b < D::N1) {
        const int l = b % kLT, mb = b / kLT;
        const LineGeo<N, AX> g(tile * kLT + l);
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) hub_store<N, AX>(A.hout[AX], g, mb + R0 * k1, M * mb + k1, s1.v[i][k1]);
        if (g.kind == 2) {
          const LineGeo<N, AX> g2 = g.second();
#pragma unroll
          for (int k1 = 0; k1 < M; ++k1) hub_store<N, AX>(A.hout[AX], g2, mb + R0 * k1, M * mb + k1, s2.v[i][k1]);
        }
      }
    }
    return;
  }

  // (C) forward stage 1, middle multiplier (forward m-, adjoint m+), inverse stage 1
#pragma unroll 1
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    const int l = b % kLT, mb = b / kLT;
    if (b < D::N1 && !(packed_tile && l >= kLT - 2)) {
      const LineGeo<N, AX> g(tile * kLT + l);
      const double s0 = g.s0(T.h);
      double2 v[M];
      T_to_s1_fwd<N>(L, v, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1;
        v[k1] = cscale(cmul(v[k1], ADJ ? T.mp[f] : T.mm[f]), kappa_at(T.h, s0, f) * sc.inv_n);
      }
      dft_r<M, true>(v);
      s1_to_T<N>(L, v, l, mb);
    }
  }
  if (__builtin_expect(packed_tile, 0)) packed_c<N>(L, Tg.kr, ADJ, sc.inv_n, tid);
  __syncthreads();

  // (D) second update, forward stage 0
  //   forward: rho <- b (b rho - dt rho0 h), transform rho
  //   adjoint: uh = v + dt rho0 t, v <- a^2 uh, transform a uh
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT;
      const StateAt<N> at(n1, tile * kLT + l);
      double2* a = s0r.a[i];
      T_to_s0_inv<N>(L, a, l, n1, T.tw);
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int x = n1 + M * m;
        if (!ADJ) {
          const double bf = T.b[x];
          const double2 ro = widen<double2>(*at(sr, m));
          const double2 rn = make_double2(bf * (bf * ro.x - sc.dt_rho0 * a[m].x),
                                          bf * (bf * ro.y - sc.dt_rho0 * a[m].y));
          *at(sr, m) = narrow(rn);
          a[m] = rn;
        } else {
          const double af = T.a[x];
          double2 uh = cscale(a[m], sc.dt_rho0);
          if (reads) uh = cadd(uh, widen<double2>(*at(su, m)));
          *at(su, m) = narrow(cscale(uh, af * af));
          a[m] = cscale(uh, af);
        }
      }
      s0_fwd_to_T<N>(L, a, l, n1, T.tw);
    }
  }
  __syncthreads();

  // (E) forward stage 1 and the output spectrum (adjoint: times m-; the
  // reader applies the sinc, common to the three components)
#pragma unroll 1
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    const int l = b % kLT, mb = b / kLT;
    if (b < D::N1 && !(packed_tile && l >= kLT - 2)) {
      const LineGeo<N, AX> g(tile * kLT + l);
      double2 v[M];
      T_to_s1_fwd<N>(L, v, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        const int f = mb + R0 * k1, p = M * mb + k1;
        hub_store<N, AX>(A.hout[AX], g, f, p, ADJ ? cmul(v[k1], T.mm[f]) : v[k1]);
      }
    }
  }
  if (__builtin_expect(packed_tile, 0)) packed_e<N, AX>(L, ADJ, A.hout[AX], tid);

  if (want_plane) {   // sum over kz of the hub read: the plane z = 0 of the pressure, / N^3
    __syncthreads();
    tput(L.T[tid], psum);
    if (tid < 2 * R0) {
      tput(L.T[kThreadsL + tid], ps1);
      tput(L.T[kThreadsL + 2 * R0 + tid], ps2);
    }
    __syncthreads();
    if (tid < kLT) {
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < kThreadsL / kLT; ++j) s = cadd(s, tget(L.T[tid + kLT * j]));
      const LineGeo<N, AX> g(tile * kLT + tid);
      if (g.kind == 2) {   // a packed pair: the sums of the packed_a threads of pair r
        const int r = tid - (kLT - 2);
        double2 s2 = make_double2(0.0, 0.0);
        s = s2;
        for (int j = 0; j < R0; ++j) {
          s = cadd(s, tget(L.T[kThreadsL + r * R0 + j]));
          s2 = cadd(s2, tget(L.T[kThreadsL + 2 * R0 + r * R0 + j]));
        }
        const LineGeo<N, AX> g2 = g.second();
        A.plane[g2.kx * N + g2.kyp] = narrow(cscale(s2, sc.inv_ntot));
      }
      s = cscale(s, sc.inv_ntot);
      A.plane[g.kx * N + g.kyp] = narrow(s);
      if (g.kind == 1) A.plane[g.kx * N + g.kyn] = make_float2((float)s.x, (float)-s.y);
    }
  }
}

template <int N, int MODE, int NH>
__global__ __launch_bounds__(kThreadsL, MODE == LM_ADJ_FINAL ? 1 : PAT_LINE_WAVES) void k_line(
    LineTables T, LineScalars sc, LineBuffers B, LineStepArgs A) {
  __shared__ LineLds<N> L;
  const int tid = threadIdx.x;
  // the three axes interleaved in dispatch order, tiles in reverse: the last
  // tile of each axis, which also carries the packed real pairs (a longer
  // path), starts first
  const int ax = blockIdx.x % 3, tile = LD<N>::NT - 1 - (int)blockIdx.x / 3;
  if (ax == 0) line_tile<N, 0, MODE, NH>(L, T, sc, B, A, tile, tid);
  else if (ax == 1) line_tile<N, 1, MODE, NH>(L, T, sc, B, A, tile, tid);
  else line_tile<N, 2, MODE, NH>(L, T, sc, B, A, tile, tid);
}

// Slab spectrum [z][kx][ky_pos] (z lines: [point][line]) -> z transform ->
// component spectrum hub[kz][kx][ky_pos], times scale.
template <int N>
__global__ __launch_bounds__(kThreadsL) void k_line_zfwd(LineTables T, const float2* __restrict__ spec, float2* hub,
                                                         double scale) {
  using D = LD<N>;
  __shared__ LineLds<N> L;
  const int tile = blockIdx.x, tid = threadIdx.x;
  double2 a[D::R0];
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
#pragma unroll
      for (int m = 0; m < D::R0; ++m) a[m] = widen<double2>(spec[(n1 + D::M * m) * D::NL + lg]);
      s0_fwd_to_T<N>(L, a, l, n1, T.tw);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, 2> g = LineGeo<N, 2>::zline(tile * kLT + l);
      double2 v[D::M];
      T_to_s1_fwd<N>(L, v, l, mb);
#pragma unroll
      for (int k1 = 0; k1 < D::M; ++k1) hub_store<N, 2>(hub, g, mb + D::R0 * k1, D::M * mb + k1, cscale(v[k1], scale));
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
#pragma unroll
  for (int i = 0; i < D::I1; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N1) {
      const int l = b % kLT, mb = b / kLT;
      const LineGeo<N, 2> g = LineGeo<N, 2>::zline(tile * kLT + l);
      double2 v[D::M];
#pragma unroll
      for (int k1 = 0; k1 < D::M; ++k1)
        v[k1] = cscale(hub_sum<N, 2>(hs, 3, g, mb + D::R0 * k1, D::M * mb + k1), scale);
      dft_r<D::M, true>(v);
      s1_to_T<N>(L, v, l, mb);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < D::I0; ++i) {
    const int b = tid + i * kThreadsL;
    if (b < D::N0) {
      const int l = b % kLT, n1 = b / kLT, lg = tile * kLT + l;
      double2 a[D::R0];
      T_to_s0_inv<N>(L, a, l, n1, T.tw);
#pragma unroll
      for (int m = 0; m < D::R0; ++m) spec[(n1 + D::M * m) * D::NL + lg] = narrow(a[m]);
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
  A.hscale = sc.c2;
  if (nt > 1) k_line<N, LM_FWD_INIT, 1><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
  const int rec = timed_span_begin(kt, K_LINE_FWD, st);
  for (int n = 0; n + 1 < nt; ++n) {
    const int cur = n & 1;
    for (int c = 0; c < 3; ++c) {
      A.hin[c] = B.hub[cur][c];
      A.hout[c] = B.hub[cur ^ 1][c];
    }
    A.plane = B.planes + (size_t)n * D::NL;
    if (n == 0) k_line<N, LM_FWD_STEP, 1><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
    else k_line<N, LM_FWD_STEP, 3><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
  }
  timed_span_end(kt, rec, K_LINE_FWD, nt - 1, st);
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
  const int rec = timed_span_begin(kt, K_LINE_ADJ, st);
  for (int j = 0; j + 1 < nt; ++j) {   // iteration of time index n = nt - 2 - j
    const int n = nt - 2 - j;
    cur = j & 1;
    for (int c = 0; c < 3; ++c) {
      A.hin[c] = B.hub[cur][c];
      A.hout[c] = B.hub[cur ^ 1][c];
    }
    A.src = B.planes + (size_t)(n + 1) * D::NL;
    if (j == 0) k_line<N, LM_ADJ_STEP, 0><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
    else k_line<N, LM_ADJ_STEP, 3><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
  }
  timed_span_end(kt, rec, K_LINE_ADJ, nt - 1, st);
  cur = (nt - 1) & 1;
  for (int c = 0; c < 3; ++c) {
    A.hin[c] = B.hub[cur][c];
    A.hout[c] = B.hub[cur ^ 1][c];
  }
  A.src = B.planes;
  if (nt == 1) k_line<N, LM_ADJ_FINAL, 0><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
  else k_line<N, LM_ADJ_FINAL, 3><<<3 * D::NT, kThreadsL, 0, st>>>(T, sc, B, A);
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
    PAT_LINE_IMPL(96),
    PAT_LINE_IMPL(128),
};

const LineImpl* find_line_impl(int nx, int ny, int nz) {
  if (nx != ny || ny != nz) return nullptr;
  for (const auto& w : kLineImpls)
    if (w.n == nx) return &w;
  return nullptr;
}

}  // namespace pat
