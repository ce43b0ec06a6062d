// C ABI of the photoacoustic-tomography hot path: plan set-up (FP64 tables,
// workspace carve-up), argument validation, the operator entry points and the
// host driver of FISTA / Bregman (App. B, Sec. 4.6). All device work is
// enqueued on the plan's stream; only calls that return host scalars sync.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fft_radix.hpp"
#include "pat_internal.hpp"
#include "sample_common.hpp"
#include "vec_common.hpp"
#include "wave_common.hpp"
#include "line_common.hpp"

namespace pat {

namespace {
thread_local char g_err[512] = "";
}

pat_status set_error(pat_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

namespace {

constexpr size_t kAlign = 256;
constexpr int kRedSlots = 16;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t u[3], rho[3], spec[4], planes2, planes, red_partial, red_out, flags;
  size_t lsu[3], lsr[3], lhub[2][3], lplanes, lspec;   // line propagator
  size_t img[7], dual, data[6];
  size_t total;
};

enum { IMG_X, IMG_XPREV, IMG_Y, IMG_G, IMG_V, IMG_QBAR, IMG_VCOPY };
enum { DAT_RX, DAT_RPREV, DAT_RY, DAT_B, DAT_D, DAT_TMP };

size_t n_voxels(const pat_grid& g) { return (size_t)g.nx * g.ny * g.nz; }
size_t n_pix(const pat_grid& g) { return (size_t)g.nx * g.ny; }
size_t n_spec(const pat_grid& g) { return (size_t)g.nz * (g.nx / 2 + 1) * g.ny; }
size_t n_dual(const pat_grid& g, int bc) {
  return bc == 1 ? 3 * (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1) : 3 * n_voxels(g);
}

Layout make_layout(const pat_grid& g, const pat_sampling& s) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t R = n_voxels(g) * sizeof(float);
  const size_t C = n_spec(g) * sizeof(float2);
  for (int i = 0; i < 3; ++i) L.u[i] = take(R);
  for (int i = 0; i < 3; ++i) L.rho[i] = take(R);
  for (int i = 0; i < 4; ++i) L.spec[i] = take(C);
  L.planes2 = take(2 * (size_t)g.nt * n_pix(g) * sizeof(float));
  L.planes = s.kind == PAT_SAMPLE_FULL ? 0 : take((size_t)g.nt * n_pix(g) * sizeof(float));
  L.red_partial = take(kRedBlocks * sizeof(double));
  L.red_out = take(kRedSlots * sizeof(double));
  L.flags = take((size_t)g.nz * sizeof(unsigned));
  for (int i = 0; i < 3; ++i) L.lsu[i] = take(C);
  for (int i = 0; i < 3; ++i) L.lsr[i] = take(C);
  for (int j = 0; j < 2; ++j)
    for (int i = 0; i < 3; ++i) L.lhub[j][i] = take(C);
  L.lplanes = take((size_t)g.nt * (g.nx / 2 + 1) * g.ny * sizeof(float2));
  L.lspec = take(C);
  for (int i = 0; i < 7; ++i) L.img[i] = take(R);
  L.dual = take(n_dual(g, 1) * sizeof(float));
  const size_t D = (size_t)g.nt * s.mc * sizeof(float);
  for (int i = 0; i < 6; ++i) L.data[i] = take(D);
  L.total = off;
  return L;
}

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

pat_status validate_grid(const pat_grid* g) {
  if (!g) return set_error(PAT_ERR_INVALID, "grid is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return set_error(PAT_ERR_INVALID, "grid sizes must be positive");
  if (!(g->dx > 0) || !(g->c0 > 0) || !(g->dt > 0) || !(g->rho0 > 0))
    return set_error(PAT_ERR_INVALID, "dx, c0, dt and rho0 must be positive and finite");
  if (!std::isfinite(g->dx) || !std::isfinite(g->c0) || !std::isfinite(g->dt) || !std::isfinite(g->rho0))
    return set_error(PAT_ERR_INVALID, "dx, c0, dt and rho0 must be finite");
  if (g->nt < 1) return set_error(PAT_ERR_INVALID, "nt must be >= 1");
  if (g->pml_size < 0 || 2 * g->pml_size >= g->nx || 2 * g->pml_size >= g->ny || 2 * g->pml_size >= g->nz)
    return set_error(PAT_ERR_INVALID, "pml_size must satisfy 0 <= 2 P < nx, ny, nz");
  if (!(g->pml_alpha >= 0) || !std::isfinite(g->pml_alpha))
    return set_error(PAT_ERR_INVALID, "pml_alpha must be finite and >= 0");
  if (!find_wave_impl(g->nx, g->ny, g->nz))
    return set_error(PAT_ERR_UNSUPPORTED, "grid %dx%dx%d is not built (cubic 16, 32, 64, 96, 128)", g->nx, g->ny, g->nz);
  return PAT_OK;
}

pat_status validate_sampling(const pat_grid* g, const pat_sampling* s) {
  if (!s) return set_error(PAT_ERR_INVALID, "sampling is NULL");
  const long np = (long)g->nx * g->ny;
  if (s->kind == PAT_SAMPLE_FULL) {
    if (s->mc != np) return set_error(PAT_ERR_INVALID, "FULL sampling needs mc == nx*ny");
    return PAT_OK;
  }
  if (s->kind != PAT_SAMPLE_POINTS && s->kind != PAT_SAMPLE_HADAMARD)
    return set_error(PAT_ERR_INVALID, "unknown sampling kind %d", s->kind);
  if (s->mc <= 0 || s->mc > np) return set_error(PAT_ERR_INVALID, "need 0 < mc <= nx*ny");
  if (!s->idx) return set_error(PAT_ERR_INVALID, "sampling idx is NULL");
  for (int j = 0; j < s->mc; ++j) {
    if (s->idx[j] < 0 || s->idx[j] >= np) return set_error(PAT_ERR_INVALID, "idx[%d] out of range", j);
    if (j > 0 && s->idx[j] <= s->idx[j - 1]) return set_error(PAT_ERR_INVALID, "idx must be strictly increasing");
  }
  if (s->kind == PAT_SAMPLE_HADAMARD) {
    if (!is_pow2(np)) return set_error(PAT_ERR_UNSUPPORTED, "Hadamard patterns need nx*ny a power of two");
    if (np > shd_max_pixels()) return set_error(PAT_ERR_UNSUPPORTED, "Hadamard plane larger than %d", shd_max_pixels());
    if (!s->perm) return set_error(PAT_ERR_INVALID, "Hadamard perm is NULL");
    std::vector<char> seen(np, 0);
    for (long i = 0; i < np; ++i) {
      const int v = s->perm[i];
      if (v < 0 || v >= np || seen[v]) return set_error(PAT_ERR_INVALID, "perm is not a permutation");
      seen[v] = 1;
    }
  }
  return PAT_OK;
}

// k of FFT bin m on an n-point axis (m' = m for m < n/2, else m - n)
double wavenumber(int m, int n, double dx) {
  const int mm = (2 * m < n) ? m : m - n;
  return 2.0 * M_PI * (double)mm / ((double)n * dx);
}

double pml_factor(double pos, int n, double seam, const pat_grid& g) {
  if (g.pml_size == 0) return 1.0;
  double dist = std::fmod(std::fabs(pos - seam), (double)n);
  dist = std::min(dist, (double)n - dist);
  const double d = std::max(0.0, 1.0 - dist / g.pml_size);
  const double sigma = g.pml_alpha * (g.c0 / g.dx) * d * d * d * d;
  return std::exp(-sigma * g.dt / 2.0);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define PAT_TRY_HIP(expr)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return set_error(PAT_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define PAT_TRY(expr)               \
  do {                              \
    pat_status s_ = (expr);         \
    if (s_ != PAT_OK) return s_;    \
  } while (0)

}  // namespace
}  // namespace pat

using namespace pat;

struct pat_plan {
  pat_grid g;
  int kind, mc;
  int npix;
  int device;
  hipStream_t stream;
  const WaveImpl* impl;
  void* tables;             // owned device allocation
  WaveTables tabs;
  WaveScalars sc;
  const int* idx;           // POINTS ids / HADAMARD rows
  const int* inv;           // POINTS: pixel -> j or -1
  const int* perm;          // HADAMARD column scramble
  const int* invperm;
  char* ws;
  Layout L;
  WaveBuffers wb;
  float* planes2;           // the two sensor-plane series of the forward propagation
  float* planes;
  double* red_partial;
  double* red_out;
  HandOff handoff;          // slab-pair flags (workspace) and launch epoch
  float* img[7];
  float* dual;
  float* data[6];
  int fftp;                 // FftPrecision of the propagator kernels
  const LineImpl* limpl;    // line propagator of this size (cubic grids), or null
  int scheme;               // PAT_SCHEME_*: which propagator runs (the line one needs FP64)
  LineTables ltabs;
  LineScalars lsc;
  LineBuffers lb;
  float* sens;              // per-pixel sensor sensitivity W_s (owned device copy) or null
  float* c2f;               // c(x)^2 of a heterogeneous medium (owned device copy) or null
  KernelTimer timer;        // active when timer.ev != nullptr
  std::vector<hipEvent_t> timer_events;
  std::vector<int> timer_ids;
  std::vector<int> timer_nl;
};

namespace {

template <typename T>
T* ws_ptr(pat_plan* p, size_t off) { return reinterpret_cast<T*>(p->ws + off); }

pat_status build_tables(pat_plan* P, const pat_sampling* s) {
  const pat_grid& g = P->g;
  const int NX = g.nx, NY = g.ny, NZ = g.nz, MX = NX / 2, NKX = MX + 1;
  struct C64 { double re, im; };
  std::vector<C64> c2;      // complex tables (FP64), concatenated
  std::vector<double> r;    // sinc argument tables (FP64)
  std::vector<float> pm;    // PML tables
  std::vector<int> iv;      // index tables
  auto twiddles = [&](int L, int count) {
    size_t o = c2.size();
    for (int j = 0; j < count; ++j) c2.push_back({std::cos(-2.0 * M_PI * j / L), std::sin(-2.0 * M_PI * j / L)});
    return o;
  };
  const size_t o_twmx = twiddles(MX, MX), o_twnx = twiddles(NX, MX + 1);
  const size_t o_twy = twiddles(NY, NY), o_twz = twiddles(NZ, NZ);
  // derivative multipliers i k exp(+-i k dx/2), exactly real at the Nyquist bin
  auto deriv = [&](int f, int n, int sgn) {
    const double k = wavenumber(f, n, g.dx);
    const double th = sgn * k * g.dx / 2.0;
    return 2 * f == n ? C64{-k * std::sin(th), 0.0} : C64{-k * std::sin(th), k * std::cos(th)};
  };
  const size_t o_mpx = c2.size();
  for (int kx = 0; kx < NKX; ++kx) c2.push_back(deriv(kx, NX, +1));
  const size_t o_mmx = c2.size();
  for (int kx = 0; kx < NKX; ++kx) c2.push_back(deriv(kx, NX, -1));
  auto axis_mult = [&](int n, int sgn) {
    size_t o = c2.size();
    for (int p = 0; p < n; ++p) c2.push_back(deriv(fft_freq(n, p), n, sgn));
    return o;
  };
  const size_t o_mpy = axis_mult(NY, +1), o_mmy = axis_mult(NY, -1);
  const size_t o_mpz = axis_mult(NZ, +1), o_mmz = axis_mult(NZ, -1);
  // line propagator: multipliers and sinc arguments by natural frequency index (cubic grid)
  const size_t o_lmp = c2.size();
  for (int k = 0; k < NX; ++k) c2.push_back(deriv(k, NX, +1));
  const size_t o_lmm = c2.size();
  for (int k = 0; k < NX; ++k) c2.push_back(deriv(k, NX, -1));
  const double hs = g.c0 * g.dt / 2.0;
  const size_t o_lh = r.size();
  for (int k = 0; k < NX; ++k) r.push_back(hs * wavenumber(k, NX, g.dx));
  // sinc(c0 dt |k| / 2) along the real lines of the line propagator, whose
  // transverse offset has |k_perp|^2 = c k_N^2 (k_N the Nyquist wavenumber), c = 0, 1, 2
  const size_t o_lkr = r.size();
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < NX; ++k) {
      const double hn = hs * wavenumber(NX / 2, NX, g.dx), hk = hs * wavenumber(k, NX, g.dx);
      const double h = std::sqrt(c * hn * hn + hk * hk);
      r.push_back(h > 0.0 ? std::sin(h) / h : 1.0);
    }
  const size_t o_hx = r.size();
  for (int kx = 0; kx < NKX; ++kx) r.push_back(hs * wavenumber(kx, NX, g.dx));
  const size_t o_hy = r.size();
  for (int p = 0; p < NY; ++p) r.push_back(hs * wavenumber(fft_freq(NY, p), NY, g.dx));
  const size_t o_hz = r.size();
  for (int q = 0; q < NZ; ++q) r.push_back(hs * wavenumber(fft_freq(NZ, q), NZ, g.dx));
  // PML factors: staggered (a) at i + 1/2, collocated (b) at i
  auto pml = [&](int n, double seam, double shift) {
    size_t o = pm.size();
    for (int i = 0; i < n; ++i) pm.push_back((float)pml_factor(i + shift, n, seam, g));
    return o;
  };
  const double seam_xy = -0.5, seam_z = (double)NZ - g.pml_size - 0.5;
  const size_t o_ax = pml(NX, seam_xy, 0.5), o_ay = pml(NY, seam_xy, 0.5), o_az = pml(NZ, seam_z, 0.5);
  const size_t o_bx = pml(NX, seam_xy, 0.0), o_by = pml(NY, seam_xy, 0.0), o_bz = pml(NZ, seam_z, 0.0);
  // index maps
  size_t o_idx = 0, o_inv = 0, o_perm = 0, o_invperm = 0;
  if (s->kind != PAT_SAMPLE_FULL) {
    o_idx = iv.size();
    iv.insert(iv.end(), s->idx, s->idx + s->mc);
  }
  if (s->kind == PAT_SAMPLE_POINTS) {
    o_inv = iv.size();
    iv.resize(iv.size() + P->npix, -1);
    for (int j = 0; j < s->mc; ++j) iv[o_inv + s->idx[j]] = j;
  }
  if (s->kind == PAT_SAMPLE_HADAMARD) {
    o_perm = iv.size();
    iv.insert(iv.end(), s->perm, s->perm + P->npix);
    o_invperm = iv.size();
    iv.resize(iv.size() + P->npix, 0);
    for (int q = 0; q < P->npix; ++q) iv[o_invperm + s->perm[q]] = q;
  }
  // device images: complex as float2 and double2, real as float and double
  std::vector<float2> cf(c2.size());
  std::vector<double2> cd(c2.size());
  for (size_t i = 0; i < c2.size(); ++i) {
    cf[i] = make_float2((float)c2[i].re, (float)c2[i].im);
    cd[i] = make_double2(c2[i].re, c2[i].im);
  }
  std::vector<float> rf(r.begin(), r.end());
  const size_t b_cf = align_up(cf.size() * sizeof(float2)), b_cd = align_up(cd.size() * sizeof(double2));
  const size_t b_rf = align_up(rf.size() * sizeof(float)), b_rd = align_up(r.size() * sizeof(double));
  const size_t b_pm = align_up(pm.size() * sizeof(float));
  const size_t b_iv = align_up(std::max<size_t>(iv.size(), 1) * sizeof(int));
  PAT_TRY_HIP(hipMalloc(&P->tables, b_cf + b_cd + b_rf + b_rd + b_pm + b_iv));
  char* base = static_cast<char*>(P->tables);
  char* p_cf = base;
  char* p_cd = p_cf + b_cf;
  char* p_rf = p_cd + b_cd;
  char* p_rd = p_rf + b_rf;
  char* p_pm = p_rd + b_rd;
  char* p_iv = p_pm + b_pm;
  PAT_TRY_HIP(hipMemcpy(p_cf, cf.data(), cf.size() * sizeof(float2), hipMemcpyHostToDevice));
  PAT_TRY_HIP(hipMemcpy(p_cd, cd.data(), cd.size() * sizeof(double2), hipMemcpyHostToDevice));
  PAT_TRY_HIP(hipMemcpy(p_rf, rf.data(), rf.size() * sizeof(float), hipMemcpyHostToDevice));
  PAT_TRY_HIP(hipMemcpy(p_rd, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice));
  PAT_TRY_HIP(hipMemcpy(p_pm, pm.data(), pm.size() * sizeof(float), hipMemcpyHostToDevice));
  if (!iv.empty()) PAT_TRY_HIP(hipMemcpy(p_iv, iv.data(), iv.size() * sizeof(int), hipMemcpyHostToDevice));
  auto fill = [&](auto& T, auto* dc, auto* dr) {
    T.tw_mx = dc + o_twmx; T.tw_nx = dc + o_twnx; T.tw_y = dc + o_twy; T.tw_z = dc + o_twz;
    T.mpx = dc + o_mpx; T.mmx = dc + o_mmx; T.mpy = dc + o_mpy; T.mmy = dc + o_mmy;
    T.mpz = dc + o_mpz; T.mmz = dc + o_mmz;
    T.hx = dr + o_hx; T.hy = dr + o_hy; T.hz = dr + o_hz;
  };
  WaveTables& t = P->tabs;
  fill(t.f, reinterpret_cast<const float2*>(p_cf), reinterpret_cast<const float*>(p_rf));
  fill(t.d, reinterpret_cast<const double2*>(p_cd), reinterpret_cast<const double*>(p_rd));
  const float* dp = reinterpret_cast<const float*>(p_pm);
  t.ax = dp + o_ax; t.ay = dp + o_ay; t.az = dp + o_az;
  t.bx = dp + o_bx; t.by = dp + o_by; t.bz = dp + o_bz;
  const int* di = reinterpret_cast<const int*>(p_iv);
  P->idx = s->kind != PAT_SAMPLE_FULL ? di + o_idx : nullptr;
  P->inv = s->kind == PAT_SAMPLE_POINTS ? di + o_inv : nullptr;
  P->perm = s->kind == PAT_SAMPLE_HADAMARD ? di + o_perm : nullptr;
  P->invperm = s->kind == PAT_SAMPLE_HADAMARD ? di + o_invperm : nullptr;
  {
    LineTables& lt = P->ltabs;
    const double2* dc = reinterpret_cast<const double2*>(p_cd);
    const double* dr = reinterpret_cast<const double*>(p_rd);
    lt.mp = dc + o_lmp;
    lt.mm = dc + o_lmm;
    lt.h = dr + o_lh;
    lt.kr = dr + o_lkr;
    lt.tw = dc + o_twz;
    lt.a[0] = t.ax; lt.a[1] = t.ay; lt.a[2] = t.az;
    lt.b[0] = t.bx; lt.b[1] = t.by; lt.b[2] = t.bz;
    LineScalars& ls = P->lsc;
    ls.c2 = g.c0 * g.c0;
    ls.dt_over_rho0 = g.dt / g.rho0;
    ls.dt_rho0 = g.dt * g.rho0;
    ls.half_dt_over_rho0 = g.dt / (2.0 * g.rho0);
    ls.inv_3c2 = 1.0 / (3.0 * g.c0 * g.c0);
    ls.inv_n = 1.0 / NX;
    ls.inv_ntot = 1.0 / ((double)NX * NY * NZ);
    ls.adj_scale = g.c0 * g.c0 * g.dt / g.rho0;
  }
  WaveScalars& sc = P->sc;
  sc.dt_over_rho0 = (float)(g.dt / g.rho0);
  sc.dt_rho0 = (float)(g.dt * g.rho0);
  sc.c2 = (float)(g.c0 * g.c0);
  sc.inv_3c2 = (float)(1.0 / (3.0 * g.c0 * g.c0));
  sc.half_dt_over_rho0 = (float)(g.dt / (2.0 * g.rho0));
  sc.inv_ntot = (float)(1.0 / ((double)NX * NY * NZ));
  return PAT_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

size_t vol_bytes(const pat_plan* P) { return n_voxels(P->g) * sizeof(float); }
size_t data_bytes(const pat_plan* P) { return (size_t)P->g.nt * P->mc * sizeof(float); }
long vol_n(const pat_plan* P) { return (long)n_voxels(P->g); }
long data_n(const pat_plan* P) { return (long)P->g.nt * P->mc; }

// ---- operator pieces used by the entry points and the solver ----------------
bool use_line(const pat_plan* P) {
  return P->scheme == PAT_SCHEME_LINE && P->limpl && P->fftp == FFT_FP64 && !P->c2f;
}

// The slab scheme tags its hand-off flags with an epoch the host advances per
// launch; a graph would replay stale epochs, so that scheme refuses capture.
pat_status check_capture(const pat_plan* P) {
  if (use_line(P)) return PAT_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(P->stream, &cs);
  if (e != hipSuccess) return set_error(PAT_ERR_HIP, "hipStreamIsCapturing: %s", hipGetErrorString(e));
  if (cs != hipStreamCaptureStatusNone)
    return set_error(PAT_ERR_UNSUPPORTED, "the slab scheme cannot be captured into a graph (use the line scheme)");
  return PAT_OK;
}

pat_status op_forward(pat_plan* P, const float* p0, float* f) {
  PAT_TRY(check_capture(P));
  float* planes = P->kind == PAT_SAMPLE_FULL ? f : P->planes;
  const long nplane = (long)P->g.nt * P->npix;
  KernelTimer* kt = P->timer.ev ? &P->timer : nullptr;
  if (use_line(P)) {
    PAT_TRY_HIP(P->limpl->forward(P->ltabs, P->lsc, P->lb, P->tabs, p0, planes, P->g.nt, P->stream, kt));
  } else {
    PAT_TRY_HIP(P->impl->forward[P->fftp](P->tabs, P->sc, P->wb, p0, P->planes2, P->g.nt, P->stream, kt,
                                          P->handoff));
    PAT_TRY_HIP(launch_sum2(P->planes2, nplane, planes, nplane, P->stream));
  }
  if (P->sens) PAT_TRY_HIP(launch_scale_pixels(planes, P->sens, planes, P->g.nt, P->npix, P->stream));
  if (P->kind == PAT_SAMPLE_POINTS)
    PAT_TRY_HIP(launch_rsp_gather(planes, P->idx, f, P->npix, P->mc, P->g.nt, P->stream));
  else if (P->kind == PAT_SAMPLE_HADAMARD)
    PAT_TRY_HIP(launch_shd_forward(planes, P->perm, P->idx, f, P->npix, P->mc, P->g.nt, P->stream));
  return PAT_OK;
}

pat_status op_adjoint(pat_plan* P, const float* f, float* p) {
  if (P->c2f)
    return set_error(PAT_ERR_UNSUPPORTED, "the adjoint is built for a homogeneous medium (clear the sound-speed field)");
  PAT_TRY(check_capture(P));
  const float* planes = f;
  if (P->kind == PAT_SAMPLE_POINTS) {
    PAT_TRY_HIP(launch_rsp_scatter(f, P->inv, P->planes, P->npix, P->mc, P->g.nt, P->stream));
    planes = P->planes;
  } else if (P->kind == PAT_SAMPLE_HADAMARD) {
    PAT_TRY_HIP(launch_shd_adjoint(f, P->invperm, P->idx, P->planes, P->npix, P->mc, P->g.nt, P->stream));
    planes = P->planes;
  }
  if (P->sens) {   // W_s is diagonal: its transpose is itself (FULL: f is read-only, scale into planes2)
    float* dst = P->kind == PAT_SAMPLE_FULL ? P->planes2 : P->planes;
    PAT_TRY_HIP(launch_scale_pixels(planes, P->sens, dst, P->g.nt, P->npix, P->stream));
    planes = dst;
  }
  KernelTimer* kt = P->timer.ev ? &P->timer : nullptr;
  if (use_line(P))
    PAT_TRY_HIP(P->limpl->adjoint(P->ltabs, P->lsc, P->lb, P->tabs, planes, p, P->g.nt, P->stream, kt));
  else
    PAT_TRY_HIP(P->impl->adjoint[P->fftp](P->tabs, P->sc, P->wb, planes, p, P->g.nt, P->stream, kt, P->handoff));
  return PAT_OK;
}

// n_iter PDHG steps for prox_{TV + (>= 0), alpha}(v) into q (v must not alias q).
pat_status op_prox(pat_plan* P, const float* v, float* q, float alpha, int n_iter, int bc, float* dual) {
  const pat_grid& g = P->g;
  float* qbar = P->img[IMG_QBAR];
  PAT_TRY_HIP(launch_pdhg_init(v, q, qbar, vol_n(P), P->stream));
  double tau = 1.0 / std::sqrt(12.0), sigma = tau;
  for (int k = 0; k < n_iter; ++k) {
    const double theta = 1.0 / std::sqrt(1.0 + 2.0 * tau);
    PAT_TRY_HIP(launch_pdhg_iter(v, q, qbar, dual, g.nx, g.ny, g.nz, bc, (float)sigma, (float)tau, (float)theta,
                                 alpha, P->stream));
    tau *= theta;
    sigma /= theta;
  }
  return PAT_OK;
}

// Copy `n` device doubles from red_out to the host (syncs).
pat_status read_slots(pat_plan* P, double* host, int n) {
  PAT_TRY_HIP(hipMemcpyAsync(host, P->red_out, n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  PAT_TRY_HIP(hipStreamSynchronize(P->stream));
  return PAT_OK;
}

pat_status op_norm2(pat_plan* P, const float* a, long n, int slot) {
  PAT_TRY_HIP(launch_reduce_vec(a, nullptr, n, 0, P->red_partial, P->red_out + slot, P->stream));
  return PAT_OK;
}

pat_status op_tv(pat_plan* P, const float* q, int bc, int slot) {
  PAT_TRY_HIP(launch_reduce_tv(q, P->g.nx, P->g.ny, P->g.nz, bc, P->red_partial, P->red_out + slot, P->stream));
  return PAT_OK;
}

pat_status op_psnr(pat_plan* P, const float* a, const float* b, int slot_maxima, int slot) {
  const pat_grid& g = P->g;
  const int Pm = g.pml_size;
  PAT_TRY_HIP(launch_psnr(a, b, g.nx, g.ny, g.nz, Pm, g.nx - Pm, Pm, g.ny - Pm, 1, g.nz - 2 * Pm, P->red_partial,
                          P->red_out + slot_maxima, P->red_out + slot, P->stream));
  return PAT_OK;
}

long psnr_count(const pat_plan* P) {
  const pat_grid& g = P->g;
  const long Pm = g.pml_size;
  return (g.nx - 2 * Pm) * (g.ny - 2 * Pm) * std::max(0L, (long)g.nz - 2 * Pm - 1);
}

double psnr_from_sum(double sum, long count) {
  if (sum == 0.0) return INFINITY;
  return -10.0 * std::log10(sum / (double)count);
}

pat_status check_plan(const pat_plan* P) {
  if (!P) return set_error(PAT_ERR_INVALID, "plan is NULL");
  return PAT_OK;
}

}  // namespace

extern "C" {

const char* pat_last_error(void) { return g_err; }

const char* pat_version(void) { return "pat-mi355x 0.1 (gfx950)"; }

size_t pat_plan_workspace_bytes(const pat_grid* grid, const pat_sampling* smp) {
  if (validate_grid(grid) != PAT_OK || validate_sampling(grid, smp) != PAT_OK) return 0;
  return make_layout(*grid, *smp).total;
}

size_t pat_tv_dual_floats(const pat_grid* grid, int32_t bc) {
  if (!grid || (bc != 0 && bc != 1) || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0) return 0;
  return n_dual(*grid, bc);
}

pat_status pat_plan_create(const pat_grid* grid, const pat_sampling* smp, void* stream, void* workspace,
                           size_t workspace_bytes, pat_plan** out) {
  if (!out) return set_error(PAT_ERR_INVALID, "out is NULL");
  *out = nullptr;
  PAT_TRY(validate_grid(grid));
  PAT_TRY(validate_sampling(grid, smp));
  const Layout L = make_layout(*grid, *smp);
  if (!workspace) return set_error(PAT_ERR_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return set_error(PAT_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < L.total)
    return set_error(PAT_ERR_NOMEM, "workspace has %zu bytes, plan needs %zu", workspace_bytes, L.total);
  pat_plan* P = new pat_plan();
  P->g = *grid;
  P->kind = smp->kind;
  P->mc = smp->mc;
  P->npix = grid->nx * grid->ny;
  P->stream = static_cast<hipStream_t>(stream);
  P->impl = find_wave_impl(grid->nx, grid->ny, grid->nz);
  P->fftp = FFT_FP64;
  P->limpl = find_line_impl(grid->nx, grid->ny, grid->nz);
  P->scheme = P->limpl ? PAT_SCHEME_LINE : PAT_SCHEME_SLAB;
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return set_error(PAT_ERR_HIP, "hipGetDevice failed (no GPU?)");
  }
  pat_status st = build_tables(P, smp);
  if (st != PAT_OK) {
    if (P->tables) (void)hipFree(P->tables);
    delete P;
    return st;
  }
  P->ws = static_cast<char*>(workspace);
  P->L = L;
  for (int i = 0; i < 3; ++i) {
    P->wb.u[i] = ws_ptr<float>(P, L.u[i]);
    P->wb.rho[i] = ws_ptr<float>(P, L.rho[i]);
  }
  for (int i = 0; i < 4; ++i) P->wb.spec[i] = ws_ptr<float2>(P, L.spec[i]);
  for (int i = 0; i < 3; ++i) {
    P->lb.su[i] = ws_ptr<float2>(P, L.lsu[i]);
    P->lb.sr[i] = ws_ptr<float2>(P, L.lsr[i]);
    for (int j = 0; j < 2; ++j) P->lb.hub[j][i] = ws_ptr<float2>(P, L.lhub[j][i]);
  }
  P->lb.planes = ws_ptr<float2>(P, L.lplanes);
  P->lb.spec = ws_ptr<float2>(P, L.lspec);
  P->planes2 = ws_ptr<float>(P, L.planes2);
  P->planes = smp->kind == PAT_SAMPLE_FULL ? nullptr : ws_ptr<float>(P, L.planes);
  P->red_partial = ws_ptr<double>(P, L.red_partial);
  P->red_out = ws_ptr<double>(P, L.red_out);
  P->handoff.flags = ws_ptr<unsigned>(P, L.flags);
  P->handoff.epoch = 0;   // launches tag the flags with epochs 1, 2, ...
  {
    hipError_t e = hipMemsetAsync(P->handoff.flags, 0, (size_t)grid->nz * sizeof(unsigned), P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) {
      (void)hipFree(P->tables);
      delete P;
      return set_error(PAT_ERR_HIP, "clearing the hand-off flags: %s", hipGetErrorString(e));
    }
  }
  for (int i = 0; i < 7; ++i) P->img[i] = ws_ptr<float>(P, L.img[i]);
  P->dual = ws_ptr<float>(P, L.dual);
  for (int i = 0; i < 6; ++i) P->data[i] = ws_ptr<float>(P, L.data[i]);
  *out = P;
  return PAT_OK;
}

pat_status pat_plan_destroy(pat_plan* plan) {
  if (!plan) return PAT_OK;
  pat_status st = PAT_OK;
  for (hipEvent_t e : plan->timer_events) (void)hipEventDestroy(e);
  if (plan->sens || plan->c2f) {
    DeviceGuard dg(plan->device);
    if (plan->sens) (void)hipFree(plan->sens);
    if (plan->c2f) (void)hipFree(plan->c2f);
  }
  if (plan->tables) {
    DeviceGuard dg(plan->device);
    hipError_t e = hipFree(plan->tables);
    if (e != hipSuccess) st = set_error(PAT_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
  }
  delete plan;
  return st;
}

pat_status pat_plan_set_stream(pat_plan* plan, void* stream) {
  PAT_TRY(check_plan(plan));
  plan->stream = static_cast<hipStream_t>(stream);
  return PAT_OK;
}

pat_status pat_plan_set_sensitivity(pat_plan* plan, const float* w) {
  PAT_TRY(check_plan(plan));
  DeviceGuard dg(plan->device);
  if (!w) {
    if (plan->sens) PAT_TRY_HIP(hipFree(plan->sens));
    plan->sens = nullptr;
    return PAT_OK;
  }
  for (int i = 0; i < plan->npix; ++i)
    if (!std::isfinite(w[i])) return set_error(PAT_ERR_INVALID, "pat_plan_set_sensitivity: w[%d] is not finite", i);
  if (!plan->sens) PAT_TRY_HIP(hipMalloc(&plan->sens, (size_t)plan->npix * sizeof(float)));
  PAT_TRY_HIP(hipMemcpy(plan->sens, w, (size_t)plan->npix * sizeof(float), hipMemcpyHostToDevice));
  return PAT_OK;
}

pat_status pat_plan_set_sound_speed(pat_plan* plan, const float* c) {
  PAT_TRY(check_plan(plan));
  DeviceGuard dg(plan->device);
  if (!c) {
    if (plan->c2f) PAT_TRY_HIP(hipFree(plan->c2f));
    plan->c2f = nullptr;
    plan->wb.c2f = nullptr;
    return PAT_OK;
  }
  const long nv = vol_n(plan);
  std::vector<float> c2(nv);
  for (long i = 0; i < nv; ++i) {
    if (!(c[i] > 0) || !std::isfinite(c[i]))
      return set_error(PAT_ERR_INVALID, "pat_plan_set_sound_speed: c[%ld] must be positive and finite", i);
    if (c[i] > plan->g.c0 * (1.0 + 1e-6))
      return set_error(PAT_ERR_INVALID, "pat_plan_set_sound_speed: c[%ld] = %g exceeds the reference c0 = %g", i,
                       (double)c[i], plan->g.c0);
    c2[i] = (float)((double)c[i] * (double)c[i]);
  }
  if (!plan->c2f) PAT_TRY_HIP(hipMalloc(&plan->c2f, (size_t)nv * sizeof(float)));
  PAT_TRY_HIP(hipMemcpy(plan->c2f, c2.data(), (size_t)nv * sizeof(float), hipMemcpyHostToDevice));
  plan->wb.c2f = plan->c2f;
  return PAT_OK;
}

pat_status pat_plan_set_fft_precision(pat_plan* plan, int32_t bits) {
  PAT_TRY(check_plan(plan));
  if (bits != 32 && bits != 64) return set_error(PAT_ERR_INVALID, "pat_plan_set_fft_precision: bits must be 32 or 64");
  plan->fftp = bits == 64 ? FFT_FP64 : FFT_FP32;
  return PAT_OK;
}

pat_status pat_plan_set_scheme(pat_plan* plan, int32_t scheme) {
  PAT_TRY(check_plan(plan));
  if (scheme != PAT_SCHEME_SLAB && scheme != PAT_SCHEME_LINE)
    return set_error(PAT_ERR_INVALID, "pat_plan_set_scheme: unknown scheme %d", (int)scheme);
  if (scheme == PAT_SCHEME_LINE && !plan->limpl)
    return set_error(PAT_ERR_UNSUPPORTED, "pat_plan_set_scheme: no line propagator for this grid");
  plan->scheme = scheme;
  return PAT_OK;
}

pat_status pat_forward(pat_plan* plan, const float* p0, float* f) {
  PAT_TRY(check_plan(plan));
  if (!p0 || !f) return set_error(PAT_ERR_INVALID, "pat_forward: null pointer");
  if (overlaps(p0, vol_bytes(plan), f, data_bytes(plan)))
    return set_error(PAT_ERR_INVALID, "pat_forward: p0 and f overlap");
  DeviceGuard dg(plan->device);
  return op_forward(plan, p0, f);
}

pat_status pat_adjoint(pat_plan* plan, const float* f, float* p) {
  PAT_TRY(check_plan(plan));
  if (!p || !f) return set_error(PAT_ERR_INVALID, "pat_adjoint: null pointer");
  if (overlaps(p, vol_bytes(plan), f, data_bytes(plan)))
    return set_error(PAT_ERR_INVALID, "pat_adjoint: f and p overlap");
  DeviceGuard dg(plan->device);
  return op_adjoint(plan, f, p);
}

pat_status pat_time_reversal(pat_plan* plan, const float* f, float* p) {
  PAT_TRY(check_plan(plan));
  if (!p || !f) return set_error(PAT_ERR_INVALID, "pat_time_reversal: null pointer");
  if (overlaps(p, vol_bytes(plan), f, data_bytes(plan)))
    return set_error(PAT_ERR_INVALID, "pat_time_reversal: f and p overlap");
  DeviceGuard dg(plan->device);
  pat_plan* P = plan;
  if (P->c2f)
    return set_error(PAT_ERR_UNSUPPORTED, "time reversal is built for a homogeneous medium (clear the sound-speed field)");
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PAT_TRY_HIP(hipStreamIsCapturing(P->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return set_error(PAT_ERR_UNSUPPORTED, "pat_time_reversal runs the slab scheme, which cannot be captured");
  }
  const float* planes = f;   // C^T f (the pseudo-inverse of C, Sec. 4.4)
  if (P->kind == PAT_SAMPLE_POINTS) {
    PAT_TRY_HIP(launch_rsp_scatter(f, P->inv, P->planes, P->npix, P->mc, P->g.nt, P->stream));
    planes = P->planes;
  } else if (P->kind == PAT_SAMPLE_HADAMARD) {
    PAT_TRY_HIP(launch_shd_adjoint(f, P->invperm, P->idx, P->planes, P->npix, P->mc, P->g.nt, P->stream));
    planes = P->planes;
  }
  float *vol = P->img[IMG_VCOPY], *pa = P->img[IMG_V], *pb = P->img[IMG_QBAR];
  PAT_TRY_HIP(P->impl->time_reversal[P->fftp](P->tabs, P->sc, P->wb, planes, vol, pa, pb, P->planes2, P->g.nt,
                                                P->stream, P->handoff));
  if (P->g.nt == 1)
    PAT_TRY_HIP(launch_scale(vol, p, 1.f, vol_n(P), P->stream));
  else
    PAT_TRY_HIP(launch_axpy(pa, pb, p, 1.f, vol_n(P), P->stream));
  return PAT_OK;
}

pat_status pat_sample(pat_plan* plan, const float* s, float* f) {
  PAT_TRY(check_plan(plan));
  if (!s || !f) return set_error(PAT_ERR_INVALID, "pat_sample: null pointer");
  DeviceGuard dg(plan->device);
  const pat_grid& g = plan->g;
  if (plan->kind == PAT_SAMPLE_FULL)
    PAT_TRY_HIP(hipMemcpyAsync(f, s, data_bytes(plan), hipMemcpyDeviceToDevice, plan->stream));
  else if (plan->kind == PAT_SAMPLE_POINTS)
    PAT_TRY_HIP(launch_rsp_gather(s, plan->idx, f, plan->npix, plan->mc, g.nt, plan->stream));
  else
    PAT_TRY_HIP(launch_shd_forward(s, plan->perm, plan->idx, f, plan->npix, plan->mc, g.nt, plan->stream));
  return PAT_OK;
}

pat_status pat_sample_adjoint(pat_plan* plan, const float* f, float* s) {
  PAT_TRY(check_plan(plan));
  if (!s || !f) return set_error(PAT_ERR_INVALID, "pat_sample_adjoint: null pointer");
  DeviceGuard dg(plan->device);
  const pat_grid& g = plan->g;
  if (plan->kind == PAT_SAMPLE_FULL)
    PAT_TRY_HIP(hipMemcpyAsync(s, f, data_bytes(plan), hipMemcpyDeviceToDevice, plan->stream));
  else if (plan->kind == PAT_SAMPLE_POINTS)
    PAT_TRY_HIP(launch_rsp_scatter(f, plan->inv, s, plan->npix, plan->mc, g.nt, plan->stream));
  else
    PAT_TRY_HIP(launch_shd_adjoint(f, plan->invperm, plan->idx, s, plan->npix, plan->mc, g.nt, plan->stream));
  return PAT_OK;
}

pat_status pat_tv_prox(pat_plan* plan, const float* v, float* q, float alpha, int32_t n_iter, int32_t bc,
                       float* dual) {
  PAT_TRY(check_plan(plan));
  if (!v || !q || !dual) return set_error(PAT_ERR_INVALID, "pat_tv_prox: null pointer");
  if (bc != 0 && bc != 1) return set_error(PAT_ERR_INVALID, "pat_tv_prox: bc must be 0 or 1");
  if (n_iter < 0) return set_error(PAT_ERR_INVALID, "pat_tv_prox: n_iter must be >= 0");
  if (!(alpha >= 0.f) || !std::isfinite(alpha)) return set_error(PAT_ERR_INVALID, "pat_tv_prox: alpha must be >= 0");
  DeviceGuard dg(plan->device);
  float* vc = plan->img[IMG_VCOPY];
  PAT_TRY_HIP(hipMemcpyAsync(vc, v, vol_bytes(plan), hipMemcpyDeviceToDevice, plan->stream));
  return op_prox(plan, vc, q, alpha, n_iter, bc, dual);
}

pat_status pat_tv_norm(pat_plan* plan, const float* p, int32_t bc, double* out) {
  PAT_TRY(check_plan(plan));
  if (!p || !out) return set_error(PAT_ERR_INVALID, "pat_tv_norm: null pointer");
  if (bc != 0 && bc != 1) return set_error(PAT_ERR_INVALID, "pat_tv_norm: bc must be 0 or 1");
  DeviceGuard dg(plan->device);
  PAT_TRY(op_tv(plan, p, bc, 0));
  return read_slots(plan, out, 1);
}

pat_status pat_psnr(pat_plan* plan, const float* p, const float* p_ref, double* out) {
  PAT_TRY(check_plan(plan));
  if (!p || !p_ref || !out) return set_error(PAT_ERR_INVALID, "pat_psnr: null pointer");
  if (psnr_count(plan) <= 0) return set_error(PAT_ERR_INVALID, "pat_psnr: empty evaluation region");
  DeviceGuard dg(plan->device);
  PAT_TRY(op_psnr(plan, p, p_ref, 2, 0));
  double sum;
  PAT_TRY(read_slots(plan, &sum, 1));
  *out = psnr_from_sum(sum, psnr_count(plan));
  return PAT_OK;
}

pat_status pat_power_iteration(pat_plan* plan, const float* x0, int32_t n_iter, double* L_out) {
  PAT_TRY(check_plan(plan));
  if (!x0 || !L_out) return set_error(PAT_ERR_INVALID, "pat_power_iteration: null pointer");
  if (n_iter < 1) return set_error(PAT_ERR_INVALID, "pat_power_iteration: n_iter must be >= 1");
  DeviceGuard dg(plan->device);
  float* x = plan->img[IMG_X];
  float* w = plan->img[IMG_G];
  float* tmp = plan->data[DAT_TMP];
  double nrm2;
  PAT_TRY(op_norm2(plan, x0, vol_n(plan), 0));
  PAT_TRY(read_slots(plan, &nrm2, 1));
  if (!(nrm2 > 0) || !std::isfinite(nrm2)) return set_error(PAT_ERR_NONFINITE, "pat_power_iteration: |x0| is 0 or not finite");
  PAT_TRY_HIP(launch_scale(x0, x, (float)(1.0 / std::sqrt(nrm2)), vol_n(plan), plan->stream));
  double lam = 0.0;
  for (int k = 0; k < n_iter; ++k) {
    PAT_TRY(op_forward(plan, x, tmp));
    PAT_TRY(op_adjoint(plan, tmp, w));
    PAT_TRY(op_norm2(plan, w, vol_n(plan), 0));
    PAT_TRY(read_slots(plan, &nrm2, 1));
    lam = std::sqrt(nrm2);
    if (!(lam > 0) || !std::isfinite(lam)) return set_error(PAT_ERR_NONFINITE, "pat_power_iteration: |w| is 0 or not finite");
    PAT_TRY_HIP(launch_scale(w, x, (float)(1.0 / lam), vol_n(plan), plan->stream));
  }
  *L_out = lam;
  return PAT_OK;
}

pat_status pat_reconstruct(pat_plan* plan, const float* f, float* p, const pat_recon_params* prm,
                           pat_recon_report* rep) {
  PAT_TRY(check_plan(plan));
  if (!f || !p || !prm) return set_error(PAT_ERR_INVALID, "pat_reconstruct: null pointer");
  if (!(prm->L > 0) || !std::isfinite(prm->L)) return set_error(PAT_ERR_INVALID, "pat_reconstruct: L must be > 0");
  if (!(prm->lambda >= 0) || !std::isfinite(prm->lambda))
    return set_error(PAT_ERR_INVALID, "pat_reconstruct: lambda must be >= 0");
  if (prm->n_outer < 1 || prm->n_inner < 0 || prm->n_prox < 0 || prm->max_backtrack < 0)
    return set_error(PAT_ERR_INVALID, "pat_reconstruct: iteration counts out of range");
  if (prm->bc != 0 && prm->bc != 1) return set_error(PAT_ERR_INVALID, "pat_reconstruct: bc must be 0 or 1");
  if (rep && rep->capacity < 0) return set_error(PAT_ERR_INVALID, "pat_reconstruct: negative report capacity");
  if (prm->p_ref && psnr_count(plan) <= 0) return set_error(PAT_ERR_INVALID, "pat_reconstruct: empty PSNR region");
  DeviceGuard dg(plan->device);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = plan->stream;
  const long nv = vol_n(plan), nd = data_n(plan);
  const double lam = prm->lambda, eta = 1.8 / prm->L;
  const int bc = prm->bc;
  float *x = plan->img[IMG_X], *xp = plan->img[IMG_XPREV], *y = plan->img[IMG_Y];
  float *g = plan->img[IMG_G], *v = plan->img[IMG_V];
  float *rx = plan->data[DAT_RX], *rp = plan->data[DAT_RPREV], *ry = plan->data[DAT_RY];
  float *b = plan->data[DAT_B], *d = plan->data[DAT_D], *tmp = plan->data[DAT_TMP];
  float* dual = plan->dual;
  if (rep) rep->n_log = 0;
  PAT_TRY_HIP(launch_fill(b, 0.f, nd, st));
  PAT_TRY_HIP(launch_fill(xp, 0.f, nv, st));   // Bregman p^0 = 0
  PAT_TRY_HIP(launch_fill(dual, 0.f, (long)n_dual(plan->g, bc), st));
  int logi = 0;

  // energy of (r, x) into h[0] = sum r^2, h[1] = TV(x); syncs
  auto energy = [&](const float* r, const float* xx, double* e, double* tv, double* res) -> pat_status {
    PAT_TRY(op_norm2(plan, r, nd, 0));
    PAT_TRY(op_tv(plan, xx, bc, 1));
    double h[2];
    PAT_TRY(read_slots(plan, h, 2));
    *e = 0.5 * h[0] + lam * h[1];
    *tv = h[1];
    *res = std::sqrt(h[0]);
    if (!std::isfinite(*e)) return set_error(PAT_ERR_NONFINITE, "pat_reconstruct: energy is not finite");
    return PAT_OK;
  };

  for (int k = 0; k < prm->n_outer; ++k) {
    // d = f + b^k ; FISTA from x0 = current p (held in xp)
    PAT_TRY_HIP(launch_axpy(f, b, d, 1.f, nd, st));
    if (k == 0) {
      PAT_TRY_HIP(launch_scale(d, rp, -1.f, nd, st));          // x0 = 0, so C A x0 = 0 and r_prev = -d
    } else {
      PAT_TRY(op_forward(plan, xp, tmp));
      PAT_TRY_HIP(launch_axpy(tmp, d, rp, -1.f, nd, st));      // r_prev = C A x0 - d
    }
    double e_prev, tv, res;
    PAT_TRY(energy(rp, xp, &e_prev, &tv, &res));
    PAT_TRY_HIP(hipMemcpyAsync(y, xp, nv * sizeof(float), hipMemcpyDeviceToDevice, st));
    PAT_TRY_HIP(hipMemcpyAsync(ry, rp, nd * sizeof(float), hipMemcpyDeviceToDevice, st));
    double t = 1.0;
    for (int it = 0; it < prm->n_inner; ++it) {
      PAT_TRY(op_adjoint(plan, ry, g));
      PAT_TRY_HIP(launch_axpy(y, g, v, (float)(-eta), nv, st));
      PAT_TRY(op_prox(plan, v, x, (float)(eta * lam), prm->n_prox, bc, dual));
      PAT_TRY(op_forward(plan, x, tmp));
      PAT_TRY_HIP(launch_axpy(tmp, d, rx, -1.f, nd, st));
      double e;
      PAT_TRY(energy(rx, x, &e, &tv, &res));
      int flag = 0;
      if (prm->restart && e > e_prev) {
        t = 1.0;
        PAT_TRY(op_adjoint(plan, rp, g));
        for (int j = 0; j <= prm->max_backtrack; ++j) {
          const double step = eta / std::ldexp(1.0, j);
          PAT_TRY_HIP(launch_axpy(xp, g, v, (float)(-step), nv, st));
          PAT_TRY(op_prox(plan, v, x, (float)(step * lam), prm->n_prox, bc, dual));
          PAT_TRY(op_forward(plan, x, tmp));
          PAT_TRY_HIP(launch_axpy(tmp, d, rx, -1.f, nd, st));
          PAT_TRY(energy(rx, x, &e, &tv, &res));
          flag = 1 + j;
          if (e <= e_prev) break;
        }
      }
      const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      const double beta = (t - 1.0) / t_next;
      PAT_TRY_HIP(launch_extrapolate(x, xp, y, (float)beta, nv, st));
      PAT_TRY_HIP(launch_extrapolate(rx, rp, ry, (float)beta, nd, st));
      if (rep && logi < rep->capacity) {
        if (rep->energy) rep->energy[logi] = e;
        if (rep->residual) rep->residual[logi] = res;
        if (rep->tv) rep->tv[logi] = tv;
        if (rep->flags) rep->flags[logi] = flag;
        if (rep->psnr) {
          if (prm->p_ref) {
            PAT_TRY(op_psnr(plan, x, prm->p_ref, 2, 0));
            double sum;
            PAT_TRY(read_slots(plan, &sum, 1));
            rep->psnr[logi] = psnr_from_sum(sum, psnr_count(plan));
          } else {
            rep->psnr[logi] = NAN;
          }
        }
        if (rep->t_ms) {
          PAT_TRY_HIP(hipStreamSynchronize(st));
          rep->t_ms[logi] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        rep->n_log = ++logi;
      }
      std::swap(x, xp);
      std::swap(rx, rp);
      e_prev = e;
      t = t_next;
    }
    // Bregman: b^{k+1} = b^k + f - C A p = -r ; log ||C A p - f|| = ||r + b^k||
    PAT_TRY_HIP(launch_reduce_vec(rp, b, nd, 2, plan->red_partial, plan->red_out, st));
    double h;
    PAT_TRY(read_slots(plan, &h, 1));
    if (rep && rep->bregman_residual) rep->bregman_residual[k] = std::sqrt(h);
    PAT_TRY_HIP(launch_scale(rp, b, -1.f, nd, st));
  }
  PAT_TRY_HIP(hipMemcpyAsync(p, xp, nv * sizeof(float), hipMemcpyDeviceToDevice, st));
  PAT_TRY_HIP(hipStreamSynchronize(st));
  return PAT_OK;
}

// Iterations it0 .. it0 + n_iter - 1 of the TV+ FISTA loop of pat_reconstruct (n_outer = 1,
// restart off). The iterate, its predecessor, the extrapolated point, their residuals and the
// prox dual live in the plan's workspace; it0 = 0 starts from x = 0, it0 > 0 continues from
// what the previous call left there (the pointer roles alternate every iteration and t follows
// its recurrence, so both are recomputed from it0).
static pat_status fista_enqueue_range(pat_plan* plan, const char* who, const float* f, float* p, double lambda,
                                      double L, int32_t it0, int32_t n_iter, int32_t n_prox, int32_t bc, double* log) {
  PAT_TRY(check_plan(plan));
  if (!f || !p) return set_error(PAT_ERR_INVALID, "%s: null pointer", who);
  if (!(L > 0) || !std::isfinite(L)) return set_error(PAT_ERR_INVALID, "%s: L must be > 0", who);
  if (!(lambda >= 0) || !std::isfinite(lambda)) return set_error(PAT_ERR_INVALID, "%s: lambda must be >= 0", who);
  if (it0 < 0 || n_iter < 0 || n_prox < 0 || n_iter > (1 << 20) || it0 > (1 << 20))
    return set_error(PAT_ERR_INVALID, "%s: iteration counts out of range", who);
  if (bc != 0 && bc != 1) return set_error(PAT_ERR_INVALID, "%s: bc must be 0 or 1", who);
  if (overlaps(p, vol_bytes(plan), f, data_bytes(plan)))
    return set_error(PAT_ERR_INVALID, "%s: f and p overlap", who);
  DeviceGuard dg(plan->device);
  hipStream_t st = plan->stream;
  const long nv = vol_n(plan), nd = data_n(plan);
  const double eta = 1.8 / L;
  float *x = plan->img[IMG_X], *xp = plan->img[IMG_XPREV], *y = plan->img[IMG_Y];
  float *g = plan->img[IMG_G], *v = plan->img[IMG_V];
  float *rx = plan->data[DAT_RX], *rp = plan->data[DAT_RPREV], *ry = plan->data[DAT_RY];
  float* tmp = plan->data[DAT_TMP];
  // the same arithmetic, in the same order, as pat_reconstruct with n_outer = 1 and restart = 0,
  // but every operand stays on the device: kernels only, no copies, no host synchronisation
  double t = 1.0;
  if (it0 == 0) {
    PAT_TRY_HIP(launch_fill(xp, 0.f, nv, st));
    PAT_TRY_HIP(launch_fill(plan->dual, 0.f, (long)n_dual(plan->g, bc), st));
    PAT_TRY_HIP(launch_scale(f, rp, -1.f, nd, st));               // x0 = 0: r_prev = -f
    PAT_TRY_HIP(launch_fill(y, 0.f, nv, st));
    PAT_TRY_HIP(launch_scale(rp, ry, 1.f, nd, st));
  } else {
    for (int it = 0; it < it0; ++it) t = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    if (it0 % 2) {
      std::swap(x, xp);
      std::swap(rx, rp);
    }
  }
  for (int it = 0; it < n_iter; ++it) {
    PAT_TRY(op_adjoint(plan, ry, g));
    PAT_TRY_HIP(launch_axpy(y, g, v, (float)(-eta), nv, st));
    PAT_TRY(op_prox(plan, v, x, (float)(eta * lambda), n_prox, bc, plan->dual));
    PAT_TRY(op_forward(plan, x, tmp));
    PAT_TRY_HIP(launch_axpy(tmp, f, rx, -1.f, nd, st));
    if (log) {
      PAT_TRY_HIP(launch_reduce_vec(rx, nullptr, nd, 0, plan->red_partial, log + 2 * it, st));
      PAT_TRY_HIP(launch_reduce_tv(x, plan->g.nx, plan->g.ny, plan->g.nz, bc, plan->red_partial, log + 2 * it + 1, st));
    }
    const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double beta = (t - 1.0) / t_next;
    PAT_TRY_HIP(launch_extrapolate(x, xp, y, (float)beta, nv, st));
    PAT_TRY_HIP(launch_extrapolate(rx, rp, ry, (float)beta, nd, st));
    std::swap(x, xp);
    std::swap(rx, rp);
    t = t_next;
  }
  PAT_TRY_HIP(launch_scale(xp, p, 1.f, nv, st));
  return PAT_OK;
}

pat_status pat_fista_enqueue(pat_plan* plan, const float* f, float* p, double lambda, double L, int32_t n_iter,
                             int32_t n_prox, int32_t bc, double* log) {
  return fista_enqueue_range(plan, "pat_fista_enqueue", f, p, lambda, L, 0, n_iter, n_prox, bc, log);
}

pat_status pat_fista_enqueue_from(pat_plan* plan, const float* f, float* p, double lambda, double L, int32_t it0,
                                  int32_t n_iter, int32_t n_prox, int32_t bc, double* log) {
  return fista_enqueue_range(plan, "pat_fista_enqueue_from", f, p, lambda, L, it0, n_iter, n_prox, bc, log);
}

pat_status pat_profile_begin(pat_plan* plan, int32_t kernel_id, int32_t max_launches) {
  PAT_TRY(check_plan(plan));
  if (plan->timer.ev) return set_error(PAT_ERR_INVALID, "pat_profile_begin: profiling already active");
  if (!(kernel_id == -2 || (kernel_id >= 0 && kernel_id < K_COUNT)))
    return set_error(PAT_ERR_INVALID, "pat_profile_begin: kernel_id must be -2 or in [0, %d)", (int)K_COUNT);
  if (max_launches < 1 || max_launches > (1 << 20))
    return set_error(PAT_ERR_INVALID, "pat_profile_begin: max_launches out of range");
  DeviceGuard dg(plan->device);
  plan->timer_events.assign(2 * (size_t)max_launches, nullptr);
  for (auto& e : plan->timer_events) {
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      for (auto& x : plan->timer_events)
        if (x) (void)hipEventDestroy(x);
      plan->timer_events.clear();
      return set_error(PAT_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(err));
    }
  }
  plan->timer_ids.assign(max_launches, -1);
  plan->timer_nl.assign(max_launches, 1);
  plan->timer.which = kernel_id;
  plan->timer.ev = plan->timer_events.data();
  plan->timer.ids = plan->timer_ids.data();
  plan->timer.nl = plan->timer_nl.data();
  plan->timer.cap = max_launches;
  plan->timer.count = 0;
  return PAT_OK;
}

pat_status pat_profile_end(pat_plan* plan, double* total_ms, int32_t* launches) {
  PAT_TRY(check_plan(plan));
  if (!plan->timer.ev) return set_error(PAT_ERR_INVALID, "pat_profile_end: profiling not active");
  DeviceGuard dg(plan->device);
  pat_status st = PAT_OK;
  hipError_t err = hipStreamSynchronize(plan->stream);
  if (err != hipSuccess) st = set_error(PAT_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
  double tot[K_COUNT] = {0};
  int cnt[K_COUNT] = {0};
  for (int i = 0; st == PAT_OK && i < plan->timer.count; ++i) {
    float ms = 0.f;
    err = hipEventElapsedTime(&ms, plan->timer.ev[2 * i], plan->timer.ev[2 * i + 1]);
    if (err != hipSuccess) {
      st = set_error(PAT_ERR_HIP, "hipEventElapsedTime: %s", hipGetErrorString(err));
      break;
    }
    tot[plan->timer.ids[i]] += ms;
    cnt[plan->timer.ids[i]] += plan->timer.nl[i];
  }
  for (hipEvent_t e : plan->timer_events) (void)hipEventDestroy(e);
  plan->timer_events.clear();
  plan->timer_ids.clear();
  plan->timer_nl.clear();
  plan->timer = KernelTimer{};
  if (st != PAT_OK) return st;
  for (int k = 0; k < K_COUNT; ++k) {
    if (total_ms) total_ms[k] = tot[k];
    if (launches) launches[k] = cnt[k];
  }
  return PAT_OK;
}

pat_status pat_copy_probe(const void* src, void* dst, int64_t nbytes, void* stream) {
  if (nbytes < 0 || nbytes % 16 || nbytes > (int64_t(1) << 40))
    return set_error(PAT_ERR_INVALID, "pat_copy_probe: nbytes must be a multiple of 16 in [0, 2^40]");
  if (nbytes == 0) return PAT_OK;
  if (!src || !dst) return set_error(PAT_ERR_INVALID, "pat_copy_probe: null pointer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u)
    return set_error(PAT_ERR_INVALID, "pat_copy_probe: src and dst must be 16-byte aligned");
  if (overlaps(src, (size_t)nbytes, dst, (size_t)nbytes))
    return set_error(PAT_ERR_INVALID, "pat_copy_probe: src and dst overlap");
  PAT_TRY_HIP(launch_copy_probe(src, dst, (long)(nbytes / 16), static_cast<hipStream_t>(stream)));
  return PAT_OK;
}

pat_status pat_kernel_info(const pat_plan* plan, int32_t kernel_id, const char** name, double* bytes_per_launch) {
  static const char* kNames[K_COUNT] = {"k_zgrad", "k_fwd_u",   "k_zmul<div>", "k_fwd_rho", "k_zmul<grad>",
                                        "k_adj_u", "k_zdiv_sum", "k_adj_rho",   "k_line<fwd>", "k_line<adj>"};
  // algorithmic HBM bytes per launch in units of C (one slab-spectrum field) and R (one real field);
  // a line step, per component: its lines (N^3/2 complex values, R bytes) of the three hub
  // spectra read, both states read and written, and one full output spectrum (C) written
  static const int kC[K_COUNT] = {4, 5, 6, 5, 6, 6, 4, 4, 3, 3};
  static const int kR[K_COUNT] = {0, 6, 0, 6, 0, 6, 0, 6, 21, 21};
  PAT_TRY(check_plan(plan));
  if (kernel_id < 0 || kernel_id >= K_COUNT) return set_error(PAT_ERR_INVALID, "pat_kernel_info: bad kernel_id");
  const double C = (double)n_spec(plan->g) * sizeof(float2), R = (double)n_voxels(plan->g) * sizeof(float);
  const double plane = (kernel_id == K_FWD_RHO || kernel_id == K_ADJ_RHO) ? (double)plan->npix * sizeof(float) : 0.0;
  if (name) *name = kNames[kernel_id];
  if (bytes_per_launch) *bytes_per_launch = kC[kernel_id] * C + kR[kernel_id] * R + plane;
  return PAT_OK;
}

pat_status pat_make_rsp_mask(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* idx_out) {
  return make_rsp_mask(n_pix, mc, seed, idx_out);
}

pat_status pat_make_shd_pattern(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* perm_out, int32_t* rows_out) {
  return make_shd_pattern(n_pix, mc, seed, perm_out, rows_out);
}

}  // extern "C"
