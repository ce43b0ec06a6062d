// Shared definitions of the wave propagator (host plan <-> kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace pat {

// Device tables of one grid, built in FP64 on the host and rounded once.
// Spectral arrays use the slab-spectrum layout [z][kx][ky_pos]:
//   kx in [0, nx/2] natural order (half spectrum of the real x transform),
//   ky_pos = position of ky after the forward y transform (digit-reversed),
//   and in the z-pencil kernels kz_pos likewise for z.
// The spectral tables exist in both arithmetic types (float2 / double2).
template <typename V, typename S>
struct SpecTables {
  const V* tw_mx;   // exp(-2 pi i j / (nx/2)), j < nx/2
  const V* tw_nx;   // exp(-2 pi i k / nx),     k <= nx/2
  const V* tw_y;    // exp(-2 pi i j / ny),     j < ny
  const V* tw_z;    // exp(-2 pi i j / nz),     j < nz
  const V* mpx;     // i kx exp(+i kx dx/2), indexed by kx
  const V* mmx;     // i kx exp(-i kx dx/2)
  const V* mpy;     // same for y, indexed by ky_pos
  const V* mmy;
  const V* mpz;     // same for z, indexed by kz_pos
  const V* mmz;
  const S* hx;      // (c0 dt / 2) kx   (argument scale of the k-space sinc)
  const S* hy;      // by ky_pos
  const S* hz;      // by kz_pos
};

struct WaveTables {
  SpecTables<float2, float> f;
  SpecTables<double2, double> d;
  const float* ax;       // PML factor at staggered points i + 1/2
  const float* ay;
  const float* az;
  const float* bx;       // PML factor at collocated points i
  const float* by;
  const float* bz;
};

struct WaveScalars {
  float dt_over_rho0;    // dt / rho0
  float dt_rho0;         // dt * rho0
  float c2;              // c0^2
  float inv_3c2;         // 1 / (3 c0^2)
  float half_dt_over_rho0;  // dt / (2 rho0)
  float inv_ntot;        // 1 / (nx ny nz): normalisation of an FFT round trip
};

// Launch helpers implemented per grid size in wave_kernels.hip.
struct WaveBuffers {
  float* u[3];           // velocity components (staggered), [nz][ny][nx]
  float* rho[3];         // split density components
  float2* spec[4];       // slab spectra [nz][nx/2+1][ny]
  const float* c2f;      // forward only: c(x)^2 [nz][ny][nx] of a heterogeneous medium, or null (c0^2)
};

// Kernels of one time step, for per-kernel timing.
enum KernelId {
  K_ZGRAD = 0,      // forward pencil pass of the gradient (2 spectra in, 2 out)
  K_FWD_U = 1,      // forward slab pass: velocity update + R2C (per component)
  K_ZDIV = 2,       // forward pencil pass of the divergences (per component)
  K_FWD_RHO = 3,    // forward slab pass: density update, sensor plane, R2C (two halves per slab)
  K_ZGRAD_ADJ = 4,  // adjoint pencil pass of the gradients (per component)
  K_ADJ_U = 5,      // adjoint slab pass: velocity update + R2C (per component)
  K_ZDIV_SUM = 6,   // adjoint pencil pass of the summed divergence (3 in, 1 out)
  K_ADJ_RHO = 7,    // adjoint slab pass: density update + source + R2C (two halves per slab)
  K_LINE_FWD = 8,   // line propagator: one forward time step of all three components
  K_LINE_ADJ = 9,   // line propagator: one adjoint time step
  K_COUNT = 10
};

// Optional HIP-event bracketing of kernel launches (which = id, or -2 for all).
struct KernelTimer {
  int which;
  hipEvent_t* ev;   // 2 per record
  int* ids;         // kernel id of each record
  int* nl;          // launches a record spans
  int cap;
  int count;
};

// Runs launch(), bracketed by timer events when kernel id is being recorded.
template <typename F>
inline void timed(KernelTimer* kt, int id, hipStream_t st, F&& launch) {
  const bool on = kt && (kt->which == id || kt->which == -2) && kt->count < kt->cap;
  if (on) (void)hipEventRecord(kt->ev[2 * kt->count], st);
  launch();
  if (on) {
    (void)hipEventRecord(kt->ev[2 * kt->count + 1], st);
    kt->ids[kt->count] = id;
    kt->nl[kt->count] = 1;
    kt->count++;
  }
}

// A run of `launches` consecutive launches of kernel id with nothing else on
// the stream between them (the time steps of one application), bracketed by
// one pair of events: per-launch events add their own gaps to every launch.
// timed_span_begin returns the record index, or -1 when not recording.
inline int timed_span_begin(KernelTimer* kt, int id, hipStream_t st) {
  const bool on = kt && (kt->which == id || kt->which == -2) && kt->count < kt->cap;
  if (!on) return -1;
  (void)hipEventRecord(kt->ev[2 * kt->count], st);
  return kt->count++;
}
inline void timed_span_end(KernelTimer* kt, int rec, int id, int launches, hipStream_t st) {
  if (rec < 0) return;
  (void)hipEventRecord(kt->ev[2 * rec + 1], st);
  kt->ids[rec] = id;
  kt->nl[rec] = launches;
}

// Hand-off flags of the slab-pair velocity passes (device, >= nz entries, zero
// at plan creation) and the host-side launch epoch that tags them.
struct HandOff {
  unsigned* flags;
  unsigned epoch;
};

// Forward: planes receives two sensor-plane series, [2][nt][ny][nx] (the two
// halves of the density pass); their sum is p on the plane z = 0.
using WaveLaunchFwd = hipError_t (*)(const WaveTables&, const WaveScalars&, const WaveBuffers&,
                                     const float* p0, float* planes2, int nt, hipStream_t, KernelTimer*, HandOff&);
using WaveLaunchAdj = hipError_t (*)(const WaveTables&, const WaveScalars&, const WaveBuffers&,
                                     const float* planes, float* p, int nt, hipStream_t, KernelTimer*, HandOff&);

// FFT arithmetic of the propagator kernels: FP32, or FP64 in registers and
// LDS with FP32 storage in HBM.
enum FftPrecision { FFT_FP32 = 0, FFT_FP64 = 1 };

// time reversal: planes [nt][ny][nx] -> p = p_a + p_b (nt > 1) or vol (nt = 1); see wave_kernels.hip
using WaveLaunchTR = hipError_t (*)(const WaveTables&, const WaveScalars&, const WaveBuffers&, const float* planes,
                                    float* vol, float* p_a, float* p_b, float* tplanes, int nt, hipStream_t,
                                    HandOff&);

struct WaveImpl {
  int nx, ny, nz;
  WaveLaunchFwd forward[2];   // indexed by FftPrecision
  WaveLaunchAdj adjoint[2];
  WaveLaunchTR time_reversal[2];
};

// Returns nullptr when the size is not built.
const WaveImpl* find_wave_impl(int nx, int ny, int nz);

}  // namespace pat
