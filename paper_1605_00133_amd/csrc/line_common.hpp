// Host <-> kernel interface of the line propagator (cubic grids).
//
// The propagator of Sec. 4.3 (k-space pseudospectral scheme with split-field
// PML) is run with each field component xi held in its own mixed space: real
// along its axis xi, Fourier-transformed along the other two. The PML factors
// of component xi depend on xi only and the derivative multipliers are
// diagonal in k, so one time step of component xi is a set of independent
// lines along xi, each needing four 1D transforms:
//   g  = F^-1[ m+ P ]                      u <- a (a u - dt/rho0 g)
//   h  = F^-1[ m- F u ]                    rho <- b (b rho - dt rho0 h)
//   out = F rho                            P' = c0^2 (out_x + out_y + out_z)
// P is the 3D spectrum of the pressure (the "hub"), read by all three
// components and summed from their three outputs. The adjoint runs the
// transposed recurrence line by line in the same way.
//
// Layouts (N = grid edge, H = N/2):
//   hub spectra      [kz][kx <= H][ky_pos]         kz natural, ky_pos digit-reversed
//   states           [point along the axis][slot], N^2/2 slots per axis: one
//                    line of each conjugate pair (-P, -Q) ~ (P, Q) of the field,
//                    the four real lines two to a slot (line_kernels.hip, LineGeo)
// so a tile of 16 consecutive slots reads 128 contiguous bytes per point.
#pragma once

#include "wave_common.hpp"

namespace pat {

// FP64 tables by natural frequency index k < n (cubic grid: the same for every axis).
struct LineTables {
  const double2* mp;   // i k exp(+i k dx/2) (real at the Nyquist bin)
  const double2* mm;   // i k exp(-i k dx/2)
  const double* h;     // (c0 dt / 2) k
  const double2* tw;   // exp(-2 pi i j / n), j < n
  const double* kr;    // sinc(c0 dt |k| / 2) on the real lines: kr[c n + k], |k_perp|^2 = c (pi/dx)^2, c < 3
  const float* a[3];   // PML factor at staggered points i + 1/2, axis x, y, z
  const float* b[3];   // PML factor at collocated points i
};

struct LineScalars {
  double c2;                 // c0^2
  double dt_over_rho0;
  double dt_rho0;
  double half_dt_over_rho0;
  double inv_3c2;
  double inv_n;              // 1 / N (one inverse 1D transform)
  double inv_ntot;           // 1 / N^3
  double adj_scale;          // c0^2 dt / rho0 (adjoint hub)
};

struct LineBuffers {
  float2* su[3];        // velocity states
  float2* sr[3];        // density states
  float2* hub[2][3];    // ping-pong component spectra
  float2* planes;       // per-step plane spectra [nt][kx <= H][ky_pos]
  float2* spec;         // slab spectrum [z][kx <= H][ky_pos]
};

// forward: p0 (real volume) -> planes_real [nt][ny][nx] (pressure on z = 0)
using LineLaunchFwd = hipError_t (*)(const LineTables&, const LineScalars&, const LineBuffers&, const WaveTables&,
                                     const float* p0, float* planes_real, int nt, hipStream_t, KernelTimer*);
// adjoint: planes_real [nt][ny][nx] -> p (real volume)
using LineLaunchAdj = hipError_t (*)(const LineTables&, const LineScalars&, const LineBuffers&, const WaveTables&,
                                     const float* planes_real, float* p, int nt, hipStream_t, KernelTimer*);

struct LineImpl {
  int n;
  LineLaunchFwd forward;
  LineLaunchAdj adjoint;
};

// nullptr when the size is not built
const LineImpl* find_line_impl(int nx, int ny, int nz);

// Plain 2D slab transforms of a batch of slabs (implemented with the slab
// machinery of the wave kernels): real [nb][N][N] <-> spectrum [nb][H+1][N]
// (ky_pos order), times scale; FP64 arithmetic.
hipError_t launch_slab_r2c(int n, const float* in, float2* out, int nb, float scale, const WaveTables& t,
                           hipStream_t st);
hipError_t launch_slab_c2r(int n, const float2* in, float* out, int nb, float scale, const WaveTables& t,
                           hipStream_t st);

}  // namespace pat
