// Launchers of the sampling kernels (sample_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace pat {

hipError_t launch_rsp_gather(const float* s, const int* idx, float* f, int npix, int mc, int nt, hipStream_t st);
hipError_t launch_rsp_scatter(const float* f, const int* inv, float* s, int npix, int mc, int nt, hipStream_t st);
hipError_t launch_shd_forward(const float* s, const int* perm, const int* rows, float* f, int npix, int mc, int nt,
                              hipStream_t st);
hipError_t launch_shd_adjoint(const float* f, const int* invperm, const int* rows, float* s, int npix, int mc, int nt,
                              hipStream_t st);
int shd_max_pixels();

}  // namespace pat
