// Host launchers of the refinement kernels (bri_refine.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bri {

constexpr int kRefineScalars = 8;

// atomicMax of |p| over a rows x cols array (double or float) into the
// non-negative double at dst (which the caller clears first).
hipError_t launch_absmax(const void* p, int elem, int64_t rows, int64_t cols, int64_t ld, double* dst,
                         hipStream_t st);
// G = sigma * Gamma in float, kb x kb, sigma = 2^-e from max |M| in scal[0].
hipError_t launch_gamma_f32(const double* M, int64_t n, int64_t ldm, int64_t kb, float* G, const double* scal,
                            hipStream_t st);
// Completes R = E_j - Gamma X after R[0:n) = -M X[0:n) (R, X: kb x b, ld b).
hipError_t launch_resid_fix(double* R, const double* X, int64_t n, int64_t kb, int b, int j, hipStream_t st);
// R32 = s R, s = 2^-e from max |R| in scal[1].
hipError_t launch_rhs_scale(const double* R, float* R32, int64_t count, const double* scal, hipStream_t st);
// X (+)= (sigma / s) D and the squared norms of the update and of X.
hipError_t launch_refine_update(double* X, const float* D, int64_t count, double* scal, int first, hipStream_t st);
hipError_t launch_scal_clear(double* scal, int from, int to, hipStream_t st);
hipError_t launch_info_unconverged(int32_t* info, hipStream_t st);

}  // namespace bri
