// Host launchers of the refinement kernels (bri_refine.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bri {

constexpr int kRefineScalars = 8;

// One problem of a (possibly merged) mixed-precision call.  Device scalars
// scal[kRefineScalars]: [0] max |M|, [1] max |R| (bit patterns of non-negative
// doubles, updated by atomicMax), [2] sum dX^2, [3] sum X^2.
struct RefItem {
  const double* M;  // n x n, leading dimension ldm
  int64_t n, ldm, kb;
  int32_t b, j;     // block order, target block column
  double* X;        // iterate, kb x b
  double* R;        // residual, kb x b
  float* R32;       // s R
  float* D;         // float solve output, kb x b
  double* scal;
};

// All launchers take a device array of count items; largest sizes bound the grid.
// atomicMax of |M| (which = 0) or |R| (which = 1) into scal[which] (cleared first).
hipError_t launch_absmax(const RefItem* items, int count, int which, int64_t max_elems, hipStream_t st);
// Completes R = E_j - Gamma X after R[0:n) = -M X[0:n).
hipError_t launch_resid_fix(const RefItem* items, int count, int64_t max_elems, hipStream_t st);
// R32 = s R, s = 2^-e from max |R|.
hipError_t launch_rhs_scale(const RefItem* items, int count, int64_t max_elems, hipStream_t st);
// X (+)= (sigma / s) D and the squared norms of the update and of X.
hipError_t launch_refine_update(const RefItem* items, int count, int64_t max_elems, int first, hipStream_t st);
// R32 = E_j.
hipError_t launch_set_ej(const RefItem* items, int count, int64_t max_elems, hipStream_t st);
// Clears scal[from, to) of every item.
hipError_t launch_scal_clear(const RefItem* items, int count, int from, int to, hipStream_t st);
// *info = -1 where *info == 0 (refinement did not converge).
hipError_t launch_info_unconverged(int32_t* info, hipStream_t st);

}  // namespace bri
