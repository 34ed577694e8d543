// Element-wise and reduction kernels of the mixed-precision refinement
// (FP64 residual, scaling into the low-precision recursion, update of the
// iterate with the norms of the convergence test).
//
// Device scalars (double scal[kRefineScalars]):
//   [0] max |M| (bit pattern of a non-negative double, updated by atomicMax),
//   [1] max |R| (same), [2] sum dX^2, [3] sum X^2.
// The power-of-two scales are derived from them on the device, so no host
// round trip sits between the residual and the correction solve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "bri_refine.h"

namespace bri {
namespace {

// 2^-e with |x| 2^-e in [0.5, 1); 1 for zero or non-finite x.
__device__ __forceinline__ double pow2_scale(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.0;
  int e = 0;
  (void)frexp(x, &e);
  return ldexp(1.0, -e);
}

__device__ __forceinline__ double bits_to_double(const double* p) {
  return __longlong_as_double(*reinterpret_cast<const long long*>(p));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_absmax(const T* p, int64_t rows, int64_t cols, int64_t ld, double* dst) {
  double m = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    const double v = fabs(static_cast<double>(p[r * ld + c]));
    m = (v > m || v != v) ? v : m;  // a NaN propagates (its bits order above +inf)
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(dst), static_cast<unsigned long long>(__double_as_longlong(m)));
}

// G = sigma * Gamma (kb x kb, leading dimension kb) in float, sigma from scal[0].
__global__ __launch_bounds__(256) void k_gamma_f32(const double* M, int64_t n, int64_t ldm, int64_t kb, float* G,
                                                   const double* scal) {
  const double sigma = pow2_scale(bits_to_double(scal));
  const int64_t total = kb * kb;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / kb, c = e - r * kb;
    const double v = (r < n && c < n) ? M[r * ldm + c] : (r == c ? 1.0 : 0.0);
    G[e] = static_cast<float>(sigma * v);
  }
}

// R = E_j - Gamma X given R[0:n) = -M X[0:n): adds the unit entries of E_j in
// rows < n and forms the identity-padding rows n <= r < kb.
__global__ __launch_bounds__(256) void k_resid_fix(double* R, const double* X, int64_t n, int64_t kb, int b,
                                                   int j) {
  const int64_t pad = kb - n;
  const int64_t total = static_cast<int64_t>(b) * (1 + pad);
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  if (e < b) {
    const int64_t r = static_cast<int64_t>(j) * b + e;
    if (r < n) R[r * b + e] += 1.0;
  } else {
    const int64_t q = e - b;
    const int64_t r = n + q / b, c = q % b;
    R[r * b + c] = (r == static_cast<int64_t>(j) * b + c ? 1.0 : 0.0) - X[r * b + c];
  }
}

// R32 = s R with s from scal[1].
__global__ __launch_bounds__(256) void k_rhs_scale(const double* R, float* R32, int64_t count, const double* scal) {
  const double s = pow2_scale(bits_to_double(scal + 1));
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    R32[e] = static_cast<float>(s * R[e]);
}

// X (+)= f D with f = sigma / s (first sweep: f = sigma, X overwritten);
// accumulates sum (f D)^2 into scal[2] and sum X^2 into scal[3].
__global__ __launch_bounds__(256) void k_refine_update(double* X, const float* D, int64_t count, double* scal,
                                                       int first) {
  const double sigma = pow2_scale(bits_to_double(scal));
  const double s = first ? 1.0 : pow2_scale(bits_to_double(scal + 1));
  const double f = sigma / s;
  double dd = 0.0, xx = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double d = f * static_cast<double>(D[e]);
    const double x = first ? d : X[e] + d;
    X[e] = x;
    dd += d * d;
    xx += x * x;
  }
  dd = wave_sum(dd);
  xx = wave_sum(xx);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(scal + 2, dd);
    atomicAdd(scal + 3, xx);
  }
}

// Clears scal[from, to).
__global__ void k_scal_clear(double* scal, int from, int to) {
  const int e = from + static_cast<int>(threadIdx.x);
  if (e < to) scal[e] = 0.0;
}

// Refinement did not converge: report -1 unless a pivot failure is recorded.
__global__ void k_info_unconverged(int32_t* info) {
  if (threadIdx.x == 0 && *info == 0) *info = -1;
}

inline int grid_for(int64_t count) {
  const int64_t g = (count + 255) / 256;
  return static_cast<int>(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

hipError_t launch_absmax(const void* p, int elem, int64_t rows, int64_t cols, int64_t ld, double* dst,
                         hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int g = grid_for(rows * cols);
  if (elem == 8)
    hipLaunchKernelGGL(k_absmax<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(p), rows, cols, ld,
                       dst);
  else
    hipLaunchKernelGGL(k_absmax<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(p), rows, cols, ld,
                       dst);
  return hipGetLastError();
}

hipError_t launch_gamma_f32(const double* M, int64_t n, int64_t ldm, int64_t kb, float* G, const double* scal,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_gamma_f32, dim3(grid_for(kb * kb)), dim3(256), 0, st, M, n, ldm, kb, G, scal);
  return hipGetLastError();
}

hipError_t launch_resid_fix(double* R, const double* X, int64_t n, int64_t kb, int b, int j, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(b) * (1 + kb - n);
  hipLaunchKernelGGL(k_resid_fix, dim3(static_cast<int>((total + 255) / 256)), dim3(256), 0, st, R, X, n, kb, b, j);
  return hipGetLastError();
}

hipError_t launch_rhs_scale(const double* R, float* R32, int64_t count, const double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_scale, dim3(grid_for(count)), dim3(256), 0, st, R, R32, count, scal);
  return hipGetLastError();
}

hipError_t launch_refine_update(double* X, const float* D, int64_t count, double* scal, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_update, dim3(grid_for(count)), dim3(256), 0, st, X, D, count, scal, first);
  return hipGetLastError();
}

hipError_t launch_scal_clear(double* scal, int from, int to, hipStream_t st) {
  hipLaunchKernelGGL(k_scal_clear, dim3(1), dim3(64), 0, st, scal, from, to);
  return hipGetLastError();
}

hipError_t launch_info_unconverged(int32_t* info, hipStream_t st) {
  hipLaunchKernelGGL(k_info_unconverged, dim3(1), dim3(64), 0, st, info);
  return hipGetLastError();
}

}  // namespace bri
