// Element-wise and reduction kernels of the mixed-precision refinement
// (FP64 residual, scaling into the low-precision recursion, update of the
// iterate with the norms of the convergence test).  Every kernel serves a
// list of problems: blockIdx.y selects the problem, the x dimension strides
// over its elements.  The power-of-two scales are derived from the device
// scalars on the device, so no host round trip sits between the residual and
// the correction solve.
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

// Maximum that propagates a NaN (fmax would drop it).
__device__ __forceinline__ double nan_max(double m, double v) { return (v > m || v != v) ? v : m; }
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reductions over the 256 threads of a workgroup (every thread gets the
// result); one atomic per workgroup then updates the problem's scalar, so
// the scalars see few atomic operations.
__device__ __forceinline__ double block_max(double v) {
  __shared__ double part[4];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = part[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) m = nan_max(m, part[w]);
  return m;
}
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double part[2][4];
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = a;
    part[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  a = part[0][0] + part[0][1] + part[0][2] + part[0][3];
  b = part[1][0] + part[1][1] + part[1][2] + part[1][3];
}

__device__ __forceinline__ int64_t first_elem() { return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t elem_stride() { return static_cast<int64_t>(gridDim.x) * blockDim.x; }

__global__ __launch_bounds__(256) void k_absmax(const RefItem* items, int which) {
  const RefItem it = items[blockIdx.y];
  const int64_t rows = which ? it.kb : it.n, cols = which ? it.b : it.n, ld = which ? it.b : it.ldm;
  const double* p = which ? it.R : it.M;
  double m = 0.0;
  for (int64_t e = first_elem(); e < rows * cols; e += elem_stride()) {
    const int64_t r = e / cols, c = e - r * cols;
    const double v = fabs(p[r * ld + c]);
    m = nan_max(m, v);  // a NaN propagates (its bits order above +inf in the atomic maximum)
  }
  m = block_max(m);
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(it.scal + which),
              static_cast<unsigned long long>(__double_as_longlong(m)));
}

// R = E_j - Gamma X given R[0:n) = -M X[0:n): adds the unit entries of E_j in
// rows < n and forms the identity-padding rows n <= r < kb.
__global__ __launch_bounds__(256) void k_resid_fix(const RefItem* items) {
  const RefItem it = items[blockIdx.y];
  const int64_t b = it.b, pad = it.kb - it.n, jb = static_cast<int64_t>(it.j) * b;
  for (int64_t e = first_elem(); e < b * (1 + pad); e += elem_stride()) {
    if (e < b) {
      const int64_t r = jb + e;
      if (r < it.n) it.R[r * b + e] += 1.0;
    } else {
      const int64_t q = e - b;
      const int64_t r = it.n + q / b, c = q % b;
      it.R[r * b + c] = (r == jb + c ? 1.0 : 0.0) - it.X[r * b + c];
    }
  }
}

// R32 = s R with s from scal[1].
__global__ __launch_bounds__(256) void k_rhs_scale(const RefItem* items) {
  const RefItem it = items[blockIdx.y];
  const double s = pow2_scale(bits_to_double(it.scal + 1));
  for (int64_t e = first_elem(); e < it.kb * it.b; e += elem_stride()) it.R32[e] = static_cast<float>(s * it.R[e]);
}

// X (+)= f D with f = sigma / s (first sweep: f = sigma, X overwritten);
// accumulates sum (f D)^2 into scal[2] and sum X^2 into scal[3].
__global__ __launch_bounds__(256) void k_refine_update(const RefItem* items, int first) {
  const RefItem it = items[blockIdx.y];
  const double sigma = pow2_scale(bits_to_double(it.scal));
  const double s = first ? 1.0 : pow2_scale(bits_to_double(it.scal + 1));
  const double f = sigma / s;
  double dd = 0.0, xx = 0.0;
  for (int64_t e = first_elem(); e < it.kb * it.b; e += elem_stride()) {
    const double d = f * static_cast<double>(it.D[e]);
    const double x = first ? d : it.X[e] + d;
    it.X[e] = x;
    dd += d * d;
    xx += x * x;
  }
  block_sum2(dd, xx);
  if (threadIdx.x == 0) {
    atomicAdd(it.scal + 2, dd);
    atomicAdd(it.scal + 3, xx);
  }
}

// R32 = E_j (the unit block column j of Gamma's order).
__global__ __launch_bounds__(256) void k_set_ej(const RefItem* items) {
  const RefItem it = items[blockIdx.y];
  const int64_t jb = static_cast<int64_t>(it.j) * it.b;
  for (int64_t e = first_elem(); e < it.kb * it.b; e += elem_stride()) {
    const int64_t r = e / it.b, c = e - r * it.b;
    it.R32[e] = (r == jb + c) ? 1.0f : 0.0f;
  }
}

__global__ void k_scal_clear(const RefItem* items, int from, int to) {
  const int e = from + static_cast<int>(threadIdx.x);
  if (e < to) items[blockIdx.y].scal[e] = 0.0;
}

// Refinement did not converge: report -1 unless a pivot failure is recorded.
__global__ void k_info_unconverged(int32_t* info) {
  if (threadIdx.x == 0 && *info == 0) *info = -1;
}

// x extent: enough workgroups for the largest problem, fewer per problem when
// there are many problems (every workgroup strides over its problem).
// Reductions: at most 256 workgroups per problem (each thread then streams
// many elements), so that few atomics reach the problem's scalars.
inline dim3 grid_reduce(int64_t max_elems, int count) {
  int64_t g = (max_elems + 255) / 256;
  int64_t cap = 65536 / (count > 0 ? count : 1);
  cap = cap < 16 ? 16 : (cap > 256 ? 256 : cap);
  g = g < 1 ? 1 : (g > cap ? cap : g);
  return dim3(static_cast<unsigned>(g), static_cast<unsigned>(count));
}

inline dim3 grid_for(int64_t max_elems, int count) {
  int64_t g = (max_elems + 255) / 256;
  int64_t cap = 65536 / (count > 0 ? count : 1);
  cap = cap < 16 ? 16 : (cap > 2048 ? 2048 : cap);
  g = g < 1 ? 1 : (g > cap ? cap : g);
  return dim3(static_cast<unsigned>(g), static_cast<unsigned>(count));
}

}  // namespace

hipError_t launch_absmax(const RefItem* items, int count, int which, int64_t max_elems, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_absmax, grid_reduce(max_elems, count), dim3(256), 0, st, items, which);
  return hipGetLastError();
}

hipError_t launch_resid_fix(const RefItem* items, int count, int64_t max_elems, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid_fix, grid_for(max_elems, count), dim3(256), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_rhs_scale(const RefItem* items, int count, int64_t max_elems, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs_scale, grid_for(max_elems, count), dim3(256), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_refine_update(const RefItem* items, int count, int64_t max_elems, int first, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_update, grid_reduce(max_elems, count), dim3(256), 0, st, items, first);
  return hipGetLastError();
}

hipError_t launch_set_ej(const RefItem* items, int count, int64_t max_elems, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_ej, grid_for(max_elems, count), dim3(256), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_scal_clear(const RefItem* items, int count, int from, int to, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scal_clear, dim3(1, count), dim3(64), 0, st, items, from, to);
  return hipGetLastError();
}

hipError_t launch_info_unconverged(int32_t* info, hipStream_t st) {
  hipLaunchKernelGGL(k_info_unconverged, dim3(1), dim3(64), 0, st, info);
  return hipGetLastError();
}

}  // namespace bri
