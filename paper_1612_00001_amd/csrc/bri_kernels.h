// Host launchers of the device kernels (bri_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bri_internal.h"

namespace bri {

template <typename T>
hipError_t launch_gemm(const GemmLaunch& L, int max_m, int max_n, hipStream_t st);
template <typename T>
hipError_t launch_getrf(const LuItem* d_items, int count, int b, hipStream_t st);
// wide: a float matrix's tile factorisations (pivot selection and the
// 32 x 32 LU with its triangular inverses) computed in double.
template <typename T>
hipError_t launch_getrf_tile(const LuItem* d_items, int count, int b, bool wide, hipStream_t st);
// Recursive LU that leaves the inverted factors in packed form (no
// triangular inversion follows); needs LuItem::tmp (a b x b shadow) and
// b = 32 * 2^m.  getrf_rec_applies() tells whether a launch of count
// matrices of order b takes it.
// lp: products of float matrices in split FP16 (1) or BF16 (2) parts, with
// range_flag as in GemmLaunch; 0 for FP32 / FP64 products.
template <typename T>
hipError_t launch_getrf_rec(const LuItem* d_items, int count, int b, bool wide, int lp, int32_t* range_flag,
                            hipStream_t st);
template <typename T>
// diag_inverted: the LU (tile pivoting) already left its diagonal 32 x 32 tiles inverted.
hipError_t launch_trtri(const LuItem* d_items, int count, int b, bool diag_inverted, hipStream_t st);
template <typename T>
hipError_t launch_load(const LoadItem* d_items, int count, int rows, int cols, hipStream_t st);
hipError_t launch_fill_int(int32_t* p, int n, int v, hipStream_t st);
// Device accounting of a plan step that has run (kind: a StepKind; elem:
// element size of its matrices): see bri_opts::d_stats.
hipError_t launch_stats(int kind, const void* items, int count, int elem, unsigned long long* stats,
                        const void* base, uint64_t limit, hipStream_t st);
// Diagonally dominant FP64 test matrices in the LU items (autotuner inputs).
hipError_t launch_fill_diag_dominant(const LuItem* d_items, int count, int b, hipStream_t st);
// Writes *src (passed by value as a kernel argument) to dst on the device.
hipError_t launch_store_rbf(RbfSource* dst, const RbfSource& src, hipStream_t st);

}  // namespace bri
