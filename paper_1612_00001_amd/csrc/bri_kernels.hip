// Device kernels of the block recursive inverse for gfx950 (CDNA4).
//
//  * k_gemm      -- batched C = beta*Cin + alpha*A*B - Sub on MFMA
//                   (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32), LDS
//                   double-buffered tiles.  Operands are views (bri::DView)
//                   that synthesise the identity padding of Gamma
//                   (eq. M_augmented), transposes, triangular masks and row
//                   permutations, so no operand is ever copied or padded.
//                   It realises every product of the Schur complement
//                   D - C A^{-1} B (eqs. SchurofA..SchurofD), the trailing
//                   updates of the LU and the recursive-doubling triangular
//                   inversion.
//  * k_getf2     -- LU with partial pivoting of one tall panel per matrix,
//                   held in registers by one 512-thread workgroup.
//  * k_laswp_trsm-- applies a panel's row interchanges to the other columns
//                   and solves the unit-lower panel system for the block row.
//  * k_trtri_diag-- inverts the 32 x 32 diagonal tiles of L and U.
//  * k_load      -- copies a view into a dense workspace block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <utility>

#include "bri_internal.h"
#include "bri_kernels.h"

namespace bri {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Views
// ---------------------------------------------------------------------------
// 2^-e with |x| 2^-e in [0.5, 1); 1 for zero or non-finite x.
__device__ __forceinline__ double pow2_scale_of(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.0;
  int e = 0;
  (void)frexp(x, &e);
  return ldexp(1.0, -e);
}

// Element (r, c) of the matrix an RbfSource describes (see its definition);
// T is the element type of the data points.
template <typename T>
__device__ __forceinline__ double rbf_element(const RbfSource& s, int64_t r, int64_t c) {
  if (r == 0 || c == 0) return (r == 0 && c == 0) ? 0.0 : 1.0;
  const T* xr = static_cast<const T*>(s.X) + (r - 1) * s.ldx;
  const T* xc = static_cast<const T*>(s.X) + (c - 1) * s.ldx;
  double d2 = 0.0;
  for (int t = 0; t < s.d; ++t) {
    const double u = static_cast<double>(xr[t]) - static_cast<double>(xc[t]);
    d2 = fma(u, u, d2);
  }
  return exp(-d2 * s.inv_two_sigma2) + (r == c ? s.inv_gamma : 0.0);
}

template <typename T>
__device__ __forceinline__ T vget(const DView& v, int x, int y) {
  if (v.tri == 1) {
    if (x == y) return T(1);
    if (x < y) return T(0);
  } else if (v.tri == 2) {
    if (x > y) return T(0);
  }
  const int xs = v.rowperm ? v.rowperm[x] : x;
  if (v.rbf) {
    if (xs < v.rows && y < v.cols)
      return static_cast<T>(rbf_element<T>(*v.rbf, static_cast<int64_t>(v.r0) + xs, static_cast<int64_t>(v.c0) + y));
    return (xs - y == v.diag) ? T(1) : T(0);
  }
  if (v.src64_max) {
    double e = (xs - y == v.diag) ? 1.0 : 0.0;
    if (xs < v.rows && y < v.cols) {
      const double* p = static_cast<const double*>(v.p);
      e = v.trans ? p[static_cast<int64_t>(y) * v.ld + xs] : p[static_cast<int64_t>(xs) * v.ld + y];
    }
    return static_cast<T>(e * pow2_scale_of(*v.src64_max));
  }
  if (xs < v.rows && y < v.cols) {
    const T* p = static_cast<const T*>(v.p);
    return v.trans ? p[static_cast<int64_t>(y) * v.ld + xs] : p[static_cast<int64_t>(xs) * v.ld + y];
  }
  return (xs - y == v.diag) ? T(1) : T(0);
}

__device__ __forceinline__ DView dense_view(const void* base, int64_t ld, int64_t r0, int64_t c0, int rows, int cols,
                                            int elem, int tri = 0) {
  DView v;
  v.p = static_cast<const char*>(base) + (r0 * ld + c0) * elem;
  v.ld = ld;
  v.rowperm = nullptr;
  v.rows = rows;
  v.cols = cols;
  v.diag = INT_MIN / 2;
  v.trans = 0;
  v.tri = static_cast<int16_t>(tri);
  v.src64_max = nullptr;
  v.rbf = nullptr;
  v.r0 = v.c0 = 0;
  return v;
}

// ---------------------------------------------------------------------------
// MFMA traits
// ---------------------------------------------------------------------------
template <typename T>
struct MF;
template <>
struct MF<double> {
  typedef d4_t acc;
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // Output element v of lane l sits at row (l/16) + 4 v, column l % 16.
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MF<float> {
  typedef f4_t acc;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // Output element v of lane l sits at row 4 (l/16) + v, column l % 16.
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Records a wavefront's largest magnitude m (non-negative, or NaN) into the
// float-bit maximum at *w.  All lanes of the wavefront take part.
__device__ __forceinline__ void note_umax(int32_t* w, float m) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float x = __shfl_xor(m, o, 64);
    m = (x > m || x != x) ? x : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int*>(w), __float_as_uint(m));
}
__device__ __forceinline__ float nan_fmax(float m, float v) { return (v > m || v != v) ? v : m; }

// ---------------------------------------------------------------------------
// GEMM work items
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__device__ bool gemm_item(const GemmLaunch& L, int idx, GemmItem& it) {
  const int E = sizeof(T);
  if (MODE == GEMM_EXPLICIT) {
    it = static_cast<const GemmItem*>(L.items)[idx];
    return true;
  }
  it.umax = nullptr;
  if (MODE == GEMM_LU_TRAILING) {
    const LuItem lu = static_cast<const LuItem*>(L.items)[idx];
    const int b = lu.b, j = L.j, w = L.w, m = b - j - w;
    if (m <= 0) return false;
    it.A = dense_view(lu.a, b, j + w, j, m, w, E);
    it.B = dense_view(lu.a, b, j, j + w, w, m, E);
    it.Cin = dense_view(lu.a, b, j + w, j + w, m, m, E);
    it.Sub = it.Cin;
    it.out = static_cast<char*>(lu.a) + (static_cast<int64_t>(j + w) * b + j + w) * E;
    it.ldo = b;
    it.M = m;
    it.N = m;
    it.K = w;
    it.has_cin = 1;
    it.has_sub = 0;
    it.alpha = -1.0;
    it.beta = 1.0;
    return true;
  }
  if (MODE == GEMM_RLU_A || MODE == GEMM_RLU_B || MODE == GEMM_RLU_C || MODE == GEMM_RLU_D) {
    // Node of the recursive LU at origin o with halves of order h.  Packed
    // block (1,1) holds L11^{-1} (strictly lower) and U11^{-1} (upper) once
    // the first half is done, likewise (2,2); the shadow sh (b x b, same
    // coordinates) holds the node's intermediate blocks at their positions.
    constexpr int P = MODE == GEMM_RLU_D ? 1 : 2;
    const int np = L.part ? 1 : P;
    const int part = L.part ? L.part - 1 : idx % P;
    const LuItem lu = static_cast<const LuItem*>(L.items)[idx / np];
    const int b = lu.b, o = L.j, h = L.s;
    if (o + 2 * h > b) return false;
    char* a = static_cast<char*>(lu.a);
    char* sh = static_cast<char*>(lu.tmp);
    it.has_cin = 0;
    it.has_sub = 0;
    it.beta = 0.0;
    it.alpha = 1.0;
    it.Cin = dense_view(a, b, 0, 0, 0, 0, E);
    it.Sub = it.Cin;
    it.M = it.N = it.K = h;
    it.ldo = b;
    // A row-permuted view: element (x, y) is stored row perm[x] (an index
    // of the b x b matrix) of column c0 + y.
    auto permuted = [&](char* base, int c0, int r0) {
      DView v = dense_view(base, b, 0, c0, b, h, E);
      v.rowperm = lu.perm + r0;
      return v;
    };
    const int64_t o1 = o, o2 = o + h;
    if (MODE == GEMM_RLU_A) {
      if (part == 0) {  // U12 = L11^{-1} (P1 A12): the block (1,2) of U, its growth recorded
        it.A = dense_view(a, b, o1, o1, h, h, E, 1);
        it.B = permuted(a, o2, o1);
        it.out = sh + (o1 * b + o2) * E;
        it.umax = lu.swaps + kUmaxWord;
      } else {          // L21 = A21 U11^{-1}
        it.A = dense_view(a, b, o2, o1, h, h, E);
        it.B = dense_view(a, b, o1, o1, h, h, E, 2);
        it.out = sh + (o2 * b + o1) * E;
      }
    } else if (MODE == GEMM_RLU_B) {
      if (part == 0) {  // A22 = A22 - L21 U12 (the Schur complement the second half factors)
        it.A = dense_view(sh, b, o2, o1, h, h, E);
        it.B = dense_view(sh, b, o1, o2, h, h, E);
        it.Cin = dense_view(a, b, o2, o2, h, h, E);
        it.has_cin = 1;
        it.beta = 1.0;
        it.alpha = -1.0;
        it.out = a + (o2 * b + o2) * E;
      } else {          // Y = U11^{-1} U12
        it.A = dense_view(a, b, o1, o1, h, h, E, 2);
        it.B = dense_view(sh, b, o1, o2, h, h, E);
        it.out = sh + (o1 * b + o1) * E;
      }
    } else if (MODE == GEMM_RLU_C) {
      if (part == 0) {  // X = L22^{-1} (P2 L21)
        it.A = dense_view(a, b, o2, o2, h, h, E, 1);
        it.B = permuted(sh, o1, o2);
        it.out = sh + (o2 * b + o2) * E;
      } else {          // block (1,2) of U^{-1}: -Y U22^{-1}
        it.A = dense_view(sh, b, o1, o1, h, h, E);
        it.B = dense_view(a, b, o2, o2, h, h, E, 2);
        it.alpha = -1.0;
        it.out = a + (o1 * b + o2) * E;
      }
    } else {            // block (2,1) of L^{-1}: -X L11^{-1}
      it.A = dense_view(sh, b, o2, o2, h, h, E);
      it.B = dense_view(a, b, o1, o1, h, h, E, 1);
      it.alpha = -1.0;
      it.out = a + (o2 * b + o1) * E;
    }
    return true;
  }
  // Recursive-doubling inversion of the packed triangular factors.  Pair pi of
  // level s covers rows/cols [o, o + s + s2), o = 2 s pi, s2 = min(s, b - o - s).
  // L part: inv([[A, 0], [C, D]]) lower-left = -D^{-1} C A^{-1}.
  // U part: inv([[A, B], [0, D]]) upper-right = -A^{-1} B D^{-1}.
  const int part = idx & 1;
  const int pi = (idx >> 1) % L.npairs;
  const int mi = (idx >> 1) / L.npairs;
  const LuItem lu = static_cast<const LuItem*>(L.items)[mi];
  const int b = lu.b, s = L.s, o = 2 * s * pi;
  if (o + s >= b) return false;
  const int s2 = min(s, b - o - s);
  char* tmp = static_cast<char*>(lu.tmp) + static_cast<int64_t>(2) * s * s * pi * E;
  it.has_cin = 0;
  it.has_sub = 0;
  it.beta = 0.0;
  it.Cin = dense_view(lu.a, b, 0, 0, 0, 0, E);
  it.Sub = it.Cin;
  if (part == 0) {
    char* tl = tmp;  // s2 x s, ld s
    if (MODE == GEMM_TRTRI_STEP1) {
      it.A = dense_view(lu.a, b, o + s, o, s2, s, E);        // C
      it.B = dense_view(lu.a, b, o, o, s, s, E, 1);          // A^{-1}, unit lower
      it.out = tl;
      it.ldo = s;
      it.M = s2;
      it.N = s;
      it.K = s;
      it.alpha = 1.0;
    } else {
      it.A = dense_view(lu.a, b, o + s, o + s, s2, s2, E, 1);  // D^{-1}, unit lower
      it.B = dense_view(tl, s, 0, 0, s2, s, E);
      it.out = static_cast<char*>(lu.a) + (static_cast<int64_t>(o + s) * b + o) * E;
      it.ldo = b;
      it.M = s2;
      it.N = s;
      it.K = s2;
      it.alpha = -1.0;
    }
  } else {
    char* tu = tmp + static_cast<int64_t>(s) * s2 * E;  // s x s2, ld s2
    if (MODE == GEMM_TRTRI_STEP1) {
      it.A = dense_view(lu.a, b, o, o + s, s, s2, E);          // B
      it.B = dense_view(lu.a, b, o + s, o + s, s2, s2, E, 2);  // D^{-1}, upper
      it.out = tu;
      it.ldo = s2;
      it.M = s;
      it.N = s2;
      it.K = s2;
      it.alpha = 1.0;
    } else {
      it.A = dense_view(lu.a, b, o, o, s, s, E, 2);            // A^{-1}, upper
      it.B = dense_view(tu, s2, 0, 0, s, s2, E);
      it.out = static_cast<char*>(lu.a) + (static_cast<int64_t>(o) * b + o + s) * E;
      it.ldo = b;
      it.M = s;
      it.N = s2;
      it.K = s;
      it.alpha = -1.0;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Operand tiles.  The fast GEMM instance handles operands that are either
// stored data covering every element the product reads (optionally through
// a row permutation and/or a triangular mask) or synthesised (no data:
// element = (x - y == diag), the identity or zero).  Loads are issued into
// raw registers and only consumed after the MFMA work of the current K-tile,
// when bounds and masks are applied on the way into LDS.  The thread-to-
// element mapping follows the contiguous direction of the stored data so that
// every load instruction is coalesced.  Operands that need element-wise view
// evaluation (tiles crossing the identity padding of Gamma) use the generic
// instance (GEN = true), chosen per item on the host.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)(p) = v;
}

template <typename T, int R, int C, int NT>
struct TileOp {
  static constexpr int E = R * C / NT;
  bool synth, trans;
  const T* p;
  int64_t ld;
  const int32_t* perm;  // LDS copy of the row permutation, or null
  int tri, diag;
  int xlim, ylim;       // product operand extent (M x K for A, K x N for B)
  int r0, dr, c0, dc;   // this thread's first local (row, col) and per-element step
  T raw[E];

  __device__ __forceinline__ void init(const DView& v, const int32_t* perm_lds, int xlim_, int ylim_, int tid) {
    trans = v.trans != 0;
    p = static_cast<const T*>(v.p);
    ld = v.ld;
    perm = v.rowperm ? perm_lds : nullptr;
    tri = v.tri;
    diag = v.diag;
    xlim = xlim_;
    ylim = ylim_;
    synth = p == nullptr;
    if (!trans) {  // contiguous along y
      r0 = tid / C;
      dr = NT / C;
      c0 = tid % C;
      dc = 0;
    } else {       // contiguous along x
      r0 = tid % R;
      dr = 0;
      c0 = tid / R;
      dc = NT / R;
    }
  }

  __device__ __forceinline__ void issue(int x0, int y0) {
    if (synth) return;
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int x = min(x0 + r0 + t * dr, xlim - 1);
      const int y = min(y0 + c0 + t * dc, ylim - 1);
      const int xs = perm ? perm[x] : x;
      raw[t] = trans ? gload(p + static_cast<int64_t>(y) * ld + xs) : gload(p + static_cast<int64_t>(xs) * ld + y);
    }
  }

  __device__ __forceinline__ T finalize(int t, int x0, int y0) const {
    const int x = x0 + r0 + t * dr, y = y0 + c0 + t * dc;
    T v;
    if (synth) {
      const int xs = perm ? perm[min(x, xlim - 1)] : x;
      v = (xs - y == diag) ? T(1) : T(0);
    } else {
      v = raw[t];
    }
    if (tri == 1) v = x > y ? v : (x == y ? T(1) : T(0));
    if (tri == 2) v = x <= y ? v : T(0);
    return (x < xlim && y < ylim) ? v : T(0);
  }

  // Element-wise path of the generic instance.
  __device__ __forceinline__ void issue_generic(const DView& v, int x0, int y0) {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int x = x0 + r0 + t * dr, y = y0 + c0 + t * dc;
      raw[t] = (x < xlim && y < ylim) ? vget<T>(v, x, y) : T(0);
    }
  }
};

// Work item and role of a workgroup of the LU step kernel: numbered item
// fastest (role t of every item before role t + 1 of any).
__device__ __forceinline__ void gemm_workgroup(int& item, int& tile) {
  const int flat = blockIdx.y * gridDim.x + blockIdx.x;
  item = flat % gridDim.y;
  tile = flat / gridDim.y;
}

// Work item and output tile of a product workgroup (grid: tiles x items).
// The dispatcher hands consecutive workgroups to the eight XCDs in turn
// (workgroup w runs on XCD w mod 8), and each XCD has its own L2.  In large
// launches the workgroups are renumbered so that every XCD takes one
// contiguous range of the item-major order (item by item, the tiles of an
// item together): the tiles an XCD runs at one time belong to one or two
// items and share their operand panels in that XCD's L2 (n = 16384, k = 8:
// -4% per call).  Small launches keep the item-fastest order (tile t of
// every item before tile t + 1 of any), which spreads them over the XCDs.
// Any numbering is correct.
__device__ __forceinline__ void product_workgroup(int& item, int& tile) {
  const int g = gridDim.x * gridDim.y;
  const int w = blockIdx.y * gridDim.x + blockIdx.x;
  if (g < 2048) {
    item = w % gridDim.y;
    tile = w / gridDim.y;
    return;
  }
  const int q = g >> 3, r = g & 7, x = w & 7, l = w >> 3;
  const int f = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
  item = f / gridDim.x;
  tile = f % gridDim.x;
}
// Output tile (tm, tn) of tile number bid of an item, row by row (column by
// column for a triangular B).  With a triangular operand the K range of a
// tile depends on its position; the heaviest tiles take the lowest numbers
// (dispatched first) so that a launch does not end on a tail of long tiles.
__device__ __forceinline__ void heavy_first(const GemmItem& it, int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  if (it.B.tri != 0 && it.A.tri == 0) {
    tn = bid / tiles_m;
    tm = bid % tiles_m;
  } else {
    tm = bid / tiles_n;
    tn = bid % tiles_n;
  }
  if (it.A.tri == 1) tm = tiles_m - 1 - tm;  // lower A: rows further down use more of K
  if (it.B.tri == 2) tn = tiles_n - 1 - tn;  // upper B: columns further right use more of K
}

// Cin and Sub values of the 16 x (16 FN) output fragments at (r0, c0) in the
// MFMA accumulator layout, for plain (stored, unpermuted) views; positions
// outside the product read its last row / column and are never stored.
template <typename T, int FN>
__device__ __forceinline__ void epilogue_operands(const GemmItem& it, int r0, int c0, int lane, T (&cv)[FN][4],
                                                  T (&sv)[FN][4]) {
  const T* cinp = static_cast<const T*>(it.Cin.p);
  const T* subp = static_cast<const T*>(it.Sub.p);
  if (it.has_cin) {
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = min(r0 + MF<T>::row(lane, v), it.M - 1), c = min(c0 + j * 16 + (lane & 15), it.N - 1);
        cv[j][v] = gload(cinp + static_cast<int64_t>(r) * it.Cin.ld + c);
      }
  }
  if (it.has_sub) {
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = min(r0 + MF<T>::row(lane, v), it.M - 1), c = min(c0 + j * 16 + (lane & 15), it.N - 1);
        sv[j][v] = gload(subp + static_cast<int64_t>(r) * it.Sub.ld + c);
      }
  }
}

// ---------------------------------------------------------------------------
// Batched MFMA GEMM.  One workgroup computes a BM x BN output tile with
// (BM/WM) x (BN/WN) wavefronts of WM x WN each; K is consumed BK at a time
// through double-buffered LDS tiles stored k-major (As[k][m], Bs[k][n]) so
// that every MFMA operand fetch reads 16 consecutive LDS words.
// MODE selects how the work items are formed (GemmMode); every mode is its
// own kernel instance so that profiles separate the Schur products from the
// LU and triangular-inversion updates.
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool GEN, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm(GemmLaunch L) {
  constexpr int NWN = BN / WN;
  constexpr int NT = (BM / WM) * NWN * 64;
  constexpr int FM = WM / 16, FN = WN / 16;
  typedef TileOp<T, BM, BK, NT> OpA;
  typedef TileOp<T, BK, BN, NT> OpB;
  constexpr int AE = OpA::E, BE = OpB::E;
  static_assert(AE * NT == BM * BK && BE * NT == BK * BN, "tile/thread mismatch");
  constexpr bool USE_PERM = (MODE == GEMM_EXPLICIT || MODE == GEMM_RLU_A || MODE == GEMM_RLU_C) && !GEN;

  GemmItem it;
  int item, tile;
  product_workgroup(item, tile);
  // Explicit items: this launch takes items [L.j, L.j + gridDim.y).
  if (!gemm_item<T, MODE>(L, item + (MODE == GEMM_EXPLICIT ? L.j : 0), it)) return;
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (tile >= tiles_m * tiles_n) return;
  int tm, tn;
  heavy_first(it, tile, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;

  int kb = 0, ke = it.K;
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  if (it.B.tri == 1) kb = max(kb, n0);
  if (it.B.tri == 2) ke = min(ke, n0 + BN);
  kb = (kb / BK) * BK;

  __shared__ T As[2][BK][BM + 1];
  __shared__ T Bs[2][BK][BN + 1];
  __shared__ int32_t s_perm[USE_PERM ? kMaxBlock : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  OpA opa;
  OpB opb;
  const int32_t* permA = nullptr;
  const int32_t* permB = nullptr;
  if (USE_PERM) {
    // At most one operand carries a row permutation (the B operand of
    // L^{-1} P B); stage it in LDS once (K entries for B).
    const int32_t* gp = it.B.rowperm ? it.B.rowperm : it.A.rowperm;
    const int np = it.B.rowperm ? it.K : it.M;
    if (gp) {
      for (int e = tid; e < np; e += NT) s_perm[e] = gp[e];
      __syncthreads();
      if (it.B.rowperm)
        permB = s_perm;
      else
        permA = s_perm;
    }
  }
  opa.init(it.A, permA, it.M, it.K, tid);
  opb.init(it.B, permB, it.K, it.N, tid);

  typename MF<T>::acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  auto issue = [&](int k0) {
    if (GEN) {
      opa.issue_generic(it.A, m0, k0);
      opb.issue_generic(it.B, k0, n0);
    } else {
      opa.issue(m0, k0);
      opb.issue(k0, n0);
    }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int t = 0; t < AE; ++t)
      As[buf][opa.c0 + t * opa.dc][opa.r0 + t * opa.dr] = GEN ? opa.raw[t] : opa.finalize(t, m0, k0);
#pragma unroll
    for (int t = 0; t < BE; ++t)
      Bs[buf][opb.r0 + t * opb.dr][opb.c0 + t * opb.dc] = GEN ? opb.raw[t] : opb.finalize(t, k0, n0);
  };

  if (kb < ke) {
    issue(kb);
    store(0, kb);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) issue(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T a[FM], bv[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = As[buf][kk + (lane >> 4)][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j) bv[j] = Bs[buf][kk + (lane >> 4)][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = MF<T>::mma(a[i], bv[j], acc[i][j]);
      }
      if (more) store(buf ^ 1, k0 + BK);
      __syncthreads();
      buf ^= 1;
    }
  }

  T* out = static_cast<T*>(it.out);
  const T alpha = static_cast<T>(it.alpha), beta = static_cast<T>(it.beta);
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    // Cin and Sub of this row of fragments are requested together (addresses
    // clamped into the product, so no load waits on a per-element branch).
    // The fast instance only receives plain Cin / Sub (gemm_item_is_fast).
    T cv[FN][4], sv[FN][4];
    if (!GEN) epilogue_operands<T, FN>(it, m0 + wm * WM + i * 16, n0 + wn * WN, lane, cv, sv);
    if (GEN) {
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = m0 + wm * WM + i * 16 + MF<T>::row(lane, v);
          const int c = n0 + wn * WN + j * 16 + (lane & 15);
          if (r < it.M && c < it.N) {
            T val = alpha * acc[i][j][v];
            if (it.has_cin) val += beta * vget<T>(it.Cin, r, c);
            if (it.has_sub) val -= vget<T>(it.Sub, r, c);
            out[static_cast<int64_t>(r) * it.ldo + c] = val;
          }
        }
    } else {
      // Every value of the row first, then the stores (a load-use wait after
      // a store would also wait for the store).
      T val[FN][4];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          val[j][v] = alpha * acc[i][j][v];
          if (it.has_cin) val[j][v] += beta * cv[j][v];
          if (it.has_sub) val[j][v] -= sv[j][v];
        }
      float um = 0.f;
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = m0 + wm * WM + i * 16 + MF<T>::row(lane, v);
          const int c = n0 + wn * WN + j * 16 + (lane & 15);
          if (r < it.M && c < it.N) {
            gstore(out + static_cast<int64_t>(r) * it.ldo + c, val[j][v]);
            um = nan_fmax(um, static_cast<float>(fabs(val[j][v])));
          }
        }
      if (it.umax) note_umax(it.umax, um);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 product with direct-to-LDS operand loads (items of gemm_item_is_direct:
// stored, untransposed A and B, even N and K, 16-byte aligned rows, plain Cin
// / Sub).  Each thread moves 16-byte pieces of the operand tiles straight
// from memory into LDS (global_load_lds_dwordx4) into three buffers: the
// loads of K step t + 2 are issued before the MFMAs of step t, and no
// register staging sits between the loads and the MFMAs.
//   LDS tiles: A row-major (BM rows of 16), its 16-byte pieces swizzled by
//   piece ^ (row & 7) so that the fragment reads of 8 consecutive rows hit
//   distinct banks; B row-major (16 rows of BN).
//   MFMA K slots: in k-step s of a 16-deep K step, lane group g = lane / 16
//   supplies k = 4 g + s (A and B alike), so every lane reads its four A
//   values as two 16-byte pieces.
// Triangular operands, the last partial K step and the row permutation of B
// are handled in the loads and in a masked variant of the K step that runs
// only where a mask applies (uniform per K step).  Out-of-range rows and
// columns load clamped addresses and feed only outputs that are not stored.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt with vmcnt = N, expcnt and lgkmcnt left at their maxima.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 16, "vmcnt field");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}
// Workgroup barrier that the compiler may not move LDS accesses across (the
// s_waitcnt and s_barrier builtins are no memory barriers to it, and a read
// hoisted above the barrier would see pieces other wavefronts have not
// loaded yet), without the memory fence of __syncthreads.  WAIT is the
// s_waitcnt immediate issued first.
template <int WAIT>
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(WAIT);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int MODE, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm_dl(GemmLaunch L) {
  constexpr int BK = 16;
  constexpr int NWN = BN / WN, NT = (BM / WM) * NWN * 64, FM = WM / 16, FN = WN / 16;
  constexpr int AC = BM * BK / 2, BC = BK * BN / 2;  // 16-byte pieces per K step
  constexpr int AI = AC / NT, BI = BC / NT;           // pieces per thread per K step
  static_assert(AI * NT == AC && BI * NT == BC && AI >= 1 && BI >= 1, "tile/thread mismatch");
  static_assert(AI + BI < 16, "outstanding loads per K step must fit the vmcnt field");
  static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "masking covers the tiles evenly");
  // One array per buffer: the compiler then tells the loads in flight into
  // one buffer from the reads of another and inserts no wait for them.
  __shared__ __attribute__((aligned(16))) double sA0[BM * BK], sA1[BM * BK], sA2[BM * BK];
  __shared__ __attribute__((aligned(16))) double sB0[BK * BN], sB1[BK * BN], sB2[BK * BN];
  __shared__ int16_t s_perm[kMaxBlock];

  GemmItem it;
  int item, tile;
  product_workgroup(item, tile);
  if (!gemm_item<double, MODE>(L, item, it)) return;
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (tile >= tiles_m * tiles_n) return;
  int tm, tn;
  heavy_first(it, tile, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;

  int kb = 0, ke = it.K;
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  if (it.B.tri == 1) kb = max(kb, n0);
  if (it.B.tri == 2) ke = min(ke, n0 + BN);
  kb = (kb / BK) * BK;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int K = it.K;
  // (The recursive LU's items keep A unpermuted and B either permuted or
  // triangular, never both.)
  const bool perm = it.B.rowperm != nullptr;
  if (perm) {
    for (int e = tid; e < K; e += NT) s_perm[e] = static_cast<int16_t>(it.B.rowperm[e]);
    __syncthreads();
  }

  typename MF<double>::acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;

  const int nk = kb < ke ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    const double* Ap = static_cast<const double*>(it.A.p);
    const double* Bp = static_cast<const double*>(it.B.p);
    const int64_t lda = it.A.ld, ldb = it.B.ld;
    // Loads of K step t into (dA, dB); steps past the last repeat the last
    // one (into a buffer no later step reads), so every step issues the same
    // number of loads.  This thread's pieces (recomputed here rather than
    // held in registers): A piece q is tile row r (clamped into the product)
    // at K offset 2 ((P & 7) ^ (r & 7)); B piece q is row P / (BN / 2) of the
    // step, columns from 2 (P % (BN / 2)) (clamped: N is even).
    auto issue = [&](int t, double* dA, double* dB) {
      const int k0 = kb + min(t, nk - 1) * BK;
#pragma unroll
      for (int q = 0; q < AI; ++q) {
        const int P = q * NT + tid, r = P >> 3;
        const int64_t row = static_cast<int64_t>(min(m0 + r, it.M - 1)) * lda;
        const int col = min(k0 + 2 * ((P & 7) ^ (r & 7)), K - 2);
        __builtin_amdgcn_global_load_lds((const void*)(Ap + row + col), (lds_void_t*)(dA + (q * NT + wave * 64) * 2),
                                         16, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < BI; ++q) {
        const int P = q * NT + tid;
        int kr = min(k0 + P / (BN / 2), K - 1);
        if (perm) kr = s_perm[kr];
        const int col = min(n0 + 2 * (P % (BN / 2)), it.N - 2);
        __builtin_amdgcn_global_load_lds((const void*)(Bp + kr * ldb + col), (lds_void_t*)(dB + (q * NT + wave * 64) * 2),
                                         16, 0, 0);
      }
    };

    const int kq = lane >> 4, li = lane & 15;
    // One K step from LDS, in two halves: k slots 2h and 2h + 1 come from one
    // 16-byte piece of A.
    // Lane parts of the fragment addresses (elements): A piece (m, kc) of
    // row m = wm WM + li (+ 16 i) sits at 2 (8 m + (kc ^ (m & 7))), and
    // m & 7 = li & 7; B element (4 kq + s, wn WN + li (+ 16 j)).
    const int a_lane = 16 * (wm * WM + li), a_x = li & 7;
    const int b_lane = 4 * kq * BN + wn * WN + li;
    auto compute = [&](const double* a_s, const double* b_s) {
      // Opaque copies: the buffer addresses are formed here in every step
      // instead of being held, three buffers' worth, across the loop.
      int al = a_lane, bl = b_lane, ax = a_x;
      asm volatile("" : "+v"(al), "+v"(bl), "+v"(ax));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double av[FM][2], bv[FN][2];
        const int apiece = 2 * ((2 * kq + h) ^ ax);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const double2 v = *reinterpret_cast<const double2*>(a_s + al + 256 * i + apiece);
          av[i][0] = v.x;
          av[i][1] = v.y;
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int u = 0; u < 2; ++u) bv[j][u] = b_s[bl + (2 * h + u) * BN + j * 16];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = MF<double>::mma(av[i][u], bv[j][u], acc[i][j]);
      }
    };
    // Whether the tiles of K step k0 need masking (uniform): a part past K,
    // or a triangular operand whose diagonal crosses the tile.
    auto needs_mask = [&](int k0) {
      return k0 + BK > K || (it.A.tri == 1 && m0 <= k0 + BK - 1) || (it.A.tri == 2 && m0 + BM - 1 > k0) ||
             (it.B.tri == 1 && k0 <= n0 + BN - 1) || (it.B.tri == 2 && k0 + BK - 1 > n0);
    };
    // Masks the landed tiles of K step k0 in place: zero past K, and the
    // triangular forms (unit lower: 1 on, 0 above the diagonal; upper: 0
    // below it) in logical coordinates.
    auto mask_tiles = [&](double* a_s, double* b_s, int k0) {
#pragma unroll
      for (int u = 0; u < BM * BK / NT; ++u) {
        const int e = tid + u * NT, r = e >> 4, kl = e & 15, x = m0 + r, k = k0 + kl;
        double* p = a_s + r * 16 + (((kl >> 1) ^ (r & 7)) << 1) + (kl & 1);
        double v = k < K ? *p : 0.0;
        if (it.A.tri == 1) v = x > k ? v : (x == k ? 1.0 : 0.0);
        if (it.A.tri == 2) v = x <= k ? v : 0.0;
        *p = v;
      }
#pragma unroll
      for (int u = 0; u < BK * BN / NT; ++u) {
        const int e = tid + u * NT, kl = e / BN, y = n0 + e % BN, k = k0 + kl;
        double v = k < K ? b_s[e] : 0.0;
        if (it.B.tri == 1) v = k > y ? v : (k == y ? 1.0 : 0.0);
        if (it.B.tri == 2) v = k <= y ? v : 0.0;
        b_s[e] = v;
      }
    };
    // Step t: after the wait, step t has landed for this thread; the barrier
    // makes that true for every thread and ends all reads of step t - 1's
    // buffer, which then receives step t + 2.
    // The loop runs a multiple of three steps; steps past the last only wait
    // and issue (their loads repeat the last step), so that every step of the
    // unrolled body has the same loads in flight.
    auto step = [&](int t, double* ra, double* rb, double* wa, double* wb) {
      // vmcnt(AI + BI): this thread's loads of step t have landed, those of
      // step t + 1 (the AI + BI issued last) may still be in flight.  Vector
      // memory loads return in issue order, so the counter reaching AI + BI
      // means every older load (and its LDS write) is done; step t + 1's
      // pieces go to a buffer that nobody reads before the next barrier.
      // lgkmcnt(0): this wavefront's reads of step t - 1's buffer are
      // complete before the barrier (the compiler places the MFMAs that
      // consume them, and their waits, after it), since once past it other
      // wavefronts load step t + 2 into that buffer.
      lds_barrier<0x0070 | (AI + BI)>();
      issue(t + 2, wa, wb);
      if (t < nk) {
        const int k0 = kb + t * BK;
        if (needs_mask(k0)) {
          mask_tiles(ra, rb, k0);
          lds_barrier<0xC07F>();  // lgkmcnt(0): this thread's LDS writes done
        }
        compute(ra, rb);
      }
    };
    issue(0, sA0, sB0);
    issue(1, sA1, sB1);
    for (int t = 0; t < nk; t += 3) {
      step(t, sA0, sB0, sA2, sB2);
      step(t + 1, sA1, sB1, sA0, sB0);
      step(t + 2, sA2, sB2, sA1, sB1);
    }
    wait_vmcnt<0>();  // no load into LDS may be in flight when the workgroup ends
  }

  double* out = static_cast<double*>(it.out);
  const double alpha = it.alpha, beta = it.beta;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double cv[FN][4], sv[FN][4];
    epilogue_operands<double, FN>(it, m0 + wm * WM + i * 16, n0 + wn * WN, lane, cv, sv);
    double val[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        val[j][v] = alpha * acc[i][j][v];
        if (it.has_cin) val[j][v] += beta * cv[j][v];
        if (it.has_sub) val[j][v] -= sv[j][v];
      }
    float um = 0.f;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * WM + i * 16 + MF<double>::row(lane, v);
        const int c = n0 + wn * WN + j * 16 + (lane & 15);
        if (r < it.M && c < it.N) {
          gstore(out + static_cast<int64_t>(r) * it.ldo + c, val[j][v]);
          um = nan_fmax(um, static_cast<float>(fabs(val[j][v])));
        }
      }
    if (MODE != GEMM_EXPLICIT && it.umax) note_umax(it.umax, um);
  }
}

// ---------------------------------------------------------------------------
// Low-precision products for the mixed-precision paths: FP32 operands are
// split into FP16 or BF16 parts on the way into LDS and multiplied on
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.
//   FP16: x = hi + lo 2^-11, three products hi hi + (hi lo + lo hi) 2^-11
//         (the scaled low part keeps small values out of FP16 subnormals);
//   BF16: x = hi + mid + lo, six products hi hi + hi mid + mid hi + hi lo +
//         lo hi + mid mid.
// A 64 x 64 output tile per workgroup, 4 wavefronts of 32 x 32, K in steps of
// 32 (one MFMA K-step); LDS tiles are k-contiguous per row (A) / per column
// (B) so that every lane fetches its 8 operand values with one 16-byte read.
// ---------------------------------------------------------------------------
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

template <int LP>
struct LPT;
template <>
struct LPT<1> {  // FP16, two parts
  typedef _Float16 E;
  typedef h8_t V;
  static constexpr int PARTS = 2;
  __device__ static void split(float x, E (&p)[2]) {
    const _Float16 hi = static_cast<_Float16>(x);
    p[0] = hi;
    p[1] = static_cast<_Float16>((x - static_cast<float>(hi)) * 2048.0f);
  }
  __device__ static f4_t mma(V a, V b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct LPT<2> {  // BF16, three parts
  typedef __bf16 E;
  typedef bf8_t V;
  static constexpr int PARTS = 3;
  __device__ static void split(float x, E (&p)[3]) {
    const __bf16 hi = static_cast<__bf16>(x);
    const float r1 = x - static_cast<float>(hi);
    const __bf16 mid = static_cast<__bf16>(r1);
    p[0] = hi;
    p[1] = mid;
    p[2] = static_cast<__bf16>(r1 - static_cast<float>(mid));
  }
  __device__ static f4_t mma(V a, V b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <int LP, int MODE, bool GEN, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm_lp(GemmLaunch L) {
  typedef LPT<LP> P;
  typedef typename P::E E;
  typedef typename P::V V;
  constexpr int NP = P::PARTS;
  constexpr int NWN = BN / WN, FM = WM / 16, FN = WN / 16;
  constexpr int BK = 32, NT = (BM / WM) * NWN * 64, KP = BK + 8;
  typedef TileOp<float, BM, BK, NT> OpA;
  typedef TileOp<float, BK, BN, NT> OpB;
  constexpr int AE = OpA::E, BE = OpB::E;

  GemmItem it;
  int item, tile;
  product_workgroup(item, tile);
  if (!gemm_item<float, MODE>(L, item + (GEN ? L.j : 0), it)) return;
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (tile >= tiles_m * tiles_n) return;
  int tm, tn;
  heavy_first(it, tile, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  int kb = 0, ke = it.K;
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  if (it.B.tri == 1) kb = max(kb, n0);
  if (it.B.tri == 2) ke = min(ke, n0 + BN);
  kb = (kb / BK) * BK;

  __shared__ __attribute__((aligned(16))) E As[2][NP][BM][KP];
  __shared__ __attribute__((aligned(16))) E Bs[2][NP][BN][KP];
  __shared__ int32_t s_perm[(MODE == GEMM_EXPLICIT && !GEN) ? kMaxBlock : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  OpA opa;
  OpB opb;
  const int32_t* permA = nullptr;
  const int32_t* permB = nullptr;
  if (MODE == GEMM_EXPLICIT && !GEN) {
    const int32_t* gp = it.B.rowperm ? it.B.rowperm : it.A.rowperm;
    const int np = it.B.rowperm ? it.K : it.M;
    if (gp) {
      for (int e = tid; e < np; e += NT) s_perm[e] = gp[e];
      __syncthreads();
      if (it.B.rowperm)
        permB = s_perm;
      else
        permA = s_perm;
    }
  }
  opa.init(it.A, permA, it.M, it.K, tid);
  opb.init(it.B, permB, it.K, it.N, tid);

  f4_t acc[FM][FN], accx[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[i][j][v] = 0.f;
        accx[i][j][v] = 0.f;
      }

  auto issue = [&](int k0) {
    if (GEN) {
      opa.issue_generic(it.A, m0, k0);
      opb.issue_generic(it.B, k0, n0);
    } else {
      opa.issue(m0, k0);
      opb.issue(k0, n0);
    }
  };
  // FP16 parts hold magnitudes below 65504 only: values outside that range
  // (or not finite) are recorded in L.range_flag, so the caller can redo the
  // products in BF16.
  bool out_of_range = false;
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int t = 0; t < AE; ++t) {
      E pa[NP];
      const float x = GEN ? opa.raw[t] : opa.finalize(t, m0, k0);
      if (LP == 1) out_of_range = out_of_range || !(fabsf(x) < 65504.0f);
      P::split(x, pa);
#pragma unroll
      for (int q = 0; q < NP; ++q) As[buf][q][opa.r0 + t * opa.dr][opa.c0 + t * opa.dc] = pa[q];
    }
#pragma unroll
    for (int t = 0; t < BE; ++t) {
      E pb[NP];
      const float y = GEN ? opb.raw[t] : opb.finalize(t, k0, n0);
      if (LP == 1) out_of_range = out_of_range || !(fabsf(y) < 65504.0f);
      P::split(y, pb);
#pragma unroll
      for (int q = 0; q < NP; ++q) Bs[buf][q][opb.c0 + t * opb.dc][opb.r0 + t * opb.dr] = pb[q];
    }
  };

  if (kb < ke) {
    issue(kb);
    store(0, kb);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) issue(k0 + BK);
      V a[FM][NP], bv[FN][NP];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int q = 0; q < NP; ++q)
          a[i][q] = *reinterpret_cast<const V*>(&As[buf][q][wm * WM + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int q = 0; q < NP; ++q)
          bv[j][q] = *reinterpret_cast<const V*>(&Bs[buf][q][wn * WN + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (LP == 1) {
            acc[i][j] = P::mma(a[i][0], bv[j][0], acc[i][j]);
            accx[i][j] = P::mma(a[i][0], bv[j][1], accx[i][j]);
            accx[i][j] = P::mma(a[i][1], bv[j][0], accx[i][j]);
          } else {
            accx[i][j] = P::mma(a[i][1], bv[j][1], accx[i][j]);
            accx[i][j] = P::mma(a[i][0], bv[j][NP - 1], accx[i][j]);
            accx[i][j] = P::mma(a[i][NP - 1], bv[j][0], accx[i][j]);
            acc[i][j] = P::mma(a[i][0], bv[j][1], acc[i][j]);
            acc[i][j] = P::mma(a[i][1], bv[j][0], acc[i][j]);
            acc[i][j] = P::mma(a[i][0], bv[j][0], acc[i][j]);
          }
        }
      if (more) store(buf ^ 1, k0 + BK);
      __syncthreads();
      buf ^= 1;
    }
  }

  if (LP == 1 && L.range_flag && __any(out_of_range) && lane == 0) atomicOr(L.range_flag, 1);
  float* out = static_cast<float*>(it.out);
  const float alpha = static_cast<float>(it.alpha), beta = static_cast<float>(it.beta);
  const float xs = (LP == 1) ? (1.0f / 2048.0f) : 1.0f;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    float cv[FN][4], sv[FN][4];
    if (!GEN) epilogue_operands<float, FN>(it, m0 + wm * WM + i * 16, n0 + wn * WN, lane, cv, sv);
    float val[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * WM + i * 16 + MF<float>::row(lane, v);
        const int c = n0 + wn * WN + j * 16 + (lane & 15);
        val[j][v] = alpha * (acc[i][j][v] + accx[i][j][v] * xs);
        if (GEN) {
          if (r < it.M && c < it.N) {
            if (it.has_cin) val[j][v] += beta * vget<float>(it.Cin, r, c);
            if (it.has_sub) val[j][v] -= vget<float>(it.Sub, r, c);
          }
        } else {
          if (it.has_cin) val[j][v] += beta * cv[j][v];
          if (it.has_sub) val[j][v] -= sv[j][v];
        }
      }
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * WM + i * 16 + MF<float>::row(lane, v);
        const int c = n0 + wn * WN + j * 16 + (lane & 15);
        if (r < it.M && c < it.N) gstore(out + static_cast<int64_t>(r) * it.ldo + c, val[j][v]);
      }
  }
}

// ---------------------------------------------------------------------------
// Split low-precision products with vectorised operand staging (used for
// FP16, LP = 1), for the explicit items of gemm_item_is_lp_vec (A and B stored untransposed,
// 16-byte aligned rows of A, a triangular form on A, a row permutation on B,
// K a multiple of 8) and the products of the recursive LU of float matrices
// (which also have triangular B operands).  Every thread stages runs of eight consecutive k: a run of
// a row of A (two 16-byte loads) or of a column of B (eight loads, each
// coalesced across the wavefront), splits them into parts and writes each
// part as one 16-byte LDS store in the layout the MFMA reads (k contiguous
// per row of A and per column of B).  Wavefronts own 64 x 64 output tiles
// (16 MFMA blocks), which halves the LDS bytes read per product compared
// with 32 x 32.  Parts and products as in k_gemm_lp.
// ---------------------------------------------------------------------------
template <int LP, int MODE, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm_lpv(GemmLaunch L) {
  typedef LPT<LP> P;
  typedef typename P::E E;
  typedef typename P::V V;
  constexpr int NP = P::PARTS;
  constexpr int NWN = BN / WN, FM = WM / 16, FN = WN / 16;
  constexpr int NT = (BM / WM) * NWN * 64, BK = 32, KP = BK + 8;
  constexpr int ACH = BM * (BK / 8) / NT, BCH = BN * (BK / 8) / NT;  // runs of 8 per thread
  static_assert(ACH * NT == BM * (BK / 8) && BCH * NT == BN * (BK / 8) && ACH >= 1 && BCH >= 1, "runs");
  __shared__ __attribute__((aligned(16))) E As[2][NP][BM][KP];
  __shared__ __attribute__((aligned(16))) E Bs[2][NP][BN][KP];
  __shared__ int16_t s_perm[kMaxBlock];

  GemmItem it;
  int item, tile;
  product_workgroup(item, tile);
  if (!gemm_item<float, MODE>(L, item, it)) return;
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (tile >= tiles_m * tiles_n) return;
  int tm, tn;
  heavy_first(it, tile, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = it.M, N = it.N, K = it.K;
  int kb = 0, ke = K;
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  if (it.B.tri == 1) kb = max(kb, n0);
  if (it.B.tri == 2) ke = min(ke, n0 + BN);
  kb = (kb / BK) * BK;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const bool perm = it.B.rowperm != nullptr;
  if (perm) {
    for (int e = tid; e < K; e += NT) s_perm[e] = static_cast<int16_t>(it.B.rowperm[e]);
    __syncthreads();
  }
  const float* Ap = static_cast<const float*>(it.A.p);
  const float* Bp = static_cast<const float*>(it.B.p);
  const int64_t lda = it.A.ld, ldb = it.B.ld;
  const int atri = it.A.tri, btri = it.B.tri;

  f4_t acc[FM][FN], accx[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[i][j][v] = 0.f;
        accx[i][j][v] = 0.f;
      }

  // This thread's runs: A run q covers row ar(q) at k offsets ak(q) .. +7,
  // B run q column bn(q) at k offsets bk(q) .. +7.
  float ra[ACH][8], rb[BCH][8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < ACH; ++q) {
      const int c = tid + q * NT, ar = c >> 2, ak = (c & 3) * 8;
      const int64_t row = min(m0 + ar, M - 1);
      const int k = min(k0 + ak, K - 8);
      const float4 lo = *reinterpret_cast<const float4*>(Ap + row * lda + k);
      const float4 hi = *reinterpret_cast<const float4*>(Ap + row * lda + k + 4);
      ra[q][0] = lo.x; ra[q][1] = lo.y; ra[q][2] = lo.z; ra[q][3] = lo.w;
      ra[q][4] = hi.x; ra[q][5] = hi.y; ra[q][6] = hi.z; ra[q][7] = hi.w;
    }
#pragma unroll
    for (int q = 0; q < BCH; ++q) {
      const int c = tid + q * NT, bn = c % BN, bk = (c / BN) * 8;
      const int col = min(n0 + bn, N - 1);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = min(k0 + bk + u, K - 1);
        const int r = perm ? s_perm[kk] : kk;
        rb[q][u] = gload(Bp + static_cast<int64_t>(r) * ldb + col);
      }
    }
  };
  bool out_of_range = false;
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int q = 0; q < ACH; ++q) {
      const int c = tid + q * NT, ar = c >> 2, ak = (c & 3) * 8;
      const int x = m0 + ar;
      V part[NP];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int y = k0 + ak + u;
        float v = y < K ? ra[q][u] : 0.f;
        if (atri == 1) v = x > y ? v : (x == y ? 1.f : 0.f);
        if (atri == 2) v = x <= y ? v : 0.f;
        if (LP == 1) out_of_range = out_of_range || !(fabsf(v) < 65504.0f);
        E pv[NP];
        P::split(v, pv);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) part[pp][u] = pv[pp];
      }
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) *reinterpret_cast<V*>(&As[buf][pp][ar][ak]) = part[pp];
    }
#pragma unroll
    for (int q = 0; q < BCH; ++q) {
      const int c = tid + q * NT, bn = c % BN, bk = (c / BN) * 8;
      const int y = n0 + bn;
      V part[NP];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int x = k0 + bk + u;
        float v = x < K ? rb[q][u] : 0.f;
        if (btri == 1) v = x > y ? v : (x == y ? 1.f : 0.f);
        if (btri == 2) v = x <= y ? v : 0.f;
        if (LP == 1) out_of_range = out_of_range || !(fabsf(v) < 65504.0f);
        E pv[NP];
        P::split(v, pv);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) part[pp][u] = pv[pp];
      }
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) *reinterpret_cast<V*>(&Bs[buf][pp][bn][bk]) = part[pp];
    }
  };

  if (kb < ke) {
    load(kb);
    store(0, kb);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) load(k0 + BK);
      V bv[FN][NP];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int pp = 0; pp < NP; ++pp)
          bv[j][pp] = *reinterpret_cast<const V*>(&Bs[buf][pp][wn * WN + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        V a[NP];
#pragma unroll
        for (int pp = 0; pp < NP; ++pp)
          a[pp] = *reinterpret_cast<const V*>(&As[buf][pp][wm * WM + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (LP == 1) {
            acc[i][j] = P::mma(a[0], bv[j][0], acc[i][j]);
            accx[i][j] = P::mma(a[0], bv[j][1], accx[i][j]);
            accx[i][j] = P::mma(a[1], bv[j][0], accx[i][j]);
          } else {
            accx[i][j] = P::mma(a[1], bv[j][1], accx[i][j]);
            accx[i][j] = P::mma(a[0], bv[j][NP - 1], accx[i][j]);
            accx[i][j] = P::mma(a[NP - 1], bv[j][0], accx[i][j]);
            acc[i][j] = P::mma(a[0], bv[j][1], acc[i][j]);
            acc[i][j] = P::mma(a[1], bv[j][0], acc[i][j]);
            acc[i][j] = P::mma(a[0], bv[j][0], acc[i][j]);
          }
        }
      }
      if (more) store(buf ^ 1, k0 + BK);
      __syncthreads();
      buf ^= 1;
    }
  }

  if (LP == 1 && L.range_flag && __any(out_of_range) && lane == 0) atomicOr(L.range_flag, 1);
  float* out = static_cast<float*>(it.out);
  const float alpha = static_cast<float>(it.alpha), beta = static_cast<float>(it.beta);
  const float xs = (LP == 1) ? (1.0f / 2048.0f) : 1.0f;
  float um = 0.f;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    float cv[FN][4], sv[FN][4];
    epilogue_operands<float, FN>(it, m0 + wm * WM + i * 16, n0 + wn * WN, lane, cv, sv);
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * WM + i * 16 + MF<float>::row(lane, v);
        const int c = n0 + wn * WN + j * 16 + (lane & 15);
        float val = alpha * (acc[i][j][v] + accx[i][j][v] * xs);
        if (it.has_cin) val += beta * cv[j][v];
        if (it.has_sub) val -= sv[j][v];
        if (r < M && c < N) {
          gstore(out + static_cast<int64_t>(r) * it.ldo + c, val);
          um = nan_fmax(um, fabsf(val));
        }
      }
  }
  if (MODE != GEMM_EXPLICIT && it.umax) note_umax(it.umax, um);
}

// ---------------------------------------------------------------------------
// Split products from operands split once (mixed FP16 / BF16 paths, large
// launches of explicit items).  k_split_ops converts every item's operands:
// A (M x K) into low-precision planes (FP16 high and low, x = hi + lo 2^-11;
// BF16 high, middle and low; as in LPT) with K contiguous per row, B (K x N)
// into the planes of its transpose (K contiguous per column), the triangular
// form of A applied and K zero-padded to the pitch kp; FP16 also checks the
// range.  k_gemm_split then moves those planes into LDS with direct loads and
// runs the products of the parts per K step (3 for FP16, 6 for BF16) with no
// conversion in its loop.  In k_gemm_lpv and k_gemm_lp every output tile
// converts its own operand panels, so an element of A is converted once per
// tile column and one of B once per tile row.
// ---------------------------------------------------------------------------
// Row tile of the k_gemm_split launches per split kind: for a triangular A,
// the split pass skips the 64 x 64 tiles outside the K range of their row tile.
template <int LP>
struct SplitShape;
template <>
struct SplitShape<1> {
  static constexpr int BM = 256, BN = 128;
};
template <>
struct SplitShape<2> {
  static constexpr int BM = 128, BN = 128;
};

template <int LP>
__global__ __launch_bounds__(256) void k_split_ops(GemmLaunch L) {
  typedef LPT<LP> P;
  typedef typename P::E E;
  typedef typename P::V V;
  constexpr int NP = P::PARTS, TM = SplitShape<LP>::BM;
  __shared__ float tb[64][65];
  const GemmItem it = static_cast<const GemmItem*>(L.items)[blockIdx.y];
  const int kp = L.split_kp, kt = kp / 64;
  E* ap = reinterpret_cast<E*>(static_cast<char*>(L.split) +
                               blockIdx.y * split_item_bytes(L.split_m, L.split_n, kp, NP));
  E* bp = ap + static_cast<int64_t>(NP) * L.split_m * kp;
  const int64_t aplane = static_cast<int64_t>(L.split_m) * kp, bplane = static_cast<int64_t>(L.split_n) * kp;
  const int tid = threadIdx.x;
  const int ta = (L.split_m + 63) / 64 * kt;
  bool bad = false;
  int t = blockIdx.x;
  if (t < ta) {
    // A: rows r0 .. r0 + 63, k0 .. k0 + 63; a thread converts runs of 8 k.
    const int r0 = (t / kt) * 64, k0 = (t % kt) * 64;
    if (r0 >= it.M) return;
    const int tm0 = r0 / TM * TM;
    if ((it.A.tri == 1 && k0 >= tm0 + TM) || (it.A.tri == 2 && k0 + 64 <= tm0)) return;
    const float* Ap = static_cast<const float*>(it.A.p);
    const int64_t lda = it.A.ld;
    const int atri = it.A.tri;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int run = tid + q * 256, x = r0 + (run >> 3), y0 = k0 + 8 * (run & 7);
      if (x >= it.M) continue;
      float v[8];
      if (y0 < it.K) {  // K is a multiple of 8: the run is stored entirely
        const float4 p0 = *reinterpret_cast<const float4*>(Ap + x * lda + y0);
        const float4 p1 = *reinterpret_cast<const float4*>(Ap + x * lda + y0 + 4);
        v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
        v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = 0.f;
      }
      V part[NP];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int y = y0 + u;
        float a = y < it.K ? v[u] : 0.f;
        if (atri == 1) a = x > y ? a : (x == y && y < it.K ? 1.f : 0.f);
        if (atri == 2) a = x <= y ? a : 0.f;
        if (LP == 1) bad = bad || !(fabsf(a) < 65504.0f);
        E pv[NP];
        P::split(a, pv);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) part[pp][u] = pv[pp];
      }
#pragma unroll
      for (int pp = 0; pp < NP; ++pp)
        *reinterpret_cast<V*>(ap + pp * aplane + static_cast<int64_t>(x) * kp + y0) = part[pp];
    }
  } else {
    // B: columns n0 .. n0 + 63, k0 .. k0 + 63, transposed through LDS.
    t -= ta;
    const int n0 = (t / kt) * 64, k0 = (t % kt) * 64;
    if (n0 >= it.N) return;
    const float* Bp = static_cast<const float*>(it.B.p);
    const int64_t ldb = it.B.ld;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int kr = (tid >> 6) + 4 * u, y = n0 + (tid & 63), k = k0 + kr;
      float v = 0.f;
      if (k < it.K && y < it.N) {
        const int row = it.B.rowperm ? it.B.rowperm[k] : k;
        v = Bp[static_cast<int64_t>(row) * ldb + y];
      }
      tb[kr][tid & 63] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int run = tid + q * 256, nr = run >> 3, c = run & 7, y = n0 + nr;
      if (y >= it.N) continue;
      V part[NP];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float b = tb[8 * c + u][nr];
        if (LP == 1) bad = bad || !(fabsf(b) < 65504.0f);
        E pv[NP];
        P::split(b, pv);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) part[pp][u] = pv[pp];
      }
#pragma unroll
      for (int pp = 0; pp < NP; ++pp)
        *reinterpret_cast<V*>(bp + pp * bplane + static_cast<int64_t>(y) * kp + k0 + 8 * c) = part[pp];
    }
  }
  if (LP == 1 && L.range_flag && __any(bad) && (tid & 63) == 0) atomicOr(L.range_flag, 1);
}

// Products of the split planes: BM x BN tiles of 64 x 64 wavefronts, K in
// steps of 32 (one MFMA K step) through three LDS buffers, loaded directly
// (16-byte pieces, eight k of one row of one plane) with the pipeline of
// k_gemm_dl.  LDS piece (plane, row r, slot s) holds k chunk s ^ ((r >> 2) & 3)
// of that row, so that the 16 rows a quarter-wavefront reads at one chunk
// fall in distinct banks.  Products and epilogue as in k_gemm_lpv.
template <int LP, int BM, int BN>
__global__ __launch_bounds__((BM / 64) * (BN / 64) * 64) void k_gemm_split(GemmLaunch L) {
  typedef LPT<LP> P;
  typedef typename P::E E;
  typedef typename P::V V;
  constexpr int NP = P::PARTS;
  constexpr int WM = 64, WN = 64, NWN = BN / WN, FM = WM / 16, FN = WN / 16;
  constexpr int NT = (BM / WM) * NWN * 64, BK = 32;
  constexpr int AC = NP * BM * 4, BC = NP * BN * 4;  // 16-byte pieces per K step (4 per row and plane)
  constexpr int AI = AC / NT, BI = BC / NT;
  static_assert(AI * NT == AC && BI * NT == BC && AI >= 1 && BI >= 1, "tile/thread mismatch");
  static_assert(AI + BI < 16, "outstanding loads per K step must fit the vmcnt field");
  __shared__ __attribute__((aligned(16))) E sA0[NP * BM * BK], sA1[NP * BM * BK], sA2[NP * BM * BK];
  __shared__ __attribute__((aligned(16))) E sB0[NP * BN * BK], sB1[NP * BN * BK], sB2[NP * BN * BK];

  GemmItem it;
  int item, tile;
  product_workgroup(item, tile);
  it = static_cast<const GemmItem*>(L.items)[item];
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (tile >= tiles_m * tiles_n) return;
  int tm, tn;
  heavy_first(it, tile, tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int kp = L.split_kp;
  int kb = 0, ke = min(it.K, kp);
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  kb = (kb / BK) * BK;

  const E* ah = reinterpret_cast<const E*>(static_cast<const char*>(L.split) +
                                           item * split_item_bytes(L.split_m, L.split_n, kp, NP));
  const E* bh = ah + static_cast<int64_t>(NP) * L.split_m * kp;
  const int64_t aplane = static_cast<int64_t>(L.split_m) * kp, bplane = static_cast<int64_t>(L.split_n) * kp;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  f4_t acc[FM][FN], accx[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[i][j][v] = 0.f;
        accx[i][j][v] = 0.f;
      }

  const int nk = kb < ke ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    // Loads of K step t into (dA, dB); steps past the last repeat the last
    // one (into a buffer no later step reads).  Piece P of a step: plane
    // P / (4 rows), row (P % (4 rows)) / 4, slot P % 4 (rows clamped into
    // the product).
    auto issue = [&](int t, E* dA, E* dB) {
      const int k0 = kb + min(t, nk - 1) * BK;
#pragma unroll
      for (int q = 0; q < AI; ++q) {
        const int P = q * NT + tid, pl = P / (BM * 4), rem = P % (BM * 4), r = rem >> 2;
        const int c = (rem & 3) ^ ((r >> 2) & 3);
        const E* src = ah + pl * aplane + static_cast<int64_t>(min(m0 + r, it.M - 1)) * kp + k0 + 8 * c;
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)(dA + (q * NT + wave * 64) * 8), 16, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < BI; ++q) {
        const int P = q * NT + tid, pl = P / (BN * 4), rem = P % (BN * 4), r = rem >> 2;
        const int c = (rem & 3) ^ ((r >> 2) & 3);
        const E* src = bh + pl * bplane + static_cast<int64_t>(min(n0 + r, it.N - 1)) * kp + k0 + 8 * c;
        __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)(dB + (q * NT + wave * 64) * 8), 16, 0, 0);
      }
    };
    // Fragment reads: lane l takes row (l & 15) of a 16-row block and k
    // chunk l >> 4 (8 elements), for A and for B transposed alike.
    const int li = lane & 15, kc = lane >> 4;
    auto compute = [&](const E* a_s, const E* b_s) {
      V bv[FN][NP], av[FM][NP];
      int boff[FN], aoff[FM];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int r = wn * WN + j * 16 + li;
        boff[j] = r * BK + 8 * (kc ^ ((r >> 2) & 3));
      }
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int r = wm * WM + i * 16 + li;
        aoff[i] = r * BK + 8 * (kc ^ ((r >> 2) & 3));
      }
      // High planes first (the first pass needs only them), then the
      // others, whose reads overlap the first passes.
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) {
#pragma unroll
        for (int j = 0; j < FN; ++j) bv[j][pp] = *reinterpret_cast<const V*>(b_s + pp * BN * BK + boff[j]);
#pragma unroll
        for (int i = 0; i < FM; ++i) av[i][pp] = *reinterpret_cast<const V*>(a_s + pp * BM * BK + aoff[i]);
      }
      // One pass per product over the 16 fragment pairs: consecutive MFMAs
      // never feed one accumulator.  FP16: hi hi into acc, the cross
      // products into accx (scaled by 2^-11 at the end); BF16: hi hi and the
      // hi-mid products into acc, the smaller ones into accx.
      auto pass = [&](f4_t (&c)[FM][FN], int pa, int pb) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) c[i][j] = P::mma(av[i][pa], bv[j][pb], c[i][j]);
      };
      pass(acc, 0, 0);
      if (LP == 1) {
        pass(accx, 0, 1);
        pass(accx, 1, 0);
      } else {
        pass(acc, 0, 1);
        pass(acc, 1, 0);
        pass(accx, 1, 1);
        pass(accx, 0, 2);
        pass(accx, 2, 0);
      }
      // Instruction order (scheduling groups: 0x100 LDS reads, 0x008
      // MFMA): the high-plane reads, then each further read after two
      // MFMAs, then the remaining MFMAs.
      constexpr int R0 = FM + FN, RX = (NP - 1) * (FM + FN), NMF = FM * FN * (LP == 1 ? 3 : 6);
      __builtin_amdgcn_sched_group_barrier(0x100, R0, 0);
#pragma unroll
      for (int q = 0; q < RX; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NMF - 2 * RX, 0);
    };
    // Step t (see k_gemm_dl): after the wait this thread's pieces of step t
    // have landed, the barrier makes that true for all and ends every read
    // of the buffer that then receives step t + 2.
    auto step = [&](int t, E* ra, E* rb, E* wa, E* wb) {
      lds_barrier<0x0070 | (AI + BI)>();
      issue(t + 2, wa, wb);
      if (t < nk) compute(ra, rb);
    };
    issue(0, sA0, sB0);
    issue(1, sA1, sB1);
    for (int t = 0; t < nk; t += 3) {
      step(t, sA0, sB0, sA2, sB2);
      step(t + 1, sA1, sB1, sA0, sB0);
      step(t + 2, sA2, sB2, sA1, sB1);
    }
    wait_vmcnt<0>();  // no load into LDS may be in flight when the workgroup ends
  }

  float* out = static_cast<float*>(it.out);
  const float alpha = static_cast<float>(it.alpha), beta = static_cast<float>(it.beta);
  const float xs = LP == 1 ? 1.0f / 2048.0f : 1.0f;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    float cv[FN][4], sv[FN][4];
    epilogue_operands<float, FN>(it, m0 + wm * WM + i * 16, n0 + wn * WN, lane, cv, sv);
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm * WM + i * 16 + MF<float>::row(lane, v);
        const int c = n0 + wn * WN + j * 16 + (lane & 15);
        float val = alpha * (acc[i][j][v] + accx[i][j][v] * xs);
        if (it.has_cin) val += beta * cv[j][v];
        if (it.has_sub) val -= sv[j][v];
        if (r < it.M && c < it.N) gstore(out + static_cast<int64_t>(r) * it.ldo + c, val);
      }
  }
}

// ---------------------------------------------------------------------------
// Wave-wide argmax with DPP: the largest value, lowest index on ties (the
// rule of LAPACK's idamax).  Every lane returns the wave's winner.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_argmax_step(double& v, int& i) {
  const int64_t bits = __double_as_longlong(v);
  const int lo = static_cast<int>(bits & 0xffffffff), hi = static_cast<int>(bits >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
  const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROW_MASK, 0xf, false);
  const double ov = __longlong_as_double((static_cast<int64_t>(ohi) << 32) | static_cast<uint32_t>(olo));
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_argmax_step(float& v, int& i) {
  const int ob = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
  const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROW_MASK, 0xf, false);
  const float ov = __int_as_float(ob);
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
  dpp_argmax_step<0xB1, 0xf>(v, i);   // quad_perm [1,0,3,2]
  dpp_argmax_step<0x4E, 0xf>(v, i);   // quad_perm [2,3,0,1]
  dpp_argmax_step<0x141, 0xf>(v, i);  // row_half_mirror
  dpp_argmax_step<0x140, 0xf>(v, i);  // row_mirror
  dpp_argmax_step<0x142, 0xa>(v, i);  // row_bcast:15 into rows 1 and 3
  dpp_argmax_step<0x143, 0xc>(v, i);  // row_bcast:31 into rows 2 and 3
  // lane 63 now holds the wave's winner
  if constexpr (sizeof(T) == 8) {
    const int64_t bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), 63);
    v = __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
  } else {
    v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  }
  i = __builtin_amdgcn_readlane(i, 63);
}

// ---------------------------------------------------------------------------
// Panel LU with partial pivoting.  Rows j..b-1, columns j..j+w-1 of one
// matrix live in registers: thread t owns panel rows t + NT q (q < R).  For
// every column: each wave finds its best row (largest magnitude, lowest
// index on ties) with DPP, its owner publishes the row in LDS, and the owner
// of the current row C publishes that row too; after one barrier every
// thread picks the global winner p, the rows C and p are exchanged, and the
// multipliers and the rank-1 update of the panel follow.  LDS buffers
// alternate between even and odd columns, so one barrier per column
// suffices.  The composite row movement is recorded as (dest, src) pairs for
// k_laswp_trsm, and the running permutation of the matrix is composed in
// it.perm.  Columns are unrolled at compile time (panel_step<C>).
// ---------------------------------------------------------------------------
template <typename T, int NB, int NW>
struct PanelShared {
  T cand[2][NW][NB];  // each wave's candidate row
  T candv[2][NW];
  int candi[2][NW];
  int cando[2][NW];   // original position of the candidate row
  T rowc[2][NB];      // the current row C
  int origc[2];
  int cnt;
};

// One column step for column C (a runtime value).  Register rows are only
// indexed statically: the pivot column is extracted and written back with
// predicated selects, which keeps one compact copy of the step in the
// instruction cache instead of NB unrolled copies.
template <typename T, int NB, int R, int NT>
__device__ __forceinline__ void panel_step(T (&a)[R][NB], int (&orig)[R], PanelShared<T, NB, NT / 64>& sh, int C,
                                           int h, int tid, int32_t* info, int node) {
  constexpr int NW = NT / 64;
  const int P = C & 1;
  const int lane = tid & 63, wave = tid >> 6;
  // Columns are grouped in quarters of NB/4; only the quarter holding C is
  // searched for the pivot column and quarters left of C are not updated.
  constexpr int QW = NB >= 8 ? NB / 4 : NB;
  constexpr int NQ = NB / QW;
  T colv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) colv[q] = T(0);
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    if (C / QW != qq) continue;
#pragma unroll
    for (int q = 0; q < R; ++q) {
#pragma unroll
      for (int t = 0; t < QW; ++t) colv[q] = (qq * QW + t == C) ? a[q][qq * QW + t] : colv[q];
    }
  }
  T best = T(-1);
  int bi = INT_MAX;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr >= C && lr < h) {
      const T v = fabs(colv[q]);
      if (v > best) {
        best = v;
        bi = lr;
      }
    }
  }
  wave_argmax(best, bi);
  // Publish the wave's candidate row and the current row C.
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr == bi) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) sh.cand[P][wave][cc] = a[q][cc];
      sh.cando[P][wave] = orig[q];
    }
  }
  if (lane == 0) {
    sh.candv[P][wave] = best;
    sh.candi[P][wave] = bi;
  }
  if (tid == C) {  // row C is owned by thread C (C < NB <= NT), slot q = 0
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) sh.rowc[P][cc] = a[0][cc];
    sh.origc[P] = orig[0];
  }
  __syncthreads();
  int ww = 0;
  best = sh.candv[P][0];
  bi = sh.candi[P][0];
#pragma unroll
  for (int wv = 1; wv < NW; ++wv) {
    const T ov = sh.candv[P][wv];
    const int oi = sh.candi[P][wv];
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
      ww = wv;
    }
  }
  const bool none = bi == INT_MAX;  // an all-NaN column keeps its row
  const int p = none ? C : bi;
  const T* prow = none ? sh.rowc[P] : sh.cand[P][ww];
  const T piv = prow[C];
  if (!(piv != T(0) && isfinite(piv)) && tid == 0 && info) atomicCAS(info, 0, node + 1);
  const T rinv = piv != T(0) ? T(1) / piv : T(0);
  T l[R];
  // Row C takes the pivot row (thread C, slot 0); row p takes row C.
  if (p != C) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * NT;
      if (lr == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) a[q][cc] = sh.rowc[P][cc];
        orig[q] = sh.origc[P];
        colv[q] = sh.rowc[P][C];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    const bool below = lr > C && lr < h;
    l[q] = below ? colv[q] * rinv : T(0);
  }
  if (tid == C) orig[0] = none ? sh.origc[P] : sh.cando[P][ww];
  // Rank-1 update by quarters; the pivot row is read from LDS once per
  // quarter (one batch of reads) and quarters left of C are skipped.
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    if (C >= (qq + 1) * QW) continue;
    T pr[QW];
#pragma unroll
    for (int t = 0; t < QW; ++t) pr[t] = prow[qq * QW + t];
#pragma unroll
    for (int t = 0; t < QW; ++t) {
      const int cc = qq * QW + t;
      if (tid == C) a[0][cc] = pr[t];
      const T pv = cc > C ? pr[t] : T(0);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        a[q][cc] -= l[q] * pv;
        if (cc == C && l[q] != T(0)) a[q][cc] = l[q];
      }
    }
  }
  if (tid == C) {
    // columns of the pivot row in finished quarters (its multipliers)
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
      if (C < (qq + 1) * QW) continue;
#pragma unroll
      for (int t = 0; t < QW; ++t) a[0][qq * QW + t] = prow[qq * QW + t];
    }
  }
}

template <typename T, int NB, int R>
__global__ __launch_bounds__(512) void k_getf2(const LuItem* items, int j) {
  constexpr int NT = 512;
  const LuItem it = items[blockIdx.x];
  T* A = static_cast<T*>(it.a);
  const int b = it.b, h = b - j, w = min(NB, h);
  const int tid = threadIdx.x;
  __shared__ PanelShared<T, NB, NT / 64> sh;

  T a[R][NB];
  int orig[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    orig[q] = lr;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      a[q][c] = (lr < h && c < w) ? A[static_cast<int64_t>(j + lr) * b + j + c] : T(0);
  }
  if (tid == 0) sh.cnt = 0;
  for (int C = 0; C < w; ++C) panel_step<T, NB, R, NT>(a, orig, sh, C, h, tid, it.info, it.node);
  __syncthreads();

  // Write the factored panel back and record the moved rows.
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr < h) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < w) A[static_cast<int64_t>(j + lr) * b + j + c] = a[q][c];
      if (orig[q] != lr) {
        const int slot = atomicAdd(&sh.cnt, 1);
        it.swaps[1 + 2 * slot] = j + lr;
        it.swaps[2 + 2 * slot] = j + orig[q];
      }
    }
  }
  int pv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    pv[q] = (lr < h) ? (j == 0 ? orig[q] : it.perm[j + orig[q]]) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr < h) it.perm[j + lr] = pv[q];
  }
  if (tid == 0) it.swaps[0] = sh.cnt;
}

// ---------------------------------------------------------------------------
// Tile-local pivoting LU, step t0: factor the kTile x kTile diagonal tile in
// one wavefront.  Lane l holds row l % 32 and columns 16 (l / 32) ..
// 16 (l / 32) + 15 of the tile.  For every column the pivot is the row of
// largest magnitude among the tile rows not chosen before (lowest index on
// near-ties).  Pivoting is implicit: rows stay in their lanes and the
// factored rows are stored in pivot order at the end, so rows move only
// inside the tile's row band.  The tile's row movement goes to
// it.swaps[1 + q] (tile position q holds original tile row swaps[1 + q]), the
// matrix permutation is composed in it.perm, and the inverses of the tile's
// unit-lower L and upper U go to it.aux (L^{-1} first, then U^{-1},
// kTile x kTile each, row-major).
// ---------------------------------------------------------------------------

// Uniform-lane read (lane is wave-uniform).
template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane) {
  if constexpr (sizeof(T) == 8) {
    const int64_t bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), lane);
    return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  }
}

// Orders this wavefront's LDS accesses for the compiler only: a wavefront's
// LDS operations execute in issue order, so rows one lane writes are seen by
// the later reads of every lane of the same (single-wavefront) workgroup.
__device__ __forceinline__ void wave_lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// 1 / d by the hardware reciprocal and two Newton steps (the pivot
// reciprocal of the tile LU; exact to about one unit in the last place).
__device__ __forceinline__ double tile_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float tile_rcp(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  const float e = fmaf(-d, r, 1.0f);
  return fmaf(r, e, r);
}

// Pivot search key of a row for a column, 32 bits: the leading bits of |y|
// (sign cleared, so the unsigned order is the order of magnitudes and a NaN
// orders above +inf) with the low five bits replaced by 31 - r; one unsigned
// maximum then picks the largest magnitude and, among magnitudes equal in
// their leading 27 bits (15 mantissa bits for double, 18 for float), the
// lowest row.  0 when the row is not a candidate.
__device__ __forceinline__ uint32_t pivot_key(double y, bool cand, int r) {
  const uint32_t hi = static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(fabs(y))) >> 32);
  return cand ? ((hi & ~31u) | static_cast<uint32_t>(31 - r)) : 0u;
}
__device__ __forceinline__ uint32_t pivot_key(float y, bool cand, int r) {
  const uint32_t bits = static_cast<uint32_t>(__float_as_int(fabsf(y)));
  return cand ? ((bits & ~31u) | static_cast<uint32_t>(31 - r)) : 0u;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_umax(uint32_t k) {
  // Every source lane is valid for the full-mask patterns, so the plain DPP
  // move (undefined old value) is used there and can fold into the maximum.
  const uint32_t o = ROW_MASK == 0xf
                         ? static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(k), CTRL, 0xf, 0xf, false))
                         : static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(k), static_cast<int>(k),
                                                                             CTRL, ROW_MASK, 0xf, false));
  return o > k ? o : k;
}
// Row of the largest key among the 32 lanes of half h (a wave-uniform value).
__device__ __forceinline__ int half_argmax(uint32_t k, int h) {
  k = dpp_umax<0xB1, 0xf>(k);   // quad_perm [1,0,3,2]
  k = dpp_umax<0x4E, 0xf>(k);   // quad_perm [2,3,0,1]
  k = dpp_umax<0x141, 0xf>(k);  // row_half_mirror
  k = dpp_umax<0x140, 0xf>(k);  // row_mirror
  k = dpp_umax<0x142, 0xa>(k);  // row_bcast:15: lanes 31 and 63 hold their half's maximum
  const int top = __builtin_amdgcn_readlane(static_cast<int>(k), h ? 63 : 31);
  return 31 - (top & 31);
}

// Buffers of tile s of the tile-pivoting LU: inverses of its L and U
// factors (kTile x kTile each, row-major, L^{-1} first) and its permutation
// (position q of the factored tile holds original tile row perm[q]).
template <typename T>
__device__ __forceinline__ T* step_inv(const LuItem& it, int s) {
  return static_cast<T*>(it.aux) + static_cast<int64_t>(s % kStepBufs) * 2 * kTile * kTile;
}
__device__ __forceinline__ int32_t* step_perm(const LuItem& it, int s) { return it.swaps + 1 + (s % kStepBufs) * kTile; }

// LDS of one tile factorisation: four kTile x (kTile + 2) arrays and kTile
// reciprocals.
constexpr int kLuLd = kTile + 2;
constexpr int kLuLdsElems = 4 * kTile * kLuLd + kTile;

// One wavefront (threads 0..63 of its workgroup; the function synchronises
// only within the wavefront) factors diagonal tile t0 / kTile.  The tile is
// read from the matrix, or from LDS (sT, leading dimension ldt) when the
// caller has just formed it there; lds is kLuLdsElems elements of scratch.
template <typename T, typename TC = T>
__device__ __forceinline__ void tile_lu_wave(const LuItem& item, int t0, const T* sT, int ldt, TC* lds) {
  constexpr int LD = kLuLd;
  const LuItem it = item;  // every field read up front, ahead of the stores
  if (t0 >= it.b) return;  // a smaller matrix of a merged batch
  T* A = static_cast<T*>(it.a);
  const int b = it.b, ts = min(kTile, b - t0), s = t0 / kTile;
  const int l = threadIdx.x & 63, r = l & 31, half = l >> 5;
  TC (*sR)[LD] = reinterpret_cast<TC (*)[LD]>(lds);                       // current rows, by original tile row
  TC (*sL)[LD] = reinterpret_cast<TC (*)[LD]>(lds + kTile * LD);          // multipliers: sL[r][C]
  TC (*sF)[LD] = reinterpret_cast<TC (*)[LD]>(lds + 2 * kTile * LD);      // factored tile in pivot order
  TC (*sFT)[LD] = reinterpret_cast<TC (*)[LD]>(lds + 3 * kTile * LD);     // its transpose
  TC* sD = lds + 4 * kTile * LD;                                         // reciprocals of U's diagonal
  // The tile (rows and columns past the matrix become identity rows): all
  // loads first, from the whole LDS tile or clamped matrix addresses, so
  // that no load waits under a per-element branch.
  TC a[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int c = 16 * half + t;
    a[t] = static_cast<TC>(sT ? sT[r * ldt + c] : gload(A + static_cast<int64_t>(t0 + min(r, ts - 1)) * b + t0 + min(c, ts - 1)));
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int c = 16 * half + t;
    if (!(r < ts && c < ts)) a[t] = r == c ? TC(1) : TC(0);
  }
  bool done = false;
  int pos = r;  // position of this row in the factored tile (rows >= ts keep theirs)
#pragma unroll
  for (int t = 0; t < 16; ++t) sR[r][16 * half + t] = a[t];
  wave_lds_order();
  // Column loop (not unrolled, so the kernel stays small for the instruction
  // cache).  Pivoting is implicit: rows stay in their lanes.  Every lane keeps
  // the current values of columns C and C + 1 of its row in registers (xc,
  // yc), so the critical path of a step is: pivot value and pivot-row value
  // by lane reads, multiplier, update of column C + 1, pivot search of
  // column C + 1.  The rest of each row is updated from the pivot row as
  // published in LDS after the previous step, column C + 2 is prepared the
  // same way, and the multipliers go to sL (so the row update needs no
  // column mask: columns left of C of unchosen rows are dead).  All those
  // LDS accesses are off the critical path.  The pivot search of column
  // C + 1 ranks the rows by |piv yc - xc u1| = |piv| |yn| (the same order as
  // |yn|), so it does not wait for the reciprocal of the pivot.
  TC xc = sR[r][0], yc = sR[r][1];
  int p = half_argmax(pivot_key(xc, half == 0 && r < ts, r), 0);
  bool bad = false;
  for (int C = 0; C < ts; ++C) {
    // Reads of the pivot row first: their latency overlaps the search.
    const int c2 = min(C + 2, kTile + 1);
    const TC y2 = sR[r][c2], u2 = sR[p][c2];
    TC prow[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) prow[t] = sR[p][16 * half + t];
    const TC piv = read_lane(xc, p);
    const TC u1 = read_lane(yc, p);
    const bool act = !done && r < ts && r != p;
    if (r == p) {
      done = true;
      pos = C;
    }
    // Pivot of column C + 1 (computed unconditionally so the step is one
    // basic block; unused after the last column), then the multiplier and
    // columns C + 1 and C + 2 of every row; the scheduling barriers keep
    // this chain ahead of the bulk row update.
    const TC ys = fma(piv, yc, -(xc * u1));
    const int pn = half_argmax(pivot_key(ys, half == 0 && !done && r < ts, r), 0);
    bad = bad || !(piv != TC(0) && isfinite(piv));
    const TC rinv = piv != TC(0) ? tile_rcp(piv) : TC(0);
    const TC lm = act ? xc * rinv : TC(0);
    const TC yn = fma(-lm, u1, yc);  // column C + 1 after this step
    const TC z = fma(-lm, u2, y2);   // column C + 2 after this step
    __builtin_amdgcn_sched_barrier(0);
    sL[r][C] = lm;  // every lane (both halves store the same value); read only for rows chosen later
#pragma unroll
    for (int t = 0; t < 16; ++t) a[t] = fma(-lm, prow[t], a[t]);  // same operations as yn and z
    wave_lds_order();
#pragma unroll
    for (int t = 0; t < 16; ++t) sR[r][16 * half + t] = a[t];
    wave_lds_order();
    xc = yn;
    yc = z;
    p = pn;
    __builtin_amdgcn_sched_barrier(0);
  }
  if (bad && l == 0 && it.info) atomicCAS(it.info, 0, it.node + 1);
  wave_lds_order();
  // Factored row in pivot order: multipliers left of its pivot column, U
  // from there on (rows past the tile edge are identity rows).
  TC fv[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) fv[t] = sL[r][16 * half + t];  // read in full, used left of pos
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int c = 16 * half + t;
    fv[t] = (r < ts && c < pos) ? fv[t] : a[t];
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int c = 16 * half + t;
    sF[pos][c] = fv[t];
    sFT[c][pos] = fv[t];
  }
  {
    // Growth: the tile's entries of U (the row from its pivot column on).
    float um = 0.f;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = 16 * half + t;
      if (r < ts && c >= pos && c < ts) um = nan_fmax(um, static_cast<float>(fabs(a[t])));
    }
    note_umax(it.swaps + kUmaxWord, um);
  }
  // Row movement of the tile: position pos holds original tile row r.  Rows
  // never leave their band, so the band's permutation entries are t0 + r.
  if (half == 0 && r < ts) {
    gstore(step_perm(it, s) + pos, r);
    gstore(it.perm + t0 + pos, t0 + r);
  }
  wave_lds_order();
  if (l < kTile) sD[l] = TC(1) / sF[l][l];
  wave_lds_order();
  // Inverses of the tile's triangular factors by forward substitution in
  // column (axpy) form, every update of a step independent:
  //   lanes 0..31 : column r of L^{-1}        (L unit lower: L[i][q] = sFT[q][i]);
  //   lanes 32..63: column r of (U^T)^{-1} = row r of U^{-1}
  //                 ((U^T)[i][q] = U[q][i] = sF[q][i], diagonal 1 / sD).
  // Element i of operand row q + 1 is read from LDS as soon as step q has
  // used element i of row q (scheduling barriers keep every step's reads
  // next to it), so one row of registers holds the operand.
  const TC* Mq = half ? &sF[0][0] : &sFT[0][0];
  TC xs[kTile];
#pragma unroll
  for (int q = 0; q < kTile; ++q) xs[q] = (q == r) ? TC(1) : TC(0);
  TC mrow[kTile];
#pragma unroll
  for (int i = 1; i < kTile; ++i) mrow[i] = Mq[i];
  TC dq = sD[0];
#pragma unroll
  for (int q = 0; q < kTile; ++q) {
    const TC xq = half ? xs[q] * dq : xs[q];
    xs[q] = xq;
    if (q + 1 < kTile) dq = sD[q + 1];
#pragma unroll
    for (int i = q + 1; i < kTile; ++i) {
      xs[i] = fma(-mrow[i], xq, xs[i]);
      if (i >= q + 2) mrow[i] = Mq[(q + 1) * LD + i];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  T* aux = step_inv<T>(it, s);
  if (half == 0) {
#pragma unroll
    for (int i = 0; i < kTile; ++i) gstore(aux + i * kTile + r, static_cast<T>(xs[i]));  // L^{-1}[i][r]
  } else {
#pragma unroll
    for (int i = 0; i < kTile; ++i) gstore(aux + kTile * kTile + r * kTile + i, static_cast<T>(xs[i]));  // U^{-1}[r][i]
  }
}

static_assert(kTrtriTile == kTile, "the tile LU inverts the diagonal tiles of the triangular inversion");

// Diagonal tile q receives its packed inverses from aux (L^{-1} below the
// diagonal, U^{-1} on and above it), the form the triangular inversion that
// follows every factorisation starts from; no kernel reads a tile's factors
// once its inverses are in aux.  The tile steps copy them (off the critical
// path); a matrix of a single tile is handled by k_tile_lu.
template <typename T>
__device__ __forceinline__ void step_diag_inverse(const LuItem& it, int q) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, tq = q * kTile, ts = min(kTile, b - tq);
  const T* inv = step_inv<T>(it, q);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int i = e >> 5, c = e & 31;
    if (i < ts && c < ts)
      gstore(A + static_cast<int64_t>(tq + i) * b + tq + c, gload(inv + (c < i ? 0 : kTile * kTile) + e));
  }
}

// C: the arithmetic of the tile factorisation (double for the mixed paths'
// float matrices: their pivot selection and smallest-block LU run in FP64).
template <typename T, typename C>
__global__ __launch_bounds__(64) void k_tile_lu(const LuItem* items, int t0) {
  __shared__ __attribute__((aligned(16))) C lds[kLuLdsElems];
  tile_lu_wave<T, C>(items[blockIdx.x], t0, nullptr, 0, lds);
  if (t0 == 0 && items[blockIdx.x].b <= kTile) {
    __threadfence();  // the inverses this wavefront stored to aux
    step_diag_inverse<T>(items[blockIdx.x], 0);
  }
}

// Element growth of the tile-pivoting LUs (words kAmaxWord.. and kUmaxWord of
// LuItem::swaps).  Before the factorisation workgroup g records the largest
// magnitude of rows [b g / P, b (g + 1) / P) (P = kAmaxParts) and workgroup 0
// clears the |U| maximum that the factorisation then raises.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_amax(const LuItem* items) {
  const LuItem it = items[blockIdx.y];
  const int b = it.b, g = blockIdx.x;
  const int64_t r0 = static_cast<int64_t>(b) * g / kAmaxParts, r1 = static_cast<int64_t>(b) * (g + 1) / kAmaxParts;
  const T* A = static_cast<const T*>(it.a);
  float m = 0.f;
  for (int64_t e = r0 * b + threadIdx.x; e < r1 * b; e += 256) m = nan_fmax(m, static_cast<float>(fabs(gload(A + e))));
  __shared__ float part[4];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = nan_fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = nan_fmax(nan_fmax(part[0], part[1]), nan_fmax(part[2], part[3]));
    it.swaps[kAmaxWord + g] = __float_as_int(m);
    if (g == 0) it.swaps[kUmaxWord] = 0;
  }
}

// After the factorisation: growth above kGrowthLimit (or a non-finite |U|)
// is reported like a failed pivot of this Schur operation.  One wavefront
// per matrix.
__global__ __launch_bounds__(64) void k_lu_check(const LuItem* items) {
  const LuItem it = items[blockIdx.x];
  const int l = threadIdx.x;
  float a = l < kAmaxParts ? __int_as_float(it.swaps[kAmaxWord + l]) : 0.f;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) a = nan_fmax(a, __shfl_xor(a, o, 64));
  const float u = __int_as_float(it.swaps[kUmaxWord]);
  if (l == 0 && it.info && !(u <= kGrowthLimit * a)) atomicCAS(it.info, 0, it.node + 1);
}

// Base case of the recursive LU (launch_getrf_rec): diagonal tile t0 / kTile
// is factored and replaced by its packed inverses (L^{-1} strictly below the
// diagonal, U^{-1} on and above it), its permutation composed into perm.
template <typename T, typename C>
__global__ __launch_bounds__(64) void k_tile_lu_inv(const LuItem* items, int t0) {
  __shared__ __attribute__((aligned(16))) C lds[kLuLdsElems];
  tile_lu_wave<T, C>(items[blockIdx.x], t0, nullptr, 0, lds);
  __threadfence();  // the inverses this wavefront stored to aux
  step_diag_inverse<T>(items[blockIdx.x], t0 / kTile);
}

// ---------------------------------------------------------------------------
// Tile step of the tile-pivoting LU.  The launch for diagonal tile s (rows
// and columns [t0, t0 + kTile)) runs after tile s has been factored, and its
// workgroups share the work that needs only tiles s - 1 and s:
//   look-ahead (first workgroup): tile s + 1 receives the update of panel s,
//       A_tt -= (A_t,s U_s^{-1}) (L_s^{-1} P_s A_s,t), and is factored, so the
//       next launch can start at once (the factorisation's critical path);
//   trailing blocks: 64 x 64 blocks of the matrix right of and below tile s
//       (tile s + 1 excepted) receive the same update; every block forms the
//       pieces of L21 = A21 U_s^{-1} and U12 = L_s^{-1} P_s A12 it needs in
//       LDS, since other blocks still read the unreduced strips;
//   strip blocks: the strips of tile s - 1, which no block reads any more,
//       are reduced in place (L21 rows with the rows of tile s's band in
//       their new order, U12 columns);
//   band blocks: the rows of tile s's band are permuted in the columns left
//       of tile s - 1 (the L part; the U part is formed in pivot order).
// All products run on MFMA from LDS operands; 256 threads per workgroup.
// ---------------------------------------------------------------------------
constexpr int kStepLd = kTile + 1;      // LDS leading dimension of 32-wide operands
constexpr int kStepLdw = 64 + 1;        // of 64-wide operands
constexpr int kStepLdsElems = 64 * kStepLd + kTile * kStepLdw + 2 * kTile * kStepLd;
static_assert(kStepLdsElems >= kTile * kStepLd + kLuLdsElems, "step LDS too small for the look-ahead");

// acc (+/-)= A[16 x kTile] B[kTile x 16] from LDS (row-major, leading dimensions lda, ldb).
template <typename T, bool NEG>
__device__ __forceinline__ void frag_mma(const T* A, int lda, const T* B, int ldb, typename MF<T>::acc& acc) {
  const int lane = threadIdx.x & 63, i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < kTile; k0 += 4) {
    const T av = A[i * lda + k0 + k];
    acc = MF<T>::mma(NEG ? -av : av, B[(k0 + k) * ldb + i], acc);
  }
}

template <typename T>
__device__ __forceinline__ void zero_acc(typename MF<T>::acc& acc) {
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = T(0);
}

// Stages the two tile inverses of step s (kTile x kTile each) into LDS.
// The staging functions below issue all their loads before any LDS store
// (one wait per function, not one per element).
constexpr int kStagePer = kTile * kTile / 256;  // elements per thread of a 32 x 32 operand
template <typename T>
__device__ __forceinline__ void stage_inverses(const LuItem& it, int s, T* sLi, T* sUi) {
  const T* inv = step_inv<T>(it, s);
  T vl[kStagePer], vu[kStagePer];
#pragma unroll
  for (int u = 0; u < kStagePer; ++u) {
    const int e = threadIdx.x + 256 * u;
    if (sLi) vl[u] = gload(inv + e);
    if (sUi) vu[u] = gload(inv + kTile * kTile + e);
  }
#pragma unroll
  for (int u = 0; u < kStagePer; ++u) {
    const int e = threadIdx.x + 256 * u, q = e >> 5, c = e & 31;
    if (sLi) sLi[q * kStepLd + c] = vl[u];
    if (sUi) sUi[q * kStepLd + c] = vu[u];
  }
}
// Stages L_s^{-1} P_s instead of L_s^{-1}: column pm[c] receives column c of
// L_s^{-1}, so that (L_s^{-1} P_s) A12 = L_s^{-1} (P_s A12) reads the band
// rows of A12 in their stored order and no load waits for the permutation.
template <typename T>
__device__ __forceinline__ void stage_linv_perm(const LuItem& it, int s, T* sLi) {
  const T* inv = step_inv<T>(it, s);
  const int32_t* pm = step_perm(it, s);
  T v[kStagePer];
  int col[kStagePer];
#pragma unroll
  for (int u = 0; u < kStagePer; ++u) {
    const int e = threadIdx.x + 256 * u;
    v[u] = gload(inv + e);
    col[u] = gload(pm + (e & 31));
  }
#pragma unroll
  for (int u = 0; u < kStagePer; ++u) {
    const int e = threadIdx.x + 256 * u;
    sLi[(e >> 5) * kStepLd + col[u]] = v[u];
  }
}

template <typename T, typename C>
__device__ __forceinline__ void step_lookahead(const LuItem& it, int t0, T* smem) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, s = t0 / kTile, t1 = t0 + kTile, ts1 = min(kTile, b - t1);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  T* sT = smem;                    // updated tile s + 1
  T* sA = sT + kTile * kStepLd;    // its rows of strip s, then L21
  T* sB = sA + kTile * kStepLd;    // its columns of band s (P_s order), then U12
  T* sLi = sB + kTile * kStepLd;
  T* sUi = sLi + kTile * kStepLd;
  const int fi = wave >> 1, fj = wave & 1;
  typename MF<T>::acc acc;  // this wavefront's 16 x 16 fragment of tile s + 1, requested first
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = 16 * fi + MF<T>::row(lane, v), y = 16 * fj + (lane & 15);
    acc[v] = gload(A + static_cast<int64_t>(min(t1 + x, b - 1)) * b + min(t1 + y, b - 1));
  }
  {
    // Rows / columns past the matrix read its last row / column and are zeroed.
    T va[kStagePer], vb[kStagePer];
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int e = tid + 256 * u, x = e >> 5, y = e & 31;
      va[u] = gload(A + static_cast<int64_t>(min(t1 + x, b - 1)) * b + t0 + y);
      vb[u] = gload(A + static_cast<int64_t>(t0 + x) * b + min(t1 + y, b - 1));
    }
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int e = tid + 256 * u, x = e >> 5, y = e & 31;
      sA[x * kStepLd + y] = x < ts1 ? va[u] : T(0);
      sB[x * kStepLd + y] = y < ts1 ? vb[u] : T(0);
    }
  }
  stage_linv_perm<T>(it, s, sLi);
  stage_inverses<T>(it, s, static_cast<T*>(nullptr), sUi);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = 16 * fi + MF<T>::row(lane, v), y = 16 * fj + (lane & 15);
    if (!(x < ts1 && y < ts1)) acc[v] = T(0);
  }
  __syncthreads();
  // L21 fragment (wave >> 1, wave & 1) and U12 fragment (wave >> 1, wave & 1)
  typename MF<T>::acc l21, u12;
  zero_acc<T>(l21);
  zero_acc<T>(u12);
  frag_mma<T, false>(sA + 16 * fi * kStepLd, kStepLd, sUi + 16 * fj, kStepLd, l21);
  frag_mma<T, false>(sLi + 16 * fi * kStepLd, kStepLd, sB + 16 * fj, kStepLd, u12);
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = 16 * fi + MF<T>::row(lane, v), y = 16 * fj + (lane & 15);
    sA[x * kStepLd + y] = l21[v];
    sB[x * kStepLd + y] = u12[v];
  }
  __syncthreads();
  frag_mma<T, true>(sA + 16 * fi * kStepLd, kStepLd, sB + 16 * fj, kStepLd, acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = 16 * fi + MF<T>::row(lane, v), y = 16 * fj + (lane & 15);
    sT[x * kStepLd + y] = acc[v];
  }
  __syncthreads();
  // (sA sits 8-byte aligned, and the workgroup's LDS holds kStepLdsElems
  // doubles, room for the factorisation's scratch in C after it)
  if (wave == 0) tile_lu_wave<T, C>(it, t1, sT, kStepLd, reinterpret_cast<C*>(sA));
}

template <typename T>
__device__ __forceinline__ void step_trailing(const LuItem& it, int t0, int ti, int tj, T* smem) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, s = t0 / kTile, t1 = t0 + kTile;
  const int r0 = t1 + 64 * ti, c0 = t1 + 64 * tj;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  T* sA = smem;                     // [64][kStepLd]: rows r0.. of strip s, then L21
  T* sB = sA + 64 * kStepLd;        // [kTile][kStepLdw]: band s (P_s order), columns c0.., then U12
  T* sLi = sB + kTile * kStepLdw;
  T* sUi = sLi + kTile * kStepLd;
  // The block of C (32 x 32 per wavefront) is requested first: its loads are
  // in flight while the strip pieces are formed.
  // (Unconditional loads from clamped addresses, zeroed past the matrix
  // once they have landed: a load under a per-element branch waits.)
  const int wr = wave >> 1, wc = wave & 1;
  typename MF<T>::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = r0 + 32 * wr + 16 * i + MF<T>::row(lane, v), gc = c0 + 32 * wc + 16 * j + (lane & 15);
        acc[i][j][v] = gload(A + static_cast<int64_t>(min(gr, b - 1)) * b + min(gc, b - 1));
      }
  {
    // Rows / columns past the matrix read its last row / column and are zeroed.
    constexpr int PER = 64 * kTile / 256;
    T va[PER], vb[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      va[u] = gload(A + static_cast<int64_t>(min(r0 + (e >> 5), b - 1)) * b + t0 + (e & 31));
      vb[u] = gload(A + static_cast<int64_t>(t0 + (e >> 6)) * b + min(c0 + (e & 63), b - 1));
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      sA[(e >> 5) * kStepLd + (e & 31)] = r0 + (e >> 5) < b ? va[u] : T(0);
      sB[(e >> 6) * kStepLdw + (e & 63)] = c0 + (e & 63) < b ? vb[u] : T(0);
    }
  }
  stage_linv_perm<T>(it, s, sLi);
  stage_inverses<T>(it, s, static_cast<T*>(nullptr), sUi);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = r0 + 32 * wr + 16 * i + MF<T>::row(lane, v), gc = c0 + 32 * wc + 16 * j + (lane & 15);
        if (!(gr < b && gc < b)) acc[i][j][v] = T(0);
      }
  __syncthreads();
  // Strip pieces: L21 (64 x 32, fragments 0..7) and U12 (32 x 64, fragments
  // 8..15); wavefront w forms fragments w, w + 4, w + 8, w + 12.
  typename MF<T>::acc pc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = wave + 4 * j;
    zero_acc<T>(pc[j]);
    if (f < 8)
      frag_mma<T, false>(sA + 16 * (f >> 1) * kStepLd, kStepLd, sUi + 16 * (f & 1), kStepLd, pc[j]);
    else
      frag_mma<T, false>(sLi + 16 * ((f - 8) >> 2) * kStepLd, kStepLd, sB + 16 * ((f - 8) & 3), kStepLdw, pc[j]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = wave + 4 * j;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int x = MF<T>::row(lane, v), y = lane & 15;
      if (f < 8)
        sA[(16 * (f >> 1) + x) * kStepLd + 16 * (f & 1) + y] = pc[j][v];
      else
        sB[(16 * ((f - 8) >> 2) + x) * kStepLdw + 16 * ((f - 8) & 3) + y] = pc[j][v];
    }
  }
  __syncthreads();
  // C -= L21 U12 on the 32 x 32 quarter of wavefront w.
#pragma unroll
  for (int k0 = 0; k0 < kTile; k0 += 4) {
    const int k = k0 + (lane >> 4);
    T av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = -sA[(32 * wr + 16 * i + (lane & 15)) * kStepLd + k];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = sB[k * kStepLdw + 32 * wc + 16 * j + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = MF<T>::mma(av[i], bv[j], acc[i][j]);
  }
  const int look = t1 + kTile;  // tile s + 1 belongs to the look-ahead workgroup
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = r0 + 32 * wr + 16 * i + MF<T>::row(lane, v), gc = c0 + 32 * wc + 16 * j + (lane & 15);
        if (gr < b && gc < b && !(gr < look && gc < look)) gstore(A + static_cast<int64_t>(gr) * b + gc, acc[i][j][v]);
      }
}

// L21 of tile s - 1 for rows [R0, R0 + 64): A21 U^{-1}, in place; rows of
// tile s's band are taken in their new order.
template <typename T>
__device__ __forceinline__ void step_strip_rows(const LuItem& it, int t0, int i, T* smem) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, s = t0 / kTile, tp = t0 - kTile, ts = min(kTile, b - t0), R0 = t0 + 64 * i;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  T* sX = smem;                   // [64][kStepLd]
  T* sUi = sX + 64 * kStepLd;
  const int32_t* pm = step_perm(it, s);
  {
    // Source rows first (rows of tile s's band through its permutation),
    // then the values; rows past the matrix read its last row, zeroed.
    constexpr int PER = 64 * kTile / 256;
    int src[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int g = R0 + ((tid + 256 * u) >> 5);
      src[u] = gload(pm + min(g - t0, ts - 1));  // used only for rows of tile s's band
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int g = R0 + ((tid + 256 * u) >> 5);
      src[u] = g < t0 + ts ? t0 + src[u] : min(g, b - 1);
    }
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = gload(A + static_cast<int64_t>(src[u]) * b + tp + ((tid + 256 * u) & 31));
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, x = e >> 5;
      sX[x * kStepLd + (e & 31)] = R0 + x < b ? v[u] : T(0);
    }
  }
  stage_inverses<T>(it, s - 1, static_cast<T*>(nullptr), sUi);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int f = wave + 4 * j, fi = f >> 1, fj = f & 1;
    typename MF<T>::acc acc;
    zero_acc<T>(acc);
    frag_mma<T, false>(sX + 16 * fi * kStepLd, kStepLd, sUi + 16 * fj, kStepLd, acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int g = R0 + 16 * fi + MF<T>::row(lane, v);
      if (g < b) gstore(A + static_cast<int64_t>(g) * b + tp + 16 * fj + (lane & 15), acc[v]);
    }
  }
}

// U12 of tile s - 1 for columns [C0, C0 + 64): L^{-1} P A12, in place.
template <typename T>
__device__ __forceinline__ void step_strip_cols(const LuItem& it, int t0, int j, T* smem) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, s = t0 / kTile, tp = t0 - kTile, C0 = t0 + 64 * j;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  T* sB = smem;                   // [kTile][kStepLdw]
  T* sLi = sB + kTile * kStepLdw;
  {
    // Columns past the matrix read its last column and are zeroed.
    constexpr int PER = kTile * 64 / 256;
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      v[u] = gload(A + static_cast<int64_t>(tp + (e >> 6)) * b + min(C0 + (e & 63), b - 1));
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      sB[(e >> 6) * kStepLdw + (e & 63)] = C0 + (e & 63) < b ? v[u] : T(0);
    }
  }
  stage_linv_perm<T>(it, s - 1, sLi);
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < 2; ++jj) {
    const int f = wave + 4 * jj, gi = f >> 2, gj = f & 3;
    typename MF<T>::acc acc;
    zero_acc<T>(acc);
    frag_mma<T, false>(sLi + 16 * gi * kStepLd, kStepLd, sB + 16 * gj, kStepLdw, acc);
    float um = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int y = C0 + 16 * gj + (lane & 15);
      if (y < b) {
        gstore(A + static_cast<int64_t>(tp + 16 * gi + MF<T>::row(lane, v)) * b + y, acc[v]);
        um = nan_fmax(um, static_cast<float>(fabs(acc[v])));
      }
    }
    note_umax(it.swaps + kUmaxWord, um);  // U12 of tile s - 1
  }
}

// Rows of tile s's band in their new order, columns [64 j, 64 j + 64) left
// of tile s - 1.
template <typename T>
__device__ __forceinline__ void step_band(const LuItem& it, int t0, int j) {
  T* A = static_cast<T*>(it.a);
  const int b = it.b, s = t0 / kTile, ts = min(kTile, b - t0), cend = t0 - kTile;
  const int32_t* pm = step_perm(it, s);
  // Permutation entries first, then the rows (clamped addresses; entries
  // past the band or the columns are not stored).
  int src[kTile * 64 / 256];
#pragma unroll
  for (int t = 0; t < kTile * 64 / 256; ++t) src[t] = gload(pm + min(static_cast<int>(threadIdx.x + 256 * t) >> 6, ts - 1));
  T v[kTile * 64 / 256];
#pragma unroll
  for (int t = 0; t < kTile * 64 / 256; ++t) {
    const int e = threadIdx.x + 256 * t, y = 64 * j + (e & 63);
    v[t] = gload(A + static_cast<int64_t>(t0 + src[t]) * b + min(y, cend - 1));
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kTile * 64 / 256; ++t) {
    const int e = threadIdx.x + 256 * t, q = e >> 6, y = 64 * j + (e & 63);
    if (q < ts && y < cend) gstore(A + static_cast<int64_t>(t0 + q) * b + y, v[t]);
  }
}

// Workgroup counts of the tile step at t0 for a matrix of order b.
struct StepShape {
  int look, trail_n, strip, band;
  __host__ __device__ StepShape(int b, int t0) {
    const int s = t0 / kTile, rest = b - t0 - kTile;
    look = rest > 0 ? 1 : 0;
    trail_n = rest > 0 ? (rest + 63) / 64 : 0;
    strip = s > 0 ? (b - t0 + 63) / 64 : 0;
    band = s > 1 ? (t0 - kTile + 63) / 64 : 0;
  }
  __host__ __device__ int total() const { return look + trail_n * trail_n + 2 * strip + band; }
};

template <typename T, typename C>
__global__ __launch_bounds__(256) void k_lu_step(const LuItem* items, int t0) {
  // kStepLdsElems doubles whatever T is: the look-ahead factorisation may
  // compute a float matrix's tile in double.
  __shared__ __attribute__((aligned(16))) double smem_raw[kStepLdsElems];
  T* smem = reinterpret_cast<T*>(smem_raw);
  // Workgroups are numbered matrix-fastest: the look-ahead workgroups of all
  // matrices come first, and consecutive workgroups (which the dispatcher
  // spreads over the XCDs in turn) of one matrix land on the same XCDs, so
  // the strips and tile inverses every block of a matrix reads stay in
  // those XCDs' L2.
  int item, role;
  gemm_workgroup(item, role);
  const LuItem it = items[item];
  if (t0 >= it.b) return;  // a smaller matrix of a merged batch
  const StepShape sh(it.b, t0);
  int bx = role;
  if (bx < sh.look) {
    step_lookahead<T, C>(it, t0, smem);
    return;
  }
  bx -= sh.look;
  if (bx < sh.trail_n * sh.trail_n) {
    step_trailing<T>(it, t0, bx / sh.trail_n, bx % sh.trail_n, smem);
    return;
  }
  bx -= sh.trail_n * sh.trail_n;
  if (bx < sh.strip) {
    step_strip_rows<T>(it, t0, bx, smem);
    return;
  }
  bx -= sh.strip;
  if (bx < sh.strip) {
    step_strip_cols<T>(it, t0, bx, smem);
    if (bx == 0) {
      // The inverses of tile s - 1 (and of the last tile, which no later
      // launch sees) go to their diagonal tiles.
      step_diag_inverse<T>(it, t0 / kTile - 1);
      if (t0 + kTile >= it.b) step_diag_inverse<T>(it, t0 / kTile);
    }
    return;
  }
  bx -= sh.strip;
  if (bx < sh.band) step_band<T>(it, t0, bx);
}

// ---------------------------------------------------------------------------
// Row interchanges of a panel applied to the columns outside it, and the
// unit-lower solve U12 = L11^{-1} A12 for the columns right of it.  A
// workgroup of 128 threads owns 128 columns: the moved rows are first read
// into LDS, then written to their destinations, then thread t solves the
// panel system for column t.
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(128) void k_laswp_trsm(const LuItem* items, int j, int w) {
  constexpr int NT = 128;
  const LuItem it = items[blockIdx.y];
  T* A = static_cast<T*>(it.a);
  const int b = it.b;
  __shared__ int s_dst[2 * NB], s_src[2 * NB];
  __shared__ T s_L[NB][NB + 1];
  __shared__ T s_rows[2 * NB][NT];
  const int tid = threadIdx.x;
  const int cnt = it.swaps[0];
  for (int e = tid; e < 2 * NB; e += NT) {
    s_dst[e] = it.swaps[1 + 2 * e];
    s_src[e] = it.swaps[2 + 2 * e];
  }
  for (int e = tid; e < NB * NB; e += NT) {
    const int r = e / NB, c = e % NB;
    s_L[r][c] = (r < w && c < w) ? A[static_cast<int64_t>(j + r) * b + j + c] : T(0);
  }
  __syncthreads();
  const int col = blockIdx.x * NT + tid;
  const bool mine = col < b && !(col >= j && col < j + w);
  if (mine) {
    for (int q = 0; q < cnt; ++q) s_rows[q][tid] = A[static_cast<int64_t>(s_src[q]) * b + col];
    for (int q = 0; q < cnt; ++q) A[static_cast<int64_t>(s_dst[q]) * b + col] = s_rows[q][tid];
  }
  if (mine && col >= j + w) {
    // Forward substitution with the unit-lower L11, column-oriented: after
    // x[s] is final, x[r] -= L[r][s] x[s] for r > s.  Register indices are
    // static (predicated), the column loop is a runtime loop.
    T x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) x[r] = (r < w) ? A[static_cast<int64_t>(j + r) * b + col] : T(0);
    for (int s2 = 0; s2 + 1 < w; ++s2) {
      T xs = T(0);
#pragma unroll
      for (int r = 0; r < NB; ++r) xs = (r == s2) ? x[r] : xs;
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (r > s2) x[r] -= s_L[r][s2] * xs;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
      if (r < w) A[static_cast<int64_t>(j + r) * b + col] = x[r];
  }
}

// ---------------------------------------------------------------------------
// Inverts the TB x TB diagonal tiles of the packed factors in place: wave 0
// solves L x = e_c (unit lower) and wave 1 solves U x = e_c for the columns c
// of the tile (lane c; TB <= 64).
// ---------------------------------------------------------------------------
template <typename T, int TB>
__global__ __launch_bounds__(128) void k_trtri_diag(const LuItem* items) {
  const LuItem it = items[blockIdx.y];
  T* A = static_cast<T*>(it.a);
  const int b = it.b;
  const int t0 = blockIdx.x * TB;
  if (t0 >= b) return;
  const int ts = min(TB, b - t0);
  __shared__ T S[TB][TB + 1];
  __shared__ T X[2][TB][64];  // per-thread solution columns
  const int tid = threadIdx.x;
  for (int e = tid; e < TB * TB; e += 128) {
    const int r = e / TB, c = e % TB;
    S[r][c] = (r < ts && c < ts) ? A[static_cast<int64_t>(t0 + r) * b + t0 + c] : (r == c ? T(1) : T(0));
  }
  __syncthreads();
  const int jc = tid & 63, part = tid >> 6;
  if (jc >= ts) return;
  T(&x)[TB][64] = X[part];
  if (part == 0) {
    // L x = e_jc, unit lower: x[r] = 0 for r < jc, x[jc] = 1.
    for (int r = jc + 1; r < ts; ++r) {
      T acc = -S[r][jc];
      for (int q = jc + 1; q < r; ++q) acc -= S[r][q] * x[q][jc];
      x[r][jc] = acc;
      A[static_cast<int64_t>(t0 + r) * b + t0 + jc] = acc;
    }
  } else {
    // U x = e_jc: x[r] = 0 for r > jc.
    for (int r = jc; r >= 0; --r) {
      T acc = (r == jc) ? T(1) : T(0);
      for (int q = r + 1; q <= jc; ++q) acc -= S[r][q] * x[q][jc];
      acc /= S[r][r];
      x[r][jc] = acc;
      A[static_cast<int64_t>(t0 + r) * b + t0 + jc] = acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_load(const LoadItem* items) {
  const LoadItem it = items[blockIdx.y];
  const int64_t total = static_cast<int64_t>(it.rows) * it.cols;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * 256) {
    const int x = static_cast<int>(e / it.cols), y = static_cast<int>(e % it.cols);
    static_cast<T*>(it.dst)[static_cast<int64_t>(x) * it.ldd + y] = vget<T>(it.src, x, y);
  }
}

__global__ void k_fill_int(int32_t* p, int n, int v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace {
inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }
}  // namespace

template <int LP, int MODE, bool GEN, int BM, int BN, int WM, int WN>
void launch_lp_shape(const GemmLaunch& L, int count, int max_m, int max_n, hipStream_t st) {
  dim3 grid(cdiv(max_m, BM) * cdiv(max_n, BN), count);
  hipLaunchKernelGGL((k_gemm_lp<LP, MODE, GEN, BM, BN, WM, WN>), grid, dim3((BM / WM) * (BN / WN) * 64), 0, st, L);
}

template <int MODE, bool GEN>
hipError_t launch_gemm_lp(const GemmLaunch& L, int count, int max_m, int max_n, hipStream_t st) {
  // 16 wavefronts per workgroup (four per SIMD hide the splitting, LDS and
  // memory latency between MFMA issues): 128 x 128 tiles of 32 x 32 per
  // wavefront from half a tile per compute unit on, 64 x 64 tiles of
  // 16 x 16 below (a single 1024 x 1024 product: 49 us instead of 84 us on
  // 64 x 64 tiles of four wavefronts).
  if constexpr (!GEN) {
    const int64_t big_tiles = static_cast<int64_t>(cdiv(max_m, 128)) * cdiv(max_n, 128) * count;
    if (max_m >= 128 && max_n >= 128 && big_tiles >= 128) {
      if (L.lp == 1)
        launch_lp_shape<1, MODE, GEN, 128, 128, 32, 32>(L, count, max_m, max_n, st);
      else
        launch_lp_shape<2, MODE, GEN, 128, 128, 32, 32>(L, count, max_m, max_n, st);
    } else if (L.lp == 1) {
      launch_lp_shape<1, MODE, GEN, 64, 64, 16, 16>(L, count, max_m, max_n, st);
    } else {
      launch_lp_shape<2, MODE, GEN, 64, 64, 16, 16>(L, count, max_m, max_n, st);
    }
    return hipGetLastError();
  }
  if (L.lp == 1)
    launch_lp_shape<1, MODE, GEN, 64, 64, 32, 32>(L, count, max_m, max_n, st);
  else
    launch_lp_shape<2, MODE, GEN, 64, 64, 32, 32>(L, count, max_m, max_n, st);
  return hipGetLastError();
}

// Tile shape of a product launch (see launch_gemm_mode).
constexpr int kTierLarge = 0, kTierMedium = 1, kTierTiny = 2, kTierSmall = 3;
inline int gemm_tier(const GemmLaunch& L, int mode, int count, int max_m, int max_n) {
  const bool tri = L.tri != 0 || mode == GEMM_TRTRI_STEP1 || mode == GEMM_TRTRI_STEP2;
  const int64_t big_tiles = static_cast<int64_t>(cdiv(max_m, 128)) * cdiv(max_n, 256) * count;
  const int64_t mid_tiles = static_cast<int64_t>(cdiv(max_m, 128)) * cdiv(max_n, 128) * count;
  if (max_m >= 128 && max_n >= 256 && big_tiles >= (tri ? 512 : 192)) return kTierLarge;
  if (max_m >= 128 && max_n >= 128 && mid_tiles >= (tri ? 512 : 128)) return kTierMedium;
  if (max_m <= 32 && max_n <= 32) return kTierTiny;
  return kTierSmall;
}

template <typename T, int MODE, bool GEN>
hipError_t launch_gemm_mode(const GemmLaunch& L, int count, int max_m, int max_n, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (L.lp) return launch_gemm_lp<MODE, GEN>(L, count, max_m, max_n, st);
  }
  // Tile shapes by the number of output tiles the launch has (four
  // wavefronts per SIMD where possible, so MFMA issue continues while other
  // wavefronts wait on LDS or memory):
  //   large: 128 x 256 tiles, 16 wavefronts of 64 x 32, K steps of 16;
  //   medium: 128 x 128 tiles, 16 wavefronts of 32 x 32, K steps of 32;
  //   small: 64 x 64 tiles, 16 wavefronts of 16 x 16, K steps of 64.
  // The fewer the output tiles per compute unit, the longer the K step, so
  // that the operand loads issued one step ahead still cover the memory
  // latency (a single 1024 x 1024 product has one 64 x 64 tile per unit).
  // The generic (element-wise view) instance and the trailing updates of the
  // partial-pivoting LU take 64 x 64 tiles of four 32 x 32 wavefronts.
  // Products with a triangular operand have uneven tiles and take the larger
  // shapes only with at least two workgroups per compute unit.  A shape is
  // used only when the products are at least as large as its tile (the
  // small levels of the triangular inversion have many 32 x 32 products:
  // 32 x 32 tiles of four 16 x 16 wavefronts).
  if constexpr (!GEN && MODE != GEMM_LU_TRAILING) {
    const int tier = gemm_tier(L, MODE, count, max_m, max_n);
    if (tier == kTierLarge) {
      dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 256), count);
      hipLaunchKernelGGL((k_gemm<T, MODE, GEN, 128, 256, 16, 64, 32>), grid, dim3(1024), 0, st, L);
    } else if (tier == kTierMedium) {
      dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 128), count);
      hipLaunchKernelGGL((k_gemm<T, MODE, GEN, 128, 128, 32, 32, 32>), grid, dim3(1024), 0, st, L);
    } else if (tier == kTierTiny) {
      dim3 grid(1, count);
      hipLaunchKernelGGL((k_gemm<T, MODE, GEN, 32, 32, 16, 16, 16>), grid, dim3(256), 0, st, L);
    } else {
      dim3 grid(cdiv(max_m, 64) * cdiv(max_n, 64), count);
      hipLaunchKernelGGL((k_gemm<T, MODE, GEN, 64, 64, 64, 16, 16>), grid, dim3(1024), 0, st, L);
    }
    return hipGetLastError();
  }
  dim3 grid(cdiv(max_m, 64) * cdiv(max_n, 64), count);
  hipLaunchKernelGGL((k_gemm<T, MODE, GEN, 64, 64, 16, 32, 32>), grid, dim3(256), 0, st, L);
  return hipGetLastError();
}

// Products of the recursive LU: every operand is a stored block at a
// multiple of 32 rows and columns of a b x b matrix (b even), so FP64 items
// all qualify for the direct-to-LDS instance (shapes as for explicit items);
// the 32 x 32 products of the lowest level and FP32 take the register-staged
// kernel.
template <typename T, int MODE>
hipError_t launch_gemm_rlu(const GemmLaunch& L, int max_m, int max_n, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    // Split FP16 recursion (mixed FP16 path): the vectorised instance from
    // halves of order 128 on (n = 16384, k = 8: its factorisations 2.27 s ->
    // 1.50 s per call).  BF16 keeps FP32 products here: its six-product
    // instance holds too many registers to run faster than them.
    if (L.lp == 1 && max_m >= 128 && max_n >= 128) {
      const int64_t tiles256 = static_cast<int64_t>(cdiv(max_m, 256)) * cdiv(max_n, 128) * L.count;
      if (tiles256 >= 256) {
        dim3 grid(cdiv(max_m, 256) * cdiv(max_n, 128), L.count);
        hipLaunchKernelGGL((k_gemm_lpv<1, MODE, 256, 128, 64, 64>), grid, dim3(512), 0, st, L);
      } else {
        dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 128), L.count);
        hipLaunchKernelGGL((k_gemm_lpv<1, MODE, 128, 128, 64, 64>), grid, dim3(256), 0, st, L);
      }
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(T) == 8) {
    const int tier = gemm_tier(L, MODE, L.count, max_m, max_n);
    if (tier == kTierSmall) {
      dim3 grid(cdiv(max_m, 64) * cdiv(max_n, 64), L.count);
      hipLaunchKernelGGL((k_gemm_dl<MODE, 64, 64, 32, 32>), grid, dim3(256), 0, st, L);
      return hipGetLastError();
    }
    if (tier != kTierTiny) {
      // Halves of order >= 1024 in launches of >= 512 tiles of 256 x 128:
      // tiles of 8 wavefronts of 64 x 64, as for the explicit products, one
      // launch per part of the node: 128 x 256 for the part whose triangular
      // operand is A (its K range ends with the tile's last row, so the
      // shorter side sits on the diagonal), 256 x 128 for the other (a full
      // product, or a triangular B whose K range follows the columns).
      // (n = 16384, k = 8: -1.9 ms per factorisation launch group at h =
      // 1024; at h = 512 the two launches took 8% longer than one of 128 x
      // 128 tiles.)
      const int64_t tiles256 = static_cast<int64_t>(cdiv(max_m, 256)) * cdiv(max_n, 128) * L.count;
      if (max_m >= 1024 && max_n >= 1024 && tiles256 >= 512) {
        if constexpr (MODE == GEMM_RLU_D) {
          dim3 grid(cdiv(max_m, 256) * cdiv(max_n, 128), L.count);
          hipLaunchKernelGGL((k_gemm_dl<MODE, 256, 128, 64, 64>), grid, dim3(512), 0, st, L);
        } else {
          // Part with the triangular A: the first for A (L11^{-1} P1 A12)
          // and C (L22^{-1} P2 L21), the second for B (U11^{-1} U12).
          constexpr int tri_a = MODE == GEMM_RLU_B ? 2 : 1;
          GemmLaunch F = L;
          F.count = L.count / 2;
          F.part = tri_a;
          dim3 gw(cdiv(max_m, 128) * cdiv(max_n, 256), F.count);
          hipLaunchKernelGGL((k_gemm_dl<MODE, 128, 256, 64, 64>), gw, dim3(512), 0, st, F);
          F.part = 3 - tri_a;
          dim3 gt(cdiv(max_m, 256) * cdiv(max_n, 128), F.count);
          hipLaunchKernelGGL((k_gemm_dl<MODE, 256, 128, 64, 64>), gt, dim3(512), 0, st, F);
        }
        return hipGetLastError();
      }
      dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 128), L.count);
      hipLaunchKernelGGL((k_gemm_dl<MODE, 128, 128, 32, 32>), grid, dim3(1024), 0, st, L);
      return hipGetLastError();
    }
  }
  // The smaller levels take the register-staged FP64 / FP32 instance (the
  // register-staged split instance stages row permutations for explicit
  // items only).
  GemmLaunch F = L;
  F.lp = 0;
  return launch_gemm_mode<T, MODE, false>(F, F.count, max_m, max_n, st);
}

template <typename T>
hipError_t launch_gemm(const GemmLaunch& L, int max_m, int max_n, hipStream_t st) {
  if (L.count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  switch (L.mode) {
    case GEMM_EXPLICIT: {
      // items [0, L.w) take the fast instance, [L.w, L.count) the generic one
      // (GemmLaunch::w carries the split; a launch takes items from
      // GemmLaunch::j on).  Except for the 32 x 32 shape, FP64 fast items
      // take the direct-to-LDS instance instead when all of them qualify
      // (L.ndl == L.w).
      const int nfast = L.w;
      int ndl = 0;
      if constexpr (sizeof(T) == 8) {
        // Only when every fast item qualifies: a second launch for the rest
        // would cost more than the direct instance gains (merged batches).
        const int tier = gemm_tier(L, GEMM_EXPLICIT, nfast, max_m, max_n);
        if (nfast > 0 && L.ndl == nfast && tier != kTierTiny) {
          // 128 x 128 tiles of 16 wavefronts of 32 x 32 for the two larger
          // shapes, 64 x 64 tiles of 4 wavefronts of 32 x 32 for the small
          // one; launches of at least 512 tiles of 256 x 128 take tiles of 8
          // wavefronts of 64 x 64, which read a quarter fewer operand bytes
          // per flop: 256 x 128 for full products, 128 x 256 for triangular
          // ones (the triangular operand is always A here, and a tile's K
          // range ends with its last row: half the overhang past the
          // diagonal).  These are the shapes the autotuner picks on the
          // MI355X in every such case it measures.
          ndl = nfast;
          int shape = tier == kTierSmall ? kShapeDl64 : kShapeDl128;
          const int64_t tiles256 = static_cast<int64_t>(cdiv(max_m, 256)) * cdiv(max_n, 128) * ndl;
          if (tier != kTierSmall && tiles256 >= 512) shape = L.tri == 0 ? kShapeDl256 : kShapeDl128w;
          const int tuned = tuned_product_shape(8, L.tri, ndl, max_m, max_n);
          if (tuned >= kShapeDl128 && tuned <= kShapeDl128w) shape = tuned;
          if (g_force_shape >= kShapeDl128 && g_force_shape <= kShapeDl128w) shape = g_force_shape;
          if (shape == kShapeDl64) {
            dim3 grid(cdiv(max_m, 64) * cdiv(max_n, 64), ndl);
            hipLaunchKernelGGL((k_gemm_dl<GEMM_EXPLICIT, 64, 64, 32, 32>), grid, dim3(256), 0, st, L);
          } else if (shape == kShapeDl128w) {
            dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 256), ndl);
            hipLaunchKernelGGL((k_gemm_dl<GEMM_EXPLICIT, 128, 256, 64, 64>), grid, dim3(512), 0, st, L);
          } else if (shape == kShapeDl256) {
            dim3 grid(cdiv(max_m, 256) * cdiv(max_n, 128), ndl);
            hipLaunchKernelGGL((k_gemm_dl<GEMM_EXPLICIT, 256, 128, 64, 64>), grid, dim3(512), 0, st, L);
          } else {
            dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 128), ndl);
            hipLaunchKernelGGL((k_gemm_dl<GEMM_EXPLICIT, 128, 128, 32, 32>), grid, dim3(1024), 0, st, L);
          }
          hipError_t e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
      } else {
        // Split products of float storage, when every fast item qualifies
        // (GemmLaunch::ndl).  Launches of fewer than 256 tiles of 256 x 128
        // keep the register-staged instance's smaller tiles (more
        // workgroups).
        const int64_t tiles256 = static_cast<int64_t>(cdiv(max_m, 256)) * cdiv(max_n, 128) * nfast;
        if (L.lp >= 1 && nfast > 0 && L.ndl == nfast && tiles256 >= 256) {
          // Launches of at least 2048 such tiles, with split scratch: the
          // operands split once (k_split_ops), then the products of the
          // planes (k_gemm_split), as many items at a time as the scratch
          // holds (n = 16384, k = 8: 32768 tiles per launch).  Otherwise FP16
          // takes the vectorised instance and BF16 the register-staged one
          // (below): at n = 4096, k = 4 (512 tiles) the split pass made the
          // mixed FP16 / BF16 calls 16% / 28% slower.
          const int parts = L.lp == 1 ? 2 : 3;
          const int kp = split_pitch(max(L.max_k, max(max_m, max_n)));
          const int64_t per = split_item_bytes(max_m, max_n, kp, parts);
          const int chunk = L.split && tiles256 >= 2048
                                ? static_cast<int>(std::min<int64_t>(nfast, L.split_bytes / per))
                                : 0;
          if (chunk > 0) {
            ndl = nfast;
            for (int c0 = 0; c0 < ndl; c0 += chunk) {
              GemmLaunch S = L;
              S.items = static_cast<const GemmItem*>(L.items) + c0;
              S.split_kp = kp;
              S.split_m = max_m;
              S.split_n = max_n;
              const int cn = min(chunk, ndl - c0);
              dim3 gs((cdiv(max_m, 64) + cdiv(max_n, 64)) * (kp / 64), cn);
              if (L.lp == 1) {
                constexpr int BM = SplitShape<1>::BM, BN = SplitShape<1>::BN;
                hipLaunchKernelGGL(k_split_ops<1>, gs, dim3(256), 0, st, S);
                dim3 grid(cdiv(max_m, BM) * cdiv(max_n, BN), cn);
                hipLaunchKernelGGL((k_gemm_split<1, BM, BN>), grid, dim3((BM / 64) * (BN / 64) * 64), 0, st, S);
              } else {
                constexpr int BM = SplitShape<2>::BM, BN = SplitShape<2>::BN;
                hipLaunchKernelGGL(k_split_ops<2>, gs, dim3(256), 0, st, S);
                dim3 grid(cdiv(max_m, BM) * cdiv(max_n, BN), cn);
                hipLaunchKernelGGL((k_gemm_split<2, BM, BN>), grid, dim3((BM / 64) * (BN / 64) * 64), 0, st, S);
              }
            }
          } else if (L.lp == 1) {
            ndl = nfast;
            dim3 grid(cdiv(max_m, 256) * cdiv(max_n, 128), ndl);
            hipLaunchKernelGGL((k_gemm_lpv<1, GEMM_EXPLICIT, 256, 128, 64, 64>), grid, dim3(512), 0, st, L);
          }
          hipError_t e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
      }
      GemmLaunch F = L;
      F.j = ndl;
      hipError_t e = launch_gemm_mode<T, GEMM_EXPLICIT, false>(F, nfast - ndl, max_m, max_n, st);
      if (e != hipSuccess) return e;
      GemmLaunch G = L;
      G.j = nfast;
      return launch_gemm_mode<T, GEMM_EXPLICIT, true>(G, L.count - nfast, max_m, max_n, st);
    }
    case GEMM_LU_TRAILING:
      return launch_gemm_mode<T, GEMM_LU_TRAILING, false>(L, L.count, max_m, max_n, st);
    case GEMM_TRTRI_STEP1:
      return launch_gemm_mode<T, GEMM_TRTRI_STEP1, false>(L, L.count, max_m, max_n, st);
    case GEMM_RLU_A:
      return launch_gemm_rlu<T, GEMM_RLU_A>(L, max_m, max_n, st);
    case GEMM_RLU_B:
      return launch_gemm_rlu<T, GEMM_RLU_B>(L, max_m, max_n, st);
    case GEMM_RLU_C:
      return launch_gemm_rlu<T, GEMM_RLU_C>(L, max_m, max_n, st);
    case GEMM_RLU_D:
      return launch_gemm_rlu<T, GEMM_RLU_D>(L, max_m, max_n, st);
    default:
      return launch_gemm_mode<T, GEMM_TRTRI_STEP2, false>(L, L.count, max_m, max_n, st);
  }
}

template <typename T, typename C>
hipError_t launch_getrf_tile_c(const LuItem* d_items, int count, int b, hipStream_t st) {
  hipLaunchKernelGGL((k_lu_amax<T>), dim3(kAmaxParts, count), dim3(256), 0, st, d_items);
  // Tile 0, then one launch per diagonal tile (k_lu_step): the launch of tile
  // s factors tile s + 1, so consecutive launches form the critical path.
  hipLaunchKernelGGL((k_tile_lu<T, C>), dim3(count), dim3(64), 0, st, d_items, 0);
  for (int t0 = 0; t0 < b; t0 += kTile) {
    const int grid = StepShape(b, t0).total();
    if (grid > 0) hipLaunchKernelGGL((k_lu_step<T, C>), dim3(grid, count), dim3(256), 0, st, d_items, t0);
  }
  hipLaunchKernelGGL(k_lu_check, dim3(count), dim3(64), 0, st, d_items);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_getrf_tile(const LuItem* d_items, int count, int b, bool wide, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (wide) return launch_getrf_tile_c<float, double>(d_items, count, b, st);
  }
  return launch_getrf_tile_c<T, T>(d_items, count, b, st);
}

// Recursive LU with inverted factors.  For a node of order 2h at origin o,
// with P1 A11 = L11 U11 and P2 S = L22 U22 (S = A22 - L21 U12 the Schur
// complement of the first half):
//   U12 = L11^{-1} P1 A12,  L21 = A21 U11^{-1},  S = A22 - L21 U12,
//   L^{-1} = [[L11^{-1}, 0], [-L22^{-1} P2 L21 L11^{-1}, L22^{-1}]],
//   U^{-1} = [[U11^{-1}, -U11^{-1} U12 U22^{-1}], [0, U22^{-1}]],
// and P = diag(P1, P2).  Every step is a product on MFMA; the recursion ends
// at kTile x kTile diagonal tiles factored (pivoting inside the tile) and
// inverted by one wavefront.  The result is the packed form the triangular
// inversion would leave (L^{-1} below the diagonal, U^{-1} on and above it)
// together with perm, so no triangular inversion follows.  Needs b =
// kTile * 2^m and a b x b shadow in LuItem::tmp.
template <typename T, typename C>
hipError_t getrf_rec_node(const LuItem* d_items, int count, int o, int n, int lp, int32_t* range_flag,
                          hipStream_t st) {
  if (n <= kTile) {
    hipLaunchKernelGGL((k_tile_lu_inv<T, C>), dim3(count), dim3(64), 0, st, d_items, o);
    return hipGetLastError();
  }
  const int h = n / 2;
  hipError_t e = getrf_rec_node<T, C>(d_items, count, o, h, lp, range_flag, st);
  if (e != hipSuccess) return e;
  GemmLaunch L{};
  L.elem = sizeof(T);
  L.lp = lp;
  L.range_flag = range_flag;
  L.items = d_items;
  L.j = o;
  L.s = h;
  L.tri = 1;
  L.count = 2 * count;
  L.mode = GEMM_RLU_A;
  if ((e = launch_gemm<T>(L, h, h, st)) != hipSuccess) return e;
  L.mode = GEMM_RLU_B;
  if ((e = launch_gemm<T>(L, h, h, st)) != hipSuccess) return e;
  if ((e = getrf_rec_node<T, C>(d_items, count, o + h, h, lp, range_flag, st)) != hipSuccess) return e;
  L.mode = GEMM_RLU_C;
  if ((e = launch_gemm<T>(L, h, h, st)) != hipSuccess) return e;
  L.mode = GEMM_RLU_D;
  L.count = count;
  return launch_gemm<T>(L, h, h, st);
}

template <typename T>
hipError_t launch_getrf_rec(const LuItem* d_items, int count, int b, bool wide, int lp, int32_t* range_flag,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_lu_amax<T>), dim3(kAmaxParts, count), dim3(256), 0, st, d_items);
  hipError_t e;
  if (sizeof(T) == 4 && wide)
    e = getrf_rec_node<T, double>(d_items, count, 0, b, lp, range_flag, st);
  else
    e = getrf_rec_node<T, T>(d_items, count, 0, b, lp, range_flag, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lu_check, dim3(count), dim3(64), 0, st, d_items);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_getrf(const LuItem* d_items, int count, int b, hipStream_t st) {
  for (int j = 0; j < b;) {
    const int h = b - j;
    const int nb = panel_width(h);
    const int w = nb < h ? nb : h;
    if (h <= 512) {
      hipLaunchKernelGGL((k_getf2<T, 32, 1>), dim3(count), dim3(512), 0, st, d_items, j);
    } else if (h <= 1024) {
      hipLaunchKernelGGL((k_getf2<T, 32, 2>), dim3(count), dim3(512), 0, st, d_items, j);
    } else if (h <= 2048) {
      hipLaunchKernelGGL((k_getf2<T, 16, 4>), dim3(count), dim3(512), 0, st, d_items, j);
    } else {
      hipLaunchKernelGGL((k_getf2<T, 8, 8>), dim3(count), dim3(512), 0, st, d_items, j);
    }
    if (j > 0 || j + w < b) {
      dim3 grid(cdiv(b, 128), count);
      if (nb == 32)
        hipLaunchKernelGGL((k_laswp_trsm<T, 32>), grid, dim3(128), 0, st, d_items, j, w);
      else if (nb == 16)
        hipLaunchKernelGGL((k_laswp_trsm<T, 16>), grid, dim3(128), 0, st, d_items, j, w);
      else
        hipLaunchKernelGGL((k_laswp_trsm<T, 8>), grid, dim3(128), 0, st, d_items, j, w);
    }
    if (j + w < b) {
      GemmLaunch L{};
      L.mode = GEMM_LU_TRAILING;
      L.elem = sizeof(T);
      L.items = d_items;
      L.count = count;
      L.j = j;
      L.w = w;
      hipError_t e = launch_gemm<T>(L, b - j - w, b - j - w, st);
      if (e != hipSuccess) return e;
    }
    j += w;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trtri(const LuItem* d_items, int count, int b, bool diag_inverted, hipStream_t st) {
  // The tile-pivoting LU leaves the inverses of its 32 x 32 diagonal tiles in
  // place; after the partial-pivoting LU they are formed here.
  if (!diag_inverted)
    hipLaunchKernelGGL((k_trtri_diag<T, kTrtriTile>), dim3(cdiv(b, kTrtriTile), count), dim3(128), 0, st, d_items);
  for (int s = kTrtriTile; s < b; s *= 2) {
    const int npairs = cdiv(b - s, 2 * s);
    GemmLaunch L{};
    L.elem = sizeof(T);
    L.items = d_items;
    L.count = count * npairs * 2;
    L.s = s;
    L.npairs = npairs;
    L.mode = GEMM_TRTRI_STEP1;
    hipError_t e = launch_gemm<T>(L, s, s, st);
    if (e != hipSuccess) return e;
    L.mode = GEMM_TRTRI_STEP2;
    e = launch_gemm<T>(L, s, s, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_load(const LoadItem* d_items, int count, int rows, int cols, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(rows) * cols;
  int gx = cdiv(total, 256);
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL((k_load<T>), dim3(gx, count), dim3(256), 0, st, d_items);
  return hipGetLastError();
}

// Fills every matrix of the LU items with a diagonally dominant pattern
// (entries in [-0.5, 0.5) from an integer hash, b added on the diagonal):
// inputs for the autotuner's factorisation timings.
__global__ __launch_bounds__(256) void k_fill_diag_dominant(const LuItem* items) {
  const LuItem it = items[blockIdx.y];
  double* a = static_cast<double*>(it.a);
  const int64_t n = static_cast<int64_t>(it.b) * it.b;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < n; e += static_cast<int64_t>(gridDim.x) * 256) {
    uint32_t h = static_cast<uint32_t>(e) * 2654435761u ^ (blockIdx.y * 40503u + 0x9e3779b9u);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    const int64_t r = e / it.b, c = e % it.b;
    a[e] = static_cast<double>(h) * (1.0 / 4294967296.0) - 0.5 + (r == c ? static_cast<double>(it.b) : 0.0);
  }
}

hipError_t launch_fill_diag_dominant(const LuItem* d_items, int count, int b, hipStream_t st) {
  int gx = cdiv(static_cast<int64_t>(b) * b, 256);
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_fill_diag_dominant, dim3(gx, count), dim3(256), 0, st, d_items);
  return hipGetLastError();
}

__global__ void k_store_rbf(RbfSource* dst, RbfSource src) {
  if (threadIdx.x == 0) *dst = src;
}

hipError_t launch_store_rbf(RbfSource* dst, const RbfSource& src, hipStream_t st) {
  hipLaunchKernelGGL(k_store_rbf, dim3(1), dim3(64), 0, st, dst, src);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device accounting of executed plan steps (optional, bri_opts::d_stats):
// one thread per item of a step that has just run reads the item's
// descriptor (the one its kernels ran on) and counts it, and records the end
// of the workspace bytes it wrote (highest offset below the workspace size).
// stats[0] pivot factorisations, stats[1] Schur products D - C X (plain and
// accumulated), stats[2] other products (triangular multiplies, final
// products), stats[3] workspace high-water mark in bytes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stats_note_end(unsigned long long* stats, const char* base, uint64_t limit,
                                               const void* p, uint64_t bytes) {
  const char* q = static_cast<const char*>(p);
  if (q < base) return;
  const uint64_t end = static_cast<uint64_t>(q - base) + bytes;
  if (end <= limit) atomicMax(stats + 3, static_cast<unsigned long long>(end));
}

__global__ void k_stats_lu(const LuItem* items, int count, int elem, int factorisation, unsigned long long* stats,
                           const char* base, uint64_t limit) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const LuItem it = items[t];
  const uint64_t bytes = static_cast<uint64_t>(it.b) * it.b * elem;
  if (factorisation) atomicAdd(stats + 0, 1ull);
  stats_note_end(stats, base, limit, it.a, bytes);
  if (it.tmp) stats_note_end(stats, base, limit, it.tmp, bytes);
}

__global__ void k_stats_gemm(const GemmItem* items, int count, int which, int elem, unsigned long long* stats,
                             const char* base, uint64_t limit) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const GemmItem it = items[t];
  atomicAdd(stats + which, 1ull);
  if (it.M > 0 && it.N > 0)
    stats_note_end(stats, base, limit, it.out,
                   (static_cast<uint64_t>(it.M - 1) * it.ldo + it.N) * static_cast<uint64_t>(elem));
}

__global__ void k_stats_load(const LoadItem* items, int count, int elem, unsigned long long* stats, const char* base,
                             uint64_t limit) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const LoadItem it = items[t];
  if (it.rows > 0 && it.cols > 0)
    stats_note_end(stats, base, limit, it.dst,
                   (static_cast<uint64_t>(it.rows - 1) * it.ldd + it.cols) * static_cast<uint64_t>(elem));
}

hipError_t launch_stats(int kind, const void* items, int count, int elem, unsigned long long* stats,
                        const void* base, uint64_t limit, hipStream_t st) {
  if (count <= 0 || !stats) return hipSuccess;
  const dim3 grid(cdiv(count, 256)), block(256);
  const char* b = static_cast<const char*>(base);
  if (kind == ST_LOAD) {
    hipLaunchKernelGGL(k_stats_load, grid, block, 0, st, static_cast<const LoadItem*>(items), count, elem, stats, b,
                       limit);
  } else if (kind == ST_GETRF || kind == ST_TRTRI) {
    // the triangular inversion writes the LU block and its scratch block
    hipLaunchKernelGGL(k_stats_lu, grid, block, 0, st, static_cast<const LuItem*>(items), count, elem,
                       kind == ST_GETRF ? 1 : 0, stats, b, limit);
  } else {
    const int which = (kind == ST_GEMM || kind == ST_GEMM_ACC) ? 1 : 2;
    hipLaunchKernelGGL(k_stats_gemm, grid, block, 0, st, static_cast<const GemmItem*>(items), count, which, elem,
                       stats, b, limit);
  }
  return hipGetLastError();
}

hipError_t launch_fill_int(int32_t* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmLaunch&, int, int, hipStream_t);
template hipError_t launch_gemm<float>(const GemmLaunch&, int, int, hipStream_t);
template hipError_t launch_getrf<double>(const LuItem*, int, int, hipStream_t);
template hipError_t launch_getrf_tile<double>(const LuItem*, int, int, bool, hipStream_t);
template hipError_t launch_getrf_rec<double>(const LuItem*, int, int, bool, int, int32_t*, hipStream_t);
template hipError_t launch_getrf_rec<float>(const LuItem*, int, int, bool, int, int32_t*, hipStream_t);
template hipError_t launch_getrf_tile<float>(const LuItem*, int, int, bool, hipStream_t);
template hipError_t launch_getrf<float>(const LuItem*, int, int, hipStream_t);
template hipError_t launch_trtri<double>(const LuItem*, int, int, bool, hipStream_t);
template hipError_t launch_trtri<float>(const LuItem*, int, int, bool, hipStream_t);
template hipError_t launch_load<double>(const LoadItem*, int, int, int, hipStream_t);
template hipError_t launch_load<float>(const LoadItem*, int, int, int, hipStream_t);

}  // namespace bri
