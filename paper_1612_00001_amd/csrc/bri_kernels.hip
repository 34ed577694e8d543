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
template <typename T>
__device__ __forceinline__ T vget(const DView& v, int x, int y) {
  if (v.tri == 1) {
    if (x == y) return T(1);
    if (x < y) return T(0);
  } else if (v.tri == 2) {
    if (x > y) return T(0);
  }
  const int xs = v.rowperm ? v.rowperm[x] : x;
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
// Batched MFMA GEMM.  One workgroup computes a BM x BN output tile with
// (BM/WM) x (BN/WN) wavefronts of WM x WN each; K is consumed BK at a time
// through double-buffered LDS tiles stored k-major (As[k][m], Bs[k][n]) so
// that every MFMA operand fetch reads 16 consecutive LDS words.
// ---------------------------------------------------------------------------
// MODE selects how the work items are formed (GemmMode); every mode is its
// own kernel instance so that profiles separate the Schur products from the
// LU and triangular-inversion updates.
template <typename T, int MODE, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm(GemmLaunch L) {
  constexpr int NWN = BN / WN;
  constexpr int NT = (BM / WM) * NWN * 64;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int AE = BM * BK / NT, BE = BK * BN / NT;
  static_assert(AE * NT == BM * BK && BE * NT == BK * BN, "tile/thread mismatch");

  GemmItem it;
  if (!gemm_item<T, MODE>(L, blockIdx.y, it)) return;
  const int tiles_n = (it.N + BN - 1) / BN;
  const int tiles_m = (it.M + BM - 1) / BM;
  if (static_cast<int>(blockIdx.x) >= tiles_m * tiles_n) return;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  int kb = 0, ke = it.K;
  if (it.A.tri == 1) ke = min(ke, m0 + BM);
  if (it.A.tri == 2) kb = max(kb, m0);
  if (it.B.tri == 1) kb = max(kb, n0);
  if (it.B.tri == 2) ke = min(ke, n0 + BN);
  kb = (kb / BK) * BK;

  __shared__ T As[2][BK][BM + 1];
  __shared__ T Bs[2][BK][BN + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  typename MF<T>::acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  T ra[AE], rb[BE];
  const bool a_plain = it.A.tri == 0 && it.A.rowperm == nullptr;
  const bool b_plain = it.B.tri == 0 && it.B.rowperm == nullptr;

  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < AE; ++t) {
      const int e = tid + t * NT;
      const int x = it.A.trans ? e % BM : e / BK;
      const int y = it.A.trans ? e / BM : e % BK;
      const int gx = m0 + x, gy = k0 + y;
      T v = T(0);
      if (gx < it.M && gy < it.K) {
        if (a_plain && gx < it.A.rows && gy < it.A.cols) {
          const T* p = static_cast<const T*>(it.A.p);
          v = it.A.trans ? p[static_cast<int64_t>(gy) * it.A.ld + gx] : p[static_cast<int64_t>(gx) * it.A.ld + gy];
        } else {
          v = vget<T>(it.A, gx, gy);
        }
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < BE; ++t) {
      const int e = tid + t * NT;
      const int x = it.B.trans ? e % BK : e / BN;
      const int y = it.B.trans ? e / BK : e % BN;
      const int gx = k0 + x, gy = n0 + y;
      T v = T(0);
      if (gx < it.K && gy < it.N) {
        if (b_plain && gx < it.B.rows && gy < it.B.cols) {
          const T* p = static_cast<const T*>(it.B.p);
          v = it.B.trans ? p[static_cast<int64_t>(gy) * it.B.ld + gx] : p[static_cast<int64_t>(gx) * it.B.ld + gy];
        } else {
          v = vget<T>(it.B, gx, gy);
        }
      }
      rb[t] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < AE; ++t) {
      const int e = tid + t * NT;
      const int x = it.A.trans ? e % BM : e / BK;
      const int y = it.A.trans ? e / BM : e % BK;
      As[buf][y][x] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < BE; ++t) {
      const int e = tid + t * NT;
      const int x = it.B.trans ? e % BK : e / BN;
      const int y = it.B.trans ? e / BK : e % BN;
      Bs[buf][x][y] = rb[t];
    }
  };

  if (kb < ke) {
    load(kb);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) load(k0 + BK);
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
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  T* out = static_cast<T*>(it.out);
  const T alpha = static_cast<T>(it.alpha), beta = static_cast<T>(it.beta);
#pragma unroll
  for (int i = 0; i < FM; ++i)
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
}

// ---------------------------------------------------------------------------
// Panel LU with partial pivoting.  Rows j..b-1, columns j..j+w-1 of one
// matrix live in registers: thread t owns panel rows t + 512 q (q < R).  For
// every column the workgroup finds the row of largest magnitude (lowest index
// on ties, as LAPACK's idamax), exchanges it with the current row through
// LDS, scales the multipliers and updates the rest of the panel.  The
// composite row movement is recorded as (dest, src) pairs for k_laswp_trsm,
// and the running permutation of the matrix is composed in it.perm.
// Columns are unrolled at compile time (panel_step<C>) so that every register
// index is static.
// ---------------------------------------------------------------------------
template <typename T, int NB>
struct PanelShared {
  T rowp[NB], rowc[NB];
  int origp, origc;
  T redv[8];
  int redi[8];
  int cnt;
};

template <typename T, int NB, int R, int C>
__device__ __forceinline__ void panel_step(T (&a)[R][NB], int (&orig)[R], PanelShared<T, NB>& sh, int h, int w,
                                           int tid, int32_t* info, int node) {
  constexpr int NT = 512;
  if (C >= w) return;
  const int lane = tid & 63, wave = tid >> 6;
  T best = T(-1);
  int bi = INT_MAX;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr >= C && lr < h) {
      const T v = fabs(a[q][C]);
      if (v > best) {
        best = v;
        bi = lr;
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    sh.redv[wave] = best;
    sh.redi[wave] = bi;
  }
  __syncthreads();
  best = sh.redv[0];
  bi = sh.redi[0];
#pragma unroll
  for (int wv = 1; wv < NT / 64; ++wv) {
    const T ov = sh.redv[wv];
    const int oi = sh.redi[wv];
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  const int p = (bi == INT_MAX) ? C : bi;  // an all-NaN column keeps its row
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr == p) {
#pragma unroll
      for (int cc = C; cc < NB; ++cc) sh.rowp[cc] = a[q][cc];
      sh.origp = orig[q];
    }
    if (lr == C) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) sh.rowc[cc] = a[q][cc];
      sh.origc = orig[q];
    }
  }
  // The pivot row's multipliers (columns < C) must travel with it as well.
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr == p) {
#pragma unroll
      for (int cc = 0; cc < C; ++cc) sh.rowp[cc] = a[q][cc];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * NT;
    if (lr == C) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) a[q][cc] = sh.rowp[cc];
      orig[q] = sh.origp;
    } else if (lr == p) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) a[q][cc] = sh.rowc[cc];
      orig[q] = sh.origc;
    }
  }
  const T piv = sh.rowp[C];
  if (!(piv != T(0) && isfinite(piv)) && tid == 0 && info) atomicCAS(info, 0, node + 1);
  if (piv != T(0)) {
    const T rinv = T(1) / piv;
    T l[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * NT;
      const bool below = lr > C && lr < h;
      l[q] = below ? a[q][C] * rinv : T(0);
      if (below) a[q][C] = l[q];
    }
#pragma unroll
    for (int cc = C + 1; cc < NB; ++cc) {
      const T pv = sh.rowp[cc];
#pragma unroll
      for (int q = 0; q < R; ++q) a[q][cc] -= l[q] * pv;
    }
  }
  __syncthreads();
}

template <typename T, int NB, int R, int... Cs>
__device__ __forceinline__ void panel_all(std::integer_sequence<int, Cs...>, T (&a)[R][NB], int (&orig)[R],
                                          PanelShared<T, NB>& sh, int h, int w, int tid, int32_t* info, int node) {
  (panel_step<T, NB, R, Cs>(a, orig, sh, h, w, tid, info, node), ...);
}

template <typename T, int NB, int R>
__global__ __launch_bounds__(512) void k_getf2(const LuItem* items, int j, int32_t* info) {
  constexpr int NT = 512;
  const LuItem it = items[blockIdx.x];
  T* A = static_cast<T*>(it.a);
  const int b = it.b, h = b - j, w = min(NB, h);
  const int tid = threadIdx.x;
  __shared__ PanelShared<T, NB> sh;

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
  panel_all<T, NB, R>(std::make_integer_sequence<int, NB>{}, a, orig, sh, h, w, tid, info, it.node);

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
    // Forward substitution with the unit-lower L11; column tid of s_rows is
    // this thread's private workspace.
    for (int r = 0; r < w; ++r) s_rows[r][tid] = A[static_cast<int64_t>(j + r) * b + col];
    for (int r = 1; r < w; ++r) {
      T acc = s_rows[r][tid];
      for (int q = 0; q < r; ++q) acc -= s_L[r][q] * s_rows[q][tid];
      s_rows[r][tid] = acc;
    }
    for (int r = 0; r < w; ++r) A[static_cast<int64_t>(j + r) * b + col] = s_rows[r][tid];
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

template <typename T, int MODE>
hipError_t launch_gemm_mode(const GemmLaunch& L, int max_m, int max_n, hipStream_t st) {
  const int64_t big_tiles = static_cast<int64_t>(cdiv(max_m, 128)) * cdiv(max_n, 128) * L.count;
  if (big_tiles >= 256) {
    dim3 grid(cdiv(max_m, 128) * cdiv(max_n, 128), L.count);
    hipLaunchKernelGGL((k_gemm<T, MODE, 128, 128, 16, 64, 64>), grid, dim3(256), 0, st, L);
  } else {
    dim3 grid(cdiv(max_m, 64) * cdiv(max_n, 64), L.count);
    hipLaunchKernelGGL((k_gemm<T, MODE, 64, 64, 16, 32, 32>), grid, dim3(256), 0, st, L);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm(const GemmLaunch& L, int max_m, int max_n, hipStream_t st) {
  if (L.count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  switch (L.mode) {
    case GEMM_EXPLICIT:
      return launch_gemm_mode<T, GEMM_EXPLICIT>(L, max_m, max_n, st);
    case GEMM_LU_TRAILING:
      return launch_gemm_mode<T, GEMM_LU_TRAILING>(L, max_m, max_n, st);
    case GEMM_TRTRI_STEP1:
      return launch_gemm_mode<T, GEMM_TRTRI_STEP1>(L, max_m, max_n, st);
    default:
      return launch_gemm_mode<T, GEMM_TRTRI_STEP2>(L, max_m, max_n, st);
  }
}

template <typename T>
hipError_t launch_getrf(const LuItem* d_items, int count, int b, int32_t* info, hipStream_t st) {
  for (int j = 0; j < b;) {
    const int h = b - j;
    const int nb = panel_width(h);
    const int w = nb < h ? nb : h;
    if (h <= 512) {
      hipLaunchKernelGGL((k_getf2<T, 32, 1>), dim3(count), dim3(512), 0, st, d_items, j, info);
    } else if (h <= 1024) {
      hipLaunchKernelGGL((k_getf2<T, 32, 2>), dim3(count), dim3(512), 0, st, d_items, j, info);
    } else if (h <= 2048) {
      hipLaunchKernelGGL((k_getf2<T, 16, 4>), dim3(count), dim3(512), 0, st, d_items, j, info);
    } else {
      hipLaunchKernelGGL((k_getf2<T, 8, 8>), dim3(count), dim3(512), 0, st, d_items, j, info);
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
hipError_t launch_trtri(const LuItem* d_items, int count, int b, hipStream_t st) {
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

hipError_t launch_fill_int(int32_t* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmLaunch&, int, int, hipStream_t);
template hipError_t launch_gemm<float>(const GemmLaunch&, int, int, hipStream_t);
template hipError_t launch_getrf<double>(const LuItem*, int, int, int32_t*, hipStream_t);
template hipError_t launch_getrf<float>(const LuItem*, int, int, int32_t*, hipStream_t);
template hipError_t launch_trtri<double>(const LuItem*, int, int, hipStream_t);
template hipError_t launch_trtri<float>(const LuItem*, int, int, hipStream_t);
template hipError_t launch_load<double>(const LoadItem*, int, int, int, hipStream_t);
template hipError_t launch_load<float>(const LoadItem*, int, int, int, hipStream_t);

}  // namespace bri
