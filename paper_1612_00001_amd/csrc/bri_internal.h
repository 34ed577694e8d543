// Internal types shared by the host planner, the executor and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace bri {

// ---------------------------------------------------------------------------
// Device-side operand view: element (x, y) of a b x b block.
//   - tri == 1: unit lower triangle of the stored data (x > y stored, x == y
//     reads 1, x < y reads 0); tri == 2: upper triangle (x <= y stored).
//   - rowperm: element (x, y) is the stored element (rowperm[x], y).
//   - Stored extent rows x cols; outside it the element is synthesised as
//     (x - y == diag) ? 1 : 0, which realises the identity padding of the
//     augmented matrix Gamma without a padded copy.
//   - trans: the stored element (x, y) lives at p[y * ld + x].
//   - src64_max: when set, the stored data are doubles and every element
//     (synthesised ones included) is multiplied by the power of two 2^-e
//     with max |M| 2^-e in [0.5, 1), max |M| being the double at src64_max
//     (the scaled matrix the mixed paths' float recursion works on).  Only
//     the block loads (k_load) read such views.
//   - rbf: when set, the elements inside the stored extent are not stored
//     but evaluated: element (x, y) is element (r0 + x, c0 + y) of the
//     matrix rbf describes (RbfSource), with (r0, c0) the view's origin.
//     Only the block loads read such views.
// ---------------------------------------------------------------------------
struct RbfSource;
struct DView {
  const void* p;
  int64_t ld;
  const int32_t* rowperm;
  int32_t rows, cols;
  int32_t diag;
  int16_t trans, tri;
  const double* src64_max;
  const RbfSource* rbf;
  int32_t r0, c0;
};

// The matrix A_gamma of the LS-SVM cross-validation (Section "Experimental
// results", eq. A), of order m = npts + 1, evaluated element by element from
// the data points x_1..x_npts (rows of X, npts x d, leading dimension ldx):
//   A(0, 0) = 0,  A(0, c) = A(c, 0) = 1,
//   A(r, c) = exp(-||x_r - x_c||^2 / (2 sigma^2)) + [r == c] / gamma   (r, c >= 1).
struct RbfSource {
  const void* X;        // double (or float for BRI_F32) data points
  int64_t ldx;
  int32_t npts, d;
  double inv_two_sigma2;  // 1 / (2 sigma^2)
  double inv_gamma;       // 1 / gamma
};

// out[x, y] = beta * Cin[x, y] + alpha * sum_t A[x, t] B[t, y] - Sub[x, y]
struct GemmItem {
  DView A, B, Cin, Sub;
  void* out;
  int64_t ldo;
  int32_t M, N, K;
  int32_t has_cin, has_sub, pad_;
  double alpha, beta;
  int32_t* umax;     // when set: the largest magnitude of the output goes here (element
                     // growth of the recursive LU, see kUmaxWord); null otherwise
};

// One b x b matrix factored in place (P A = L U, unit L strictly below the
// diagonal, U on and above), later overwritten by L^{-1} and U^{-1} in the
// same packed layout.
struct LuItem {
  void* a;           // dense b x b, leading dimension b
  int32_t* perm;     // b entries: row x of P A is row perm[x] of A
  int32_t* swaps;    // partial pivoting: per-panel list of moved rows [count, (dest, src) ...];
                     // tile pivoting: kStepBufs tile permutations of kTile entries after word 0
  void* tmp;         // b x b scratch for the triangular inversion
  void* aux;         // kAuxElems elements: inverses of the L and U factors of recent diagonal tiles
  int32_t* info;     // device status word of the problem this matrix belongs to (or null)
  int32_t node;      // Schur operation index reported through *info
  int32_t b;
};

// Tile of the tile-local pivoting LU: the pivot search of column c runs over
// the rows of the kTile x kTile diagonal tile that holds c.
constexpr int kTile = 32;
// The tile-step launch of tile s reads the factors of tiles s - 1 and s while
// it factors tile s + 1, so the tile inverses and permutations rotate through
// three buffers.
constexpr int kStepBufs = 3;
constexpr int kAuxElems = kStepBufs * 2 * kTile * kTile;

struct LoadItem {
  DView src;
  void* dst;
  int64_t ldd;
  int32_t rows, cols;
};

enum GemmMode : int32_t {
  GEMM_EXPLICIT = 0,    // items[] are GemmItem
  GEMM_LU_TRAILING = 1, // trailing update of a right-looking LU step
  GEMM_TRTRI_STEP1 = 2, // recursive-doubling triangular inversion, first product
  GEMM_TRTRI_STEP2 = 3, // second product
  // Recursive LU with inverted factors (launch_getrf_rec): the products of
  // one node (origin j, halves of order s) of the recursion, formed on the
  // device from the LuItem (a: the matrix, tmp: a b x b shadow of it).
  GEMM_RLU_A = 4,       // U12 = L11^{-1} P1 A12 and L21 = A21 U11^{-1}, into the shadow
  GEMM_RLU_B = 5,       // A22 -= L21 U12 and Y = U11^{-1} U12 (shadow)
  GEMM_RLU_C = 6,       // X = L22^{-1} P2 L21 (shadow) and A12 <- -Y U22^{-1}
  GEMM_RLU_D = 7,       // A21 <- -X L11^{-1}
};

struct GemmLaunch {
  int32_t mode;
  int32_t elem;         // 8 = double, 4 = float
  const void* items;    // GemmItem* or LuItem*
  int32_t count;        // items for GEMM_EXPLICIT, matrices otherwise
  int32_t j, w;         // LU step: panel start and width.  GEMM_EXPLICIT:
                        // w = number of leading items the fast instance
                        // takes (see gemm_item_is_fast), j = item offset
  int32_t s;            // TRTRI level: half-block size
  int32_t npairs;       // TRTRI level: block pairs per matrix
  int32_t lp;           // float storage only: 0 FP32 MFMA, 1 FP16 split, 2 BF16 split
  int32_t tri;          // items have a triangular operand (uneven K per output tile)
  int32_t ndl;          // GEMM_EXPLICIT: the first ndl fast items also qualify for
                        // the direct-to-LDS FP64 instance (gemm_item_is_direct)
  int32_t* range_flag;  // FP16 split products: set to 1 when an operand value lies
                        // outside the FP16 range (or is not finite); may be null
  int32_t part;         // recursive LU modes: 0 = every part of each node (count =
                        // matrices x parts), 1 / 2 = only the first / second part
                        // (count = matrices)
  // FP16 split products of float storage (GEMM_EXPLICIT): scratch for the
  // operands split once before the product (split_item_bytes per item), or
  // null; the launch then takes as many items at a time as it holds.
  void* split;
  int64_t split_bytes;
  int32_t max_k;                       // largest inner order K of the items (0: at most
                                       // max(max_m, max_n), as for block products)
  int32_t split_kp, split_m, split_n;  // set by the launch: K pitch, A rows, B columns
};

// Bytes of one item's pre-split operands: the parts (2 FP16 or 3 BF16
// planes) of A (m rows) and of B transposed (n rows), kp elements per row.
constexpr int64_t split_item_bytes(int m, int n, int kp, int parts) {
  return 2 * static_cast<int64_t>(parts) * (m + n) * kp;
}
// The K pitch of the split operands of products of inner order up to k.
constexpr int split_pitch(int k) { return (k + 63) / 64 * 64; }

constexpr int kMaxBlock = 4096;  // == BRI_MAX_BLOCK

// True when every element the product reads from A and B is either stored
// (inside the view's stored extent) or synthesised without stored data, so
// the fast GEMM instance can stream the operands.
inline bool view_fast(const DView& v, int xlim, int ylim) {
  if (v.p == nullptr) return v.rows == 0;
  if (v.trans && v.rowperm) return false;
  const int need_rows = v.rowperm ? xlim : xlim;  // permuted rows are < xlim as well
  return need_rows <= v.rows && ylim <= v.cols;
}
// Plain: stored, untransposed, unpermuted, untriangular and covering M x N.
inline bool view_plain(const DView& v, int xlim, int ylim) {
  return v.p != nullptr && !v.trans && !v.rowperm && v.tri == 0 && xlim <= v.rows && ylim <= v.cols;
}
// Direct-to-LDS operand: stored, untransposed, covering the product, rows
// starting on 16-byte boundaries (the operand tiles move to LDS in 16-byte
// pieces, two FP64 elements each).
inline bool view_direct(const DView& v, int xlim, int ylim, int elem) {
  return v.p != nullptr && !v.trans && xlim <= v.rows && ylim <= v.cols &&
         reinterpret_cast<uintptr_t>(v.p) % 16 == 0 && (v.ld * elem) % 16 == 0;
}
// An item of the direct-to-LDS FP64 instance: A and B direct (a row
// permutation only on B, a triangular form only on A, the forms the
// explicit steps produce and the tests cover), even N and K (no 16-byte
// piece crosses the edge of an operand), plain Cin / Sub.
inline bool gemm_item_is_direct(const GemmItem& g, int elem) {
  return elem == 8 && g.M > 0 && g.N > 0 && g.K > 0 && g.N % 2 == 0 && g.K % 2 == 0 &&
         view_direct(g.A, g.M, g.K, elem) && g.A.rowperm == nullptr && view_direct(g.B, g.K, g.N, elem) &&
         g.B.tri == 0 &&
         (g.B.rowperm == nullptr || g.K <= kMaxBlock) &&
         (!g.has_cin || view_plain(g.Cin, g.M, g.N)) && (!g.has_sub || view_plain(g.Sub, g.M, g.N));
}
// An item of the vectorised split FP16 instance (float storage,
// k_gemm_lpv) and of the split pass (k_split_ops): A stored untransposed
// with 16-byte aligned rows, unpermuted, possibly triangular; B stored
// untransposed, untriangular, possibly with a row permutation; K a multiple
// of 8 (runs of eight k never cross it) and at most kMaxBlock; plain Cin /
// Sub; no element conversion or evaluation.
inline bool gemm_item_is_lp_vec(const GemmItem& g) {
  return g.M > 0 && g.N > 0 && g.K > 0 && g.K % 8 == 0 && g.K <= kMaxBlock &&
         view_direct(g.A, g.M, g.K, 4) && g.A.rowperm == nullptr && g.A.src64_max == nullptr && g.A.rbf == nullptr &&
         g.B.p != nullptr && !g.B.trans && g.B.tri == 0 && g.K <= g.B.rows && g.N <= g.B.cols &&
         g.B.src64_max == nullptr && g.B.rbf == nullptr &&
         (!g.has_cin || view_plain(g.Cin, g.M, g.N)) && (!g.has_sub || view_plain(g.Sub, g.M, g.N));
}
inline bool gemm_item_is_fast(const GemmItem& g) {
  return view_fast(g.A, g.M, g.K) && view_fast(g.B, g.K, g.N) && (!g.has_cin || view_plain(g.Cin, g.M, g.N)) &&
         (!g.has_sub || view_plain(g.Sub, g.M, g.N));
}

constexpr int kSwapWords = 1 + 2 * 2 * 64;  // count + up to 128 (dest, src) pairs
static_assert(1 + kStepBufs * kTile <= kSwapWords, "tile permutations exceed the swap words");
// Element growth of the tile-pivoting LUs, in the swap words they leave
// free: kAmaxParts partial maxima of |A| over bands of rows (taken before
// the factorisation) from word kAmaxWord on, and the largest |U| entry formed
// (float bits, updated by atomic maximum) in word kUmaxWord.  A
// factorisation whose largest |U| exceeds kGrowthLimit times the largest |A|
// is reported through info like a failed pivot (partial pivoting keeps this
// ratio near 10 on Gaussian matrices of these orders; SPD and diagonally
// dominant matrices keep it at most 1 and 2).
constexpr int kAmaxParts = 64;
constexpr int kAmaxWord = 128;
constexpr int kUmaxWord = kSwapWords - 1;
constexpr float kGrowthLimit = 64.0f;
static_assert(1 + kStepBufs * kTile <= kAmaxWord && kAmaxWord + kAmaxParts <= kUmaxWord, "growth words");
constexpr int kTrtriTile = 32;                // diagonal tile of the triangular inversion

// Width of the LU panel held in registers for a panel of h rows (512 threads
// hold ceil(h / 512) rows of at most 64 doubles each).
inline int panel_width(int h) { return h <= 1024 ? 32 : (h <= 2048 ? 16 : 8); }

// ---------------------------------------------------------------------------
// Host plan: batched steps over b x b workspace slots.
// ---------------------------------------------------------------------------
// OPND_RHS: block row a of the right-hand side of a solve plan (the extra
// block column k of the bordered matrix [Gamma | R]).
enum OpndKind : int8_t { OPND_NONE = 0, OPND_SLOT = 1, OPND_MBLK = 2, OPND_IDENT = 3, OPND_OUT = 4, OPND_RHS = 5 };

struct Opnd {
  int8_t kind = OPND_NONE;
  int32_t a = 0, b = 0;
  static Opnd none() { return Opnd(); }
  static Opnd slot(int s) { Opnd o; o.kind = OPND_SLOT; o.a = s; return o; }
  static Opnd mblk(int r, int c) { Opnd o; o.kind = OPND_MBLK; o.a = r; o.b = c; return o; }
  static Opnd ident() { Opnd o; o.kind = OPND_IDENT; return o; }
  static Opnd outp() { Opnd o; o.kind = OPND_OUT; return o; }
  static Opnd out_blk(int r) { Opnd o; o.kind = OPND_OUT; o.a = r; return o; }
  static Opnd rhs(int r) { Opnd o; o.kind = OPND_RHS; o.a = r; return o; }
};

enum StepKind : int32_t {
  ST_LOAD = 1,      // dst <- x
  ST_GETRF = 2,     // dst <- LU(dst)
  ST_TRTRI = 3,     // dst (LU) <- packed inverses of L and U; x = scratch slot
  ST_TRMM_L = 4,    // dst <- L(x)^{-1} P(x) y
  ST_TRMM_U = 5,    // dst <- U(x)^{-1} y
  ST_GEMM = 6,      // dst <- cin - x * y - sub
  ST_GEMM_ACC = 7,  // dst <- cin + x * y   (cin may be none)
  ST_GEMM_NEG = 8,  // dst <- -x * y
};

struct StepItem {
  Opnd dst, x, y, cin, sub;
  int32_t node = -1;
};

struct Step {
  StepKind kind;
  std::vector<StepItem> items;
};

struct Plan {
  int64_t n = 0;
  int k = 0, i = 0, j = 0;
  int b = 0;
  int width = 1;
  int transpose = 0;        // operands are blocks of Gamma^T
  std::vector<Step> steps;
  int nslots = 0;           // high-water mark of simultaneously live slots
  int64_t schur_ops = 0;
  int64_t final_inversions = 0;
  int64_t launches = 0;     // kernel launches with tile pivoting
  double executed_flops = 0;
  double algorithmic_flops = 0;
};

// Builds the plan of invert_block for target (i, j) with batch width W.
Plan make_block_plan(int64_t n, int k, int i, int j, int width);
// Builds the plan of bri_block_column (block column j of Gamma^{-1}).
Plan make_column_plan(int64_t n, int k, int j, int width);

// Plans of the mixed-precision refinement for block column j, sharing one
// slot numbering:
//   column: the block column plan that also keeps the factored pivot of
//           every back-substitution position in a reserved slot;
//   solve:  X = Gamma^{-1} R for a general (k b) x b right-hand side R
//           (operands OPND_RHS), by the same back substitution whose Schur
//           complements are recomputed, reusing the kept pivots.
struct RefinePlans {
  Plan column, solve;
  std::vector<int> kept;         // kept[pos]: slot of the pivot of elimination position pos
  bool column_gives_x0 = true;   // false: the column plan only factors the pivots (reuse)
};
RefinePlans make_refine_plans(int64_t n, int k, int j, int width, bool reuse);

// Blocks of Gamma read by the products of a step are first converted into
// slots by a load step (slot numbers from base, live for that step only);
// returns the most slots one step needed.  Used where M is read through
// converting or evaluating loads only (mixed precisions, matrix-free M).
int stage_matrix_blocks(Plan& p, int base);
// make_block_plan with every block of M staged that way.
Plan make_block_plan_staged(int64_t n, int k, int i, int j, int width);

// The plan of invert_block in the paper's literal frame order (Sections
// "Forward recursive procedure" and "Backward recursive procedure"): typed
// frames whose Schur complements may pivot on non-principal blocks, block
// rows 0 <-> j and columns 0 <-> i exchanged, the root's (M/D) inverted.
Plan make_block_plan_literal(int64_t n, int k, int i, int j, int width);

// The plan of invert_block with the k - 1 elimination pivots kept and reused
// (each Schur node then has three children; the paper's suggested reuse
// across branches).  Same result, fewer operations, k - 1 kept b x b blocks.
Plan make_block_plan_reuse(int64_t n, int k, int i, int j, int width);

// Launch/flop accounting of the kernels that realise a step.
// Kernel launches of one batched LU (tile pivoting, or panels with partial pivoting).
// LU variants: tile-step LU (tile pivoting), panel LU (partial pivoting),
// recursive LU with inverted factors (tile pivoting; no triangular
// inversion follows).
enum LuKind : int { LU_TILE = 0, LU_PANEL = 1, LU_RECURSIVE = 2 };
// The recursive LU halves the matrix down to kTile x kTile tiles: b must be
// kTile times a power of two.
inline bool getrf_rec_possible(int b) { return b >= 2 * kTile && b <= kMaxBlock && (b & (b - 1)) == 0; }
// Variant of a factorisation launch of count matrices of order b (uniform:
// all of that order).  choice: 0 automatic, 1 tile steps, 2 recursive where
// possible.  Automatic: the recursion's products keep the MFMA pipes busy
// when there are many or large matrices; for few small ones the tile-step
// LU's shorter chain of launches wins.
// Autotuned choices (bri_tune.cpp), loaded from the tuning cache on first
// use: -1 when the table holds nothing for the case.
int tuned_lu_kind(int count, int b);
int tuned_product_shape(int elem, int tri, int count, int m, int n);
// Overrides for the autotuner's timing runs (-1: none), per host thread.
extern thread_local int g_force_shape;
extern thread_local int g_force_lu;
// Tile shapes of the FP64 explicit products that the autotuner chooses from:
// 128 x 128, 64 x 64, 256 x 128 and 128 x 256 (rows x columns).
constexpr int kShapeDl128 = 1, kShapeDl64 = 2, kShapeDl256 = 3, kShapeDl128w = 4;

inline LuKind lu_kind(int count, int b, bool panel_pivoting, bool uniform, int choice) {
  if (panel_pivoting) return LU_PANEL;
  if (!uniform || !getrf_rec_possible(b) || choice == 1) return LU_TILE;
  if (choice == 2) return LU_RECURSIVE;
  if (g_force_lu == LU_TILE || g_force_lu == LU_RECURSIVE) return static_cast<LuKind>(g_force_lu);
  const int tuned = tuned_lu_kind(count, b);
  if (tuned == LU_TILE || tuned == LU_RECURSIVE) return static_cast<LuKind>(tuned);
  const double work = static_cast<double>(count) * b * b * b;
  return work >= 64.0 * 1024.0 * 1024.0 * 1024.0 ? LU_RECURSIVE : LU_TILE;
}
int64_t getrf_launches(int b, LuKind kind);
int64_t trtri_launches(int b, LuKind kind);
double getrf_flops(int b);
double trtri_flops(int b);

}  // namespace bri
