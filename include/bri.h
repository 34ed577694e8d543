/*
 * bri.h -- C ABI of the MI355X block recursive inverse (BRI) library.
 *
 * The library returns one chosen b x b block N_ij of M^{-1} for a nonsingular
 * n x n matrix M partitioned into k x k square blocks of order b = ceil(n/k)
 * (Section "Preliminaries", eqs. blockmatricesnxn and
 * inverseblockmatricesnxn).  The block is computed by recursive Schur
 * complement splitting (Section "Block Recursive Inversion algorithm"): every
 * intermediate block is a Schur complement v(r, c, I) = M_rc - M_rI M_II^{-1}
 * M_Ic that is recomputed rather than stored, so the device workspace is a
 * small multiple of b^2 per concurrently evaluated branch (Section
 * "Implementation", Theorem "MC_BRI").  When k does not divide n the matrix is
 * treated as the augmented Gamma = [[M, 0], [0, I_l]] (eq. M_augmented) and the
 * returned block is the block of Gamma^{-1} (eq. inverse_M_augmented): rows or
 * columns past n of the last block hold the identity / zero padding.
 *
 * Conventions for every entry point below:
 *  - Matrices are row-major.  Element (r, c) of M is M[r * ldm + c].
 *  - Block indices i, j are 0-based: the paper's N_11 is (i, j) = (0, 0).
 *  - Every matrix pointer is a DEVICE pointer owned by the caller.  M is only
 *    read.  The library never allocates device memory: the caller passes a
 *    workspace of at least bri_workspace_size() bytes.
 *  - All work is enqueued on opts->stream; calls return once the work is
 *    enqueued (asynchronous).  The caller keeps M, out and the workspace alive
 *    until the stream has executed the work.
 *  - Calls that share a workspace must not overlap in time.
 *
 * Error behaviour:
 *  - Synchronous argument checks return -p when argument p (1-based position
 *    in the C signature) is invalid, in the style of LAPACK's info; nothing is
 *    enqueued then.
 *  - BRI_ERR_WORKSPACE: the workspace is smaller than bri_workspace_size().
 *  - BRI_ERR_UNSUPPORTED: a size or precision this build does not support
 *    (b > BRI_MAX_BLOCK, or a precision not available for the entry point).
 *  - BRI_ERR_HIP: a HIP launch or copy failed; the stream state is undefined.
 *  - Numerical failures are only known on the device and are written to
 *    *opts->d_info (a device int32; may be NULL): 0 = success, t > 0 = the
 *    pivot factorisation of Schur operation t-1 (in execution order; the final
 *    inversion counts as the last operation) met an exactly zero or
 *    non-finite pivot.  The result is then undefined, as with LAPACK getrf.
 *    For the mixed-precision paths d_info = -1 means that iterative refinement
 *    did not reach the requested tolerance within refine_max_iters.
 */
#ifndef BRI_H
#define BRI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BRI_OK 0
#define BRI_ERR_HIP (-1000)
#define BRI_ERR_WORKSPACE (-1001)
#define BRI_ERR_UNSUPPORTED (-1002)

/* Largest block order b supported by the pivot factorisation kernels. */
#define BRI_MAX_BLOCK 4096

/* Element type of M / out and the arithmetic the Schur updates run in. */
typedef enum {
  BRI_F64 = 0,        /* M, out: double.  All arithmetic FP64 (FP64 MFMA).        */
  BRI_F32 = 1,        /* M, out: float.   All arithmetic FP32 (FP32 MFMA).        */
  BRI_MIXED_F32 = 2,  /* M, out: double.  Schur products in FP32, FP64 refinement. */
  BRI_MIXED_F16 = 3,  /* M, out: double.  Schur products in FP16 MFMA (FP32 acc).  */
  BRI_MIXED_BF16 = 4  /* M, out: double.  Schur products in BF16 MFMA (FP32 acc).  */
} bri_precision;

/* Pivoting of the b x b pivot factorisations (the method itself never
 * pivots across blocks: every pivot is a principal Schur complement). */
typedef enum {
  BRI_PIVOT_TILE = 0,   /* partial pivoting inside each 32-row diagonal tile.  Stable
                           for SPD and diagonally dominant matrices (whose pivot
                           blocks, principal Schur complements, stay such).  A
                           factorisation whose largest |U| exceeds 64 times its
                           largest |A| (element growth; partial pivoting keeps this
                           ratio near 10 on Gaussian matrices) is reported through
                           d_info like a failed pivot.                            */
  BRI_PIVOT_PANEL = 1,  /* partial pivoting over all rows of the pivot block (LAPACK getrf) */
  BRI_PIVOT_AUTO = 2    /* default: tile pivoting; the call then waits for the stream
                           and, if a factorisation reported a failed pivot or element
                           growth, computes the block again with panel pivoting
                           (batched calls: the flagged problems, one by one, in the
                           same workspace).  Synchronous.                            */
} bri_pivoting;

/* Elimination order of the recursion. */
typedef enum {
  BRI_ORDER_PRINCIPAL = 0, /* default: every Schur complement is taken with respect to a
                              principal pivot block v(p, p, I) (eq. SchurofA with the
                              pivot moved to the leading position); for a target
                              (i, j) the other blocks are eliminated in ascending
                              order, then j (i != j) or the largest other index, and an
                              off-diagonal block is assembled by eq. invSchur          */
  BRI_ORDER_PAPER = 1      /* the literal frame procedure of Sections "Forward recursive
                              procedure" and "Backward recursive procedure": block rows
                              0 <-> j and columns 0 <-> i exchanged, typed frames
                              reduced by (M/D), (M/C), (M/B) or (M/A), the root's (M/D)
                              inverted.  For k >= 5 some pivots are non-principal
                              blocks, which may be singular or ill-conditioned where
                              the principal order's are not.  invert_block and its
                              size / describe / dump queries only, BRI_F64 and BRI_F32,
                              without reuse; elsewhere BRI_ERR_UNSUPPORTED (size
                              queries: 0)                                              */
} bri_order;

typedef struct {
  int precision;           /* a bri_precision value                                   */
  int concurrency;         /* W: Schur operations evaluated side by side; <= 0: auto  */
  int pivoting;            /* a bri_pivoting value                                    */
  int reuse;               /* 0: recompute every Schur complement (the paper's
                              procedure); 1: keep the k - 1 factored elimination
                              pivots and reuse them (the paper's suggested reuse
                              across branches: 3 children per Schur node instead of
                              4, k - 1 more b x b blocks of workspace)            */
  int refine_max_iters;    /* mixed paths: refinement sweeps (0 = none)               */
  double refine_tol;       /* mixed paths: stop when the correction dX_t, or from the
                              second sweep the bound rho/(1-rho) ||dX_t||_F with
                              rho = ||dX_t|| / ||dX_{t-1}|| < 1/2, is <= tol ||X||_F   */
  void* workspace;         /* device workspace, >= bri_workspace_size() bytes         */
  size_t workspace_bytes;  /* its size                                                */
  int32_t* d_info;         /* device int32 status (see above), or NULL                */
  hipStream_t stream;      /* stream the work is enqueued on (NULL = default stream)  */
  int factorization;       /* the LU of each pivot block (with tile pivoting):
                              0 automatic; 1 tile steps (one launch per 32-column
                              diagonal tile) followed by a triangular inversion;
                              2 recursive halving with inverted factors (block
                              orders 32 * 2^m only, else tile steps)              */
  size_t workspace_budget; /* 0: none.  Otherwise, with automatic concurrency, the
                              width is the widest one (the automatic width, then
                              down by factors of 4) whose workspace fits in this
                              many bytes: fewer Schur operations side by side,
                              more launches (the memory / time trade-off of
                              Theorem "MC_BRI").  Size queries return 0 and calls
                              BRI_ERR_WORKSPACE when even width 1 does not fit.
                              Batched calls ignore it.                            */
  int order;               /* a bri_order value (default BRI_ORDER_PRINCIPAL)         */
  int64_t* d_stats;        /* device accounting of the work a call executes, or NULL:
                              4 device int64 words, zeroed at the start of the call's
                              last pass (automatic pivoting: the panel pass when it
                              ran; mixed: the BF16 pass after an FP16 range restart)
                              and filled by small kernels after every plan step from
                              the descriptors that step ran on: [0] pivot
                              factorisations (Theorem "C_BRI": T(k) Schur operations
                              + the final inversion), [1] Schur products D - C X,
                              [2] other products (triangular multiplies, final
                              products), [3] workspace high-water mark: the end of
                              the highest workspace byte a step wrote, relative to
                              workspace (Theorem "MC_BRI").  invert_block (plain and
                              mixed precisions, noalloc included); calls with it do
                              not replay captured graphs.  Costs one small launch
                              per plan step.                                          */
} bri_opts;

/* Fills *o with defaults: BRI_F64, automatic concurrency, automatic pivoting
 * (BRI_PIVOT_AUTO), no reuse, 10 refinement sweeps, tolerance 1e-12, no
 * workspace, no d_info, default stream, automatic factorisation, no
 * workspace budget. */
void bri_default_opts(bri_opts* o);

/* Bytes of device workspace invert_block() needs for (n, k, i, j) with the
 * precision and concurrency of *o (the workspace fields of *o are ignored).
 * Returns 0 for invalid arguments. */
size_t bri_workspace_size(int64_t n, int k, int i, int j, const bri_opts* o);

/* Block N_ij of M^{-1} (of Gamma^{-1} when k does not divide n).
 *   M    : n x n, leading dimension ldm >= n, element type per precision.
 *   k    : number of block rows/columns, 2 <= k <= n.
 *   i, j : target block, 0 <= i, j < k.
 *   out  : b x b result, b = ceil(n / k), leading dimension ldo >= b.
 * Recursive Schur splitting of Sections "Forward recursive procedure" and
 * "Backward recursive procedure" in the principal elimination order; for
 * i != j the last step takes the lower-left block of eq. invSchur. */
int invert_block(const void* M, int64_t n, int64_t ldm, int k, int i, int j,
                 void* out, int64_t ldo, const bri_opts* o);

/* Block column j of M^{-1} (Gamma^{-1}): X = Gamma^{-1} E_j, (k*b) x b with
 * leading dimension ldx >= b, by block back substitution whose Schur
 * complements are recomputed by the same recursion.  With transpose != 0 the
 * block column of (M^T)^{-1} is returned instead (its transpose is block row j
 * of M^{-1}).  Workspace: bri_block_column_workspace_size(). */
size_t bri_block_column_workspace_size(int64_t n, int k, int j, const bri_opts* o);
int bri_block_column(const void* M, int64_t n, int64_t ldm, int k, int j, int transpose,
                     void* X, int64_t ldx, const bri_opts* o);

/* Batched form: count independent problems (M[t], n[t], k[t], i[t], j[t]) ->
 * out[t]; all arrays are HOST arrays (of device pointers where pointers).  All
 * problems share one workspace of bri_batched_workspace_size() bytes (its size
 * depends on the precision and pivoting in *o).  d_info, if not NULL, points
 * to count device int32s (one status per problem).  With BRI_F64 / BRI_F32
 * and tile pivoting the problems are merged: problems whose plans have the
 * same step structure (same k, diagonal or off-diagonal target) share every
 * kernel launch, each work item carrying its own block order b = ceil(n/k)
 * (Section "Block Recursive Inversion algorithm" per problem; the paper's
 * remark that blocks can be computed in an embarrassingly parallel fashion,
 * Section "Conclusion").  Other precisions and panel pivoting evaluate the
 * problems one after another on the stream.  Argument codes: -p for argument
 * p of this signature when any problem's entry is invalid. */
size_t bri_batched_workspace_size(int count, const int64_t* n, const int* k, const int* i,
                                  const int* j, const bri_opts* o);
int invert_block_batched(int count, const void* const* M, const int64_t* n, const int64_t* ldm,
                         const int* k, const int* i, const int* j, void* const* out,
                         const int64_t* ldo, const bri_opts* o);

/* invert_block for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it).  Same
 * arguments and result as invert_block (BRI_F64 and BRI_F32; o->workspace
 * and o->workspace_bytes are ignored), but the workspace is a static device
 * array of BRI_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends, and the step descriptors are staged
 * through a static host buffer: no device or pinned host memory is
 * allocated (the host plan of a new shape is built and cached in ordinary
 * host memory on its first call).  With automatic concurrency the width is
 * the widest whose workspace fits the array; problems that do not fit even
 * at width 1 return BRI_ERR_WORKSPACE (and mixed precisions
 * BRI_ERR_UNSUPPORTED).  All calls on one GPU share the array, which keeps
 * the last call's contents: calls that overlap in time on one GPU race. */
#define BRI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
size_t bri_noalloc_scratch_bytes(void);
int invert_block_noalloc(const void* M, int64_t n, int64_t ldm, int k, int i, int j,
                         void* out, int64_t ldo, const bri_opts* o);

/* Several blocks of one matrix: blocks (i[t], j[t]) of M^{-1}, t < count, to
 * out[t] (b x b, leading dimension ldo[t]).  i, j, out and ldo are HOST
 * arrays.  All k^2 blocks, or any selection (such as the band of blocks near
 * the diagonal), follow the paper's remark that the blocks can be computed
 * independently and in parallel (Section "Conclusion"; Section
 * "Implementation" obtains every block by its own run): the targets are the
 * problems of one merged batch over the same M (invert_block_batched with
 * M[t] = M), sharing its launches.  Workspace:
 * bri_blocks_workspace_size().  d_info, if not NULL, holds count statuses.
 * Argument codes: -p for argument p of this signature. */
size_t bri_blocks_workspace_size(int64_t n, int k, int count, const int* i, const int* j, const bri_opts* o);
int invert_blocks(const void* M, int64_t n, int64_t ldm, int k, int count, const int* i, const int* j,
                  void* const* out, const int64_t* ldo, const bri_opts* o);

/* Matrix-free M: block N_ij of A_gamma^{-1} for the LS-SVM cross-validation
 * matrix of Section "Experimental results" (eq. A), of order m = npts + 1,
 *   A_gamma = [[0, 1^T], [1, K + I / gamma]],  K_rc = exp(-||x_r - x_c||^2 / (2 sigma^2)),
 * never stored: every block of it the recursion reads is evaluated from the
 * data points by the block loads (the paper's remark that such a matrix can
 * be computed element by element from the much smaller input data, Section
 * "Implementation").
 *   X   : npts x d data points, row-major, leading dimension ldx >= d; double
 *         for BRI_F64, float for BRI_F32 (the other precisions: unsupported).
 *   sigma, gamma > 0; k, i, j, out, ldo as for invert_block with n = npts + 1.
 * Workspace: bri_rbf_workspace_size(); argument codes -p as usual. */
size_t bri_rbf_workspace_size(int64_t npts, int d, int k, int i, int j, const bri_opts* o);
int invert_block_rbf(const void* X, int64_t npts, int64_t ldx, int d, double sigma, double gamma,
                     int k, int i, int j, void* out, int64_t ldo, const bri_opts* o);

/* Adjoint of invert_block: for L = sum(G .* N_ij), writes
 *   grad_M = dL/dM = -(N_{i,:})^T G (N_{:,j})^T            (n x n, ld ldgm)
 * where N_{i,:} and N_{:,j} are block row i and block column j of M^{-1},
 * recomputed through the recursion (nothing is stored by the forward call).
 * G is b x b with leading dimension ldg.  Precisions: BRI_F64, BRI_F32.
 * Workspace: bri_backward_workspace_size(). */
size_t bri_backward_workspace_size(int64_t n, int k, int i, int j, const bri_opts* o);
int invert_block_backward(const void* M, int64_t n, int64_t ldm, int k, int i, int j,
                          const void* G, int64_t ldg, void* grad_M, int64_t ldgm,
                          const bri_opts* o);

/* The Schur-update product kernel on plain operands: for t < count,
 *   C[t] = beta * C[t] + alpha * A[t] B[t]     (C[t]: m x n, A[t]: m x kk, B[t]: kk x n)
 * row-major with leading dimensions lda, ldb, ldc; A, B, C are HOST arrays of
 * DEVICE pointers.  precision BRI_F64 (double) or BRI_F32 (float); C may not
 * alias A or B.  Uses o->stream and, for its descriptors, o->workspace of at
 * least bri_gemm_workspace_size(count) bytes.  This is the MFMA kernel every
 * Schur complement D - C A^{-1} B of the recursion runs its products on
 * (eqs. SchurofA..SchurofD); it is exported to measure and test it alone.
 * BRI_MIXED_F16 / BRI_MIXED_BF16 (float operands, split products): workspace
 * beyond bri_gemm_workspace_size(count) is scratch for the operands split
 * once before the products, 2 p (m + n) ceil(kk / 64) 64 bytes per item
 * (p = 2 FP16 or 3 BF16 parts), as many items at a time as it holds (used
 * for launches of 2048 or more output tiles of 256 x 128 when kk is a
 * multiple of 8 and the rows of A are 16-byte aligned). */
size_t bri_gemm_workspace_size(int count);
int bri_gemm(int count, int64_t m, int64_t n, int64_t kk, double alpha, const void* const* A, int64_t lda,
             const void* const* B, int64_t ldb, double beta, void* const* C, int64_t ldc, const bri_opts* o);

/* Structure of the evaluation plan for (n, k, i, j) under *o, without running
 * it (host only).  Counts are per call of invert_block. */
typedef struct {
  int64_t schur_ops;        /* Schur complement operations executed                  */
  int64_t final_inversions; /* b x b inversions after the recursion (1)              */
  int64_t slots;            /* b x b workspace blocks live at the high-water mark    */
  int64_t batch_width;      /* W actually used                                       */
  int64_t steps;            /* batched plan steps                                    */
  int64_t kernel_launches;  /* kernel launches one call enqueues                     */
  int64_t block;            /* b                                                     */
  double algorithmic_flops; /* T(k) (14/3) b^3 + 2 b^3 (+ 2 b^3 if i != j)          */
  double executed_flops;    /* flops the kernels execute                             */
  size_t workspace_bytes;   /* == bri_workspace_size()                               */
} bri_plan_stats;
int bri_plan_describe(int64_t n, int k, int i, int j, const bri_opts* o, bri_plan_stats* s);

/* Host-only description of the plan's steps for inspection by tests:
 * writes up to cap int64 words, returns the number needed (or < 0 on bad
 * arguments).  Format: for every step, [kind, nitems] followed per item by 16
 * words: dst(kind, a, b), x(kind, a, b), y(kind, a, b), cin(kind, a, b),
 * sub(kind, a, b), node.  Operand kinds: 0 none, 1 slot a, 2 block (a, b) of
 * M, 3 identity, 4 out.  Step kinds: 1 load, 2 getrf, 3 trtri, 4 trmm_lower,
 * 5 trmm_upper, 6 gemm (dst = cin - x * y - sub), 7 gemm_acc (dst = cin + x * y),
 * 8 gemm_neg (dst = -x * y). */
int64_t bri_plan_dump(int64_t n, int k, int i, int j, const bri_opts* o, int64_t* words,
                      int64_t cap);

/* The two plans of the mixed-precision refinement for block column j
 * (which = 0: the float block column plan that keeps its pivots; 1: the
 * correction solve X = Gamma^{-1} R, with R as operand kind 5 "rhs block a";
 * 2: the k slots holding the kept pivots, by elimination position), in the
 * format of bri_plan_dump.  Host only; returns the number of words needed or
 * < 0 on bad arguments. */
int64_t bri_refine_plan_dump(int64_t n, int k, int j, int which, const bri_opts* o, int64_t* words,
                             int64_t cap);

/* Step timing, a profiling aid.  While enabled, every plan step that
 * invert_block / bri_block_column enqueue is bracketed by two HIP events on
 * the caller's stream.  bri_profile_read() waits for those events and writes,
 * for each step kind t (entry t, kinds as in bri_plan_dump; entry 0 unused),
 * the number of steps, of kernel launches, the summed GPU time between the
 * events in milliseconds and the algorithmic flops of the steps (getrf and
 * triangular inversion 2/3 b^3, triangular products b^3, products 2 b^3 per
 * item); it then clears the record.  Returns the number of entries written. */
typedef struct {
  int64_t steps;
  int64_t launches;
  double ms;
  double flops;
} bri_profile_entry;
#define BRI_PROFILE_KINDS 9
int bri_profile_enable(int on);
int bri_profile_read(bri_profile_entry* entries, int cap);

/* Diagnostics of the calling thread's last mixed-precision invert_block:
 * the number of refinement sweeps it ran, the relative size
 * ||dX||_F / ||X||_F of its last correction, and whether its FP16 split
 * products met an operand outside the FP16 range and the call was computed
 * again with BF16 split products (0, 0 and 0 before any such call).  Any
 * pointer may be NULL. */
int bri_refine_last(int* sweeps, double* last_update, int* bf16_fallback);

/* Autotuner.  bri_autotune() measures on this GPU, with synthetic inputs in
 * o->workspace (at least 64 MiB; larger workspaces cover larger cases, up to
 * about 4 GiB for all of them) on o->stream, (1) which tile shape the FP64
 * products of a plan step run fastest in, for 1..64 items of order
 * 256..2048, plain and triangular, and (2) which LU variant (tile steps or
 * recursive halving) factors 1..64 matrices of order 256..2048 fastest.  It
 * writes the decisions to the text cache at path (NULL: $BRI_TUNE_CACHE, else
 * $HOME/.cache/bri-mi355x/tune.txt), loads them, and returns the number of
 * decisions (< 0: an error code).  Later calls of this process, and every
 * process that finds the cache, take these decisions where the automatic
 * choices apply (bri_opts.factorization = 0); the built-in rules cover the
 * cases the cache lacks.  bri_tune_load() (re)loads a cache (NULL: the
 * default path) and returns its number of decisions, or BRI_ERR_UNSUPPORTED
 * when it cannot be read.  Synchronous. */
int bri_autotune(const bri_opts* o, const char* path);
int bri_tune_load(const char* path);

/* Human-readable text for a status code returned by any entry point. */
const char* bri_status_string(int status);

/* Library version string. */
const char* bri_version(void);

/* sizeof(bri_opts) as the library was built with (for bindings that lay the
 * struct out themselves). */
size_t bri_opts_size(void);

#ifdef __cplusplus
}
#endif

#endif /* BRI_H */
