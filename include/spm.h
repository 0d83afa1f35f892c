/*
 * spm.h -- C ABI of the MI355X (gfx950) sparse assembly + CSC SpMM library (libspm.so).
 *
 * The operations follow Sanderson & Curtin, "A User-Friendly Hybrid Sparse Matrix Class in C++"
 * (LNCS 10931, 2018; arXiv:1805.03380):
 *   - COO (Section 3.2): an unordered list of (row, column, value) triplets held as three
 *     arrays; duplicates of one location are allowed and accumulate (the += element update of
 *     Fig. 1), in input order.
 *   - CSC (Section 3.1): values[N], row_indices[N] and column offsets c[n_cols+1] with c[0] = 0,
 *     c[n_cols] = N, zero-based indices; column i holds c[i+1] - c[i] elements, stored in
 *     increasing row order (the ordered traversal of Section 3.3 emits column-major order).
 *   - the product of a dense operand with the sparse matrix (Section 3, use case (iv)).
 *
 * Conventions shared by every entry point
 *   Memory.   Every array argument is DEVICE memory owned by the caller, except where marked
 *             "host".  The library never allocates, frees or keeps a pointer after returning;
 *             scratch memory comes in through a caller-provided workspace (ws, ws_bytes) whose
 *             size the matching *_workspace / *_size call reports.  Device buffers must be
 *             256-byte aligned where noted (PyTorch allocations are).
 *   Streams.  `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every
 *             call only enqueues work on that stream; none synchronizes it.
 *   Errors.   Arguments that can be checked on the host are checked before anything is
 *             enqueued; on failure the call returns that status and enqueues nothing.
 *             Conditions only the device can see (an out-of-range triplet, a malformed CSC)
 *             are written to the device status word info[1].  Out-of-range triplets are
 *             skipped and the outputs describe the others; a plan built from a malformed CSC
 *             is unspecified.  Either way no kernel reads or writes outside the buffers
 *             described here.
 *             A failed HIP launch returns SPM_EHIP.
 *   Sizes.    Dimensions and counts are int64_t on the ABI; n_rows, n_cols, nnz and every
 *             offset must fit in int32 (SPM_EOVERFLOW otherwise).
 *   Dense.    Dense operands are row-major with a leading dimension (elements between rows):
 *             X is n_cols x k (row c of X multiplies column c of A), Y and G are n_rows x k.
 *   Numerics. Assembly folds duplicates left to right in input order in binary64 and rounds
 *             once to the output type; a location whose fold compares equal to 0.0 is not
 *             stored (so -0.0 and cancelled sums are dropped; NaN and Inf are kept).  SpMM
 *             accumulates every output sequentially in a fixed order (ascending column for Y,
 *             ascending row for dX) in binary64, or in binary32 when a dense operand is
 *             bfloat16 and no operand is binary64, and rounds once.  Results do not depend
 *             on tuning, launch shape or batching: the batched entry point is bitwise equal
 *             to the per-matrix entry points.
 */
#ifndef SPM_H
#define SPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Under C++ the enumerations have int as their underlying type, so every int a C caller
 * passes is a value of the type (an unknown one is then rejected by the checks below); in C an
 * enumeration is an int already. */
#ifdef __cplusplus
#define SPM_ENUM_INT : int
#else
#define SPM_ENUM_INT
#endif

typedef enum spm_status SPM_ENUM_INT {
  SPM_OK = 0,
  SPM_EINVAL = 1,     /* null pointer, negative size, k < 1, bad leading dimension, bad CSC */
  SPM_EBOUNDS = 2,    /* (device) a triplet's row or column is outside the matrix */
  SPM_EOVERFLOW = 3,  /* a size or offset does not fit in int32 */
  SPM_EWORKSPACE = 4, /* workspace / plan buffer smaller than reported */
  SPM_EDTYPE = 5,     /* unsupported element-type combination */
  SPM_EHIP = 6        /* a HIP runtime call or kernel launch failed */
} spm_status;

typedef enum spm_dtype SPM_ENUM_INT {
  SPM_F64 = 0,  /* IEEE binary64 */
  SPM_F32 = 1,  /* IEEE binary32 */
  SPM_BF16 = 2  /* bfloat16, stored as uint16 */
} spm_dtype;

/* Order of the stored values handed to the forward product:
 *   SPM_ORDER_CSC   val[p] for CSC slot p (as assembled); the product reads val[perm[q]].
 *   SPM_ORDER_PLAN  val[q] for plan slot q, i.e. val_csc[perm[q]] (as written by
 *                   spm_csc_plan_build with values); the product reads val[q] contiguously.
 * Plan-order values are a copy: after the CSC values change they must be rebuilt (or the
 * CSC order used). */
typedef enum spm_val_order SPM_ENUM_INT { SPM_ORDER_CSC = 0, SPM_ORDER_PLAN = 1 } spm_val_order;

/* Human-readable name of a status code (static string, never NULL). */
const char *spm_status_string(int status);

/* Library version string, e.g. "0.1.0 gfx950". */
const char *spm_version(void);

/* ------------------------------------------------------------------------------------------
 * COO -> CSC bulk assembly  (Section 3.2 -> Section 3.1; duplicates accumulate as in Fig. 1,
 * location order is the column-major index order row + col * n_rows of Section 3.3).
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Bytes of workspace spm_coo_to_csc needs for these sizes (*ws_bytes, host).
 * Returns SPM_EINVAL / SPM_EOVERFLOW for sizes spm_coo_to_csc would reject. */
spm_status spm_coo_to_csc_workspace(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                    size_t *ws_bytes);

/* Assemble nnz_in triplets (row[t], col[t], val[t]) of an n_rows x n_cols matrix into CSC.
 *   row, col  int32[nnz_in]; val[nnz_in] of type val_type (F64, F32 or BF16).
 *   col_ptr   int32[n_cols + 1], fully written: col_ptr[0] = 0, col_ptr[n_cols] = nnz_out.
 *   row_idx   int32[nnz_in] capacity; the first nnz_out entries are written.
 *   val_out   capacity nnz_in elements of out_type (F64 or F32); first nnz_out written.
 *   info      int32[2], written on the stream: info[0] = nnz_out, info[1] = device status
 *             (0, or SPM_EBOUNDS when some triplet lies outside the matrix; out-of-range
 *             triplets are then skipped and the outputs describe the remaining ones).
 *   ws        workspace of at least spm_coo_to_csc_workspace() bytes, 256-byte aligned.
 * nnz_in = 0 is legal (all-zero col_ptr); n_cols = 0 gives col_ptr = {0}. */
spm_status spm_coo_to_csc(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t *row,
                          const int32_t *col, const void *val, spm_dtype val_type,
                          int32_t *col_ptr, int32_t *row_idx, void *val_out,
                          spm_dtype out_type, int32_t *info, void *ws, size_t ws_bytes,
                          void *stream);

/* ------------------------------------------------------------------------------------------
 * Row index ("plan") of a CSC pattern: the structural transpose the forward product walks.
 * Deriving the layout an operation needs from the canonical CSC and keeping it alongside is
 * the hybrid-storage idea of Section 3.4; the transpose itself is X.t() of Table 1.
 * Plan layout (int32, each part starting on a 256-byte boundary):
 *   row_ptr[n_rows + 1] | col_t[nnz_cap] | perm[nnz_cap]
 * where for q in [row_ptr[r], row_ptr[r+1]) the stored element (r, col_t[q]) sits at CSC
 * slot perm[q], and columns increase with q inside each row.
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Plan size and plan-build workspace size for a CSC with capacity nnz_cap. */
spm_status spm_csc_plan_size(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                             size_t *plan_bytes, size_t *ws_bytes);

/* Host only.  The plan size alone (the plan_bytes of spm_csc_plan_size). */
spm_status spm_csc_plan_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                              size_t *plan_bytes);

/* Build the plan of the CSC pattern (col_ptr[n_cols+1], row_idx[nnz]) where nnz =
 * col_ptr[n_cols] is read on the device and must not exceed nnz_cap.
 *   val, val_plan  optional (both NULL, or both given): the CSC values (val_type F64 or F32,
 *         nnz_cap capacity) and a buffer of nnz_cap elements of the same type that receives
 *         them in plan order, val_plan[q] = val[perm[q]] (see SPM_ORDER_PLAN).  The values
 *         travel with the pattern through the grouping, so this costs a contiguous write
 *         rather than a gather.
 *   info  int32[2]: info[0] = nnz seen, info[1] = 0, SPM_EINVAL (col_ptr not monotone,
 *         col_ptr[0] != 0 or nnz > nnz_cap) or SPM_EBOUNDS (a row index out of range). */
spm_status spm_csc_plan_build(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                              const int32_t *col_ptr, const int32_t *row_idx, const void *val,
                              spm_dtype val_type, void *plan, size_t plan_bytes,
                              void *val_plan, int32_t *info, void *ws, size_t ws_bytes,
                              void *stream);

/* ------------------------------------------------------------------------------------------
 * Assembly and plan in one call (Sections 3.2 -> 3.1 and the row index of Section 3.4): the
 * same outputs as spm_coo_to_csc followed by spm_csc_plan_build with nnz_cap = nnz_in (and,
 * when val_plan is given, the assembled values carried to plan order), bit for bit.  The
 * assembled elements go straight from the assembly's grouping into the plan's, so the plan
 * does not re-read the CSC it was just given.  Shapes that the fused grouping does not cover
 * run the two builds one after the other; the results are the same either way.
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Plan bytes (as spm_csc_plan_size with nnz_cap = nnz_in) and workspace bytes of
 * spm_coo_to_csc_plan. */
spm_status spm_coo_to_csc_plan_size(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                    size_t *plan_bytes, size_t *ws_bytes);

/* Arguments as in spm_coo_to_csc, plus
 *   plan       plan buffer (layout above, nnz_cap = nnz_in) of at least plan_bytes, 256-byte
 *              aligned.
 *   val_plan   optional (NULL for none): nnz_in elements of out_type; receives the
 *              assembled values in plan order, val_plan[q] = val_out[perm[q]].
 *   plan_info  int32[2]: plan_info[0] = nnz_out, plan_info[1] = 0 (the CSC is valid by
 *              construction; out-of-range triplets are reported in info[1]).
 *   ws         at least the ws_bytes of spm_coo_to_csc_plan_size, 256-byte aligned.
 * Errors: as spm_coo_to_csc; SPM_EINVAL also for a NULL or misaligned plan / plan_info. */
spm_status spm_coo_to_csc_plan(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                               const int32_t *row, const int32_t *col, const void *val,
                               spm_dtype val_type, int32_t *col_ptr, int32_t *row_idx,
                               void *val_out, spm_dtype out_type, int32_t *info, void *plan,
                               size_t plan_bytes, void *val_plan, int32_t *plan_info, void *ws,
                               size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): spm_coo_to_csc_plan with the workspace taken from a
 * fixed array inside the library instead of the caller.
 *   The array is SPM_NOALLOC_SCRATCH_BYTES (64 MiB) of device memory that every GPU the
 *   library runs this call on holds from the first such call until the process ends.  Sizes
 *   whose workspace (spm_coo_to_csc_plan_size) exceeds it return SPM_EWORKSPACE before
 *   anything is enqueued (about 1.2e6 triplets at the default tuning).  The call allocates
 *   nothing; the caller still passes every input and output as for spm_coo_to_csc_plan,
 *   with the same results bit for bit.
 *   All calls on one GPU share that GPU's array: calls that overlap in time on one GPU (on
 *   different streams, or from several host threads without ordering) race on it and their
 *   results are unspecified.  Calls in one stream are ordered and safe.  The array keeps the
 *   last call's contents; every call clears what it needs itself.
 *   SPM_EHIP if the array's device address cannot be obtained. */
#define SPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
spm_status spm_coo_to_csc_plan_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz_in,
                                       const int32_t *row, const int32_t *col, const void *val,
                                       spm_dtype val_type, int32_t *col_ptr, int32_t *row_idx,
                                       void *val_out, spm_dtype out_type, int32_t *info,
                                       void *plan, size_t plan_bytes, void *val_plan,
                                       int32_t *plan_info, void *stream);

/* ------------------------------------------------------------------------------------------
 * Batch insertion into an existing CSC (Section 3.1: the elements to be inserted are sorted
 * and then merged with the existing arrays), accumulating like X(r,c) += v of Fig. 1: at a
 * location the existing value comes first, then the new values in input order, folded in
 * binary64 and rounded once to out_type; a location whose result compares equal to 0.0 is
 * not stored.  The result is a new CSC (outputs must not overlap the existing arrays).  Only
 * the new triplets are sorted (by column, row and input position); the existing arrays are
 * read once by a merge that cuts the work by position in the merged sequence (merge path),
 * so long columns are shared by many threads.
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Workspace of spm_csc_insert for an existing CSC of capacity cap_a and nnz_t new
 * triplets. */
spm_status spm_csc_insert_workspace(int64_t n_rows, int64_t n_cols, int64_t cap_a,
                                    int64_t nnz_t, size_t *ws_bytes);

/* Insert nnz_t triplets (row[t], col[t], val[t]) into the n_rows x n_cols CSC
 * (a_col_ptr[n_cols+1], a_row_idx / a_val with capacity cap_a; the number of existing
 * elements a_col_ptr[n_cols] is read on the device).
 *   val_type   type of a_val and val alike: F64 or F32.
 *   col_ptr    int32[n_cols + 1], fully written; row_idx / val_out (out_type F64 or F32) have
 *              capacity cap_a + nnz_t, the first nnz_out entries are written.
 *   info       int32[2]: info[0] = nnz_out, info[1] = 0, SPM_EBOUNDS (a new triplet, or an
 *              existing row index, outside the matrix; skipped) or SPM_EINVAL (a_col_ptr not
 *              monotone, a_col_ptr[0] != 0 or more than cap_a elements, or existing rows not
 *              increasing down a column: then the outputs hold unspecified values, written
 *              only within their capacity).
 *   ws         at least spm_csc_insert_workspace() bytes, 256-byte aligned.
 * The existing rows must increase strictly within each column (a valid CSC).  n_cols >= 1;
 * shapes the assembly's partition does not cover return SPM_EINVAL.  cap_a + nnz_t must fit
 * in int32 (SPM_EOVERFLOW). */
spm_status spm_csc_insert(int64_t n_rows, int64_t n_cols, int64_t cap_a,
                          const int32_t *a_col_ptr, const int32_t *a_row_idx, const void *a_val,
                          int64_t nnz_t, const int32_t *row, const int32_t *col, const void *val,
                          spm_dtype val_type, int32_t *col_ptr, int32_t *row_idx, void *val_out,
                          spm_dtype out_type, int32_t *info, void *ws, size_t ws_bytes,
                          void *stream);

/* ------------------------------------------------------------------------------------------
 * Forward product Y = A . X  (Section 3 use case (iv), through the plan of A's pattern).
 *   val      values of A, val_type F64 or F32, in val_order: CSC order (indexed through
 *            plan.perm) or plan order (read contiguously; from spm_csc_plan_build).
 *   X        n_cols x k, x_type F64, F32 or BF16, leading dimension ldx >= k.
 *   Y        n_rows x k, y_type F64 or F32, leading dimension ldy >= k; fully written
 *            (rows with no stored element are 0).
 * Y[r, j] = sum over q in row r, ascending column, of val[perm[q]] * X[col_t[q], j]; the
 * order of the values changes where they are read from, never the result.
 * ------------------------------------------------------------------------------------------ */
spm_status spm_csc_spmm(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k,
                        const void *plan, const void *val, spm_dtype val_type,
                        spm_val_order val_order, const void *X, int64_t ldx, spm_dtype x_type,
                        void *Y, int64_t ldy, spm_dtype y_type, void *stream);

/* ------------------------------------------------------------------------------------------
 * Adjoint of Y = A . X for a loss with dL/dY = G (n_rows x k):
 *   dX[c, j]  = sum over p in column c (ascending row) of val[p] * G[row_idx[p], j]
 *               -- A^T . G by a walk down each CSC column, the traversal of the row-vector
 *               times CSC product of Fig. 1;
 *   dval[p]   = sum_j G[row_idx[p], j] * X[c, j]  -- G . X^T sampled on A's pattern.
 * G has an element type of its own, g_type (F64, F32 or BF16), independent of x_type (F64,
 * F32 or BF16): G arrives in Y's type (binary64 when the values are binary64, whatever X is)
 * and is read as such, never narrowed.  Sums run in binary64, or in binary32 when one of
 * G and X is bfloat16 and none of the values, G and X is binary64.
 * dX (n_cols x k, ld lddx, dx_type F64 or F32) and dval (nnz elements, dval_type F64 or F32)
 * may each be NULL to skip that output; nnz = col_ptr[n_cols] is read on the device and
 * clamped to nnz_cap.
 * ------------------------------------------------------------------------------------------ */
spm_status spm_csc_spmm_backward(int64_t n_rows, int64_t n_cols, int64_t nnz_cap, int64_t k,
                                 const int32_t *col_ptr, const int32_t *row_idx,
                                 const void *val, spm_dtype val_type, const void *G,
                                 int64_t ldg, spm_dtype g_type, const void *X, int64_t ldx,
                                 spm_dtype x_type, void *dX, int64_t lddx, spm_dtype dx_type,
                                 void *dval, spm_dtype dval_type, void *stream);

/* ------------------------------------------------------------------------------------------
 * Sum A + B of two CSCs of one shape, by the merge of batch insertion: B's stored elements are
 * inserted into A, so a location stored in both holds A's value plus B's (binary64, A's
 * first), and a 0.0 result is not stored.
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Workspace of spm_csc_add. */
spm_status spm_csc_add_workspace(int64_t n_rows, int64_t n_cols, int64_t a_cap, int64_t b_cap,
                                 size_t *ws_bytes);

/* A (a_col_ptr, a_row_idx, a_val; capacity a_cap) and B (b_*; capacity b_cap): valid CSCs,
 * n_rows x n_cols, rows increasing down each column; the stored counts are read on the device.
 *   val_type   F64 or F32, the type of a_val and b_val.
 *   col_ptr    int32[n_cols + 1]; row_idx / val_out (out_type F64 or F32) have capacity
 *              a_cap + b_cap.
 *   info       int32[2]: info[0] = nnz of the sum, info[1] = 0, SPM_EINVAL (a malformed
 *              CSC) or SPM_EBOUNDS (a stored row outside the matrix).
 *   ws         at least spm_csc_add_workspace() bytes, 256-byte aligned.
 * n_cols must be at least 1 (SPM_EINVAL otherwise, as for spm_csc_insert).  The two CSCs are
 * merged by merge path (as in spm_csc_insert, with B in place of the sorted new triplets);
 * rows not increasing down a column of A or B are also reported as SPM_EINVAL, after which
 * the outputs hold unspecified values, written only within their capacity; with SPM_EBOUNDS
 * the locations outside the matrix are skipped. */
spm_status spm_csc_add(int64_t n_rows, int64_t n_cols, int64_t a_cap, const int32_t *a_col_ptr,
                       const int32_t *a_row_idx, const void *a_val, int64_t b_cap,
                       const int32_t *b_col_ptr, const int32_t *b_row_idx, const void *b_val,
                       spm_dtype val_type, int32_t *col_ptr, int32_t *row_idx, void *val_out,
                       spm_dtype out_type, int32_t *info, void *ws, size_t ws_bytes,
                       void *stream);

/* ------------------------------------------------------------------------------------------
 * Transpose X.t() (Table 1) as a CSC of the n_cols x n_rows result: the row index of A that
 * spm_csc_plan_build derives is the CSC of A^T, here written into separate arrays with the
 * values carried along (moved, not changed).
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Workspace of spm_csc_transpose. */
spm_status spm_csc_transpose_workspace(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                                       size_t *ws_bytes);

/* A^T of the CSC (col_ptr[n_cols+1], row_idx / val of capacity nnz_cap; nnz =
 * col_ptr[n_cols] is read on the device).
 *   val_type   F64 or F32, also the type of t_val.
 *   t_col_ptr  int32[n_rows + 1], fully written; t_row_idx / t_val have capacity nnz_cap,
 *              the first nnz entries are written (column r of A^T lists row r of A by
 *              increasing column).
 *   info       int32[2] as for spm_csc_plan_build (nnz; 0, SPM_EINVAL or SPM_EBOUNDS).
 *   ws         at least spm_csc_transpose_workspace() bytes, 256-byte aligned. */
spm_status spm_csc_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz_cap,
                             const int32_t *col_ptr, const int32_t *row_idx, const void *val,
                             spm_dtype val_type, int32_t *t_col_ptr, int32_t *t_row_idx,
                             void *t_val, int32_t *info, void *ws, size_t ws_bytes,
                             void *stream);

/* ------------------------------------------------------------------------------------------
 * trace(A^T B) of two CSC matrices of one shape without forming A^T or the product (Section 2's
 * example of an expression evaluated from its parts; Table 1): entry (j, j) of A^T B is the
 * dot product of column j of A with column j of B, so the trace is the sum, over locations
 * stored in both, of A[i,j] * B[i,j].  A location stored in only one matrix meets a structural
 * zero and adds nothing (an Inf or NaN there does not reach the result).
 * ------------------------------------------------------------------------------------------ */

/* Host only.  Workspace of spm_csc_trace_atb (about 16 bytes per 16 columns). */
spm_status spm_csc_trace_atb_workspace(int64_t n_cols, size_t *ws_bytes);

/* A and B: n_rows x n_cols CSCs (col_ptr[n_cols+1]; row_idx / val of capacity a_cap, b_cap),
 * rows strictly increasing down each column, as spm_coo_to_csc writes them.
 *   val_type  F64 or F32, the type of both a_val and b_val; products and sums in binary64.
 *   out       double[1] (device): the trace.
 *   info      int32[2] (device): info[0] = number of locations stored in both, info[1] = 0,
 *             SPM_EINVAL (offsets not starting at 0, decreasing or beyond the capacity, or
 *             rows not increasing in a column) or SPM_EBOUNDS (a stored row outside the
 *             matrix); on a nonzero status out is unspecified.
 *   ws        at least spm_csc_trace_atb_workspace() bytes, 256-byte aligned.
 * n_cols above 2^28 returns SPM_EOVERFLOW (one launch covers at most 2^32 lanes).
 * Summation order: in each column A's elements by increasing position, dealt round-robin to
 * 64 partial sums that combine by halving; columns in chunks of 16 added in order; the chunk
 * sums in a fixed two-level order.  The result depends on n_cols and the data only, never on
 * the tuning, and is within the a-priori bound of a dot product of the matched terms. */
spm_status spm_csc_trace_atb(int64_t n_rows, int64_t n_cols, int64_t a_cap,
                             const int32_t *a_col_ptr, const int32_t *a_row_idx,
                             const void *a_val, int64_t b_cap, const int32_t *b_col_ptr,
                             const int32_t *b_row_idx, const void *b_val, spm_dtype val_type,
                             double *out, int32_t *info, void *ws, size_t ws_bytes,
                             void *stream);

/* ------------------------------------------------------------------------------------------
 * Gradient with respect to each input triplet's value, for assembly (spm_coo_to_csc) followed
 * by Y = A . X and a loss with dL/dY = G.  A[r,c] is the sum of the values of the triplets at
 * (r, c) (the += of Fig. 1; a zero sum is only not stored), so every triplet t at (r, c) has
 *     dv[t] = sum_j G[r, j] * X[c, j],
 * shared by duplicates and defined also where the location summed to zero; a triplet outside
 * the matrix (skipped by assembly) gets 0.
 * ------------------------------------------------------------------------------------------ */

/* row, col  int32[nnz_in], the triplets' locations as given to assembly.
 * val_type  F64 or F32: the assembled values' type; it takes part in the accumulation rule
 *           of the adjoint (binary32 only when one of G and X is bfloat16 and none of the
 *           values, G and X is binary64; otherwise binary64).
 * G         n_rows x k of g_type, X n_cols x k of x_type (each F64, F32 or BF16, leading
 *           dimensions ldg, ldx >= k).
 * dv        nnz_in elements of dv_type (F64 or F32), rounded once.
 * Summation order: the adjoint's dvalues order (lane pieces of 4 in ascending order, then a
 * fixed lane tree that depends on k alone).  No workspace, no device status (a triplet out
 * of range is not an error here). */
spm_status spm_coo_triplet_grad(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                                const int32_t *row, const int32_t *col, spm_dtype val_type,
                                const void *G, int64_t ldg, spm_dtype g_type, const void *X,
                                int64_t ldx, spm_dtype x_type, void *dv, spm_dtype dv_type,
                                void *stream);

/* The same gradients read from the adjoint's dvalues (spm_csc_spmm_backward on the CSC that
 * assembly produced from these triplets: col_ptr, row_idx of capacity nnz_cap, dval of type
 * dval_type F64 or F32): a binary search in the triplet's column finds its slot p and
 * dv[t] = dval[p] (rounded to dv_type).  A triplet whose location is not stored (its values
 * summed to zero) gets the dot product as in spm_coo_triplet_grad, one outside the matrix 0.
 * Only dropped locations read rows of G and X, so this form costs a lookup per triplet. */
spm_status spm_coo_triplet_grad_csc(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                                    const int32_t *row, const int32_t *col, int64_t nnz_cap,
                                    const int32_t *col_ptr, const int32_t *row_idx,
                                    const void *dval, spm_dtype dval_type, spm_dtype val_type,
                                    const void *G, int64_t ldg, spm_dtype g_type,
                                    const void *X, int64_t ldx, spm_dtype x_type, void *dv,
                                    spm_dtype dv_type, void *stream);

/* ------------------------------------------------------------------------------------------
 * Batched path: many independent matrices assembled, planned, multiplied forward and
 * backward by launches on the stream: a persistent grouping launch (one workgroup per matrix
 * at a time, matrices taken from a device queue in the order given, largest first
 * recommended), then the products, as one grid over all rows (forward) and all columns
 * (adjoint) of all matrices.  When the workspace cannot hold the batch's row and column
 * prefixes (16 bytes per matrix), the products run one workgroup per matrix instead.
 * All per-matrix arrays are packed; item b describes where matrix b lives.  Element offsets
 * are in elements of the respective array.  For matrix b with nnz_in triplets:
 *   triplets       row/col/val[trip_off .. trip_off + nnz_in)
 *   CSC            col_ptr[colptr_off .. + n_cols + 1), row_idx/val_out[trip_off .. + nnz_in)
 *   plan           row_ptr[rowptr_off .. + n_rows + 1), col_t/perm[trip_off .. + nnz_in)
 *   dense          X and dX at x_off (n_cols x k, ld k), G and Y at g_off (n_rows x k, ld k)
 *   dval           dval[trip_off .. + nnz_in)
 *   info           info[2b] = nnz_out, info[2b + 1] = status of matrix b
 * Types: val_type F32 or BF16 (values assembled into F32), x_type (X and G) F32 or BF16;
 * val_out, Y, dX and dval are F32.  Each matrix's results are bitwise equal to what
 * spm_coo_to_csc + spm_csc_plan_build + spm_csc_spmm + spm_csc_spmm_backward give for it.
 * ------------------------------------------------------------------------------------------ */
typedef struct spm_batch_item {
  int32_t n_rows, n_cols, nnz_in, reserved;
  int64_t trip_off, colptr_off, rowptr_off, x_off, g_off;
} spm_batch_item;

/* Host only.  Workspace for a batch whose matrices all have n_rows, n_cols <= max_dim and
 * nnz_in <= max_nnz_in, run with `workers` persistent workgroups (0 = the library's choice,
 * which is also what spm_batch_run uses for 0). */
spm_status spm_batch_workspace(int64_t max_dim, int64_t max_nnz_in, int32_t workers,
                               size_t *ws_bytes);

/* Host only.  Longest-processing-time-first order of the items (host arrays): order[i] is
 * the index of the i-th matrix to start; cost is estimated from nnz_in, n and k. */
spm_status spm_batch_schedule(const spm_batch_item *items_host, int32_t batch, int64_t k,
                              int32_t *order_host);

/* Run the whole batch.  items and order are device copies (batch entries each); items whose
 * sizes exceed max_dim / max_nnz_in get info status SPM_EINVAL and are skipped. */
spm_status spm_batch_run(int32_t batch, int64_t k, const spm_batch_item *items,
                         const int32_t *order, const int32_t *row, const int32_t *col,
                         const void *val, spm_dtype val_type, const void *X, const void *G,
                         spm_dtype x_type, int32_t *col_ptr, int32_t *row_idx, float *val_out,
                         int32_t *row_ptr, int32_t *col_t, int32_t *perm, float *Y, float *dX,
                         float *dval, int32_t *info, int64_t max_dim, int64_t max_nnz_in,
                         int32_t workers, void *ws, size_t ws_bytes, void *stream);

/* spm_batch_run with the named tuning tune_key (spm_tuning_register) in effect for this call
 * only (NULL: the tuning already in effect; SPM_EINVAL for an unknown key, nothing enqueued). */
spm_status spm_batch_coo_to_csc_spmm(int32_t batch, int64_t k, const spm_batch_item *items,
                                     const int32_t *order, const int32_t *row,
                                     const int32_t *col, const void *val, spm_dtype val_type,
                                     const void *X, const void *G, spm_dtype x_type,
                                     int32_t *col_ptr, int32_t *row_idx, float *val_out,
                                     int32_t *row_ptr, int32_t *col_t, int32_t *perm, float *Y,
                                     float *dX, float *dval, int32_t *info, int64_t max_dim,
                                     int64_t max_nnz_in, int32_t workers, void *ws,
                                     size_t ws_bytes, const char *tune_key, void *stream);

/* ------------------------------------------------------------------------------------------
 * Tuning.  Launch-shape parameters that never change results (see Numerics above): they
 * decide how work is cut into workgroups, never the order in which any output is summed.
 * spm_tuning_set validates and copies process-wide values (host only); named tunings below
 * give a thread or a call values of its own.  The grouping parameters change the workspace
 * sizes that spm_coo_to_csc_workspace and spm_csc_plan_size report: ask for sizes after
 * setting the tuning (a call made with a smaller workspace fails with SPM_EWORKSPACE, it never
 * overruns).
 * ------------------------------------------------------------------------------------------ */
typedef struct spm_tuning {
  int32_t spmm_block;          /* threads per workgroup of the forward / backward kernels:
                                  64, 128 or 256 */
  int32_t spmm_blocks_per_cu;  /* forward / backward grid cap, in workgroups per compute unit
                                  (1..64); rows or columns beyond it are strided */
  int32_t batch_wg_per_cu;     /* persistent batched workgroups per compute unit (1..8) */
  int32_t part_bucket_target;  /* assembly / plan grouping: target elements per coarse bucket
                                  (256..2048, power of two) */
  int32_t part_max_tiles;      /* assembly / plan grouping: at most this many first-level
                                  tiles (64..4096, power of two) */
  int32_t batch_spmm_wg_per_cu; /* persistent workgroups per compute unit of the batch's
                                   products launch (1..32; 0 = the library's default, 8) */
  int32_t trace_group_width;   /* lanes per column of spm_csc_trace_atb: 16, 32 or 64
                                  (0 = chosen from the average column length) */
  int32_t reserved;
} spm_tuning;

/* The tuning in effect for the calling thread (its selection, else the process-wide values). */
spm_status spm_tuning_get(spm_tuning *out);
/* Set the process-wide values (SPM_EINVAL for a value outside the ranges above). */
spm_status spm_tuning_set(const spm_tuning *in);

/* Named tunings ("tune keys"), so that callers with different shapes in one process do not
 * share one mutable setting: spm_tuning_register stores a validated copy under key (replacing
 * an earlier one); spm_tuning_select makes it the calling thread's tuning for every later call
 * from that thread (NULL: back to the process-wide values; SPM_EINVAL for an unknown key).
 * Workspace sizes follow the tuning in effect, as above. */
spm_status spm_tuning_register(const char *key, const spm_tuning *in);
spm_status spm_tuning_select(const char *key);

#ifdef __cplusplus
}
#endif

#endif /* SPM_H */
