/*
 * csrk.h — C ABI of the CSR-k sparse matrix-vector library for AMD Instinct
 * MI355X (gfx950).
 *
 * The operation is y = A x for a square sparse matrix A held in CSR-k form
 * (Lane & Booth, "Heterogeneous Sparse Matrix-Vector Multiplication via
 * Compressed Sparse Row Format"): plain CSR arrays (row_ptr, col_idx, vals;
 * Section 2.1) of the reordered matrix plus two pointer arrays, sr_ptr
 * (running count of rows per super-row) and ssr_ptr (running count of
 * super-rows per super-super-row) (Section 2.2, Fig. 1).  The library builds
 * the reordering and grouping on the host (Band-k, Section 2.2), picks the
 * group sizes with a constant-time model (Section 4.1), and runs the product,
 * its adjoint and batched multi-right-hand-side forms in HIP kernels.
 *
 * Conventions shared by every call:
 *  - Every call returns a csrk_status and never throws across the ABI.  On
 *    failure csrk_last_error_detail() returns a thread-local text.
 *  - Indices are 32-bit (Section 2.1): n < 2^31 and nnz < 2^31.
 *  - "perm" maps reordered to input rows: perm[new] = old.  The reordered
 *    matrix is A' = P A P^T, A'[i', j'] = A[perm[i'], perm[j']].  Vectors in
 *    "permuted space" are indexed by reordered rows: x'[i'] = x[perm[i']].
 *  - Device pointers are HIP device addresses; streams are hipStream_t passed
 *    as void* (NULL = the default stream).  Device calls are enqueued
 *    asynchronously on that stream and never synchronise implicitly.
 *  - Blocks of right-hand sides are row-major n x nrhs.
 *  - A handle's structure is immutable after it is built; concurrent device
 *    calls on one handle from different streams are safe.  csrk_set_launch
 *    and csrk_destroy must not overlap calls still in flight (synchronise the
 *    stream first).
 */
#ifndef CSRK_H
#define CSRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum csrk_status {
    CSRK_OK = 0,
    CSRK_ERR_ARG = 1,          /* bad argument: null pointer, size <= 0 where forbidden, bad enum, misaligned pointer */
    /* 2 is not used: a matrix is given by its n rows and columns in [0, n), so a
       non-square input shows up as CSRK_ERR_COL_RANGE */
    CSRK_ERR_BAD_ROWPTR = 3,   /* row_ptr[0] != 0, decreasing, or row_ptr[n] != nnz */
    CSRK_ERR_COL_RANGE = 4,    /* a column index outside [0, n) */
    CSRK_ERR_DUPLICATE = 5,    /* the same column twice in one row */
    CSRK_ERR_ALLOC = 6,        /* host or device allocation failed */
    CSRK_ERR_DEVICE = 7,       /* a HIP runtime error, or no GPU */
    CSRK_ERR_UNSUPPORTED = 8   /* valid but not supported (e.g. device call on a host-only handle) */
} csrk_status;

/* Storage type of the matrix values.  F64 pairs with FP64 vectors and FP64
 * accumulation; F32 and BF16 pair with FP32 vectors and FP32 accumulation. */
/* Rows with more nonzeros than this are computed by a workgroup of their own
 * instead of by their super-row's wavefront (see csrk_info.long_rows). */
#define CSRK_LONG_ROW 1024

typedef enum csrk_dtype { CSRK_F64 = 0, CSRK_F32 = 1, CSRK_BF16 = 2 } csrk_dtype;

/* Size models.  VOLTA and AMPERE are the paper's fitted GPU formulas (Section
 * 4.1); MI355X is this library's fit of the same form for gfx950; HOST_CPU is
 * the paper's constant-time CPU choice (Section 4.2): CSR-2 with SRS = 96 for
 * every matrix, the fallback when the matrix is not tuned individually. */
typedef enum csrk_model {
    CSRK_MODEL_MI355X = 0,
    CSRK_MODEL_VOLTA = 1,
    CSRK_MODEL_AMPERE = 2,
    CSRK_MODEL_HOST_CPU = 3
} csrk_model;

/* Row orderings: Band-k (Section 2.2; this library's deterministic reading),
 * reverse Cuthill-McKee of the symmetrised pattern, or the input order. */
typedef enum csrk_reorder { CSRK_REORDER_BANDK = 0, CSRK_REORDER_RCM = 1, CSRK_REORDER_NONE = 2 } csrk_reorder;

/* Tuning parameters.  srs = rows per super-row (SRS), ssrs = super-rows per
 * super-super-row (SSRS) (Section 4.1).  lanes_per_row (1, 2, 4, ..., 64) is
 * the number of wavefront lanes that reduce one row; waves_per_wg (1..16) the
 * wavefronts per workgroup.  k is the number of CSR-k levels, 2..8 (Section
 * 2.2 defines CSR-k for every k >= 2): k - 1 grouping levels above the rows.
 * k = 3 (CSR-3): super-rows and super-super-rows.  k = 2 (CSR-2): one
 * coarsening level, Band-k orders the coarse graph by reverse Cuthill-McKee;
 * the super-rows are then grouped ssrs at a time in order for the launch,
 * which is what ssr_ptr holds for k = 2.  k >= 4: every level above the
 * super-row groups ssrs units of the level below (this library's reading; the
 * paper sizes only k <= 3), Band-k coarsens k - 1 times; the GPU kernels use
 * the super-row and super-super-row levels, csrk_level_ptr gives the others. */
typedef struct csrk_params {
    int32_t k;
    int32_t srs;
    int32_t ssrs;
    int32_t lanes_per_row;
    int32_t waves_per_wg;
    int32_t reorder;  /* csrk_reorder */
} csrk_params;

/* Statistics of a built handle (Section 5.3 and Table 1 quantities). */
typedef struct csrk_info {
    int32_t n;
    int64_t nnz;
    int32_t nsr;              /* number of super-rows */
    int32_t nssr;             /* number of super-super-rows */
    double rdensity;          /* nnz / n (Section 4.1) */
    double row_variance;      /* variance of nonzeros per row (Section 5.3) */
    int32_t max_row;          /* maximum nonzeros in a row (Table 1 MAX) */
    int32_t bandwidth_input;  /* max |i - j| of the input */
    int32_t bandwidth;        /* max |i - j| after reordering */
    double symmetry;          /* fraction of off-diagonal entries whose mirror is stored (Table 1 SY) */
    int32_t max_sr_nnz;       /* largest nonzero count of a super-row */
    int32_t max_ssr_rows;     /* largest row count of a super-super-row */
    int32_t on_device;        /* 1 when device arrays exist */
    int32_t store;            /* csrk_dtype of the device values (valid when on_device) */
    int32_t long_rows;        /* rows with more than CSRK_LONG_ROW nonzeros: each is computed
                                 by a workgroup of its own (Section 7 names computing
                                 dense rows in parallel as the fix for irregular matrices) */
    int32_t values_symmetric; /* 1 when uploaded and A' equals A'^T exactly: the adjoint then
                                 reads the forward's values instead of a transposed copy */
    csrk_params params;
    int32_t adjoint_union;    /* 1 when uploaded with a nonsymmetric pattern whose union
                                 pattern (A' + A'^T) fits the staging windows: the
                                 adjoint (one or several right-hand sides) then takes both
                                 gradients in one pass over the union instead of a pass
                                 over A' and one over A'^T */
} csrk_info;

typedef struct csrk_matrix *csrk_handle;
typedef struct csrk_batch_s *csrk_batch;

/* Text of a status code (static storage). */
const char *csrk_status_string(csrk_status s);

/* Thread-local detail of the last failure on this thread ("" if none). */
const char *csrk_last_error_detail(void);

/*
 * csrk_tune — constant-time choice of the tuning parameters from n and nnz
 * alone (rdensity = nnz / n; Section 4.1).  VOLTA/AMPERE reproduce the
 * paper's formulas: round-half-up logarithmic fits and the per-case
 * adjustments, "SRSS" read as SSRS, results clamped to >= 1.  MI355X uses
 * this library's constants of the same form.  HOST_CPU gives k = 2,
 * srs = 96, ssrs = 1 (each super-row is one unit of the host kernel's
 * parallel loop; Section 4.2) for any n and nnz.  O(1), no allocation.
 * Errors: CSRK_ERR_ARG for n <= 0, nnz <= 0, unknown model or out == NULL.
 */
csrk_status csrk_tune(int64_t n, int64_t nnz, csrk_model model, csrk_params *out);

/*
 * csrk_tune_rhs — csrk_tune for a matrix that will be multiplied by blocks
 * of nrhs right-hand sides (nrhs >= 1; nrhs == 1 is csrk_tune).  The paper's
 * model is for one vector (Section 4.1); for nrhs > 1 the MI355X model halves
 * its SRS (snapped to the {2^i, 1.5 * 2^i} set) and sets SSRS = waves per
 * workgroup = 4, this library's measurement on the multi-right-hand-side
 * kernels (a batch of 64 7-point matrices with 8 right-hand sides, one
 * workgroup per work item: forward + adjoint 1.24 ms at (SRS 32, SSRS 4)
 * against 1.34 ms at (64, 8) and 1.88 ms at (16, 2)).  VOLTA/AMPERE ignore
 * nrhs.
 * Errors: as csrk_tune, and CSRK_ERR_ARG for nrhs < 1.
 */
csrk_status csrk_tune_rhs(int64_t n, int64_t nnz, int32_t nrhs, csrk_model model, csrk_params *out);

/*
 * csrk_build_host — validate the CSR input, build the symmetrised graph,
 * reorder (Band-k / RCM / none), apply the symmetric permutation (columns
 * sorted within rows) and form sr_ptr / ssr_ptr (Section 2.2).  Host only: no
 * HIP call.  row_ptr[n+1], col_idx[nnz] and vals[nnz] are borrowed for the
 * call and copied.  vals holds nnz values of in_dtype (F64: double, F32:
 * float, BF16: the 16-bit patterns as uint16_t), or is NULL for a
 * pattern-only build (values then 0).  The host keeps the values in FP64;
 * FP32 and BF16 inputs widen exactly, so a later upload in the input's own
 * type reproduces them bit for bit.
 * Columns may be unsorted within a row; duplicates are rejected.  p == NULL
 * uses csrk_tune(n, nnz, CSRK_MODEL_MI355X).  The result is deterministic:
 * the same input gives a bit-identical structure.
 * Irregular matrices: after the grouping, a super-row whose nonzeros (rows
 * longer than CSRK_LONG_ROW not counted) exceed the budget
 * B = max(2048, ceil(4 * SRS * nnz / n)) is cut greedily into consecutive
 * pieces of at most B, each piece becoming a super-row; the pieces of a
 * super-super-row are regrouped SSRS at a time.  A regular matrix (no
 * super-row above B) keeps the plain grouping.  This is this library's
 * extension: the paper leaves load balance on irregular matrices as future
 * work (Section 7).
 * Errors: CSRK_ERR_ARG (also for an unknown in_dtype), CSRK_ERR_BAD_ROWPTR,
 * CSRK_ERR_COL_RANGE, CSRK_ERR_DUPLICATE, CSRK_ERR_ALLOC.
 */
csrk_status csrk_build_host(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                            const void *vals, csrk_dtype in_dtype, const csrk_params *p, csrk_handle *out);

/*
 * csrk_build_from_groups — like csrk_build_host but with a caller-given
 * ordering perm[n] (perm[new] = old) and grouping: nsr super-rows of
 * sr_sizes[s] >= 1 rows each (sum = n) and nssr super-super-rows of
 * ssr_sizes[t] >= 1 super-rows each (sum = nsr).  This is how uneven groups
 * such as those of Fig. 1 are expressed.  p->k must be 2 or 3 here (the
 * caller gives two levels); CSRK_ERR_ARG otherwise.
 */
csrk_status csrk_build_from_groups(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                   const void *vals, csrk_dtype in_dtype, const int32_t *perm, int32_t nsr,
                                   const int32_t *sr_sizes, int32_t nssr, const int32_t *ssr_sizes,
                                   const csrk_params *p, csrk_handle *out);

/*
 * csrk_upload — copy a host-built handle's arrays to the current HIP device
 * and convert the values to `store` there (FP64 -> FP32 round to nearest
 * even; BF16 = BF16(FP32(v)), both steps round to nearest even).  Synchronous.
 * Calling it again replaces the device copy.  Errors: CSRK_ERR_DEVICE,
 * CSRK_ERR_ALLOC, CSRK_ERR_ARG.
 */
csrk_status csrk_upload(csrk_handle h, csrk_dtype store);

/* csrk_build = csrk_build_host followed by csrk_upload(store).  On failure
 * *out is NULL and nothing is left allocated. */
csrk_status csrk_build(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const void *vals,
                       csrk_dtype in_dtype, csrk_dtype store, const csrk_params *p, csrk_handle *out);

/*
 * csrk_set_launch — change the kernel launch shape of a built handle
 * (lanes_per_row: 1, 2, 4, ..., 64; waves_per_wg: 1..16) without rebuilding
 * its structure: the shape does not affect the ordering or grouping.  Used by
 * the autotuner.  Must not overlap device calls on the same handle.
 * Errors: CSRK_ERR_ARG.
 */
csrk_status csrk_set_launch(csrk_handle h, int32_t lanes_per_row, int32_t waves_per_wg);

/* Statistics and parameters of a handle. */
csrk_status csrk_get_info(csrk_handle h, csrk_info *out);

/*
 * csrk_level_ptr — the pointer array of grouping level `level` (Section 2.2,
 * Fig. 1): level 1 = sr_ptr (rows per super-row), level 2 = ssr_ptr
 * (super-rows per super-super-row), level l >= 3 (k >= 4) = running counts of
 * level-(l-1) units per level-l unit.  Valid levels: 1 .. max(2, k - 1).
 * *count receives the number of level-l units; out, if not NULL, must hold
 * *count + 1 entries and receives the array.  Host only.
 * Errors: CSRK_ERR_ARG (null handle or count, level out of range).
 */
csrk_status csrk_level_ptr(csrk_handle h, int32_t level, int32_t *count, int32_t *out);

/*
 * csrk_copy_union — the union-pattern index a nonsymmetric A' gets for its
 * one-pass adjoint (built on the host with the structure; see adjoint_union
 * in csrk_info).  *nu receives the number of union entries, padding included
 * (0 when the pattern is symmetric or some super-row has more than 64 rows or
 * more than 504 union entries: then the adjoint walks A' and A'^T).  Super-row
 * s owns union entries [sr_begin[s], sr_end[s]): its A' entries in A' order
 * (u_col = their columns), then its rows' extras, the columns j with (j, i) in
 * A' but (i, j) not, row by row by increasing column; each super-row's extras
 * are padded (column = its first row, source -1) to a multiple of 8.  u_src
 * gives the position in A' of the mirror entry (j, i) of union entry (i, j),
 * -1 where A' has none; erow_ptr[n+1] counts extras before each row (no
 * padding).  Buffers: u_col[nu], u_src[nu], erow_ptr[n+1], sr_begin[nsr],
 * sr_end[nsr]; any may be NULL.  Host only.  Errors: CSRK_ERR_ARG.
 */
csrk_status csrk_copy_union(csrk_handle h, int64_t *nu, int32_t *u_col, int32_t *u_src, int32_t *erow_ptr,
                            int32_t *sr_begin, int32_t *sr_end);

/*
 * csrk_copy_structure — copy the host structure into caller buffers; any
 * pointer may be NULL.  perm[n], row_ptr[n+1], col_idx[nnz] and vals[nnz]
 * (FP64 master values) describe A' as plain CSR, which is what keeps CSR-k
 * readable by any CSR consumer (Section 2.2); vmap[nnz] gives the input
 * position of each entry of A'; sr_ptr[nsr+1], ssr_ptr[nssr+1].
 */
csrk_status csrk_copy_structure(csrk_handle h, int32_t *perm, int32_t *row_ptr, int32_t *col_idx, double *vals,
                                int64_t *vmap, int32_t *sr_ptr, int32_t *ssr_ptr);

/*
 * csrk_device_vals — the handle's device value array (nnz entries of the
 * storage type, CSR-k order, 16-byte aligned).  Owned by the handle and
 * meant to be read (e.g. copied as the initial value tensor): the adjoint
 * with the handle's own values uses a transposed copy made at upload (or
 * this same array when the matrix is symmetric), so values written here
 * reach csrk_spmv but not csrk_spmv_adjoint; pass changed values to both
 * calls through their vals_dev argument instead.
 */
csrk_status csrk_device_vals(csrk_handle h, void **vals_dev);

/*
 * csrk_copy_device_vals — enqueue on `stream` a device-to-device copy of the
 * handle's stored values (nnz entries of the storage type, CSR-k order) into
 * the caller's buffer dst_dev (at least nnz * element size bytes, caller
 * owned).  Asynchronous like the products.  Errors: CSRK_ERR_ARG (null
 * handle or destination), CSRK_ERR_UNSUPPORTED (host-only handle),
 * CSRK_ERR_DEVICE.
 */
csrk_status csrk_copy_device_vals(csrk_handle h, void *dst_dev, void *stream);

/*
 * csrk_spmv — y' = A' x' (Section 1 statement of SpMV on the CSR-k arrays;
 * one super-super-row per workgroup, one super-row per wavefront, Section 3).
 * vals_dev: NULL = the handle's values, else nnz values of the storage type
 * in CSR-k order (16-byte aligned).  x_dev, y_dev: n x nrhs row-major in
 * permuted space; FP64 for F64 storage, FP32 otherwise.  y must not alias x.
 * Rows without nonzeros give 0.  nrhs >= 1.  Errors: CSRK_ERR_ARG,
 * CSRK_ERR_UNSUPPORTED (host-only handle), CSRK_ERR_DEVICE (launch failure).
 */
csrk_status csrk_spmv(csrk_handle h, const void *vals_dev, const void *x_dev, void *y_dev, int32_t nrhs,
                      void *stream);

/*
 * csrk_spmv_plain — the same product with a plain CSR kernel that ignores the
 * super-row levels (rows spread over the grid in fixed-size blocks).  The
 * baseline against which CSR-k is measured; same arguments as csrk_spmv.
 */
csrk_status csrk_spmv_plain(csrk_handle h, const void *vals_dev, const void *x_dev, void *y_dev, int32_t nrhs,
                            void *stream);

/*
 * csrk_spmv_host — the product on the host CPU over the same handle (the
 * paper's CPU kernel, Section 2.2 listing): super-super-rows in parallel
 * (OpenMP, static schedule), then their super-rows, then their rows, each row
 * summed left to right in FP64.  x (n doubles) and y (n doubles) are host
 * arrays in permuted space; values are the handle's FP64 master copy.
 * nthreads <= 0 uses the OpenMP default.  Needs no device.  Errors:
 * CSRK_ERR_ARG for a null handle or pointer.
 */
csrk_status csrk_spmv_host(csrk_handle h, const double *x, double *y, int32_t nthreads);

/*
 * csrk_cg — conjugate gradients for A' x' = b' (A' symmetric positive
 * definite), the iterative-solver use the paper names for the format
 * (Section 1 and the conclusions).  Each iteration is one CSR-k product in
 * the handle's storage precision (FP32 copies of the direction vector feed
 * FP32/BF16 storage) plus FP64 vector updates; x', r', p' and every
 * reduction are FP64 and reduced in a fixed order, so the iteration is
 * reproducible.  b_dev (n doubles) and x_dev (n doubles, the initial guess
 * on entry, the solution on exit) are device arrays in permuted space.  Stops
 * when ||r||_2 <= rtol * ||b||_2 (r the recurrence residual, checked every
 * check_every iterations) or after max_iter iterations; *iters_out and
 * *rel_resid_out (both may be NULL) receive the iteration count and
 * ||r||_2 / ||b||_2.  Allocates, for the call, one device block holding 3
 * work vectors (4 with FP32/BF16 storage) and one FP64 partial sum per
 * workgroup of the product (p'Ap is summed by the product's own workgroups),
 * and synchronises
 * `stream` before returning.  Errors: CSRK_ERR_ARG (null
 * vectors, rtol <= 0, max_iter < 0, check_every < 1), CSRK_ERR_UNSUPPORTED on
 * a breakdown (p'A p <= 0: the stored matrix is not positive definite),
 * CSRK_ERR_ALLOC, CSRK_ERR_DEVICE.
 */
csrk_status csrk_cg(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter,
                    int32_t check_every, void *stream, int32_t *iters_out, double *rel_resid_out);

/*
 * csrk_cg_noalloc — csrk_cg for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, hosts that forbid
 * allocation during a solve).  Same arguments, iteration, results and errors
 * as csrk_cg, bit for bit, but the work vectors, partial sums and scalars live
 * in one fixed array of CSRK_CG_NOALLOC_BYTES bytes per device, owned by the
 * library, created when the library's code is loaded on the device and held
 * until the process ends; the call makes no device allocation or free.
 * csrk_cg_noalloc_bytes reports the work memory a handle needs (3 or 4
 * vectors of n entries, one FP64 partial sum per workgroup of the product,
 * rounded to 256-byte boundaries); a handle that needs more than
 * CSRK_CG_NOALLOC_BYTES (FP64 and FP32/BF16 storage alike: about
 * 2.7 million rows) is rejected with CSRK_ERR_ARG before any device work.
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (different host threads, or different streams) race and
 * give wrong results; the caller orders them.  The array keeps the last
 * call's contents; nothing in it needs clearing, since each solve writes every
 * work entry before reading it.  Synchronises `stream` before returning.
 */
#define CSRK_CG_NOALLOC_BYTES (64ll << 20)
csrk_status csrk_cg_noalloc_bytes(csrk_handle h, int64_t *bytes_out);
csrk_status csrk_cg_noalloc(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter,
                            int32_t check_every, void *stream, int32_t *iters_out, double *rel_resid_out);

/*
 * csrk_spmv_adjoint — gradients of L = <g', A' x'> (not in the paper):
 * grad_x' = A'^T g' (n x nrhs, same type as x) and grad_vals'[k] =
 * sum_c g'[row(k), c] x'[col(k), c] (nnz values in CSR-k order, FP64 for F64
 * storage, FP32 otherwise).  Either output may be NULL to skip it.  No
 * atomics: grad_x is computed row by row over the transposed index structure
 * built at upload, so both outputs are the same on every run.  Same errors
 * as csrk_spmv.
 */
csrk_status csrk_spmv_adjoint(csrk_handle h, const void *vals_dev, const void *x_dev, const void *g_dev,
                              void *grad_x_dev, void *grad_vals_dev, int32_t nrhs, void *stream);

/*
 * csrk_permute — move a vector block between input and permuted space:
 * direction 0: out[i', c] = in[perm[i'], c] (to permuted space);
 * direction 1: out[perm[i'], c] = in[i', c] (back to input order).
 * elem_bytes is 4 or 8.  in and out must not alias.
 */
csrk_status csrk_permute(csrk_handle h, int32_t direction, const void *in_dev, void *out_dev, int32_t nrhs,
                         int32_t elem_bytes, void *stream);

/* Free the handle and its host and device memory. */
csrk_status csrk_destroy(csrk_handle h);

/*
 * Batched forms (not in the paper): many matrices of uneven size, each with
 * an n_b x nrhs block, in one launch over a work list of
 * (matrix, super-super-row) items.  All handles must be on the device with
 * the same storage type; they must outlive the batch.  The batch owns the
 * work list and one device pointer table per direction, rewritten on the
 * call's stream when the pointers change: calls on one batch from different
 * streams (or host threads) must be ordered by the caller, or the table can
 * change under a launch still reading it.  The work list is cut into one
 * contiguous range per workgroup, with 16 workgroups per CU or more.
 */
csrk_status csrk_batch_create(const csrk_handle *handles, int32_t count, csrk_batch *out);

/* y_b = A_b x_b for every b.  vals/x/y are arrays of `count` device pointers
 * (vals may be NULL, or hold NULL entries, for the handles' own values). */
csrk_status csrk_batch_spmv(csrk_batch b, const void *const *vals, const void *const *x, void *const *y, int32_t nrhs,
                            void *stream);

/* Adjoint of every product of the batch; grad_x / grad_vals arrays may be NULL. */
csrk_status csrk_batch_spmv_adjoint(csrk_batch b, const void *const *vals, const void *const *x, const void *const *g,
                                    void *const *grad_x, void *const *grad_vals, int32_t nrhs, void *stream);

/*
 * csrk_batch_set_launch — launch shape of a batch's kernels: at least
 * blocks_per_cu workgroups per compute unit in the grid, each taking a
 * contiguous range of (matrix, super-super-row) items (0 = the library's
 * default: one workgroup per item), and waves_per_wg wavefronts per
 * workgroup (0 = keep the first handle's).  The grouping of the matrices is not changed.  Used by the
 * autotuner.  Must not overlap calls in flight on the batch.
 * Errors: CSRK_ERR_ARG (null batch, blocks_per_cu outside 0..256,
 * waves_per_wg outside 0..16).
 */
csrk_status csrk_batch_set_launch(csrk_batch b, int32_t blocks_per_cu, int32_t waves_per_wg);

csrk_status csrk_batch_destroy(csrk_batch b);

/*
 * Bandwidth probes (measurement aids, not part of the product): the HBM rate
 * attainable on the device, against which the products' achieved rates are
 * read (Section 1 explains why SpMV is bound by memory bandwidth).
 * csrk_probe_read streams `bytes` of device memory (a multiple of 16, buf_dev
 * 16-byte aligned) with 16-byte non-temporal loads and writes 4096 doubles of
 * checksum to part_dev (caller owned); csrk_probe_copy copies `bytes` from
 * src_dev to dst_dev (both 16-byte aligned, not overlapping) with 16-byte
 * non-temporal loads and stores.  Asynchronous on `stream`.  Errors:
 * CSRK_ERR_ARG, CSRK_ERR_DEVICE.
 */
csrk_status csrk_probe_read(const void *buf_dev, int64_t bytes, double *part_dev, void *stream);
csrk_status csrk_probe_copy(const void *src_dev, void *dst_dev, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CSRK_H */
