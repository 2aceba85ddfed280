// Launchers of the gfx950 kernels (device/forward.hip, adjoint.hip, batch.hip,
// util.hip, cg.hip).  C++ linkage, used only by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../../include/csrk.h"

namespace csrk {
namespace dev {

// Rows with more nonzeros than this are computed by a workgroup of their own
// (split over its wavefronts) instead of by their super-row's wavefront; the
// handle lists them at upload.
constexpr int32_t kLongRow = CSRK_LONG_ROW;

// A nonsymmetric pattern gets a union-pattern index (one-pass adjoint) when
// every super-row has at most kUnionRows rows and at most kUnionWindow union
// entries: one wavefront's staging window (512 entries) less one load step of
// the widest entry group (8), as the window walk requires.
constexpr int32_t kUnionRows = 64;
constexpr int32_t kUnionWindow = 512 - 8;

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin
// by block index.  SSR block b (counted after the long-row blocks, a multiple
// of 8 of them) runs super-super-row b[b % 8] + b / 8 of XCD b % 8's
// contiguous range [b[x], b[x+1]); blocks past the end of their range exit at
// once.  The ranges are cut so that each XCD gets about the same work.
constexpr int kXcds = 8;
struct XcdSplit {
    int32_t b[kXcds + 1] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t width = 0;  // largest range: the grid is width * kXcds blocks
};

// Bounds of one super-row: rows [r0, r1) and their entries [e0, e1).  The
// handle keeps one record per (super-super-row, slot), slot w < stride holding
// the SSR's w-th super-row (empty records, r0 == r1, pad short SSRs), so a
// workgroup finds its super-rows' rows and entries with one load instead of
// the chain ssr_ptr -> sr_ptr -> row_ptr.
struct __attribute__((aligned(16))) SrRec {
    int32_t r0, r1, e0, e1;
};

// Device arrays of one CSR-k matrix.
struct Arrays {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t nsr = 0;
    int32_t nssr = 0;
    const int32_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const int32_t *sr_ptr = nullptr;
    const int32_t *ssr_ptr = nullptr;
    const int32_t *perm = nullptr;
    // A'^T: row j lists column j of A' by increasing row (t_col) with each
    // entry's position in A' (t_src).  For a symmetric pattern t_row_ptr and
    // t_col are row_ptr and col_idx.
    const int32_t *t_row_ptr = nullptr;
    const int32_t *t_col = nullptr;
    const int32_t *t_src = nullptr;
    const void *vals_t = nullptr;  // the handle's values in A'^T order (aligned with t_col)
    bool sym = false;              // pattern of A' is symmetric: A'^T has the pattern of A'
    // Rows of A' (long_rows) and of A'^T (t_long_rows) longer than kLongRow,
    // ascending; for a symmetric pattern the two lists are the same.
    const int32_t *long_rows = nullptr;
    int32_t nlong = 0;
    const int32_t *t_long_rows = nullptr;
    int32_t t_nlong = 0;
    XcdSplit split_fwd;  // by the forward's work (rows of A')
    XcdSplit split_adj;  // by the adjoint's work (rows of A' and of A'^T)
    int32_t max_row = 0;  // longest row of A' or of A'^T (nonzeros)
    const SrRec *srec = nullptr;    // nssr * srec_stride super-row records
    const SrRec *srec_t = nullptr;  // the same rows of A'^T (entries of t_row_ptr); == srec if symmetric
    int32_t srec_stride = 0;        // most super-rows in one super-super-row
    // Union pattern of a nonsymmetric A' (host union_index): per super-row its
    // A' entries, then its rows' extras (entries of A'^T missing from A'),
    // each U entry (i, j) carrying a'_ji.  Present (srec_u != nullptr) only
    // when every super-row fits one staging window; the single-right-hand-side
    // adjoint then takes both gradients in one pass over it.
    const int32_t *u_col = nullptr;
    const int32_t *u_src = nullptr;  // position of a'_ji in A', -1 where A' has no (j, i) (value 0)
    const void *u_vals = nullptr;    // the handle's values a'_ji in U order (0 where u_src is -1)
    const int32_t *erow_ptr = nullptr;  // extras of the rows before row i
    const SrRec *srec_u = nullptr;      // per (SSR, slot): rows [r0, r1), U entries [e0, e1)
    int64_t nu = 0;                     // U entries (with padding)
};

// Per-matrix record of a batched launch (device-resident table).
struct MatDesc {
    const int32_t *ssr_ptr;
    const int32_t *sr_ptr;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const int32_t *t_row_ptr;
    const int32_t *t_col;
    const int32_t *t_src;
    const void *vals;
    const void *x;
    void *y;
    const void *g;
    void *gx;
    void *gv;
    int64_t nnz;
    int32_t n;
    int32_t nssr;
    int32_t sym;
    int32_t uni;  // the matrix has a union-pattern index (Arrays::u_col ...): the adjoint takes one pass
    const int32_t *u_col;
    const int32_t *u_src;
    const int32_t *erow_ptr;
    const void *u_vals;
    int64_t nu;
};

// Kernel-shape knobs: lanes per row in the reduction, wavefronts per workgroup.
struct Shape {
    int lanes_per_row = 1;
    int waves = 4;
};

// y = A'x (one right-hand side) and part[w] = the partial sum of y_i pdot_i
// over workgroup w's rows, for w < spmv_grid(a) (CG's p . Ap; FP64).
int spmv_grid(const Arrays &a);
hipError_t spmv_dot(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, const double *pdot,
                    double *part, Shape s, hipStream_t st);

hipError_t spmv(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, int nrhs, Shape s,
                hipStream_t st);
hipError_t spmv_plain(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, int nrhs,
                      Shape s, hipStream_t st);
hipError_t adjoint(const Arrays &a, csrk_dtype store, const void *vals, const void *x, const void *g, void *gx,
                   void *gv, int nrhs, Shape s, hipStream_t st);
// vals_t[p] = vals[t_src[p]]: the values in A'^T order.
hipError_t transpose_values(const Arrays &a, csrk_dtype store, const void *vals, void *vals_t, hipStream_t st);
// out[p] = vals[idx[p]] (0 where idx[p] < 0) for p < count, storage type `store`.
hipError_t gather_values(const int32_t *idx, int64_t count, csrk_dtype store, const void *vals, void *out,
                         hipStream_t st);
hipError_t permute(const Arrays &a, int dir, const void *in, void *out, int nrhs, int elem_bytes, hipStream_t st);
hipError_t convert_values(const double *src, void *dst, int64_t count, csrk_dtype store, hipStream_t st);

// Batched launches: one grid over `nitems` (matrix, super-super-row) items.
// `vec`: every right-hand-side block pointer is 16-byte aligned.
// `brec`: per item, `stride` super-row records (SrRec) of its SSR.
hipError_t batch_forward(const MatDesc *descs, const int2 *items, const SrRec *brec, int32_t stride, int32_t nitems,
                         csrk_dtype store, int nrhs, Shape s, int grid, bool vec, hipStream_t st);
// `ind`: the descriptors' vals are caller values in CSR-k order (reached
// through t_src); otherwise they are the handles' transposed copies.
// `all_sym`: every matrix of the batch has a symmetric pattern; `both`: both
// gradients are wanted (then a multi-right-hand-side launch with FP32
// accumulation runs the fused-only kernel).
// `brec_u`: per item, the same slots' union-pattern records (for matrices
// with uni set; other slots repeat brec).
hipError_t batch_adjoint(const MatDesc *descs, const int2 *items, const SrRec *brec, const SrRec *brec_u,
                         int32_t stride, int32_t nitems, csrk_dtype store, int nrhs, Shape s, int grid, bool ind,
                         bool vec, bool all_sym, bool both, hipStream_t st);

// Workgroups per CU the batched kernels can keep resident (for sizing the grid).
int batch_occupancy(csrk_dtype store, int nrhs, Shape s, bool adjoint, bool ind, bool vec, bool all_sym,
                    bool both);

// Bandwidth probes (device/util.hip): a streaming read of `bytes` (a multiple of
// 16, 16-byte aligned) writing one word per workgroup to part[0 .. probe_grid()),
// and a copy of `bytes` from src to dst.
int probe_grid();
hipError_t probe_read(const void *buf, int64_t bytes, double *part, hipStream_t st);
hipError_t probe_copy(const void *src, void *dst, int64_t bytes, hipStream_t st);

// Conjugate-gradient vector kernels (device/cg.hip).  FP64 vectors; q (the
// product's output) is FP32 when q_f32.  part holds kCgGrid partial sums
// (or spmv_grid's, for cg_alpha_parts); s the scalars rr, pq, alpha, beta,
// rr_new, bb at s[0..5].
constexpr int kCgGrid = 1024;
int cg_grid(int64_t n);
// r = b - q, s[0] = r . r
hipError_t cg_residual(const double *b, const void *q, bool q_f32, double *r, int64_t n, double *part, double *s,
                       hipStream_t st);
// s[5] = b . b
hipError_t cg_norm2(const double *b, int64_t n, double *part, double *s, hipStream_t st);
// p = r + beta p (p = r when !use_beta); p_lo = float(p) when p_lo != NULL
hipError_t cg_set_p(const double *r, double *p, float *p_lo, const double *s, int64_t n, bool use_beta,
                    hipStream_t st);
// s[1] = sum of part[0..count) (p . q from spmv_dot), s[2] = alpha = s[0] / s[1]
hipError_t cg_alpha_parts(const double *part, int count, double *s, hipStream_t st);
// r -= alpha q, s[4] = r . r, s[3] = beta = s[4] / s[0], s[0] = s[4]
hipError_t cg_update_r(double *r, const void *q, bool q_f32, int64_t n, double *part, double *s, hipStream_t st);
// x += alpha p, then p = r + beta p (one pass over the old p); p_lo = float(p) when p_lo != NULL
hipError_t cg_update_xp(double *x, double *p, float *p_lo, const double *r, const double *s, int64_t n,
                        hipStream_t st);
// out = float(v)
hipError_t cg_round(const double *v, float *out, int64_t n, hipStream_t st);

}  // namespace dev
}  // namespace csrk
