/*
 * Oracle: plain FP64 CSR sparse matrix-vector product and its adjoint in C —
 * TEST INFRASTRUCTURE ONLY (host timing of the oracle and a second check of
 * the Python oracle).  Shares nothing with the library.
 *
 * Forward (Section 1 definition of SpMV over the CSR arrays of Section 2.1):
 *   y_i = sum over k in [row_ptr[i], row_ptr[i+1]) of vals[k] * x[col_idx[k]],
 * each row summed from 0.0 in storage order; rows are split over OpenMP
 * threads with a static schedule, as the paper runs its CPU kernels
 * (Section 5.2).
 *
 * Adjoint: grad_x[col_idx[k]] += vals[k] * g[i] for every stored entry in
 * storage order (serial: a plain scatter), grad_vals[k] = g[i] * x[col_idx[k]].
 * The gather form computes the same sums column by column: grad_x[j] = sum of
 * vals[k] * g[row(k)] over the entries k of column j taken by increasing row
 * (the order the scatter adds them in, so the two agree bit for bit), with the
 * columns split over OpenMP threads; the column index (t_ptr, t_row, t_pos)
 * is built by the caller before timing.
 *
 * Pins: tests/test_oracle_cref.py (dense brute force, Laplacian times ones).
 */
#include <stdint.h>
#include <string.h>
#include <omp.h>

void oracle_spmv_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *vals, const double *x, double *y)
{
    int32_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc += vals[k] * x[col_idx[k]];
        y[i] = acc;
    }
}

void oracle_spmv_adjoint_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             const double *vals, const double *x, const double *g,
                             double *grad_x, double *grad_vals)
{
    memset(grad_x, 0, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            grad_x[col_idx[k]] += vals[k] * g[i];
            grad_vals[k] = g[i] * x[col_idx[k]];
        }
    }
}

void oracle_spmv_adjoint_gather_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                    const double *vals, const int32_t *t_ptr, const int32_t *t_row,
                                    const int32_t *t_pos, const double *x, const double *g,
                                    double *grad_x, double *grad_vals)
{
    int32_t i, j;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            grad_vals[k] = g[i] * x[col_idx[k]];
#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int32_t p = t_ptr[j]; p < t_ptr[j + 1]; ++p)
            acc += vals[t_pos[p]] * g[t_row[p]];
        grad_x[j] = acc;
    }
}

int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads of every later parallel region (the timing runs on 1 core and on all). */
void oracle_set_threads(int t) { omp_set_num_threads(t); }

/* Runs the forward product `reps` times back to back and returns the wall seconds. */
double oracle_time_spmv_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            const double *vals, const double *x, double *y, int reps)
{
    double t0 = omp_get_wtime();
    for (int r = 0; r < reps; ++r)
        oracle_spmv_f64(n, row_ptr, col_idx, vals, x, y);
    return omp_get_wtime() - t0;
}

/* Runs the adjoint `reps` times and returns the wall seconds. */
double oracle_time_adjoint_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                               const double *vals, const double *x, const double *g,
                               double *grad_x, double *grad_vals, int reps)
{
    double t0 = omp_get_wtime();
    for (int r = 0; r < reps; ++r)
        oracle_spmv_adjoint_f64(n, row_ptr, col_idx, vals, x, g, grad_x, grad_vals);
    return omp_get_wtime() - t0;
}

/* Runs the gather form of the adjoint `reps` times and returns the wall seconds. */
double oracle_time_adjoint_gather_f64(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                      const double *vals, const int32_t *t_ptr, const int32_t *t_row,
                                      const int32_t *t_pos, const double *x, const double *g,
                                      double *grad_x, double *grad_vals, int reps)
{
    double t0 = omp_get_wtime();
    for (int r = 0; r < reps; ++r)
        oracle_spmv_adjoint_gather_f64(n, row_ptr, col_idx, vals, t_ptr, t_row, t_pos, x, g, grad_x, grad_vals);
    return omp_get_wtime() - t0;
}
