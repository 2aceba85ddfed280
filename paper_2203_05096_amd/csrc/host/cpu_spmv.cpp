// The CSR-k product on the host CPU (the paper's CPU kernel, Section 2.2
// listing): one parallel loop over super-super-rows, then the super-rows of
// each, then their rows.  Plain C++ with OpenMP; the same handle serves the
// GPU kernels, which is the paper's point of a heterogeneous format.
#include <omp.h>

#include "host.hpp"

namespace csrk {

void spmv_host(int64_t nssr, const int32_t *ssr_ptr, const int32_t *sr_ptr, const int32_t *row_ptr,
               const int32_t *col_idx, const double *vals, const double *x, double *y, int nthreads) {
    const int threads = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t t = 0; t < nssr; ++t) {
        for (int32_t s = ssr_ptr[t]; s < ssr_ptr[t + 1]; ++s) {
            for (int32_t i = sr_ptr[s]; i < sr_ptr[s + 1]; ++i) {
                double acc = 0.0;
                for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) acc += vals[k] * x[col_idx[k]];
                y[i] = acc;
            }
        }
    }
}

}  // namespace csrk
