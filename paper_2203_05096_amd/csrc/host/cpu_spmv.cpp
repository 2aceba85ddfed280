// The CSR-k product on the host CPU over the same handle as the GPU kernels,
// which is the point of a heterogeneous format (Section 2.2 gives the CPU
// kernel).  The unit of parallel work is a super-super-row, split over OpenMP
// threads with a static schedule (Section 5.2).  The rows of a super-super-row
// are contiguous (its super-rows are consecutive and so are their rows), so
// each unit walks one row range and one contiguous run of nonzeros, with no
// inner loop over super-rows; every row is summed from 0.0 left to right, so
// the result is the same as the row-by-row traversal bit for bit.
#include <omp.h>

#include "host.hpp"

namespace csrk {

void spmv_host(int64_t nssr, const int32_t *ssr_ptr, const int32_t *sr_ptr, const int32_t *row_ptr,
               const int32_t *col_idx, const double *vals, const double *x, double *y, int nthreads) {
    const int threads = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t t = 0; t < nssr; ++t) {
        const int32_t first = sr_ptr[ssr_ptr[t]], last = sr_ptr[ssr_ptr[t + 1]];
        int64_t k = row_ptr[first];
        for (int32_t i = first; i < last; ++i) {
            const int64_t end = row_ptr[i + 1];
            double acc = 0.0;
            for (; k < end; ++k) acc += vals[k] * x[col_idx[k]];
            y[i] = acc;
        }
    }
}

}  // namespace csrk
