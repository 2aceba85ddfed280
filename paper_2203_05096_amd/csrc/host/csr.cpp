// CSR validation, the symmetric permutation A' = P A P^T, and row statistics.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.hpp"

namespace csrk {

void validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx) {
    if (n < 0) throw Error{CSRK_ERR_ARG, "n must be >= 0"};
    if (nnz < 0 || nnz > INT32_MAX) throw Error{CSRK_ERR_ARG, "nnz must be in [0, 2^31)"};
    if (!row_ptr) throw Error{CSRK_ERR_ARG, "row_ptr is NULL"};
    if (nnz > 0 && !col_idx) throw Error{CSRK_ERR_ARG, "col_idx is NULL"};
    if (row_ptr[0] != 0) throw Error{CSRK_ERR_BAD_ROWPTR, "row_ptr[0] != 0"};
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            throw Error{CSRK_ERR_BAD_ROWPTR, "row_ptr decreases at row " + std::to_string(i)};
    if (row_ptr[n] != nnz) throw Error{CSRK_ERR_BAD_ROWPTR, "row_ptr[n] != nnz"};
    std::vector<int32_t> last(n, -1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = col_idx[k];
            if (j < 0 || j >= n)
                throw Error{CSRK_ERR_COL_RANGE, "column " + std::to_string(j) + " out of range in row " + std::to_string(i)};
            if (last[j] == i)
                throw Error{CSRK_ERR_DUPLICATE, "column " + std::to_string(j) + " repeated in row " + std::to_string(i)};
            last[j] = i;
        }
}

Permuted permute(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *vals,
                 const std::vector<int32_t> &perm) {
    Permuted p;
    std::vector<int32_t> iperm(n);
    for (int32_t i = 0; i < n; ++i) iperm[perm[i]] = i;
    p.row_ptr.assign(static_cast<size_t>(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i) p.row_ptr[i + 1] = p.row_ptr[i] + (row_ptr[perm[i] + 1] - row_ptr[perm[i]]);
    const int64_t nnz = p.row_ptr[n];
    p.col_idx.resize(nnz);
    p.vals.resize(nnz);
    p.vmap.resize(nnz);
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t old = perm[i];
        row.clear();
        for (int32_t k = row_ptr[old]; k < row_ptr[old + 1]; ++k) row.emplace_back(iperm[col_idx[k]], k);
        std::sort(row.begin(), row.end());
        int32_t o = p.row_ptr[i];
        for (const auto &e : row) {
            p.col_idx[o] = e.first;
            p.vmap[o] = e.second;
            p.vals[o] = vals ? vals[e.second] : 0.0;
            ++o;
        }
    }
    return p;
}

Transposed transpose_index(int32_t n, const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &col_idx) {
    Transposed t;
    const int64_t nnz = row_ptr[n];
    t.t_row_ptr.assign(static_cast<size_t>(n) + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) ++t.t_row_ptr[col_idx[k] + 1];
    for (int32_t j = 0; j < n; ++j) t.t_row_ptr[j + 1] += t.t_row_ptr[j];
    t.t_col.resize(nnz);
    t.t_src.resize(nnz);
    std::vector<int32_t> fill(t.t_row_ptr.begin(), t.t_row_ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int32_t p = fill[col_idx[k]]++;
            t.t_col[p] = i;
            t.t_src[p] = k;
        }
    t.symmetric = (t.t_row_ptr == row_ptr) && (t.t_col == col_idx);
    if (t.symmetric) {
        t.t_row_ptr.clear();
        t.t_row_ptr.shrink_to_fit();
        t.t_col.clear();
        t.t_col.shrink_to_fit();
    }
    return t;
}

int32_t bandwidth(int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
    int64_t bw = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) bw = std::max<int64_t>(bw, std::llabs(int64_t(i) - col_idx[k]));
    return static_cast<int32_t>(bw);
}

Stats row_stats(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, bool sorted_rows) {
    Stats s;
    if (n == 0) return s;
    const double nnz = row_ptr[n];
    s.rdensity = nnz / n;
    double acc = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t len = row_ptr[i + 1] - row_ptr[i];
        s.max_row = std::max(s.max_row, len);
        const double d = len - s.rdensity;
        acc += d * d;
    }
    s.row_variance = acc / n;
    s.bandwidth = bandwidth(n, row_ptr, col_idx);
    if (sorted_rows) {
        int64_t off = 0, mirrored = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int32_t j = col_idx[k];
                if (j == i) continue;
                ++off;
                if (std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], i)) ++mirrored;
            }
        s.symmetry = off ? double(mirrored) / double(off) : 1.0;
    }
    return s;
}

}  // namespace csrk
