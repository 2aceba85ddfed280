// CSR validation, the symmetric permutation A' = P A P^T, row statistics, and the
// union-pattern index of a nonsymmetric A' for the one-pass adjoint.
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

namespace csrk {

UnionIndex union_index(int32_t n, const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &col_idx,
                       const std::vector<int32_t> &sr_ptr, const Transposed &tr, int32_t max_rows,
                       int32_t max_entries) {
    UnionIndex u;
    if (tr.symmetric || n == 0) return u;
    const size_t nsr = sr_ptr.size() - 1;
    // per row: the mirror source of each A' entry, and the extras
    std::vector<int32_t> mirror(col_idx.size(), -1);
    std::vector<int32_t> xcol, xsrc;
    u.erow_ptr.assign(size_t(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t k = row_ptr[i], p = tr.t_row_ptr[i];
        const int32_t ke = row_ptr[i + 1], pe = tr.t_row_ptr[i + 1];
        while (k < ke || p < pe) {  // both rows by increasing column
            if (p == pe || (k < ke && col_idx[k] < tr.t_col[p])) {
                ++k;
            } else if (k == ke || tr.t_col[p] < col_idx[k]) {
                xcol.push_back(tr.t_col[p]);
                xsrc.push_back(tr.t_src[p]);
                ++p;
            } else {
                mirror[size_t(k)] = tr.t_src[p];
                ++k;
                ++p;
            }
        }
        u.erow_ptr[size_t(i) + 1] = static_cast<int32_t>(xcol.size());
    }
    u.sr_begin.resize(nsr);
    u.sr_end.resize(nsr);
    int64_t e = 0;  // U entries of earlier super-rows' extras and padding
    for (size_t s = 0; s < nsr; ++s) {
        const int32_t r0 = sr_ptr[s], r1 = sr_ptr[s + 1];
        const int64_t na = row_ptr[r1] - row_ptr[r0], nx = u.erow_ptr[r1] - u.erow_ptr[r0];
        if (r1 - r0 > max_rows || na + nx > max_entries) return {};
        if (int64_t(row_ptr[n]) + e + nx + kUnionAlign > INT32_MAX) return {};  // U positions are int32
        u.sr_begin[s] = static_cast<int32_t>(row_ptr[r0] + e);
        u.sr_end[s] = static_cast<int32_t>(row_ptr[r1] + e + nx);
        e += (nx + kUnionAlign - 1) / kUnionAlign * kUnionAlign;
    }
    const size_t nu = size_t(row_ptr[n] + e);
    u.u_col.assign(nu, 0);
    u.u_src.assign(nu, -1);
    for (size_t s = 0; s < nsr; ++s) {
        const int32_t r0 = sr_ptr[s], r1 = sr_ptr[s + 1];
        size_t q = size_t(u.sr_begin[s]);
        for (int32_t k = row_ptr[r0]; k < row_ptr[r1]; ++k, ++q) {
            u.u_col[q] = col_idx[size_t(k)];
            u.u_src[q] = mirror[size_t(k)];
        }
        for (int32_t x = u.erow_ptr[r0]; x < u.erow_ptr[r1]; ++x, ++q) {
            u.u_col[q] = xcol[size_t(x)];
            u.u_src[q] = xsrc[size_t(x)];
        }
        const int32_t nx = u.erow_ptr[r1] - u.erow_ptr[r0];
        const size_t padded_end = size_t(u.sr_end[s]) + size_t((kUnionAlign - nx % kUnionAlign) % kUnionAlign);
        for (; q < padded_end; ++q) u.u_col[q] = r0;  // padding: a valid column, no source (value 0)
    }
    u.ok = true;
    return u;
}

}  // namespace csrk
