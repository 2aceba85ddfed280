// Host-side preprocessing of the CSR-k library: validation, the symmetrised
// graph, orderings (weighted Cuthill-McKee, Band-k), the symmetric
// permutation, grouping into super-rows / super-super-rows, statistics and
// the constant-time size model.  Plain C++17, no HIP: it builds and is tested
// on machines without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../../include/csrk.h"

namespace csrk {

// Error raised inside the host code; the C ABI turns it into a status.
struct Error {
    csrk_status status;
    std::string detail;
};

// ---------------------------------------------------------------- graphs

// Undirected weighted graph in CSR form.  Adjacency lists are sorted by
// vertex index and hold each neighbour once.  ident[v] is the vertex's id for
// tie-breaking: the smallest input row it stands for.  Vertices are numbered
// in increasing ident, so comparing indices and comparing idents agree.
struct Graph {
    int32_t n = 0;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
    std::vector<int64_t> wgt;
    std::vector<int64_t> ident;
    int64_t degree(int32_t v) const { return xadj[v + 1] - xadj[v]; }
};

// Grouping of the vertices of one level into coarse vertices.
struct Aggregation {
    int32_t ncoarse = 0;
    std::vector<int32_t> owner;      // fine vertex -> coarse vertex
    std::vector<int64_t> child_ptr;  // coarse vertex c owns children[child_ptr[c] .. child_ptr[c+1])
    std::vector<int32_t> children;
    std::vector<int64_t> ident;      // coarse vertex ids (smallest input row)
};

// G0: pattern of A + A^T without the diagonal, unit weights (Section 2.2 turns
// the matrix into a graph; symmetrising is this library's reading).
Graph graph_from_csr(int32_t n, const int32_t *row_ptr, const int32_t *col_idx);

// Weighted Cuthill-McKee: repeated FIFO breadth-first searches started at the
// unvisited vertex with the smallest (degree, id); a dequeued vertex's
// unvisited neighbours are queued by (-edge weight, degree, id).
std::vector<int32_t> cuthill_mckee(const Graph &g);

// Consecutive chunks of `chunk` vertices of cuthill_mckee(g) (the last may be
// shorter); coarse vertices numbered by increasing id.
Aggregation aggregate(const Graph &g, int32_t chunk);

// Quotient graph: coarse edge weight = sum of fine edge weights between the
// two aggregates.
Graph quotient(const Graph &g, const Aggregation &a);

// Emit the fine vertices of each coarse vertex, coarse vertices taken in
// `order_up`.  Inside a coarse vertex: start at the not-yet-emitted child with
// the smallest (-wp, degree, id), wp = total edge weight to vertices already
// emitted, then breadth-first search restricted to the children with the
// Cuthill-McKee neighbour key; repeat until all children are emitted.
std::vector<int32_t> expand(const Graph &g, const std::vector<int32_t> &order_up, const Aggregation &a);

// Ordering + grouping result: perm[new] = old; sr_ptr / ssr_ptr running counts.
// For k >= 4, upper[l - 3] is the pointer array of grouping level l = 3 .. k-1
// (running counts of level-(l-1) units per level-l unit; level 2 is the SSR).
struct Grouping {
    std::vector<int32_t> perm;
    std::vector<int32_t> sr_ptr;
    std::vector<int32_t> ssr_ptr;
    std::vector<std::vector<int32_t>> upper;
};

// Largest k accepted (CSR-k is defined for every k >= 2, Section 2.2).
constexpr int32_t kMaxK = 8;

// Band-k with k = 3 (Section 2.2): coarsen by SRS, coarsen again by SSRS,
// reverse Cuthill-McKee of the coarsest graph, expand twice.
Grouping bandk(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t ssrs);

// Band-k with any k >= 2 levels of pointers: coarsen k - 1 times by the group
// sizes sizes[0..k-2] (fine to coarse), reverse Cuthill-McKee of the coarsest
// graph, expand level by level.  Fills sr_ptr (level 1), ssr_ptr (level 2;
// for k = 2 the super-rows grouped sizes[0]... see bandk2) and upper.  For
// k = 3 the result is bandk's.
Grouping bandk_levels(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const std::vector<int32_t> &sizes);

// Levels 3 .. k-1 over a grouping whose SR and SSR levels exist: consecutive
// chunks of `t` units of the level below (orders other than Band-k).
void chunk_upper(Grouping &g, int32_t k, int32_t t);

// Band-k with k = 2 (CSR-2): coarsen once by SRS, reverse Cuthill-McKee of the
// coarse graph, expand.  The format has no super-super-row level; for the GPU
// launch the super-rows are grouped `group` at a time in order (ssr_ptr).
Grouping bandk2(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t group);

// Fixed-size chunks over a given order (input order or RCM of G0).
Grouping chunked(std::vector<int32_t> perm, int32_t srs, int32_t ssrs);
Grouping rcm_chunked(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t ssrs);

// Grouping from explicit sizes.
Grouping from_sizes(std::vector<int32_t> perm, const int32_t *sr_sizes, int32_t nsr, const int32_t *ssr_sizes,
                    int32_t nssr);

// Nonzero budget of a super-row: max(2048, ceil(4 * srs * nnz / n)).
int64_t sr_budget(int32_t n, int64_t nnz, int32_t srs);

// Cuts every super-row whose cost (its rows' nonzeros, rows longer than
// CSRK_LONG_ROW counted as 0) exceeds `budget` greedily into consecutive
// pieces of cost <= budget, and regroups the pieces of each super-super-row
// `ssrs` at a time.  row_ptr is the input matrix's (rows in input order).
// Levels above the SSR keep their row ranges: upper[0] is recounted over the
// new SSRs (every old SSR start is still an SSR start).
void balance(Grouping &g, const int32_t *row_ptr, int64_t budget, int32_t ssrs);

// ---------------------------------------------------------------- CSR

// Checks row_ptr / col_idx; throws Error with the matching status.
void validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx);

// A' = P A P^T with columns sorted inside each row; vmap[k'] = input position.
struct Permuted {
    std::vector<int32_t> row_ptr;
    std::vector<int32_t> col_idx;
    std::vector<double> vals;
    std::vector<int64_t> vmap;
};
Permuted permute(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *vals,
                 const std::vector<int32_t> &perm);

// Transposed index structure of A' used by the adjoint: row j of A'^T lists
// the entries of column j of A' by increasing row, as (row, position in A').
// When the pattern is symmetric, t_row_ptr / t_col equal row_ptr / col_idx
// and only t_src (the position of each entry's mirror) is needed.
struct Transposed {
    bool symmetric = true;
    std::vector<int32_t> t_row_ptr;
    std::vector<int32_t> t_col;
    std::vector<int32_t> t_src;
};
Transposed transpose_index(int32_t n, const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &col_idx);

// Index structure of the union pattern U = pattern(A' + A'^T) of a
// nonsymmetric A', laid out so that the adjoint can take both gradients in
// one pass over it.  Super-row s (rows [r0, r1)) owns the U range
// [row_ptr[r0] + e[s], row_ptr[r1] + e[s] + extras(s)): first the A' entries
// of its rows, in A' order (column col_idx[k]; source = position in A' of the
// mirror entry (j, i), or -1 when A' has no (j, i)), then its rows' extras:
// for row i, the columns j with (j, i) in A' but (i, j) not in A', by
// increasing column (source = position of (j, i) in A').  A U entry (i, j)
// carries the value a'_ji, so row i of U times g is row i of A'^T times g.
// e[s] is the number of U entries that earlier super-rows' extras and padding
// take; each super-row's extras are padded (column r0, source -1) to a
// multiple of kUnionAlign, so e[s] keeps the A' part at A''s own alignment.
// erow_ptr[i] counts the extras of rows before i (no padding).  `ok` is false (and the vectors empty) when the
// pattern is symmetric or some super-row has more than max_rows rows or more
// than max_entries U entries (its A' part plus its extras).
constexpr int32_t kUnionAlign = 8;
struct UnionIndex {
    bool ok = false;
    std::vector<int32_t> u_col, u_src, erow_ptr;
    std::vector<int32_t> sr_begin, sr_end;  // per super-row: its U range
};
UnionIndex union_index(int32_t n, const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &col_idx,
                       const std::vector<int32_t> &sr_ptr, const Transposed &tr, int32_t max_rows,
                       int32_t max_entries);

// Row statistics (Section 5.3 / Table 1).
struct Stats {
    double rdensity = 0, row_variance = 0, symmetry = 1;
    int32_t max_row = 0, bandwidth = 0;
};
Stats row_stats(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, bool sorted_rows);
int32_t bandwidth(int32_t n, const int32_t *row_ptr, const int32_t *col_idx);

// ---------------------------------------------------------------- CPU kernel

// y = A' x on the host: super-super-rows in parallel (OpenMP, static
// schedule), rows summed left to right (Section 2.2 listing).
void spmv_host(int64_t nssr, const int32_t *ssr_ptr, const int32_t *sr_ptr, const int32_t *row_ptr,
               const int32_t *col_idx, const double *vals, const double *x, double *y, int nthreads);

// ---------------------------------------------------------------- model

// Constant-time size model (Section 4.1); see csrk_tune.
csrk_status tune(int64_t n, int64_t nnz, csrk_model model, csrk_params *out);
// tune for blocks of nrhs right-hand sides (nrhs == 1: tune)
csrk_status tune_rhs(int64_t n, int64_t nnz, int32_t nrhs, csrk_model model, csrk_params *out);

// Sanity-checks parameters (throws Error CSRK_ERR_ARG).
void check_params(const csrk_params &p);

}  // namespace csrk
