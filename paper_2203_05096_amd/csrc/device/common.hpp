// Device building blocks shared by the kernel translation units (forward,
// adjoint, batched, utilities): storage types, the windowed super-row walks
// and the dispatch helpers.  Everything here is internal to one translation
// unit (anonymous namespace); the kernels and their launchers live in the
// .hip files that include it.
//
// Mapping (Section 3 maps one super-super-row to a thread block and super-rows
// to a block dimension; here the same hierarchy is laid onto CDNA4):
//   super-super-row (SSR) -> one workgroup,
//   super-row (SR)        -> one 64-lane wavefront (SRs of an SSR are dealt
//                            round-robin to the workgroup's wavefronts),
//   row                   -> `L` lanes of that wavefront during the reduction.
// Because the rows of an SR are contiguous, the SR's nonzeros are one
// contiguous range of vals/col_idx.  A wavefront streams a window of whole
// rows of that range with 16-byte vector loads (fully coalesced whatever the
// row lengths), gathers x, multiplies, and stages the products in LDS; then
// each row is summed out of LDS by its L lanes (wavefront shuffles when L > 1).
// No MFMA: SpMV is not a dense contraction and is bound by HBM bandwidth.
//
// Workgroups are renumbered so that each of the 8 XCDs (which receive
// workgroups round-robin and each own an L2) works on a contiguous range of
// SSRs; neighbouring SSRs share most of their x window after a band-limiting
// ordering, so x is fetched into each L2 roughly once.  The ranges are cut by
// work (nonzeros plus rows), not by SSR count: on a power-law matrix the
// band ordering gathers the heavy rows together, and equal counts left one
// XCD with nearly half of the work.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <type_traits>

#include "launch.hpp"

namespace csrk {
namespace dev {

namespace {

constexpr int kWave = 64;
constexpr int kStageEntries = 512;  // nonzeros staged per window and wavefront
// Products are staged at window offsets -kStagePad .. kStageEntries - 1: a
// lane's first 16-byte step may start up to 7 entries before the window, and
// those lanes write their (unused) products into the pad instead of branching.
constexpr int kStagePad = 8;
constexpr int kStageBytes = (kStageEntries + kStagePad) * 8;  // LDS for one window (FP64 worst case)
static_assert(kUnionRows == kWave && kUnionWindow <= kStageEntries - 8, "a union super-row must fit one window");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

template <typename VT>
struct Store;
template <>
struct Store<double> {
    using X = double;  // vector element type
    using A = double;  // accumulation type
    static constexpr int V = 2;  // values per 16-byte load
    __device__ static double widen(double v) { return v; }
};
template <>
struct Store<float> {
    using X = float;
    using A = float;
    static constexpr int V = 4;
    __device__ static float widen(float v) { return v; }
};
template <>
struct Store<uint16_t> {
    using X = float;
    using A = float;
    static constexpr int V = 8;
    __device__ static float widen(uint16_t v) { return bf16_to_f32(v); }
};

// Super-super-row of block b under the work-balanced XCD ranges, or -1 for a
// padding block.  b counts from the first SSR block, which the long-row blocks
// in front of it (a multiple of 8 of them) leave on XCD 0.
__device__ __forceinline__ int32_t ssr_of_block(const XcdSplit &sp, int32_t b) {
    const int32_t xcd = b % kXcds;
    const int32_t t = sp.b[xcd] + b / kXcds;
    return t < sp.b[xcd + 1] ? t : -1;
}

// Logical block index such that each XCD (blockIdx % 8 under round-robin
// dispatch) receives a contiguous range of logical indices.  A bijection on
// [0, grid).
__device__ __forceinline__ int32_t xcd_contiguous(int32_t b, int32_t grid) {
    const int32_t xcd = b % kXcds;
    const int32_t per = grid / kXcds, extra = grid % kXcds;
    return xcd * per + min(xcd, extra) + b / kXcds;
}

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// A device pointer read from memory (a batch's descriptor table) is generic:
// the compiler must then access it with flat instructions, which count
// against the LDS wait counter as well, so every wait for an LDS read also
// waits for all gathers in flight.  Passing it through the global address
// space lets the accesses become global loads and stores (kernel-argument
// pointers are global already).  The empty asm keeps the compiler from folding
// the generic -> global -> generic round trip away before it infers the
// address space of the accesses.  p must point to device (global) memory and
// be the same for the whole wavefront (it lives in scalar registers).
template <typename T>
__device__ __forceinline__ T *global_ptr(T *p) {
    using G = __attribute__((address_space(1))) T *;
    G q = (G)p;
    asm("" : "+s"(q));
    return (T *)q;
}

// Make LDS writes of this wavefront visible to its own later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Products of one window staged in LDS at their offset from the window's
// 16-byte-aligned start: lane l's V products of step u go to
// buf[u * 64 * V + l * V ..], one aligned vector write per lane and step (no
// bank conflicts between lanes), and entry k of a window starting at entry cs
// sits at buf[k - (cs & ~(V - 1))].  Products of entries outside the window
// land where no row sum reads.
template <typename A, int U, int V>
__device__ __forceinline__ void stage_products(A *__restrict__ buf, const A (&p)[U][V], int lane) {
    typedef A PV __attribute__((ext_vector_type(V)));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        PV t;
#pragma unroll
        for (int e = 0; e < V; ++e) t[e] = p[u][e];
        *reinterpret_cast<PV *>(buf + u * kWave * V + lane * V) = t;
    }
}

// V consecutive column indices starting at pos (pos % V == 0) and the values
// of those entries: vals[pos + e], or vals[src[pos + e]] when the values are
// reached through an index map (IND; a negative map entry reads as 0).
// Entries at or beyond nnz read as 0.
// The value stream is read with non-temporal loads: each value is used once
// per product, and keeping it out of the caches leaves the Infinity Cache to
// col_idx, row_ptr and the vectors, which the forward and the adjoint of a
// step share (measured: the forward + adjoint step on a 128^3 7-point matrix
// runs about 4% faster; loading col_idx the same way made it slower).
template <typename VT, bool IND>
__device__ __forceinline__ void load_vec(const VT *__restrict__ vals, const int32_t *__restrict__ cols,
                                         const int32_t *__restrict__ src, int64_t pos, int64_t nnz,
                                         typename Store<VT>::A (&v)[Store<VT>::V], int32_t (&c)[Store<VT>::V]) {
    constexpr int V = Store<VT>::V;
    typedef int32_t CV __attribute__((ext_vector_type(V)));
    if (pos + V <= nnz) {
        const CV cv = *reinterpret_cast<const CV *>(cols + pos);
        if constexpr (IND) {
            const CV sv = *reinterpret_cast<const CV *>(src + pos);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                c[e] = cv[e];
                v[e] = sv[e] >= 0 ? Store<VT>::widen(vals[sv[e]]) : typename Store<VT>::A(0);
            }
        } else {
            typedef VT VV __attribute__((ext_vector_type(V)));
            const VV vv = __builtin_nontemporal_load(reinterpret_cast<const VV *>(vals + pos));
#pragma unroll
            for (int e = 0; e < V; ++e) {
                c[e] = cv[e];
                v[e] = Store<VT>::widen(vv[e]);
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const bool ok = pos + e < nnz;
            c[e] = ok ? cols[pos + e] : 0;
            const int64_t at = ok ? (IND ? int64_t(src[pos + e]) : pos + e) : -1;
            v[e] = at >= 0 ? Store<VT>::widen(vals[at]) : typename Store<VT>::A(0);
        }
    }
}

// ------------------------------------------------------------------ rows longer than a window
//
// A row with more nonzeros than a staging window is streamed in windows of
// kStageEntries entries by one wavefront: every lane issues all its 16-byte
// loads of a window before the dependent gathers, as in the windowed path, and
// keeps a running partial sum; the lanes are summed at the end.  Rows longer
// than kLongRow are not left to one wavefront at all: they are listed at
// upload and each is split over the wavefronts of a workgroup of its own, in
// front of the super-super-row workgroups of the same launch; the paper names
// computing very dense rows in parallel as the fix for irregular matrices
// (Section 7, GPU performance).

// Sum over entries [k0, k1) of value(k) * x[col(k)] (value(k) = vals[k], or
// vals[src[k]] with IND) by one wavefront; every lane returns the sum.
template <typename VT, bool IND>
__device__ __forceinline__ typename Store<VT>::A range_dot(int64_t k0, int64_t k1, const int32_t *__restrict__ cols,
                                                           const int32_t *__restrict__ src,
                                                           const VT *__restrict__ vals,
                                                           const typename Store<VT>::X *__restrict__ x, int64_t nnz,
                                                           int lane) {
    using A = typename Store<VT>::A;
    constexpr int V = Store<VT>::V;
    constexpr int U = kStageEntries / (kWave * V);
    A acc = 0;
    for (int64_t w0 = k0 & ~int64_t(V - 1); w0 < k1; w0 += kStageEntries) {
        const int64_t base = w0 + int64_t(lane) * V;
        A v[U][V];
        int32_t c[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            if (pos < k1) {
                load_vec<VT, IND>(vals, cols, src, pos, nnz, v[u], c[u]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v[u][e] = A(0);
                    c[u][e] = 0;
                }
            }
        }
        A xv[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                xv[u][e] = (k >= k0 && k < k1) ? A(x[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                if (k >= k0 && k < k1) acc += v[u][e] * xv[u][e];
            }
    }
    return group_sum<kWave>(acc);
}

// grad_vals[k] = gi * x[cols[k]] over entries [k0, k1) of one row, by one
// wavefront: 16-byte column loads, then the gathers, then 16-byte stores.
template <typename VT>
__device__ __forceinline__ void range_grad_vals(int64_t k0, int64_t k1, typename Store<VT>::A gi,
                                                const int32_t *__restrict__ cols,
                                                const typename Store<VT>::X *__restrict__ x,
                                                typename Store<VT>::A *__restrict__ gv, int64_t nnz, int lane) {
    using A = typename Store<VT>::A;
    constexpr int VA = 16 / int(sizeof(A));
    constexpr int U = kStageEntries / (kWave * VA);
    typedef A AV __attribute__((ext_vector_type(VA)));
    typedef int32_t CV __attribute__((ext_vector_type(VA)));
    for (int64_t w0 = k0 & ~int64_t(VA - 1); w0 < k1; w0 += kStageEntries) {
        const int64_t base = w0 + int64_t(lane) * VA;
        int32_t c[U][VA];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * VA;
            if (pos < k1 && pos + VA <= nnz) {
                const CV cv = *reinterpret_cast<const CV *>(cols + pos);
#pragma unroll
                for (int e = 0; e < VA; ++e) c[u][e] = cv[e];
            } else {
#pragma unroll
                for (int e = 0; e < VA; ++e) c[u][e] = (pos < k1 && pos + e < nnz) ? cols[pos + e] : 0;
            }
        }
        A out[U][VA];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < VA; ++e) {
                const int64_t k = base + int64_t(u) * kWave * VA + e;
                out[u][e] = (k >= k0 && k < k1) ? gi * A(x[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * VA;
            if (pos >= k0 && pos + VA <= k1) {
                AV ov;
#pragma unroll
                for (int e = 0; e < VA; ++e) ov[e] = out[u][e];
                *reinterpret_cast<AV *>(gv + pos) = ov;
            } else {
#pragma unroll
                for (int e = 0; e < VA; ++e) {
                    const int64_t k = pos + e;
                    if (k >= k0 && k < k1) gv[k] = out[u][e];
                }
            }
        }
    }
}

// Both gradients over entries [k0, k1) of row i of a symmetric pattern, by one
// wavefront: grad_vals[k] = gi * x[cols[k]] and the returned sum of
// valueT(k) * g[cols[k]] (a part of grad_x[i]); every lane returns the sum.
template <typename VT, bool IND>
__device__ __forceinline__ typename Store<VT>::A range_adjoint(int64_t k0, int64_t k1, typename Store<VT>::A gi,
                                                               const int32_t *__restrict__ cols,
                                                               const int32_t *__restrict__ src,
                                                               const VT *__restrict__ valsT,
                                                               const typename Store<VT>::X *__restrict__ x,
                                                               const typename Store<VT>::X *__restrict__ g,
                                                               typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                               int lane) {
    using A = typename Store<VT>::A;
    constexpr int V = Store<VT>::V;
    constexpr int U = kStageEntries / (kWave * V);
    typedef A AV __attribute__((ext_vector_type(V)));
    A acc = 0;
    for (int64_t w0 = k0 & ~int64_t(V - 1); w0 < k1; w0 += kStageEntries) {
        const int64_t base = w0 + int64_t(lane) * V;
        A v[U][V];
        int32_t c[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            if (pos < k1) {
                load_vec<VT, IND>(valsT, cols, src, pos, nnz, v[u], c[u]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v[u][e] = A(0);
                    c[u][e] = 0;
                }
            }
        }
        A xs[U][V], gs[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                xs[u][e] = (k >= k0 && k < k1) ? A(x[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                gs[u][e] = (k >= k0 && k < k1) ? A(g[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            A gvv[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = pos + e;
                const bool ok = k >= k0 && k < k1;
                gvv[e] = ok ? gi * xs[u][e] : A(0);
                if (ok) acc += v[u][e] * gs[u][e];
            }
            if (pos >= k0 && pos + V <= k1) {
                AV ov;
#pragma unroll
                for (int e = 0; e < V; ++e) ov[e] = gvv[e];
                *reinterpret_cast<AV *>(gv + pos) = ov;
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int64_t k = pos + e;
                    if (k >= k0 && k < k1) gv[k] = gvv[e];
                }
            }
        }
    }
    return group_sum<kWave>(acc);
}

// ------------------------------------------------------------------ forward

// y[r0..r1) = rows r0..r1-1 of (values) * x, one super-row, single right-hand
// side; with skip_long, rows longer than kLongRow are left out (their own
// kernel computes them).  The wavefront walks the super-row in windows of at most 64 whole
// rows whose nonzeros fit its LDS staging area.  Per window: every lane issues
// all its 16-byte loads of col_idx / values for the whole window before the
// dependent x gathers; the row ends of the next window are fetched meanwhile;
// products go to LDS and each row is then summed by L lanes.
// Row sums of a staged window: row rr (0 <= rr < nrows) owns the products
// buf[end(rr-1) .. end(rr)), window offsets, where end(rr) = my_end of lane rr
// minus cs; emit(rr, sum) is called by one lane per row.  Rows are reduced by
// L lanes each, the launch shape's choice for the matrix's average row.  With
// ADAPT (matrices with rows much longer than that shape expects), a window
// that holds few rows gives each row more lanes, up to the whole wavefront,
// so that a row of hundreds of products is not summed by L lanes while the
// rest of the wavefront idles.
template <int L, bool ADAPT, typename A, typename F>
__device__ __forceinline__ void window_row_sums(const A *__restrict__ buf, int nrows, int32_t my_end, int32_t cs,
                                                int lane, F &&emit) {
    int lw = L;
    if constexpr (ADAPT)
        while (lw < kWave && nrows * lw * 2 <= kWave) lw *= 2;  // wavefront-uniform
    if (!ADAPT || lw == L) {
#pragma unroll 1
        for (int b = 0; b < nrows; b += kWave / L) {
            const int rr = b + lane / L;
            const bool act = rr < nrows;
            const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
            const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
            const int32_t rbeg = rr == 0 ? 0 : prev;
            A acc = 0;
            if (act)
                for (int32_t k = rbeg + (lane % L); k < rend; k += L) acc += buf[k];
            acc = group_sum<L>(acc);
            if (act && (lane % L) == 0) emit(rr, acc);
        }
        return;
    }
    // lw * nrows <= kWave: one pass, lw lanes per row
    const int rr = lane / lw;
    const bool act = rr < nrows;
    const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
    const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
    const int32_t rbeg = rr == 0 ? 0 : prev;
    A acc = 0;
    if (act)
        for (int32_t k = rbeg + (lane % lw); k < rend; k += lw) acc += buf[k];
    for (int off = lw / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (act && (lane % lw) == 0) emit(rr, acc);
}

// With DOT, the lane that stores y[i] also adds y[i] * pdot[i] (FP64, y as
// stored) to *dot: the product's inner product with a vector, for CG.
template <typename VT, int L, bool IND, bool ADAPT = false, bool DOT = false>
__device__ __forceinline__ void sr_forward(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                           const VT *__restrict__ vals, const typename Store<VT>::X *__restrict__ x,
                                           typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                           typename Store<VT>::A *__restrict__ buf, int lane, bool skip_long,
                                           const double *__restrict__ pdot = nullptr, double *dot = nullptr) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);  // unrolled stream steps covering CAP entries
    constexpr int WIN = CAP - V;          // window limit: an unaligned window still fits U steps
    static_assert(U >= 1 && U * kWave * V == CAP, "staging area must be a whole number of steps");
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool in = ra + lane < r1;
        const bool fits = in && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            // Row ra alone exceeds the staging window: stream it in windows, or
            // leave it to the long-row workgroups.
            const int32_t re = uniform(__shfl(my_end, 0));
            if (!(skip_long && re - cs > kLongRow)) {
                const A acc = range_dot<VT, IND>(cs, re, cols, src, vals, x, nnz, lane);
                if (lane == 0) {
                    y[ra] = X(acc);
                    if constexpr (DOT) *dot += double(X(acc)) * pdot[ra];
                }
            }
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
        A v[U][V];
        int32_t c[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            if (pos < ce) {
                load_vec<VT, IND>(vals, cols, src, pos, nnz, v[u], c[u]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v[u][e] = A(0);
                    c[u][e] = 0;
                }
            }
        }
        // Every loaded column index is a valid one (entries of neighbouring rows
        // at the window's edges, or 0), so the gathers need no guard; products
        // of entries outside the window land in the pad or past the window's
        // end, where the reduction does not read.
        A xv[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) xv[u][e] = A(x[c[u][e]]);
        A pr[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) pr[u][e] = v[u][e] * xv[u][e];
        stage_products<A, U, V>(buf, pr, lane);
        wave_lds_sync();
        window_row_sums<L, ADAPT>(buf + (cs - (cs & ~(V - 1))), nrows, my_end, cs, lane, [&](int rr, A acc) {
            y[ra + rr] = X(acc);
            if constexpr (DOT) *dot += double(X(acc)) * pdot[ra + rr];
        });
        wave_lds_sync();
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// y for the rows of one super-row given by its record.  When the whole
// super-row fits one window (the common case), its stream and its row ends
// are requested together straight from the record, instead of after reading
// sr_ptr and then row_ptr: a workgroup's first loads then depend on one load
// (the record) rather than three.  Otherwise sr_forward walks it in windows.
// Results are bit for bit those of sr_forward.
template <typename VT, int L, bool IND, bool ADAPT = false, bool DOT = false>
__device__ __forceinline__ void sr_forward_rec(const SrRec &rec, const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                               const VT *__restrict__ vals, const typename Store<VT>::X *__restrict__ x,
                                               typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                               typename Store<VT>::A *__restrict__ buf, int lane, bool skip_long,
                                               const double *__restrict__ pdot = nullptr, double *dot = nullptr) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int U = kStageEntries / (kWave * V);
    constexpr int WIN = kStageEntries - V;
    const int32_t r0 = rec.r0, r1 = rec.r1, cs = rec.e0, ce = rec.e1;
    const int nrows = r1 - r0;
    if (nrows > kWave || ce - cs > WIN) {
        sr_forward<VT, L, IND, ADAPT, DOT>(r0, r1, row_ptr, cols, src, vals, x, y, nnz, buf, lane, skip_long, pdot,
                                           dot);
        return;
    }
    const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
    A v[U][V];
    int32_t c[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        if (pos < ce) {
            load_vec<VT, IND>(vals, cols, src, pos, nnz, v[u], c[u]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                v[u][e] = A(0);
                c[u][e] = 0;
            }
        }
    }
    const int32_t my_end = lane < nrows ? row_ptr[r0 + lane + 1] : 0;
    A xv[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) xv[u][e] = A(x[c[u][e]]);
    A pr[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) pr[u][e] = v[u][e] * xv[u][e];
    stage_products<A, U, V>(buf, pr, lane);
    wave_lds_sync();
    window_row_sums<L, ADAPT>(buf + (cs - (cs & ~(V - 1))), nrows, my_end, cs, lane, [&](int rr, A acc) {
        y[r0 + rr] = X(acc);
        if constexpr (DOT) *dot += double(X(acc)) * pdot[r0 + rr];
    });
    wave_lds_sync();
}

// ------------------------------------------------------------------ rows longer than kLongRow
//
// The main kernels leave rows longer than kLongRow to blocks of their own in
// front of the SSR blocks of the same grid (so they start first and run
// alongside the rest): the block's wavefronts take contiguous slices of the
// row (slice lengths a multiple of the 16-byte load width), and the slices'
// sums are added in slice order, so results do not depend on timing.

template <int V>
__device__ __forceinline__ void long_slice(int64_t k0, int64_t k1, int wave, int nw, int64_t &a, int64_t &b) {
    const int64_t per = ((k1 - k0 + nw - 1) / nw + V - 1) / V * V;
    a = min(k1, k0 + int64_t(wave) * per);
    b = min(k1, a + per);
}

// Adds the wavefronts' partial sums in order; the result is valid in thread 0.
template <typename A>
__device__ __forceinline__ A block_total(A sum, unsigned char *smem, int wave, int nw, int lane) {
    A *part = reinterpret_cast<A *>(smem);
    if (lane == 0) part[wave] = sum;
    __syncthreads();
    A t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += part[w];
    return t;
}

// y[r] for long row r by the whole workgroup (with pdot: thread 0 adds
// y[r] * pdot[r] to *dot).
template <typename VT>
__device__ __forceinline__ void long_row_forward(int32_t r, const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                 const typename Store<VT>::X *__restrict__ x,
                                                 typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                                 unsigned char *smem, int wave, int nw, int lane,
                                                 const double *__restrict__ pdot = nullptr, double *dot = nullptr) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    int64_t a, b;
    long_slice<Store<VT>::V>(row_ptr[r], row_ptr[r + 1], wave, nw, a, b);
    const A sum = (a < b) ? range_dot<VT, false>(a, b, cols, nullptr, vals, x, nnz, lane) : A(0);
    const A t = block_total(sum, smem, wave, nw, lane);
    if (threadIdx.x == 0) {
        y[r] = X(t);
        if (pdot) *dot += double(X(t)) * pdot[r];
    }
}

// Long-row item `item` of the adjoint: items [0, na) are long rows of A'
// (grad_vals of the row, plus grad_x of the same row when FUSED), items
// [na, na + nt) long rows of A'^T (grad_x only; never with FUSED).
template <typename VT, bool IND, bool FUSED>
__device__ __forceinline__ void long_row_adjoint(int32_t item, const int32_t *__restrict__ rows, int32_t na,
                                                 const int32_t *__restrict__ t_rows,
                                                 const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                                                 const int32_t *__restrict__ t_row_ptr,
                                                 const int32_t *__restrict__ t_col, const int32_t *__restrict__ t_src,
                                                 const VT *__restrict__ valsT,
                                                 const typename Store<VT>::X *__restrict__ x,
                                                 const typename Store<VT>::X *__restrict__ g,
                                                 typename Store<VT>::X *__restrict__ gx,
                                                 typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                 unsigned char *smem, int wave, int nw, int lane) {
    using A = typename Store<VT>::A;
    const bool a_item = item < na;
    const int32_t r = a_item ? rows[item] : t_rows[item - na];
    const int32_t *rp = a_item ? row_ptr : t_row_ptr;
    int64_t a, b;
    long_slice<Store<VT>::V>(rp[r], rp[r + 1], wave, nw, a, b);
    A sum = 0;
    if constexpr (FUSED) {
        if (a < b) sum = range_adjoint<VT, IND>(a, b, A(g[r]), cols, t_src, valsT, x, g, gv, nnz, lane);
    } else {
        if (a_item) {
            if (a < b) range_grad_vals<VT>(a, b, A(g[r]), cols, x, gv, nnz, lane);
            return;  // uniform over the workgroup
        }
        if (a < b) sum = range_dot<VT, IND>(a, b, t_col, t_src, valsT, g, nnz, lane);
    }
    const A t = block_total(sum, smem, wave, nw, lane);
    if (threadIdx.x == 0) gx[r] = typename Store<VT>::X(t);
}


// LDS bytes per wavefront of the multi-right-hand-side kernels: a window of
// (value, column) pairs, or (value, column, grad_vals) triples of 4-byte
// values in the fused adjoint; sized for the largest.
constexpr int kMrhsLds = kStageEntries * (8 + 4);
// Entries per window of the fused multi-column adjoint: half a window for
// 8-byte values, so that its values, columns and grad_vals take no more LDS
// than the FP32 window (more resident wavefronts).
template <typename A>
__host__ __device__ constexpr int mrhs_fused_cap() {
    return sizeof(A) == 8 ? kStageEntries / 2 : kStageEntries;
}
// LDS bytes per wavefront of a multi-column adjoint: the fused window's
// values, columns and grad_vals, and at least what the other multi-column
// layouts take.
template <typename VT>
__host__ __device__ constexpr int mrhs_adjoint_lds() {
    using A = typename Store<VT>::A;
    constexpr int f = mrhs_fused_cap<A>() * int(2 * sizeof(A) + sizeof(int32_t));
    return f > kMrhsLds ? f : kMrhsLds;
}
// LDS bytes per wavefront of a multi-column adjoint that may take the union
// window (values, columns and grad_vals of a full window).
template <typename VT>
__host__ __device__ constexpr int union_mrhs_lds() {
    constexpr int f = kStageEntries * int(2 * sizeof(typename Store<VT>::A) + sizeof(int32_t));
    return f > mrhs_adjoint_lds<VT>() ? f : mrhs_adjoint_lds<VT>();
}
// The multi-column forward needs only its own storage type's pairs.
template <typename VT>
__host__ __device__ constexpr int mrhs_forward_lds() {
    return kStageEntries * int(sizeof(typename Store<VT>::A) + sizeof(int32_t));
}
// LDS bytes per wavefront of the batched forward.
template <typename VT>
__host__ __device__ constexpr int batch_forward_lds(int nrhs) {
    return nrhs == 1 ? kStageBytes : mrhs_forward_lds<VT>();
}

// VX consecutive right-hand-side columns starting at p (16-byte aligned when VX > 1).
template <typename X, int VX>
__device__ __forceinline__ void load_cols(const X *__restrict__ p, X (&out)[VX]) {
    if constexpr (VX == 1) {
        out[0] = p[0];
    } else {
        typedef X XV __attribute__((ext_vector_type(VX)));
        const XV t = *reinterpret_cast<const XV *>(p);
#pragma unroll
        for (int e = 0; e < VX; ++e) out[e] = t[e];
    }
}

template <typename X, int VX>
__device__ __forceinline__ void store_cols(X *__restrict__ p, const X (&in)[VX]) {
    if constexpr (VX == 1) {
        p[0] = in[0];
    } else {
        typedef X XV __attribute__((ext_vector_type(VX)));
        XV t;
#pragma unroll
        for (int e = 0; e < VX; ++e) t[e] = in[e];
        *reinterpret_cast<XV *>(p) = t;
    }
}

// Sum over the lanes that share lane % RL (the entry slices of a long row).
template <int RL, typename T>
__device__ __forceinline__ T slice_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off >= RL; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One window of the multi-right-hand-side product: rows [ra, ra + nrows)
// with entries [cs, ce) (lane i holds the end of row ra + i in my_end).  The
// (value, column) pairs are streamed into LDS with 16-byte loads, staged at
// their offset from the window's 16-byte-aligned start so that each lane's
// step is one aligned LDS write; then RL lanes per row each accumulate VX
// consecutive columns, gathering VX-wide slices of the x rows (64/RL rows per
// pass).  Returns after a closing wavefront sync (the LDS may be reused).
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void mrhs_forward_window(int32_t ra, int nrows, int32_t cs, int32_t ce, int32_t my_end,
                                                    const int32_t *__restrict__ cols,
                                                    const int32_t *__restrict__ src, const VT *__restrict__ vals,
                                                    const typename Store<VT>::X *__restrict__ x,
                                                    typename Store<VT>::X *__restrict__ y, int64_t nnz, int nrhs,
                                                    unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);
    constexpr int RPP = kWave / RL;  // rows per pass
    constexpr int CPP = RL * VX;     // columns per pass
    A *sval = reinterpret_cast<A *>(lds);
    int32_t *scol = reinterpret_cast<int32_t *>(lds + CAP * sizeof(A));
    const int q = lane % RL;
    const int rsub = lane / RL;
    const int32_t cs0 = cs & ~(V - 1);
    const int32_t off = cs - cs0;  // LDS index of entry cs
    const int64_t base = int64_t(cs0) + int64_t(lane) * V;
    A v[U][V];
    int32_t c[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        if (pos < ce) {
            load_vec<VT, IND>(vals, cols, src, pos, nnz, v[u], c[u]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                v[u][e] = A(0);
                c[u][e] = 0;
            }
        }
    }
    // aligned staging: the lane's V entries of step u at LDS index u*64*V + lane*V
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            sval[u * kWave * V + lane * V + e] = v[u][e];
            scol[u * kWave * V + lane * V + e] = c[u][e];
        }
    wave_lds_sync();
#pragma unroll 1
    for (int b = 0; b < nrows; b += RPP) {
        const int rr = b + rsub;
        const bool act = rr < nrows;
        const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
        const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
        const int32_t rbeg = rr == 0 ? 0 : prev;
        if (!act) continue;
        for (int cb = 0; cb < nrhs; cb += CPP) {
            const int col0 = cb + q * VX;
            if (col0 >= nrhs) continue;
            A acc[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) acc[e] = A(0);
            // four entries at a time: their x slices are all requested before any is used
            for (int32_t k0 = rbeg; k0 < rend; k0 += 4) {
                X xv[4][VX];
                A a[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = k0 + t < rend;
                    a[t] = ok ? sval[off + k0 + t] : A(0);
                    if (ok) {
                        load_cols<X, VX>(x + int64_t(scol[off + k0 + t]) * nrhs + col0, xv[t]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VX; ++e) xv[t][e] = X(0);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int e = 0; e < VX; ++e) acc[e] += a[t] * A(xv[t][e]);
            }
            X out[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) out[e] = X(acc[e]);
            store_cols<X, VX>(y + int64_t(ra + rr) * nrhs + col0, out);
        }
    }
    wave_lds_sync();
}

// y for rows r0..r1-1 with nrhs right-hand sides (row-major n x nrhs), in
// windows of whole rows (mrhs_forward_window).  Values are vals[k] or
// vals[src[k]] (IND).  VX > 1 requires nrhs % VX == 0 and 16-byte aligned
// x / y.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void sr_forward_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                                const VT *__restrict__ vals,
                                                const typename Store<VT>::X *__restrict__ x,
                                                typename Store<VT>::X *__restrict__ y, int64_t nnz, int nrhs,
                                                unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int WIN = kStageEntries - V;
    constexpr int RPP = kWave / RL;  // rows per pass
    constexpr int CPP = RL * VX;     // columns per pass
    const int q = lane % RL;
    const int rsub = lane / RL;
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool fits = (ra + lane < r1) && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            // Row ra alone exceeds the window: entry slices of RPP lanes, RL lanes over columns.
            const int32_t re = uniform(__shfl(my_end, 0));
            for (int cb = 0; cb < nrhs; cb += CPP) {
                const int col0 = cb + q * VX;
                const bool cok = col0 < nrhs;
                A acc[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) acc[e] = A(0);
                for (int64_t k = int64_t(cs) + rsub; k < re; k += RPP) {
                    if (!cok) continue;
                    const A a = Store<VT>::widen(vals[IND ? src[k] : k]);
                    X xv[VX];
                    load_cols<X, VX>(x + int64_t(cols[k]) * nrhs + col0, xv);
#pragma unroll
                    for (int e = 0; e < VX; ++e) acc[e] += a * A(xv[e]);
                }
                X out[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) out[e] = X(slice_sum<RL>(acc[e]));
                if (rsub == 0 && cok) store_cols<X, VX>(y + int64_t(ra) * nrhs + col0, out);
            }
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        mrhs_forward_window<VT, RL, VX, IND>(ra, nrows, cs, ce, my_end, cols, src, vals, x, y, nnz, nrhs, lds, lane);
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// The multi-right-hand-side product of one super-row given by its record:
// a super-row that fits one window is streamed straight from the record
// (its stream and row ends requested together); otherwise sr_forward_mrhs.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void sr_forward_mrhs_rec(const SrRec &rec, const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                                    const VT *__restrict__ vals,
                                                    const typename Store<VT>::X *__restrict__ x,
                                                    typename Store<VT>::X *__restrict__ y, int64_t nnz, int nrhs,
                                                    unsigned char *__restrict__ lds, int lane) {
    constexpr int WIN = kStageEntries - Store<VT>::V;
    const int nrows = rec.r1 - rec.r0;
    if (nrows > kWave || rec.e1 - rec.e0 > WIN) {
        sr_forward_mrhs<VT, RL, VX, IND>(rec.r0, rec.r1, row_ptr, cols, src, vals, x, y, nnz, nrhs, lds, lane);
        return;
    }
    const int32_t my_end = lane < nrows ? row_ptr[rec.r0 + lane + 1] : 0;
    mrhs_forward_window<VT, RL, VX, IND>(rec.r0, nrows, rec.e0, rec.e1, my_end, cols, src, vals, x, y, nnz, nrhs, lds,
                                         lane);
}


// ------------------------------------------------------------------ adjoint
//
// No atomics: both gradients are row-local.
//   grad_vals[k] = g_i x_j for the entries k of rows i of the super-row
//     (a pure stream: coalesced col_idx loads and grad_vals stores);
//   grad_x[j] = sum over column j of A' of a_ij g_i = row j of A'^T times g,
//     computed like the forward product over the transposed index structure
//     (t_row_ptr, t_col) with each value fetched through t_src.
// Both use the rows of the same super-row, so the SSR -> workgroup and
// SR -> wavefront mapping carries over unchanged.

// grad_vals for rows r0..r1-1, single right-hand side, in windows of whole
// rows like the forward.  Each window's rows write their local index over
// their entries in an LDS byte map, so the stream can find g_i for any entry.
// All column loads of a window are issued first, then all x gathers, then the
// 16-byte stores.
template <typename VT>
__device__ __forceinline__ void sr_grad_vals(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                             const int32_t *__restrict__ cols,
                                             const typename Store<VT>::X *__restrict__ x,
                                             const typename Store<VT>::X *__restrict__ g,
                                             typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                             unsigned char *__restrict__ lds, int lane, bool skip_long) {
    using A = typename Store<VT>::A;
    constexpr int VA = 16 / int(sizeof(A));  // grad_vals entries per 16-byte store
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * VA);
    constexpr int WIN = CAP - VA;
    static_assert(U >= 1 && U * kWave * VA == CAP, "window must be a whole number of steps");
    typedef A AV __attribute__((ext_vector_type(VA)));
    typedef int32_t CV __attribute__((ext_vector_type(VA)));
    unsigned char *rowid = lds;
    A *gwin = reinterpret_cast<A *>(lds + CAP);
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool in = ra + lane < r1;
        const bool fits = in && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            const int32_t re = uniform(__shfl(my_end, 0));
            if (!(skip_long && re - cs > kLongRow)) range_grad_vals<VT>(cs, re, A(g[ra]), cols, x, gv, nnz, lane);
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        const int32_t prev_end = __shfl(my_end, lane > 0 ? lane - 1 : 0);
        const int64_t base = int64_t(cs & ~(VA - 1)) + int64_t(lane) * VA;
        int32_t c[U][VA];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * VA;
            if (pos < ce && pos + VA <= nnz) {
                const CV cv = *reinterpret_cast<const CV *>(cols + pos);
#pragma unroll
                for (int e = 0; e < VA; ++e) c[u][e] = cv[e];
            } else {
#pragma unroll
                for (int e = 0; e < VA; ++e) c[u][e] = (pos < ce && pos + e < nnz) ? cols[pos + e] : 0;
            }
        }
        if (lane < nrows) {
            gwin[lane] = A(g[ra + lane]);
            for (int32_t k = (lane == 0 ? cs : prev_end); k < my_end; ++k) rowid[k - cs] = uint8_t(lane);
        }
        A xs[U][VA];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < VA; ++e) {
                const int64_t k = base + int64_t(u) * kWave * VA + e;
                xs[u][e] = (k >= cs && k < ce) ? A(x[c[u][e]]) : A(0);
            }
        wave_lds_sync();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * VA;
            A out[VA];
#pragma unroll
            for (int e = 0; e < VA; ++e) {
                const int64_t k = pos + e;
                out[e] = (k >= cs && k < ce) ? gwin[rowid[k - cs]] * xs[u][e] : A(0);
            }
            if (pos >= cs && pos + VA <= ce) {
                AV ov;
#pragma unroll
                for (int e = 0; e < VA; ++e) ov[e] = out[e];
                *reinterpret_cast<AV *>(gv + pos) = ov;
            } else {
#pragma unroll
                for (int e = 0; e < VA; ++e) {
                    const int64_t k = pos + e;
                    if (k >= cs && k < ce) gv[k] = out[e];
                }
            }
        }
        wave_lds_sync();
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// grad_vals for the rows of one super-row given by its record.  When the
// whole super-row fits one window, its column stream, row ends and the g of
// its rows are requested together straight from the record (the row map is
// built while the stream is in flight); otherwise sr_grad_vals walks it in
// windows.  Results are bit for bit those of sr_grad_vals.
template <typename VT>
__device__ __forceinline__ void sr_grad_vals_rec(const SrRec &rec, const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ cols,
                                                 const typename Store<VT>::X *__restrict__ x,
                                                 const typename Store<VT>::X *__restrict__ g,
                                                 typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                 unsigned char *__restrict__ lds, int lane, bool skip_long) {
    using A = typename Store<VT>::A;
    constexpr int VA = 16 / int(sizeof(A));
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * VA);
    constexpr int WIN = CAP - VA;
    typedef A AV __attribute__((ext_vector_type(VA)));
    typedef int32_t CV __attribute__((ext_vector_type(VA)));
    const int32_t r0 = rec.r0, cs = rec.e0, ce = rec.e1;
    const int nrows = rec.r1 - rec.r0;
    if (nrows > kWave || ce - cs > WIN) {
        sr_grad_vals<VT>(rec.r0, rec.r1, row_ptr, cols, x, g, gv, nnz, lds, lane, skip_long);
        return;
    }
    unsigned char *rowid = lds;
    A *gwin = reinterpret_cast<A *>(lds + CAP);
    const int32_t my_end = lane < nrows ? row_ptr[r0 + lane + 1] : 0;
    const A gi = lane < nrows ? A(g[r0 + lane]) : A(0);
    const int64_t base = int64_t(cs & ~(VA - 1)) + int64_t(lane) * VA;
    int32_t c[U][VA];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * VA;
        if (pos < ce && pos + VA <= nnz) {
            const CV cv = *reinterpret_cast<const CV *>(cols + pos);
#pragma unroll
            for (int e = 0; e < VA; ++e) c[u][e] = cv[e];
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e) c[u][e] = (pos < ce && pos + e < nnz) ? cols[pos + e] : 0;
        }
    }
    const int32_t prev_end = __shfl(my_end, lane > 0 ? lane - 1 : 0);
    if (lane < nrows) {
        gwin[lane] = gi;
        for (int32_t k = (lane == 0 ? cs : prev_end); k < my_end; ++k) rowid[k - cs] = uint8_t(lane);
    }
    A xs[U][VA];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VA; ++e) {
            const int64_t k = base + int64_t(u) * kWave * VA + e;
            xs[u][e] = (k >= cs && k < ce) ? A(x[c[u][e]]) : A(0);
        }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * VA;
        A out[VA];
#pragma unroll
        for (int e = 0; e < VA; ++e) {
            const int64_t k = pos + e;
            out[e] = (k >= cs && k < ce) ? gwin[rowid[k - cs]] * xs[u][e] : A(0);
        }
        if (pos >= cs && pos + VA <= ce) {
            AV ov;
#pragma unroll
            for (int e = 0; e < VA; ++e) ov[e] = out[e];
            *reinterpret_cast<AV *>(gv + pos) = ov;
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e) {
                const int64_t k = pos + e;
                if (k >= cs && k < ce) gv[k] = out[e];
            }
        }
    }
    wave_lds_sync();
}

// grad_vals for several right-hand sides: grad_vals[k] = sum_c g[i,c] x[j,c].
// Per window, the column indices are streamed into LDS; RL lanes per row each
// take VX columns of g_i and of the gathered x_j rows, the partial dot
// products are summed across the RL lanes with shuffles into LDS, and the
// window's results are written out with 16-byte stores.
template <typename VT, int RL, int VX>
__device__ __forceinline__ void sr_grad_vals_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ cols,
                                                  const typename Store<VT>::X *__restrict__ x,
                                                  const typename Store<VT>::X *__restrict__ g,
                                                  typename Store<VT>::A *__restrict__ gv, int64_t nnz, int nrhs,
                                                  unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int VC = 4;  // column indices per 16-byte load
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * VC);
    constexpr int WIN = CAP - VC;
    constexpr int RPP = kWave / RL;
    constexpr int CPP = RL * VX;
    constexpr int VA = 16 / int(sizeof(A));  // grad_vals entries per 16-byte store
    typedef int32_t CV __attribute__((ext_vector_type(VC)));
    typedef A AV __attribute__((ext_vector_type(VA)));
    int32_t *scol = reinterpret_cast<int32_t *>(lds);
    A *sgv = reinterpret_cast<A *>(lds + CAP * sizeof(int32_t));
    const int q = lane % RL;
    const int rsub = lane / RL;
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool fits = (ra + lane < r1) && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            const int32_t re = uniform(__shfl(my_end, 0));
            // entry slices of RPP lanes; each slice's RL lanes reduce one entry
            for (int64_t kb = int64_t(cs); kb < re; kb += RPP) {
                const int64_t k = kb + rsub;
                const bool kok = k < re;
                const int64_t j = kok ? cols[k] : 0;
                A p = 0;
                for (int cb = 0; cb < nrhs; cb += CPP) {
                    const int col0 = cb + q * VX;
                    if (!kok || col0 >= nrhs) continue;
                    X gi[VX], xv[VX];
                    load_cols<X, VX>(g + int64_t(ra) * nrhs + col0, gi);
                    load_cols<X, VX>(x + j * nrhs + col0, xv);
#pragma unroll
                    for (int e = 0; e < VX; ++e) p += A(gi[e]) * A(xv[e]);
                }
                p = group_sum<RL>(p);
                if (kok && q == 0) gv[k] = p;
            }
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        const int64_t base = int64_t(cs & ~(VC - 1)) + int64_t(lane) * VC;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * VC;
            int32_t c[VC];
            if (pos < ce && pos + VC <= nnz) {
                const CV cv = *reinterpret_cast<const CV *>(cols + pos);
#pragma unroll
                for (int e = 0; e < VC; ++e) c[e] = cv[e];
            } else {
#pragma unroll
                for (int e = 0; e < VC; ++e) c[e] = (pos < ce && pos + e < nnz) ? cols[pos + e] : 0;
            }
#pragma unroll
            for (int e = 0; e < VC; ++e) {
                const int64_t k = pos + e;
                if (k >= cs && k < ce) scol[k - cs] = c[e];
            }
        }
        wave_lds_sync();
#pragma unroll 1
        for (int b = 0; b < nrows; b += RPP) {
            const int rr = b + rsub;
            const bool act = rr < nrows;
            const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
            const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
            const int32_t rbeg = rr == 0 ? 0 : prev;
            if (!act) continue;  // a row's RL lanes are active or idle together
            for (int cb = 0; cb < nrhs; cb += CPP) {
                const int col0 = cb + q * VX;
                const bool cok = col0 < nrhs;
                X gi[VX];
                if (cok) {
                    load_cols<X, VX>(g + int64_t(ra + rr) * nrhs + col0, gi);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e) gi[e] = X(0);
                }
                // eight entries at a time (measured: 3% faster than four here,
                // while the forward product is faster with four)
                for (int32_t k0 = rbeg; k0 < rend; k0 += 8) {
                    X xv[8][VX];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        if (cok && k0 + t < rend) {
                            load_cols<X, VX>(x + int64_t(scol[k0 + t]) * nrhs + col0, xv[t]);
                        } else {
#pragma unroll
                            for (int e = 0; e < VX; ++e) xv[t][e] = X(0);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        A p = 0;
#pragma unroll
                        for (int e = 0; e < VX; ++e) p += A(gi[e]) * A(xv[t][e]);
                        p = group_sum<RL>(p);
                        if (q == 0 && k0 + t < rend) sgv[k0 + t] = cb == 0 ? p : sgv[k0 + t] + p;
                    }
                }
            }
        }
        wave_lds_sync();
        // the window's grad_vals leave LDS as 16-byte stores
        for (int64_t pos = int64_t(cs & ~(VA - 1)) + int64_t(lane) * VA; pos < ce; pos += int64_t(kWave) * VA) {
            if (pos >= cs && pos + VA <= ce) {
                AV ov;
#pragma unroll
                for (int e = 0; e < VA; ++e) ov[e] = sgv[pos + e - cs];
                *reinterpret_cast<AV *>(gv + pos) = ov;
            } else {
#pragma unroll
                for (int e = 0; e < VA; ++e) {
                    const int64_t k = pos + e;
                    if (k >= cs && k < ce) gv[k] = sgv[k - cs];
                }
            }
        }
        wave_lds_sync();
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// Both gradients of one super-row, symmetric pattern, single right-hand side,
// in one pass: row i of A'^T has the pattern of row i of A', so the same
// stream of col_idx serves grad_vals[k] = g_i x_j and the products
// a_ji g_j of grad_x[i].  Transposed values come from valsT[k] (the handle's
// stored transposed copy) or vals[src[k]] (IND: values passed by the caller).
// LDS per wavefront: products (kStageBytes) | row map (CAP bytes) | g of the
// window's rows (64 entries).
template <typename VT, int L, bool IND, bool ADAPT = false>
__device__ __forceinline__ void sr_adjoint_fused(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                                 const VT *__restrict__ valsT,
                                                 const typename Store<VT>::X *__restrict__ x,
                                                 const typename Store<VT>::X *__restrict__ g,
                                                 typename Store<VT>::X *__restrict__ gx,
                                                 typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                 unsigned char *__restrict__ lds, int lane, bool skip_long) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);
    constexpr int WIN = CAP - V;
    typedef A AV __attribute__((ext_vector_type(V)));
    A *buf = reinterpret_cast<A *>(lds) + kStagePad;
    unsigned char *rowid = lds + kStageBytes;
    A *gwin = reinterpret_cast<A *>(lds + kStageBytes + CAP);
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool in = ra + lane < r1;
        const bool fits = in && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            // Row ra alone exceeds the staging window: stream it in windows, or
            // leave it to the long-row workgroups.
            const int32_t re = uniform(__shfl(my_end, 0));
            if (!(skip_long && re - cs > kLongRow)) {
                const A acc = range_adjoint<VT, IND>(cs, re, A(g[ra]), cols, src, valsT, x, g, gv, nnz, lane);
                if (lane == 0) gx[ra] = X(acc);
            }
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        const int32_t prev_end = __shfl(my_end, lane > 0 ? lane - 1 : 0);
        const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
        A v[U][V];
        int32_t c[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            if (pos < ce) {
                load_vec<VT, IND>(valsT, cols, src, pos, nnz, v[u], c[u]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v[u][e] = A(0);
                    c[u][e] = 0;
                }
            }
        }
        if (lane < nrows) {
            gwin[lane] = A(g[ra + lane]);
            for (int32_t k = (lane == 0 ? cs : prev_end); k < my_end; ++k) rowid[k - cs] = uint8_t(lane);
        }
        // All x gathers, then all g gathers, before any LDS or store work: the
        // compiler does not move them past those on its own, and issuing them
        // together keeps far more requests in flight.  (Here the guarded form
        // measured faster than sr_forward's unguarded one for FP32 storage.)
        A xs[U][V], gs[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                xs[u][e] = (k >= cs && k < ce) ? A(x[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                gs[u][e] = (k >= cs && k < ce) ? A(g[c[u][e]]) : A(0);
            }
        wave_lds_sync();
        A pr[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            A gvv[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = pos + e;
                const bool ok = k >= cs && k < ce;
                const A xj = xs[u][e];
                const A gj = gs[u][e];
                gvv[e] = ok ? gwin[rowid[k - cs]] * xj : A(0);
                pr[u][e] = v[u][e] * gj;
            }
            if (pos >= cs && pos + V <= ce) {
                AV ov;
#pragma unroll
                for (int e = 0; e < V; ++e) ov[e] = gvv[e];
                *reinterpret_cast<AV *>(gv + pos) = ov;
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int64_t k = pos + e;
                    if (k >= cs && k < ce) gv[k] = gvv[e];
                }
            }
        }
        stage_products<A, U, V>(buf, pr, lane);
        wave_lds_sync();
        window_row_sums<L, ADAPT>(buf + (cs - (cs & ~(V - 1))), nrows, my_end, cs, lane,
                                  [&](int rr, A acc) { gx[ra + rr] = X(acc); });
        wave_lds_sync();
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// Both gradients of one super-row of a symmetric pattern given by its record
// (the fused adjoint).  When the whole super-row fits one window, its stream,
// its row ends and the g of its rows are requested together straight from the
// record; otherwise sr_adjoint_fused walks it in windows.  Results are bit for
// bit those of sr_adjoint_fused.
template <typename VT, int L, bool IND, bool ADAPT = false>
__device__ __forceinline__ void sr_adjoint_fused_rec(const SrRec &rec, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ cols, const int32_t *__restrict__ src,
                                                     const VT *__restrict__ valsT,
                                                     const typename Store<VT>::X *__restrict__ x,
                                                     const typename Store<VT>::X *__restrict__ g,
                                                     typename Store<VT>::X *__restrict__ gx,
                                                     typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                     unsigned char *__restrict__ lds, int lane, bool skip_long) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);
    constexpr int WIN = CAP - V;
    typedef A AV __attribute__((ext_vector_type(V)));
    const int32_t r0 = rec.r0, r1 = rec.r1, cs = rec.e0, ce = rec.e1;
    const int nrows = r1 - r0;
    if (nrows > kWave || ce - cs > WIN) {
        sr_adjoint_fused<VT, L, IND, ADAPT>(r0, r1, row_ptr, cols, src, valsT, x, g, gx, gv, nnz, lds, lane,
                                            skip_long);
        return;
    }
    A *buf = reinterpret_cast<A *>(lds) + kStagePad;
    unsigned char *rowid = lds + kStageBytes;
    A *gwin = reinterpret_cast<A *>(lds + kStageBytes + CAP);
    const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
    A v[U][V];
    int32_t c[U][V];
    auto stream = [&]() {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = base + int64_t(u) * kWave * V;
            if (pos < ce) {
                load_vec<VT, IND>(valsT, cols, src, pos, nnz, v[u], c[u]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    v[u][e] = A(0);
                    c[u][e] = 0;
                }
            }
        }
    };
    A xs[U][V], gs[U][V];
    auto gathers = [&]() {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                xs[u][e] = (k >= cs && k < ce) ? A(x[c[u][e]]) : A(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = base + int64_t(u) * kWave * V + e;
                gs[u][e] = (k >= cs && k < ce) ? A(g[c[u][e]]) : A(0);
            }
    };
    int32_t my_end = 0;
    A gi = A(0);
    auto row_map = [&]() {
        const int32_t prev_end = __shfl(my_end, lane > 0 ? lane - 1 : 0);
        if (lane < nrows) {
            gwin[lane] = gi;
            for (int32_t k = (lane == 0 ? cs : prev_end); k < my_end; ++k) rowid[k - cs] = uint8_t(lane);
        }
    };
    // Order of the requests (measured): with 16-byte loads of 8 entries (BF16)
    // the row ends come first and the row map is built while the stream is in
    // flight; with 2 or 4 entries per load the stream comes first and the row
    // map is built while the gathers are in flight (27-point 100^3 FP64
    // adjoint 141 -> 120 us, BF16 111 -> 96 us for the better order).
    if constexpr (V >= 8) {
        my_end = lane < nrows ? row_ptr[r0 + lane + 1] : 0;
        gi = lane < nrows ? A(g[r0 + lane]) : A(0);
        stream();
        row_map();
        gathers();
    } else {
        stream();
        my_end = lane < nrows ? row_ptr[r0 + lane + 1] : 0;
        gi = lane < nrows ? A(g[r0 + lane]) : A(0);
        gathers();
        row_map();
    }
    wave_lds_sync();
    A pr[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        A gvv[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int64_t k = pos + e;
            const bool ok = k >= cs && k < ce;
            gvv[e] = ok ? gwin[rowid[k - cs]] * xs[u][e] : A(0);
            pr[u][e] = v[u][e] * gs[u][e];
        }
        if (pos >= cs && pos + V <= ce) {
            AV ov;
#pragma unroll
            for (int e = 0; e < V; ++e) ov[e] = gvv[e];
            *reinterpret_cast<AV *>(gv + pos) = ov;
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = pos + e;
                if (k >= cs && k < ce) gv[k] = gvv[e];
            }
        }
    }
    stage_products<A, U, V>(buf, pr, lane);
    wave_lds_sync();
    window_row_sums<L, ADAPT>(buf + (cs - (cs & ~(V - 1))), nrows, my_end, cs, lane,
                              [&](int rr, A acc) { gx[r0 + rr] = X(acc); });
    wave_lds_sync();
}

// Both gradients of one super-row of a nonsymmetric pattern in one pass over
// its union-pattern range (Arrays::u_col): the super-row's A' entries (at a
// fixed offset `e` from their A' positions), then its rows' extras.  Each U
// entry (i, j) carries a'_ji (0 where A' has no (j, i)), so row i of U times g
// is grad_x[i]: it is summed over two segments, the row's A' part and its
// extras.  grad_vals[k] = g_i x_j is written for the A' part only, at U
// position k + e.  `ra` is the super-row's record in A' (entries [e0, e1)),
// `ru` its record in U; the host builds U only when every super-row has at
// most 64 rows and fits one window (U entries <= kStageEntries - 8), which
// also leaves no row longer than kLongRow.  Values are vals[k] of U order, or
// the caller's values vals[src[k]] (IND).
template <typename VT, int L, bool IND>
__device__ __forceinline__ void sr_adjoint_union_rec(const SrRec &ra, const SrRec &ru,
                                                     const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ erow_ptr,
                                                     const int32_t *__restrict__ ucols,
                                                     const int32_t *__restrict__ usrc, const VT *__restrict__ vals,
                                                     const typename Store<VT>::X *__restrict__ x,
                                                     const typename Store<VT>::X *__restrict__ g,
                                                     typename Store<VT>::X *__restrict__ gx,
                                                     typename Store<VT>::A *__restrict__ gv, int64_t nu,
                                                     unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);
    typedef A AV __attribute__((ext_vector_type(V)));
    const int32_t r0 = ra.r0, r1 = ra.r1;
    const int nrows = r1 - r0;
    const int32_t cs = ru.e0, ce = ru.e1;  // the super-row's U range (no padding)
    const int32_t e = ru.e0 - ra.e0;       // U position of A' entry k is k + e (e % 8 == 0)
    const int32_t ca = ra.e1 + e;          // end of the A' part
    A *buf = reinterpret_cast<A *>(lds) + kStagePad;
    unsigned char *rowid = lds + kStageBytes;
    A *gwin = reinterpret_cast<A *>(lds + kStageBytes + CAP);
    const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
    // Row ends in U coordinates, of the A' part (a_end) and of the extras
    // (x_end), and the rows' g, requested before the stream (measured: 2%
    // faster than after it on the 2D 9-point 2048^2 matrix with 10% dropped)
    const int32_t eb = uniform(erow_ptr[r0]);
    const int32_t a_end = lane < nrows ? row_ptr[r0 + lane + 1] + e : 0;
    const int32_t x_end = lane < nrows ? ca + (erow_ptr[r0 + lane + 1] - eb) : 0;
    const A gi = lane < nrows ? A(g[r0 + lane]) : A(0);
    A v[U][V];
    int32_t c[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        if (pos < ce) {
            load_vec<VT, IND>(vals, ucols, usrc, pos, nu, v[u], c[u]);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                v[u][q] = A(0);
                c[u][q] = 0;
            }
        }
    }
    A xs[U][V], gs[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const int64_t k = base + int64_t(u) * kWave * V + q;
            xs[u][q] = (k >= cs && k < ca) ? A(x[c[u][q]]) : A(0);
        }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const int64_t k = base + int64_t(u) * kWave * V + q;
            gs[u][q] = (k >= cs && k < ce) ? A(g[c[u][q]]) : A(0);
        }
    {
        // the A' part's row map: entry k of row rr has rowid[k - cs] = rr
        const int32_t prev_end = __shfl(a_end, lane > 0 ? lane - 1 : 0);
        if (lane < nrows) {
            gwin[lane] = gi;
            for (int32_t k = (lane == 0 ? cs : prev_end); k < a_end; ++k) rowid[k - cs] = uint8_t(lane);
        }
    }
    wave_lds_sync();
    A pr[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        A gvv[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const int64_t k = pos + q;
            gvv[q] = (k >= cs && k < ca) ? gwin[rowid[k - cs]] * xs[u][q] : A(0);
            pr[u][q] = v[u][q] * gs[u][q];
        }
        if (pos >= cs && pos + V <= ca) {
            AV ov;
#pragma unroll
            for (int q = 0; q < V; ++q) ov[q] = gvv[q];
            *reinterpret_cast<AV *>(gv + (pos - e)) = ov;
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t k = pos + q;
                if (k >= cs && k < ca) gv[k - e] = gvv[q];
            }
        }
    }
    stage_products<A, U, V>(buf, pr, lane);
    wave_lds_sync();
    // grad_x of row rr: its A' part, then its extras, L lanes per row
    const A *w = buf + (cs - (cs & ~(V - 1)));
#pragma unroll 1
    for (int b = 0; b < nrows; b += kWave / L) {
        const int rr = b + lane / L;
        const bool act = rr < nrows;
        const int src = act ? rr : 0, prv = (act && rr > 0) ? rr - 1 : 0;
        const int32_t a1 = __shfl(a_end, src) - cs;
        const int32_t a0p = __shfl(a_end, prv) - cs;
        const int32_t x1 = __shfl(x_end, src) - cs;
        const int32_t x0p = __shfl(x_end, prv) - cs;
        const int32_t a0 = rr > 0 ? a0p : 0;
        const int32_t x0 = rr > 0 ? x0p : ca - cs;
        A acc = 0;
        if (act) {
            for (int32_t k = a0 + (lane % L); k < a1; k += L) acc += w[k];
            for (int32_t k = x0 + (lane % L); k < x1; k += L) acc += w[k];
        }
        acc = group_sum<L>(acc);
        if (act && (lane % L) == 0) gx[r0 + rr] = X(acc);
    }
    wave_lds_sync();
}

// Both gradients of one super-row, single right-hand side.  `valsT` holds the
// transposed values (aligned with t_col) unless IND, in which case it holds the
// caller's values in CSR-k order and each transposed value is vals[t_src[p]].
template <typename VT, int L, bool IND>
__device__ __forceinline__ void sr_adjoint(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ cols, const int32_t *__restrict__ t_row_ptr,
                                           const int32_t *__restrict__ t_col, const int32_t *__restrict__ t_src,
                                           const VT *__restrict__ valsT, const typename Store<VT>::X *__restrict__ x,
                                           const typename Store<VT>::X *__restrict__ g,
                                           typename Store<VT>::X *__restrict__ gx,
                                           typename Store<VT>::A *__restrict__ gv, int64_t nnz, bool sym,
                                           unsigned char *__restrict__ lds, int lane, bool skip_long) {
    using A = typename Store<VT>::A;
    if (sym && gx && gv) {
        sr_adjoint_fused<VT, L, IND>(r0, r1, row_ptr, cols, t_src, valsT, x, g, gx, gv, nnz, lds, lane, skip_long);
        return;
    }
    if (gv) sr_grad_vals<VT>(r0, r1, row_ptr, cols, x, g, gv, nnz, lds, lane, skip_long);
    if (gx)
        sr_forward<VT, L, IND>(r0, r1, t_row_ptr, t_col, t_src, valsT, g, gx, nnz,
                               reinterpret_cast<A *>(lds) + kStagePad, lane, skip_long);
}

// One window of the fused multi-right-hand-side adjoint (symmetric pattern):
// rows [ra, ra + nrows) with entries [cs, ce), lane i holding the end of row
// ra + i in my_end.  The (transposed value, column) pairs are staged in LDS at
// their offset from the window's 16-byte-aligned start (one aligned write per
// lane and step); then RL lanes per row, VX columns each, gather the x and g
// slices of every entry j of row i, add a_ji g_j into grad_x[i] and sum
// g_i . x_j over the columns into grad_vals (LDS, then 16-byte stores).
// Ends with a wavefront sync.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void mrhs_adjoint_fused_window(int32_t ra, int nrows, int32_t cs, int32_t ce,
                                                          int32_t my_end, const int32_t *__restrict__ cols,
                                                          const int32_t *__restrict__ src,
                                                          const VT *__restrict__ valsT,
                                                          const typename Store<VT>::X *__restrict__ x,
                                                          const typename Store<VT>::X *__restrict__ g,
                                                          typename Store<VT>::X *__restrict__ gx,
                                                          typename Store<VT>::A *__restrict__ gv, int64_t nnz,
                                                          int nrhs, unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = mrhs_fused_cap<A>();
    constexpr int U = CAP / (kWave * V);
    constexpr int RPP = kWave / RL;
    constexpr int CPP = RL * VX;
    constexpr int VA = 16 / int(sizeof(A));
    typedef A AV __attribute__((ext_vector_type(VA)));
    A *sval = reinterpret_cast<A *>(lds);
    int32_t *scol = reinterpret_cast<int32_t *>(lds + CAP * sizeof(A));
    A *sgv = reinterpret_cast<A *>(lds + CAP * (sizeof(A) + sizeof(int32_t)));
    const int q = lane % RL;
    const int rsub = lane / RL;
    const int32_t off = cs - (cs & ~(V - 1));  // LDS index of entry cs
    const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
    A v[U][V];
    int32_t c[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        if (pos < ce) {
            load_vec<VT, IND>(valsT, cols, src, pos, nnz, v[u], c[u]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                v[u][e] = A(0);
                c[u][e] = 0;
            }
        }
    }
    // aligned staging: the lane's V entries of step u at LDS index u*64*V + lane*V
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            sval[u * kWave * V + lane * V + e] = v[u][e];
            scol[u * kWave * V + lane * V + e] = c[u][e];
        }
    wave_lds_sync();
#pragma unroll 1
    for (int b = 0; b < nrows; b += RPP) {
        const int rr = b + rsub;
        const bool act = rr < nrows;
        const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
        const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
        const int32_t rbeg = rr == 0 ? 0 : prev;
        if (!act) continue;  // a row's RL lanes are active or idle together
        for (int cb = 0; cb < nrhs; cb += CPP) {
            const int col0 = cb + q * VX;
            const bool cok = col0 < nrhs;
            X gi[VX];
            A acc[VX];
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                gi[e] = X(0);
                acc[e] = A(0);
            }
            if (cok) load_cols<X, VX>(g + int64_t(ra + rr) * nrhs + col0, gi);
            // four entries at a time: their x and g slices are all requested before any is used
            for (int32_t k0 = rbeg; k0 < rend; k0 += 4) {
                X xv[4][VX], gj[4][VX];
                A a[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = cok && k0 + t < rend;
                    a[t] = ok ? sval[off + k0 + t] : A(0);
                    if (ok) {
                        const int64_t j = scol[off + k0 + t];
                        load_cols<X, VX>(x + j * nrhs + col0, xv[t]);
                        load_cols<X, VX>(g + j * nrhs + col0, gj[t]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VX; ++e) xv[t][e] = gj[t][e] = X(0);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    A p = 0;
#pragma unroll
                    for (int e = 0; e < VX; ++e) {
                        p += A(gi[e]) * A(xv[t][e]);
                        acc[e] += a[t] * A(gj[t][e]);
                    }
                    p = group_sum<RL>(p);
                    if (q == 0 && k0 + t < rend) sgv[k0 + t] = cb == 0 ? p : sgv[k0 + t] + p;
                }
            }
            if (cok) {
                X out[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) out[e] = X(acc[e]);
                store_cols<X, VX>(gx + int64_t(ra + rr) * nrhs + col0, out);
            }
        }
    }
    wave_lds_sync();
    for (int64_t pos = int64_t(cs & ~(VA - 1)) + int64_t(lane) * VA; pos < ce; pos += int64_t(kWave) * VA) {
        if (pos >= cs && pos + VA <= ce) {
            AV ov;
#pragma unroll
            for (int e = 0; e < VA; ++e) ov[e] = sgv[pos + e - cs];
            *reinterpret_cast<AV *>(gv + pos) = ov;
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e) {
                const int64_t k = pos + e;
                if (k >= cs && k < ce) gv[k] = sgv[k - cs];
            }
        }
    }
    wave_lds_sync();
}

// Both gradients of one super-row of a symmetric pattern, several right-hand
// sides, in one pass (the multi-column form of sr_adjoint_fused): per window
// the (transposed value, column) pairs are staged in LDS once; then RL lanes
// per row, VX columns each, gather the x and g slices of every entry j of
// row i, add a_ji g_j into grad_x[i] and sum g_i . x_j over the columns into
// grad_vals (LDS, then 16-byte stores).  LDS per wavefront: values, columns
// and grad_vals of a window (mrhs_adjoint_lds).
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void sr_adjoint_fused_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ cols,
                                                      const int32_t *__restrict__ src, const VT *__restrict__ valsT,
                                                      const typename Store<VT>::X *__restrict__ x,
                                                      const typename Store<VT>::X *__restrict__ g,
                                                      typename Store<VT>::X *__restrict__ gx,
                                                      typename Store<VT>::A *__restrict__ gv, int64_t nnz, int nrhs,
                                                      unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int WIN = mrhs_fused_cap<A>() - V;
    constexpr int RPP = kWave / RL;
    constexpr int CPP = RL * VX;
    const int q = lane % RL;
    const int rsub = lane / RL;
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    int32_t my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
    while (ra < r1) {
        const bool fits = (ra + lane < r1) && (my_end - cs <= WIN);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            // Row ra alone exceeds the window: entry slices of RPP lanes, RL lanes over columns.
            const int32_t re = uniform(__shfl(my_end, 0));
            for (int cb = 0; cb < nrhs; cb += CPP) {
                const int col0 = cb + q * VX;
                const bool cok = col0 < nrhs;
                X gi[VX];
                A acc[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    gi[e] = X(0);
                    acc[e] = A(0);
                }
                if (cok) load_cols<X, VX>(g + int64_t(ra) * nrhs + col0, gi);
                for (int64_t kb = int64_t(cs); kb < re; kb += RPP) {
                    const int64_t k = kb + rsub;
                    const bool kok = k < re;
                    A p = 0;
                    if (kok && cok) {
                        const int64_t j = cols[k];
                        const A a = Store<VT>::widen(valsT[IND ? src[k] : k]);
                        X xv[VX], gj[VX];
                        load_cols<X, VX>(x + j * nrhs + col0, xv);
                        load_cols<X, VX>(g + j * nrhs + col0, gj);
#pragma unroll
                        for (int e = 0; e < VX; ++e) {
                            p += A(gi[e]) * A(xv[e]);
                            acc[e] += a * A(gj[e]);
                        }
                    }
                    p = group_sum<RL>(p);
                    if (kok && q == 0) gv[k] = cb == 0 ? p : gv[k] + p;
                }
                X out[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) out[e] = X(slice_sum<RL>(acc[e]));
                if (rsub == 0 && cok) store_cols<X, VX>(gx + int64_t(ra) * nrhs + col0, out);
            }
            cs = re;
            ++ra;
            my_end = (ra + lane < r1) ? row_ptr[ra + lane + 1] : 0;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        const int32_t nra = ra + nrows;
        const int32_t next_end = (nra + lane < r1) ? row_ptr[nra + lane + 1] : 0;
        mrhs_adjoint_fused_window<VT, RL, VX, IND>(ra, nrows, cs, ce, my_end, cols, src, valsT, x, g, gx, gv, nnz,
                                                   nrhs, lds, lane);
        cs = ce;
        ra = nra;
        my_end = next_end;
    }
}

// The fused multi-right-hand-side adjoint of one super-row given by its
// record: a super-row that fits one window is streamed straight from the
// record; otherwise sr_adjoint_fused_mrhs.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void sr_adjoint_fused_mrhs_rec(const SrRec &rec, const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ cols,
                                                          const int32_t *__restrict__ src,
                                                          const VT *__restrict__ valsT,
                                                          const typename Store<VT>::X *__restrict__ x,
                                                          const typename Store<VT>::X *__restrict__ g,
                                                          typename Store<VT>::X *__restrict__ gx,
                                                          typename Store<VT>::A *__restrict__ gv, int64_t nnz, int nrhs,
                                                          unsigned char *__restrict__ lds, int lane) {
    constexpr int WIN = mrhs_fused_cap<typename Store<VT>::A>() - Store<VT>::V;
    const int nrows = rec.r1 - rec.r0;
    if (nrows > kWave || rec.e1 - rec.e0 > WIN) {
        sr_adjoint_fused_mrhs<VT, RL, VX, IND>(rec.r0, rec.r1, row_ptr, cols, src, valsT, x, g, gx, gv, nnz, nrhs, lds,
                                               lane);
        return;
    }
    const int32_t my_end = lane < nrows ? row_ptr[rec.r0 + lane + 1] : 0;
    mrhs_adjoint_fused_window<VT, RL, VX, IND>(rec.r0, nrows, rec.e0, rec.e1, my_end, cols, src, valsT, x, g, gx, gv,
                                               nnz, nrhs, lds, lane);
}

// Both gradients of one super-row of a nonsymmetric pattern, several
// right-hand sides, in one pass over its union-pattern range (the
// multi-column form of sr_adjoint_union_rec): per row, RL lanes x VX columns
// walk the row's A' part, gathering the x and g slices of every column j
// (grad_vals[k] = sum_c g_ic x_jc, grad_x[i] += a'_ji g_j), then its extras,
// gathering g only.  `ra` / `ru`: the super-row's records in A' and in U; the
// host builds U only when every super-row has at most 64 rows and fits one
// window.  LDS per wavefront: union_mrhs_lds.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void mrhs_adjoint_union_window(const SrRec &ra, const SrRec &ru,
                                                          const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ erow_ptr,
                                                          const int32_t *__restrict__ ucols,
                                                          const int32_t *__restrict__ usrc, const VT *__restrict__ vals,
                                                          const typename Store<VT>::X *__restrict__ x,
                                                          const typename Store<VT>::X *__restrict__ g,
                                                          typename Store<VT>::X *__restrict__ gx,
                                                          typename Store<VT>::A *__restrict__ gv, int64_t nu,
                                                          int nrhs, unsigned char *__restrict__ lds, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageEntries;
    constexpr int U = CAP / (kWave * V);
    constexpr int RPP = kWave / RL;
    constexpr int CPP = RL * VX;
    constexpr int VA = 16 / int(sizeof(A));
    typedef A AV __attribute__((ext_vector_type(VA)));
    A *sval = reinterpret_cast<A *>(lds);
    int32_t *scol = reinterpret_cast<int32_t *>(lds + CAP * sizeof(A));
    A *sgv = reinterpret_cast<A *>(lds + CAP * (sizeof(A) + sizeof(int32_t)));
    const int32_t r0 = ra.r0;
    const int nrows = ra.r1 - ra.r0;
    const int32_t cs = ru.e0, ce = ru.e1;  // U range (no padding)
    const int32_t e = ru.e0 - ra.e0;       // U position of A' entry k is k + e (e % 8 == 0)
    const int32_t ca = ra.e1 + e;          // end of the A' part
    const int q = lane % RL;
    const int rsub = lane / RL;
    const int32_t off = cs - (cs & ~(V - 1));  // LDS index of entry cs
    const int64_t base = int64_t(cs & ~(V - 1)) + int64_t(lane) * V;
    // row ends in U coordinates: of the A' part (a_end) and of the extras (x_end)
    const int32_t eb = uniform(erow_ptr[r0]);
    const int32_t a_end = lane < nrows ? row_ptr[r0 + lane + 1] + e : 0;
    const int32_t x_end = lane < nrows ? ca + (erow_ptr[r0 + lane + 1] - eb) : 0;
    A v[U][V];
    int32_t c[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t pos = base + int64_t(u) * kWave * V;
        if (pos < ce) {
            load_vec<VT, IND>(vals, ucols, usrc, pos, nu, v[u], c[u]);
        } else {
#pragma unroll
            for (int t = 0; t < V; ++t) {
                v[u][t] = A(0);
                c[u][t] = 0;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < V; ++t) {
            sval[u * kWave * V + lane * V + t] = v[u][t];
            scol[u * kWave * V + lane * V + t] = c[u][t];
        }
    wave_lds_sync();
#pragma unroll 1
    for (int b = 0; b < nrows; b += RPP) {
        const int rr = b + rsub;
        const bool act = rr < nrows;
        const int src = act ? rr : 0, prv = (act && rr > 0) ? rr - 1 : 0;
        const int32_t a1 = __shfl(a_end, src) - cs, a0p = __shfl(a_end, prv) - cs;
        const int32_t x1 = __shfl(x_end, src) - cs, x0p = __shfl(x_end, prv) - cs;
        const int32_t a0 = rr > 0 ? a0p : 0;
        const int32_t x0 = rr > 0 ? x0p : ca - cs;
        if (!act) continue;  // a row's RL lanes are active or idle together
        for (int cb = 0; cb < nrhs; cb += CPP) {
            const int col0 = cb + q * VX;
            const bool cok = col0 < nrhs;
            X gi[VX];
            A acc[VX];
#pragma unroll
            for (int t = 0; t < VX; ++t) {
                gi[t] = X(0);
                acc[t] = A(0);
            }
            if (cok) load_cols<X, VX>(g + int64_t(r0 + rr) * nrhs + col0, gi);
            // the A' part, four entries at a time: x and g slices all requested before any is used
            for (int32_t k0 = a0; k0 < a1; k0 += 4) {
                X xv[4][VX], gj[4][VX];
                A a[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = cok && k0 + t < a1;
                    a[t] = ok ? sval[off + k0 + t] : A(0);
                    if (ok) {
                        const int64_t j = scol[off + k0 + t];
                        load_cols<X, VX>(x + j * nrhs + col0, xv[t]);
                        load_cols<X, VX>(g + j * nrhs + col0, gj[t]);
                    } else {
#pragma unroll
                        for (int z = 0; z < VX; ++z) xv[t][z] = gj[t][z] = X(0);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    A p = 0;
#pragma unroll
                    for (int z = 0; z < VX; ++z) {
                        p += A(gi[z]) * A(xv[t][z]);
                        acc[z] += a[t] * A(gj[t][z]);
                    }
                    p = group_sum<RL>(p);
                    if (q == 0 && k0 + t < a1) sgv[k0 + t] = cb == 0 ? p : sgv[k0 + t] + p;
                }
            }
            // the extras: g slices only
            for (int32_t k0 = x0; k0 < x1; k0 += 4) {
                X gj[4][VX];
                A a[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = cok && k0 + t < x1;
                    a[t] = ok ? sval[off + k0 + t] : A(0);
                    if (ok) {
                        load_cols<X, VX>(g + int64_t(scol[off + k0 + t]) * nrhs + col0, gj[t]);
                    } else {
#pragma unroll
                        for (int z = 0; z < VX; ++z) gj[t][z] = X(0);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int z = 0; z < VX; ++z) acc[z] += a[t] * A(gj[t][z]);
            }
            if (cok) {
                X out[VX];
#pragma unroll
                for (int t = 0; t < VX; ++t) out[t] = X(acc[t]);
                store_cols<X, VX>(gx + int64_t(r0 + rr) * nrhs + col0, out);
            }
        }
    }
    wave_lds_sync();
    // grad_vals of the A' part, from LDS, at A' positions (U position - e)
    for (int64_t pos = int64_t(cs & ~(VA - 1)) + int64_t(lane) * VA; pos < ca; pos += int64_t(kWave) * VA) {
        if (pos >= cs && pos + VA <= ca) {
            AV ov;
#pragma unroll
            for (int t = 0; t < VA; ++t) ov[t] = sgv[pos + t - cs];
            *reinterpret_cast<AV *>(gv + (pos - e)) = ov;
        } else {
#pragma unroll
            for (int t = 0; t < VA; ++t) {
                const int64_t k = pos + t;
                if (k >= cs && k < ca) gv[k - e] = sgv[k - cs];
            }
        }
    }
    wave_lds_sync();
}

// Both gradients of one super-row, several right-hand sides (RL lanes x VX
// columns per row): one fused pass for a symmetric pattern with both outputs
// and FP32 accumulation, else grad_vals and then grad_x over A'^T.
template <typename VT, int RL, int VX, bool IND>
__device__ __forceinline__ void sr_adjoint_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ cols, const int32_t *__restrict__ t_row_ptr,
                                                const int32_t *__restrict__ t_col, const int32_t *__restrict__ t_src,
                                                const VT *__restrict__ valsT,
                                                const typename Store<VT>::X *__restrict__ x,
                                                const typename Store<VT>::X *__restrict__ g,
                                                typename Store<VT>::X *__restrict__ gx,
                                                typename Store<VT>::A *__restrict__ gv, int64_t nnz, int nrhs,
                                                bool sym, unsigned char *__restrict__ lds, int lane) {
    if (sym && gx && gv) {
        sr_adjoint_fused_mrhs<VT, RL, VX, IND>(r0, r1, row_ptr, cols, t_src, valsT, x, g, gx, gv, nnz, nrhs, lds, lane);
        return;
    }
    if (gv) sr_grad_vals_mrhs<VT, RL, VX>(r0, r1, row_ptr, cols, x, g, gv, nnz, nrhs, lds, lane);
    if (gx) sr_forward_mrhs<VT, RL, VX, IND>(r0, r1, t_row_ptr, t_col, t_src, valsT, g, gx, nnz, nrhs, lds, lane);
}

// LDS bytes per wavefront of the adjoint kernels: products, a one-byte row map
// per staged entry, g of 64 rows.
constexpr int kAdjointLds = kStageBytes + kStageEntries + 64 * 8;
// LDS bytes per wavefront of the batched kernels (any direction, any nrhs).
constexpr int kBatchLds = kMrhsLds > kAdjointLds ? kMrhsLds : kAdjointLds;


// ------------------------------------------------------------------ dispatch helpers

inline int pow2_at_least(int v) {
    int p = 1;
    while (p < v && p < 64) p <<= 1;
    return p;
}

// Calls f.template operator()<VT>() for the storage type.
template <typename F>
hipError_t by_dtype(csrk_dtype st, F &&f) {
    switch (st) {
    case CSRK_F64:
        return f(double{});
    case CSRK_F32:
        return f(float{});
    case CSRK_BF16:
        return f(uint16_t{});
    }
    return hipErrorInvalidValue;
}

template <typename F>
hipError_t by_lanes(int L, F &&f) {
    switch (L) {
    case 1:
        return f(std::integral_constant<int, 1>{});
    case 2:
        return f(std::integral_constant<int, 2>{});
    case 4:
        return f(std::integral_constant<int, 4>{});
    case 8:
        return f(std::integral_constant<int, 8>{});
    case 16:
        return f(std::integral_constant<int, 16>{});
    case 32:
        return f(std::integral_constant<int, 32>{});
    case 64:
        return f(std::integral_constant<int, 64>{});
    }
    return hipErrorInvalidValue;
}

// Columns per lane for multi-right-hand-side kernels: 16 bytes of columns when
// nrhs is a multiple of that width and every block pointer is 16-byte aligned.
template <typename X>
int vec_cols(int nrhs, std::initializer_list<const void *> ptrs) {
    constexpr int VXM = 16 / int(sizeof(X));
    if (nrhs % VXM) return 1;
    for (const void *p : ptrs)
        if (p && reinterpret_cast<uintptr_t>(p) % 16) return 1;
    return VXM;
}

// Calls f with std::integral_constant<int, VX> for VX in {1, 16 / sizeof(X)}.
template <typename X, typename F>
hipError_t by_vx(int vx, F &&f) {
    if (vx == 1) return f(std::integral_constant<int, 1>{});
    return f(std::integral_constant<int, 16 / int(sizeof(X))>{});
}

// Lanes per row for a multi-right-hand-side kernel with VX columns per lane.
inline int rhs_lanes(int nrhs, int vx) { return pow2_at_least((nrhs + vx - 1) / vx); }

// Whether windows of few rows get more lanes per row (window_row_sums): only
// for matrices with rows far longer than L lanes per row is meant for, so that
// regular matrices run the plain reduction.
inline bool adapt_windows(const Arrays &a, int L) { return a.max_row > 16 * L; }

// Calls f(std::bool_constant<ADAPT>); the adaptive reduction is instantiated
// for up to 4 lanes per row (wider groups already suit long rows).
template <int L, typename F>
void by_adapt(bool adapt, F &&f) {
    if constexpr (L <= 4) {
        if (adapt) {
            f(std::true_type{});
            return;
        }
    }
    f(std::false_type{});
}

inline int grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return int(g);
}

}  // namespace

}  // namespace dev
}  // namespace csrk
