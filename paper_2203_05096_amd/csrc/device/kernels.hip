// gfx950 kernels of the CSR-k library.
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
// ordering, so x is fetched into each L2 roughly once.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace csrk {
namespace dev {

namespace {

constexpr int kWave = 64;
constexpr int kStageBytes = 4096;  // LDS staging window per wavefront
constexpr int kXcds = 8;

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

// Logical block index such that each XCD (blockIdx % 8 under round-robin
// dispatch) receives a contiguous range of logical indices.  A bijection on
// [0, grid).
__device__ __forceinline__ int32_t xcd_contiguous(int32_t b, int32_t grid) {
    const int32_t xcd = b % kXcds;
    const int32_t per = grid / kXcds, extra = grid % kXcds;
    return xcd * per + min(xcd, extra) + b / kXcds;
}

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

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

// V consecutive values / column indices starting at pos (pos % V == 0); the
// tail beyond nnz (array end) is read element by element.
template <typename VT>
__device__ __forceinline__ void load_vec(const VT *__restrict__ vals, const int32_t *__restrict__ cols, int64_t pos,
                                         int64_t nnz, typename Store<VT>::A (&v)[Store<VT>::V],
                                         int32_t (&c)[Store<VT>::V]) {
    constexpr int V = Store<VT>::V;
    if (pos + V <= nnz) {
        typedef VT VV __attribute__((ext_vector_type(V)));
        typedef int32_t CV __attribute__((ext_vector_type(V)));
        const VV vv = *reinterpret_cast<const VV *>(vals + pos);
        const CV cv = *reinterpret_cast<const CV *>(cols + pos);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            v[e] = Store<VT>::widen(vv[e]);
            c[e] = cv[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const bool ok = pos + e < nnz;
            v[e] = ok ? Store<VT>::widen(vals[pos + e]) : typename Store<VT>::A(0);
            c[e] = ok ? cols[pos + e] : 0;
        }
    }
}

// ------------------------------------------------------------------ forward

// y[r0..r1) for one super-row, single right-hand side.
template <typename VT, int L>
__device__ __forceinline__ void sr_forward(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                           const typename Store<VT>::X *__restrict__ x,
                                           typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                           typename Store<VT>::A *__restrict__ buf, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int V = Store<VT>::V;
    constexpr int CAP = kStageBytes / int(sizeof(A));
    int32_t ra = r0;
    int32_t cs = uniform(row_ptr[r0]);
    while (ra < r1) {
        const int32_t my_row = ra + lane;
        const bool in = my_row < r1;
        const int32_t my_end = in ? row_ptr[my_row + 1] : 0;
        const bool fits = in && (my_end - cs <= CAP);
        const uint64_t mask = __ballot(fits);
        const int nrows = (~mask == 0ull) ? kWave : __builtin_ctzll(~mask);
        if (nrows == 0) {
            // Row ra alone exceeds the staging window: sum it straight from memory.
            const int32_t re = uniform(__shfl(my_end, 0));
            A acc = 0;
            for (int64_t k = int64_t(cs) + lane; k < re; k += kWave)
                acc += Store<VT>::widen(vals[k]) * A(x[cols[k]]);
            acc = group_sum<kWave>(acc);
            if (lane == 0) y[ra] = X(acc);
            cs = re;
            ++ra;
            continue;
        }
        const int32_t ce = uniform(__shfl(my_end, nrows - 1));
        for (int64_t pos = int64_t(cs & ~(V - 1)) + int64_t(lane) * V; pos < ce; pos += int64_t(kWave) * V) {
            A v[V];
            int32_t c[V];
            load_vec<VT>(vals, cols, pos, nnz, v, c);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t k = pos + e;
                if (k >= cs && k < ce) buf[k - cs] = v[e] * A(x[c[e]]);
            }
        }
        wave_lds_sync();
#pragma unroll 1
        for (int base = 0; base < nrows; base += kWave / L) {
            const int rr = base + lane / L;
            const bool act = rr < nrows;
            const int32_t rend = __shfl(my_end, act ? rr : 0) - cs;
            const int32_t prev = __shfl(my_end, (act && rr > 0) ? rr - 1 : 0) - cs;
            const int32_t rbeg = rr == 0 ? 0 : prev;
            A acc = 0;
            if (act)
                for (int32_t k = rbeg + (lane % L); k < rend; k += L) acc += buf[k];
            acc = group_sum<L>(acc);
            if (act && (lane % L) == 0) y[ra + rr] = X(acc);
        }
        wave_lds_sync();
        cs = ce;
        ra += nrows;
    }
}

template <typename VT, int L>
__global__ void __launch_bounds__(1024) k_spmv_csrk(const int32_t *__restrict__ ssr_ptr, const int32_t *__restrict__ sr_ptr,
                                                    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                                                    const VT *__restrict__ vals, const typename Store<VT>::X *__restrict__ x,
                                                    typename Store<VT>::X *__restrict__ y, int64_t nnz) {
    using A = typename Store<VT>::A;
    constexpr int CAP = kStageBytes / int(sizeof(A));
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    A *buf = reinterpret_cast<A *>(smem) + wave * CAP;
    const int32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t s0 = ssr_ptr[t], s1 = ssr_ptr[t + 1];
    for (int32_t s = s0 + wave; s < s1; s += nw)
        sr_forward<VT, L>(uniform(sr_ptr[s]), uniform(sr_ptr[s + 1]), row_ptr, cols, vals, x, y, nnz, buf, lane);
}

// y for one super-row, nrhs right-hand sides (row-major): R lanes per row cover
// R consecutive columns of the block; 64/R rows per pass.
template <typename VT, int R>
__device__ __forceinline__ void sr_forward_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                const typename Store<VT>::X *__restrict__ x,
                                                typename Store<VT>::X *__restrict__ y, int nrhs, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    const int c = lane % R;
    const int rr = lane / R;
    for (int cb = 0; cb < nrhs; cb += R) {
        const int col = cb + c;
        const bool cok = col < nrhs;
        for (int32_t rb = r0; rb < r1; rb += kWave / R) {
            const int32_t row = rb + rr;
            if (row < r1 && cok) {
                A acc = 0;
                const int32_t kb = row_ptr[row], ke = row_ptr[row + 1];
#pragma unroll 4
                for (int32_t k = kb; k < ke; ++k)
                    acc += Store<VT>::widen(vals[k]) * A(x[int64_t(cols[k]) * nrhs + col]);
                y[int64_t(row) * nrhs + col] = X(acc);
            }
        }
    }
}

template <typename VT, int R>
__global__ void __launch_bounds__(1024) k_spmv_csrk_mrhs(const int32_t *__restrict__ ssr_ptr,
                                                         const int32_t *__restrict__ sr_ptr,
                                                         const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                         const typename Store<VT>::X *__restrict__ x,
                                                         typename Store<VT>::X *__restrict__ y, int nrhs) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t s0 = ssr_ptr[t], s1 = ssr_ptr[t + 1];
    for (int32_t s = s0 + wave; s < s1; s += nw)
        sr_forward_mrhs<VT, R>(uniform(sr_ptr[s]), uniform(sr_ptr[s + 1]), row_ptr, cols, vals, x, y, nrhs, lane);
}

// ------------------------------------------------------------------ adjoint

// grad_x += A^T g (atomics) and grad_vals = g_i x_j for one super-row.
// L lanes per row stride over the row's nonzeros; R lanes cover RHS columns.
template <typename VT, int L>
__device__ __forceinline__ void sr_adjoint(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                           const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                           const typename Store<VT>::X *__restrict__ x,
                                           const typename Store<VT>::X *__restrict__ g,
                                           typename Store<VT>::X *__restrict__ gx, typename Store<VT>::A *__restrict__ gv,
                                           int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    const int sub = lane % L;
    for (int32_t rb = r0; rb < r1; rb += kWave / L) {
        const int32_t row = rb + lane / L;
        if (row < r1) {
            const A gi = A(g[row]);
            const int32_t ke = row_ptr[row + 1];
            for (int32_t k = row_ptr[row] + sub; k < ke; k += L) {
                const int32_t j = cols[k];
                if (gv) gv[k] = gi * A(x[j]);
                if (gx) unsafeAtomicAdd(&gx[j], X(Store<VT>::widen(vals[k]) * gi));
            }
        }
    }
}

template <typename VT, int R>
__device__ __forceinline__ void sr_adjoint_mrhs(int32_t r0, int32_t r1, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                const typename Store<VT>::X *__restrict__ x,
                                                const typename Store<VT>::X *__restrict__ g,
                                                typename Store<VT>::X *__restrict__ gx,
                                                typename Store<VT>::A *__restrict__ gv, int nrhs, int lane) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    const int c = lane % R;
    const int rr = lane / R;
    for (int cb = 0; cb < nrhs; cb += R) {
        const int col = cb + c;
        const bool cok = col < nrhs;
        for (int32_t rb = r0; rb < r1; rb += kWave / R) {
            const int32_t row = rb + rr;
            if (row < r1) {
                const A gi = cok ? A(g[int64_t(row) * nrhs + col]) : A(0);
                const int32_t ke = row_ptr[row + 1];
                for (int32_t k = row_ptr[row]; k < ke; ++k) {
                    const int64_t j = cols[k];
                    if (gx && cok) unsafeAtomicAdd(&gx[j * nrhs + col], X(Store<VT>::widen(vals[k]) * gi));
                    A p = cok ? gi * A(x[j * nrhs + col]) : A(0);
                    p = group_sum<R>(p);
                    if (gv && c == 0) gv[k] = cb == 0 ? p : gv[k] + p;
                }
            }
        }
    }
}

template <typename VT, int L>
__global__ void __launch_bounds__(1024) k_adjoint_csrk(const int32_t *__restrict__ ssr_ptr, const int32_t *__restrict__ sr_ptr,
                                                       const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                       const typename Store<VT>::X *__restrict__ x,
                                                       const typename Store<VT>::X *__restrict__ g,
                                                       typename Store<VT>::X *__restrict__ gx,
                                                       typename Store<VT>::A *__restrict__ gv, int nrhs) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t s0 = ssr_ptr[t], s1 = ssr_ptr[t + 1];
    for (int32_t s = s0 + wave; s < s1; s += nw) {
        const int32_t r0 = uniform(sr_ptr[s]), r1 = uniform(sr_ptr[s + 1]);
        if (nrhs == 1)
            sr_adjoint<VT, L>(r0, r1, row_ptr, cols, vals, x, g, gx, gv, lane);
        else
            sr_adjoint_mrhs<VT, L>(r0, r1, row_ptr, cols, vals, x, g, gx, gv, nrhs, lane);
    }
}

// ------------------------------------------------------------------ plain CSR baseline

// Classic CSR-vector kernel: groups of L lanes per row, rows dealt to the grid
// in order, no super-row levels and no LDS staging.
template <typename VT, int L>
__global__ void __launch_bounds__(256) k_spmv_plain(int32_t n, const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                    const typename Store<VT>::X *__restrict__ x,
                                                    typename Store<VT>::X *__restrict__ y, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int sub = int(gid % L);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x / L;
    if (nrhs == 1) {
        for (int64_t row = gid / L; row < n; row += stride) {
            A acc = 0;
            const int32_t ke = row_ptr[row + 1];
            for (int32_t k = row_ptr[row] + sub; k < ke; k += L) acc += Store<VT>::widen(vals[k]) * A(x[cols[k]]);
            acc = group_sum<L>(acc);
            if (sub == 0) y[row] = X(acc);
        }
    } else {
        // L lanes cover L right-hand-side columns of one row
        for (int64_t row = gid / L; row < n; row += stride) {
            for (int cb = 0; cb < nrhs; cb += L) {
                const int col = cb + sub;
                if (col >= nrhs) continue;
                A acc = 0;
                const int32_t ke = row_ptr[row + 1];
                for (int32_t k = row_ptr[row]; k < ke; ++k)
                    acc += Store<VT>::widen(vals[k]) * A(x[int64_t(cols[k]) * nrhs + col]);
                y[row * nrhs + col] = X(acc);
            }
        }
    }
}

// ------------------------------------------------------------------ utilities

template <typename T>
__global__ void k_fill_zero(T *__restrict__ p, int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = T(0);
}

template <typename T>
__global__ void k_permute(int32_t n, int nrhs, const int32_t *__restrict__ perm, const T *__restrict__ in,
                          T *__restrict__ out, int dir) {
    const int64_t total = int64_t(n) * nrhs;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = idx / nrhs, c = idx % nrhs;
        const int64_t p = perm[i];
        if (dir == 0)
            out[idx] = in[p * nrhs + c];
        else
            out[p * nrhs + c] = in[idx];
    }
}

// FP64 -> FP32, round to nearest even (the conversion instruction's default mode).
__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = float(src[i]);
}

// FP64 -> FP32 -> BF16, both steps round to nearest even; NaN stays quiet NaN.
__global__ void k_to_bf16(const double *__restrict__ src, uint16_t *__restrict__ dst, int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x) {
        const float f = float(src[i]);
        uint32_t u = __float_as_uint(f);
        uint16_t h;
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
            h = uint16_t((u >> 16) | 0x40u);
        else
            h = uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        dst[i] = h;
    }
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ batched

// Persistent batched forward: logical block b takes the contiguous item range
// [b*per, (b+1)*per) of the (matrix, SSR) work list; logical indices are laid
// out so each XCD owns a contiguous part of the list.
template <typename VT, int L, int R>
__global__ void __launch_bounds__(1024) k_batch_forward(const MatDesc *__restrict__ descs, const int2 *__restrict__ items,
                                                        int32_t nitems, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    constexpr int CAP = kStageBytes / int(sizeof(A));
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    A *buf = reinterpret_cast<A *>(smem) + wave * CAP;
    const int32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t per = (nitems + gridDim.x - 1) / gridDim.x;
    const int32_t i0 = b * per, i1 = min(nitems, i0 + per);
    for (int32_t it = i0; it < i1; ++it) {
        const int2 item = items[it];
        const MatDesc d = descs[item.x];
        const int32_t s0 = d.ssr_ptr[item.y], s1 = d.ssr_ptr[item.y + 1];
        const VT *vals = static_cast<const VT *>(d.vals);
        const X *x = static_cast<const X *>(d.x);
        X *y = static_cast<X *>(d.y);
        for (int32_t s = s0 + wave; s < s1; s += nw) {
            const int32_t r0 = uniform(d.sr_ptr[s]), r1 = uniform(d.sr_ptr[s + 1]);
            if (nrhs == 1)
                sr_forward<VT, L>(r0, r1, d.row_ptr, d.col_idx, vals, x, y, d.nnz, buf, lane);
            else
                sr_forward_mrhs<VT, R>(r0, r1, d.row_ptr, d.col_idx, vals, x, y, nrhs, lane);
        }
    }
}

template <typename VT, int L, int R>
__global__ void __launch_bounds__(1024) k_batch_adjoint(const MatDesc *__restrict__ descs, const int2 *__restrict__ items,
                                                        int32_t nitems, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t per = (nitems + gridDim.x - 1) / gridDim.x;
    const int32_t i0 = b * per, i1 = min(nitems, i0 + per);
    for (int32_t it = i0; it < i1; ++it) {
        const int2 item = items[it];
        const MatDesc d = descs[item.x];
        const int32_t s0 = d.ssr_ptr[item.y], s1 = d.ssr_ptr[item.y + 1];
        const VT *vals = static_cast<const VT *>(d.vals);
        const X *x = static_cast<const X *>(d.x);
        const X *g = static_cast<const X *>(d.g);
        X *gx = static_cast<X *>(d.gx);
        A *gv = static_cast<A *>(d.gv);
        for (int32_t s = s0 + wave; s < s1; s += nw) {
            const int32_t r0 = uniform(d.sr_ptr[s]), r1 = uniform(d.sr_ptr[s + 1]);
            if (nrhs == 1)
                sr_adjoint<VT, L>(r0, r1, d.row_ptr, d.col_idx, vals, x, g, gx, gv, lane);
            else
                sr_adjoint_mrhs<VT, R>(r0, r1, d.row_ptr, d.col_idx, vals, x, g, gx, gv, nrhs, lane);
        }
    }
}

// Zero every matrix's grad_x block (blockIdx.y = matrix).
template <typename X>
__global__ void k_batch_zero_gx(const MatDesc *__restrict__ descs, int nrhs) {
    const MatDesc d = descs[blockIdx.y];
    if (!d.gx) return;
    X *gx = static_cast<X *>(d.gx);
    const int64_t total = int64_t(d.n) * nrhs;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x)
        gx[i] = X(0);
}

// ------------------------------------------------------------------ dispatch helpers

int pow2_at_least(int v) {
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

int grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return int(g);
}

// Lanes per row used by the adjoint (its loads go straight to memory, so
// lanes stride along a row): the power of two covering the typical row.
int adjoint_lanes(const Arrays &a) {
    const double r = a.n ? double(a.nnz) / a.n : 1.0;
    int L = 4;
    while (L < 64 && L < r) L <<= 1;
    return L;
}

}  // namespace

hipError_t spmv(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, int nrhs, Shape s,
                hipStream_t st) {
    if (a.nssr == 0) return hipSuccess;
    const int block = s.waves * kWave;
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        if (nrhs == 1) {
            return by_lanes(s.lanes_per_row, [&](auto lc) -> hipError_t {
                constexpr int L = decltype(lc)::value;
                hipLaunchKernelGGL((k_spmv_csrk<VT, L>), dim3(a.nssr), dim3(block), size_t(s.waves) * kStageBytes, st,
                                   a.ssr_ptr, a.sr_ptr, a.row_ptr, a.col_idx, static_cast<const VT *>(vals),
                                   static_cast<const X *>(x), static_cast<X *>(y), a.nnz);
                return hipGetLastError();
            });
        }
        return by_lanes(pow2_at_least(nrhs), [&](auto rc) -> hipError_t {
            constexpr int R = decltype(rc)::value;
            hipLaunchKernelGGL((k_spmv_csrk_mrhs<VT, R>), dim3(a.nssr), dim3(block), 0, st, a.ssr_ptr, a.sr_ptr,
                               a.row_ptr, a.col_idx, static_cast<const VT *>(vals), static_cast<const X *>(x),
                               static_cast<X *>(y), nrhs);
            return hipGetLastError();
        });
    });
}

hipError_t spmv_plain(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, int nrhs,
                      Shape s, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const double r = double(a.nnz) / a.n;
    int L = 1;
    if (nrhs == 1) {
        while (L < 64 && L < r) L <<= 1;  // lanes covering a typical row
        if (L > 1 && r <= 0.75 * L) L >>= 1;
    } else {
        L = pow2_at_least(nrhs);
    }
    (void)s;
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        return by_lanes(L, [&](auto lc) -> hipError_t {
            constexpr int LL = decltype(lc)::value;
            const int grid = grid_for(int64_t(a.n) * LL, 256);
            hipLaunchKernelGGL((k_spmv_plain<VT, LL>), dim3(grid), dim3(256), 0, st, a.n, a.row_ptr, a.col_idx,
                               static_cast<const VT *>(vals), static_cast<const X *>(x), static_cast<X *>(y), nrhs);
            return hipGetLastError();
        });
    });
}

hipError_t adjoint(const Arrays &a, csrk_dtype store, const void *vals, const void *x, const void *g, void *gx,
                   void *gv, int nrhs, Shape s, hipStream_t st) {
    if (a.nssr == 0) return hipSuccess;
    const int block = s.waves * kWave;
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        using A = typename Store<VT>::A;
        if (gx) {
            const int64_t cnt = int64_t(a.n) * nrhs;
            hipLaunchKernelGGL((k_fill_zero<X>), dim3(grid_for(cnt, 256)), dim3(256), 0, st, static_cast<X *>(gx), cnt);
        }
        const int L = nrhs == 1 ? adjoint_lanes(a) : pow2_at_least(nrhs);
        return by_lanes(L, [&](auto lc) -> hipError_t {
            constexpr int LL = decltype(lc)::value;
            hipLaunchKernelGGL((k_adjoint_csrk<VT, LL>), dim3(a.nssr), dim3(block), 0, st, a.ssr_ptr, a.sr_ptr,
                               a.row_ptr, a.col_idx, static_cast<const VT *>(vals), static_cast<const X *>(x),
                               static_cast<const X *>(g), static_cast<X *>(gx), static_cast<A *>(gv), nrhs);
            return hipGetLastError();
        });
    });
}

hipError_t permute(const Arrays &a, int dir, const void *in, void *out, int nrhs, int elem_bytes, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const int grid = grid_for(int64_t(a.n) * nrhs, 256);
    if (elem_bytes == 8)
        hipLaunchKernelGGL((k_permute<double>), dim3(grid), dim3(256), 0, st, a.n, nrhs, a.perm,
                           static_cast<const double *>(in), static_cast<double *>(out), dir);
    else
        hipLaunchKernelGGL((k_permute<float>), dim3(grid), dim3(256), 0, st, a.n, nrhs, a.perm,
                           static_cast<const float *>(in), static_cast<float *>(out), dir);
    return hipGetLastError();
}

hipError_t convert_values(const double *src, void *dst, int64_t count, csrk_dtype store, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const int grid = grid_for(count, 256);
    switch (store) {
    case CSRK_F64:
        hipLaunchKernelGGL(k_copy_f64, dim3(grid), dim3(256), 0, st, src, static_cast<double *>(dst), count);
        break;
    case CSRK_F32:
        hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(256), 0, st, src, static_cast<float *>(dst), count);
        break;
    case CSRK_BF16:
        hipLaunchKernelGGL(k_to_bf16, dim3(grid), dim3(256), 0, st, src, static_cast<uint16_t *>(dst), count);
        break;
    }
    return hipGetLastError();
}

hipError_t batch_forward(const MatDesc *descs, const int2 *items, int32_t nitems, csrk_dtype store, int nrhs,
                         Shape s, int grid, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    const int R = pow2_at_least(nrhs);
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        return by_lanes(nrhs == 1 ? s.lanes_per_row : R, [&](auto lc) -> hipError_t {
            constexpr int LL = decltype(lc)::value;
            hipLaunchKernelGGL((k_batch_forward<VT, LL, LL>), dim3(grid), dim3(block),
                               nrhs == 1 ? size_t(s.waves) * kStageBytes : 0, st, descs, items, nitems, nrhs);
            return hipGetLastError();
        });
    });
}

hipError_t batch_adjoint(const MatDesc *descs, const int2 *items, int32_t nitems, int32_t nmat, int32_t max_n,
                         csrk_dtype store, int nrhs, Shape s, int grid, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    const int R = pow2_at_least(nrhs);
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        const int zgrid = grid_for(int64_t(max_n) * nrhs, 256);
        hipLaunchKernelGGL((k_batch_zero_gx<X>), dim3(zgrid < 1024 ? zgrid : 1024, nmat), dim3(256), 0, st, descs, nrhs);
        return by_lanes(nrhs == 1 ? s.lanes_per_row : R, [&](auto lc) -> hipError_t {
            constexpr int LL = decltype(lc)::value;
            hipLaunchKernelGGL((k_batch_adjoint<VT, LL, LL>), dim3(grid), dim3(block), 0, st, descs, items, nitems,
                               nrhs);
            return hipGetLastError();
        });
    });
}

int batch_occupancy(csrk_dtype store, int nrhs, Shape s, bool adj) {
    int blocks = 1;
    const int block = s.waves * kWave;
    const int R = pow2_at_least(nrhs);
    const hipError_t e = by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        return by_lanes(nrhs == 1 ? s.lanes_per_row : R, [&](auto lc) -> hipError_t {
            constexpr int LL = decltype(lc)::value;
            if (adj)
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_adjoint<VT, LL, LL>, block, 0);
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_forward<VT, LL, LL>, block,
                                                                nrhs == 1 ? size_t(s.waves) * kStageBytes : 0);
        });
    });
    return (e != hipSuccess || blocks < 1) ? 1 : blocks;
}

}  // namespace dev
}  // namespace csrk
