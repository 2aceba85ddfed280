// Forward kernels: the CSR-k product for one and for several right-hand sides,
// the product with a fused partial inner product (for CG), and the plain CSR
// baseline; with their launchers.
#include "common.hpp"

namespace csrk {
namespace dev {

namespace {

template <typename VT, int L, bool ADAPT>
__global__ void __launch_bounds__(1024) k_spmv_csrk(const SrRec *__restrict__ srec, int32_t stride,
                                                    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                                                    const VT *__restrict__ vals, const typename Store<VT>::X *__restrict__ x,
                                                    typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                                    const int32_t *__restrict__ long_rows, int32_t nlong,
                                                    int32_t long_blocks, XcdSplit split) {
    using A = typename Store<VT>::A;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t bid = int32_t(blockIdx.x);
    if (bid < long_blocks) {
        if (bid < nlong) long_row_forward<VT>(long_rows[bid], row_ptr, cols, vals, x, y, nnz, smem, wave, nw, lane);
        return;
    }
    A *buf = reinterpret_cast<A *>(smem + size_t(wave) * kStageBytes) + kStagePad;
    const int32_t t = ssr_of_block(split, bid - long_blocks);
    if (t < 0) return;
    // the SSR's super-rows from its records (slots past its last SR are empty)
    for (int32_t w = wave; w < stride; w += nw) {
        const SrRec rec = srec[int64_t(t) * stride + w];
        if (rec.r0 >= rec.r1) break;
        sr_forward_rec<VT, L, false, ADAPT>(rec, row_ptr, cols, nullptr, vals, x, y, nnz, buf, lane, true);
    }
}

// The forward product y = A'x plus, per workgroup, the partial inner product
// sum_i y_i pdot_i (FP64, y as stored), written to part[blockIdx.x] by every
// workgroup (0 where it has no rows).  Each lane accumulates the rows it
// stores, in storage order; lanes, then wavefronts, are added in a fixed
// order, so the partials do not depend on timing.  Used by CG for p . Ap.
template <typename VT, int L>
__global__ void __launch_bounds__(1024) k_spmv_csrk_dot(const SrRec *__restrict__ srec, int32_t stride,
                                                        const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                        const typename Store<VT>::X *__restrict__ x,
                                                        typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                                        const int32_t *__restrict__ long_rows, int32_t nlong,
                                                        int32_t long_blocks, XcdSplit split,
                                                        const double *__restrict__ pdot, double *__restrict__ part) {
    using A = typename Store<VT>::A;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double wsum[1024 / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t bid = int32_t(blockIdx.x);
    double dot = 0;
    if (bid < long_blocks) {
        if (bid < nlong)
            long_row_forward<VT>(long_rows[bid], row_ptr, cols, vals, x, y, nnz, smem, wave, nw, lane, pdot, &dot);
    } else {
        A *buf = reinterpret_cast<A *>(smem + size_t(wave) * kStageBytes) + kStagePad;
        const int32_t t = ssr_of_block(split, bid - long_blocks);
        if (t >= 0) {
            for (int32_t w = wave; w < stride; w += nw) {
                const SrRec rec = srec[int64_t(t) * stride + w];
                if (rec.r0 >= rec.r1) break;
                sr_forward_rec<VT, L, false, false, true>(rec, row_ptr, cols, nullptr, vals, x, y, nnz, buf, lane, true,
                                                          pdot, &dot);
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) dot += __shfl_xor(dot, off);
    if (lane == 0) wsum[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < nw; ++w) t += wsum[w];
        part[bid] = t;
    }
}

template <typename VT, int RL, int VX>
__global__ void __launch_bounds__(1024) k_spmv_csrk_mrhs(const SrRec *__restrict__ srec, int32_t stride,
                                                         const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ cols, const VT *__restrict__ vals,
                                                         const typename Store<VT>::X *__restrict__ x,
                                                         typename Store<VT>::X *__restrict__ y, int64_t nnz,
                                                         int nrhs, XcdSplit split) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    unsigned char *lds = smem + size_t(wave) * mrhs_forward_lds<VT>();
    const int32_t t = ssr_of_block(split, int32_t(blockIdx.x));
    if (t < 0) return;
    for (int32_t w = wave; w < stride; w += nw) {
        const SrRec rec = srec[int64_t(t) * stride + w];
        if (rec.r0 >= rec.r1) break;
        sr_forward_mrhs_rec<VT, RL, VX, false>(rec, row_ptr, cols, nullptr, vals, x, y, nnz, nrhs, lds, lane);
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
                const int32_t long_blocks = (a.nlong + kXcds - 1) / kXcds * kXcds;
                by_adapt<L>(adapt_windows(a, L), [&](auto ac) {
                    hipLaunchKernelGGL((k_spmv_csrk<VT, L, decltype(ac)::value>),
                                       dim3(long_blocks + a.split_fwd.width * kXcds), dim3(block),
                                       size_t(s.waves) * kStageBytes, st, a.srec, a.srec_stride, a.row_ptr,
                                       a.col_idx, static_cast<const VT *>(vals), static_cast<const X *>(x),
                                       static_cast<X *>(y), a.nnz, a.long_rows, a.nlong, long_blocks, a.split_fwd);
                });
                return hipGetLastError();
            });
        }
        const int vx = vec_cols<X>(nrhs, {x, y});
        return by_vx<X>(vx, [&](auto vc) -> hipError_t {
            constexpr int VX = decltype(vc)::value;
            return by_lanes(rhs_lanes(nrhs, VX), [&](auto rc) -> hipError_t {
                constexpr int RL = decltype(rc)::value;
                hipLaunchKernelGGL((k_spmv_csrk_mrhs<VT, RL, VX>), dim3(a.split_fwd.width * kXcds), dim3(block),
                                   size_t(s.waves) * mrhs_forward_lds<VT>(), st, a.srec, a.srec_stride, a.row_ptr,
                                   a.col_idx,
                                   static_cast<const VT *>(vals), static_cast<const X *>(x), static_cast<X *>(y),
                                   a.nnz, nrhs, a.split_fwd);
                return hipGetLastError();
            });
        });
    });
}

int spmv_grid(const Arrays &a) {
    return (a.nlong + kXcds - 1) / kXcds * kXcds + a.split_fwd.width * kXcds;
}

hipError_t spmv_dot(const Arrays &a, csrk_dtype store, const void *vals, const void *x, void *y, const double *pdot,
                    double *part, Shape s, hipStream_t st) {
    if (a.nssr == 0) return hipSuccess;
    const int block = s.waves * kWave;
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        return by_lanes(s.lanes_per_row, [&](auto lc) -> hipError_t {
            constexpr int L = decltype(lc)::value;
            const int32_t long_blocks = (a.nlong + kXcds - 1) / kXcds * kXcds;
            hipLaunchKernelGGL((k_spmv_csrk_dot<VT, L>), dim3(spmv_grid(a)), dim3(block),
                               size_t(s.waves) * kStageBytes, st, a.srec, a.srec_stride, a.row_ptr, a.col_idx,
                               static_cast<const VT *>(vals), static_cast<const X *>(x), static_cast<X *>(y), a.nnz,
                               a.long_rows, a.nlong, long_blocks, a.split_fwd, pdot, part);
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

}  // namespace dev
}  // namespace csrk
