// Batched kernels: one launch over a work list of (matrix, super-super-row)
// items for many matrices, forward and adjoint; with their launchers.
#include "common.hpp"

namespace csrk {
namespace dev {

namespace {

// ------------------------------------------------------------------ batched

// Batched forward: logical block b takes the contiguous item range
// [b*per, (b+1)*per) of the (matrix, SSR) work list; logical indices are laid
// out so each XCD owns a contiguous part of the list.  L is the lanes per row
// (single right-hand side) or per row group (several: L lanes x VX columns).
template <typename VT, int L, int VX>
__global__ void __launch_bounds__(1024) k_batch_forward(const MatDesc *__restrict__ descs, const int2 *__restrict__ items,
                                                        int32_t nitems, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    unsigned char *lds = smem + size_t(wave) * batch_forward_lds<VT>(nrhs);
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
                sr_forward<VT, L, false>(r0, r1, d.row_ptr, d.col_idx, nullptr, vals, x, y, d.nnz,
                                         reinterpret_cast<A *>(lds) + kStagePad, lane, false);
            else
                sr_forward_mrhs<VT, L, VX, false>(r0, r1, d.row_ptr, d.col_idx, nullptr, vals, x, y, d.nnz, nrhs, lds,
                                                  lane);
        }
    }
}

template <typename VT, int L, int VX, bool IND>
__global__ void __launch_bounds__(1024) k_batch_adjoint(const MatDesc *__restrict__ descs, const int2 *__restrict__ items,
                                                        int32_t nitems, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    unsigned char *lds = smem + size_t(wave) * kBatchLds;
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
                sr_adjoint<VT, L, IND>(r0, r1, d.row_ptr, d.col_idx, d.t_row_ptr, d.t_col, d.t_src, vals, x, g, gx,
                                       gv, d.nnz, d.sym != 0, lds, lane, false);
            else
                sr_adjoint_mrhs<VT, L, VX, IND>(r0, r1, d.row_ptr, d.col_idx, d.t_row_ptr, d.t_col, d.t_src, vals, x,
                                                g, gx, gv, d.nnz, nrhs, d.sym != 0, lds, lane);
        }
    }
}

}  // namespace

namespace {

// Calls f(VT{}, integral_constant<VX>, integral_constant<L>) with the
// instantiation the batched kernels use for this storage type, column count
// and launch shape (the same choice for the launch and its occupancy query).
template <typename F>
hipError_t by_batch_shape(csrk_dtype store, int nrhs, const Shape &s, bool vec, F &&f) {
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using X = typename Store<decltype(vt)>::X;
        const int vx = (nrhs > 1 && vec && nrhs % (16 / int(sizeof(X))) == 0) ? 16 / int(sizeof(X)) : 1;
        return by_vx<X>(vx, [&](auto vc) -> hipError_t {
            return by_lanes(nrhs == 1 ? s.lanes_per_row : rhs_lanes(nrhs, decltype(vc)::value),
                            [&](auto lc) -> hipError_t { return f(vt, vc, lc); });
        });
    });
}

}  // namespace

hipError_t batch_forward(const MatDesc *descs, const int2 *items, int32_t nitems, csrk_dtype store, int nrhs,
                         Shape s, int grid, bool vec, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    return by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        hipLaunchKernelGGL((k_batch_forward<VT, LL, VX>), dim3(grid), dim3(block),
                           size_t(s.waves) * batch_forward_lds<VT>(nrhs), st, descs, items, nitems, nrhs);
        return hipGetLastError();
    });
}

hipError_t batch_adjoint(const MatDesc *descs, const int2 *items, int32_t nitems, csrk_dtype store, int nrhs,
                         Shape s, int grid, bool ind, bool vec, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    const size_t lds = size_t(s.waves) * kBatchLds;
    return by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        if (ind)
            hipLaunchKernelGGL((k_batch_adjoint<VT, LL, VX, true>), dim3(grid), dim3(block), lds, st, descs, items,
                               nitems, nrhs);
        else
            hipLaunchKernelGGL((k_batch_adjoint<VT, LL, VX, false>), dim3(grid), dim3(block), lds, st, descs, items,
                               nitems, nrhs);
        return hipGetLastError();
    });
}

int batch_occupancy(csrk_dtype store, int nrhs, Shape s, bool adj, bool ind, bool vec) {
    int blocks = 1;
    const int block = s.waves * kWave;
    const hipError_t e = by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        if (adj) {
            const size_t lds = size_t(s.waves) * kBatchLds;
            return ind ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_adjoint<VT, LL, VX, true>,
                                                                      block, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_adjoint<VT, LL, VX, false>,
                                                                      block, lds);
        }
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_forward<VT, LL, VX>, block,
                                                            size_t(s.waves) * batch_forward_lds<VT>(nrhs));
    });
    return (e != hipSuccess || blocks < 1) ? 1 : blocks;
}


}  // namespace dev
}  // namespace csrk
