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
                                                        const SrRec *__restrict__ brec, int32_t stride,
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
        const VT *vals = global_ptr(static_cast<const VT *>(d.vals));
        const X *x = global_ptr(static_cast<const X *>(d.x));
        X *y = global_ptr(static_cast<X *>(d.y));
        const int32_t *row_ptr = global_ptr(d.row_ptr), *col_idx = global_ptr(d.col_idx);
        // the item's super-rows from its records (slots past its last SR are empty)
        for (int32_t w = wave; w < stride; w += nw) {
            const SrRec rec = brec[int64_t(it) * stride + w];
            if (rec.r0 >= rec.r1) break;
            if (nrhs == 1)
                sr_forward_rec<VT, L, false>(rec, row_ptr, col_idx, nullptr, vals, x, y, d.nnz,
                                             reinterpret_cast<A *>(lds) + kStagePad, lane, false);
            else
                sr_forward_mrhs_rec<VT, L, VX, false>(rec, row_ptr, col_idx, nullptr, vals, x, y, d.nnz, nrhs, lds,
                                                      lane);
        }
    }
}

// Adjoint paths of a batched launch, one instantiation each so that a launch
// carries only its own path's registers: one right-hand side (fused or
// two-phase per matrix), several right-hand sides with every matrix
// symmetric (fused only), several right-hand sides in general (fused or
// two-phase per matrix).
enum BatchAdjPath { kAdjSingle = 0, kAdjMrhsFused = 1, kAdjMrhsAny = 2 };

// LDS bytes per wavefront of a batched adjoint path (the general
// multi-column path may take the union window).
template <typename VT, int PATH>
__host__ __device__ constexpr int adj_lds() {
    return PATH == kAdjSingle ? kBatchLds : PATH == kAdjMrhsFused ? mrhs_adjoint_lds<VT>() : union_mrhs_lds<VT>();
}

template <typename VT, int L, int VX, bool IND, int PATH>
__global__ void __launch_bounds__(1024) k_batch_adjoint(const MatDesc *__restrict__ descs, const int2 *__restrict__ items,
                                                        const SrRec *__restrict__ brec,
                                                        const SrRec *__restrict__ brec_u, int32_t stride,
                                                        int32_t nitems, int nrhs) {
    using A = typename Store<VT>::A;
    using X = typename Store<VT>::X;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    unsigned char *lds = smem + size_t(wave) * adj_lds<VT, PATH>();
    const int32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int32_t per = (nitems + gridDim.x - 1) / gridDim.x;
    const int32_t i0 = b * per, i1 = min(nitems, i0 + per);
    for (int32_t it = i0; it < i1; ++it) {
        const int2 item = items[it];
        const MatDesc d = descs[item.x];
        const VT *vals = global_ptr(static_cast<const VT *>(d.vals));
        const X *x = global_ptr(static_cast<const X *>(d.x));
        const X *g = global_ptr(static_cast<const X *>(d.g));
        X *gx = global_ptr(static_cast<X *>(d.gx));
        A *gv = global_ptr(static_cast<A *>(d.gv));
        const int32_t *row_ptr = global_ptr(d.row_ptr), *col_idx = global_ptr(d.col_idx);
        const int32_t *t_row_ptr = global_ptr(d.t_row_ptr), *t_col = global_ptr(d.t_col);
        const int32_t *t_src = global_ptr(d.t_src);
        // the item's super-rows from its records (slots past its last SR are empty)
        for (int32_t w = wave; w < stride; w += nw) {
            const SrRec rec = brec[int64_t(it) * stride + w];
            if (rec.r0 >= rec.r1) break;
            const int32_t r0 = rec.r0, r1 = rec.r1;
            // a nonsymmetric matrix with a union-pattern index: both gradients in one pass over it (values
            // reached through u_src when the caller passes them)
            const bool uni = d.uni != 0 && gx && gv;
            if constexpr (PATH == kAdjSingle) {
                if (uni) {
                    sr_adjoint_union_rec<VT, L, IND>(rec, brec_u[int64_t(it) * stride + w], row_ptr,
                                                     global_ptr(d.erow_ptr), global_ptr(d.u_col),
                                                     global_ptr(d.u_src),
                                                     IND ? vals : global_ptr(static_cast<const VT *>(d.u_vals)), x, g,
                                                     gx, gv, d.nu, lds, lane);
                    continue;
                }
                sr_adjoint<VT, L, IND>(r0, r1, row_ptr, col_idx, t_row_ptr, t_col, t_src, vals, x, g, gx, gv, d.nnz,
                                       d.sym != 0, lds, lane, false);
            } else if constexpr (PATH == kAdjMrhsFused) {
                sr_adjoint_fused_mrhs_rec<VT, L, VX, IND>(rec, row_ptr, col_idx, t_src, vals, x, g, gx, gv, d.nnz,
                                                          nrhs, lds, lane);
            } else {
                if (uni) {
                    mrhs_adjoint_union_window<VT, L, VX, IND>(
                        rec, brec_u[int64_t(it) * stride + w], row_ptr, global_ptr(d.erow_ptr), global_ptr(d.u_col),
                        global_ptr(d.u_src), IND ? vals : global_ptr(static_cast<const VT *>(d.u_vals)), x, g, gx, gv,
                        d.nu, nrhs, lds, lane);
                    continue;
                }
                sr_adjoint_mrhs<VT, L, VX, IND>(r0, r1, row_ptr, col_idx, t_row_ptr, t_col, t_src, vals, x, g, gx, gv,
                                                d.nnz, nrhs, d.sym != 0, lds, lane);
            }
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

hipError_t batch_forward(const MatDesc *descs, const int2 *items, const SrRec *brec, int32_t stride, int32_t nitems,
                         csrk_dtype store, int nrhs, Shape s, int grid, bool vec, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    return by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        hipLaunchKernelGGL((k_batch_forward<VT, LL, VX>), dim3(grid), dim3(block),
                           size_t(s.waves) * batch_forward_lds<VT>(nrhs), st, descs, items, brec, stride, nitems,
                           nrhs);
        return hipGetLastError();
    });
}

// The adjoint path for a launch: several right-hand sides over symmetric
// patterns with both outputs take the fused-only instantiation.
inline int adj_path(int nrhs, bool all_sym, bool both) {
    if (nrhs == 1) return kAdjSingle;
    return (all_sym && both) ? kAdjMrhsFused : kAdjMrhsAny;
}

// Instantiations that a launch can choose: one right-hand side runs with one
// column per lane.
template <typename VT, int VX, int PATH>
constexpr bool adj_variant_exists() {
    if constexpr (PATH == kAdjSingle) return VX == 1;
    return true;
}

// Calls f(integral_constant<bool, IND>, integral_constant<int, PATH>).
template <typename F>
hipError_t by_adj_variant(bool ind, int path, F &&f) {
    auto with_path = [&](auto ic) -> hipError_t {
        switch (path) {
        case kAdjSingle:
            return f(ic, std::integral_constant<int, kAdjSingle>{});
        case kAdjMrhsFused:
            return f(ic, std::integral_constant<int, kAdjMrhsFused>{});
        default:
            return f(ic, std::integral_constant<int, kAdjMrhsAny>{});
        }
    };
    return ind ? with_path(std::true_type{}) : with_path(std::false_type{});
}

hipError_t batch_adjoint(const MatDesc *descs, const int2 *items, const SrRec *brec, const SrRec *brec_u,
                         int32_t stride, int32_t nitems, csrk_dtype store, int nrhs, Shape s, int grid, bool ind,
                         bool vec, bool all_sym, bool both, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const int block = s.waves * kWave;
    const int path = adj_path(nrhs, all_sym, both);
    return by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        return by_adj_variant(ind, path, [&](auto ic, auto pc) -> hipError_t {
            constexpr bool IND = decltype(ic)::value;
            constexpr int PATH = decltype(pc)::value;
            if constexpr (!adj_variant_exists<VT, VX, PATH>()) {
                return hipErrorInvalidValue;  // never chosen (see adj_variant_exists)
            } else {
                const size_t lds = size_t(s.waves) * adj_lds<VT, PATH>();
                hipLaunchKernelGGL((k_batch_adjoint<VT, LL, VX, IND, PATH>), dim3(grid), dim3(block), lds, st, descs,
                                   items, brec, brec_u, stride, nitems, nrhs);
                return hipGetLastError();
            }
        });
    });
}

int batch_occupancy(csrk_dtype store, int nrhs, Shape s, bool adj, bool ind, bool vec, bool all_sym, bool both) {
    int blocks = 1;
    const int block = s.waves * kWave;
    const hipError_t e = by_batch_shape(store, nrhs, s, vec, [&](auto vt, auto vc, auto lc) -> hipError_t {
        using VT = decltype(vt);
        constexpr int VX = decltype(vc)::value, LL = decltype(lc)::value;
        if (adj) {
            return by_adj_variant(ind, adj_path(nrhs, all_sym, both), [&](auto ic, auto pc) -> hipError_t {
                constexpr bool IND = decltype(ic)::value;
                constexpr int PATH = decltype(pc)::value;
                if constexpr (!adj_variant_exists<VT, VX, PATH>())
                    return hipErrorInvalidValue;
                else
                    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &blocks, k_batch_adjoint<VT, LL, VX, IND, PATH>, block, size_t(s.waves) * adj_lds<VT, PATH>());
            });
        }
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_forward<VT, LL, VX>, block,
                                                            size_t(s.waves) * batch_forward_lds<VT>(nrhs));
    });
    return (e != hipSuccess || blocks < 1) ? 1 : blocks;
}


}  // namespace dev
}  // namespace csrk
