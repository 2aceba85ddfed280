// Adjoint kernels (grad_x = A'^T g, grad_vals = g_i x_j) for one and for
// several right-hand sides, with their launcher.
#include "common.hpp"

namespace csrk {
namespace dev {

namespace {

// How the single-right-hand-side adjoint walks a matrix: grad_vals over A'
// and then grad_x over the same rows of A'^T (two-phase), one pass over A'
// for a symmetric pattern (fused), or one pass over the union pattern of a
// nonsymmetric A' (union; srec_t then holds the union records).
enum AdjMode { kTwoPhase = 0, kFused = 1, kUnion = 2 };

template <typename VT, int L, bool IND, int MODE, bool ADAPT>
__global__ void __launch_bounds__(1024) k_adjoint_csrk(const SrRec *__restrict__ srec, const SrRec *__restrict__ srec_t,
                                                       int32_t stride,
                                                       const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ cols,
                                                       const int32_t *__restrict__ t_row_ptr,
                                                       const int32_t *__restrict__ t_col,
                                                       const int32_t *__restrict__ t_src, const VT *__restrict__ valsT,
                                                       const typename Store<VT>::X *__restrict__ x,
                                                       const typename Store<VT>::X *__restrict__ g,
                                                       typename Store<VT>::X *__restrict__ gx,
                                                       typename Store<VT>::A *__restrict__ gv, int64_t nnz, int sym,
                                                       const int32_t *__restrict__ long_rows, int32_t na,
                                                       const int32_t *__restrict__ t_long_rows, int32_t nt,
                                                       int32_t long_blocks, XcdSplit split,
                                                       const int32_t *__restrict__ erow_ptr, int64_t nu) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const int32_t bid = int32_t(blockIdx.x);
    if (bid < long_blocks) {
        if constexpr (MODE != kUnion) {
            if (bid < na + nt)
                long_row_adjoint<VT, IND, MODE == kFused>(bid, long_rows, na, t_long_rows, row_ptr, cols, t_row_ptr,
                                                          t_col, t_src, valsT, x, g, gx, gv, nnz, smem, wave, nw,
                                                          lane);
        }
        return;
    }
    unsigned char *lds = smem + size_t(wave) * kAdjointLds;
    const int32_t t = ssr_of_block(split, bid - long_blocks);
    if (t < 0) return;
    // one instantiation per path keeps the other path's registers out of it
    using A = typename Store<VT>::A;
    // the SSR's super-rows from its records (slots past its last SR are empty)
    for (int32_t w = wave; w < stride; w += nw) {
        const SrRec rec = srec[int64_t(t) * stride + w];
        if (rec.r0 >= rec.r1) break;
        if constexpr (MODE == kFused) {
            sr_adjoint_fused_rec<VT, L, IND, ADAPT>(rec, row_ptr, cols, t_src, valsT, x, g, gx, gv, nnz, lds, lane,
                                                    true);
        } else if constexpr (MODE == kUnion) {
            // t_col / t_src / valsT are the union pattern's columns, sources and values here
            sr_adjoint_union_rec<VT, L, IND>(rec, srec_t[int64_t(t) * stride + w], row_ptr, erow_ptr, t_col, t_src,
                                             valsT, x, g, gx, gv, nu, lds, lane);
        } else {
            // the same rows of A'^T (grad_x = their product with g)
            const SrRec rect = srec_t[int64_t(t) * stride + w];
            if (gv) sr_grad_vals_rec<VT>(rec, row_ptr, cols, x, g, gv, nnz, lds, lane, true);
            if (gx)
                sr_forward_rec<VT, L, IND, ADAPT>(rect, t_row_ptr, t_col, t_src, valsT, g, gx, nnz,
                                                  reinterpret_cast<A *>(lds) + kStagePad, lane, true);
        }
    }
}

template <typename VT, int RL, int VX, bool IND>
__global__ void __launch_bounds__(1024) k_adjoint_csrk_mrhs(
    const SrRec *__restrict__ srec, int32_t stride, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ cols, const int32_t *__restrict__ t_row_ptr, const int32_t *__restrict__ t_col,
    const int32_t *__restrict__ t_src, const VT *__restrict__ valsT, const typename Store<VT>::X *__restrict__ x,
    const typename Store<VT>::X *__restrict__ g, typename Store<VT>::X *__restrict__ gx,
    typename Store<VT>::A *__restrict__ gv, int64_t nnz, int nrhs, int sym, XcdSplit split,
    const SrRec *__restrict__ srec_u, const int32_t *__restrict__ erow_ptr, const int32_t *__restrict__ u_col,
    const int32_t *__restrict__ u_src, const VT *__restrict__ u_vals, int64_t nu) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    unsigned char *lds = smem + size_t(wave) * (srec_u ? union_mrhs_lds<VT>() : mrhs_adjoint_lds<VT>());
    const int32_t t = ssr_of_block(split, int32_t(blockIdx.x));
    if (t < 0) return;
    for (int32_t w = wave; w < stride; w += nw) {
        const SrRec rec = srec[int64_t(t) * stride + w];
        if (rec.r0 >= rec.r1) break;
        if (sym != 0 && gx && gv) {
            sr_adjoint_fused_mrhs_rec<VT, RL, VX, IND>(rec, row_ptr, cols, t_src, valsT, x, g, gx, gv, nnz, nrhs, lds,
                                                       lane);
            continue;
        }
        if (srec_u && gx && gv) {  // nonsymmetric: one pass over the union pattern
            mrhs_adjoint_union_window<VT, RL, VX, IND>(rec, srec_u[int64_t(t) * stride + w], row_ptr, erow_ptr, u_col,
                                                       u_src, IND ? valsT : u_vals, x, g, gx, gv, nu, nrhs, lds, lane);
            continue;
        }
        sr_adjoint_mrhs<VT, RL, VX, IND>(rec.r0, rec.r1, row_ptr, cols, t_row_ptr, t_col, t_src, valsT, x, g, gx, gv,
                                         nnz, nrhs, sym != 0, lds, lane);
    }
}

}  // namespace

hipError_t adjoint(const Arrays &a, csrk_dtype store, const void *vals, const void *x, const void *g, void *gx,
                   void *gv, int nrhs, Shape s, hipStream_t st) {
    if (a.nssr == 0) return hipSuccess;
    const int block = s.waves * kWave;
    // Values passed by the caller are reached through the transposed map (the
    // union's source map on the union path); the handle's own values use its
    // stored transposed (union) copy.
    const bool ind = vals != nullptr;
    return by_dtype(store, [&](auto vt) -> hipError_t {
        using VT = decltype(vt);
        using X = typename Store<VT>::X;
        using A = typename Store<VT>::A;
        auto launch = [&](auto indc) -> hipError_t {
            constexpr bool IND = decltype(indc)::value;
            if (nrhs == 1) {
                return by_lanes(s.lanes_per_row, [&](auto lc) -> hipError_t {
                    constexpr int LL = decltype(lc)::value;
                    // The long rows the main blocks leave out: long rows of A' for
                    // grad_vals (and grad_x when fused), long rows of A'^T for grad_x
                    // otherwise.
                    const bool fused = a.sym && gx && gv;
                    const bool adapt = adapt_windows(a, LL);
                    // a nonsymmetric pattern whose union fits the windows takes one pass (no long rows there)
                    const bool uni = !a.sym && gx && gv && a.srec_u && !adapt;
                    const int32_t na = uni ? 0 : (fused || gv) ? a.nlong : 0;
                    const int32_t nt = uni ? 0 : (!fused && gx) ? a.t_nlong : 0;
                    const int32_t long_blocks = (na + nt + kXcds - 1) / kXcds * kXcds;
                    auto go = [&](auto mc) {
                        constexpr int M = decltype(mc)::value;
                        const VT *vsrc = static_cast<const VT *>(ind ? vals : M == kUnion ? a.u_vals : a.vals_t);
                        const int32_t *tcol = M == kUnion ? a.u_col : a.t_col;
                        const int32_t *tsrc = M == kUnion ? a.u_src : a.t_src;
                        const SrRec *rec_t = M == kUnion ? a.srec_u : a.srec_t;
                        by_adapt<LL>(M != kUnion && adapt, [&](auto ac) {
                            hipLaunchKernelGGL((k_adjoint_csrk<VT, LL, IND, M, decltype(ac)::value>),
                                               dim3(long_blocks + a.split_adj.width * kXcds), dim3(block),
                                               size_t(s.waves) * kAdjointLds, st, a.srec, rec_t, a.srec_stride,
                                               a.row_ptr, a.col_idx, a.t_row_ptr, tcol, tsrc, vsrc,
                                               static_cast<const X *>(x), static_cast<const X *>(g),
                                               static_cast<X *>(gx), static_cast<A *>(gv), a.nnz, int(a.sym),
                                               a.long_rows, na, a.t_long_rows, nt, long_blocks, a.split_adj,
                                               a.erow_ptr, a.nu);
                        });
                    };
                    if (fused)
                        go(std::integral_constant<int, kFused>{});
                    else if (uni)
                        go(std::integral_constant<int, kUnion>{});
                    else
                        go(std::integral_constant<int, kTwoPhase>{});
                    return hipGetLastError();
                });
            }
            const VT *vsrc = static_cast<const VT *>(ind ? vals : a.vals_t);
            const SrRec *srec_u = a.sym ? nullptr : a.srec_u;
            const size_t lds = size_t(s.waves) * (srec_u ? union_mrhs_lds<VT>() : mrhs_adjoint_lds<VT>());
            const int vx = vec_cols<X>(nrhs, {x, g, gx});
            return by_vx<X>(vx, [&](auto vc) -> hipError_t {
                constexpr int VX = decltype(vc)::value;
                return by_lanes(rhs_lanes(nrhs, VX), [&](auto rc) -> hipError_t {
                    constexpr int RL = decltype(rc)::value;
                    // with caller values the union pass reaches them through u_src (valsT is then the caller's)
                    hipLaunchKernelGGL((k_adjoint_csrk_mrhs<VT, RL, VX, IND>), dim3(a.split_adj.width * kXcds),
                                       dim3(block), lds, st, a.srec, a.srec_stride, a.row_ptr, a.col_idx,
                                       a.t_row_ptr, a.t_col, a.t_src, vsrc, static_cast<const X *>(x),
                                       static_cast<const X *>(g), static_cast<X *>(gx), static_cast<A *>(gv), a.nnz,
                                       nrhs, int(a.sym), a.split_adj, srec_u, a.erow_ptr, a.u_col, a.u_src,
                                       static_cast<const VT *>(a.u_vals), a.nu);
                    return hipGetLastError();
                });
            });
        };
        return ind ? launch(std::true_type{}) : launch(std::false_type{});
    });
}

}  // namespace dev
}  // namespace csrk
