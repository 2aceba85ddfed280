// Conjugate gradients on top of the CSR-k product (the paper names CG for
// PDE systems as the application its format is meant for: Section 1 and the
// conclusions).  The matrix product runs in the handle's storage precision;
// the CG vectors x, r, p and every reduction are FP64, so the residual that
// decides convergence is accumulated in FP64 whatever the matrix storage.
//
// Reductions are deterministic: a fixed grid writes one FP64 partial sum per
// workgroup (each summed in a fixed order), and one workgroup adds the
// partials in index order.  p . Ap comes the same way from the workgroups of
// the product itself (spmv_dot), so p and q are not read again for it, and
// x moves in the pass that rebuilds p.  The scalars rr, pq, alpha, beta stay
// on the device, so an iteration is a sequence of launches on one stream with
// no host round trip; the host only reads rr when it checks convergence.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace csrk {
namespace dev {

namespace {

constexpr int kBlock = 256;
constexpr int kWaveSize = 64;

// Sum of v over the workgroup (kBlock threads) in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int off = kWaveSize / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x / kWaveSize;
    if ((threadIdx.x % kWaveSize) == 0) sh[wave] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / kWaveSize; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// part[block] = sum over this block's grid-stride share of a[i] * b[i].
template <typename TB>
__global__ void __launch_bounds__(kBlock) k_dot_partial(const double *__restrict__ a, const TB *__restrict__ b,
                                                        int64_t n, double *__restrict__ part) {
    __shared__ double sh[kBlock / kWaveSize];
    double acc = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
        acc += a[i] * double(b[i]);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

constexpr int kFinishBlock = 1024;

// s[slot] = sum of part[0..count) (one workgroup); then, for mode 1:
// alpha = rr / pq; mode 2: beta = rr_new / rr, rr = rr_new.  Thread t adds
// part[t], part[t + 1024], ... in that order (coalesced; the loads of a
// thread are independent, so they are issued together), then the threads'
// sums are combined in a fixed order.  Scalars: s[0] = rr, s[1] = pq,
// s[2] = alpha, s[3] = beta, s[4] = rr_new, s[5] = b . b.
__global__ void __launch_bounds__(kFinishBlock) k_finish(const double *__restrict__ part, int count,
                                                         double *__restrict__ s, int slot, int mode) {
    __shared__ double sh[kFinishBlock / kWaveSize];
    double acc = 0;
#pragma unroll 8
    for (int i = threadIdx.x; i < count; i += kFinishBlock) acc += part[i];
#pragma unroll
    for (int off = kWaveSize / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x % kWaveSize) == 0) sh[threadIdx.x / kWaveSize] = acc;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kFinishBlock / kWaveSize; ++w) t += sh[w];
    if (threadIdx.x == 0) {
        s[slot] = t;
        if (mode == 1) s[2] = s[0] / s[1];
        if (mode == 2) {
            s[3] = t / s[0];
            s[0] = t;
        }
    }
}

// r -= alpha q; part[block] = partial sum of r . r.  (x moves in
// k_update_xp, which reads p anyway.)
template <typename TQ>
__global__ void __launch_bounds__(kBlock) k_update_r(double *__restrict__ r, const TQ *__restrict__ q,
                                                     const double *__restrict__ s, int64_t n,
                                                     double *__restrict__ part) {
    __shared__ double sh[kBlock / kWaveSize];
    const double alpha = s[2];
    double acc = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const double ri = r[i] - alpha * double(q[i]);
        r[i] = ri;
        acc += ri * ri;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += alpha p (the direction of this iteration), then p = r + beta p.
__global__ void __launch_bounds__(kBlock) k_update_xp(double *__restrict__ x, double *__restrict__ p,
                                                      float *__restrict__ p_lo, const double *__restrict__ r,
                                                      const double *__restrict__ s, int64_t n) {
    const double alpha = s[2], beta = s[3];
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const double pi = p[i];
        x[i] += alpha * pi;
        const double pn = r[i] + beta * pi;
        p[i] = pn;
        if (p_lo) p_lo[i] = float(pn);
    }
}

// p = r + beta p (beta_from_s: beta = s[3]; otherwise p = r); p_lo = p rounded
// to the product's vector type when that is not FP64.
__global__ void __launch_bounds__(kBlock) k_update_p(const double *__restrict__ r, double *__restrict__ p,
                                                     float *__restrict__ p_lo, const double *__restrict__ s,
                                                     int64_t n, int beta_from_s) {
    const double beta = beta_from_s ? s[3] : 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const double pi = r[i] + beta * (beta_from_s ? p[i] : 0.0);
        p[i] = pi;
        if (p_lo) p_lo[i] = float(pi);
    }
}

// r = b - q (q = A x0), part = partial sums of r . r.
template <typename TQ>
__global__ void __launch_bounds__(kBlock) k_residual(const double *__restrict__ b, const TQ *__restrict__ q,
                                                     double *__restrict__ r, int64_t n, double *__restrict__ part) {
    __shared__ double sh[kBlock / kWaveSize];
    double acc = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const double ri = b[i] - double(q[i]);
        r[i] = ri;
        acc += ri * ri;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_round_f32(const double *__restrict__ v, float *__restrict__ out,
                                                      int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
        out[i] = float(v[i]);
}

}  // namespace

int cg_grid(int64_t n) {
    const int64_t g = (n + kBlock - 1) / kBlock;
    return int(g < 1 ? 1 : (g > kCgGrid ? kCgGrid : g));
}

hipError_t cg_residual(const double *b, const void *q, bool q_f32, double *r, int64_t n, double *part, double *s,
                       hipStream_t st) {
    const int grid = cg_grid(n);
    if (q_f32)
        hipLaunchKernelGGL((k_residual<float>), dim3(grid), dim3(kBlock), 0, st, b, static_cast<const float *>(q),
                           r, n, part);
    else
        hipLaunchKernelGGL((k_residual<double>), dim3(grid), dim3(kBlock), 0, st, b, static_cast<const double *>(q),
                           r, n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, part, grid, s, 0, 0);
    return hipGetLastError();
}

hipError_t cg_norm2(const double *b, int64_t n, double *part, double *s, hipStream_t st) {
    const int grid = cg_grid(n);
    hipLaunchKernelGGL((k_dot_partial<double>), dim3(grid), dim3(kBlock), 0, st, b, b, n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, part, grid, s, 5, 0);
    return hipGetLastError();
}

hipError_t cg_set_p(const double *r, double *p, float *p_lo, const double *s, int64_t n, bool use_beta,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_update_p, dim3(cg_grid(n)), dim3(kBlock), 0, st, r, p, p_lo, s, n, use_beta ? 1 : 0);
    return hipGetLastError();
}

hipError_t cg_alpha_parts(const double *part, int count, double *s, hipStream_t st) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, part, count, s, 1, 1);
    return hipGetLastError();
}

hipError_t cg_update_r(double *r, const void *q, bool q_f32, int64_t n, double *part, double *s, hipStream_t st) {
    const int grid = cg_grid(n);
    if (q_f32)
        hipLaunchKernelGGL((k_update_r<float>), dim3(grid), dim3(kBlock), 0, st, r, static_cast<const float *>(q), s,
                           n, part);
    else
        hipLaunchKernelGGL((k_update_r<double>), dim3(grid), dim3(kBlock), 0, st, r, static_cast<const double *>(q),
                           s, n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, part, grid, s, 4, 2);
    return hipGetLastError();
}

hipError_t cg_update_xp(double *x, double *p, float *p_lo, const double *r, const double *s, int64_t n,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_update_xp, dim3(cg_grid(n)), dim3(kBlock), 0, st, x, p, p_lo, r, s, n);
    return hipGetLastError();
}

hipError_t cg_round(const double *v, float *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_round_f32, dim3(cg_grid(n)), dim3(kBlock), 0, st, v, out, n);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace csrk
