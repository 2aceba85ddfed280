// Utility kernels: value conversion at upload, the transposed value copy and
// vector permutation; with their launchers.  Also two bandwidth probes (a
// streaming read and a copy with 16-byte non-temporal accesses) that measure
// the HBM rate attainable on the device, against which the products' achieved
// rates are read.
#include "common.hpp"

namespace csrk {
namespace dev {

namespace {

// ------------------------------------------------------------------ utilities

// out[p] = in[idx[p]] for p < count (0 where idx[p] < 0).
template <typename T>
__global__ void k_gather(const int32_t *__restrict__ idx, const T *__restrict__ in, T *__restrict__ out, int64_t count) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += int64_t(gridDim.x) * blockDim.x) {
        const int32_t i = idx[p];
        out[p] = i >= 0 ? in[i] : T(0);
    }
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

// Streaming read of n16 16-byte words: four independent non-temporal loads per
// lane in flight, a running xor per lane, one word per workgroup written to
// part[blockIdx.x] so the loads cannot be dropped.
constexpr int kProbeGrid = 4096, kProbeBlock = 256;
typedef uint32_t U4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kProbeBlock) k_probe_read(const U4 *__restrict__ p, int64_t n16,
                                                            double *__restrict__ part) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    uint32_t acc = 0;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        U4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
    }
    for (; i < n16; i += stride) {
        const U4 v = __builtin_nontemporal_load(p + i);
        acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
    }
    for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off);
    __shared__ uint32_t w[kProbeBlock / 64];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kProbeBlock / 64; ++k) t ^= w[k];
        part[blockIdx.x] = double(t);
    }
}

// Copy of n16 16-byte words with non-temporal loads and stores, four in flight per lane.
__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const U4 *__restrict__ src, U4 *__restrict__ dst,
                                                            int64_t n16) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        U4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

int probe_grid() { return kProbeGrid; }

hipError_t probe_read(const void *buf, int64_t bytes, double *part, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_read, dim3(kProbeGrid), dim3(kProbeBlock), 0, st, static_cast<const U4 *>(buf),
                       bytes / 16, part);
    return hipGetLastError();
}

hipError_t probe_copy(const void *src, void *dst, int64_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_copy, dim3(kProbeGrid), dim3(kProbeBlock), 0, st, static_cast<const U4 *>(src),
                       static_cast<U4 *>(dst), bytes / 16);
    return hipGetLastError();
}

hipError_t gather_values(const int32_t *idx, int64_t count, csrk_dtype store, const void *vals, void *out,
                         hipStream_t st) {
    if (count == 0) return hipSuccess;
    const int grid = grid_for(count, 256);
    switch (store) {
    case CSRK_F64:
        hipLaunchKernelGGL((k_gather<double>), dim3(grid), dim3(256), 0, st, idx, static_cast<const double *>(vals),
                           static_cast<double *>(out), count);
        break;
    case CSRK_F32:
        hipLaunchKernelGGL((k_gather<float>), dim3(grid), dim3(256), 0, st, idx, static_cast<const float *>(vals),
                           static_cast<float *>(out), count);
        break;
    case CSRK_BF16:
        hipLaunchKernelGGL((k_gather<uint16_t>), dim3(grid), dim3(256), 0, st, idx,
                           static_cast<const uint16_t *>(vals), static_cast<uint16_t *>(out), count);
        break;
    }
    return hipGetLastError();
}

hipError_t transpose_values(const Arrays &a, csrk_dtype store, const void *vals, void *vals_t, hipStream_t st) {
    return gather_values(a.t_src, a.nnz, store, vals, vals_t, st);
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

}  // namespace dev
}  // namespace csrk
