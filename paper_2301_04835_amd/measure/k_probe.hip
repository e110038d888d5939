// Bandwidth probes: a plain streaming read and a plain copy of a known
// number of bytes.  They calibrate the hardware traffic counters (bytes
// fetched / written per byte moved) and give the achievable streaming rate
// of the device next to its nominal HBM peak.
#include <hip/hip_runtime.h>

#include "../../include/sampx_measure.h"

namespace {

constexpr int kBlock = 256;

typedef float nt_f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ float4 ld(const float4 *p)
{
    if (NT) {
        const nt_f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f32x4 *>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    }
    return *p;
}

// grid-stride float4 read; each workgroup writes one float so the loads
// cannot be dropped
template <bool NT>
__global__ void __launch_bounds__(kBlock) k_read(const float4 *__restrict__ src, int64_t n4, float *sink)
{
    __shared__ float red[kBlock / 64];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kBlock * 4;
    for (int64_t i = (int64_t)blockIdx.x * kBlock * 4 + threadIdx.x; i < n4; i += stride) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = i + u * kBlock < n4 ? ld<NT>(src + i + u * kBlock) : make_float4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one workgroup that does nothing: what a launch costs by itself
__global__ void __launch_bounds__(64) k_noop() {}

__global__ void __launch_bounds__(kBlock) k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" sx_status sx_probe_read(const void *src, size_t bytes, float *sink, int32_t grid, int32_t nontemporal,
                                   void *stream)
{
    if (!src || !sink || bytes % 16 || grid < 1) return SX_EINVAL;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const float4 *p = static_cast<const float4 *>(src);
    if (nontemporal)
        hipLaunchKernelGGL(k_read<true>, dim3(grid), dim3(kBlock), 0, s, p, (int64_t)(bytes / 16), sink);
    else
        hipLaunchKernelGGL(k_read<false>, dim3(grid), dim3(kBlock), 0, s, p, (int64_t)(bytes / 16), sink);
    return hipGetLastError() == hipSuccess ? SX_OK : SX_EDEVICE;
}

extern "C" sx_status sx_probe_noop(void *stream)
{
    hipLaunchKernelGGL(k_noop, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? SX_OK : SX_EDEVICE;
}

extern "C" sx_status sx_probe_copy(void *dst, const void *src, size_t bytes, int32_t grid, void *stream)
{
    if (!src || !dst || bytes % 16 || grid < 1) return SX_EINVAL;
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), (int64_t)(bytes / 16));
    return hipGetLastError() == hipSuccess ? SX_OK : SX_EDEVICE;
}
