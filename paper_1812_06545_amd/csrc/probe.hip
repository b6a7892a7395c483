// Streaming copy kernel: the yardstick for achievable HBM bandwidth and for
// scaling hardware byte counters, and the serving loop's host-to-device
// staging copy (it reads pinned host memory across the link).
#include <algorithm>

#include "ldpc_internal.h"

namespace {

// Each thread moves 4 float4 per step, all loads before the stores, so
// enough bytes are in flight to cover the memory latency.
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n)
{
    constexpr int kU = 4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + (kU - 1) * stride < n; i += kU * stride) {
        float4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

namespace ldpc {

ldpc_status launch_copy16(void *dst, const void *src, size_t bytes, int cus, hipStream_t stream)
{
    if (!dst || !src || bytes == 0 || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) ||
        (reinterpret_cast<uintptr_t>(src) & 15) || cus < 1)
        return LDPC_EINVAL;
    const int64_t n = static_cast<int64_t>(bytes / 16);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, static_cast<int64_t>(cus) * 32);
    ProfScope ps(LDPC_KERNEL_OTHER, stream);
    hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

}  // namespace ldpc

extern "C" ldpc_status ldpc_copy_probe(void *dst, const void *src, size_t bytes, void *stream)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LDPC_EDEVICE;
    return ldpc::launch_copy16(dst, src, bytes, cus, static_cast<hipStream_t>(stream));
}
