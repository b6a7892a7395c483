// Streaming copy kernels: the yardstick for achievable HBM bandwidth and for
// scaling hardware byte counters, and the serving loop's host-to-device
// staging copy (it reads pinned host memory across the link).
#include <algorithm>

#include "ldpc_internal.h"

namespace {

// One 16-byte element per thread over a grid that covers the buffer, with
// non-temporal loads and stores (streamed data, no reuse).  On MI355X this
// reaches about 6.5 TB/s for 1 GiB; a persistent grid-stride loop over the
// same buffer reaches only 4.1-5.1 TB/s.
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const v4f *__restrict__ src, v4f *__restrict__ dst, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// The link copy: a small fixed grid, each thread keeping kLinkUnroll 16-byte
// loads in flight per round.  Reads of pinned host memory wait microseconds
// on the link; a full grid would park one wave per 16 bytes on those waits
// and take the compute units' wave slots from kernels running beside it,
// while a few waves per compute unit already keep the link saturated.
constexpr int kLinkUnroll = 8;
__global__ __launch_bounds__(256) void k_copy_link(const v4f *__restrict__ src, v4f *__restrict__ dst, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; base < n;
         base += stride * kLinkUnroll) {
        v4f v[kLinkUnroll];
#pragma unroll
        for (int k = 0; k < kLinkUnroll; ++k) {
            const int64_t i = base + k * stride;
            if (i < n)
                v[k] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int k = 0; k < kLinkUnroll; ++k) {
            const int64_t i = base + k * stride;
            if (i < n)
                __builtin_nontemporal_store(v[k], dst + i);
        }
    }
}

bool copy_args_ok(const void *dst, const void *src, size_t bytes)
{
    return dst && src && bytes != 0 && bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(src) & 15) == 0 && bytes / 16 / 256 <= 0x7fffffff;
}

}  // namespace

namespace ldpc {

ldpc_status launch_link_copy16(void *dst, const void *src, size_t bytes, int32_t max_blocks, hipStream_t stream)
{
    if (!copy_args_ok(dst, src, bytes) || max_blocks < 1)
        return LDPC_EINVAL;
    const int64_t n = static_cast<int64_t>(bytes / 16);
    const int64_t blocks = std::min<int64_t>(max_blocks, (n + 255) / 256);
    ProfScope ps(LDPC_KERNEL_OTHER, stream);
    LDPC_LAUNCH(ps, k_copy_link, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                static_cast<const v4f *>(src), static_cast<v4f *>(dst), n);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

ldpc_status launch_copy16(void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    if (!copy_args_ok(dst, src, bytes))
        return LDPC_EINVAL;
    const int64_t n = static_cast<int64_t>(bytes / 16);
    const int64_t blocks = (n + 255) / 256;
    ProfScope ps(LDPC_KERNEL_OTHER, stream);
    LDPC_LAUNCH(ps, k_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, static_cast<const v4f *>(src),
                static_cast<v4f *>(dst), n);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

}  // namespace ldpc

extern "C" ldpc_status ldpc_copy_probe(void *dst, const void *src, size_t bytes, void *stream)
try {
    return ldpc::launch_copy16(dst, src, bytes, static_cast<hipStream_t>(stream));
} catch (...) {
    return ldpc::status_of_exception();
}
