// membw.hip -- a streaming copy kernel that sets the achievable HBM bandwidth
// the traversal's memory traffic is compared against.
//
// Each lane moves 16-byte words (dwordx4 loads and stores) in a grid-stride
// loop with four words in flight; loads and stores are non-temporal so the
// copy streams through the caches instead of filling them.  The grid is a
// fixed number of workgroups per compute unit, so every CU keeps many waves of
// outstanding requests whatever the size.
#include <hip/hip_runtime.h>

#include "rsi_internal.h"

namespace rsi {
namespace {

typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr int kCopyBlocksPerCU = 8;
constexpr int kCopyInFlight = 4;

__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const U32x4 *__restrict__ src, U32x4 *__restrict__ dst,
                                                            int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kCopyInFlight - 1) * stride < n; i += kCopyInFlight * stride) {
        U32x4 v[kCopyInFlight];
#pragma unroll
        for (int k = 0; k < kCopyInFlight; ++k)
            v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < kCopyInFlight; ++k)
            __builtin_nontemporal_store(v[k], dst + i + k * stride);
    }
    for (; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

hipError_t launch_stream_copy(void *dst, const void *src, int64_t n16, hipStream_t s) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = (n16 + kCopyThreads - 1) / kCopyThreads;
    const int64_t cap = (int64_t)cus * kCopyBlocksPerCU;
    const int grid = (int)(want < cap ? want : cap);
    if (grid > 0)
        k_stream_copy<<<grid, kCopyThreads, 0, s>>>(static_cast<const U32x4 *>(src), static_cast<U32x4 *>(dst), n16);
    return hipGetLastError();
}

}  // namespace rsi
