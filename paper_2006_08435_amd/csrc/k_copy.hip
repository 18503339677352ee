// Streaming device copy: the practical HBM bandwidth that the transform
// passes are measured against.  One 16-byte non-temporal load and store per
// element, one element per thread in a single sweep (grid-stride beyond
// 2^20 workgroups).
#include <hip/hip_runtime.h>

#include "registry.hpp"

namespace fft3d {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr long kCopyMaxBlocks = 1L << 20;

__global__ void __launch_bounds__(kCopyThreads) k_stream_copy(const f4v* __restrict__ src, f4v* __restrict__ dst,
                                                              long n)
{
    const long stride = (long)gridDim.x * kCopyThreads;
    for (long i = (long)blockIdx.x * kCopyThreads + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void* src, void* dst, long n16, hipStream_t st)
{
    if (n16 == 0) return hipSuccess;
    long blocks = (n16 + kCopyThreads - 1) / kCopyThreads;
    if (blocks > kCopyMaxBlocks) blocks = kCopyMaxBlocks;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st,
                       static_cast<const f4v*>(src), static_cast<f4v*>(dst), n16);
    return hipGetLastError();
}

}  // namespace fft3d
