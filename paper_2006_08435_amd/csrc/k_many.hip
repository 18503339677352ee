// Heterogeneous persistent kernel instances (both signs, 512 or 1024 threads).
#include "kernels_many.hpp"
#include "registry.hpp"

namespace fft3d {

template <int S, int T>
static hipError_t launch(const ManyArgs& a, int grid, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((k_many<S, T>), dim3((unsigned)grid), dim3(T), lds, st, a);
    return hipGetLastError();
}

template <int T>
static int occ(size_t lds)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_many<-1, T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_many<1, T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_many<-1, T>), T, lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t launch_many(const ManyArgs& a, int sign, int threads, int grid, size_t lds, hipStream_t st)
{
    if (threads == 512) return sign < 0 ? launch<-1, 512>(a, grid, lds, st) : launch<1, 512>(a, grid, lds, st);
    return sign < 0 ? launch<-1, 1024>(a, grid, lds, st) : launch<1, 1024>(a, grid, lds, st);
}

int many_blocks_per_cu(int threads, size_t lds) { return threads == 512 ? occ<512>(lds) : occ<1024>(lds); }

bool many_size_ok(int n) { return many_size_supported(n); }

size_t many_lds_bytes(int n, int threads)
{
    switch (n) {
#define FFT3D_MANY_LDS(m)                                                                                  \
    case m:                                                                                                \
        return sizeof(float2) * (threads == 1024 ? many_lds_need<m, 1024>() : many_lds_need<m, 512>());
        FFT3D_FOR_EACH_MANY_SIZE(FFT3D_MANY_LDS)
#undef FFT3D_MANY_LDS
    default: return 0;
    }
}

int many_per_item(int n, int threads)
{
    switch (n) {
#define FFT3D_MANY_PER(m)                                                                                  \
    case m:                                                                                                \
        return threads == 1024 ? many_per<m, 1024>() : many_per<m, 512>();
        FFT3D_FOR_EACH_MANY_SIZE(FFT3D_MANY_PER)
#undef FFT3D_MANY_PER
    default: return 1;
    }
}

}  // namespace fft3d
