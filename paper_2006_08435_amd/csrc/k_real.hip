// Real-grid (r2c / c2r) plane-pass instances for every even supported N.
#include "kernels_real.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N>
static int real_occ(bool forward)
{
    int nb = 0;
    const void* k = forward ? reinterpret_cast<const void*>(&k_plane_r2c<N, -1>)
                            : reinterpret_cast<const void*>(&k_plane_c2r<N, 1>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, RealGeom<N>::T, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

template <int N>
static hipError_t launch_r2c(const void* in, void* out, const float2* tw_x, const float2* tw_y, const float2* rt,
                             long planes, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_plane_r2c<N, -1>), dim3((unsigned)grid), dim3(RealGeom<N>::T), 0, st,
                       static_cast<const float*>(in), static_cast<float2*>(out), tw_x, tw_y, rt, planes);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_c2r(const void* in, void* out, const float2* tw_x, const float2* tw_y, const float2* rt,
                             long planes, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_plane_c2r<N, 1>), dim3((unsigned)grid), dim3(RealGeom<N>::T), 0, st,
                       static_cast<const float2*>(in), static_cast<float*>(out), tw_x, tw_y, rt, planes);
    return hipGetLastError();
}

#define FFT3D_REAL_CASE(n)                                                     \
    case n:                                                                    \
        return forward ? &launch_r2c<n> : &launch_c2r<n>;
#define FFT3D_REAL_OCC(n)                                                      \
    case n:                                                                    \
        return real_occ<n>(forward);
#define FFT3D_REAL_INFO(n)                                                     \
    case n:                                                                    \
        return {RealGeom<n>::T, (int)(RealGeom<n>::WORDS * sizeof(float2))};

RealPlaneFn real_plane_fn(int n, bool forward)
{
    switch (n) {
        FFT3D_FOR_EACH_EVEN_SIZE(FFT3D_REAL_CASE)
    default: return nullptr;
    }
}

int real_blocks_per_cu(int n, bool forward)
{
    switch (n) {
        FFT3D_FOR_EACH_EVEN_SIZE(FFT3D_REAL_OCC)
    default: return 1;
    }
}

KernelInfo real_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_EVEN_SIZE(FFT3D_REAL_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
