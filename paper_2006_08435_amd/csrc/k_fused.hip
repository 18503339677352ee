// Persistent fused (plane + z-slab) kernel instances, cubic N.
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N, int S>
static hipError_t launch_fused(const float2* in, float2* out, const float2* tw, FusedCtl* ctl, int batch, int lag,
                               int grid, int chunk, hipStream_t st)
{
    hipLaunchKernelGGL((k_fused<N, S>), dim3((unsigned)grid), dim3(PlaneGeom<N>::T), 0, st, in, out, tw, ctl, batch,
                       lag, chunk);
    return hipGetLastError();
}

template <int N>
static int occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_fused<N, -1>),
                                                     PlaneGeom<N>::T, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

template <int N, int S>
static hipError_t launch_fused_xcd(const float2* in, float2* out, const float2* tw, FusedCtl* ctl, int batch, int lag,
                                   int grid, int q, hipStream_t st)
{
    hipLaunchKernelGGL((k_fused_xcd<N, S>), dim3((unsigned)grid), dim3(PlaneGeom<N>::T), 0, st, in, out, tw,
                       reinterpret_cast<XcdCtl*>(ctl), batch, q, lag);
    return hipGetLastError();
}

template <int N>
static int occupancy_xcd()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_fused_xcd<N, -1>),
                                                     PlaneGeom<N>::T, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

#define FFT3D_FUSED_XCD_OCC(n)                                                 \
    case n:                                                                    \
        return occupancy_xcd<n>();

int fused_xcd_blocks_per_cu(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_FUSED_SIZE(FFT3D_FUSED_XCD_OCC)
    default: return 1;
    }
}

#define FFT3D_FUSED_XCD_CASE(n)                                                \
    case n:                                                                    \
        return sign < 0 ? &launch_fused_xcd<n, -1> : &launch_fused_xcd<n, 1>;

FusedXcdFn fused_xcd_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_FUSED_SIZE(FFT3D_FUSED_XCD_CASE)
    default: return nullptr;
    }
}

#define FFT3D_FUSED_CASE(n)                                                    \
    case n:                                                                    \
        return sign < 0 ? &launch_fused<n, -1> : &launch_fused<n, 1>;
#define FFT3D_FUSED_OCC(n)                                                     \
    case n:                                                                    \
        return occupancy<n>();
#define FFT3D_FUSED_INFO(n)                                                    \
    case n:                                                                    \
        return {PlaneGeom<n>::T, (int)(PlaneGeom<n>::WORDS * sizeof(float2))};

FusedFn fused_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_FUSED_SIZE(FFT3D_FUSED_CASE)
    default: return nullptr;
    }
}

int fused_blocks_per_cu(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_FUSED_SIZE(FFT3D_FUSED_OCC)
    default: return 1;
    }
}

KernelInfo fused_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_FUSED_SIZE(FFT3D_FUSED_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
