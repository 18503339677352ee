// Whole-grid-in-LDS kernel instances (cubic N <= kCubeMaxN).
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N, int S>
static hipError_t launch_cube(const float2* in, float2* out, const float2* tw, long grids, hipStream_t st)
{
    hipLaunchKernelGGL((k_cube<N, S>), dim3((unsigned)grids), dim3(CubeGeom<N>::T), 0, st, in, out, tw);
    return hipGetLastError();
}

#define FFT3D_CUBE_CASE(n)                                                     \
    case n:                                                                    \
        return sign < 0 ? &launch_cube<n, -1> : &launch_cube<n, 1>;
#define FFT3D_CUBE_INFO(n)                                                     \
    case n:                                                                    \
        return {CubeGeom<n>::T, (int)(CubeGeom<n>::WORDS * sizeof(float2))};

CubeFn cube_fn(int n, int sign)
{
    switch (n) {
        FFT3D_CUBE_CASE(1) FFT3D_CUBE_CASE(2) FFT3D_CUBE_CASE(3) FFT3D_CUBE_CASE(4)
        FFT3D_CUBE_CASE(5) FFT3D_CUBE_CASE(6) FFT3D_CUBE_CASE(8) FFT3D_CUBE_CASE(9)
        FFT3D_CUBE_CASE(10) FFT3D_CUBE_CASE(12) FFT3D_CUBE_CASE(15) FFT3D_CUBE_CASE(16)
    default: return nullptr;
    }
}

KernelInfo cube_info(int n)
{
    switch (n) {
        FFT3D_CUBE_INFO(1) FFT3D_CUBE_INFO(2) FFT3D_CUBE_INFO(3) FFT3D_CUBE_INFO(4)
        FFT3D_CUBE_INFO(5) FFT3D_CUBE_INFO(6) FFT3D_CUBE_INFO(8) FFT3D_CUBE_INFO(9)
        FFT3D_CUBE_INFO(10) FFT3D_CUBE_INFO(12) FFT3D_CUBE_INFO(15) FFT3D_CUBE_INFO(16)
    default: return {0, 0};
    }
}

}  // namespace fft3d
