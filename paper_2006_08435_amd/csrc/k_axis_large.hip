// Three-pass form for lengths above 128: the row (x) and strided (y, z)
// kernels with fewer lines per workgroup, so that a tile of whole lines
// still fits LDS (16 rows or 32 strided lines of up to 512 points).
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

// Adjacent lines per strided workgroup: 32, i.e. 256 contiguous bytes per
// element (16 lines, 128 bytes, measured 14% slower at 512^3), N * 33 * 8
// bytes of LDS (<= 135 KB at N = 512); rows per row-pass workgroup: 16
// (8 measured no faster at 512).
template <int N>
constexpr int large_lines()
{
    return 32;
}
template <int N>
constexpr int large_rows()
{
    return 16;
}

template <int N, int S>
static hipError_t launch_str_large(const float2* in, float2* out, const float2* tw, const AxisMap& m, int energy,
                                   const float*, double*, long, hipStream_t st)
{
    if (energy) return hipErrorInvalidValue;   // the energy form is provided up to 128 only
    constexpr int L = large_lines<N>();
    const long blocks = (m.lines + L - 1) / L;
    hipLaunchKernelGGL((k_axis_str<N, S, L, false>), dim3((unsigned)blocks), dim3(AxisGeom<N, L>::T), 0, st, in, out,
                       tw, m, nullptr, nullptr, 0L, 0.0, nullptr, 0L);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_row_large(const float2* in, float2* out, const float2* tw, long rows, hipStream_t st)
{
    constexpr int L = large_rows<N>();
    const long blocks = (rows + L - 1) / L;
    hipLaunchKernelGGL((k_axis_row<N, S, L>), dim3((unsigned)blocks), dim3(RowGeom<N, L>::T), 0, st, in, out, tw,
                       rows);
    return hipGetLastError();
}

#define FFT3D_STR_LARGE_CASE(n)                                                \
    case n:                                                                    \
        return sign < 0 ? &launch_str_large<n, -1> : &launch_str_large<n, 1>;
#define FFT3D_ROW_LARGE_CASE(n)                                                \
    case n:                                                                    \
        return sign < 0 ? &launch_row_large<n, -1> : &launch_row_large<n, 1>;
#define FFT3D_STR_LARGE_INFO(n)                                                \
    case n:                                                                    \
        return {AxisGeom<n, large_lines<n>()>::T, (int)(AxisGeom<n, large_lines<n>()>::WORDS * sizeof(float2))};
#define FFT3D_ROW_LARGE_INFO(n)                                                \
    case n:                                                                    \
        return {RowGeom<n, large_rows<n>()>::T, (int)(RowGeom<n, large_rows<n>()>::WORDS * sizeof(float2))};

AxisStrFn axis_str_large_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_LARGE_SIZE(FFT3D_STR_LARGE_CASE)
    default: return nullptr;
    }
}

AxisRowFn axis_row_large_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_LARGE_SIZE(FFT3D_ROW_LARGE_CASE)
    default: return nullptr;
    }
}

KernelInfo axis_str_large_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_LARGE_SIZE(FFT3D_STR_LARGE_INFO)
    default: return {0, 0};
    }
}

KernelInfo axis_row_large_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_LARGE_SIZE(FFT3D_ROW_LARGE_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
