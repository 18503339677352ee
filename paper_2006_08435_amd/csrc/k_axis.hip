// Single-axis pass kernel instances: strided (y, z) and row (x) forms.
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N, int S>
static hipError_t launch_axis_str(const float2* in, float2* out, const float2* tw, const AxisMap& m,
                                  hipStream_t st)
{
    const long blocks = (m.lines + kAxisLines - 1) / kAxisLines;
    hipLaunchKernelGGL((k_axis_str<N, S, kAxisLines>), dim3((unsigned)blocks), dim3(AxisGeom<N, kAxisLines>::T), 0,
                       st, in, out, tw, m);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_axis_row(const float2* in, float2* out, const float2* tw, long rows, hipStream_t st)
{
    const long blocks = (rows + kRowLines - 1) / kRowLines;
    hipLaunchKernelGGL((k_axis_row<N, S, kRowLines>), dim3((unsigned)blocks), dim3(RowGeom<N, kRowLines>::T), 0, st,
                       in, out, tw, rows);
    return hipGetLastError();
}

#define FFT3D_STR_CASE(n)                                                      \
    case n:                                                                    \
        return sign < 0 ? &launch_axis_str<n, -1> : &launch_axis_str<n, 1>;
#define FFT3D_ROW_CASE(n)                                                      \
    case n:                                                                    \
        return sign < 0 ? &launch_axis_row<n, -1> : &launch_axis_row<n, 1>;
#define FFT3D_STR_INFO(n)                                                      \
    case n:                                                                    \
        return {AxisGeom<n, kAxisLines>::T,                                    \
                (int)((Plan1D<n>::stages > 1 ? AxisGeom<n, kAxisLines>::WORDS : 1) * sizeof(float2))};
#define FFT3D_ROW_INFO(n)                                                      \
    case n:                                                                    \
        return {RowGeom<n, kRowLines>::T, (int)(RowGeom<n, kRowLines>::WORDS * sizeof(float2))};

AxisStrFn axis_str_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_STR_CASE)
    default: return nullptr;
    }
}

AxisRowFn axis_row_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_ROW_CASE)
    default: return nullptr;
    }
}

KernelInfo axis_str_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_STR_INFO)
    default: return {0, 0};
    }
}

KernelInfo axis_row_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_ROW_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
