// Schedule variants of the two dense passes for the batched form's
// autotuner: the plane pass and the z pass with the alternative radix order
// (schedule kind 2), and the z pass with 32-line tiles, for every size of
// the heterogeneous batches.  Kind 0 with 64-line tiles is the default pair
// (plane_pf_fn / axis_str_fn).
#include "kernels_fp32.hpp"
#include "many_sizes.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N, int S, int K>
static hipError_t launch_plane_v(const float2* in, float2* out, const float2* tw, long planes, int grid, bool stream,
                                 hipStream_t st)
{
    const dim3 g((unsigned)grid), b(PlaneGeom<N>::T);
    constexpr long pb = (long)N * N * sizeof(float2);
    if (stream && planes * pb >= kStreamMinBytes)
        hipLaunchKernelGGL((k_plane_pf<N, S, false, true, K>), g, b, 0, st, in, out, tw, planes, nullptr, nullptr, N,
                           streamed_store_planes(planes, pb));
    else
        hipLaunchKernelGGL((k_plane_pf<N, S, false, false, K>), g, b, 0, st, in, out, tw, planes, nullptr, nullptr, N,
                           0L);
    return hipGetLastError();
}

template <int N, int S, int K, int L>
static hipError_t launch_axis_v(const float2* in, float2* out, const float2* tw, const AxisMap& m, hipStream_t st)
{
    const long blocks = (m.lines + L - 1) / L;
    hipLaunchKernelGGL((k_axis_str<N, S, L, false, 0, K>), dim3((unsigned)blocks), dim3(AxisGeom<N, L>::T), 0, st, in,
                       out, tw, m, nullptr, nullptr, 0L, 0.0, nullptr, 0L);
    return hipGetLastError();
}

#define FFT3D_PLANE_V_CASE(n)                                                  \
    case n:                                                                    \
        return sign < 0 ? &launch_plane_v<n, -1, 2> : &launch_plane_v<n, 1, 2>;

PlaneVarFn plane_variant_fn(int n, int sign, int kind)
{
    if (kind != 2) return nullptr;
    switch (n) {
        FFT3D_FOR_EACH_MANY_SIZE(FFT3D_PLANE_V_CASE)
    default: return nullptr;
    }
}

#define FFT3D_AXIS_V_CASE(n)                                                                   \
    case n:                                                                                    \
        if (kind == 2 && lines == 64) return sign < 0 ? &launch_axis_v<n, -1, 2, 64> : &launch_axis_v<n, 1, 2, 64>; \
        if (kind == 2 && lines == 32) return sign < 0 ? &launch_axis_v<n, -1, 2, 32> : &launch_axis_v<n, 1, 2, 32>; \
        if (kind == 0 && lines == 32) return sign < 0 ? &launch_axis_v<n, -1, 0, 32> : &launch_axis_v<n, 1, 0, 32>; \
        return nullptr;

AxisVarFn axis_variant_fn(int n, int sign, int kind, int lines)
{
    switch (n) {
        FFT3D_FOR_EACH_MANY_SIZE(FFT3D_AXIS_V_CASE)
    default: return nullptr;
    }
}

}  // namespace fft3d
