// xy-plane (pass A) kernel instances, Nx = Ny = N for every supported N.
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

template <int N, int S>
static hipError_t launch_plane(const float2* in, float2* out, const float2* tw, long planes, hipStream_t st)
{
    hipLaunchKernelGGL((k_plane<N, S>), dim3((unsigned)planes), dim3(PlaneGeom<N>::T), 0, st, in, out, tw);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_plane_pf(const float2* in, float2* out, const float2* tw, long planes, int grid, int scale,
                                  const float* V, const double* gE, int nz, bool stream, hipStream_t st)
{
    const dim3 g((unsigned)grid), b(PlaneGeom<N>::T);
    if constexpr (stream_plane(N)) {
        constexpr long pb = (long)N * N * sizeof(float2);
        if (stream && planes * pb >= kStreamMinBytes) {
            const long ntp = streamed_store_planes(planes, pb);   // used where the stores are paired
            if (scale)
                hipLaunchKernelGGL((k_plane_pf<N, S, true, true>), g, b, 0, st, in, out, tw, planes, V, gE, nz, ntp);
            else
                hipLaunchKernelGGL((k_plane_pf<N, S, false, true>), g, b, 0, st, in, out, tw, planes, V, gE, nz, ntp);
            return hipGetLastError();
        }
    }
    if (scale)
        hipLaunchKernelGGL((k_plane_pf<N, S, true>), g, b, 0, st, in, out, tw, planes, V, gE, nz, 0L);
    else
        hipLaunchKernelGGL((k_plane_pf<N, S, false>), g, b, 0, st, in, out, tw, planes, V, gE, nz, 0L);
    return hipGetLastError();
}

template <int N>
static int plane_pf_occ()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_plane_pf<N, -1, false>),
                                                     PlaneGeom<N>::T, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb > 0 ? nb : 1;
}

#define FFT3D_PLANE_PF_CASE(n)                                                 \
    case n:                                                                    \
        return sign < 0 ? &launch_plane_pf<n, -1> : &launch_plane_pf<n, 1>;
#define FFT3D_PLANE_PF_OCC(n)                                                  \
    case n:                                                                    \
        return plane_pf_occ<n>();

PlanePfFn plane_pf_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_PF_CASE)
    default: return nullptr;
    }
}

int plane_pf_blocks_per_cu(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_PF_OCC)
    default: return 1;
    }
}

template <int N, int S>
static hipError_t launch_plane_pruned(const float2* in, float2* out, const float2* tw, long planes, int grid,
                                      const int* zlist, int nzp, int nz, double R2, const SphereRow* rows, long npts,
                                      hipStream_t st)
{
    // inverse plans prune planes and row loads (optionally gathering from a
    // packed sphere), forward plans the stores
    if constexpr (S > 0) {
        if (rows) {
            hipLaunchKernelGGL((k_plane_pruned<N, S, 0, true>), dim3((unsigned)grid), dim3(PlaneGeom<N>::T), 0, st,
                               in, out, tw, planes, zlist, nzp, nz, R2, rows, npts);
            return hipGetLastError();
        }
    } else {
        if (rows) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_plane_pruned<N, S, (S < 0 ? 1 : 0)>), dim3((unsigned)grid), dim3(PlaneGeom<N>::T), 0, st,
                       in, out, tw, planes, zlist, nzp, nz, R2, nullptr, 0L);
    return hipGetLastError();
}

// Forward plane pass over the planes of zlist, storing only the sphere
// (the last pass of the local-potential operator with a cutoff).
template <int N>
static hipError_t launch_plane_ball(const float2* in, float2* out, const float2* tw, long planes, int grid,
                                    const int* zlist, int nzp, int nz, double R2, const SphereRow*, long,
                                    hipStream_t st)
{
    hipLaunchKernelGGL((k_plane_pruned<N, -1, 2>), dim3((unsigned)grid), dim3(PlaneGeom<N>::T), 0, st, in, out, tw,
                       planes, zlist, nzp, nz, R2, nullptr, 0L);
    return hipGetLastError();
}

#define FFT3D_PLANE_BALL_CASE(n)                                               \
    case n:                                                                    \
        return &launch_plane_ball<n>;

PlanePrunedFn plane_ball_fwd_fn(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_BALL_CASE)
    default: return nullptr;
    }
}

#define FFT3D_PLANE_PRUNED_CASE(n)                                             \
    case n:                                                                    \
        return sign < 0 ? &launch_plane_pruned<n, -1> : &launch_plane_pruned<n, 1>;

PlanePrunedFn plane_pruned_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_PRUNED_CASE)
    default: return nullptr;
    }
}

#define FFT3D_PLANE_CASE(n)                                                    \
    case n:                                                                    \
        return sign < 0 ? &launch_plane<n, -1> : &launch_plane<n, 1>;
#define FFT3D_PLANE_INFO(n)                                                    \
    case n:                                                                    \
        return {PlaneGeom<n>::T, (int)(PlaneGeom<n>::WORDS * sizeof(float2))};

PlaneFn plane_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_CASE)
    default: return nullptr;
    }
}

KernelInfo plane_info(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_PLANE_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
