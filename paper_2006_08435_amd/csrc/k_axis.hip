// Single-axis pass kernel instances: strided (y, z) and row (x) forms.
#include "kernels_fp32.hpp"
#include "registry.hpp"

namespace fft3d {

// Sum of n FP64 partials in a fixed order (one workgroup of 256 threads).
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ p, long n, double* __restrict__ out)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (long i = tid; i < n; i += 256) s += p[i];
    red[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[0] = red[0];
}

long axis_str_blocks(long lines) { return (lines + kAxisLines - 1) / kAxisLines; }

hipError_t launch_sum_partials(const double* partials, long n, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, n, out);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_axis_str(const float2* in, float2* out, const float2* tw, const AxisMap& m, int energy,
                                  const float* V, double* partials, long vol, hipStream_t st)
{
    const long blocks = axis_str_blocks(m.lines);
    if (energy == 2) {
        hipLaunchKernelGGL((k_axis_energy<N, S, kAxisLines>), dim3((unsigned)blocks),
                           dim3(AxisGeom<N, kAxisLines>::T), 0, st, in, tw, m, V, partials, vol);
        return hipGetLastError();
    }
    if (energy)
        hipLaunchKernelGGL((k_axis_str<N, S, kAxisLines, true>), dim3((unsigned)blocks),
                           dim3(AxisGeom<N, kAxisLines>::T), 0, st, in, out, tw, m, V, partials, vol, 0.0);
    else
        hipLaunchKernelGGL((k_axis_str<N, S, kAxisLines, false>), dim3((unsigned)blocks),
                           dim3(AxisGeom<N, kAxisLines>::T), 0, st, in, out, tw, m, V, partials, vol, 0.0);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_axis_str_pruned(const float2* in, float2* out, const float2* tw, const AxisMap& m, double R2,
                                         const SphereRow* rows, long npts, hipStream_t st)
{
    const long blocks = axis_str_blocks(m.lines);
    // inverse plans prune the loads (sphere-limited input), forward plans
    // lines and stores (optionally scattering into a packed sphere)
    if constexpr (S < 0) {
        if (rows) {
            hipLaunchKernelGGL((k_axis_str<N, S, kAxisLines, false, 3>), dim3((unsigned)blocks),
                               dim3(AxisGeom<N, kAxisLines>::T), 0, st, in, out, tw, m, nullptr, nullptr, 0L, R2, rows,
                               npts);
            return hipGetLastError();
        }
    } else {
        if (rows) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_axis_str<N, S, kAxisLines, false, (S > 0 ? 1 : 2)>), dim3((unsigned)blocks),
                       dim3(AxisGeom<N, kAxisLines>::T), 0, st, in, out, tw, m, nullptr, nullptr, 0L, R2, nullptr, 0L);
    return hipGetLastError();
}

#define FFT3D_STR_PRUNED_CASE(n)                                               \
    case n:                                                                    \
        return sign < 0 ? &launch_axis_str_pruned<n, -1> : &launch_axis_str_pruned<n, 1>;

AxisStrPrunedFn axis_str_pruned_fn(int n, int sign)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_STR_PRUNED_CASE)
    default: return nullptr;
    }
}

template <int N>
static hipError_t launch_hloc(float2* buf, const float2* tw_inv, const float2* tw_fwd, const AxisMap& m,
                              const float* V, const double* scale, float mult, double* partials, long vol, double R2,
                              int mode, hipStream_t st)
{
    const long blocks = axis_str_blocks(m.lines);
    if (mode)
        hipLaunchKernelGGL((k_axis_hloc<N, kAxisLines, 1>), dim3((unsigned)blocks), dim3(AxisGeom<N, kAxisLines>::T),
                           0, st, buf, tw_inv, tw_fwd, m, V, scale, mult, partials, vol, R2);
    else
        hipLaunchKernelGGL((k_axis_hloc<N, kAxisLines, 0>), dim3((unsigned)blocks), dim3(AxisGeom<N, kAxisLines>::T),
                           0, st, buf, tw_inv, tw_fwd, m, V, scale, mult, partials, vol, R2);
    return hipGetLastError();
}

#define FFT3D_HLOC_CASE(n)                                                     \
    case n:                                                                    \
        return &launch_hloc<n>;

HlocFn axis_hloc_fn(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_HLOC_CASE)
    default: return nullptr;
    }
}

constexpr int kDensityLines = 32;

template <int N>
static hipError_t launch_density(const float2* buf, const float2* tw, const AxisMap& m, int batch, long vol,
                                 const float* occ, float* rho, double R2, int mode, hipStream_t st)
{
    const long blocks = (m.lines + kDensityLines - 1) / kDensityLines;
    if (mode)
        hipLaunchKernelGGL((k_axis_density<N, kDensityLines, 1>), dim3((unsigned)blocks),
                           dim3(AxisGeom<N, kDensityLines>::T), 0, st, buf, tw, m, batch, vol, occ, rho, R2);
    else
        hipLaunchKernelGGL((k_axis_density<N, kDensityLines, 0>), dim3((unsigned)blocks),
                           dim3(AxisGeom<N, kDensityLines>::T), 0, st, buf, tw, m, batch, vol, occ, rho, R2);
    return hipGetLastError();
}

#define FFT3D_DENSITY_CASE(n)                                                  \
    case n:                                                                    \
        return &launch_density<n>;

DensityFn axis_density_fn(int n)
{
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_DENSITY_CASE)
    default: return nullptr;
    }
}

hipError_t launch_sphere_copy(bool pack, const float2* src, float2* dst, const SphereRow* rows, long npts, int nx,
                              long nyz, long total, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    long blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;   // grid-stride beyond 2M points
    if (pack)
        hipLaunchKernelGGL((k_sphere_copy<true>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, rows, npts, nx,
                           nyz, total);
    else
        hipLaunchKernelGGL((k_sphere_copy<false>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, rows, npts, nx,
                           nyz, total);
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
    if (n > 128) return axis_str_large_fn(n, sign);
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_STR_CASE)
    default: return nullptr;
    }
}

AxisRowFn axis_row_fn(int n, int sign)
{
    if (n > 128) return axis_row_large_fn(n, sign);
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_ROW_CASE)
    default: return nullptr;
    }
}

KernelInfo axis_str_info(int n)
{
    if (n > 128) return axis_str_large_info(n);
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_STR_INFO)
    default: return {0, 0};
    }
}

KernelInfo axis_row_info(int n)
{
    if (n > 128) return axis_row_large_info(n);
    switch (n) {
        FFT3D_FOR_EACH_SIZE(FFT3D_ROW_INFO)
    default: return {0, 0};
    }
}

}  // namespace fft3d
