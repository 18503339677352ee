// Reduced-precision (scaled16) kernel instances and launchers.
#include "kernels_q16.hpp"
#include "registry.hpp"

namespace fft3d {

// Persistent launches: as many workgroups as fit the device at once (the
// occupancy of the kernel times the compute units), capped by the work.
static long resident_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        return 1;
    }
    return cus;
}

template <class K>
static long persistent_grid(K kernel, int threads, long work)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kernel), threads, 0) !=
            hipSuccess ||
        nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    const long g = (long)nb * resident_cus();
    return work < g ? work : g;
}

// fmt: 1 binary16, 2 bfloat16; +16 selects the vector-ALU radix-16 stage.
template <int N, int S, int F, bool M>
static void plane_k(const unsigned* ip, const signed char* ie, unsigned* mp, signed char* me, const float2* tw,
                    long planes, hipStream_t st)
{
    // streaming input loads as in the FP32 plane pass (same lengths, passes
    // of at least kStreamMinBytes of payload)
    if constexpr (stream_plane(N)) {
        if (planes * N * N * (long)sizeof(unsigned) >= kStreamMinBytes) {
            const long grid = persistent_grid(&k_q16_plane<N, S, F, M, true>, Q16Geom<N>::T, planes);
            hipLaunchKernelGGL((k_q16_plane<N, S, F, M, true>), dim3((unsigned)grid), dim3(Q16Geom<N>::T), 0, st, ip,
                               ie, mp, me, tw, planes);
            return;
        }
    }
    const long grid = persistent_grid(&k_q16_plane<N, S, F, M>, Q16Geom<N>::T, planes);
    hipLaunchKernelGGL((k_q16_plane<N, S, F, M>), dim3((unsigned)grid), dim3(Q16Geom<N>::T), 0, st, ip, ie, mp, me,
                       tw, planes);
}

template <int N, int S, int F, bool M>
static void slab_k(const unsigned* mp, const signed char* me, unsigned* op, signed char* oe, const float2* tw,
                   long slabs, hipStream_t st)
{
    const long grid = persistent_grid(&k_q16_slab<N, S, F, M>, Q16Geom<N>::T, slabs);
    hipLaunchKernelGGL((k_q16_slab<N, S, F, M>), dim3((unsigned)grid), dim3(Q16Geom<N>::T), 0, st, mp, me, op, oe,
                       tw, slabs);
}

template <int N, int S>
static hipError_t launch_plane(const unsigned* ip, const signed char* ie, unsigned* mp, signed char* me,
                               const float2* tw, long planes, int fmt_in, hipStream_t st)
{
    const bool valu = fmt_in & 16;
    const int f = fmt_in & 15;
    if (f == kFmtF16) (valu ? plane_k<N, S, kFmtF16, false> : plane_k<N, S, kFmtF16, true>)(ip, ie, mp, me, tw, planes, st);
    else (valu ? plane_k<N, S, kFmtBF16, false> : plane_k<N, S, kFmtBF16, true>)(ip, ie, mp, me, tw, planes, st);
    return hipGetLastError();
}

template <int N, int S>
static hipError_t launch_slab(const unsigned* mp, const signed char* me, unsigned* op, signed char* oe,
                              const float2* tw, long slabs, int fmt_out, hipStream_t st)
{
    const bool valu = fmt_out & 16;
    const int f = fmt_out & 15;
    if (f == kFmtF16) (valu ? slab_k<N, S, kFmtF16, false> : slab_k<N, S, kFmtF16, true>)(mp, me, op, oe, tw, slabs, st);
    else (valu ? slab_k<N, S, kFmtBF16, false> : slab_k<N, S, kFmtBF16, true>)(mp, me, op, oe, tw, slabs, st);
    return hipGetLastError();
}

#define FFT3D_Q16_SIZES(X) X(16) X(32) X(48) X(64) X(80) X(96) X(128)

Q16PlaneFn q16_plane_fn(int n, int sign)
{
    switch (n) {
#define C(m) \
    case m: return sign < 0 ? &launch_plane<m, -1> : &launch_plane<m, 1>;
        FFT3D_Q16_SIZES(C)
#undef C
    default: return nullptr;
    }
}

Q16SlabFn q16_slab_fn(int n, int sign)
{
    switch (n) {
#define C(m) \
    case m: return sign < 0 ? &launch_slab<m, -1> : &launch_slab<m, 1>;
        FFT3D_Q16_SIZES(C)
#undef C
    default: return nullptr;
    }
}

KernelInfo q16_info(int n)
{
    switch (n) {
#define C(m) \
    case m: return {Q16Geom<m>::T, (int)(Q16Geom<m>::WORDS * sizeof(float2) + m * sizeof(int))};
        FFT3D_Q16_SIZES(C)
#undef C
    default: return {0, 0};
    }
}

hipError_t launch_quantize(int fmt, const float2* in, long rows, int C, unsigned* pay, signed char* ex,
                           hipStream_t st)
{
    const long blocks = (rows + 3) / 4;
    if (blocks == 0) return hipSuccess;
    if (fmt == kFmtF16)
        hipLaunchKernelGGL(k_q16_quantize<kFmtF16>, dim3((unsigned)blocks), dim3(256), 0, st, in, rows, C, pay, ex);
    else
        hipLaunchKernelGGL(k_q16_quantize<kFmtBF16>, dim3((unsigned)blocks), dim3(256), 0, st, in, rows, C, pay, ex);
    return hipGetLastError();
}

hipError_t launch_dequantize(int fmt, const unsigned* pay, const signed char* ex, long rows, int C, float2* out,
                             hipStream_t st)
{
    const long blocks = (rows * C + 255) / 256;
    if (blocks == 0) return hipSuccess;
    if (fmt == kFmtF16)
        hipLaunchKernelGGL(k_q16_dequantize<kFmtF16>, dim3((unsigned)blocks), dim3(256), 0, st, pay, ex, rows, C, out);
    else
        hipLaunchKernelGGL(k_q16_dequantize<kFmtBF16>, dim3((unsigned)blocks), dim3(256), 0, st, pay, ex, rows, C,
                           out);
    return hipGetLastError();
}

}  // namespace fft3d
