// fft3d_energy_noalloc: the local-potential energy E = sum V |psi|^2 of
// fft3d_energy (psi = unnormalised inverse transform of the orbitals, summed
// on chip, never written) for callers that cannot allocate device memory.
// No plan: the twiddle tables and the per-workgroup FP64 partial sums,
// which a plan keeps in memory it allocated, live here in one fixed device
// array per GPU.  The kernels are exactly those of fft3d_energy (xy-plane
// pass, E-only z pass, fixed-order partial sum) with the same host-generated
// tables, so E is bit-identical to fft3d_energy's.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "plan_internal.hpp"

// One copy per GPU, held until the process ends: 1 MiB (see the layout
// below).  In host code this name is only a handle for hipGetSymbolAddress,
// never a device address.
static __device__ __align__(256) unsigned char scratch[size_t(1) << 20];

namespace fft3d {
namespace {

// Layout of the per-device array: the two twiddle tables (x and z, sign +1,
// kTabCap complex values each), then the partial sums from kPartialsOff on.
constexpr size_t kScratchBytes = sizeof(scratch);
constexpr int kTabCap = 128;   // a length-n table (n <= 128) has fewer than n entries
constexpr size_t kPartialsOff = 4096;
constexpr long kMaxPartials = (long)((kScratchBytes - kPartialsOff) / sizeof(double));
constexpr int kMaxDevices = 64;
static_assert(2 * kTabCap * sizeof(float2) <= kPartialsOff, "tables overlap the partials");

// Both tables travel by value in the launch arguments (no host-to-device
// copy, so the call can be captured in a graph) and are written to the array.
struct Tables {
    float2 v[2 * kTabCap];
};

__global__ void __launch_bounds__(256) k_fill_tables(Tables t, float2* __restrict__ dst)
{
    for (int i = threadIdx.x; i < 2 * kTabCap; i += 256) dst[i] = t.v[i];
}

std::mutex g_mu;
void* g_scratch[kMaxDevices];
int g_cus[kMaxDevices];

// Address of device `dev`'s array, and its compute-unit count, looked up
// once per device with that device current (the caller's current device).
int device_scratch(int dev, void** ptr, int* cus)
{
    if (dev < 0 || dev >= kMaxDevices) return FFT3D_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return FFT3D_E_LAUNCH;
        }
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) {
            (void)hipGetLastError();
            n = 1;
        }
        g_cus[dev] = n;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    *cus = g_cus[dev];
    return FFT3D_OK;
}

}  // namespace
}  // namespace fft3d

using namespace fft3d;

extern "C" int fft3d_energy_noalloc(int nx, int ny, int nz, int batch, const void* c, const float* V, void* work,
                                    double* E_dev, fft3d_stream_t stream)
{
    if (!c || !V || !work || !E_dev || nx < 1 || ny < 1 || nz < 1 || batch < 1) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)c % 16) || ((uintptr_t)work % 16) || ((uintptr_t)V % 16) || ((uintptr_t)E_dev % 8))
        return FFT3D_E_ALIGNMENT;
    if (!size_supported(nx) || !size_supported(ny) || !size_supported(nz)) return FFT3D_E_UNSUPPORTED_SIZE;
    if (nx != ny) return FFT3D_E_UNSUPPORTED;
    const long vol = (long)nx * ny * nz;
    if ((long)batch * vol > (1L << 36)) return FFT3D_E_INVALID_ARG;
    const long lines = (long)batch * ny * nx;
    const long n_partials = axis_str_blocks(lines);
    if (n_partials > kMaxPartials) return FFT3D_E_SCRATCH;
    const PlanePfFn plane = plane_pf_fn(nx, FFT3D_INVERSE);
    const AxisStrFn zpass = axis_str_fn(nz, FFT3D_INVERSE);
    if (!plane || !zpass) return FFT3D_E_UNSUPPORTED;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_NO_DEVICE;
    }
    void* base = nullptr;
    int cus = 1;
    const int rc = device_scratch(dev, &base, &cus);
    if (rc != FFT3D_OK) return rc;
    Tables t{};
    if (twiddles_into(t.v, kTabCap, nx, FFT3D_INVERSE) < 0 || twiddles_into(t.v + kTabCap, kTabCap, nz, FFT3D_INVERSE) < 0)
        return FFT3D_E_UNSUPPORTED;
    float2* tab = static_cast<float2*>(base);
    double* partials = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kPartialsOff);

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fill_tables, dim3(1), dim3(256), 0, st, t, tab);
    hipError_t e = hipGetLastError();
    const long planes = (long)batch * nz;
    const long resident = (long)plane_pf_blocks_per_cu(nx) * cus;
    const int grid = (int)(planes < resident ? planes : resident);
    if (e == hipSuccess)
        e = plane(static_cast<const float2*>(c), static_cast<float2*>(work), tab, planes, grid, 0, nullptr, nullptr, nz,
                  true, st);
    const AxisMap zmap{lines, nx, ny, vol, (long)nx, (long)nx * ny};
    if (e == hipSuccess)
        e = zpass(static_cast<float2*>(work), static_cast<float2*>(work), tab + kTabCap, zmap, 2, V, partials, vol, st);
    if (e == hipSuccess) e = launch_sum_partials(partials, n_partials, E_dev, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}
