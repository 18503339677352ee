// Internal launcher tables of the FP32 kernels, one entry per supported
// transform length and sign.  Each launcher checks nothing: the planner has
// validated the geometry before calling it.
#pragma once
#include <hip/hip_runtime.h>

namespace fft3d {

struct AxisMap;

using CubeFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long grids, hipStream_t st);
using PlaneFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long planes, hipStream_t st);
using AxisStrFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, const AxisMap& m,
                                 hipStream_t st);
using AxisRowFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long rows, hipStream_t st);

// Largest cubic length handled by the whole-grid-in-LDS kernel.
constexpr int kCubeMaxN = 16;
// Lines per workgroup of the strided-axis and row kernels.
constexpr int kAxisLines = 64;
constexpr int kRowLines = 16;

CubeFn cube_fn(int n, int sign);
PlaneFn plane_fn(int n, int sign);
AxisStrFn axis_str_fn(int n, int sign);
AxisRowFn axis_row_fn(int n, int sign);

// Kernel geometry (threads, LDS bytes) for diagnostics.
struct KernelInfo {
    int threads;
    int lds_bytes;
};
KernelInfo cube_info(int n);
KernelInfo plane_info(int n);
KernelInfo axis_str_info(int n);
KernelInfo axis_row_info(int n);

}  // namespace fft3d
