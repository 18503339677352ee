// Internal launcher tables of the FP32 kernels, one entry per supported
// transform length and sign.  Each launcher checks nothing: the planner has
// validated the geometry before calling it.
#pragma once
#include <hip/hip_runtime.h>

namespace fft3d {

struct AxisMap;
struct FusedCtl;
struct ManyArgs;
struct SphereRow;

using CubeFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long grids, hipStream_t st);
using PlaneFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long planes, hipStream_t st);
// scale != 0: fused prologue, input at r multiplied by 2 gE[0] V[r].
// stream: the input is cold (not just written by the pass before), so its
// loads may stream (stream_plane, kStreamMinBytes).
using PlanePfFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long planes, int grid, int scale,
                                 const float* V, const double* gE, int nz, bool stream, hipStream_t st);
// energy != 0: fused epilogue, V[r]|out(r)|^2 summed into one FP64 partial
// per workgroup (axis_str_blocks(m) of them) at `partials`; energy == 2: the
// sum only, `out` is not written.
using AxisStrFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, const AxisMap& m, int energy,
                                 const float* V, double* partials, long vol, hipStream_t st);
using AxisRowFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long rows, hipStream_t st);
using FusedFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, FusedCtl* ctl, int batch, int lag,
                               int grid, int chunk, hipStream_t st);

// Largest cubic length handled by the whole-grid-in-LDS kernel.
constexpr int kCubeMaxN = 16;
// Lines per workgroup of the strided-axis and row kernels.
constexpr int kAxisLines = 64;
constexpr int kRowLines = 16;

CubeFn cube_fn(int n, int sign);
long axis_str_blocks(long lines);
hipError_t launch_sum_partials(const double* partials, long n, double* out, hipStream_t st);
PlaneFn plane_fn(int n, int sign);
PlanePfFn plane_pf_fn(int n, int sign);
// Pruned transforms for the sphere |G|^2 < R2 (signed frequencies), both in
// the dense order (xy planes, then z).  Inverse (sign +1, input vanishing
// outside the sphere): plane pass over the planes of zlist reading only rows
// inside the sphere, then the z pass with zero loads for the other planes.
// Forward (sign -1, output wanted inside the sphere only): plane pass over
// every plane storing only the z-lines the sphere meets, then the z pass
// over those lines storing only the sphere.
// rows != nullptr selects the packed-sphere forms: the inverse plane pass
// gathers its input from a packed sphere of npts points per grid, the
// forward z pass scatters its output into one.
using PlanePrunedFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long planes, int grid,
                                     const int* zlist, int nzp, int nz, double R2, const SphereRow* rows, long npts,
                                     hipStream_t st);
using AxisStrPrunedFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, const AxisMap& m, double R2,
                                       const SphereRow* rows, long npts, hipStream_t st);
// Dense [batch][nz][ny][nx] <-> packed [batch][npts] (pack: gather, else scatter with zeros).
hipError_t launch_sphere_copy(bool pack, const float2* src, float2* dst, const SphereRow* rows, long npts, int nx,
                              long nyz, long total, hipStream_t st);
PlanePrunedFn plane_pruned_fn(int n, int sign);
// Forward plane pass over the planes of zlist storing only the sphere.
PlanePrunedFn plane_ball_fwd_fn(int n);
// z part of the local-potential operator (see k_axis_hloc); mode 1 = cutoff
// R2 (loads and stores limited to Gz^2 < R2).  partials: one FP64 per
// workgroup (axis_str_blocks(m.lines) of them), may be null.
using HlocFn = hipError_t (*)(float2* buf, const float2* tw_inv, const float2* tw_fwd, const AxisMap& m,
                              const float* V, const double* scale, float mult, double* partials, long vol, double R2,
                              int mode, hipStream_t st);
HlocFn axis_hloc_fn(int n);
// Density epilogue (see k_axis_density): m maps the z-lines of ONE grid,
// orbitals are `vol` apart in buf; mode 1 = cutoff R2.
using DensityFn = hipError_t (*)(const float2* buf, const float2* tw, const AxisMap& m, int batch, long vol,
                                 const float* occ, float* rho, double R2, int mode, hipStream_t st);
DensityFn axis_density_fn(int n);
AxisStrPrunedFn axis_str_pruned_fn(int n, int sign);
int plane_pf_blocks_per_cu(int n);
AxisStrFn axis_str_fn(int n, int sign);
AxisRowFn axis_row_fn(int n, int sign);
FusedFn fused_fn(int n, int sign);
// XCD-local variant; the control block is an XcdCtl (larger than FusedCtl).
using FusedXcdFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, FusedCtl* ctl, int batch, int lag,
                                  int grid, int q, hipStream_t st);
FusedXcdFn fused_xcd_fn(int n, int sign);
// Workgroups of the fused kernel (and of its XCD-local form) that fit on
// one compute unit at once.
int fused_blocks_per_cu(int n);
int fused_xcd_blocks_per_cu(int n);

// Schedule variants of the dense passes for the batched form's autotuner
// (k_variants.hip), sizes of FFT3D_FOR_EACH_MANY_SIZE: kind 2 = the
// alternative radix order (make_sched_alt; its twiddle table is
// twiddles(n, sign, 2)), z tiles of `lines` = 32 or 64 lines.  nullptr for
// combinations that are not compiled (kind 0 with 64 lines is the default
// pair, plane_pf_fn / axis_str_fn).
using PlaneVarFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, long planes, int grid, bool stream,
                                  hipStream_t st);
using AxisVarFn = hipError_t (*)(const float2* in, float2* out, const float2* tw, const AxisMap& m, hipStream_t st);
PlaneVarFn plane_variant_fn(int n, int sign, int kind);
AxisVarFn axis_variant_fn(int n, int sign, int kind, int lines);

// Heterogeneous persistent kernel (kernels_many.hpp); threads is 512 or 1024.
hipError_t launch_many(const ManyArgs& a, int sign, int threads, int grid, size_t lds_bytes, hipStream_t st);
int many_blocks_per_cu(int threads, size_t lds_bytes);
bool many_size_ok(int n);
size_t many_lds_bytes(int n, int threads);   // dynamic LDS one size-n item needs
int many_per_item(int n, int threads);       // planes (slabs) per work item

// Reduced-precision (scaled16) passes; fmt 1 = binary16, 2 = bfloat16.
using Q16PlaneFn = hipError_t (*)(const unsigned* in_pay, const signed char* in_exp, unsigned* mid_pay,
                                  signed char* mid_exp, const float2* tw, long planes, int fmt_in, hipStream_t st);
using Q16SlabFn = hipError_t (*)(const unsigned* mid_pay, const signed char* mid_exp, unsigned* out_pay,
                                 signed char* out_exp, const float2* tw, long slabs, int fmt_out, hipStream_t st);
Q16PlaneFn q16_plane_fn(int n, int sign);
Q16SlabFn q16_slab_fn(int n, int sign);
hipError_t launch_quantize(int fmt, const float2* in, long rows, int C, unsigned* pay, signed char* ex,
                           hipStream_t st);
hipError_t launch_dequantize(int fmt, const unsigned* pay, const signed char* ex, long rows, int C, float2* out,
                             hipStream_t st);

// Streaming copy of n16 16-byte elements (k_copy.hip).
hipError_t launch_stream_copy(const void* src, void* dst, long n16, hipStream_t st);

// Kernel geometry (threads, LDS bytes) for diagnostics.
struct KernelInfo {
    int threads;
    int lds_bytes;
};
KernelInfo cube_info(int n);
KernelInfo plane_info(int n);
KernelInfo axis_str_info(int n);
KernelInfo axis_row_info(int n);
KernelInfo fused_info(int n);
KernelInfo q16_info(int n);
// Lengths above 128 (three-pass form only); axis_str_fn / axis_row_fn and
// their _info functions forward to these for n > 128.
AxisStrFn axis_str_large_fn(int n, int sign);
AxisRowFn axis_row_large_fn(int n, int sign);
KernelInfo axis_str_large_info(int n);
KernelInfo axis_row_large_info(int n);

// Real-grid plane passes (Nx = Ny = n even): r2c (forward) real planes ->
// half-spectrum planes [n][n/2+1], c2r (inverse) the reverse.  tw_x is the
// length-n/2 table, tw_y the length-n table, rt the split/merge roots.
using RealPlaneFn = hipError_t (*)(const void* in, void* out, const float2* tw_x, const float2* tw_y,
                                   const float2* rt, long planes, int grid, hipStream_t st);
RealPlaneFn real_plane_fn(int n, bool forward);
int real_blocks_per_cu(int n, bool forward);
KernelInfo real_info(int n);

}  // namespace fft3d
