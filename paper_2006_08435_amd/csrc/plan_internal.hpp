// Internal plan state shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fft3d.h"
#include "kernels_fp32.hpp"
#include "many_args.hpp"
#include "many_sizes.hpp"
#include "registry.hpp"
#include "sched.hpp"

namespace fft3d {

int set_error(int code);
int last_error_value();
void clear_error();
bool env_flag(const char* name);
// Twiddle table of a length-n transform for exponent sign `sign` (sched.hpp layout).
std::vector<float2> twiddles(int n, int sign, int kind = 0);
// The same table written to t[0 .. len) without allocating; returns len, or
// -1 if it exceeds cap.
int twiddles_into(float2* t, int cap, int n, int sign, int kind = 0);

// One kernel launch of an exec.  The first pass reads the caller's input,
// every later pass works in place on the output buffer.
struct Pass {
    enum Kind { kCubeK, kPlaneK, kPlanePfK, kRowK, kStrK, kFusedK, kQ16PlaneK, kQ16SlabK, kPlanePrunedK, kStrPrunedK, kRealK } kind;
    int n;        // transform length of this pass
    long count;   // grids / planes / rows (cube, plane, row kinds)
    AxisMap map;  // strided kind
    long tw;      // offset of this pass's twiddle table in d_tw
    int grid;     // workgroups of a persistent launch
};

// Heterogeneous batch (fft3d_plan_many): groups of cubic grids, one
// persistent launch over a host-built work list.
struct ManyPlan {
    int ngroups = 0;
    int n[kMaxGroups] = {};
    int batch[kMaxGroups] = {};
    std::vector<ManyGrid> grids;
    ManyGrid* d_grids = nullptr;
    unsigned* d_items = nullptr;
    long nitems = 0;
    long items_cap = 0;
    int* d_twoff = nullptr;
    int threads = 1024;   // 0: grouped mode (two plain passes per group) instead of the persistent kernel
    int chunk = 2;
    // hybrid mode: the groups marked big (enough planes to fill the device)
    // run their two plain passes, the others share one persistent launch
    bool hybrid = false;
    bool big[kMaxGroups] = {};
    int twoff_host[129] = {};   // offset of the length-n table in the plan's twiddles
    int twoff_alt[129] = {};    // offset of the length-n table of the alternative radix order
    // per group, for its plain passes (grouped mode, and the big groups of
    // the hybrid mode): radix order (0 default, 2 alternative) and z-tile
    // lines (64 or 32); chosen by the tuner or fft3d_plan_set_group_schedule
    int kind[kMaxGroups] = {};
    int zlines[kMaxGroups] = {};
    int grid = 1;
    size_t lds = 0;
    bool tuned = false;
    double tuned_ms = 0.0;
};

}  // namespace fft3d

struct fft3d_plan_s {
    int nx, ny, nz, batch, precision, direction;
    int scheme;
    int device;
    float2* d_tw;              // all tables of the plan, one allocation
    long tw_x, tw_y, tw_z;     // offsets (elements) of each dimension's table
    long tw_rx, tw_ry, tw_rz;  // the same tables for the opposite sign
    long vol;
    double* partials;          // energy: one FP64 partial per z-pass workgroup (nx == ny plans)
    long n_partials;
    int pf_grid;               // workgroups of the persistent plane pass (nx == ny plans)
    std::vector<fft3d::Pass> passes;
    fft3d::FusedCtl* ctl;      // persistent-kernel control block (fused / many)
    size_t ctl_bytes;          // its allocated size
    int fused_grid;            // workgroups of the persistent launch
    int fused_lag;             // dependency lag in grids
    int fused_chunk;           // items per queue claim (0: static round robin)
    int fused_xcd;             // > 0: XCD-local variant with this many queues
    bool q16_valu;             // scaled16 plans: radix-16 stage on the vector ALUs instead of MFMA
    double cut_r2;             // > 0: sphere cutoff of the pruned inverse (fft3d_plan_set_cutoff)
    int* d_zlist;              // z-planes with Gz^2 < cut_r2 (device), n_zlist of them
    int n_zlist;
    fft3d::SphereRow* d_rows;  // packed-sphere row table [nz][ny] (device)
    long sphere_pts;           // points per grid inside the cutoff sphere
    std::vector<fft3d::Pass> dense_passes;   // schedule without the cutoff
    bool real;                 // plan from fft3d_plan_real (r2c forward / c2r inverse)
    long tw_rt;                // real plans: offset of the split/merge roots W_N^{direction*k}, k <= N/4
    bool many;                 // plan from fft3d_plan_many
    fft3d::ManyPlan mp;
};

namespace fft3d {
// fft3d_plan_describe text of a plan from fft3d_plan_many.
int many_describe(fft3d_plan_t p, char* buf, size_t len);
}  // namespace fft3d
