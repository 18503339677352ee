// Arguments of the heterogeneous persistent kernel (kernels_many.hpp), shared
// with the host code that builds its work list.
#pragma once
#include <hip/hip_runtime.h>

namespace fft3d {

struct FusedCtl;

constexpr int kMaxGroups = 16;

struct ManyGrid {
    int n;        // cubic size of this grid
    int group;    // index into the exec's in/out pointer arrays
    long offset;  // first element of the grid in its group's buffers
};

struct ManyArgs {
    const float2* in[kMaxGroups];
    float2* out[kMaxGroups];
    const ManyGrid* grids;
    const unsigned* items;
    long nitems;
    const float2* tw;    // twiddle tables of every size in the plan
    const int* tw_off;   // tw_off[n]: offset of the length-n table
    FusedCtl* ctl;
    int chunk;
    int ngrids;
};

// item = grid << 8 | slab << 7 | index
__host__ __device__ constexpr unsigned many_item(unsigned grid, unsigned slab, unsigned idx)
{
    return grid << 8 | slab << 7 | idx;
}

}  // namespace fft3d
