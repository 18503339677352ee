// Persistent kernel over a heterogeneous work list: many grids of different
// cubic sizes (and batch groups) transformed by ONE launch.
//
// The host builds a list of 32-bit work items in a global order: for every
// grid its N xy-plane items, and later its N xz-slab items (a slab item of a
// grid always comes after all plane items of that grid, at least `lag` items
// later).  Workgroups claim `chunk` consecutive items at a time from one
// queue counter and process them in order; a slab item waits (bounded spin)
// until its grid's plane counter reaches N.  Because items are claimed in
// list order, every item a slab item waits for is already held by a running
// workgroup (or done), so the wait always ends.  Hand-off between workgroups
// uses the device-coherent store/load protocol of k_fused.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels_fp32.hpp"
#include "many_args.hpp"
#include "many_sizes.hpp"

namespace fft3d {

struct ManyState {
    int pending;   // grid of this workgroup's last unpublished plane item, or -1
};

template <int T>
__device__ __forceinline__ void many_publish(FusedCtl* ctl, ManyState& st, int tid)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (st.pending >= 0 && tid == 0)
        __hip_atomic_fetch_add(&ctl->done[st.pending], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st.pending = -1;
}

// Group buffer pointers by a uniform select chain (no dynamic indexing of
// the by-value argument block, which would go through scratch memory).
__device__ __forceinline__ void group_ptrs(const ManyArgs& a, int g, const float2*& in, float2*& out)
{
    in = a.in[0];
    out = a.out[0];
#pragma unroll
    for (int k = 1; k < kMaxGroups; ++k)
        if (g == k) {
            in = a.in[k];
            out = a.out[k];
        }
}

// Planes (or slabs) per work item: items of grids with N <= 64 run four at
// once when the workgroup has 1024 threads (two when 4 does not divide N),
// each with its own LDS tile and T / PER threads (thread group h takes
// index idx + h).  On the mixed batch (256 x 64^3 + 48^3 ... 120^3) the
// single persistent launch took 0.527 ms with two and 0.456 ms with four:
// the 64^3 planes are latency-bound and want as many in flight per compute
// unit as the largest grid's LDS tile leaves room for.
template <int N, int T>
constexpr int many_per()
{
    return T == 1024 && N <= 64 ? (N % 4 == 0 ? 4 : 2) : 1;
}

// LDS floats2 needed by one size-N item.
template <int N, int T>
constexpr int many_lds_need()
{
    return many_per<N, T>() * PlaneGeom<N>::WORDS;
}

// One work item of a size-N grid; returns the workgroup's new unpublished
// plane-item grid (or -1).  Kept out of line so that every size gets its own
// register allocation instead of the maximum over all sizes.
template <int N, int S, int T>
__device__ __noinline__ int many_body(const float2* in, float2* out, const float2* __restrict__ tw, FusedCtl* ctl,
                                      long offset, int grid, int slab, int idx, float2* lds, int tid, int pending)
{
    constexpr unsigned PER = many_per<N, T>();    // planes/slabs per item
    constexpr int TH = T / PER;                     // threads per plane/slab
    constexpr int RS = PlaneGeom<N>::RS;
    const int sub = PER > 1 ? tid / TH : 0;
    const int ltid = PER > 1 ? tid % TH : tid;
    float2* my = lds + sub * PlaneGeom<N>::WORDS;
    const int j = idx + sub;
    ManyState st{pending};
    if (!slab) {
        const long base = offset + (long)j * N * N;
        tile_to_lds<N, N, RS, TH>(in + base, my, ltid);
        many_publish<T>(ctl, st, tid);   // the previous plane's stores are complete by now
        fft_lds_all<N, S, N, TH, RS, 1>(my, tw, ltid);
        const LdsAcc<1, RS> col{my};
        const PlaneColOut<N, true> dst{out + base};
        run_tail<N, S, N, TH, 0, false>(col, dst, tw, ltid);
        return grid;
    }
    many_publish<T>(ctl, st, tid);
    if (tid == 0) {
        unsigned n = 0;
        // one increment per plane item: N / PER items per grid
        while (__hip_atomic_load(&ctl->done[grid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < N / PER) {
            if (++n >= kSpinLimit) {
                atomicAdd(&ctl->timeouts, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    const long base = offset + (long)j * N;
    slab_body<N, S, TH, true>(out + base, out + base, (long)N * N, tw, my, ltid);
    return -1;
}

template <int S, int T>
__global__ void __launch_bounds__(T) k_many(ManyArgs a)
{
    extern __shared__ float2 lds[];
    __shared__ long item_sh;
    const int tid = threadIdx.x;
    ManyState st{-1};
    long next = 0, end = 0;
    for (;;) {
        if (next >= end) {
            if (tid == 0) item_sh = (long)atomicAdd(&a.ctl->head, (unsigned)a.chunk);
            __syncthreads();
            next = item_sh;
            end = next + a.chunk;
            __syncthreads();
        }
        if (next >= a.nitems) break;
        const unsigned it = a.items[next++];
        const int grid = (int)(it >> 8), slab = (int)((it >> 7) & 1), idx = (int)(it & 127);
        const ManyGrid gd = a.grids[grid];
        const float2* in;
        float2* out;
        group_ptrs(a, gd.group, in, out);
        switch (gd.n) {
#define FFT3D_MANY_CASE(m)                                                                                       \
    case m:                                                                                                      \
        st.pending = many_body<m, S, T>(in, out, a.tw + a.tw_off[m], a.ctl, gd.offset, grid, slab, idx, lds, tid, \
                                        st.pending);                                                            \
        break;
            FFT3D_FOR_EACH_MANY_SIZE(FFT3D_MANY_CASE)
#undef FFT3D_MANY_CASE
        default: break;
        }
        __syncthreads();   // LDS reuse
    }
    many_publish<T>(a.ctl, st, tid);
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&a.ctl->exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            for (int g = 0; g < a.ngrids; ++g) a.ctl->done[g] = 0;
            a.ctl->head = 0;
            __hip_atomic_store(&a.ctl->exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace fft3d
