// Workgroup-level engine for batches of 1D Stockham transforms.
//
// A workgroup holds a tile of L "lines" (independent 1D transforms of length
// N).  Every stage of the radix schedule (sched.hpp) is one call of
// fft_stage: each thread takes butterflies b = tid, tid + T, ...; reads its R
// inputs through a source accessor, applies twiddles and the R-point DFT, and
// writes its R outputs through a destination accessor.  Accessors map
// (line, element) to an address, so the same stage code runs from global
// memory into LDS, LDS to LDS, or LDS to global memory with any layout.
//
// Mapping of butterfly index b to (line, j):
//   LINE_FAST: line = b mod L, j = b / L -- consecutive lanes take
//              consecutive lines; used wherever consecutive lines are
//              adjacent in memory (coalesced global access, conflict-free LDS
//              with an odd line stride).  When L is a multiple of 64 every
//              lane of a wave has the same j, so the twiddle index is
//              wave-uniform and twiddles come through scalar loads.
//   J_FAST:    j = b mod (N/R), line = b / (N/R).
#pragma once
#include <hip/hip_runtime.h>

#include "codelets.hpp"
#include "sched.hpp"

namespace fft3d {

// KIND 0: default schedule; KIND 1: radix-16 first (make_sched16).
template <int N, int KIND = 0>
struct Plan1D {
    static constexpr int n = N;
    static constexpr Sched sc = make_sched_kind(N, KIND);
    static constexpr int stages = sc.count;
    static constexpr int radix(int s) { return sc.r[s]; }
    static constexpr int ns(int s) { return sched_ns(sc, s); }
    static constexpr int tw_off(int s) { return sched_tw_off(sc, s); }
    static constexpr int tw_len = sched_tw_len(sc);
    static constexpr int max_radix = sched_max_radix(sc);
    static constexpr int min_radix = sched_min_radix(sc);
};

// ---------------------------------------------------------------- accessors --

// LDS tile: address = line * LS + e * ES (float2 units).
template <int LS, int ES>
struct LdsAcc {
    float2* p;
    __device__ __forceinline__ float2 load(int line, int e) const { return p[line * LS + e * ES]; }
    __device__ __forceinline__ void store(int line, int e, float2 v) const { p[line * LS + e * ES] = v; }
};

// Global memory, line base offsets given per line by a functor-free form:
// address = base + line * LS + e * ES (element units).
template <long LS, long ES>
struct GlobAcc {
    const float2* src;
    float2* dst;
    __device__ __forceinline__ float2 load(int line, int e) const { return src[(long)line * LS + (long)e * ES]; }
    __device__ __forceinline__ void store(int line, int e, float2 v) const { dst[(long)line * LS + (long)e * ES] = v; }
};

// Streaming (non-temporal) 8-byte global load: the data bypass the
// retention policy of the caches.  Used only where measured to pay; see
// stream_plane.
__device__ __forceinline__ float2 ld_stream(const float2* p)
{
    const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
    return __builtin_bit_cast(float2, u);
}

// Whether the xy-plane passes of length n stream their plane loads.  They
// read each input plane once, and streaming those loads keeps the input out
// of the Infinity Cache, which then still holds the plane pass's own output
// (default-policy stores) when the z pass reads it, last-written first
// (rev_tile).  Measured on whole inverse+forward steps over ~512 MB
// batches: 2-7% faster at every length from 32 to 120 except 90 (no
// change); 128 and 125 gain on the pass itself as well.  An earlier sweep
// that timed the plane pass alone, with its stores streamed too, had found
// lengths 72-120 slower: it could not see the effect on the z pass.
constexpr bool stream_plane(int n) { return n >= 16; }
// Streaming loads pay on batches that do not stay in the caches between
// passes; below this many bytes per pass (a single 128^3 grid is 16 MB) the
// default policy is faster.
constexpr long kStreamMinBytes = 32L << 20;
// The streamed plane passes with paired 16-byte stores (N = 64, 128) store
// the output of their first planes with the streaming policy too, all but
// the last kPlaneCachedTail bytes: the planes written first leave the
// Infinity Cache (256 MB) before the z pass, which reads the last-written
// first, reaches them, and caching them only displaces the tail it does
// find there.
constexpr long kPlaneCachedTail = 320L << 20;

__host__ __device__ constexpr long streamed_store_planes(long planes, long plane_bytes)
{
    return planes > kPlaneCachedTail / plane_bytes ? planes - kPlaneCachedTail / plane_bytes : 0;
}

// Global memory with a runtime element stride and a per-thread line base
// (the line index passed in is ignored; the caller has folded it into base).
struct GlobStrided {
    const float2* src;
    float2* dst;
    long es;
    __device__ __forceinline__ float2 load(int, int e) const { return src[(long)e * es]; }
    __device__ __forceinline__ void store(int, int e, float2 v) const { dst[(long)e * es] = v; }
};

// Device-coherent 8-byte global accesses: the load misses every cache that
// is not coherent across the device's L2 slices and the store writes through
// them (agent-scope relaxed atomics, i.e. sc1 accesses on gfx950).  Used for
// data handed from one workgroup to another inside one kernel launch.
__device__ __forceinline__ float2 load_coherent(const float2* p)
{
    const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, b);
}
__device__ __forceinline__ void store_coherent(float2* p, float2 v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 8-byte global load that misses the compute unit's L1 cache and is served
// by the L2 of the XCD the workgroup runs on (sc0 on gfx950): it sees every
// store that another compute unit of the same XCD has completed into that
// L2 (the XCD's L2 is shared by its 32 compute units; only the L1 caches
// are private).
__device__ __forceinline__ float2 load_xcd_coherent(const float2* p)
{
    const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_bit_cast(float2, b);
}

// Global memory, lines adjacent (line stride 1), runtime element stride.
// COH_LOAD: 0 plain loads, 1 device-coherent loads (load_coherent), 2 loads
// coherent within the XCD (load_xcd_coherent).
template <int COH_LOAD = 0>
struct GlobLines {
    const float2* src;
    float2* dst;
    long es;
    __device__ __forceinline__ float2 load(int line, int e) const
    {
        const float2* p = src + line + (long)e * es;
        if constexpr (COH_LOAD == 1) return load_coherent(p);
        else if constexpr (COH_LOAD == 2) return load_xcd_coherent(p);
        else return *p;
    }
    __device__ __forceinline__ void store(int line, int e, float2 v) const { dst[line + (long)e * es] = v; }
};

// ------------------------------------------------------------------- stage --

// One Stockham stage of the length-N schedule (stage index ST) over L lines
// with T threads.  `valid(line)` masks lines beyond a ragged tile end.
// SYNC: barrier between the read phase and the write phase (needed when
// source and destination alias in LDS).
template <class P, int ST, int S, int L, int T, bool LINE_FAST, bool SYNC, class Src, class Dst>
__device__ __forceinline__ void fft_stage_p(const Src& src, const Dst& dst, const float2* __restrict__ tw,
                                          int tid, int valid_lines = L)
{
    constexpr int N = P::n;
    constexpr int R = P::radix(ST);
    constexpr int NS = P::ns(ST);
    constexpr int M = N / R;
    constexpr int NB = L * M;
    constexpr int IT = (NB + T - 1) / T;
    constexpr bool UNIFORM = LINE_FAST && (L % 64 == 0) && (T % 64 == 0);
    const float2* __restrict__ tws = tw + P::tw_off(ST);

    float2 v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * T;
        const int line = LINE_FAST ? b % L : b / M;
        int j = LINE_FAST ? b / L : b % M;
        if (UNIFORM) j = __builtin_amdgcn_readfirstlane(j);
        if ((NB % T == 0 || b < NB) && line < valid_lines) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[it][q] = src.load(line, j + q * M);
            if constexpr (NS > 1) {
                const float2* __restrict__ w = tws + (j % NS) * (R - 1);
#pragma unroll
                for (int q = 1; q < R; ++q) v[it][q] = cmul(v[it][q], w[q - 1]);
            }
            dft<R, S>(v[it]);
        }
    }
    if constexpr (SYNC) __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * T;
        const int line = LINE_FAST ? b % L : b / M;
        const int j = LINE_FAST ? b / L : b % M;
        if ((NB % T == 0 || b < NB) && line < valid_lines) {
            const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
            for (int q = 0; q < R; ++q) dst.store(line, base + q * NS, v[it][q]);
        }
    }
}

// K: schedule kind of the length-N transform (Plan1D).
template <int N, int ST, int S, int L, int T, bool LINE_FAST, bool SYNC, int K = 0, class Src, class Dst>
__device__ __forceinline__ void fft_stage(const Src& src, const Dst& dst, const float2* __restrict__ tw, int tid,
                                          int valid_lines = L)
{
    fft_stage_p<Plan1D<N, K>, ST, S, L, T, LINE_FAST, SYNC>(src, dst, tw, tid, valid_lines);
}

// All stages of a length-N transform on an LDS tile, in place.
// The tile is left in natural order; ends with a barrier.  Every stage but
// the last needs a barrier between its reads and its writes; in the last
// stage each thread writes exactly the positions it read (j + q N/R), so it
// needs none.
template <int N, int S, int L, int T, int LS, int ES, int KIND = 0>
__device__ __forceinline__ void fft_lds_all(float2* lds, const float2* __restrict__ tw, int tid,
                                            int valid_lines = L)
{
    using P = Plan1D<N, KIND>;
    constexpr int K = P::stages;
    constexpr int D = KIND;
    const LdsAcc<LS, ES> a{lds};
    if constexpr (K > 0) { fft_stage<N, 0, S, L, T, true, (K > 1), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 1) { fft_stage<N, 1, S, L, T, true, (K > 2), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 2) { fft_stage<N, 2, S, L, T, true, (K > 3), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 3) { fft_stage<N, 3, S, L, T, true, (K > 4), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 4) { fft_stage<N, 4, S, L, T, true, (K > 5), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 5) { fft_stage<N, 5, S, L, T, true, (K > 6), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 6) { fft_stage<N, 6, S, L, T, true, (K > 7), D>(a, a, tw, tid, valid_lines); __syncthreads(); }
    if constexpr (K > 7) { fft_stage<N, 7, S, L, T, true, false, D>(a, a, tw, tid, valid_lines); __syncthreads(); }
}

}  // namespace fft3d
