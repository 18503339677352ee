// FP32 complex-to-complex kernels for gfx950, templated on transform length
// and exponent sign.  Layout of every grid: [batch][z][y][x], x contiguous,
// interleaved complex64.
//
//   k_cube<N,S>      one whole N^3 grid per workgroup, all three 1D passes in
//                    LDS (grids small enough to live on one compute unit).
//   k_plane<N,S>     pass A of the two-pass form: one xy-plane (Nx = Ny = N)
//                    per workgroup; x transform, LDS transpose by access
//                    pattern, y transform, store.
//   k_axis_str<N,S,L> one 1D pass along a strided axis (y or z): a workgroup
//                    owns L adjacent lines (consecutive x), reads and writes
//                    global memory directly with lanes along x.
//   k_axis_row<N,S,L> one 1D pass along x: L whole rows per workgroup,
//                    staged through LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace fft3d {

constexpr int odd_stride(int n) { return (n % 2 == 0) ? n + 1 : n; }

constexpr int round_up(int a, int m) { return (a + m - 1) / m * m; }

// Threads for a tile of `lines` transforms of length N: one butterfly of the
// largest radix per thread, clamped to [64, 1024].
template <int N>
constexpr int threads_for(int lines)
{
    int t = round_up(lines * N / Plan1D<N>::max_radix, 64);
    return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

// 2D LDS accessor: line -> (hi, lo) = (line / LDIV, line % LDIV);
// address = hi * LHI + lo * LLO + e * ES.
template <int LDIV, int LHI, int LLO, int ES>
struct LdsAcc2 {
    float2* p;
    __device__ __forceinline__ int addr(int line, int e) const
    {
        return (line / LDIV) * LHI + (line % LDIV) * LLO + e * ES;
    }
    __device__ __forceinline__ float2 load(int line, int e) const { return p[addr(line, e)]; }
    __device__ __forceinline__ void store(int line, int e, float2 v) const { p[addr(line, e)] = v; }
};

// Run stages [ST, stages) of the length-N schedule from LDS accessor `a` in
// place, the last stage writing to `last` instead.  LAST_SYNC: `last`
// aliases `a`, so the last stage also needs a barrier between its reads and
// its writes.
template <int N, int S, int L, int T, int ST, bool LAST_SYNC, class A, class D>
__device__ __forceinline__ void run_tail(const A& a, const D& last, const float2* __restrict__ tw, int tid,
                                         int valid = L)
{
    using P = Plan1D<N>;
    if constexpr (ST < P::stages) {
        if constexpr (ST == P::stages - 1) {
            fft_stage<N, ST, S, L, T, true, LAST_SYNC>(a, last, tw, tid, valid);
        } else {
            fft_stage<N, ST, S, L, T, true, true>(a, a, tw, tid, valid);
            __syncthreads();
            run_tail<N, S, L, T, ST + 1, LAST_SYNC>(a, last, tw, tid, valid);
        }
    }
}

// ------------------------------------------------------------------ cube --

template <int N>
struct CubeGeom {
    static constexpr int YS = odd_stride(N);
    static constexpr int ZS = N * YS;
    static constexpr int WORDS = N * ZS;
    static constexpr int T = threads_for<N>(N * N);
};

template <int N, int S>
__global__ void __launch_bounds__(CubeGeom<N>::T)
k_cube(const float2* in, float2* out, const float2* __restrict__ tw)
{
    using G = CubeGeom<N>;
    constexpr int T = G::T;
    constexpr int V = N * N * N;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * V;
    for (int i = tid; i < V; i += T) {
        const int x = i % N, y = (i / N) % N, z = i / (N * N);
        lds[z * G::ZS + y * G::YS + x] = in[base + i];
    }
    __syncthreads();
    // x: lines (z, y), contiguous elements
    fft_lds_all<N, S, N * N, T, G::YS, 1>(lds, tw, tid);
    // y: lines (z, x), element stride YS
    {
        const LdsAcc2<N, G::ZS, 1, G::YS> a{lds};
        run_tail<N, S, N * N, T, 0, true>(a, a, tw, tid);
        __syncthreads();
    }
    // z: lines (y, x), element stride ZS
    {
        const LdsAcc2<N, G::YS, 1, G::ZS> a{lds};
        run_tail<N, S, N * N, T, 0, true>(a, a, tw, tid);
        __syncthreads();
    }
    for (int i = tid; i < V; i += T) {
        const int x = i % N, y = (i / N) % N, z = i / (N * N);
        out[base + i] = lds[z * G::ZS + y * G::YS + x];
    }
}

// ----------------------------------------------------------------- plane --

template <int N>
struct PlaneGeom {
    static constexpr int RS = odd_stride(N);
    static constexpr int WORDS = N * RS;
    static constexpr int T = threads_for<N>(N);
};

// Global accessor for the y pass's final store: line = x, element = y.
template <int N>
struct PlaneColOut {
    float2* p;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const { p[y * N + x] = v; }
};

template <int N, int S>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_plane(const float2* in, float2* out, const float2* __restrict__ tw)
{
    using G = PlaneGeom<N>;
    constexpr int T = G::T;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * N * N;
    for (int i = tid; i < N * N; i += T) lds[(i / N) * G::RS + (i % N)] = in[base + i];
    __syncthreads();
    // x transform: lines = y
    fft_lds_all<N, S, N, T, G::RS, 1>(lds, tw, tid);
    // y transform: lines = x; last stage straight to global
    const LdsAcc<1, G::RS> col{lds};
    const PlaneColOut<N> dst{out + base};
    run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
}

// ---------------------------------------------------------- strided axis --

// Lines are enumerated (o, x), x fastest; line li has global base
//   (o / odiv) * shi + (o % odiv) * slo + x,  o = li / nx, x = li % nx,
// and its elements are es apart.
struct AxisMap {
    long lines;
    int nx;
    int odiv;
    long shi, slo, es;
};

template <int N, int L>
struct AxisGeom {
    static constexpr int LP = odd_stride(L);
    static constexpr int WORDS = N * LP;
    static constexpr int T = threads_for<N>(L);
    static_assert(T % L == 0 || L % T == 0, "tile lines and threads must nest");
};

template <int N, int S, int L>
__global__ void __launch_bounds__((AxisGeom<N, L>::T))
k_axis_str(const float2* in, float2* out, const float2* __restrict__ tw, AxisMap m)
{
    using G = AxisGeom<N, L>;
    using P = Plan1D<N>;
    constexpr int T = G::T;
    static_assert(T % L == 0, "each thread keeps one line");
    __shared__ float2 lds[P::stages > 1 ? G::WORDS : 1];
    const int tid = threadIdx.x;
    const long l0 = (long)blockIdx.x * L;
    const int myline = tid % L;
    const long li = l0 + myline;
    const int valid = (int)((m.lines - l0) < L ? (m.lines - l0) : L);
    long gbase = 0;
    if (li < m.lines) {
        const long o = li / m.nx;
        const long x = li - o * m.nx;
        gbase = (o / m.odiv) * m.shi + (o % m.odiv) * m.slo + x;
    }
    const GlobStrided g{in + gbase, out + gbase, m.es};
    if constexpr (P::stages == 1) {
        fft_stage<N, 0, S, L, T, true, false>(g, g, tw, tid, valid);
    } else {
        const LdsAcc<1, G::LP> a{lds};
        fft_stage<N, 0, S, L, T, true, false>(g, a, tw, tid, valid);
        __syncthreads();
        run_tail<N, S, L, T, 1, false>(a, g, tw, tid, valid);
    }
}

// --------------------------------------------------------------- x rows --

template <int N, int L>
struct RowGeom {
    static constexpr int RS = odd_stride(N);
    static constexpr int WORDS = L * RS;
    static constexpr int T = threads_for<N>(L);
};

template <int N, int S, int L>
__global__ void __launch_bounds__((RowGeom<N, L>::T))
k_axis_row(const float2* in, float2* out, const float2* __restrict__ tw, long rows)
{
    using G = RowGeom<N, L>;
    constexpr int T = G::T;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    const long r0 = (long)blockIdx.x * L;
    const int valid = (int)((rows - r0) < L ? (rows - r0) : L);
    const long base = r0 * N;
    for (int i = tid; i < valid * N; i += T) lds[(i / N) * G::RS + (i % N)] = in[base + i];
    __syncthreads();
    fft_lds_all<N, S, L, T, G::RS, 1>(lds, tw, tid, valid);
    for (int i = tid; i < valid * N; i += T) out[base + i] = lds[(i / N) * G::RS + (i % N)];
}

}  // namespace fft3d
