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

#include <type_traits>

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

template <int N, int KIND>
constexpr int threads_for_kind(int lines)
{
    int t = round_up(lines * N / Plan1D<N, KIND>::max_radix, 64);
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
// aliases `a` with another layout, so the last stage also needs a barrier
// between its reads and its writes.  With last == a it needs none: the last
// stage of a Stockham schedule writes exactly the positions it read.
// K: schedule kind (Plan1D).
template <int N, int S, int L, int T, int ST, bool LAST_SYNC, int K = 0, class A, class D>
__device__ __forceinline__ void run_tail(const A& a, const D& last, const float2* __restrict__ tw, int tid,
                                         int valid = L)
{
    using P = Plan1D<N, K>;
    if constexpr (ST < P::stages) {
        if constexpr (ST == P::stages - 1) {
            fft_stage<N, ST, S, L, T, true, LAST_SYNC, K>(a, last, tw, tid, valid);
        } else {
            fft_stage<N, ST, S, L, T, true, true, K>(a, a, tw, tid, valid);
            __syncthreads();
            run_tail<N, S, L, T, ST + 1, LAST_SYNC, K>(a, last, tw, tid, valid);
        }
    }
}

// Copy a contiguous run of ROWS * ROW complex values between global memory
// and an LDS tile with row stride RS, all loads issued before any LDS store
// (and all LDS reads before any global store).  Even-length rows move as
// 16-byte pairs.  `rows` <= ROWS masks a ragged tail.
template <int ROWS, int ROW, int RS, int T>
__device__ __forceinline__ void tile_to_lds(const float2* g, float2* lds, int tid, int rows = ROWS)
{
    if constexpr (ROW % 2 == 0) {
        constexpr int PAIRS = ROWS * ROW / 2, IT = (PAIRS + T - 1) / T;
        const float4* g4 = reinterpret_cast<const float4*>(g);
        float4 r[IT];
        const int lim = rows * ROW / 2;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) r[k] = g4[i];
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) {
                const int e = 2 * i, row = e / ROW, col = e % ROW;
                lds[row * RS + col] = make_float2(r[k].x, r[k].y);
                lds[row * RS + col + 1] = make_float2(r[k].z, r[k].w);
            }
        }
    } else {
        constexpr int E = ROWS * ROW, IT = (E + T - 1) / T;
        float2 r[IT];
        const int lim = rows * ROW;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) r[k] = g[i];
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) lds[(i / ROW) * RS + (i % ROW)] = r[k];
        }
    }
}

// The same copy split in two halves so the global loads of the next tile can
// be in flight while the current tile is being transformed.  NT: load()
// streams (ld_stream).
template <int ROWS, int ROW, int T, bool NT = false>
struct TileRegs {
    static constexpr bool PAIRS = ROW % 2 == 0;
    static constexpr int UNITS = PAIRS ? ROWS * ROW / 2 : ROWS * ROW;
    static constexpr int IT = (UNITS + T - 1) / T;
    using U = typename std::conditional<PAIRS, float4, float2>::type;
    U r[IT];

    __device__ __forceinline__ void load(const float2* g, int tid)
    {
        const U* gu = reinterpret_cast<const U*>(g);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                if constexpr (NT) {
                    if constexpr (PAIRS) {
                        typedef float f4v __attribute__((ext_vector_type(4)));
                        const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(gu + i));
                        r[k] = make_float4(t.x, t.y, t.z, t.w);
                    } else {
                        r[k] = ld_stream(reinterpret_cast<const float2*>(gu + i));
                    }
                } else {
                    r[k] = gu[i];
                }
            }
        }
    }
    // Load with a row predicate: rows for which row_ok(row) is false are not
    // read and hold zeros.
    template <class RowOk>
    __device__ __forceinline__ void load_rows(const float2* g, int tid, const RowOk& row_ok)
    {
        const U* gu = reinterpret_cast<const U*>(g);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                const int row = PAIRS ? (2 * i) / ROW : i / ROW;
                if (row_ok(row)) r[k] = gu[i];
                else r[k] = U{};
            }
        }
    }
    // Load the real factors f[e] matching this tile's elements (same unit
    // pattern: pairs of floats for even rows, single floats otherwise).
    template <class FR>
    __device__ __forceinline__ void load_factors(FR& fr, const float* f, int tid) const
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                if constexpr (PAIRS) fr.r[k] = reinterpret_cast<const float2*>(f)[i];
                else fr.r[k] = f[i];
            }
        }
    }
    template <int RS, class FR>
    __device__ __forceinline__ void store_lds_scaled(float2* lds, int tid, const FR& fr, float s) const
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                if constexpr (PAIRS) {
                    const int e = 2 * i, row = e / ROW, col = e % ROW;
                    const float a = s * fr.r[k].x, b = s * fr.r[k].y;
                    lds[row * RS + col] = make_float2(a * r[k].x, a * r[k].y);
                    lds[row * RS + col + 1] = make_float2(b * r[k].z, b * r[k].w);
                } else {
                    const float a = s * fr.r[k];
                    lds[(i / ROW) * RS + (i % ROW)] = make_float2(a * r[k].x, a * r[k].y);
                }
            }
        }
    }
    template <int RS>
    __device__ __forceinline__ void store_lds(float2* lds, int tid) const
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                if constexpr (PAIRS) {
                    const int e = 2 * i, row = e / ROW, col = e % ROW;
                    lds[row * RS + col] = make_float2(r[k].x, r[k].y);
                    lds[row * RS + col + 1] = make_float2(r[k].z, r[k].w);
                } else {
                    lds[(i / ROW) * RS + (i % ROW)] = r[k];
                }
            }
        }
    }
};

// Register copy of the real factors of one tile (see TileRegs::load_factors).
template <int ROWS, int ROW, int T>
struct FactorRegs {
    using TR = TileRegs<ROWS, ROW, T>;
    using U = typename std::conditional<TR::PAIRS, float2, float>::type;
    U r[TR::IT];
};

template <int ROWS, int ROW, int RS, int T>
__device__ __forceinline__ void lds_to_tile(const float2* lds, float2* g, int tid, int rows = ROWS)
{
    if constexpr (ROW % 2 == 0) {
        constexpr int PAIRS = ROWS * ROW / 2, IT = (PAIRS + T - 1) / T;
        float4* g4 = reinterpret_cast<float4*>(g);
        float4 r[IT];
        const int lim = rows * ROW / 2;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) {
                const int e = 2 * i, row = e / ROW, col = e % ROW;
                const float2 a = lds[row * RS + col], b = lds[row * RS + col + 1];
                r[k] = make_float4(a.x, a.y, b.x, b.y);
            }
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) g4[i] = r[k];
        }
    } else {
        constexpr int E = ROWS * ROW, IT = (E + T - 1) / T;
        float2 r[IT];
        const int lim = rows * ROW;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) r[k] = lds[(i / ROW) * RS + (i % ROW)];
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (i < lim) g[i] = r[k];
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
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    const long base = (long)blockIdx.x * (N * N * N);
    tile_to_lds<N * N, N, G::YS, T>(in + base, lds, tid);
    __syncthreads();
    // x: lines (z, y), contiguous elements
    fft_lds_all<N, S, N * N, T, G::YS, 1>(lds, tw, tid);
    // y: lines (z, x), element stride YS
    {
        const LdsAcc2<N, G::ZS, 1, G::YS> a{lds};
        run_tail<N, S, N * N, T, 0, false>(a, a, tw, tid);
        __syncthreads();
    }
    // z: lines (y, x), element stride ZS
    {
        const LdsAcc2<N, G::YS, 1, G::ZS> a{lds};
        run_tail<N, S, N * N, T, 0, false>(a, a, tw, tid);
        __syncthreads();
    }
    lds_to_tile<N * N, N, G::YS, T>(lds, out + base, tid);
}

// ----------------------------------------------------------------- plane --

template <int N>
struct PlaneGeom {
    static constexpr int RS = odd_stride(N);
    static constexpr int WORDS = N * RS;
    static constexpr int T = threads_for<N>(N);
};

// Global accessor for the y pass's final store: line = x, element = y.
// COH: device-coherent (write-through) stores.
template <int N, bool COH = false>
struct PlaneColOut {
    float2* p;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const
    {
        if constexpr (COH) store_coherent(p + y * N + x, v);
        else p[y * N + x] = v;
    }
};

// One xy-plane: `in` and `out` point at the plane's first element.
// COH: the plane's output is stored device-coherently.
template <int N, int S, int T, bool COH = false>
__device__ __forceinline__ void plane_body(const float2* in, float2* out, const float2* __restrict__ tw,
                                           float2* lds, int tid)
{
    constexpr int RS = PlaneGeom<N>::RS;
    tile_to_lds<N, N, RS, T>(in, lds, tid);
    __syncthreads();
    // x transform: lines = y
    fft_lds_all<N, S, N, T, RS, 1>(lds, tw, tid);
    // y transform: lines = x; last stage straight to global
    const LdsAcc<1, RS> col{lds};
    const PlaneColOut<N, COH> dst{out};
    run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
}

template <int N, int S>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_plane(const float2* in, float2* out, const float2* __restrict__ tw)
{
    __shared__ float2 lds[PlaneGeom<N>::WORDS];
    const long base = (long)blockIdx.x * N * N;
    plane_body<N, S, PlaneGeom<N>::T>(in + base, out + base, tw, lds, threadIdx.x);
}

// Last stage of a length-N transform over L lines held in LDS (line x,
// element e at src.load(x, e)), with the lines adjacent in global memory:
// output element r of line x goes to out[x + r * es], stored as 16-byte
// pairs of adjacent lines.  The 64 lanes of a wave take the wave's 64
// lines in the order 0, 2, 4, ... (lanes 0-31) then 1, 3, 5, ... (lanes
// 32-63); after the butterfly one v_permlane32_swap per value component
// gives lane l < 32 the outputs of lines x, x + 1 for the upper half of the
// butterfly's output elements and lane l + 32 the same two lines for the
// lower half, each stored as one 16-byte write: half the store
// instructions of one 8-byte value per lane, every wave store still whole
// runs of adjacent lines.  The LDS reads cover the same 64 consecutive lines
// per wave as the plain stage, conflict-free.
template <int N, int L, int K>
constexpr bool pairs_ok(int T)
{
    using P = Plan1D<N, K>;
    return L % 64 == 0 && P::radix(P::stages - 1) % 2 == 0 && (L * (N / P::radix(P::stages - 1))) % T == 0 &&
           T % 64 == 0;
}

template <int N, int S, int L, int T, int K, bool NTS = false, class A>
__device__ __forceinline__ void last_stage_pairs(const A& src, float2* out, long es, const float2* __restrict__ tw,
                                                 int tid)
{
    using P = Plan1D<N, K>;
    constexpr int ST = P::stages - 1, R = P::radix(ST), NS = P::ns(ST), M = N / R, NB = L * M, IT = NB / T;
    static_assert(pairs_ok<N, L, K>(T), "64-line waves, an even last radix, whole iterations");
    const float2* __restrict__ tws = tw + P::tw_off(ST);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * T, lane = b & 63, b0 = b - lane;
        const int j = __builtin_amdgcn_readfirstlane(b0 / L);
        const int xe = b0 % L + 2 * (lane & 31), x = xe + (lane >> 5);
        float2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = src.load(x, j + q * M);
        if constexpr (NS > 1) {
            const float2* __restrict__ w = tws + (j % NS) * (R - 1);
#pragma unroll
            for (int q = 1; q < R; ++q) v[q] = cmul(v[q], w[q - 1]);
        }
        dft<R, S>(v);
        const int base = (j / NS) * NS * R + (j % NS);
        const bool lower = lane >= 32;
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            // new v[k + R/2] register: lanes 0-31 keep line xe, lanes 32-63 receive
            // line xe of v[k]; new v[k] register: line xe + 1 of the same elements
            const auto re = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v[k + R / 2].x),
                                                             __builtin_bit_cast(unsigned, v[k].x), false, false);
            const auto im = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v[k + R / 2].y),
                                                             __builtin_bit_cast(unsigned, v[k].y), false, false);
            const long r = base + (lower ? k : k + R / 2) * NS;
            typedef float f4v __attribute__((ext_vector_type(4)));
            const f4v val = {__builtin_bit_cast(float, (unsigned)re[0]), __builtin_bit_cast(float, (unsigned)im[0]),
                             __builtin_bit_cast(float, (unsigned)re[1]), __builtin_bit_cast(float, (unsigned)im[1])};
            f4v* dst = reinterpret_cast<f4v*>(out + xe + r * es);
            if constexpr (NTS) __builtin_nontemporal_store(val, dst);   // streaming store
            else *dst = val;
        }
    }
}

// All stages but the last of a length-N transform over L lines in LDS (in
// place, each followed by a barrier), then the last one stored as pairs.
template <int N, int S, int L, int T, int K, int FIRST, bool NTS = false, class A>
__device__ __forceinline__ void tail_pairs(const A& a, float2* out, long es, const float2* __restrict__ tw, int tid)
{
    constexpr int ST = Plan1D<N, K>::stages - 1;
    static_assert(ST - FIRST <= 3, "at most three stages before the last");
    if constexpr (FIRST < ST) { fft_stage<N, FIRST, S, L, T, true, true, K>(a, a, tw, tid); __syncthreads(); }
    if constexpr (FIRST + 1 < ST) { fft_stage<N, FIRST + 1, S, L, T, true, true, K>(a, a, tw, tid); __syncthreads(); }
    if constexpr (FIRST + 2 < ST) { fft_stage<N, FIRST + 2, S, L, T, true, true, K>(a, a, tw, tid); __syncthreads(); }
    last_stage_pairs<N, S, L, T, K, NTS>(a, out, es, tw, tid);
}

// Persistent form of the plane pass: workgroup w transforms planes
// w, w + G, w + 2G, ... and loads plane p + G into registers while plane p is
// being transformed, so HBM latency overlaps the LDS/VALU phases.
//
// SCALE: every input value at grid position r is first multiplied by the real
// factor 2 * gE[0] * V[r] (V: one [nz][N][N] grid shared by the batch) -- the
// prologue of the energy gradient.
// NT: streaming plane loads (see stream_plane); planes below nt_planes
// (streamed_store_planes) also stream their stores, the rest keep the
// default policy so that the z pass after it finds the last part of the
// output in the caches.
// K: schedule kind of both 1D transforms (0 default, 2 the tuner's
// alternative order; the twiddle table must be of the same kind).
template <int N, int S, bool SCALE = false, bool NT = false, int K = 0>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_plane_pf(const float2* in, float2* out, const float2* __restrict__ tw, long planes, const float* __restrict__ V,
           const double* __restrict__ gE, int nz, long nt_planes)
{
    constexpr int T = PlaneGeom<N>::T, RS = PlaneGeom<N>::RS;
    __shared__ float2 lds[PlaneGeom<N>::WORDS];
    const int tid = threadIdx.x;
    // N not a multiple of 64: a wave's butterflies of one stage span two
    // twiddle groups, so the stages read their twiddles per lane; those reads
    // go to an LDS copy of the table instead of global memory
    constexpr bool TWL = N % 64 != 0;
    constexpr int TWN = Plan1D<N, K>::tw_len;
    __shared__ float2 tw_lds[TWL && TWN > 0 ? TWN : 1];
    if constexpr (TWL && TWN > 0) {
        for (int i = tid; i < TWN; i += T) tw_lds[i] = tw[i];   // visible after the first barrier below
        tw = tw_lds;
    }
    TileRegs<N, N, T, NT> regs;
    FactorRegs<N, N, T> vr;
    float scale = 0.f;
    if constexpr (SCALE) scale = (float)(2.0 * gE[0]);
    long p = blockIdx.x;
    if (p < planes) {
        regs.load(in + p * N * N, tid);
        if constexpr (SCALE) regs.load_factors(vr, V + (p % nz) * N * N, tid);
    }
    for (; p < planes; p += gridDim.x) {
        if constexpr (SCALE) regs.template store_lds_scaled<RS>(lds, tid, vr, scale);
        else regs.template store_lds<RS>(lds, tid);
        __syncthreads();
        const long pn = p + gridDim.x;
        if (pn < planes) {
            regs.load(in + pn * N * N, tid);
            if constexpr (SCALE) regs.load_factors(vr, V + (pn % nz) * N * N, tid);
        }
        fft_lds_all<N, S, N, T, RS, 1, K>(lds, tw, tid);
        if constexpr (pairs_ok<N, N, K>(T)) {   // y transform: lines = x, rows y N apart
            if (NT && p < nt_planes)   // uniform: the store policy is chosen per plane
                tail_pairs<N, S, N, T, K, 0, NT>(LdsAcc<1, RS>{lds}, out + p * N * N, (long)N, tw, tid);
            else
                tail_pairs<N, S, N, T, K, 0>(LdsAcc<1, RS>{lds}, out + p * N * N, (long)N, tw, tid);
        } else {
            const LdsAcc<1, RS> col{lds};
            const PlaneColOut<N> dst{out + p * N * N};
            run_tail<N, S, N, T, 0, false, K>(col, dst, tw, tid);
        }
        __syncthreads();
    }
}

// Signed frequency of index k on a length-n axis (k for k < n/2, k - n above).
__host__ __device__ __forceinline__ int signed_freq(int k, int n) { return 2 * k < n ? k : k - n; }

// Packed sphere: the points of a grid inside the sphere, in the grid's own
// order ([kz][ky][kx] ascending), grid after grid.  Row (kz, ky) of a grid
// holds cnt of them at packed offset off: kx = 0 .. npos-1, then
// kx = n - (cnt - npos) .. n - 1 (the non-negative, then the negative
// frequencies).  The table has one entry per (kz, ky).
struct SphereRow {
    int off, cnt, npos, pad;
};

__host__ __device__ __forceinline__ bool sphere_has(const SphereRow& r, int x, int n)
{
    return x < r.npos || x >= n - (r.cnt - r.npos);
}

// Packed index (within the grid) of point kx = x of row r; x must be inside.
__host__ __device__ __forceinline__ int sphere_rank(const SphereRow& r, int x, int n)
{
    return r.off + (x < r.npos ? x : x - (n - r.cnt));
}

// One N x N plane gathered from a packed sphere into registers (zeros at the
// points outside it), in the element order of a plane tile.
template <int N, int T>
struct PackedRegs {
    static constexpr int E = N * N;
    static constexpr int IT = (E + T - 1) / T;
    float2 r[IT];

    __device__ __forceinline__ void load(const float2* packed, const SphereRow* rows, int tid)
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (E % T == 0 || i < E) {
                const int y = i / N, x = i % N;
                const SphereRow rw = rows[y];
                r[k] = sphere_has(rw, x, N) ? packed[sphere_rank(rw, x, N)] : make_float2(0.f, 0.f);
            }
        }
    }
    template <int RS>
    __device__ __forceinline__ void store_lds(float2* lds, int tid) const
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (E % T == 0 || i < E) lds[(i / N) * RS + (i % N)] = r[k];
        }
    }
};

// Plane output that stores only the points with Gx^2 + Gy^2 < R2.
template <int N>
struct PlaneColOutDisk {
    float2* p;
    double R2;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const
    {
        const int gx = signed_freq(x, N), gy = signed_freq(y, N);
        if ((double)(gx * gx + gy * gy) < R2) p[y * N + x] = v;
    }
};

// Plane output of plane kz (gz2 = Gz^2) storing only the points inside the
// sphere Gx^2 + Gy^2 + gz2 < R2.
template <int N>
struct PlaneColOutBall {
    float2* p;
    int gz2;
    double R2;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const
    {
        const int gx = signed_freq(x, N), gy = signed_freq(y, N);
        if ((double)(gx * gx + gy * gy + gz2) < R2) p[y * N + x] = v;
    }
};

// The xy-plane pass of a pruned transform with the sphere |G|^2 < R2
// (G = signed frequencies) on grids [batch][nz][N][N].
//   OUT = false (inverse, input vanishing outside the sphere): only the
//     planes kz of zlist (those with Gz^2 < R2, nzp of them; `planes` =
//     batch * nzp) are transformed, and in each only the rows with
//     Gy^2 + Gz^2 < R2 are read, the other rows being zeros.  Whole planes
//     are written; the other planes are neither read nor written.
//   KIND 1 (forward, output wanted inside the sphere only): every plane
//     (`planes` = batch * nz, zlist unused) is read whole and transformed;
//     only the points with Gx^2 + Gy^2 < R2, the z-lines the sphere meets,
//     are written.
//   KIND 2 (last pass of a forward whose z pass came first, output wanted
//     inside the sphere only): only the planes of zlist are read (whole) and
//     transformed, and only their points inside the sphere are written.
//   KIND 0 is the inverse (first form above).
//   PACKED (with KIND 0): `in` is a packed sphere of `npts` points per grid
//     with row table `rows` ([kz][ky]); the rows are gathered from it.
template <int N, int S, int KIND, bool PACKED = false>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_plane_pruned(const float2* in, float2* out, const float2* __restrict__ tw, long planes, const int* __restrict__ zlist,
               int nzp, int nz, double R2, const SphereRow* __restrict__ rows = nullptr, long npts = 0)
{
    constexpr bool OUT = KIND == 1;
    static_assert(KIND == 0 || !PACKED, "the packed form of the plane pass is the inverse's");
    constexpr int T = PlaneGeom<N>::T, RS = PlaneGeom<N>::RS;
    __shared__ float2 lds[PlaneGeom<N>::WORDS];
    const int tid = threadIdx.x;
    typename std::conditional<PACKED, PackedRegs<N, T>, TileRegs<N, N, T, stream_plane(N)>>::type regs;
    auto plane_base = [&](long i) {
        if constexpr (OUT) return i * N * N;
        const long b = i / nzp;
        return (b * nz + zlist[i % nzp]) * (long)N * N;
    };
    auto load = [&](long i) {
        if constexpr (PACKED) {
            const long g = i / nzp;
            regs.load(in + g * npts, rows + (long)zlist[i % nzp] * N, tid);
        } else if constexpr (KIND != 0) {
            regs.load(in + plane_base(i), tid);
        } else {
            const int gz = signed_freq(zlist[i % nzp], nz), gz2 = gz * gz;
            regs.load_rows(in + plane_base(i), tid, [gz2, R2](int y) {
                const int gy = signed_freq(y, N);
                return (double)(gy * gy + gz2) < R2;
            });
        }
    };
    long p = blockIdx.x;
    if (p < planes) load(p);
    for (; p < planes; p += gridDim.x) {
        regs.template store_lds<RS>(lds, tid);
        __syncthreads();
        const long pn = p + gridDim.x;
        if (pn < planes) load(pn);
        fft_lds_all<N, S, N, T, RS, 1>(lds, tw, tid);
        const LdsAcc<1, RS> col{lds};
        if constexpr (KIND == 1) {
            const PlaneColOutDisk<N> dst{out + plane_base(p), R2};
            run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
        } else if constexpr (KIND == 2) {
            const int gz = signed_freq(zlist[p % nzp], nz);
            const PlaneColOutBall<N> dst{out + plane_base(p), gz * gz, R2};
            run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
        } else {
            const PlaneColOut<N> dst{out + plane_base(p)};
            run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
        }
        __syncthreads();
    }
}

// Dense grids [batch][nz][ny][nx] <-> packed spheres [batch][npts]
// (PACK: gather the points inside the sphere; otherwise scatter them and
// write zeros everywhere else).  nyz = nz * ny rows per grid.
template <bool PACK>
__global__ void __launch_bounds__(256)
k_sphere_copy(const float2* __restrict__ src, float2* __restrict__ dst, const SphereRow* __restrict__ rows, long npts,
              int nx, long nyz, long total)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const long row = i / nx;
        const int x = (int)(i - row * nx);
        const long b = row / nyz;
        const SphereRow r = rows[row - b * nyz];
        const bool in = sphere_has(r, x, nx);
        const long p = b * npts + (in ? sphere_rank(r, x, nx) : 0);
        if constexpr (PACK) {
            if (in) dst[p] = src[i];
        } else {
            dst[i] = in ? src[p] : make_float2(0.f, 0.f);
        }
    }
}

// One xz-slab for fixed (b, y): N lines (all x) of N points along z, element
// z of line x at base[z * es + x].  Loads and stores run with lanes along x.
// COH: how the slab's input is loaded (GlobLines: 0 plain, 1 device-coherent,
// 2 coherent within the XCD).
template <int N, int S, int T, int COH = 0>
__device__ __forceinline__ void slab_body(const float2* in, float2* out, long es, const float2* __restrict__ tw,
                                          float2* lds, int tid)
{
    constexpr int LP = PlaneGeom<N>::RS;
    using P = Plan1D<N>;
    const GlobLines<COH> g{in, out, es};
    if constexpr (P::stages == 1) {
        fft_stage<N, 0, S, N, T, true, false>(g, g, tw, tid);
    } else {
        const LdsAcc<1, LP> a{lds};
        fft_stage<N, 0, S, N, T, true, false>(g, a, tw, tid);
        __syncthreads();
        run_tail<N, S, N, T, 1, false>(a, g, tw, tid);
    }
}

// ------------------------------------------------------------ fused pass --

// Control block of the persistent kernel (device memory owned by the plan,
// zero between executions: the last workgroup to leave resets it).
struct FusedCtl {
    unsigned head;     // next work item
    unsigned exited;   // workgroups that have left the item loop
    unsigned timeouts; // bounded waits that expired (0 in correct operation)
    unsigned pad;
    unsigned done[1];  // per grid: plane items completed (batch entries)
};

// Work item order for `batch` grids with dependency lag `lag` (in grids):
// phase p emits the N plane items of grid p (p < batch) followed by the N
// slab items of grid p - lag (p >= lag).  Every plane item of grid g is
// dequeued before any slab item of g, so a slab item only ever waits for
// items already held by running workgroups.
struct Item {
    int slab;
    int g;
    int idx;
};

__device__ __forceinline__ Item decode_item(long i, int N, int batch, int lag)
{
    const int n1 = lag < batch ? lag : batch;
    const long s1 = (long)n1 * N;
    if (i < s1) return {0, (int)(i / N), (int)(i % N)};
    i -= s1;
    const int n2 = batch > lag ? batch - lag : 0;
    const long s2 = (long)n2 * 2 * N;
    if (i < s2) {
        const int ph = (int)(i / (2 * N)), r = (int)(i % (2 * N)), p = lag + ph;
        return r < N ? Item{0, p, r} : Item{1, p - lag, r - N};
    }
    i -= s2;
    return {1, n2 + (int)(i / N), (int)(i % N)};
}

constexpr unsigned kSpinLimit = 1u << 22;

// Hand-off protocol between workgroups (one launch, no cache-wide
// write-back or invalidate): plane items store their output with
// device-coherent write-through stores; a plane item is published (its
// grid's counter incremented) only after every wave of the workgroup has
// waited for all its outstanding memory operations, which includes those
// stores; slab items read the intermediate with device-coherent loads issued
// after they have observed the counter.  Publishing is deferred to the next
// item's load phase so that the store latency overlaps useful work.
template <int N, int S>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_fused(const float2* in, float2* out, const float2* __restrict__ tw, FusedCtl* ctl, int batch, int lag,
        int chunk)
{
    constexpr int T = PlaneGeom<N>::T;
    constexpr long V = (long)N * N * N;
    __shared__ float2 lds[PlaneGeom<N>::WORDS];
    __shared__ int item_sh;
    const int tid = threadIdx.x;
    const long total = 2L * batch * N;
    int pending = -1;
    long next = -1, chunk_end = -1;   // items of the current chunk (dynamic) or stride (static)   // grid of this workgroup's last unpublished plane item (uniform)
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (pending >= 0 && tid == 0)
            __hip_atomic_fetch_add(&ctl->done[pending], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pending = -1;
    };
    for (;;) {
        long it;
        if (chunk <= 0) {                    // static round robin
            it = next < 0 ? (long)blockIdx.x : next + gridDim.x;
            next = it;
        } else {
            if (next < 0 || next + 1 >= chunk_end) {
                if (tid == 0) item_sh = (int)atomicAdd(&ctl->head, (unsigned)chunk);
                __syncthreads();
                next = item_sh;
                chunk_end = next + chunk;
            } else {
                ++next;
            }
            it = next;
        }
        if (it >= total) break;
        const Item w = decode_item(it, N, batch, lag);
        if (!w.slab) {
            const long base = w.g * V + (long)w.idx * N * N;
            constexpr int RS = PlaneGeom<N>::RS;
            tile_to_lds<N, N, RS, T>(in + base, lds, tid);
            publish();   // previous plane's stores are complete by now
            fft_lds_all<N, S, N, T, RS, 1>(lds, tw, tid);
            const LdsAcc<1, RS> col{lds};
            const PlaneColOut<N, true> dst{out + base};
            run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
            pending = w.g;
        } else {
            publish();
            if (tid == 0) {
                unsigned n = 0;
                while (__hip_atomic_load(&ctl->done[w.g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)N) {
                    if (++n >= kSpinLimit) {
                        atomicAdd(&ctl->timeouts, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            const long base = w.g * V + (long)w.idx * N;
            slab_body<N, S, T, true>(out + base, out + base, (long)N * N, tw, lds, tid);
        }
        __syncthreads();   // LDS and item_sh reuse
    }
    publish();
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            for (int g = 0; g < batch; ++g) ctl->done[g] = 0;
            ctl->head = 0;
            __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// XCD-local form of the fused kernel.  Each XCD (accelerator complex die,
// with its own L2 shared by its 32 compute units) owns the grids g with
// g mod Q == its XCC id mod Q and has its own item queue, so a grid's planes
// and slabs are transformed by workgroups that share one L2.  With a lag of
// one grid at most two grids' intermediates are live per XCD (2 x 2 MiB at
// 64^3, the size of the L2), so the intermediate is handed over through the
// L2 instead of through HBM:
//   * plane items store with ordinary stores (the L1 writes through to the
//     L2); a plane item is published (its grid's counter incremented) after
//     every wave has waited for all its memory operations, i.e. after its
//     stores have completed into the L2;
//   * slab items read the intermediate with loads that miss the L1 and are
//     served by the L2 (load_xcd_coherent), issued after they have observed
//     the counter, so no stale L1 line (e.g. of an in-place input) is used.
// Workgroups claim one item ahead: while an item is transformed, the input
// plane of the next item (when it is a plane item) is already loading into
// registers (streaming loads: each input plane is read once).  Items are
// still claimed in list order, so the earliest unfinished item is always
// held by a running workgroup as its current item and progresses.  The last
// workgroup to leave checks that every queue was fully claimed (an XCD
// without workgroups would leave its grids untransformed; that is reported
// through the timeout counter).
struct XcdCtl {
    unsigned head[8][32];   // one queue counter per XCD, 128 bytes apart
    unsigned exited;
    unsigned timeouts;
    unsigned pad[30];
    unsigned done[1];       // per grid: plane items completed
};

__device__ __forceinline__ unsigned xcc_id()
{
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);   // HW_REG_XCC_ID[3:0]
}

template <int N, int S>
__global__ void __launch_bounds__(PlaneGeom<N>::T)
k_fused_xcd(const float2* in, float2* out, const float2* __restrict__ tw, XcdCtl* ctl, int batch, int q, int lag)
{
    constexpr int T = PlaneGeom<N>::T, RS = PlaneGeom<N>::RS;
    constexpr long V = (long)N * N * N;
    __shared__ float2 lds[PlaneGeom<N>::WORDS];
    __shared__ int item_sh;
    const int tid = threadIdx.x;
    const int x = (int)(xcc_id() % (unsigned)q);
    const int bq = (batch - x + q - 1) / q;     // grids of this XCD's queue
    const long total = 2L * bq * N;
    int pending = -1;
    TileRegs<N, N, T, true> regs;
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (pending >= 0 && tid == 0)
            __hip_atomic_fetch_add(&ctl->done[pending], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pending = -1;
    };
    auto claim = [&]() -> long {
        if (tid == 0) item_sh = (int)atomicAdd(&ctl->head[x][0], 1u);
        __syncthreads();
        const long it = item_sh;
        __syncthreads();
        return it;
    };
    // input plane of item `it` into registers, if it is a plane item
    auto prefetch = [&](long it) {
        if (it < total) {
            const Item w = decode_item(it, N, bq, lag);
            if (!w.slab) regs.load(in + (w.g * q + x) * V + (long)w.idx * N * N, tid);
        }
    };
    long cur = claim();
    prefetch(cur);
    while (cur < total) {
        const Item w = decode_item(cur, N, bq, lag);
        const int g = w.g * q + x;
        const long nxt = claim();
        if (!w.slab) {
            const long base = g * V + (long)w.idx * N * N;
            regs.template store_lds<RS>(lds, tid);
            publish();   // the previous plane's stores are complete by now
            prefetch(nxt);
            fft_lds_all<N, S, N, T, RS, 1>(lds, tw, tid);
            const LdsAcc<1, RS> col{lds};
            const PlaneColOut<N, false> dst{out + base};
            run_tail<N, S, N, T, 0, false>(col, dst, tw, tid);
            pending = g;
        } else {
            publish();
            prefetch(nxt);
            if (tid == 0) {
                unsigned n = 0;
                while (__hip_atomic_load(&ctl->done[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)N) {
                    if (++n >= kSpinLimit) {
                        atomicAdd(&ctl->timeouts, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            const long base = g * V + (long)w.idx * N;
            slab_body<N, S, T, 2>(out + base, out + base, (long)N * N, tw, lds, tid);
        }
        __syncthreads();   // LDS reuse
        cur = nxt;
    }
    publish();
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            for (int y = 0; y < q; ++y) {
                const int by = (batch - y + q - 1) / q;
                // queue not drained (each workgroup claims once past the end)
                if (ctl->head[y][0] < (unsigned)(2L * by * N)) atomicAdd(&ctl->timeouts, 1u);
                ctl->head[y][0] = 0;
            }
            for (int gg = 0; gg < batch; ++gg) ctl->done[gg] = 0;
            __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
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

// Final-store accessor of the energy epilogue: stores psi and accumulates
// V[r] |psi(r)|^2 (FP32 product, FP64 running sum) for this thread's points.
// STORE = false: the sum only, psi is not written.
template <bool STORE>
struct EnergyStoreT {
    const float2* src;
    float2* dst;
    long es;
    const float* v;
    mutable double acc;
    __device__ __forceinline__ float2 load(int, int e) const { return src[(long)e * es]; }
    __device__ __forceinline__ void store(int, int e, float2 val) const
    {
        if constexpr (STORE) dst[(long)e * es] = val;
        acc += (double)(v[(long)e * es] * fmaf(val.x, val.x, val.y * val.y));
    }
};
using EnergyStore = EnergyStoreT<true>;

// Fixed-order workgroup sum of one double per thread; result valid in thread 0.
template <int T>
__device__ __forceinline__ double block_sum(double x, double* red, int tid)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = x;
    __syncthreads();
    double t = 0.0;
    if (tid == 0)
        for (int w = 0; w < T / 64; ++w) t += red[w];
    return t;
}

// Strided access of one z-line of a pruned transform with the sphere
// |G|^2 < R2; gxy2 = Gx^2 + Gy^2 of the line, e the z index.
// MODE 1 (z pass of the pruned inverse): loads of elements with
//   Gz^2 >= R2 read zeros (those planes were never written by the plane
//   pass); every element is stored.
// MODE 2 (z pass of the pruned forward): a line with gxy2 >= R2 loads zeros
//   (the plane pass did not write it) and every element outside the sphere
//   is left unstored.
template <int MODE>
struct GlobStridedPruned {
    const float2* src;
    float2* dst;
    long es;
    int n;
    int gxy2;
    double R2;
    __device__ __forceinline__ float2 load(int, int e) const
    {
        if constexpr (MODE == 1) {
            const int g = signed_freq(e, n);
            return (double)(g * g) < R2 ? src[(long)e * es] : make_float2(0.f, 0.f);
        } else {
            return (double)gxy2 < R2 ? src[(long)e * es] : make_float2(0.f, 0.f);
        }
    }
    __device__ __forceinline__ void store(int, int e, float2 v) const
    {
        if constexpr (MODE == 2) {
            const int g = signed_freq(e, n);
            if ((double)(gxy2 + g * g) < R2) dst[(long)e * es] = v;
        } else {
            dst[(long)e * es] = v;
        }
    }
};

// Z-line (x, y) of grid b in the last pass of the pruned forward with a
// packed output: loads as GlobStridedPruned<2>; element z is stored to the
// packed sphere when row (z, y) holds point x.
struct GlobZPacked {
    const float2* src;
    float2* packed;                 // this grid's packed sphere
    const SphereRow* rows;          // [kz][ky] table
    long es;
    int x, y, ny, nx;
    bool line_in;                   // Gx^2 + Gy^2 < R2
    __device__ __forceinline__ float2 load(int, int e) const
    {
        return line_in ? src[(long)e * es] : make_float2(0.f, 0.f);
    }
    __device__ __forceinline__ void store(int, int e, float2 v) const
    {
        if (!line_in) return;
        const SphereRow r = rows[(long)e * ny + y];
        if (sphere_has(r, x, nx)) packed[sphere_rank(r, x, nx)] = v;
    }
};

// Tile of this workgroup in the strided (z) passes, in reverse launch
// order.  Workgroups start roughly in blockIdx order and the plane passes
// run their planes in increasing order, so a z pass that takes the highest
// tiles first begins on the data the plane pass before it wrote last (still
// in the Infinity Cache) and ends on the lowest, where the plane pass after
// it begins.  Measured on 32 x 128^3 inverse+forward: 0.757 -> 0.731 ms per
// step, with the plane pass's stores left in the caches (default policy).
__device__ __forceinline__ long rev_tile() { return (long)(gridDim.x - 1 - blockIdx.x); }

// ENERGY: the pass is the last one of an inverse transform psi = IFFT(c);
// while storing psi it accumulates sum V |psi|^2 and writes one FP64 partial
// per tile to partials[tile] (V indexed by position in the grid).
// PRUNE: 0 dense; 1 z pass of the pruned inverse, 2 z pass of the pruned
// forward (GlobStridedPruned), 3 z pass of the pruned forward into a packed
// sphere (GlobZPacked: `out` is the packed buffer, npts points per grid).
// 1 to 3 require the z-pass AxisMap.
// K: schedule kind (dense form only: 0 default, 2 the tuner's alternative
// order, with a twiddle table of the same kind).
template <int N, int S, int L, bool ENERGY = false, int PRUNE = 0, int K = 0>
__global__ void __launch_bounds__((AxisGeom<N, L>::T))
k_axis_str(const float2* in, float2* out, const float2* __restrict__ tw, AxisMap m, const float* __restrict__ V,
           double* __restrict__ partials, long vol, double R2 = 0.0, const SphereRow* __restrict__ rows = nullptr,
           long npts = 0)
{
    static_assert(K == 0 || (!ENERGY && PRUNE == 0), "schedule kinds other than 0 serve the dense form only");
    using G = AxisGeom<N, L>;
    using P = Plan1D<N, K>;
    constexpr int T = G::T;
    static_assert(T % L == 0, "each thread keeps one line");
    __shared__ float2 lds[P::stages > 1 ? G::WORDS : 1];
    const int tid = threadIdx.x;
    // tiles of fewer than 64 lines: a wave's butterflies span several twiddle
    // groups and read their twiddles per lane, from an LDS copy of the table
    // (stage 0 reads none; the barrier after it publishes the copy).  At
    // 512^3 (32-line tiles) the y and z passes 0.392 / 0.465 -> 0.386 /
    // 0.460 ms, at 4 x 256^3 0.169 / 0.211 -> 0.164 / 0.205 ms.
    constexpr bool TWL = L % 64 != 0 && P::stages > 1 && P::tw_len > 0;
    __shared__ float2 tw_lds[TWL ? P::tw_len : 1];
    if constexpr (TWL) {
        for (int i = tid; i < P::tw_len; i += T) tw_lds[i] = tw[i];
        tw = tw_lds;
    }
    const long tile = rev_tile();
    const long l0 = tile * L;
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
    if constexpr (ENERGY) {
        __shared__ double red[T / 64];
        const EnergyStore eg{in + gbase, out + gbase, m.es, V + (gbase % vol), 0.0};
        if constexpr (P::stages == 1) {
            fft_stage<N, 0, S, L, T, true, false>(g, eg, tw, tid, valid);
        } else {
            const LdsAcc<1, G::LP> a{lds};
            fft_stage<N, 0, S, L, T, true, false>(g, a, tw, tid, valid);
            __syncthreads();
            run_tail<N, S, L, T, 1, false>(a, eg, tw, tid, valid);
        }
        const double t = block_sum<T>(eg.acc, red, tid);
        if (tid == 0) partials[tile] = t;
    } else if constexpr (PRUNE == 3) {
        const long o = li / m.nx;
        const int x = (int)(li - o * m.nx), y = (int)(o % m.odiv);
        const long b = o / m.odiv;
        const int gx = signed_freq(x, (int)m.nx), gy = signed_freq(y, (int)m.odiv);
        const GlobZPacked gp{in + gbase, out + b * npts, rows, m.es, x, y, (int)m.odiv, (int)m.nx,
                             (double)(gx * gx + gy * gy) < R2 && li < m.lines};
        if constexpr (P::stages == 1) {
            fft_stage<N, 0, S, L, T, true, false>(gp, gp, tw, tid, valid);
        } else {
            const LdsAcc<1, G::LP> a{lds};
            fft_stage<N, 0, S, L, T, true, false>(gp, a, tw, tid, valid);
            __syncthreads();
            run_tail<N, S, L, T, 1, false>(a, gp, tw, tid, valid);
        }
    } else if constexpr (PRUNE != 0) {
        int gxy2 = 0;
        if constexpr (PRUNE == 2) {   // z pass: line li = (b * ny + y) * nx + x with odiv = ny
            const long o = li / m.nx;
            const int gx = signed_freq((int)(li - o * m.nx), (int)m.nx);
            const int gy = signed_freq((int)(o % m.odiv), (int)m.odiv);
            gxy2 = gx * gx + gy * gy;
        }
        const GlobStridedPruned<PRUNE> gp{in + gbase, out + gbase, m.es, N, gxy2, R2};
        if constexpr (P::stages == 1) {
            fft_stage<N, 0, S, L, T, true, false>(gp, gp, tw, tid, valid);
        } else {
            const LdsAcc<1, G::LP> a{lds};
            fft_stage<N, 0, S, L, T, true, false>(gp, a, tw, tid, valid);
            __syncthreads();
            run_tail<N, S, L, T, 1, false>(a, gp, tw, tid, valid);
        }
    } else {
        if constexpr (P::stages == 1) {
            fft_stage<N, 0, S, L, T, true, false, K>(g, g, tw, tid, valid);
        } else {
            const LdsAcc<1, G::LP> a{lds};
            fft_stage<N, 0, S, L, T, true, false, K>(g, a, tw, tid, valid);
            __syncthreads();
            // (16-byte paired stores, as in the plane pass, measured no faster here:
            // this pass already runs at the streaming-copy rate)
            run_tail<N, S, L, T, 1, false, K>(a, g, tw, tid, valid);
        }
    }
}


// The energy pass without its output: the last pass of psi = IFFT(c), its
// values only summed into sum V |psi|^2 (one FP64 partial per workgroup,
// partials[tile], the same products in the same order as the ENERGY
// form of k_axis_str) and never written.
template <int N, int S, int L>
__global__ void __launch_bounds__((AxisGeom<N, L>::T))
k_axis_energy(const float2* in, const float2* __restrict__ tw, AxisMap m, const float* __restrict__ V,
              double* __restrict__ partials, long vol)
{
    using G = AxisGeom<N, L>;
    using P = Plan1D<N>;
    constexpr int T = G::T;
    static_assert(T % L == 0, "each thread keeps one line");
    __shared__ float2 lds[P::stages > 1 ? G::WORDS : 1];
    __shared__ double red[T / 64];
    const int tid = threadIdx.x;
    const long tile = rev_tile();
    const long l0 = tile * L;
    const long li = l0 + tid % L;
    const int valid = (int)((m.lines - l0) < L ? (m.lines - l0) : L);
    long gbase = 0;
    if (li < m.lines) {
        const long o = li / m.nx;
        const long x = li - o * m.nx;
        gbase = (o / m.odiv) * m.shi + (o % m.odiv) * m.slo + x;
    }
    const GlobStrided g{in + gbase, nullptr, m.es};
    const EnergyStoreT<false> eg{in + gbase, nullptr, m.es, V + (gbase % vol), 0.0};
    if constexpr (P::stages == 1) {
        fft_stage<N, 0, S, L, T, true, false>(g, eg, tw, tid, valid);
    } else {
        const LdsAcc<1, G::LP> a{lds};
        fft_stage<N, 0, S, L, T, true, false>(g, a, tw, tid, valid);
        __syncthreads();
        run_tail<N, S, L, T, 1, false>(a, eg, tw, tid, valid);
    }
    const double t = block_sum<T>(eg.acc, red, tid);
    if (tid == 0) partials[tile] = t;
}

// --------------------------------------------------------------- x rows --

// The z part of the local-potential operator of a plane-wave code,
// out = forward(V * inverse(c)) with the transforms split as [inverse xy
// planes] [this kernel] [forward xy planes]: each workgroup takes L adjacent
// z-lines of the intermediate `buf`, runs the inverse z-transform into LDS
// (psi of those lines, which never reaches HBM), accumulates sum V |psi|^2
// (one FP64 partial per workgroup), multiplies psi by s V with
// s = mult * (scale ? scale[0] : 1), runs the forward z-transform and stores
// in place.  MODE 1 (sphere cutoff R2): only the elements with Gz^2 < R2 are
// loaded (the others were never written by the pruned inverse plane pass)
// and stored (the pruned forward plane pass reads only those planes).
template <int N, int L, int MODE>
__global__ void __launch_bounds__((AxisGeom<N, L>::T))
k_axis_hloc(float2* buf, const float2* __restrict__ tw_inv, const float2* __restrict__ tw_fwd, AxisMap m,
            const float* __restrict__ V, const double* __restrict__ scale, float mult, double* __restrict__ partials,
            long vol, double R2)
{
    using G = AxisGeom<N, L>;
    using P = Plan1D<N>;
    constexpr int T = G::T;
    static_assert(T % L == 0, "each thread keeps one line");
    __shared__ float2 lds[G::WORDS];
    __shared__ double red[T / 64];
    const int tid = threadIdx.x;
    const long tile = rev_tile();
    const long l0 = tile * L;
    const int myline = tid % L;
    const long li = l0 + myline;
    const int valid = (int)((m.lines - l0) < L ? (m.lines - l0) : L);
    long gbase = 0;
    if (li < m.lines) {
        const long o = li / m.nx;
        const long x = li - o * m.nx;
        gbase = (o / m.odiv) * m.shi + (o % m.odiv) * m.slo + x;
    }
    using Acc = typename std::conditional<MODE == 1, GlobStridedPruned<1>, GlobStrided>::type;
    using Out = typename std::conditional<MODE == 1, GlobStridedPruned<2>, GlobStrided>::type;
    Acc src{};
    Out dst{};
    if constexpr (MODE == 1) {
        src = Acc{buf + gbase, buf + gbase, m.es, N, 0, R2};
        dst = Out{buf + gbase, buf + gbase, m.es, N, 0, R2};
    } else {
        src = Acc{buf + gbase, buf + gbase, m.es};
        dst = Out{buf + gbase, buf + gbase, m.es};
    }
    const LdsAcc<1, G::LP> a{lds};
    // inverse z-transform into LDS
    fft_stage<N, 0, 1, L, T, true, false>(src, a, tw_inv, tid, valid);
    __syncthreads();
    if constexpr (P::stages > 1) {
        run_tail<N, 1, L, T, 1, false>(a, a, tw_inv, tid, valid);
        __syncthreads();
    }
    // psi -> energy partial, s V psi
    const float s = mult * (scale ? (float)scale[0] : 1.f);
    double acc = 0.0;
    if (myline < valid) {
        const float* v = V + (gbase % vol);
        for (int e = tid / L; e < N; e += T / L) {
            const float2 p = lds[e * G::LP + myline];
            const float vv = v[(long)e * m.es];
            acc += (double)(vv * fmaf(p.x, p.x, p.y * p.y));
            const float f = s * vv;
            lds[e * G::LP + myline] = make_float2(f * p.x, f * p.y);
        }
    }
    const double t = block_sum<T>(acc, red, tid);   // contains the barrier before the forward stages
    if (tid == 0 && partials) partials[tile] = t;
    // forward z-transform, stored in place
    if constexpr (P::stages == 1) {
        fft_stage<N, 0, -1, L, T, true, false>(a, dst, tw_fwd, tid, valid);
    } else {
        fft_stage<N, 0, -1, L, T, true, true>(a, a, tw_fwd, tid, valid);
        __syncthreads();
        run_tail<N, -1, L, T, 1, false>(a, dst, tw_fwd, tid, valid);
    }
}

// Density epilogue of the inverse transform: rho(r) = sum_b occ[b]
// |psi_b(r)|^2, psi_b the inverse z-transform of orbital b of `buf` (already
// transformed along x and y; orbitals `vol` apart).  Each workgroup owns L
// adjacent z-lines of the grid (map: the lines of ONE grid) and loops over
// the orbitals: stage 0 from HBM into LDS, the other stages in LDS, then each
// thread adds occ[b] |psi|^2 at its fixed points in registers (FP32 FMA, in
// fixed orbital order, last first: deterministic).  psi is never stored; rho ([z][y][x] real)
// is written once.  MODE 1 (cutoff R2): loads only of the planes with
// Gz^2 < R2 (the others were not written by the pruned plane pass).
template <int N, int L, int MODE>
__global__ void __launch_bounds__((AxisGeom<N, L>::T))
k_axis_density(const float2* buf, const float2* __restrict__ tw, AxisMap m, int batch, long vol,
               const float* __restrict__ occ, float* __restrict__ rho, double R2)
{
    using G = AxisGeom<N, L>;
    using P = Plan1D<N>;
    constexpr int T = G::T;
    static_assert(T % L == 0, "each thread keeps one line");
    constexpr int PER = (N * L + T - 1) / T;   // points per thread
    // stage 0 (radix R0, no twiddles) is split into its loads, issued one
    // orbital ahead into registers, and its butterflies
    constexpr int R0 = P::radix(0), M0 = N / R0, NB0 = L * M0, IT0 = (NB0 + T - 1) / T;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    // tiles of fewer than 64 lines read their twiddles per lane: from an LDS
    // copy, made once for all orbitals (published by the first barrier)
    constexpr bool TWL = L % 64 != 0 && P::stages > 1 && P::tw_len > 0;
    __shared__ float2 tw_lds[TWL ? P::tw_len : 1];
    if constexpr (TWL) {
        for (int i = tid; i < P::tw_len; i += T) tw_lds[i] = tw[i];
        tw = tw_lds;
    }
    const long tile = rev_tile();
    const long l0 = tile * L;
    const int myline = tid % L;
    const long li = l0 + myline;
    const int valid = (int)((m.lines - l0) < L ? (m.lines - l0) : L);
    long gbase = 0;
    if (li < m.lines) {
        const long o = li / m.nx;
        const long x = li - o * m.nx;
        gbase = (o / m.odiv) * m.shi + (o % m.odiv) * m.slo + x;
    }
    float2 pre[IT0][R0];
    auto load0 = [&](int b) {
        const float2* src = buf + (long)b * vol + gbase;
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int bb = tid + it * T, j = bb / L;
            if ((NB0 % T == 0 || bb < NB0) && myline < valid) {
#pragma unroll
                for (int q = 0; q < R0; ++q) {
                    const int e = j + q * M0;
                    if constexpr (MODE == 1) {
                        const int g = signed_freq(e, N);
                        pre[it][q] = (double)(g * g) < R2 ? src[(long)e * m.es] : make_float2(0.f, 0.f);
                    } else {
                        pre[it][q] = src[(long)e * m.es];
                    }
                }
            }
        }
    };
    float acc[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = 0.f;
    const LdsAcc<1, G::LP> a{lds};
    // orbitals from the last to the first: the plane pass before this one
    // wrote the last orbitals last, so they are the ones still in the caches
    if (batch > 0) load0(batch - 1);
    for (int b = batch - 1; b >= 0; --b) {
#pragma unroll
        for (int it = 0; it < IT0; ++it) {
            const int bb = tid + it * T, j = bb / L;
            if ((NB0 % T == 0 || bb < NB0) && myline < valid) {
                dft<R0, 1>(pre[it]);
#pragma unroll
                for (int q = 0; q < R0; ++q) lds[(j * R0 + q) * G::LP + myline] = pre[it][q];
            }
        }
        __syncthreads();
        if (b > 0) load0(b - 1);
        if constexpr (P::stages > 1) {
            run_tail<N, 1, L, T, 1, false>(a, a, tw, tid, valid);
            __syncthreads();
        }
        const float f = occ[b];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * T;
            if ((N * L) % T == 0 || i < N * L) {
                const float2 p = lds[(i / L) * G::LP + myline];
                acc[k] = fmaf(f, fmaf(p.x, p.x, p.y * p.y), acc[k]);
            }
        }
        __syncthreads();   // the next orbital's stage 0 overwrites the tile
    }
    if (myline < valid) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * T;
            if ((N * L) % T == 0 || i < N * L) rho[gbase + (long)(i / L) * m.es] = acc[k];
        }
    }
}

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
    // (an LDS copy of the twiddle table, as the strided pass makes for tiles
    // of fewer than 64 lines, measured slower here: 0.385 -> 0.419 ms for the
    // x pass of 512^3, one 4 KB table per 16-row tile)
    const long r0 = (long)blockIdx.x * L;
    const int valid = (int)((rows - r0) < L ? (rows - r0) : L);
    const long base = r0 * N;
    tile_to_lds<L, N, G::RS, T>(in + base, lds, tid, valid);
    __syncthreads();
    fft_lds_all<N, S, L, T, G::RS, 1>(lds, tw, tid, valid);
    lds_to_tile<L, N, G::RS, T>(lds, out + base, tid, valid);
}

}  // namespace fft3d
