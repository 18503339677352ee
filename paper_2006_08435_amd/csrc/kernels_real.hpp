// Real-grid transforms: the xy-plane passes of r2c (forward) and c2r
// (inverse) for Nx = Ny = N even.
//
// A real row f[0..N) is read as M = N/2 complex values z[m] = f[2m] +
// i f[2m+1] (the same bytes), transformed with a length-M FFT, and split into
// the half spectrum X[0..M] of f:
//   E_k = (Z_k + conj Z_{M-k}) / 2,  O_k = (Z_k - conj Z_{M-k}) / (2i),
//   X_k = E_k + W_N^k O_k,  X_{M-k} = conj(E_k - W_N^k O_k),
// (E and O are the DFTs of the even and odd samples; W_N = exp(-2 pi i/N)).
// The inverse merges a half spectrum h[0..M] into
//   Z'_k = (h_k + conj h_{M-k}) + i W_N^{-k} (h_k - conj h_{M-k}),
//   Z'_{M-k} = conj of the same with the sign of the second term flipped,
// whose unnormalised length-M inverse FFT holds f[2m] + i f[2m+1] of the
// unnormalised real inverse (the imaginary parts of h_0 and h_M are dropped,
// as the real inverse of a Hermitian extension ignores them).
//
// Half-spectrum planes are [y][M+1] complex; the z pass is the ordinary
// strided kernel over the half layout.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels_fp32.hpp"

namespace fft3d {

// Even supported lengths (r2c / c2r need Nx even).
#define FFT3D_FOR_EACH_EVEN_SIZE(X)                                            \
    X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(18) X(20) X(24) X(30) X(32) X(36)  \
    X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80) X(90) X(96) X(100) X(108)  \
    X(120) X(128)

template <int N>
struct RealGeom {
    static constexpr int M = N / 2, H = M + 1;
    static constexpr int RS = odd_stride(H);   // LDS row stride (complex values)
    static constexpr int WORDS = N * RS;
    static constexpr int TX = threads_for<M>(N), TY = threads_for<N>(H);
    static constexpr int T = TX > TY ? TX : TY;
    static constexpr int PAIRS = M / 2 + 1;    // (k, M-k) pairs per row
};

// Forward split of one row in LDS (k in [0, M/2]); w = W_N^k.
template <int N>
__device__ __forceinline__ void r2c_split(float2* row, int k, float2 w)
{
    constexpr int M = N / 2;
    if (k == 0) {
        const float2 a = row[0];
        row[0] = make_float2(a.x + a.y, 0.f);
        row[M] = make_float2(a.x - a.y, 0.f);
        return;
    }
    const float2 A = row[k], B = row[M - k];
    const float2 E = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
    const float2 O = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
    const float2 WO = cmul(w, O);
    row[k] = make_float2(E.x + WO.x, E.y + WO.y);
    if (2 * k != M) row[M - k] = make_float2(E.x - WO.x, WO.y - E.y);
}

// Inverse merge of one row in LDS (k in [0, M/2]); w = W_N^{-k}.
template <int N>
__device__ __forceinline__ void c2r_merge(float2* row, int k, float2 w)
{
    constexpr int M = N / 2;
    if (k == 0) {
        const float a = row[0].x, b = row[M].x;
        row[0] = make_float2(a + b, a - b);
        return;
    }
    const float2 A = row[k], B = row[M - k];
    const float2 P = make_float2(A.x + B.x, A.y - B.y);   // h_k + conj h_{M-k}
    const float2 D = make_float2(A.x - B.x, A.y + B.y);   // h_k - conj h_{M-k}
    const float2 WD = cmul(w, D);
    const float2 Q = make_float2(-WD.y, WD.x);            // i W^{-k} D
    row[k] = make_float2(P.x + Q.x, P.y + Q.y);
    if (2 * k != M) row[M - k] = make_float2(P.x - Q.x, Q.y - P.y);
}

// y-pass store of a half-spectrum plane: line = x in [0, M], element = y.
template <int N>
struct HalfColOut {
    float2* p;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const { p[y * (N / 2 + 1) + x] = v; }
};

// r2c plane pass (S = -1): real planes [planes][N][N] -> half-spectrum planes
// [planes][N][M+1], x split then y transform.  Persistent over planes with
// the next plane prefetched into registers.  tw_x: length-M table, tw_y:
// length-N table, rt[k] = W_N^k for k <= M/2.
template <int N, int S>
__global__ void __launch_bounds__(RealGeom<N>::T)
k_plane_r2c(const float* in, float2* out, const float2* __restrict__ tw_x, const float2* __restrict__ tw_y,
            const float2* __restrict__ rt, long planes)
{
    using G = RealGeom<N>;
    constexpr int M = G::M, H = G::H, T = G::T, RS = G::RS;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    const float2* in2 = reinterpret_cast<const float2*>(in);
    TileRegs<N, M, T, stream_plane(N)> regs;
    long p = blockIdx.x;
    if (p < planes) regs.load(in2 + p * N * M, tid);
    for (; p < planes; p += gridDim.x) {
        regs.template store_lds<RS>(lds, tid);
        __syncthreads();
        const long pn = p + gridDim.x;
        if (pn < planes) regs.load(in2 + pn * N * M, tid);
        fft_lds_all<M, S, N, T, RS, 1>(lds, tw_x, tid);
        for (int i = tid; i < N * G::PAIRS; i += T) {
            const int y = i / G::PAIRS, k = i % G::PAIRS;
            r2c_split<N>(lds + y * RS, k, rt[k]);
        }
        __syncthreads();
        const LdsAcc<1, RS> col{lds};
        const HalfColOut<N> dst{out + p * N * H};
        run_tail<N, S, H, T, 0, false>(col, dst, tw_y, tid);
        __syncthreads();
    }
}

// c2r plane pass (S = +1): half-spectrum planes [planes][N][M+1] (after the
// z pass) -> real planes [planes][N][N]: y transform, merge, x transform,
// coalesced row store.  rt[k] = W_N^{-k} for k <= M/2.
template <int N, int S>
__global__ void __launch_bounds__(RealGeom<N>::T)
k_plane_c2r(const float2* in, float* out, const float2* __restrict__ tw_x, const float2* __restrict__ tw_y,
            const float2* __restrict__ rt, long planes)
{
    using G = RealGeom<N>;
    constexpr int M = G::M, H = G::H, T = G::T, RS = G::RS;
    __shared__ float2 lds[G::WORDS];
    const int tid = threadIdx.x;
    float2* out2 = reinterpret_cast<float2*>(out);
    TileRegs<N, H, T, stream_plane(N)> regs;
    long p = blockIdx.x;
    if (p < planes) regs.load(in + p * N * H, tid);
    for (; p < planes; p += gridDim.x) {
        regs.template store_lds<RS>(lds, tid);
        __syncthreads();
        const long pn = p + gridDim.x;
        if (pn < planes) regs.load(in + pn * N * H, tid);
        fft_lds_all<N, S, H, T, 1, RS>(lds, tw_y, tid);
        for (int i = tid; i < N * G::PAIRS; i += T) {
            const int y = i / G::PAIRS, k = i % G::PAIRS;
            c2r_merge<N>(lds + y * RS, k, rt[k]);
        }
        __syncthreads();
        fft_lds_all<M, S, N, T, RS, 1>(lds, tw_x, tid);
        lds_to_tile<N, M, RS, T>(lds, out2 + p * N * M, tid);
        __syncthreads();
    }
}

}  // namespace fft3d
