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
//
// Columns x = 0 and x = M of a plane are real along y in the forward pass
// (X_0 and X_M of every row are real), and in the inverse only the real
// parts of their y transforms are used.  Both passes therefore transform
// M lines along y, not M + 1: column 0 carries c = a + i b, a and b the two
// real columns.  The forward splits C = FFT(c) afterwards into the two
// Hermitian transforms A_k = (C_k + conj C_{N-k}) / 2 and
// B_k = (C_k - conj C_{N-k}) / (2i); the inverse packs beforehand
// p = H(h_0) + i H(h_M) with H(h)_k = (h_k + conj h_{N-k}) / 2, whose inverse
// transform is Re IFFT(h_0) + i Re IFFT(h_M).  M lines per plane keep the y
// stages whole (65 lines of a 128 plane left one wave a second butterfly).
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
    static constexpr int TX = threads_for<M>(N), TY = threads_for<N>(M);
    // at most 512 threads: two workgroups per compute unit at N = 128
    static constexpr int T = (TX > TY ? TX : TY) > 512 ? 512 : (TX > TY ? TX : TY);
    static constexpr int PAIRS = M / 2 + 1;    // (k, M-k) pairs per row
};

// Forward split of one row in LDS (k in [0, M/2]); w = W_N^k.  The two real
// values X_0 and X_M go to slot 0 as X_0 + i X_M.
template <int N>
__device__ __forceinline__ void r2c_split(float2* row, int k, float2 w)
{
    constexpr int M = N / 2;
    if (k == 0) {
        const float2 a = row[0];
        row[0] = make_float2(a.x + a.y, a.x - a.y);
        return;
    }
    const float2 A = row[k], B = row[M - k];
    const float2 E = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
    const float2 O = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
    const float2 WO = cmul(w, O);
    row[k] = make_float2(E.x + WO.x, E.y + WO.y);
    if (2 * k != M) row[M - k] = make_float2(E.x - WO.x, WO.y - E.y);
}

// Inverse merge of one row in LDS (k in [0, M/2]); w = W_N^{-k}.  Slot 0
// holds Re h_0 + i Re h_M of the row (after the packed y transform).
template <int N>
__device__ __forceinline__ void c2r_merge(float2* row, int k, float2 w)
{
    constexpr int M = N / 2;
    if (k == 0) {
        const float a = row[0].x, b = row[0].y;
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

// y-pass store of a half-spectrum plane: line = x in [0, M), element = y;
// line 0 (the packed columns 0 and M) stays in the LDS tile (row stride RS)
// for the split that follows.
template <int N, int RS>
struct HalfColOut {
    float2* p;
    float2* lds;
    __device__ __forceinline__ float2 load(int, int) const { return float2{}; }
    __device__ __forceinline__ void store(int x, int y, float2 v) const
    {
        if (x == 0) lds[y * RS] = v;
        else p[y * (N / 2 + 1) + x] = v;
    }
};

// Forward: split the packed column C (slot 0 of every row of the tile) into
// columns 0 and M of the half-spectrum plane.  A thread takes the pair
// (k, N - k), so it reads only what it writes.
template <int N, int RS, int T>
__device__ __forceinline__ void r2c_unpack_cols(const float2* lds, float2* out, int tid)
{
    constexpr int M = N / 2, H = M + 1;
    for (int k = tid; k <= N / 2; k += T) {
        const int kn = (N - k) % N;
        const float2 c = lds[k * RS], d = lds[kn * RS];
        const float2 a = make_float2(0.5f * (c.x + d.x), 0.5f * (c.y - d.y));   // (C_k + conj C_{N-k}) / 2
        const float2 q = make_float2(0.5f * (c.x - d.x), 0.5f * (c.y + d.y));   // (C_k - conj C_{N-k}) / 2
        const float2 b = make_float2(q.y, -q.x);                                // q / i
        out[k * H] = a;
        out[k * H + M] = b;
        if (kn != k) {   // A and B are Hermitian
            out[kn * H] = make_float2(a.x, -a.y);
            out[kn * H + M] = make_float2(b.x, -b.y);
        }
    }
}

// Inverse: pack columns 0 and M of the tile into slot 0 as
// H(h_0) + i H(h_M).  A thread takes the pair (k, N - k).
template <int N, int RS, int T>
__device__ __forceinline__ void c2r_pack_cols(float2* lds, int tid)
{
    constexpr int M = N / 2;
    for (int k = tid; k <= N / 2; k += T) {
        const int kn = (N - k) % N;
        const float2 h0k = lds[k * RS], h0n = lds[kn * RS], hmk = lds[k * RS + M], hmn = lds[kn * RS + M];
        const float2 e = make_float2(0.5f * (h0k.x + h0n.x), 0.5f * (h0k.y - h0n.y));   // H(h_0)_k
        const float2 f = make_float2(0.5f * (hmk.x + hmn.x), 0.5f * (hmk.y - hmn.y));   // H(h_M)_k
        lds[k * RS] = make_float2(e.x - f.y, e.y + f.x);                              // e + i f
        if (kn != k) lds[kn * RS] = make_float2(e.x + f.y, f.x - e.y);                // conj e + i conj f
    }
}

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
    __shared__ float2 rts[G::PAIRS];   // the split's twiddles, read by every plane
    const int tid = threadIdx.x;
    const float2* in2 = reinterpret_cast<const float2*>(in);
    TileRegs<N, M, T, stream_plane(N)> regs;
    for (int k = tid; k < G::PAIRS; k += T) rts[k] = rt[k];   // visible after the first barrier below
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
            r2c_split<N>(lds + y * RS, k, rts[k]);
        }
        __syncthreads();
        const LdsAcc<1, RS> col{lds};
        const HalfColOut<N, RS> dst{out + p * N * H, lds};
        run_tail<N, S, M, T, 0, false>(col, dst, tw_y, tid);
        __syncthreads();
        r2c_unpack_cols<N, RS, T>(lds, out + p * N * H, tid);
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
    __shared__ float2 rts[G::PAIRS];   // the merge's twiddles, read by every plane
    const int tid = threadIdx.x;
    float2* out2 = reinterpret_cast<float2*>(out);
    TileRegs<N, H, T, stream_plane(N)> regs;
    for (int k = tid; k < G::PAIRS; k += T) rts[k] = rt[k];   // visible after the first barrier below
    long p = blockIdx.x;
    if (p < planes) regs.load(in + p * N * H, tid);
    for (; p < planes; p += gridDim.x) {
        regs.template store_lds<RS>(lds, tid);
        __syncthreads();
        const long pn = p + gridDim.x;
        if (pn < planes) regs.load(in + pn * N * H, tid);
        c2r_pack_cols<N, RS, T>(lds, tid);
        __syncthreads();
        fft_lds_all<N, S, M, T, 1, RS>(lds, tw_y, tid);
        for (int i = tid; i < N * G::PAIRS; i += T) {
            const int y = i / G::PAIRS, k = i % G::PAIRS;
            c2r_merge<N>(lds + y * RS, k, rts[k]);
        }
        __syncthreads();
        fft_lds_all<M, S, N, T, RS, 1>(lds, tw_x, tid);
        lds_to_tile<N, M, RS, T>(lds, out2 + p * N * M, tid);
        __syncthreads();
    }
}

}  // namespace fft3d
