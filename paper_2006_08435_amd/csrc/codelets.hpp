// Register-resident R-point DFT butterflies (R = 1, 2, 3, 4, 5, 6, 8, 9, 10,
// 12, 15, 16) on
// float2 complex values, for exponent sign S (-1 forward, +1 inverse):
//   X[k] = sum_n x[n] exp(S * 2 pi i n k / R),  in place on v[0..R).
// Constants are written to float precision from their closed forms.
#pragma once
#include <hip/hip_runtime.h>

namespace fft3d {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w)
{
    return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// S * i * a
template <int S> __device__ __forceinline__ float2 mul_si(float2 a)
{
    return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// a * exp(S * 2 pi i / 8) = a * (1 + S i) / sqrt(2)
template <int S> __device__ __forceinline__ float2 mul_w8(float2 a)
{
    constexpr float h = 0.70710678118654752f;
    return S > 0 ? make_float2((a.x - a.y) * h, (a.y + a.x) * h)
                 : make_float2((a.x + a.y) * h, (a.y - a.x) * h);
}

// a * exp(S * 2 pi i * 3 / 8) = a * (-1 + S i) / sqrt(2)
template <int S> __device__ __forceinline__ float2 mul_w8_3(float2 a)
{
    constexpr float h = 0.70710678118654752f;
    return S > 0 ? make_float2((-a.x - a.y) * h, (a.x - a.y) * h)
                 : make_float2((a.y - a.x) * h, (-a.x - a.y) * h);
}

// a * (c + S i s) for constants c, s
template <int S> __device__ __forceinline__ float2 mul_cs(float2 a, float c, float s)
{
    const float ss = S > 0 ? s : -s;
    return make_float2(fmaf(a.x, c, -a.y * ss), fmaf(a.x, ss, a.y * c));
}

template <int S> __device__ __forceinline__ void dft2(float2& a, float2& b)
{
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int S> __device__ __forceinline__ void dft3(float2& a, float2& b, float2& c)
{
    constexpr float h = 0.86602540378443865f;   // sqrt(3)/2
    const float2 t = cadd(b, c);
    const float2 d = csub(b, c);
    const float2 m = make_float2(fmaf(-0.5f, t.x, a.x), fmaf(-0.5f, t.y, a.y));
    const float2 r = mul_si<S>(cscale(d, h));
    a = cadd(a, t);
    b = cadd(m, r);
    c = csub(m, r);
}

template <int S> __device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d)
{
    const float2 t0 = cadd(a, c), t1 = csub(a, c);
    const float2 t2 = cadd(b, d), t3 = mul_si<S>(csub(b, d));
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, t3);
    d = csub(t1, t3);
}

template <int S> __device__ __forceinline__ void dft5(float2& a, float2& b, float2& c, float2& d, float2& e)
{
    constexpr float c1 = 0.30901699437494742f;    // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742f;   // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357f;    // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247313f;    // sin(4 pi / 5)
    const float2 t1 = cadd(b, e), d1 = csub(b, e);
    const float2 t2 = cadd(c, d), d2 = csub(c, d);
    const float2 m1 = make_float2(fmaf(c1, t1.x, fmaf(c2, t2.x, a.x)), fmaf(c1, t1.y, fmaf(c2, t2.y, a.y)));
    const float2 m2 = make_float2(fmaf(c2, t1.x, fmaf(c1, t2.x, a.x)), fmaf(c2, t1.y, fmaf(c1, t2.y, a.y)));
    const float2 r1 = mul_si<S>(make_float2(fmaf(s1, d1.x, s2 * d2.x), fmaf(s1, d1.y, s2 * d2.y)));
    const float2 r2 = mul_si<S>(make_float2(fmaf(s2, d1.x, -s1 * d2.x), fmaf(s2, d1.y, -s1 * d2.y)));
    a = cadd(a, cadd(t1, t2));
    b = cadd(m1, r1);
    e = csub(m1, r1);
    c = cadd(m2, r2);
    d = csub(m2, r2);
}

// 8 points: radix-2 split x[n] +/- x[n+4], then two 4-point DFTs.
template <int S> __device__ __forceinline__ void dft8(float2* v)
{
    float2 a0 = cadd(v[0], v[4]), b0 = csub(v[0], v[4]);
    float2 a1 = cadd(v[1], v[5]), b1 = csub(v[1], v[5]);
    float2 a2 = cadd(v[2], v[6]), b2 = csub(v[2], v[6]);
    float2 a3 = cadd(v[3], v[7]), b3 = csub(v[3], v[7]);
    b1 = mul_w8<S>(b1);
    b2 = mul_si<S>(b2);
    b3 = mul_w8_3<S>(b3);
    dft4<S>(a0, a1, a2, a3);
    dft4<S>(b0, b1, b2, b3);
    v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
    v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

// 16 points as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <int S> __device__ __forceinline__ void dft16(float2* v)
{
    constexpr float C1 = 0.92387953251128676f;   // cos(pi / 8)
    constexpr float S1 = 0.38268343236508977f;   // sin(pi / 8)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<S>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] now holds Y_{n2}[k1]; twiddle by W16^{n2 k1}
    v[5] = mul_cs<S>(v[5], C1, S1);      // n2=1,k1=1: W^1
    v[6] = mul_w8<S>(v[6]);              // n2=2,k1=1: W^2
    v[7] = mul_cs<S>(v[7], S1, C1);      // n2=3,k1=1: W^3
    v[9] = mul_w8<S>(v[9]);              // n2=1,k1=2: W^2
    v[10] = mul_si<S>(v[10]);            // n2=2,k1=2: W^4
    v[11] = mul_w8_3<S>(v[11]);          // n2=3,k1=2: W^6
    v[13] = mul_cs<S>(v[13], S1, C1);    // n2=1,k1=3: W^3
    v[14] = mul_w8_3<S>(v[14]);          // n2=2,k1=3: W^6
    v[15] = mul_cs<S>(v[15], -C1, -S1);  // n2=3,k1=3: W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<S>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]; transpose 4x4 into natural order
    float2 t;
    t = v[1]; v[1] = v[4]; v[4] = t;
    t = v[2]; v[2] = v[8]; v[8] = t;
    t = v[3]; v[3] = v[12]; v[12] = t;
    t = v[6]; v[6] = v[9]; v[9] = t;
    t = v[7]; v[7] = v[13]; v[13] = t;
    t = v[11]; v[11] = v[14]; v[14] = t;
}

template <int R, int S> __device__ __forceinline__ void dft(float2* v);

// Index k in [0, R1 R2) with k = k1 (mod R1) and k = k2 (mod R2) (Chinese
// remainder map; R1, R2 coprime).
template <int R1, int R2>
__host__ __device__ constexpr int crt_index(int k1, int k2)
{
    for (int k = 0; k < R1 * R2; ++k)
        if (k % R1 == k1 && k % R2 == k2) return k;
    return 0;
}

// R1 R2 points with R1, R2 coprime by the prime-factor (Good-Thomas) mapping:
// input n = (n1 R2 + n2 R1) mod R and output k = CRT(k1, k2) turn the DFT
// into R2 DFTs of length R1 followed by R1 DFTs of length R2 with no
// twiddle factors.  All indices are compile-time constants, so the
// permutations are register renaming.
template <int R1, int R2, int S> __device__ __forceinline__ void dft_pfa(float2* v)
{
    constexpr int R = R1 * R2;
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[(n1 * R2 + n2 * R1) % R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) dft<R1, S>(a[n2]);
    float2 b[R1][R2];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) b[k1][n2] = a[n2][k1];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) dft<R2, S>(b[k1]);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[crt_index<R1, R2>(k1, k2)] = b[k1][k2];
}

// 9 points as 3 x 3: n = 3 n1 + n2, k = k1 + 3 k2, twiddles W9^(n2 k1).
template <int S> __device__ __forceinline__ void dft9(float2* v)
{
    constexpr float C1 = 0.76604444311897804f, S1 = 0.64278760968653933f;    // 2 pi / 9
    constexpr float C2 = 0.17364817766693035f, S2 = 0.98480775301220806f;    // 4 pi / 9
    constexpr float C4 = -0.93969262078590838f, S4 = 0.34202014332566873f;   // 8 pi / 9
    float2 a[3][3];   // a[n2][.]
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
        a[n2][0] = v[n2];
        a[n2][1] = v[3 + n2];
        a[n2][2] = v[6 + n2];
        dft3<S>(a[n2][0], a[n2][1], a[n2][2]);   // a[n2][k1]
    }
    a[1][1] = mul_cs<S>(a[1][1], C1, S1);
    a[1][2] = mul_cs<S>(a[1][2], C2, S2);
    a[2][1] = mul_cs<S>(a[2][1], C2, S2);
    a[2][2] = mul_cs<S>(a[2][2], C4, S4);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        float2 x0 = a[0][k1], x1 = a[1][k1], x2 = a[2][k1];
        dft3<S>(x0, x1, x2);
        v[k1] = x0;
        v[k1 + 3] = x1;
        v[k1 + 6] = x2;
    }
}

template <int R, int S> __device__ __forceinline__ void dft(float2* v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        dft2<S>(v[0], v[1]);
    } else if constexpr (R == 3) {
        dft3<S>(v[0], v[1], v[2]);
    } else if constexpr (R == 4) {
        dft4<S>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 5) {
        dft5<S>(v[0], v[1], v[2], v[3], v[4]);
    } else if constexpr (R == 6) {
        dft_pfa<2, 3, S>(v);
    } else if constexpr (R == 8) {
        dft8<S>(v);
    } else if constexpr (R == 9) {
        dft9<S>(v);
    } else if constexpr (R == 10) {
        dft_pfa<2, 5, S>(v);
    } else if constexpr (R == 12) {
        dft_pfa<4, 3, S>(v);
    } else if constexpr (R == 15) {
        dft_pfa<3, 5, S>(v);
    } else if constexpr (R == 16) {
        dft16<S>(v);
    } else {
        static_assert(R == 16, "unsupported radix");
    }
}

}  // namespace fft3d
