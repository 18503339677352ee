// Radix schedules and twiddle-table geometry shared by the host planner and
// the device kernels of the FP32 path.
//
// A 1D transform of length N (2*3*5-smooth, 1 <= N <= 512) is computed as a
// sequence of self-sorting (Stockham) radix-R stages.  Stage s has radix r[s]
// and "span" NS(s) = r[0] * ... * r[s-1]; its butterfly j reads elements
// j + q*N/R (q < R), multiplies element q by W_{NS*R}^{(j mod NS) q}, applies
// the R-point DFT and writes element (j / NS) * NS * R + (j mod NS) + q * NS.
// After the last stage the result is in natural order.
//
// Twiddle table of a length-N transform and sign S: for every stage s >= 1,
// NS(s) * (R - 1) complex values tw[off(s) + k * (R - 1) + (q - 1)] =
// exp(S * 2 pi i * k q / (NS(s) * R)), k < NS(s), 1 <= q < R.
#pragma once

namespace fft3d {

struct Sched {
    int count;
    int r[8];
};

__host__ __device__ constexpr Sched make_sched_pow2(int n);

// Radices with a register codelet.
__host__ __device__ constexpr bool radix_ok(int r)
{
    return r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 8 || r == 9 || r == 10 || r == 12 || r == 15 ||
           r == 16;
}

// Schedule of n: powers of two keep their measured table; eight lengths take
// a measured two-stage order; any other n with a factor 3 or 5 takes the
// fewest stages over the radices above (each stage is one pass through LDS),
// then the smallest largest radix (fewer registers per butterfly), then
// non-increasing radices, searched over ordered factorizations of up to 4
// stages (n <= 512).
__host__ __device__ constexpr Sched make_sched(int n)
{
    int m = n;
    while (m % 2 == 0) m /= 2;
    if (n == 1 || m == 1) return make_sched_pow2(n);
    // two-stage orders measured fastest (planes + z lines, both signs) where
    // they differ from the rule below
    {
        int r0 = 0, r1 = 0;
        switch (n) {
        case 24: r0 = 8; r1 = 3; break;
        case 40: r0 = 5; r1 = 8; break;
        case 48: r0 = 16; r1 = 3; break;
        case 72: r0 = 12; r1 = 6; break;
        case 75: r0 = 5; r1 = 15; break;
        case 80: r0 = 8; r1 = 10; break;
        case 108: r0 = 9; r1 = 12; break;
        case 120: r0 = 8; r1 = 15; break;
        default: break;
        }
        if (r0) return Sched{2, {r0, r1, 0, 0, 0, 0, 0, 0}};
    }
    Sched best{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    int best_max = 1 << 30;
    const int rs[11] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
    for (int stages = 1; stages <= 4 && best.count == 0; ++stages) {
        // enumerate non-increasing radix sequences of length `stages` with product n
        int idx[4] = {0, 0, 0, 0};
        for (;;) {
            long prod = 1;
            bool ordered = true;
            for (int i = 0; i < stages; ++i) {
                prod *= rs[idx[i]];
                if (i > 0 && rs[idx[i]] > rs[idx[i - 1]]) ordered = false;
            }
            if (ordered && prod == n) {
                const int mx = rs[idx[0]];
                if (mx < best_max) {
                    best_max = mx;
                    best.count = stages;
                    for (int i = 0; i < stages; ++i) best.r[i] = rs[idx[i]];
                }
            }
            int k = stages - 1;
            while (k >= 0 && idx[k] == 10) { idx[k] = 0; --k; }
            if (k < 0) break;
            ++idx[k];
        }
    }
    if (best.count) return best;
    // not reachable for 2*3*5-smooth n <= 512; fall back to single factors
    Sched s = make_sched_pow2(n / m * 1);
    while (m % 3 == 0) { s.r[s.count++] = 3; m /= 3; }
    while (m % 5 == 0) { s.r[s.count++] = 5; m /= 5; }
    return s;
}

// Powers of two (and the power-of-two part of other lengths).
__host__ __device__ constexpr Sched make_sched_pow2(int n)
{
    Sched s{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    if (n == 1) {
        s.r[s.count++] = 1;
        return s;
    }
    int m = n, p2 = 0;
    while (m % 2 == 0) { m /= 2; ++p2; }
    switch (p2) {
    case 0: break;
    case 1: s.r[s.count++] = 2; break;
    case 2: s.r[s.count++] = 4; break;
    case 3: s.r[s.count++] = 8; break;
    case 4: s.r[s.count++] = 16; break;
    case 5: s.r[s.count++] = 8; s.r[s.count++] = 4; break;
    case 6: s.r[s.count++] = 8; s.r[s.count++] = 8; break;
    case 7: s.r[s.count++] = 8; s.r[s.count++] = 16; break;
    case 8: s.r[s.count++] = 16; s.r[s.count++] = 16; break;
    default: s.r[s.count++] = 8; s.r[s.count++] = 8; s.r[s.count++] = 8; break;   // 512
    }
    while (m % 3 == 0) { s.r[s.count++] = 3; m /= 3; }
    while (m % 5 == 0) { s.r[s.count++] = 5; m /= 5; }
    return s;
}

// Schedule of the reduced-precision form: a radix-16 first stage (computed
// as a DFT-matrix product on the matrix cores) followed by the default
// schedule of N / 16.  Requires 16 | N.
__host__ __device__ constexpr Sched make_sched16(int n)
{
    Sched s{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    s.r[s.count++] = 16;
    if (n / 16 > 1) {
        const Sched t = make_sched(n / 16);
        for (int i = 0; i < t.count; ++i) s.r[s.count++] = t.r[i];
    }
    return s;
}

// The autotuner's alternative schedule of n (kind 2): the default's two
// radices in the other order, or, where the default repeats one radix, the
// length split another way; lengths with neither keep the default.
__host__ __device__ constexpr Sched make_sched_alt(int n)
{
    Sched s = make_sched(n);
    if (s.count == 2 && s.r[0] != s.r[1]) {
        const int t = s.r[0];
        s.r[0] = s.r[1];
        s.r[1] = t;
        return s;
    }
    switch (n) {
    case 16: return Sched{2, {4, 4, 0, 0, 0, 0, 0, 0}};
    case 36: return Sched{2, {9, 4, 0, 0, 0, 0, 0, 0}};
    case 64: return Sched{2, {16, 4, 0, 0, 0, 0, 0, 0}};
    case 100: return Sched{3, {4, 5, 5, 0, 0, 0, 0, 0}};
    default: return s;
    }
}

// kind 0: default; 1: radix 16 first (reduced-precision form); 2: the
// autotuner's alternative order.
__host__ __device__ constexpr Sched make_sched_kind(int n, int kind)
{
    return kind == 1 ? make_sched16(n) : (kind == 2 ? make_sched_alt(n) : make_sched(n));
}

__host__ __device__ constexpr int sched_ns(const Sched& s, int stage)
{
    int p = 1;
    for (int i = 0; i < stage; ++i) p *= s.r[i];
    return p;
}

__host__ __device__ constexpr int sched_tw_off(const Sched& s, int stage)
{
    int o = 0;
    for (int i = 1; i < stage; ++i) o += sched_ns(s, i) * (s.r[i] - 1);
    return o;
}

__host__ __device__ constexpr int sched_tw_len(const Sched& s)
{
    return sched_tw_off(s, s.count);
}

__host__ __device__ constexpr int sched_max_radix(const Sched& s)
{
    int m = 1;
    for (int i = 0; i < s.count; ++i) m = s.r[i] > m ? s.r[i] : m;
    return m;
}

__host__ __device__ constexpr int sched_min_radix(const Sched& s)
{
    int m = 1 << 30;
    for (int i = 0; i < s.count; ++i) m = s.r[i] < m ? s.r[i] : m;
    return m;
}

__host__ __device__ constexpr bool smooth235(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

// Lengths of every form: 2*3*5-smooth, 1..128.
__host__ __device__ constexpr bool size_supported(int n) { return n <= 128 && smooth235(n); }

// Lengths of the three-pass form only (one line of up to 512 points per
// transform, lines of 16..32 per workgroup): 2*3*5-smooth, 129..512.
__host__ __device__ constexpr bool size_supported_large(int n) { return n > 128 && n <= 512 && smooth235(n); }

}  // namespace fft3d

// X-macro over the cubic lengths served by the persistent fused kernel
// (smaller cubes use the whole-grid-in-LDS kernel).
#define FFT3D_FOR_EACH_FUSED_SIZE(X)                                           \
    X(18) X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(50)    \
    X(54) X(60) X(64) X(72) X(75) X(80) X(81) X(90) X(96) X(100) X(108)        \
    X(120) X(125) X(128)

// X-macro over every supported length.
#define FFT3D_FOR_EACH_SIZE(X)                                                 \
    X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18)      \
    X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(50) X(54)    \
    X(60) X(64) X(72) X(75) X(80) X(81) X(90) X(96) X(100) X(108) X(120)       \
    X(125) X(128)

// X-macro over the lengths of the three-pass form above 128.
#define FFT3D_FOR_EACH_LARGE_SIZE(X)                                           \
    X(135) X(144) X(150) X(160) X(162) X(180) X(192) X(200) X(216) X(225)      \
    X(240) X(243) X(250) X(256) X(270) X(288) X(300) X(320) X(324) X(360)      \
    X(375) X(384) X(400) X(405) X(432) X(450) X(480) X(486) X(500) X(512)
