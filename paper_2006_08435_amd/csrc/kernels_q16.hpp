// Reduced-precision form: scaled 16-bit storage with FP32 arithmetic; the
// radix-16 stage runs either as an FP32 butterfly on the vector ALUs (the
// default: faster and more accurate on MI355X) or as a DFT-matrix product on
// the matrix cores.
//
// Storage ("scaled16"): a buffer of R rows of C complex values holds a
// payload of R*C 32-bit words (low half = real part, high half = imaginary
// part, each a binary16 or bfloat16 pattern) followed by R int8 exponents;
// the value of an entry is payload * 2^exponent.  Exponent rule per row:
// m = max |re|, |im| over the row; e = 0 if m == 0, else
// clamp(ilogb(m) - 14, -128, 127), so the scaled row maximum lies in
// [2^14, 2^15).  Conversions round to nearest, ties to even.
//
// Transform (cubic N, 16 | N): the 1D schedule is radix 16 first, then the
// default schedule of N / 16.  The matrix-core radix-16 stage multiplies 16-point columns
// by the DFT matrix written as a real 32x32 matrix [[C, -sS], [sS, C]]
// (C = cos, S = sin of 2 pi m k / 16, s = exponent sign) with
// v_mfma_f32_16x16x32_f16: FP16 operands (each column scaled by a power of
// two so its largest component lies in [2^14, 2^15)), FP32 accumulation.
// Twiddles and the other radices run in FP32 on the vector ALUs.  Pass A
// (xy-planes) stores its intermediate as scaled FP16 whatever the output
// format; pass B (xz-slabs) stores the result in the plan's format.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels_fp32.hpp"

namespace fft3d {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kFmtF16 = 1;
constexpr int kFmtBF16 = 2;

template <int FMT>
__device__ __forceinline__ float dec16(unsigned h)
{
    if constexpr (FMT == kFmtF16) return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
    else return __builtin_bit_cast(float, h << 16);
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// One payload word from a complex value: low half the real part, high half
// the imaginary part, each rounded to nearest, ties to even (one packed
// conversion instruction on gfx950 for either format).
template <int FMT>
__device__ __forceinline__ unsigned enc16x2(float re, float im)
{
    const f32x2_t f = {re, im};
    if constexpr (FMT == kFmtF16) return __builtin_bit_cast(unsigned, __builtin_convertvector(f, f16x2_t));
    else return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2_t));
}

// max(m, |v.re|, |v.im|).  The NaN-propagating maximum compiles to
// v_maximum3_f32 with absolute-value operand modifiers; maxnum (fmaxf)
// would first quiet every operand with an extra instruction.
__device__ __forceinline__ float absmax(float m, float2 v)
{
    return __builtin_elementwise_maximum(m, __builtin_elementwise_maximum(fabsf(v.x), fabsf(v.y)));
}

__device__ __forceinline__ unsigned fbits(float x) { return __builtin_bit_cast(unsigned, x); }

// Maxima of absolute values run on their bit patterns: non-negative floats
// order like their patterns as unsigned integers, and an integer maximum
// takes a DPP operand in the same instruction (v_max_u32_dpp).

// max(m, the pattern DPP control CTL moves into this lane); a lane outside
// ROW_MASK reads 0, the identity of the maximum.
template <int CTL, int ROW_MASK = 0xF>
__device__ __forceinline__ unsigned dpp_max(unsigned m)
{
    return max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, CTL, ROW_MASK, 0xF, false));
}

// Maximum over each row of 16 lanes, in every lane of the row: lanes 1
// apart, then 2 apart (quad permutations), then the two quads of each half
// (half-row mirror), then the two halves (row mirror).  Every lane must be
// active.
__device__ __forceinline__ unsigned rowmax16(unsigned m)
{
    m = dpp_max<0xB1>(m);       // quad_perm [1,0,3,2]
    m = dpp_max<0x4E>(m);       // quad_perm [2,3,0,1]
    m = dpp_max<0x141>(m);      // row_half_mirror
    return dpp_max<0x140>(m);   // row_mirror
}

// Maximum over the wave, wave-uniform: the row maxima, then row 0's into
// row 1 and row 2's into row 3 (row_bcast15), then row 1's into rows 2 and
// 3 (row_bcast31), so that lane 63 holds the maximum of all four rows.
// Every lane must be active.
__device__ __forceinline__ unsigned wavemax(unsigned m)
{
    m = rowmax16(m);
    m = dpp_max<0x142, 0xA>(m);
    m = dpp_max<0x143, 0xC>(m);
    return (unsigned)__builtin_amdgcn_readlane((int)m, 63);
}

// Wave maxima of R = 4 or 8 values per lane at once, by halving exchanges
// that also transpose: v_permlane32_swap pairs value i with i + R/2 (after
// the maximum, lanes 0-31 hold value i's partial maximum and lanes 32-63
// value i + R/2's), then v_permlane16_swap pairs the results again, so that
// each row of 16 lanes holds one value's partial maximum; a row reduction
// finishes them.  out[q]: the maximum of value q, wave-uniform.  Every lane
// must be active.
template <int R>
__device__ __forceinline__ void wavemax_many(const unsigned (&m)[R], unsigned (&out)[R])
{
    static_assert(R == 4 || R == 8, "four or eight values");
    constexpr int H = R / 2, Q = R / 4;
    unsigned n[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {   // n[i]: value i in lanes 0-31, value i + H in lanes 32-63
        const auto sw = __builtin_amdgcn_permlane32_swap(m[i], m[i + H], false, false);
        n[i] = max((unsigned)sw[0], (unsigned)sw[1]);
    }
    unsigned p[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {   // p[i]: values i, i + Q, i + H, i + H + Q in rows 0, 1, 2, 3
        const auto sw = __builtin_amdgcn_permlane16_swap(n[i], n[i + Q], false, false);
        p[i] = rowmax16(max((unsigned)sw[0], (unsigned)sw[1]));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        out[i] = (unsigned)__builtin_amdgcn_readlane((int)p[i], 0);
        out[i + Q] = (unsigned)__builtin_amdgcn_readlane((int)p[i], 16);
        out[i + H] = (unsigned)__builtin_amdgcn_readlane((int)p[i], 32);
        out[i + H + Q] = (unsigned)__builtin_amdgcn_readlane((int)p[i], 48);
    }
}

// Row exponent of the storage rule for a finite row maximum m >= 0 given
// by its bit pattern b: ilogb(m) - 14 = (biased exponent - 127) - 14 for a
// normal m; every m below 2^-114 (subnormals included) clamps to -128, and
// the largest finite m gives 113, so only the lower clamp is needed.
__device__ __forceinline__ int row_exponent_bits(unsigned b)
{
    if (b == 0) return 0;
    const int e = (int)(b >> 23) - 127 - 14;
    return e < -128 ? -128 : e;
}

template <int N>
struct Q16Geom {
    static constexpr int RS = odd_stride(N);
    static constexpr int WORDS = N * RS;
    static constexpr int T = threads_for_kind<N, 1>(N);
};

// NR rows of N scaled16 payload words held in registers (one 4-byte word
// per lane and load, consecutive lanes on consecutive points: coalesced
// loads, conflict-free LDS stores), plus the row exponent of row `tid`: the
// next tile is loaded while the current one is being transformed.
template <int NR, int N, int T>
struct Q16Regs {
    static constexpr int UNITS = NR * N, IT = (UNITS + T - 1) / T;
    static_assert(NR <= T, "one exponent per thread");
    unsigned u[IT];
    int ev;
    // rows r at pay + r * rstride, exponents at ex[r * estride]; OFF32:
    // 32-bit element offsets from pay (the tile spans < 2^32 elements); NT:
    // streaming payload loads (see stream_plane)
    template <bool OFF32 = false, bool NT = false>
    __device__ __forceinline__ void load(const unsigned* pay, long rstride, const signed char* ex, long estride,
                                         int tid)
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                if constexpr (OFF32) u[k] = pay[(unsigned)((i / N) * rstride + (i % N))];
                else if constexpr (NT) u[k] = __builtin_nontemporal_load(pay + (i / N) * rstride + (i % N));
                else u[k] = pay[(i / N) * rstride + (i % N)];
            }
        }
        if (tid < NR) ev = OFF32 ? ex[(unsigned)(tid * estride)] : ex[tid * estride];
    }
    // exact FP32 values into the LDS tile (row stride RS); lds_e must hold
    // the exponents (see put_exponent) and be visible to every thread
    template <int RS, int FMT>
    __device__ __forceinline__ void to_lds(float2* lds, const int* lds_e, int tid) const
    {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int i = tid + k * T;
            if (UNITS % T == 0 || i < UNITS) {
                const int r = i / N, x = i % N, e = lds_e[r];
                lds[r * RS + x] = make_float2(ldexpf(dec16<FMT>(u[k] & 0xFFFFu), e), ldexpf(dec16<FMT>(u[k] >> 16), e));
            }
        }
    }
    __device__ __forceinline__ void put_exponent(int* lds_e, int tid) const
    {
        if (tid < NR) lds_e[tid] = ev;
    }
};

// Requantize NR rows of N FP32 values from the LDS tile to scaled16: one
// wave per row (lanes along the row), row maximum by a wave reduction.
template <int NR, int N, int RS, int T, int FMT>
__device__ __forceinline__ void q16_store_rows(const float2* lds, unsigned* pay, long rstride, signed char* ex,
                                               long estride, int tid)
{
    constexpr int W = T / 64, PER = (N + 63) / 64;
    const int lane = tid & 63, wave = tid >> 6;
    for (int r = wave; r < NR; r += W) {
        float2 v[PER];
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int x = lane + 64 * k;
            v[k] = x < N ? lds[r * RS + x] : make_float2(0.f, 0.f);
            m = absmax(m, v[k]);
        }
        const int e = row_exponent_bits(wavemax(fbits(m)));
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int x = lane + 64 * k;
            if (x < N) pay[r * rstride + x] = enc16x2<FMT>(ldexpf(v[k].x, -e), ldexpf(v[k].y, -e));
        }
        if (lane == 0) ex[r * estride] = (signed char)e;
    }
}

// cos and sin of 2 pi t / 16, t = 0..15.
__device__ __forceinline__ float cos16(int t)
{
    constexpr float c[16] = {1.0f, 0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                             -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128676f, -1.0f,
                             -0.92387953251128676f, -0.70710678118654752f, -0.38268343236508977f, 0.0f,
                             0.38268343236508977f, 0.70710678118654752f, 0.92387953251128676f};
    return c[t & 15];
}
__device__ __forceinline__ float sin16(int t) { return cos16(t + 12); }   // sin x = cos(x - pi/2)

// Radix-16 stage 0 of schedule KIND 1 on an LDS tile (L lines of N, line
// stride LS, element stride ES), in place, on the matrix cores.  A wave takes
// 16 columns (line, j) at a time: lane l holds 8 real or 8 imaginary parts
// of column l % 16 (operand row block 8 * (l / 16)); two 16x16x32 products
// give the real and imaginary outputs, 4 per lane (rows 4 * (l / 16) + i).
template <int N, int S, int L, int T, int LS, int ES>
__device__ __forceinline__ void mfma_stage16(float2* lds, int tid)
{
    constexpr int M = N / 16, COLS = L * M, GROUPS = COLS / 16, W = T / 64, GPW = (GROUPS + W - 1) / W;
    static_assert(COLS % 16 == 0, "columns come in groups of 16");
    const int lane = tid & 63, wave = tid >> 6, c16 = lane & 15, h = lane >> 4;
    half8_t are, aim;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int kk = 8 * h + i, k = kk & 15, t = (c16 * k) & 15;
        const float c = cos16(t), sn = (S > 0 ? 1.f : -1.f) * sin16(t);
        are[i] = (_Float16)(kk < 16 ? c : -sn);
        aim[i] = (_Float16)(kk < 16 ? sn : c);
    }
    float2 outv[GPW][4];
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
        const int G = wave + g * W;
        if (GROUPS % W == 0 || G < GROUPS) {
            const int col = G * 16 + c16, line = col % L, j = col / L;
            const float* f = reinterpret_cast<const float*>(lds + line * LS + j * ES) + (h >> 1);
            float v[8], mx = 0.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int p = 8 * (h & 1) + i;
                v[i] = f[2 * p * M * ES];
                mx = fmaxf(mx, fabsf(v[i]));
            }
            mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
            mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
            const int e2 = mx > 0.f ? __builtin_amdgcn_frexp_expf(mx) : 0;   // mx in [2^(e2-1), 2^e2)
            half8_t b;
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = (_Float16)ldexpf(v[i], 15 - e2);
            const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
            const f32x4_t dre = __builtin_amdgcn_mfma_f32_16x16x32_f16(are, b, z, 0, 0, 0);
            const f32x4_t dim = __builtin_amdgcn_mfma_f32_16x16x32_f16(aim, b, z, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) outv[g][i] = make_float2(ldexpf(dre[i], e2 - 15), ldexpf(dim[i], e2 - 15));
        }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
        const int G = wave + g * W;
        if (GROUPS % W == 0 || G < GROUPS) {
            const int col = G * 16 + c16, line = col % L, j = col / L;
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[line * LS + (j * 16 + 4 * h + i) * ES] = outv[g][i];
        }
    }
}

// All stages of a length-N KIND-1 transform on an LDS tile, in place; ends
// with a barrier.  MFMA: radix-16 stage on the matrix cores (else the same
// stage as an FP32 radix-16 butterfly on the vector ALUs).  The last vector
// stage writes exactly the positions each thread read, so it needs no
// barrier between its reads and writes.
// SKIP_LAST: stop before the last stage (q16_last_stage_store runs it).
template <int N, int S, int L, int T, int LS, int ES, bool MFMA, bool SKIP_LAST = false>
__device__ __forceinline__ void q16_fft_lds(float2* lds, const float2* __restrict__ tw, int tid)
{
    using P = Plan1D<N, 1>;
    constexpr int K = SKIP_LAST ? P::stages - 1 : P::stages;
    static_assert(K >= 1, "at least one stage runs here");
    const LdsAcc<LS, ES> a{lds};
    // a stage needs the barrier between its reads and writes unless it is
    // the schedule's true last stage
    constexpr int KL = P::stages;
    if constexpr (MFMA) mfma_stage16<N, S, L, T, LS, ES>(lds, tid);
    else fft_stage_p<P, 0, S, L, T, true, (KL > 1)>(a, a, tw, tid);
    __syncthreads();
    if constexpr (K > 1) { fft_stage_p<P, 1, S, L, T, true, (KL > 2)>(a, a, tw, tid); __syncthreads(); }
    if constexpr (K > 2) { fft_stage_p<P, 2, S, L, T, true, (KL > 3)>(a, a, tw, tid); __syncthreads(); }
    if constexpr (K > 3) { fft_stage_p<P, 3, S, L, T, true, (KL > 4)>(a, a, tw, tid); __syncthreads(); }
    if constexpr (K > 4) { fft_stage_p<P, 4, S, L, T, true, false>(a, a, tw, tid); __syncthreads(); }
}

// Whether the last stage of a length-N KIND-1 transform over N lines can run
// with one wave per butterfly index j: the stage has N / R butterflies per
// line, so T / 64 == N / R waves each take all N lines (N / 64 per lane) of
// one j, and every output row j + q N / R lies inside one wave.
template <int N, int T>
constexpr bool q16_wave_rows()
{
    using P = Plan1D<N, 1>;
    return P::stages > 1 && N % 64 == 0 && T == 64 * (N / P::radix(P::stages - 1));
}

// Last stage of the transform along the tile's elements (lines = x, LDS
// address x + e * ES) with one wave per butterfly index, requantized
// straight from registers: output row r = element index, stored as scaled16
// at pay[r * rstride + x] with its exponent at ex[r * estride].  The same
// butterflies, twiddles, row maxima and roundings as running the stage in
// LDS and then q16_store_rows, without writing the tile back to LDS and
// reading it again (the compiler may contract a few multiply-adds
// differently, so single values can differ in the last place).  Used by
// both passes; the slab pass loads its tile with 32-bit offsets
// (Q16Regs::load<true>), which frees the registers this stage needs.
template <int N, int S, int T, int ES, int FMT>
__device__ __forceinline__ void q16_last_stage_store(const float2* lds, const float2* __restrict__ tw,
                                                     unsigned* pay, int rstride, signed char* ex, int estride,
                                                     int tid)
{
    using P = Plan1D<N, 1>;
    constexpr int ST = P::stages - 1, R = P::radix(ST), NS = P::ns(ST), M = N / R, IT = N / 64;
    static_assert(q16_wave_rows<N, T>() && NS == M, "one wave per butterfly index of the last stage");
    const int lane = tid & 63;
    const int j = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float2* __restrict__ w = tw + P::tw_off(ST) + (j % NS) * (R - 1);
    float2 v[IT][R];
    float m[R];
#pragma unroll
    for (int q = 0; q < R; ++q) m[q] = 0.f;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int x = lane + 64 * it;
#pragma unroll
        for (int q = 0; q < R; ++q) v[it][q] = lds[x + (j + q * M) * ES];
#pragma unroll
        for (int q = 1; q < R; ++q) v[it][q] = cmul(v[it][q], w[q - 1]);
        dft<R, S>(v[it]);
#pragma unroll
        for (int q = 0; q < R; ++q) m[q] = absmax(m[q], v[it][q]);
    }
    unsigned mb[R], wm[R];
#pragma unroll
    for (int q = 0; q < R; ++q) mb[q] = fbits(m[q]);
    if constexpr (R == 4 || R == 8) {
        wavemax_many<R>(mb, wm);
    } else {
#pragma unroll
        for (int q = 0; q < R; ++q) wm[q] = wavemax(mb[q]);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = j + q * NS, e = row_exponent_bits(wm[q]);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int x = lane + 64 * it;
            pay[(unsigned)(r * rstride + x)] = enc16x2<FMT>(ldexpf(v[it][q].x, -e), ldexpf(v[it][q].y, -e));
        }
        if (lane == 0) ex[(unsigned)(r * estride)] = (signed char)e;
    }
}

// A tile's input held for the first stage of the transform across its rows
// straight from registers: thread (x = tid % N, j = tid / N) holds the 16
// inputs e = j + q N/16 (q < 16) of its radix-16 butterfly of column x,
// one scaled16 word each (lanes along x: every load instruction reads whole
// rows), and the row exponents.  Row e starts RSTRIDE words and its
// exponent ESTRIDE bytes after row 0 (slab pass: rows z of an xz-slab, N*N
// and N; plane pass: rows y of an xy-plane, N and 1).  When N is a multiple
// of 64 a wave shares j, so lane q < 16 loads the exponent of row
// j + q N/16 and the others are taken from it with readlane; otherwise
// every thread loads its 16 exponents.  Offsets are 32-bit from the tile's
// base (a tile spans < 2^32 elements).  Threads from N N/16 on (T is
// rounded up to whole waves) hold nothing.
template <int N, int T, int RSTRIDE = N * N, int ESTRIDE = N>
struct Q16ColRegs {
    static constexpr int M0 = N / 16, NB = N * M0;
    static_assert(T >= NB && (N % 64 != 0 || T == NB), "one first-stage butterfly per thread");
    static constexpr bool WAVE_J = N % 64 == 0;
    unsigned u[16];
    int e[WAVE_J ? 1 : 4];   // else the 16 exponents as bytes, four per word
    // NT: streaming payload loads (see stream_plane)
    template <bool NT = false>
    __device__ __forceinline__ void load(const unsigned* pay, const signed char* ex, int tid)
    {
        if (NB < T && tid >= NB) return;
        const int x = tid % N, j = tid / N;
        if constexpr (WAVE_J) {
            // row addresses in scalar registers, the lane offset x in a vector one
            // (a 32-bit byte offset, so that the load takes the scalar base + vector offset form)
            const int js = __builtin_amdgcn_readfirstlane(j);
            const unsigned bx = 4u * (unsigned)x;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const char* row = reinterpret_cast<const char*>(pay + (unsigned)((js + M0 * q) * RSTRIDE));
                const unsigned* a = reinterpret_cast<const unsigned*>(row + bx);
                if constexpr (NT) u[q] = __builtin_nontemporal_load(a);
                else u[q] = *a;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if constexpr (NT) u[q] = __builtin_nontemporal_load(pay + (unsigned)((j + M0 * q) * RSTRIDE + x));
                else u[q] = pay[(unsigned)((j + M0 * q) * RSTRIDE + x)];
            }
        }
        if constexpr (WAVE_J) {
            const int lane = tid & 63;
            e[0] = lane < 16 ? (int)ex[(unsigned)((j + M0 * lane) * ESTRIDE)] : 0;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) e[k] = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                e[q >> 2] |= ((int)(unsigned char)ex[(unsigned)((j + M0 * q) * ESTRIDE)]) << (8 * (q & 3));
        }
    }
    template <int FMT>
    __device__ __forceinline__ float2 value(int q) const
    {
        int eq;
        if constexpr (WAVE_J) eq = __builtin_amdgcn_readlane(e[0], q);
        else eq = (int)(signed char)(e[q >> 2] >> (8 * (q & 3)));
        return make_float2(ldexpf(dec16<FMT>(u[q] & 0xFFFFu), eq), ldexpf(dec16<FMT>(u[q] >> 16), eq));
    }
    // Stage 0 of the KIND-1 schedule (radix 16, no twiddles) on the held
    // values, written to the LDS tile (lines = x, element stride ES) in the
    // stage's Stockham output order: element 16 j + q.
    template <int S, int ES, int FMT>
    __device__ __forceinline__ void stage0_to_lds(float2* lds, int tid) const
    {
        if (NB < T && tid >= NB) return;
        const int x = tid % N, j = tid / N;
        float2 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = value<FMT>(q);
        dft<16, S>(v);
#pragma unroll
        for (int q = 0; q < 16; ++q) lds[x + (16 * j + q) * ES] = v[q];
    }
};

// 2^d as an FP32 value for -126 <= d <= 127, from its bit pattern (exact;
// wave-uniform callers compute it on the scalar unit without branches).
__device__ __forceinline__ float pow2f(int d) { return __builtin_bit_cast(float, (unsigned)(d + 127) << 23); }

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf16x4_bits_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// The same first stage (radix 16 across the tile's rows, from registers) on
// the matrix cores, straight from the binary16 payloads.  With x_q = h_q
// 2^(e_q) the 16 inputs of butterfly j (payload h_q, row exponent e_q of
// row j + M0 q),
//   X_f = sum_q W^(f q) x_q = 2^E sum_q (W^(f q) 2^(e_q - E)) h_q,
// E the largest exponent of the rows that are not all zero: the row
// exponents fold into the DFT matrix (entries at most 1 in size, rounded to
// binary16) and the payloads, as loaded, are the other operand.  An all-zero
// row's exponent (0 by the storage rule) says nothing about its scale, so
// it is left out of E and its matrix columns are 0.
// v_mfma_f32_32x32x8_f16 takes 32 lines at a time: B (8 x 32) is 4
// payload halves per lane, A (32 x 8) stacks the real-output rows 0-15 over
// the imaginary-output rows 16-31, and four instructions accumulate the 32
// real inputs (16 rows, re and im).  Lane l: line n = l % 32 of the block,
// K half kb = l / 32; in instruction kk it holds rows q = 4 kk + 2 kb + t
// (t < 2), one payload word (re, im) each, and the matching A entries for
// output row l % 32; its results are frequencies f = 4 kb + c and
// 8 + 4 kb + c (c < 4) of line n.  A wave takes one butterfly index j and 64
// lines (two blocks).  Same layout conventions and interface as Q16ColRegs.
// bfloat16 payloads (PF = kFmtBF16) go to v_mfma_f32_32x32x8_bf16 as loaded
// (same operand layout); the matrix is then the sum of two bfloat16
// matrices, its entries rounded to bfloat16 and the remainders rounded
// again (about 16 significant bits, more than the binary16 matrix's 11),
// and each product pair accumulates both.  The remainders depend on the
// lane only; they sit in a 2 KB LDS table (kMfmaLoWords words, filled by
// wave 0 in init, read after the caller's next barrier) rather than in 8
// more registers per lane.
constexpr int kMfmaLoWords = 8 * 64;

template <int N, int T, int RSTRIDE = N * N, int ESTRIDE = N, int PF = kFmtF16>
struct Q16MfmaCols {
    static constexpr int M0 = N / 16, WPJ = N / 64;
    static_assert(N % 64 == 0 && T == N * M0, "a wave per butterfly index and 64 lines");
    unsigned u[2][4][2];   // [line block][kk][t]
    int ev;                // lane q < 16: exponent of row j + M0 q
    unsigned ab[4][2];     // A entries before scaling: 16-bit (re-input, im-input) pairs in the payload format
    const unsigned* lo;    // bfloat16 payloads: the entries' remainders, word (2 kk + t) * 64 + lane

    // lo_tab: kMfmaLoWords words of LDS (bfloat16 payloads only)
    template <int S>
    __device__ __forceinline__ void init(int tid, unsigned* lo_tab = nullptr)
    {
        lo = lo_tab;
        const int lane = tid & 63, m = lane & 31, kb = lane >> 5, f = m & 15;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int th = (f * (4 * kk + 2 * kb + t)) & 15;
                const float c = cos16(th), s = (S > 0 ? 1.f : -1.f) * sin16(th);
                const float v0 = m < 16 ? c : s, v1 = m < 16 ? -s : c;
                if constexpr (PF == kFmtF16) {
                    ab[kk][t] = enc16x2<kFmtF16>(v0, v1);
                } else {
                    const unsigned hi = enc16x2<kFmtBF16>(v0, v1);
                    ab[kk][t] = hi;
                    if (tid < 64)
                        lo_tab[(2 * kk + t) * 64 + lane] =
                            enc16x2<kFmtBF16>(v0 - __builtin_bit_cast(float, hi << 16),
                                              v1 - __builtin_bit_cast(float, hi & 0xFFFF0000u));
                }
            }
    }
    template <bool NT = false>
    __device__ __forceinline__ void load(const unsigned* pay, const signed char* ex, int tid)
    {
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        const int j = w / WPJ, x = 64 * (w % WPJ) + (lane & 31), kb = lane >> 5;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const unsigned* p = pay + (unsigned)((j + M0 * (4 * kk + 2 * kb + t)) * RSTRIDE + x + 32 * b);
                    if constexpr (NT) u[b][kk][t] = __builtin_nontemporal_load(p);
                    else u[b][kk][t] = *p;
                }
        ev = lane < 16 ? (int)ex[(unsigned)((j + M0 * lane) * ESTRIDE)] : 0;
    }
    template <int S, int ES, int FMT>
    __device__ __forceinline__ void stage0_to_lds(float2* lds, int tid) const
    {
        static_assert(FMT == PF, "the payload format the matrix was built for");
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        const int j = w / WPJ, x = 64 * (w % WPJ) + (lane & 31), kb = lane >> 5;
        // which rows hold a nonzero value on this wave's 64 lines (either sign of zero counts as zero)
        bool nz[16];
        int e[16];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const unsigned long long m =
                    __builtin_amdgcn_ballot_w64(((u[0][kk][t] | u[1][kk][t]) & 0x7FFF7FFFu) != 0u);
                nz[4 * kk + t] = (unsigned)m != 0u;
                nz[4 * kk + 2 + t] = (unsigned)(m >> 32) != 0u;
            }
        // an all-zero row takes exponent -1000: it never sets E, and its
        // scale 2^(-1000 - E) is 0
        int E = -1000;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int eq = __builtin_amdgcn_readlane(ev, q);
            e[q] = nz[q] ? eq : -1000;
            E = e[q] > E ? e[q] : E;
        }
        half4_t a[4];
        unsigned ah[4][2], al[4][2];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int q0 = 4 * kk + t, q1 = q0 + 2;
                const int d0 = e[q0] - E, d1 = e[q1] - E;
                const int d = kb ? d1 : d0;
                if constexpr (PF == kFmtF16) {
                    // 2^(e_q - E) (0 for an all-zero row), rounded to binary16 in
                    // both halves by one packed conversion: subnormal or 0 far below E
                    const float sc = kb ? pow2f(d1 < -100 ? -100 : d1) : pow2f(d0 < -100 ? -100 : d0);
                    const f16x2_t v = __builtin_bit_cast(f16x2_t, ab[kk][t]) *
                                      __builtin_convertvector(f32x2_t{sc, sc}, f16x2_t);
                    a[kk][2 * t] = v[0];
                    a[kk][2 * t + 1] = v[1];
                } else {
                    // 2^(e_q - E), exact in bfloat16; 0 for an all-zero row and
                    // below 2^-100 (far under FP32 rounding of the sum)
                    const float sc = d < -100 ? 0.f : pow2f(d < -100 ? -100 : d);
                    const unsigned h = ab[kk][t], l = lo[(2 * kk + t) * 64 + lane];
                    ah[kk][t] = enc16x2<kFmtBF16>(sc * __builtin_bit_cast(float, h << 16),
                                                  sc * __builtin_bit_cast(float, h & 0xFFFF0000u));
                    al[kk][t] = enc16x2<kFmtBF16>(sc * __builtin_bit_cast(float, l << 16),
                                                  sc * __builtin_bit_cast(float, l & 0xFFFF0000u));
                }
            }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            f32x16_t acc = {};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const unsigned w2[2] = {u[b][kk][0], u[b][kk][1]};
                if constexpr (PF == kFmtF16) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x8f16(a[kk], __builtin_bit_cast(half4_t, w2), acc, 0, 0, 0);
                } else {
                    const bf16x4_bits_t bv = __builtin_bit_cast(bf16x4_bits_t, w2);
                    const unsigned h2[2] = {ah[kk][0], ah[kk][1]}, l2[2] = {al[kk][0], al[kk][1]};
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4_bits_t, h2), bv, acc, 0,
                                                                   0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(bf16x4_bits_t, l2), bv, acc, 0,
                                                                   0, 0);
                }
            }
            const int xb = x + 32 * b;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                lds[xb + (16 * j + 4 * kb + c) * ES] = make_float2(ldexpf(acc[c], E), ldexpf(acc[8 + c], E));
                lds[xb + (16 * j + 8 + 4 * kb + c) * ES] = make_float2(ldexpf(acc[4 + c], E), ldexpf(acc[12 + c], E));
            }
        }
    }
};

// Whether the first stage along the rows runs on the matrix cores from the
// payloads (Q16MfmaCols) for this length and payload format.
template <int N, int FMT>
constexpr bool q16_mfma_cols(int T)
{
    return (FMT == kFmtF16 || FMT == kFmtBF16) && N % 64 == 0 && Plan1D<N, 1>::stages == 2 && T == N * (N / 16);
}

// Last stage of the transform along the rows of an LDS tile (lines = rows,
// row stride RS, elements contiguous), requantized straight from registers
// row by row: output row r is stored as scaled16 at pay[r * N + x] with its
// exponent at ex[r].  The stage is the last of a two-stage KIND-1 schedule
// (radix 16, then R = N / 16), so every row has 16 butterflies; 16
// consecutive lanes take the 16 butterflies of one row, find the row
// maximum with a 16-lane reduction and store their R values each.  The
// stage writes the positions it read, so no LDS barrier precedes it beyond
// the one after the previous stage.
template <int N, int S, int T, int RS, int FMT>
__device__ __forceinline__ void q16_row_last_stage_store(const float2* lds, const float2* __restrict__ tw,
                                                         unsigned* pay, signed char* ex, int tid)
{
    using P = Plan1D<N, 1>;
    constexpr int ST = P::stages - 1, R = P::radix(ST), NS = P::ns(ST), M = N / R;
    static_assert(P::stages == 2 && M == 16 && NS == 16, "a radix-16 stage then the last stage");
    static_assert(T % 64 == 0, "row groups of 16 lanes stay inside waves");
    constexpr int NB = N * M, IT = (NB + T - 1) / T;
    const float2* __restrict__ tws = tw + P::tw_off(ST);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * T;
        const int j = b % M, row = b / M;
        const bool live = NB % T == 0 || b < NB;   // uniform per 16-lane group
        float2 v[R];
        float m = 0.f;
        if (live) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[q] = lds[row * RS + j + q * M];
            const float2* __restrict__ w = tws + j * (R - 1);
#pragma unroll
            for (int q = 1; q < R; ++q) v[q] = cmul(v[q], w[q - 1]);
            dft<R, S>(v);
#pragma unroll
            for (int q = 0; q < R; ++q) m = absmax(m, v[q]);
        }
        const unsigned mr = rowmax16(fbits(m));
        if (live) {
            const int e = row_exponent_bits(mr);
#pragma unroll
            for (int q = 0; q < R; ++q)
                pay[(unsigned)(row * N + j + q * M)] = enc16x2<FMT>(ldexpf(v[q].x, -e), ldexpf(v[q].y, -e));
            if (j == 0) ex[(unsigned)row] = (signed char)e;
        }
    }
}

// Pass A: planes p = b * N + z, persistent over `planes` with the next plane
// prefetched into registers.  Rows of the input (b, z, y) -> rows of the FP16
// intermediate (b, z, ky).  NT: streaming input loads.
template <int N, int S, int FMT_IN, bool MFMA, bool NT = false>
__global__ void __launch_bounds__(Q16Geom<N>::T)
k_q16_plane(const unsigned* in_pay, const signed char* in_exp, unsigned* mid_pay, signed char* mid_exp,
            const float2* __restrict__ tw, long planes)
{
    using G = Q16Geom<N>;
    constexpr int T = G::T, RS = G::RS;
    __shared__ float2 lds[G::WORDS];
    __shared__ int lds_e[N];
    const int tid = threadIdx.x;
    long p = blockIdx.x;
    constexpr bool MC = MFMA && q16_mfma_cols<N, FMT_IN>(T);
    if constexpr ((!MFMA || MC) && Plan1D<N, 1>::stages == 2) {
        // y transform first, its radix-16 stage straight from the loaded
        // registers (on the matrix cores with the MFMA engine); x transform
        // last, requantized row by row from registers: three LDS sweeps and
        // four barriers per plane instead of four and seven (the same DFT;
        // rounding differs from the x-first order only at FP32 level).
        using CR = typename std::conditional<MC, Q16MfmaCols<N, T, N, 1, FMT_IN>, Q16ColRegs<N, T, N, 1>>::type;
        CR cr;
        if constexpr (MC && FMT_IN == kFmtBF16) {
            __shared__ unsigned lo_tab[kMfmaLoWords];
            cr.template init<S>(tid, lo_tab);
            __syncthreads();
        } else if constexpr (MC) {
            cr.template init<S>(tid);
        }
        if (p < planes) cr.template load<NT>(in_pay + p * N * N, in_exp + p * N, tid);
        for (; p < planes; p += gridDim.x) {
            cr.template stage0_to_lds<S, RS, FMT_IN>(lds, tid);   // y stage 0: lines = x
            const long pn = p + gridDim.x;
            if (pn < planes) cr.template load<NT>(in_pay + pn * N * N, in_exp + pn * N, tid);
            __syncthreads();
            {
                const LdsAcc<1, RS> a{lds};                       // y stage 1 (the last of y), in place
                fft_stage_p<Plan1D<N, 1>, 1, S, N, T, true, false>(a, a, tw, tid);
            }
            __syncthreads();
            {
                const LdsAcc<RS, 1> a{lds};                       // x stage 0: lines = rows
                fft_stage_p<Plan1D<N, 1>, 0, S, N, T, true, true>(a, a, tw, tid);
            }
            __syncthreads();
            q16_row_last_stage_store<N, S, T, RS, kFmtF16>(lds, tw, mid_pay + p * N * N, mid_exp + p * N, tid);
            __syncthreads();   // the tile is read before the next plane's stage 0 writes it
        }
        return;
    }
    Q16Regs<N, N, T> regs;
    if (p < planes) regs.template load<false, NT>(in_pay + p * N * N, N, in_exp + p * N, 1, tid);
    for (; p < planes; p += gridDim.x) {
        regs.put_exponent(lds_e, tid);
        __syncthreads();   // exponents visible; the previous plane is done with the tile
        regs.template to_lds<RS, FMT_IN>(lds, lds_e, tid);
        const long pn = p + gridDim.x;
        if (pn < planes) regs.template load<false, NT>(in_pay + pn * N * N, N, in_exp + pn * N, 1, tid);
        __syncthreads();
        q16_fft_lds<N, S, N, T, RS, 1, MFMA>(lds, tw, tid);   // x: lines = rows
        if constexpr (q16_wave_rows<N, T>()) {                // y: lines = columns
            q16_fft_lds<N, S, N, T, 1, RS, MFMA, true>(lds, tw, tid);
            q16_last_stage_store<N, S, T, RS, kFmtF16>(lds, tw, mid_pay + p * N * N, N, mid_exp + p * N, 1, tid);
        } else {
            q16_fft_lds<N, S, N, T, 1, RS, MFMA>(lds, tw, tid);
            q16_store_rows<N, N, RS, T, kFmtF16>(lds, mid_pay + p * N * N, N, mid_exp + p * N, 1, tid);
        }
    }
}

// Pass B: slabs s = b * N + y, persistent likewise; rows (b, z, y) of the
// intermediate for all z -> rows (b, kz, y) of the output.
template <int N, int S, int FMT_OUT, bool MFMA>
__global__ void __launch_bounds__(Q16Geom<N>::T)
k_q16_slab(const unsigned* mid_pay, const signed char* mid_exp, unsigned* out_pay, signed char* out_exp,
           const float2* __restrict__ tw, long slabs)
{
    using G = Q16Geom<N>;
    constexpr int T = G::T, RS = G::RS;
    __shared__ float2 lds[G::WORDS];
    __shared__ int lds_e[N];
    const int tid = threadIdx.x;
    Q16Regs<N, N, T> regs;
    // row index of (b, z = 0, y) of the k-th slab taken, rows of successive
    // z N apart; slabs are taken in reverse (b, y) order, so the pass begins
    // with the planes the plane pass wrote last (still in the caches)
    auto row0 = [slabs](long k) {
        const long s = slabs - 1 - k;
        return (s / N) * N * N + (s % N);
    };
    long s = blockIdx.x;
    constexpr bool MC = MFMA && q16_mfma_cols<N, kFmtF16>(T);
    if constexpr ((!MFMA || MC) && Plan1D<N, 1>::stages == 2) {
        // First z stage straight from the loaded registers (on the matrix
        // cores with the MFMA engine): one LDS write, one barrier, then the
        // last stage (one LDS sweep and a barrier fewer per slab than
        // staging the dequantized slab through LDS).
        using CR = typename std::conditional<MC, Q16MfmaCols<N, T>, Q16ColRegs<N, T>>::type;
        CR cr;
        if constexpr (MC) cr.template init<S>(tid);
        if (s < slabs) cr.load(mid_pay + row0(s) * N, mid_exp + row0(s), tid);
        for (; s < slabs; s += gridDim.x) {
            cr.template stage0_to_lds<S, RS, kFmtF16>(lds, tid);
            const long sn = s + gridDim.x;
            if (sn < slabs) cr.load(mid_pay + row0(sn) * N, mid_exp + row0(sn), tid);
            __syncthreads();
            if constexpr (q16_wave_rows<N, T>()) {
                q16_last_stage_store<N, S, T, RS, FMT_OUT>(lds, tw, out_pay + row0(s) * N, N * N, out_exp + row0(s),
                                                           N, tid);
            } else {
                const LdsAcc<1, RS> a{lds};
                fft_stage_p<Plan1D<N, 1>, 1, S, N, T, true, false>(a, a, tw, tid);
                __syncthreads();
                q16_store_rows<N, N, RS, T, FMT_OUT>(lds, out_pay + row0(s) * N, (long)N * N, out_exp + row0(s), N,
                                                     tid);
            }
            __syncthreads();   // the tile is read before the next slab's stage 0 writes it
        }
        return;
    }
    if (s < slabs) regs.template load<true>(mid_pay + row0(s) * N, (long)N * N, mid_exp + row0(s), N, tid);
    for (; s < slabs; s += gridDim.x) {
        regs.put_exponent(lds_e, tid);
        __syncthreads();
        regs.template to_lds<RS, kFmtF16>(lds, lds_e, tid);
        const long sn = s + gridDim.x;
        if (sn < slabs) regs.template load<true>(mid_pay + row0(sn) * N, (long)N * N, mid_exp + row0(sn), N, tid);
        __syncthreads();
        // z: lines = x, elements along z (LDS rows)
        if constexpr (q16_wave_rows<N, T>()) {
            q16_fft_lds<N, S, N, T, 1, RS, MFMA, true>(lds, tw, tid);
            q16_last_stage_store<N, S, T, RS, FMT_OUT>(lds, tw, out_pay + row0(s) * N, N * N, out_exp + row0(s), N,
                                                       tid);
        } else {
            q16_fft_lds<N, S, N, T, 1, RS, MFMA>(lds, tw, tid);
            q16_store_rows<N, N, RS, T, FMT_OUT>(lds, out_pay + row0(s) * N, (long)N * N, out_exp + row0(s), N,
                                                 tid);
        }
    }
}

// Standalone conversions (fft3d_quantize / fft3d_dequantize): one wave per
// row of C values; rows of FP32 complex in, scaled16 out, and back.
template <int FMT>
__global__ void __launch_bounds__(256) k_q16_quantize(const float2* in, long rows, int C, unsigned* pay,
                                                      signed char* ex)
{
    const int lane = threadIdx.x & 63;
    const long r = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const float2* row = in + r * C;
    float m = 0.f;
    for (int x = lane; x < C; x += 64) m = absmax(m, row[x]);
    const int e = row_exponent_bits(wavemax(fbits(m)));
    for (int x = lane; x < C; x += 64) pay[r * C + x] = enc16x2<FMT>(ldexpf(row[x].x, -e), ldexpf(row[x].y, -e));
    if (lane == 0) ex[r] = (signed char)e;
}

template <int FMT>
__global__ void __launch_bounds__(256) k_q16_dequantize(const unsigned* pay, const signed char* ex, long rows, int C,
                                                        float2* out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * C) return;
    const int e = ex[i / C];
    const unsigned u = pay[i];
    out[i] = make_float2(ldexpf(dec16<FMT>(u & 0xFFFFu), e), ldexpf(dec16<FMT>(u >> 16), e));
}

}  // namespace fft3d
