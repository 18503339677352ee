/*
 * FP64 CPU oracle for the complex-to-complex 3D DFT and the forms built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it (through oracle/__init__.py).  It shares no
 * code, header, table or constant with the GPU implementation.
 *
 * What it computes (paper: "Efficient Ab-Initio Molecular Dynamic Simulations
 * by Offloading Fast Fourier Transformations to FPGAs", Ramaswami et al.):
 *
 *   * Eq. (1), Section II: F(kx,ky,kz) = sum_{z,y,x} f(x,y,z) W^{x kx} W^{y ky}
 *     W^{z kz} with W_N = exp(-2 pi i / N) per dimension, no normalisation.
 *     The sign of the exponent is a parameter: -1 is Eq. (1) itself, +1 is the
 *     unnormalised inverse (the paper does not define an inverse; the reading
 *     used everywhere in this project is "opposite sign, no scaling", so
 *     inverse(forward(f)) = Nx*Ny*Nz*f).
 *   * dft3d_naive: Eq. (1) written out term by term, O((NxNyNz)^2).
 *   * fft3d: the decomposition stated in Section II -- 1D transforms along x,
 *     then y, then z -- where each 1D transform is a recursive mixed-radix
 *     decimation-in-time FFT taking factors 5, then 3, then 2.
 *
 * Layout everywhere: C order [batch][z][y][x], x contiguous, each complex
 * value stored as (re, im) doubles.  Roots of unity are evaluated with cos/sin
 * in double on an index already reduced modulo N, so no large argument ever
 * reaches cos/sin.
 *
 * Real-grid transforms (r2c / c2r), the scaled 16-bit storage format and the
 * plane-wave local-potential energy are the other forms this project builds
 * on top of the transform; they
 * are defined here from their plain definitions (see the comments on each
 * function).  All rounding to 16-bit formats is written out from the IEEE
 * definitions of binary16 and bfloat16 (round to nearest, ties to even).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Roots of unity                                                            */
/* ------------------------------------------------------------------------ */

/* w[2e], w[2e+1] = cos(2 pi e / n), sign * sin(2 pi e / n) for e in [0, n). */
static void root_table(int n, int sign, double *w)
{
    for (int e = 0; e < n; ++e) {
        double a = 2.0 * M_PI * (double)e / (double)n;
        w[2 * e] = cos(a);
        w[2 * e + 1] = (double)sign * sin(a);
    }
}

/* ------------------------------------------------------------------------ */
/* O1: Eq. (1) term by term                                                  */
/* ------------------------------------------------------------------------ */

int oracle_dft3d_naive(int nx, int ny, int nz, int batch, int sign,
                       const double *in, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1 || (sign != 1 && sign != -1))
        return -1;
    double *wx = malloc(sizeof(double) * 2 * nx);
    double *wy = malloc(sizeof(double) * 2 * ny);
    double *wz = malloc(sizeof(double) * 2 * nz);
    if (!wx || !wy || !wz) { free(wx); free(wy); free(wz); return -4; }
    root_table(nx, sign, wx);
    root_table(ny, sign, wy);
    root_table(nz, sign, wz);
    const long vol = (long)nx * ny * nz;
    for (int b = 0; b < batch; ++b) {
        const double *f = in + 2 * vol * b;
        double *F = out + 2 * vol * b;
#pragma omp parallel for collapse(2) schedule(static)
        for (int kz = 0; kz < nz; ++kz)
            for (int ky = 0; ky < ny; ++ky)
                for (int kx = 0; kx < nx; ++kx) {
                    double re = 0.0, im = 0.0;
                    for (int z = 0; z < nz; ++z) {
                        const double *a = wz + 2 * (((long)z * kz) % nz);
                        for (int y = 0; y < ny; ++y) {
                            const double *c = wy + 2 * (((long)y * ky) % ny);
                            /* W_z^{z kz} * W_y^{y ky} */
                            double pr = a[0] * c[0] - a[1] * c[1];
                            double pi = a[0] * c[1] + a[1] * c[0];
                            for (int x = 0; x < nx; ++x) {
                                const double *d = wx + 2 * (((long)x * kx) % nx);
                                double tr = pr * d[0] - pi * d[1];
                                double ti = pr * d[1] + pi * d[0];
                                long i = ((long)z * ny + y) * nx + x;
                                double fr = f[2 * i], fi = f[2 * i + 1];
                                re += fr * tr - fi * ti;
                                im += fr * ti + fi * tr;
                            }
                        }
                    }
                    long o = ((long)kz * ny + ky) * nx + kx;
                    F[2 * o] = re;
                    F[2 * o + 1] = im;
                }
    }
    free(wx); free(wy); free(wz);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2: recursive mixed-radix FFT (decimation in time)                        */
/* ------------------------------------------------------------------------ */

/* Factor taken at each level: 5, then 3, then 2; any other prime factor is
 * handled by the same combine step (which is then a plain DFT of that size). */
static int pick_factor(int n)
{
    if (n % 5 == 0) return 5;
    if (n % 3 == 0) return 3;
    if (n % 2 == 0) return 2;
    for (int p = 7; (long)p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/*
 * X[0..n) = DFT_n of x[0], x[xs], x[2 xs], ... (complex, interleaved).
 * w is the root table of the top-level length N; W_n^e = W_N^{e N/n}.
 *
 * With n = p m and x_q[j] = x[q + p j]:
 *   Y_q = DFT_m(x_q),   X[k + s m] = sum_q W_n^{q (k + s m)} Y_q[k].
 * Y_q is written to X[q m .. q m + m); for a fixed k the p values Y_q[k] and
 * the p outputs X[k + s m] occupy the same p slots, so the combine is done in
 * place one k at a time.
 */
static void fft_rec(int n, int N, const double *w, const double *x, long xs,
                    double *X, double *t)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    int p = pick_factor(n), m = n / p;
    for (int q = 0; q < p; ++q)
        fft_rec(m, N, w, x + 2 * (long)q * xs, xs * p, X + 2 * (long)q * m, t);
    const long step = N / n;
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) {
            t[2 * q] = X[2 * ((long)q * m + k)];
            t[2 * q + 1] = X[2 * ((long)q * m + k) + 1];
        }
        for (int s = 0; s < p; ++s) {
            long kk = k + (long)s * m;
            double re = 0.0, im = 0.0;
            for (int q = 0; q < p; ++q) {
                long e = ((long)q * kk) % n;
                const double *c = w + 2 * (e * step);
                re += t[2 * q] * c[0] - t[2 * q + 1] * c[1];
                im += t[2 * q] * c[1] + t[2 * q + 1] * c[0];
            }
            X[2 * kk] = re;
            X[2 * kk + 1] = im;
        }
    }
}

int oracle_fft1d(int n, int sign, const double *in, double *out)
{
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    double *w = malloc(sizeof(double) * 2 * n);
    double *t = malloc(sizeof(double) * 2 * n);
    if (!w || !t) { free(w); free(t); return -4; }
    root_table(n, sign, w);
    fft_rec(n, n, w, in, 1, out, t);
    free(w); free(t);
    return 0;
}

/* One batched 1D pass along `axis` (0 = x, 1 = y, 2 = z), in place on a. */
static int axis_pass(int nx, int ny, int nz, int batch, int sign, int axis,
                     double *a)
{
    const int dims[3] = {nx, ny, nz};
    const int n = dims[axis];
    const long stride = axis == 0 ? 1 : (axis == 1 ? (long)nx : (long)nx * ny);
    const long vol = (long)nx * ny * nz;
    const long per = vol / n;             /* pencils per batch member */
    const long total = per * batch;
    double *w = malloc(sizeof(double) * 2 * n);
    if (!w) return -4;
    root_table(n, sign, w);
    int err = 0;
#pragma omp parallel
    {
        double *buf = malloc(sizeof(double) * 6 * n);
        if (!buf) {
#pragma omp atomic write
            err = -4;
        } else {
            double *pin = buf, *pout = buf + 2 * n, *tmp = buf + 4 * n;
#pragma omp for schedule(static)
            for (long pc = 0; pc < total; ++pc) {
                long b = pc / per, r = pc % per, base;
                if (axis == 0) {            /* r enumerates (z, y) */
                    base = r * nx;
                } else if (axis == 1) {     /* r enumerates (z, x) */
                    long z = r / nx, x = r % nx;
                    base = z * (long)nx * ny + x;
                } else {                    /* r enumerates (y, x) */
                    base = r;
                }
                double *pen = a + 2 * (b * vol + base);
                for (int i = 0; i < n; ++i) {
                    pin[2 * i] = pen[2 * i * stride];
                    pin[2 * i + 1] = pen[2 * i * stride + 1];
                }
                fft_rec(n, n, w, pin, 1, pout, tmp);
                for (int i = 0; i < n; ++i) {
                    pen[2 * i * stride] = pout[2 * i];
                    pen[2 * i * stride + 1] = pout[2 * i + 1];
                }
            }
            free(buf);
        }
    }
    free(w);
    return err;
}

/* Separable 3D transform with the 1D passes applied in the given axis order
 * (order = {0,1,2} is x, then y, then z, as Section II states it). */
int oracle_fft3d_order(int nx, int ny, int nz, int batch, int sign,
                       const double *in, double *out, const int *order)
{
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1 || (sign != 1 && sign != -1))
        return -1;
    int seen = 0;
    for (int i = 0; i < 3; ++i) {
        if (order[i] < 0 || order[i] > 2) return -1;
        seen |= 1 << order[i];
    }
    if (seen != 7) return -1;
    const long vol = (long)nx * ny * nz;
    if (out != in) memcpy(out, in, sizeof(double) * 2 * vol * batch);
    for (int i = 0; i < 3; ++i) {
        int err = axis_pass(nx, ny, nz, batch, sign, order[i], out);
        if (err) return err;
    }
    return 0;
}

int oracle_fft3d(int nx, int ny, int nz, int batch, int sign,
                 const double *in, double *out)
{
    static const int xyz[3] = {0, 1, 2};
    return oracle_fft3d_order(nx, ny, nz, batch, sign, in, out, xyz);
}

/* ------------------------------------------------------------------------ */
/* Real grids (densities and potentials are real)                            */
/* ------------------------------------------------------------------------ */

/*
 * r2c: Eq. (1) of a real grid f (imaginary parts zero), sign -1, keeping the
 * half kx = 0 .. nx/2 of the x frequencies; the other half follows from
 * F(-k) = conj F(k).  in: real [batch][z][y][x]; out: complex
 * [batch][z][y][nx/2 + 1].  nx must be even.
 */
int oracle_r2c3d(int nx, int ny, int nz, int batch, const double *in, double *out)
{
    if (nx < 2 || nx % 2 || ny < 1 || nz < 1 || batch < 1) return -1;
    const long vol = (long)nx * ny * nz, rows = (long)ny * nz * batch;
    const int h = nx / 2 + 1;
    double *full = malloc(sizeof(double) * 2 * vol * batch);
    if (!full) return -4;
    for (long i = 0; i < vol * batch; ++i) {
        full[2 * i] = in[i];
        full[2 * i + 1] = 0.0;
    }
    int err = oracle_fft3d(nx, ny, nz, batch, -1, full, full);
    if (!err)
        for (long r = 0; r < rows; ++r)
            for (int k = 0; k < h; ++k) {
                out[2 * (r * h + k)] = full[2 * (r * nx + k)];
                out[2 * (r * h + k) + 1] = full[2 * (r * nx + k) + 1];
            }
    free(full);
    return err;
}

/*
 * c2r: the unnormalised inverse of a half spectrum H [batch][z][y][nx/2 + 1]
 * (the inverse of its Hermitian extension, the sign +1 form of Eq. (1)):
 * complex inverse transforms along z and y, then along x the real sum
 *   f(x) = Re H_0 + (-1)^x Re H_{nx/2}
 *          + 2 sum_{0 < k < nx/2} (Re H_k cos(2 pi k x / nx) - Im H_k sin(2 pi k x / nx)),
 * so the imaginary parts of the kx = 0 and kx = nx/2 entries do not
 * contribute.  out: real [batch][z][y][x].  nx must be even.
 */
int oracle_c2r3d(int nx, int ny, int nz, int batch, const double *in, double *out)
{
    if (nx < 2 || nx % 2 || ny < 1 || nz < 1 || batch < 1) return -1;
    const int h = nx / 2 + 1;
    const long hvol = (long)h * ny * nz, rows = (long)ny * nz * batch;
    double *t = malloc(sizeof(double) * 2 * hvol * batch);
    double *w = malloc(sizeof(double) * 2 * nx);
    if (!t || !w) {
        free(t);
        free(w);
        return -4;
    }
    memcpy(t, in, sizeof(double) * 2 * hvol * batch);
    int err = axis_pass(h, ny, nz, batch, +1, 1, t);
    if (!err) err = axis_pass(h, ny, nz, batch, +1, 2, t);
    if (!err) {
        root_table(nx, +1, w);
#pragma omp parallel for schedule(static)
        for (long r = 0; r < rows; ++r) {
            const double *H = t + 2 * r * h;
            for (int x = 0; x < nx; ++x) {
                double v = H[0] + ((x & 1) ? -H[2 * (nx / 2)] : H[2 * (nx / 2)]);
                for (int k = 1; k < nx / 2; ++k) {
                    const long e = ((long)k * x) % nx;
                    v += 2.0 * (H[2 * k] * w[2 * e] - H[2 * k + 1] * w[2 * e + 1]);
                }
                out[r * nx + x] = v;
            }
        }
    }
    free(t);
    free(w);
    return err;
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 16-bit formats, from the IEEE definitions (round to nearest, ties even)   */
/* ------------------------------------------------------------------------ */

/* Round the real number v (finite) to an integer, ties to even. */
static double rne_int(double v)
{
    double f = floor(v), d = v - f;
    if (d > 0.5) return f + 1.0;
    if (d < 0.5) return f;
    return fmod(f, 2.0) == 0.0 ? f : f + 1.0;
}

/*
 * Round v to a binary floating-point format with `mant` stored fraction bits,
 * minimum normal exponent emin and maximum exponent emax; return the rounded
 * value (as a double; +-inf on overflow).  Works on the value, not on bits:
 * v = m * 2^(e - mant) with the quantum 2^(max(e, emin) - mant).
 */
static double round_format(double v, int mant, int emin, int emax)
{
    if (v == 0.0 || !isfinite(v)) return v;
    double a = fabs(v);
    int e = ilogb(a);
    if (e < emin) e = emin;                       /* subnormal quantum */
    double q = ldexp(1.0, e - mant);
    double r = rne_int(a / q) * q;
    /* largest finite value: (2 - 2^-mant) * 2^emax */
    double maxv = ldexp(2.0 - ldexp(1.0, -mant), emax);
    if (r > maxv) r = INFINITY;
    return v < 0 ? -r : r;
}

/* Encode a value already rounded to the format into its 16-bit pattern. */
static uint16_t pack_format(double r, int mant, int ebits)
{
    uint16_t s = signbit(r) ? (uint16_t)(1u << 15) : 0;
    double a = fabs(r);
    const int bias = (1 << (ebits - 1)) - 1;
    if (isinf(a)) return s | (uint16_t)(((1u << ebits) - 1) << mant);
    if (a == 0.0) return s;
    int e = ilogb(a);
    if (e < 1 - bias) {                           /* subnormal */
        double m = a / ldexp(1.0, 1 - bias - mant);
        return s | (uint16_t)m;
    }
    double frac = a / ldexp(1.0, e) - 1.0;        /* in [0, 1) */
    uint16_t m = (uint16_t)(frac * (double)(1u << mant));
    return s | (uint16_t)((e + bias) << mant) | m;
}

static double unpack_format(uint16_t h, int mant, int ebits)
{
    const int bias = (1 << (ebits - 1)) - 1;
    int s = h >> 15;
    int e = (h >> mant) & ((1 << ebits) - 1);
    int m = h & ((1 << mant) - 1);
    double v;
    if (e == 0)
        v = ldexp((double)m, 1 - bias - mant);
    else if (e == (1 << ebits) - 1)
        v = m ? NAN : INFINITY;
    else
        v = ldexp(1.0 + (double)m / (double)(1u << mant), e - bias);
    return s ? -v : v;
}

/* binary16: 10 fraction bits, 5 exponent bits, normal exponents [-14, 15].
 * bfloat16: 7 fraction bits, 8 exponent bits, normal exponents [-126, 127]. */
uint16_t oracle_round_fp16(double v) { return pack_format(round_format(v, 10, -14, 15), 10, 5); }
uint16_t oracle_round_bf16(double v) { return pack_format(round_format(v, 7, -126, 127), 7, 8); }
double oracle_fp16_value(uint16_t h) { return unpack_format(h, 10, 5); }
double oracle_bf16_value(uint16_t h) { return unpack_format(h, 7, 8); }

/*
 * Scaled 16-bit storage ("scaled16"): every row of `row_len` complex values
 * carries one int8 exponent e; the stored value is payload * 2^e.
 * Exponent rule (per row): m = max over the row of |re| and |im|;
 * e = 0 if m == 0, else e = clamp(ilogb(m) - 14, -128, 127), which puts the
 * scaled row maximum in [2^14, 2^15), inside the binary16 range.
 * fmt: 1 = binary16 payload, 2 = bfloat16 payload.  `in` holds FP32 values.
 */
int oracle_q16_encode(int fmt, long rows, int row_len, const float *in,
                      uint16_t *payload, int8_t *exps)
{
    if ((fmt != 1 && fmt != 2) || rows < 0 || row_len < 1) return -1;
    for (long r = 0; r < rows; ++r) {
        const float *v = in + 2 * r * row_len;
        double m = 0.0;
        for (int i = 0; i < 2 * row_len; ++i) {
            double a = fabs((double)v[i]);
            if (a > m) m = a;
        }
        int e = 0;
        if (m > 0.0) {
            e = ilogb(m) - 14;
            if (e < -128) e = -128;
            if (e > 127) e = 127;
        }
        exps[r] = (int8_t)e;
        for (int i = 0; i < 2 * row_len; ++i) {
            double s = ldexp((double)v[i], -e);
            payload[2 * r * row_len + i] =
                fmt == 1 ? oracle_round_fp16(s) : oracle_round_bf16(s);
        }
    }
    return 0;
}

int oracle_q16_decode(int fmt, long rows, int row_len, const uint16_t *payload,
                      const int8_t *exps, double *out)
{
    if ((fmt != 1 && fmt != 2) || rows < 0 || row_len < 1) return -1;
    for (long r = 0; r < rows; ++r)
        for (int i = 0; i < 2 * row_len; ++i) {
            uint16_t h = payload[2 * r * row_len + i];
            double v = fmt == 1 ? oracle_fp16_value(h) : oracle_bf16_value(h);
            out[2 * r * row_len + i] = ldexp(v, exps[r]);
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Plane-wave local-potential energy and its gradient                        */
/* ------------------------------------------------------------------------ */

/*
 * The local-potential operator of a plane-wave code applied to coefficient
 * grids c_n: out_n = forward transform (sign -1) of V * inverse transform
 * (sign +1) of c_n, both unnormalised (so a constant V = v gives
 * out = v * Nx*Ny*Nz * c).  This is half the gradient of oracle_energy's E.
 */
int oracle_apply_potential(int nx, int ny, int nz, int batch, const double *c,
                           const double *V, double *out)
{
    const long vol = (long)nx * ny * nz;
    const int inverse = +1, forward = -1;
    double *p = malloc(sizeof(double) * 2 * vol * batch);
    if (!p) return -4;
    int err = oracle_fft3d(nx, ny, nz, batch, inverse, c, p);
    if (!err) {
        for (int b = 0; b < batch; ++b)
            for (long i = 0; i < vol; ++i) {
                p[2 * (b * vol + i)] *= V[i];
                p[2 * (b * vol + i) + 1] *= V[i];
            }
        err = oracle_fft3d(nx, ny, nz, batch, forward, p, out);
    }
    free(p);
    return err;
}

/*
 * The electron density of a plane-wave code from its orbital coefficients:
 * rho(r) = sum_n f_n |psi_n(r)|^2 with psi_n the unnormalised inverse
 * transform (sign +1) of c_n and f_n the occupation of orbital n.  rho is a
 * real [z][y][x] grid.
 */
int oracle_density(int nx, int ny, int nz, int batch, const double *c,
                   const double *occ, double *rho)
{
    const long vol = (long)nx * ny * nz;
    const int inverse_sign = +1;
    double *p = malloc(sizeof(double) * 2 * vol * batch);
    if (!p) return -4;
    int err = oracle_fft3d(nx, ny, nz, batch, inverse_sign, c, p);
    if (!err) {
        for (long i = 0; i < vol; ++i) rho[i] = 0.0;
        for (int b = 0; b < batch; ++b)
            for (long i = 0; i < vol; ++i) {
                const double re = p[2 * (b * vol + i)], im = p[2 * (b * vol + i) + 1];
                rho[i] += occ[b] * (re * re + im * im);
            }
    }
    free(p);
    return err;
}

/*
 * psi_n = unnormalised inverse transform of c_n (sign +1), for every orbital n
 * of the batch;  E = sum_n sum_r V(r) |psi_n(r)|^2 (V real, shared).
 * Gradient in the convention dE/dRe(c) + i dE/dIm(c) (what automatic
 * differentiation of a real function of complex inputs returns):
 *   grad_n = 2 * forward transform (sign -1) of V * psi_n,
 * because E is a Hermitian form in c and the adjoint of the unnormalised
 * inverse is the unnormalised forward transform.
 * psi and grad may be NULL.
 */
int oracle_energy(int nx, int ny, int nz, int batch, const double *c,
                  const double *V, double *E, double *psi, double *grad)
{
    const long vol = (long)nx * ny * nz;
    double *p = malloc(sizeof(double) * 2 * vol * batch);
    if (!p) return -4;
    int err = oracle_fft3d(nx, ny, nz, batch, +1, c, p);
    if (err) { free(p); return err; }
    double acc = 0.0;
    for (int b = 0; b < batch; ++b)
        for (long i = 0; i < vol; ++i) {
            double re = p[2 * (b * vol + i)], im = p[2 * (b * vol + i) + 1];
            acc += V[i] * (re * re + im * im);
        }
    *E = acc;
    if (psi) memcpy(psi, p, sizeof(double) * 2 * vol * batch);
    if (grad) {
        for (int b = 0; b < batch; ++b)
            for (long i = 0; i < vol; ++i) {
                p[2 * (b * vol + i)] *= 2.0 * V[i];
                p[2 * (b * vol + i) + 1] *= 2.0 * V[i];
            }
        err = oracle_fft3d(nx, ny, nz, batch, -1, p, grad);
    }
    free(p);
    return err;
}
