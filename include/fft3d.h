/*
 * fft3d.h -- C ABI of libfft3d.so, a complex-to-complex 3D FFT for AMD
 * Instinct MI355X (gfx950).
 *
 * The operation is Eq. (1) of Ramaswami, Kenter, Kuehne, Plessl, "Efficient
 * Ab-Initio Molecular Dynamic Simulations by Offloading Fast Fourier
 * Transformations to FPGAs" (Section II):
 *
 *   out[b][kz][ky][kx] = sum_{z,y,x} in[b][z][y][x]
 *                        * exp(s * 2 pi i * (x kx / Nx + y ky / Ny + z kz / Nz))
 *
 * with s = -1 (FFT3D_FORWARD, Eq. (1) itself: W_N = exp(-2 pi i / N)) or
 * s = +1 (FFT3D_INVERSE, the unnormalised inverse; the paper defines no
 * inverse, and this library follows the convention that inverse(forward(f))
 * = Nx Ny Nz f).  No normalisation is applied in either direction.  The
 * transform is computed, as Section II decomposes it, as batched 1D FFTs
 * along x, then y, then z.
 *
 * Data layout: C order [batch][z][y][x], x contiguous, complex values as
 * interleaved (re, im) pairs.  FFT3D_FP32 buffers hold complex64 (8 bytes per
 * point).  Output is in natural order, in the same layout as the input.
 *
 * Scaled 16-bit buffers (FFT3D_FP16_SCALED / FFT3D_BF16_SCALED; the paper's
 * reduced-precision direction, Section I and the closing paragraph of
 * Section III): a payload of one 32-bit word per point (low 16 bits the real
 * part, high 16 bits the imaginary part, as binary16 or bfloat16 patterns),
 * followed at byte offset 4 * batch * nx*ny*nz by one int8 exponent per
 * x-row ([batch][z][y], batch*nz*ny bytes).  A point's value is payload *
 * 2^exponent.  Exponents follow the rule of fft3d_quantize.  These plans need
 * nx == ny == nz with 16 | n (16, 32, 48, 64, 80, 96, 128); all arithmetic
 * is FP32 (the radix-16 stage as an FP32 butterfly on the vector ALUs; with
 * the environment variable FFT3D_Q16_MFMA=1 at plan time it runs instead as
 * a DFT-matrix product with FP32 accumulation on the matrix cores: binary16
 * operands, or for bfloat16 input the payloads as loaded times a DFT matrix
 * held as two bfloat16 terms); the intermediate between the xy and z passes
 * is stored as scaled binary16.
 *
 * Memory: every data pointer passed to an exec call is a DEVICE pointer
 * (hipMalloc / torch CUDA tensor memory) on the device the plan was created
 * on, aligned to 16 bytes.  The caller owns all buffers and the stream.  A
 * plan owns its device-side tables (allocated at plan time, freed by
 * fft3d_destroy); execution never allocates and never synchronises the host.
 *
 * Streams: `stream` is a hipStream_t (NULL selects the null stream).  Calls
 * are enqueued asynchronously in stream order.  A plan must not be executed
 * concurrently on two streams.
 *
 * Errors: functions returning int return FFT3D_OK (0) or a negative
 * fft3d_status.  Plan constructors return NULL on error and record the code,
 * readable with fft3d_last_error() (per host thread).  Argument checks run
 * before any HIP call.
 */
#ifndef FFT3D_H
#define FFT3D_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *fft3d_stream_t; /* the same type as hipStream_t */
typedef struct fft3d_plan_s *fft3d_plan_t;   /* opaque */

enum fft3d_precision {
    FFT3D_FP32 = 0,        /* complex64 in, complex64 out, FP32 arithmetic */
    FFT3D_FP16_SCALED = 1, /* scaled 16-bit storage, binary16 payload */
    FFT3D_BF16_SCALED = 2  /* scaled 16-bit storage, bfloat16 payload */
};

enum fft3d_direction {
    FFT3D_FORWARD = -1, /* exponent sign -1: Eq. (1) */
    FFT3D_INVERSE = 1   /* exponent sign +1, unnormalised */
};

enum fft3d_status {
    FFT3D_OK = 0,
    FFT3D_E_INVALID_ARG = -1,      /* NULL plan/pointer, bad enum, batch < 1, size < 1 */
    FFT3D_E_UNSUPPORTED_SIZE = -2, /* a dimension > 512 or not of the form 2^a 3^b 5^c */
    FFT3D_E_NO_DEVICE = -3,        /* no usable HIP device */
    FFT3D_E_ALLOC = -4,            /* device allocation failed at plan time */
    FFT3D_E_LAUNCH = -5,           /* a kernel launch or HIP call failed */
    FFT3D_E_ALIGNMENT = -6,        /* a data pointer is not 16-byte aligned */
    FFT3D_E_UNSUPPORTED = -7,      /* valid arguments, combination not provided */
    FFT3D_E_TIMEOUT = -8,          /* a bounded in-kernel wait expired (see fft3d_plan_check) */
    FFT3D_E_SCRATCH = -9           /* problem too large for the fixed scratch of fft3d_energy_noalloc */
};

/*
 * Create a plan for `batch` grids of nx * ny * nz points (Section II, Eq. (1)).
 * 1 <= nx, ny, nz <= 512, each 2^a 3^b 5^c; batch >= 1; precision one of
 * fft3d_precision; direction FFT3D_FORWARD or FFT3D_INVERSE.  Builds the
 * radix schedule, generates the twiddle factors in double precision (rounded
 * once to the working precision) and uploads them to the current device.
 * Grids with a dimension above 128 (the larger sizes the paper names as
 * future work, Section III) use the three-pass form: one 1D pass per axis
 * (x rows, then strided y and z lines), FP32 only (FFT3D_E_UNSUPPORTED for
 * the scaled 16-bit precisions); every other entry point that takes a plan
 * (energy, cutoff, real grids, heterogeneous batches) is limited to 128.
 * Returns NULL on error (see fft3d_last_error).
 */
fft3d_plan_t fft3d_plan(int nx, int ny, int nz, int batch, int precision, int direction);

/*
 * Real grids.  Densities and potentials, the other grids a plane-wave code
 * transforms (Section I), are real; their transform under Eq. (1) is
 * Hermitian, F(-k) = conj F(k), so half of it is kept: kx = 0 .. nx/2.
 * Plan `batch` real transforms with nx == ny, nx even, each dimension
 * 2^a 3^b 5^c in 1..128, FP32.
 *   FORWARD (r2c): in = real float32 [batch][nz][ny][nx], out = complex64
 *     [batch][nz][ny][nx/2 + 1], the kx <= nx/2 half of Eq. (1).
 *   INVERSE (c2r): in = complex64 [batch][nz][ny][nx/2 + 1], out = real
 *     float32 [batch][nz][ny][nx]: the unnormalised inverse of the Hermitian
 *     extension (complex inverse along z and y, then the real inverse along
 *     x, which ignores the imaginary parts of the kx = 0 and kx = nx/2
 *     entries); c2r(r2c(f)) = nx*ny*nz*f.  The input buffer is used as the
 *     workspace of the z pass and is OVERWRITTEN.
 * fft3d_exec(plan, in, out, stream) runs it; in and out must be distinct
 * (FFT3D_E_INVALID_ARG otherwise).  fft3d_buffer_bytes returns the bytes of
 * the complex side, fft3d_real_bytes those of the real side (0 for plans
 * that are not real).  Passes (fft3d_exec_pass): r2c = [plane in -> out,
 * z in place on out]; c2r = [z in place on `in`, plane in -> out].  The z
 * pass always works in place on the complex-side buffer (out of an r2c, in
 * of a c2r) whatever the other pointer is.
 * Returns NULL with FFT3D_E_UNSUPPORTED for nx != ny or nx odd; other
 * errors as fft3d_plan.  Energy and cutoff entry points reject real plans.
 */
fft3d_plan_t fft3d_plan_real(int nx, int ny, int nz, int batch, int direction);
size_t fft3d_real_bytes(fft3d_plan_t plan);

/*
 * Enqueue the transform of `in` into `out` on `stream`.  Both are device
 * buffers of fft3d_buffer_bytes(plan) bytes.  in == out (in place) is
 * allowed; out-of-place calls leave `in` unmodified.  Returns FFT3D_OK,
 * FFT3D_E_INVALID_ARG (NULL plan or pointer), FFT3D_E_ALIGNMENT or
 * FFT3D_E_LAUNCH.
 */
int fft3d_exec(fft3d_plan_t plan, const void *in, void *out, fft3d_stream_t stream);

/* Release a plan and its device tables.  NULL is a no-op.  Returns FFT3D_OK. */
int fft3d_destroy(fft3d_plan_t plan);

/* Code of the last failed plan construction on this host thread (FFT3D_OK if none). */
int fft3d_last_error(void);

/* Static, human-readable text for a status code. */
const char *fft3d_strerror(int code);

/* Bytes of one input (and one output) buffer of the plan; 0 for NULL. */
size_t fft3d_buffer_bytes(fft3d_plan_t plan);

/*
 * Write a one-line description of the plan's kernel schedule (kernels,
 * radices, threads, LDS bytes) into buf (NUL-terminated, truncated to len).
 * Returns the untruncated length, or a negative status.
 */
int fft3d_plan_describe(fft3d_plan_t plan, char *buf, size_t len);

/*
 * Pruned transforms for a sphere cutoff in frequency space.  In a plane-wave
 * code the coefficients that enter the inverse transform of Eq. (1), and the
 * ones kept after the forward transform, are those inside a sphere (the 3D
 * FFTs that evaluate the quantum-mechanical operators, Section I, and the
 * cutoff restriction of the evaluation in Section III).  With the signed
 * frequency G_d = k_d for k_d < N_d/2 and k_d - N_d otherwise, the sphere is
 * Gx^2 + Gy^2 + Gz^2 < r2.
 *   INVERSE plan: the caller promises that every input point outside the
 *     sphere is zero (those points are never read).  The plane pass handles
 *     only the xy-planes with Gz^2 < r2 and reads in each only the x-rows
 *     with Gy^2 + Gz^2 < r2; the z pass skips the loads of the other planes.
 *     The result is the dense transform of the same input, computed by the
 *     same butterflies in the same order.
 *   FORWARD plan: only the output inside the sphere is wanted.  The plane
 *     pass transforms every plane but stores only the points with
 *     Gx^2 + Gy^2 < r2 (the z-lines the sphere meets); the z pass transforms
 *     only those lines and stores only the points inside the sphere, which
 *     hold the dense transform's values; all other output points are left
 *     unspecified (they may hold intermediate values).
 *   Both use the dense schedule's butterflies in the dense order; the
 *   compiler may contract a few multiply-adds of the pruned kernels into
 *   FMAs differently, so results agree with the dense plan's to FP32
 *   rounding (in practice the inverse reproduces them bit for bit).
 * Applies to fft3d_exec and fft3d_exec_pass (the pass list keeps its two
 * passes, plane then z, with pruned kernels); the energy entry points are
 * not affected.
 *   r2 > 0   set the cutoff (replacing an earlier one); r2 <= 0 clears it.
 * Returns FFT3D_E_UNSUPPORTED unless the plan is an FP32 plan with nx == ny
 * from fft3d_plan; FFT3D_E_INVALID_ARG for NULL or NaN; FFT3D_E_ALLOC if the
 * plane list cannot be allocated (the plan is then unchanged).  Not
 * thread-safe against a concurrent exec of the same plan.
 */
int fft3d_plan_set_cutoff(fft3d_plan_t plan, double r2);

/*
 * Packed spheres.  Plane-wave codes keep only the coefficients inside the
 * cutoff sphere.  The packed form of a plan with a cutoff (see above) lists,
 * for each grid of the batch in turn, the points inside the sphere in the
 * grid's own order (kz, then ky, then kx ascending): exactly the points
 * dense[b][kz][ky][kx] with Gx^2 + Gy^2 + Gz^2 < r2, as a boolean-mask
 * selection in row-major order would list them.  A packed buffer holds
 * batch * fft3d_plan_sphere_points(plan) complex64 values, grid after grid.
 *
 * fft3d_plan_sphere_points: points per grid inside the sphere, or
 *   FFT3D_E_INVALID_ARG (NULL) / FFT3D_E_UNSUPPORTED (no cutoff set).
 * fft3d_sphere_pack: gather dense [batch][nz][ny][nx] -> packed.
 * fft3d_sphere_unpack: scatter packed -> dense, writing zeros at every point
 *   outside the sphere.
 * fft3d_exec_packed: the pruned transform with the sphere in packed form.
 *   INVERSE plan: reads `packed`, writes the dense result to `dense` (the
 *     plane pass gathers its rows straight from the packed sphere); equal to
 *     fft3d_exec on the unpacked input.
 *   FORWARD plan: reads `dense`, which is also used as the workspace of the
 *     first pass and is overwritten, and writes the points inside the
 *     sphere to `packed` (the z pass scatters them there directly).
 * All three copy/transform calls are enqueued on `stream`.  Pointers must be
 * 16-byte aligned device pointers to distinct buffers.  Return FFT3D_OK,
 * FFT3D_E_INVALID_ARG (NULL, or the same buffer twice), FFT3D_E_ALIGNMENT,
 * FFT3D_E_UNSUPPORTED (no cutoff set) or FFT3D_E_LAUNCH.
 */
long long fft3d_plan_sphere_points(fft3d_plan_t plan);
int fft3d_sphere_pack(fft3d_plan_t plan, const void *dense, void *packed, fft3d_stream_t stream);
int fft3d_sphere_unpack(fft3d_plan_t plan, const void *packed, void *dense, fft3d_stream_t stream);
int fft3d_exec_packed(fft3d_plan_t plan, void *dense, void *packed, fft3d_stream_t stream);

/*
 * Measurement hooks.  An exec is a fixed sequence of kernel launches
 * ("passes": e.g. the xy-plane pass and the z pass of Section II's
 * decomposition).  fft3d_plan_passes returns how many; fft3d_exec_pass
 * enqueues pass `pass` alone (0-based), reading `in` and writing `out`, so a
 * profiler can time each kernel.  Running passes 0..k-1 in order with
 * in -> out for pass 0 and out -> out afterwards is exactly fft3d_exec.
 * Returns FFT3D_E_INVALID_ARG for a NULL plan/pointer or a pass out of range.
 */
int fft3d_plan_passes(fft3d_plan_t plan);
/*
 * Health check of a plan's device-side state.  Batches of cubic grids run as
 * one persistent kernel in which the z pass of a grid waits, with a bounded
 * spin, for that grid's xy-plane pass; if any such wait ever expired (which
 * would mean an invalid result) this returns FFT3D_E_TIMEOUT once and clears
 * the flag.  Synchronises the device: for tests and diagnostics, not for the
 * hot path.  Returns FFT3D_OK, FFT3D_E_INVALID_ARG or FFT3D_E_LAUNCH.
 */
int fft3d_plan_check(fft3d_plan_t plan);
int fft3d_exec_pass(fft3d_plan_t plan, int pass, const void *in, void *out, fft3d_stream_t stream);

/*
 * Conversions between complex64 rows and scaled 16-bit storage, on `stream`.
 * `rows` rows of `row_len` complex values; in the scaled buffer the payload
 * (rows*row_len 32-bit words) is followed by `rows` int8 exponents.  Rule per
 * row: m = max of |re| and |im| over the row; e = 0 if m == 0, otherwise
 * e = clamp(ilogb(m) - 14, -128, 127); payload = value * 2^-e rounded to
 * nearest even (so the row maximum is stored in [2^14, 2^15)).
 * fft3d_dequantize returns the exact values payload * 2^e.  precision is
 * FFT3D_FP16_SCALED or FFT3D_BF16_SCALED.  Returns FFT3D_OK,
 * FFT3D_E_INVALID_ARG, FFT3D_E_ALIGNMENT (16-byte device pointers) or
 * FFT3D_E_LAUNCH.  Inputs must be finite with magnitude below 2^127.
 */
int fft3d_quantize(int precision, long rows, int row_len, const void *in_c64, void *out_scaled,
                   fft3d_stream_t stream);
int fft3d_dequantize(int precision, long rows, int row_len, const void *in_scaled, void *out_c64,
                     fft3d_stream_t stream);

/*
 * Measurement aid, not part of the transform: copies `bytes` bytes from src
 * to dst (device pointers, 16-byte aligned, not overlapping; bytes a
 * multiple of 16) on `stream` with 16-byte non-temporal loads and stores in
 * one sweep.  Timing it on buffers the size of a transform's input gives the
 * practical HBM bandwidth (read + write) that the transform passes are
 * compared with, beside the nominal 8 TB/s.  bytes == 0 is a no-op.
 * Returns FFT3D_OK, FFT3D_E_INVALID_ARG, FFT3D_E_ALIGNMENT or FFT3D_E_LAUNCH.
 */
int fft3d_stream_copy(const void *src, void *dst, size_t bytes, fft3d_stream_t stream);

/*
 * Heterogeneous batches in one launch.  `count` groups (1 <= count <= 16);
 * group g holds batch[g] cubic grids of nx[g] = ny[g] = nz[g] points per
 * side (sizes 24, 30, 32, 36, 40, 48, 50, 60, 64, 72, 80, 90, 96, 100, 120,
 * 128; FP32).  fft3d_exec_many transforms every grid of every group with ONE
 * persistent kernel launch: workgroups claim work items (xy-planes, then
 * xz-slabs of each grid) from a queue, and a grid's z work waits on a
 * per-grid counter of its finished planes.  A plan can instead run in the
 * grouped mode (two plain launches per group, the dense kernels) or a hybrid
 * of the two (see fft3d_plan_set_schedule), which the tuner picks when they
 * measure faster (few, large groups).  `in` and `out` are HOST arrays of
 * `count` device pointers, group g's buffer holding batch[g] grids in the
 * layout of fft3d_exec (in[g] == out[g] allowed).  The launch is
 * graph-capturable; a plan must not run concurrently with itself or with
 * another persistent launch on a different stream.
 *
 * Returns NULL / FFT3D_E_UNSUPPORTED for non-cubic or unlisted sizes and
 * other precisions.  The schedule (launch mode, threads per workgroup, items
 * per queue claim, and per group the radix order and z-tile width of its
 * plain passes) is taken from the tuning cache ($FFT3D_TUNE_CACHE, default
 * ~/.cache/fft3d/tune.json), else tuned at plan time when FFT3D_TUNE=1,
 * else a default.  The results are valid only while fft3d_plan_check
 * reports no expired wait (see there).
 */
fft3d_plan_t fft3d_plan_many(int count, const int *nx, const int *ny, const int *nz, const int *batch,
                             int precision, int direction);
int fft3d_exec_many(fft3d_plan_t plan, const void *const *in, void *const *out, fft3d_stream_t stream);
/* Force a schedule of a many-plan: threads 512 or 1024 (the persistent
 * kernel, chunk 1..64 items per claim), threads 0 (grouped mode: each
 * group's plane pass and z pass as plain launches, chunk ignored), or
 * threads -512 / -1024 (hybrid mode: a group whose batch*n planes fill every
 * compute unit with the plane kernel runs as in grouped mode, all other
 * groups share one persistent launch with 512 / 1024 threads).  The tuner
 * times all of them. */
int fft3d_plan_set_schedule(fft3d_plan_t plan, int threads, int chunk);
/* Force the schedule of group `group`'s plain passes (grouped mode, and
 * the big groups of the hybrid mode): radix_order 0 = the default radix
 * order of its length, 1 = the alternative order (the default's two radices
 * swapped, or the length split another way: 36 = 9x4, 64 = 16x4,
 * 100 = 4x5x5); z_lines = 64 or 32 adjacent z-lines per workgroup of the z
 * pass.  Returns FFT3D_OK or FFT3D_E_INVALID_ARG. */
int fft3d_plan_set_group_schedule(fft3d_plan_t plan, int group, int radix_order, int z_lines);
/* Time every schedule candidate on scratch buffers (synchronous), keep the
 * fastest and record it in the tuning cache: first, per group, the radix
 * order and z-tile width of its plain passes (that group alone); then the
 * launch mode with its threads and chunk. */
int fft3d_plan_tune(fft3d_plan_t plan);

/*
 * Plane-wave local-potential energy and its gradient (the operator
 * evaluation through 3D FFTs that Section I places on the critical path of
 * plane-wave DFT; the FP32-vs-FP64 energy comparison of Section III is its
 * accuracy question).  For a plan of `batch` orbitals c_n (FP32, nx == ny,
 * either direction):
 *
 *   fft3d_energy_fwd:  psi_n = unnormalised inverse transform of c_n (sign
 *     +1), written to `psi` (device, same size as c; psi == c allowed), and
 *     E = sum_n sum_r V(r) |psi_n(r)|^2 written to E_dev[0] (device double).
 *     V is a device float array [nz][ny][nx] shared by all orbitals.  The
 *     products are FP32, the sum is FP64 in a fixed order (deterministic).
 *   fft3d_energy_bwd:  grad_c = forward transform (sign -1) of
 *     2 * gE_dev[0] * V * psi_n -- the gradient of gE * E in the convention
 *     dE/dRe(c) + i dE/dIm(c) (the adjoint of the unnormalised inverse is the
 *     unnormalised forward transform).  If have_psi != 0, c_or_psi holds psi
 *     (e.g. from fft3d_energy_fwd); otherwise it holds c and the gradient
 *     is computed by the fused operator below (psi is not stored).  grad_c
 *     may equal c_or_psi.
 *
 * Both enqueue on `stream` without host synchronisation.  Returns FFT3D_OK,
 * FFT3D_E_INVALID_ARG (NULL pointer), FFT3D_E_ALIGNMENT (data not 16-byte,
 * doubles not 8-byte aligned), FFT3D_E_UNSUPPORTED (plan not FP32 or
 * nx != ny) or FFT3D_E_LAUNCH.
 */
int fft3d_energy_fwd(fft3d_plan_t plan, const void *c, const float *V, void *psi, double *E_dev,
                     fft3d_stream_t stream);

/*
 * E alone, for schedules that recompute psi in the backward pass
 * (fft3d_energy_bwd with have_psi == 0): the same E as fft3d_energy_fwd (the
 * same FP32 products summed in the same FP64 order, so bit-identical), with
 * psi summed on chip and never written.  `work` (device, the size of c)
 * receives the xy-transformed intermediate; its contents afterwards are
 * unspecified.  work == c is allowed and then overwrites c.  One read of c,
 * one write and one read of the intermediate: 3 sweeps instead of 4.
 * Plans and return codes as for fft3d_energy_fwd.
 */
int fft3d_energy(fft3d_plan_t plan, const void *c, const float *V, void *work, double *E_dev,
                 fft3d_stream_t stream);

/*
 * fft3d_energy without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same E as fft3d_energy on a plan of `batch`
 * orbitals of nx * ny * nz points (bit-identical: the same kernels, tables
 * and summation order), without a plan.  The twiddle tables and the
 * per-workgroup partial sums live in a fixed 1 MiB device array of the
 * library, one per GPU it runs on, held until the process ends.  The call
 * allocates nothing; it enqueues on `stream` a table fill, the xy-plane
 * pass c -> work, the E-only z pass and the final sum into E_dev[0].
 *   Limits: nx == ny; every dimension 2^a 3^b 5^c in 1..128; the partial
 *   sums, ceil(batch*ny*nx / 64) doubles, must fit the array: batch*nx*ny
 *   <= 8,355,840 (e.g. batch <= 510 at 128^2, <= 906 at 96^2); beyond it
 *   FFT3D_E_SCRATCH.
 *   Every call on one GPU uses that GPU's single array, which keeps the
 *   last call's contents: calls that overlap on one GPU (two streams, two
 *   host threads without ordering) race and give wrong results.  The first
 *   call on a device looks the array up (hipGetSymbolAddress) and must not
 *   itself be under stream capture; later calls may be captured.
 * c, work: device complex64 [batch][nz][ny][nx] (work receives the
 * xy-transformed orbitals, contents afterwards unspecified; work == c
 * allowed and then overwrites c); V: device float [nz][ny][nx]; E_dev:
 * device double.  Returns FFT3D_OK, FFT3D_E_INVALID_ARG (NULL pointer,
 * size or batch < 1), FFT3D_E_ALIGNMENT (c, work, V not 16-byte, E_dev not
 * 8-byte aligned), FFT3D_E_UNSUPPORTED_SIZE, FFT3D_E_UNSUPPORTED
 * (nx != ny), FFT3D_E_SCRATCH, FFT3D_E_NO_DEVICE or FFT3D_E_LAUNCH.
 */
int fft3d_energy_noalloc(int nx, int ny, int nz, int batch, const void *c, const float *V, void *work,
                         double *E_dev, fft3d_stream_t stream);

/*
 * The local-potential operator itself, out_n = s * forward(V * inverse(c_n))
 * (both unnormalised; s = scale_dev[0] if scale_dev is not NULL, else 1):
 * the product of Section I's operator evaluation, and half the energy
 * gradient.  Three passes instead of four: inverse xy planes, then one
 * fused z kernel (inverse z transform, the energy sum and the product with
 * V, forward z transform, with psi held on chip and never written to HBM),
 * then forward xy planes.  If E_dev is not NULL it receives
 * E = sum_n sum_r V(r) |psi_n(r)|^2 as in fft3d_energy_fwd.  With a cutoff
 * set on the plan (fft3d_plan_set_cutoff) the pruned passes are used: c must
 * vanish outside the sphere, and only the points of `out` inside the sphere
 * are written (the rest are unspecified).  c == out is allowed.  The
 * forward transform runs z before xy, so results agree with fft3d_exec's
 * forward to FP32 rounding.  Plans as for the energy entry points; returns
 * the same codes.  fft3d_energy_bwd with have_psi == 0 uses this path (with
 * s = 2 gE, dense).
 */
int fft3d_apply_potential(fft3d_plan_t plan, const void *c, const float *V, void *out, double *E_dev,
                          const double *scale_dev, fft3d_stream_t stream);

/*
 * Electron density from orbital coefficients, the real-space product that
 * follows the inverse transforms of Section I's plane-wave operators:
 * rho(r) = sum_n occ[n] |psi_n(r)|^2, psi_n the unnormalised inverse
 * transform (sign +1) of c_n, for the plan's `batch` orbitals.  occ: device
 * float[batch]; rho: device float [nz][ny][nx] (written, not accumulated);
 * work: device buffer of the size of c (the xy-transformed orbitals; may
 * equal c, which is then overwritten).  Two passes: the inverse xy planes
 * into `work`, then one kernel per group of z-lines that runs the inverse
 * z transform of every orbital in turn and sums occ |psi|^2 in registers
 * (FP32, fixed orbital order: deterministic), so psi is never stored.  With a
 * cutoff on the plan, c must vanish outside the sphere and the pruned plane
 * pass is used.  Plans as for the energy entry points; returns the same
 * codes (FFT3D_E_ALIGNMENT: c / work not 16-byte, occ / rho not 4-byte
 * aligned).
 */
int fft3d_density(fft3d_plan_t plan, const void *c, const float *occ, float *rho, void *work,
                  fft3d_stream_t stream);
int fft3d_energy_bwd(fft3d_plan_t plan, const void *c_or_psi, int have_psi, const float *V, const double *gE_dev,
                     void *grad_c, fft3d_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FFT3D_H */
