// Host side of libfft3d: argument validation, planning (schedule choice and
// FP64 twiddle generation), and stream-ordered execution of the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plan_internal.hpp"

namespace fft3d {

namespace {
thread_local int g_last_error = FFT3D_OK;
}  // namespace

enum Scheme {
    kCube = 0,    // whole grid per workgroup
    kPlaneZ = 1,  // xy-plane pass + strided z pass (Nx == Ny)
    kAxes = 2,    // x rows, strided y, strided z
    kFused = 3,   // persistent plane + z-slab kernel (cubic)
    kQ16 = 4,     // scaled 16-bit storage, radix-16 on the matrix cores (cubic, 16 | N)
};

int set_error(int code)
{
    g_last_error = code;
    return code;
}

// Angles are reduced to an integer index modulo the root order before
// cos/sin (double precision), then rounded once to float.
int twiddles_into(float2* t, int cap, int n, int sign, int kind)
{
    const Sched sc = make_sched_kind(n, kind);
    const int len = sched_tw_len(sc) > 0 ? sched_tw_len(sc) : 0;
    if (len > cap) return -1;
    for (int s = 1; s < sc.count; ++s) {
        const int R = sc.r[s], NS = sched_ns(sc, s), order = NS * R;
        const int off = sched_tw_off(sc, s);
        for (int k = 0; k < NS; ++k)
            for (int q = 1; q < R; ++q) {
                const long m = ((long)k * q) % order;
                const double a = 2.0 * M_PI * (double)m / (double)order;
                t[off + k * (R - 1) + (q - 1)] = make_float2((float)std::cos(a), (float)(sign * std::sin(a)));
            }
    }
    return len;
}

std::vector<float2> twiddles(int n, int sign, int kind)
{
    const Sched sc = make_sched_kind(n, kind);
    std::vector<float2> t(sched_tw_len(sc) > 0 ? sched_tw_len(sc) : 0);
    if (!t.empty()) twiddles_into(t.data(), (int)t.size(), n, sign, kind);
    return t;
}

bool env_flag(const char* name)
{
    const char* e = std::getenv(name);
    return e && e[0] == '1';
}

static bool test_fail_alloc() { return env_flag("FFT3D_TEST_FAIL_ALLOC"); }

// FFT3D_FUSED: 1 = persistent plane+slab kernel, 2 = its XCD-local variant.
static int fused_mode()
{
    const char* e = std::getenv("FFT3D_FUSED");
    return e ? std::atoi(e) : 0;
}

int last_error_value() { return g_last_error; }
void clear_error() { g_last_error = FFT3D_OK; }

}  // namespace fft3d

using namespace fft3d;

extern "C" {

const char* fft3d_strerror(int code)
{
    switch (code) {
    case FFT3D_OK: return "success";
    case FFT3D_E_INVALID_ARG: return "invalid argument";
    case FFT3D_E_UNSUPPORTED_SIZE: return "unsupported size (each dimension must be 2^a 3^b 5^c, 1..512)";
    case FFT3D_E_NO_DEVICE: return "no usable HIP device";
    case FFT3D_E_ALLOC: return "device allocation failed";
    case FFT3D_E_LAUNCH: return "kernel launch or HIP call failed";
    case FFT3D_E_ALIGNMENT: return "data pointer not 16-byte aligned";
    case FFT3D_E_UNSUPPORTED: return "valid arguments, combination not provided";
    case FFT3D_E_TIMEOUT: return "a bounded in-kernel wait expired (result invalid)";
    case FFT3D_E_SCRATCH: return "problem exceeds the fixed scratch array of the no-allocation entry point";
    default: return "unknown status";
    }
}

int fft3d_last_error(void) { return last_error_value(); }

fft3d_plan_t fft3d_plan(int nx, int ny, int nz, int batch, int precision, int direction)
{
    clear_error();
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    if (precision != FFT3D_FP32 && precision != FFT3D_FP16_SCALED && precision != FFT3D_BF16_SCALED) {
        set_error(FFT3D_E_INVALID_ARG);
        return nullptr;
    }
    if (direction != FFT3D_FORWARD && direction != FFT3D_INVERSE) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    auto size_ok = [](int n) { return size_supported(n) || size_supported_large(n); };
    if (!size_ok(nx) || !size_ok(ny) || !size_ok(nz)) {
        set_error(FFT3D_E_UNSUPPORTED_SIZE);
        return nullptr;
    }
    // lengths above 128: FP32, three-pass form only
    const bool large = nx > 128 || ny > 128 || nz > 128;
    if (large && precision != FFT3D_FP32) { set_error(FFT3D_E_UNSUPPORTED); return nullptr; }
    const long vol = (long)nx * ny * nz;
    // 2^36 points (512 GiB of complex64) bounds every grid dimension of every
    // launch below 2^31 workgroups.
    if ((long)batch * vol > (1L << 36)) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    const bool q16 = precision != FFT3D_FP32;
    if (q16 && (nx != ny || ny != nz || !q16_plane_fn(nx, direction))) { set_error(FFT3D_E_UNSUPPORTED); return nullptr; }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error(FFT3D_E_NO_DEVICE);
        return nullptr;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error(FFT3D_E_NO_DEVICE); return nullptr; }

    fft3d_plan_s* p = new (std::nothrow) fft3d_plan_s{};
    if (!p) { set_error(FFT3D_E_ALLOC); return nullptr; }
    p->nx = nx; p->ny = ny; p->nz = nz; p->batch = batch;
    p->precision = precision; p->direction = direction; p->device = dev; p->vol = vol;
    if (q16) {
        p->scheme = kQ16;
        // radix-16 stage on the vector ALUs unless FFT3D_Q16_MFMA=1 asks for the matrix cores
        // (the vector-ALU stage measured faster and more accurate on MI355X)
        p->q16_valu = !env_flag("FFT3D_Q16_MFMA");
    }
    else if (large) p->scheme = kAxes;
    else if (nx == ny && ny == nz && nx <= kCubeMaxN) p->scheme = kCube;
    else if (nx == ny && ny == nz && fused_fn(nx, direction) && fused_mode() > 0) p->scheme = kFused;
    else if (nx == ny) p->scheme = kPlaneZ;
    else p->scheme = kAxes;

    // One table per dimension (identical lengths share nothing on purpose:
    // the tables are tiny and separate offsets keep the exec path simple).
    std::vector<float2> tab;
    const int kind = q16 ? 1 : 0;
    auto append = [&](int n, int sign) {
        const long off = (long)tab.size();
        std::vector<float2> t = twiddles(n, sign, kind);
        tab.insert(tab.end(), t.begin(), t.end());
        // keep every table 16-byte aligned
        if (tab.size() % 2) tab.push_back(make_float2(0.f, 0.f));
        return off;
    };
    p->tw_x = append(nx, direction);
    p->tw_y = append(ny, direction);
    p->tw_z = append(nz, direction);
    p->tw_rx = append(nx, -direction);
    p->tw_ry = append(ny, -direction);
    p->tw_rz = append(nz, -direction);
    if (tab.empty()) tab.push_back(make_float2(0.f, 0.f));
    const size_t bytes = tab.size() * sizeof(float2);
    if (test_fail_alloc() || hipMalloc((void**)&p->d_tw, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        set_error(FFT3D_E_ALLOC);
        return nullptr;
    }
    if (hipMemcpy(p->d_tw, tab.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p->d_tw);
        delete p;
        set_error(FFT3D_E_LAUNCH);
        return nullptr;
    }
    if (nx == ny && !q16 && !large) {
        // energy path: persistent plane pass + strided z pass with fused epilogue
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        const long resident = (long)plane_pf_blocks_per_cu(nx) * cus, planes = (long)batch * nz;
        p->pf_grid = (int)(planes < resident ? planes : resident);
        p->n_partials = axis_str_blocks((long)batch * ny * nx);
        if (hipMalloc((void**)&p->partials, sizeof(double) * p->n_partials) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(p->d_tw);
            delete p;
            set_error(FFT3D_E_ALLOC);
            return nullptr;
        }
    }
    const long B = batch;
    const AxisMap zmap{B * ny * nx, nx, ny, vol, (long)nx, (long)nx * ny};
    const AxisMap ymap{B * nz * nx, nx, nz, vol, (long)nx * ny, (long)nx};
    if (p->scheme == kQ16) {
        p->passes.push_back({Pass::kQ16PlaneK, nx, B * nz, {}, p->tw_x, 0});
        p->passes.push_back({Pass::kQ16SlabK, nx, B * ny, {}, p->tw_x, 0});
    } else if (p->scheme == kFused) {
        // room for either control-block layout (XcdCtl is the larger one)
        const size_t cb = (sizeof(XcdCtl) > sizeof(FusedCtl) ? sizeof(XcdCtl) : sizeof(FusedCtl)) +
                          sizeof(unsigned) * (size_t)batch;
        p->ctl_bytes = cb;
        if (hipMalloc((void**)&p->ctl, cb) != hipSuccess || hipMemset(p->ctl, 0, cb) != hipSuccess) {
            (void)hipGetLastError();
            if (p->ctl) (void)hipFree(p->ctl);
            (void)hipFree(p->d_tw);
            delete p;
            set_error(FFT3D_E_ALLOC);
            return nullptr;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        const int resident = fused_blocks_per_cu(nx) * cus;
        const long items = 2L * batch * nx;
        p->fused_grid = (int)(items < resident ? items : resident);
        p->fused_lag = (resident + nx - 1) / nx + 1;
        const char* ck = std::getenv("FFT3D_FUSED_CHUNK");
        p->fused_chunk = ck ? std::atoi(ck) : 1;
        int nxcc = 1;
        if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nxcc < 1) {
            (void)hipGetLastError();
            nxcc = 1;
        }
        if (nxcc > 8) nxcc = 8;
        if (env_flag("FFT3D_LOG")) std::fprintf(stderr, "fft3d_plan: %d XCDs, %d resident workgroups\n", nxcc, resident);
        p->fused_xcd = fused_mode() == 2 ? nxcc : 0;
        if (p->fused_xcd) {
            // lag, in grids: every workgroup holds two claimed items (the
            // current one and the next), so a slab item is claimed only
            // after twice the XCD's resident workgroups' worth of items
            // have been claimed since its grid's planes, plus two grids.
            // Measured at 256 x 64^3 (lags 1, 2, 3, 5, 6, 8, 11, 16:
            // 1.05, 0.77, 0.59, 0.34, 0.35, 0.36, 0.39, 0.42 ms per
            // transform): shorter lags make slab items wait, longer ones
            // keep more intermediates in flight.  FFT3D_FUSED_LAG overrides.
            const int res_x = fused_xcd_blocks_per_cu(nx) * cus;
            p->fused_grid = (int)(items < res_x ? items : res_x);
            const char* lg = std::getenv("FFT3D_FUSED_LAG");
            p->fused_lag = lg && std::atoi(lg) > 0 ? std::atoi(lg) : (2 * (res_x / nxcc) + nx - 1) / nx + 2;
        }
        p->passes.push_back({Pass::kFusedK, nx, B, {}, p->tw_x});
    } else if (p->scheme == kCube) {
        p->passes.push_back({Pass::kCubeK, nx, B, {}, p->tw_x});
    } else if (p->scheme == kPlaneZ) {
        if (plane_pf_fn(nx, direction) && !env_flag("FFT3D_NO_PLANE_PF")) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 1;
            const long resident = (long)plane_pf_blocks_per_cu(nx) * cus;
            const long planes = B * nz;
            p->passes.push_back({Pass::kPlanePfK, nx, planes, {}, p->tw_x, p->pf_grid});
        } else {
            p->passes.push_back({Pass::kPlaneK, nx, B * nz, {}, p->tw_x});
        }
        if (nz > 1) p->passes.push_back({Pass::kStrK, nz, 0, zmap, p->tw_z});
    } else {
        if (nx > 1) p->passes.push_back({Pass::kRowK, nx, B * nz * ny, {}, p->tw_x});
        if (ny > 1) p->passes.push_back({Pass::kStrK, ny, 0, ymap, p->tw_y});
        if (nz > 1) p->passes.push_back({Pass::kStrK, nz, 0, zmap, p->tw_z});
    }
    return p;
}

fft3d_plan_t fft3d_plan_real(int nx, int ny, int nz, int batch, int direction)
{
    clear_error();
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    if (direction != FFT3D_FORWARD && direction != FFT3D_INVERSE) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    if (!size_supported(nx) || !size_supported(ny) || !size_supported(nz)) {
        set_error(FFT3D_E_UNSUPPORTED_SIZE);
        return nullptr;
    }
    if (nx != ny || nx % 2 || !real_plane_fn(nx, direction < 0)) { set_error(FFT3D_E_UNSUPPORTED); return nullptr; }
    const long vol = (long)nx * ny * nz;
    if ((long)batch * vol > (1L << 36)) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        set_error(FFT3D_E_NO_DEVICE);
        return nullptr;
    }
    fft3d_plan_s* p = new (std::nothrow) fft3d_plan_s{};
    if (!p) { set_error(FFT3D_E_ALLOC); return nullptr; }
    p->nx = nx; p->ny = ny; p->nz = nz; p->batch = batch;
    p->precision = FFT3D_FP32; p->direction = direction; p->device = dev; p->vol = vol;
    p->real = true;
    p->scheme = kPlaneZ;
    const int M = nx / 2, H = M + 1;
    std::vector<float2> tab;
    auto append = [&](const std::vector<float2>& t) {
        const long off = (long)tab.size();
        tab.insert(tab.end(), t.begin(), t.end());
        if (tab.size() % 2) tab.push_back(make_float2(0.f, 0.f));
        return off;
    };
    p->tw_x = append(twiddles(M, direction));
    p->tw_y = append(twiddles(ny, direction));
    p->tw_z = append(twiddles(nz, direction));
    // split/merge roots exp(direction * 2 pi i k / nx), k = 0 .. M/2
    std::vector<float2> rt(M / 2 + 1);
    for (int k = 0; k <= M / 2; ++k) {
        const double a = 2.0 * M_PI * (double)k / (double)nx;
        rt[k] = make_float2((float)std::cos(a), (float)(direction * std::sin(a)));
    }
    p->tw_rt = append(rt);
    const size_t bytes = tab.size() * sizeof(float2);
    if (test_fail_alloc() || hipMalloc((void**)&p->d_tw, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        set_error(FFT3D_E_ALLOC);
        return nullptr;
    }
    if (hipMemcpy(p->d_tw, tab.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p->d_tw);
        delete p;
        set_error(FFT3D_E_LAUNCH);
        return nullptr;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        cus = 1;
    }
    const long planes = (long)batch * nz;
    const long resident = (long)real_blocks_per_cu(nx, direction < 0) * cus;
    const Pass plane{Pass::kRealK, nx, planes, {}, 0, (int)(planes < resident ? planes : resident)};
    // z pass over the half layout [batch][z][y][H]
    const AxisMap zmap{(long)batch * ny * H, H, ny, (long)nz * ny * H, (long)H, (long)ny * H};
    const Pass zpass{Pass::kStrK, nz, 0, zmap, p->tw_z, 0};
    if (direction == FFT3D_FORWARD) {
        p->passes.push_back(plane);
        if (nz > 1) p->passes.push_back(zpass);
    } else {
        if (nz > 1) p->passes.push_back(zpass);
        p->passes.push_back(plane);
    }
    return p;
}

size_t fft3d_real_bytes(fft3d_plan_t p)
{
    if (!p || !p->real) return 0;
    return (size_t)p->batch * (size_t)p->vol * sizeof(float);
}

int fft3d_destroy(fft3d_plan_t p)
{
    if (!p) return FFT3D_OK;
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->ctl) (void)hipFree(p->ctl);
    if (p->partials) (void)hipFree(p->partials);
    if (p->mp.d_grids) (void)hipFree(p->mp.d_grids);
    if (p->mp.d_items) (void)hipFree(p->mp.d_items);
    if (p->mp.d_twoff) (void)hipFree(p->mp.d_twoff);
    if (p->d_zlist) (void)hipFree(p->d_zlist);
    if (p->d_rows) (void)hipFree(p->d_rows);
    delete p;
    return FFT3D_OK;
}

size_t fft3d_buffer_bytes(fft3d_plan_t p)
{
    if (!p) return 0;
    if (p->many) {
        size_t b = 0;
        for (int g = 0; g < p->mp.ngroups; ++g)
            b += (size_t)p->mp.batch[g] * p->mp.n[g] * p->mp.n[g] * p->mp.n[g] * sizeof(float2);
        return b;
    }
    if (p->real)   // the complex half-spectrum side
        return (size_t)p->batch * p->nz * p->ny * (p->nx / 2 + 1) * sizeof(float2);
    if (p->precision != FFT3D_FP32)   // payload (4 B per point) + one exponent byte per x-row
        return (size_t)p->batch * (size_t)p->vol * 4 + (size_t)p->batch * p->nz * p->ny;
    return (size_t)p->batch * (size_t)p->vol * sizeof(float2);
}

static hipError_t run_pass(const fft3d_plan_s* p, const Pass& ps, const float2* src, float2* dst,
                           hipStream_t st)
{
    const int S = p->direction;
    const float2* tw = p->d_tw + ps.tw;
    switch (ps.kind) {
    case Pass::kCubeK: return cube_fn(ps.n, S)(src, dst, tw, ps.count, st);
    case Pass::kPlaneK: return plane_fn(ps.n, S)(src, dst, tw, ps.count, st);
    case Pass::kPlanePfK:
        return plane_pf_fn(ps.n, S)(src, dst, tw, ps.count, ps.grid, 0, nullptr, nullptr, 1, true, st);
    case Pass::kRowK: return axis_row_fn(ps.n, S)(src, dst, tw, ps.count, st);
    case Pass::kStrK: return axis_str_fn(ps.n, S)(src, dst, tw, ps.map, 0, nullptr, nullptr, 0, st);
    case Pass::kPlanePrunedK:
        return plane_pruned_fn(ps.n, S)(src, dst, tw, ps.count, ps.grid, p->d_zlist, p->n_zlist, p->nz, p->cut_r2,
                                        nullptr, 0, st);
    case Pass::kStrPrunedK: return axis_str_pruned_fn(ps.n, S)(src, dst, tw, ps.map, p->cut_r2, nullptr, 0, st);
    case Pass::kRealK:
        return real_plane_fn(ps.n, S < 0)(src, dst, p->d_tw + p->tw_x, p->d_tw + p->tw_y, p->d_tw + p->tw_rt,
                                          ps.count, ps.grid, st);
    case Pass::kQ16PlaneK:
    case Pass::kQ16SlabK: {
        const size_t pay = (size_t)p->batch * p->vol * 4;
        const unsigned* ip = reinterpret_cast<const unsigned*>(src);
        const signed char* ie = reinterpret_cast<const signed char*>(src) + pay;
        unsigned* op = reinterpret_cast<unsigned*>(dst);
        signed char* oe = reinterpret_cast<signed char*>(dst) + pay;
        const int f = p->precision | (p->q16_valu ? 16 : 0);
        if (ps.kind == Pass::kQ16PlaneK) return q16_plane_fn(ps.n, S)(ip, ie, op, oe, tw, ps.count, f, st);
        return q16_slab_fn(ps.n, S)(ip, ie, op, oe, tw, ps.count, f, st);
    }
    case Pass::kFusedK:
        if (p->ctl_bytes < sizeof(XcdCtl) + sizeof(unsigned) * (size_t)p->batch) return hipErrorInvalidValue;
        if (p->fused_xcd)
            return fused_xcd_fn(ps.n, S)(src, dst, tw, p->ctl, p->batch, p->fused_lag, p->fused_grid, p->fused_xcd, st);
        return fused_fn(ps.n, S)(src, dst, tw, p->ctl, p->batch, p->fused_lag, p->fused_grid, p->fused_chunk, st);
    }
    return hipErrorInvalidValue;
}

static int check_ptrs(fft3d_plan_t p, const void* in, const void* out)
{
    if (!p || !in || !out) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)in % 16) || ((uintptr_t)out % 16)) return FFT3D_E_ALIGNMENT;
    return FFT3D_OK;
}

int fft3d_exec(fft3d_plan_t p, const void* in, void* out, fft3d_stream_t stream)
{
    const int rc = check_ptrs(p, in, out);
    if (rc != FFT3D_OK) return rc;
    if (p->many) return FFT3D_E_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float2* src = static_cast<const float2*>(in);
    float2* dst = static_cast<float2*>(out);
    hipError_t e = hipSuccess;
    if (p->real) {
        // r2c: plane pass in -> out, z pass in place on out.  c2r: z pass in
        // place on the input (which it overwrites), plane pass in -> out.
        if (in == out) return FFT3D_E_INVALID_ARG;
        float2* work = p->direction == FFT3D_INVERSE ? const_cast<float2*>(src) : dst;
        for (size_t i = 0; i < p->passes.size() && e == hipSuccess; ++i) {
            const Pass& ps = p->passes[i];
            e = ps.kind == Pass::kRealK ? run_pass(p, ps, src, dst, st) : run_pass(p, ps, work, work, st);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return FFT3D_E_LAUNCH;
        }
        return FFT3D_OK;
    }
    for (size_t i = 0; i < p->passes.size() && e == hipSuccess; ++i)
        e = run_pass(p, p->passes[i], i == 0 ? src : dst, dst, st);
    if (e == hipSuccess && p->passes.empty() && src != dst)
        e = hipMemcpyAsync(dst, src, fft3d_buffer_bytes(p), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_plan_passes(fft3d_plan_t p)
{
    if (!p) return FFT3D_E_INVALID_ARG;
    if (p->many) return 1;
    return (int)p->passes.size();
}

int fft3d_exec_pass(fft3d_plan_t p, int pass, const void* in, void* out, fft3d_stream_t stream)
{
    const int rc = check_ptrs(p, in, out);
    if (rc != FFT3D_OK) return rc;
    if (p->many || pass < 0 || pass >= (int)p->passes.size()) return FFT3D_E_INVALID_ARG;
    const Pass& ps = p->passes[pass];
    const float2* src = static_cast<const float2*>(in);
    float2* dst = static_cast<float2*>(out);
    if (p->real && ps.kind != Pass::kRealK) {
        // the z pass of a real plan works in place on the complex (half
        // spectrum) side: `out` of an r2c, `in` of a c2r; the other pointer
        // may be the smaller real buffer and is never touched by it
        float2* work = p->direction == FFT3D_INVERSE ? const_cast<float2*>(src) : dst;
        src = work;
        dst = work;
    }
    const hipError_t e = run_pass(p, ps, src, dst, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

// Two-pass transform of sign `sign` (plane pass, then z pass) with the
// optional gradient prologue (V, gE) and energy epilogue (V, E partials).
// epilogue: 0 none, 1 E summed while psi is stored, 2 E only (dst then
// holds the xy-transformed intermediate).
static hipError_t energy_transform(const fft3d_plan_s* p, int sign, const float2* src, float2* dst,
                                   const float* V, const double* gE, int epilogue, hipStream_t st)
{
    const int n = p->nx, nz = p->nz;
    const bool same = sign == p->direction;
    const float2* twx = p->d_tw + (same ? p->tw_x : p->tw_rx);
    const float2* twz = p->d_tw + (same ? p->tw_z : p->tw_rz);
    const long planes = (long)p->batch * nz;
    hipError_t e = plane_pf_fn(n, sign)(src, dst, twx, planes, p->pf_grid, gE != nullptr, V, gE, nz, true, st);
    if (e != hipSuccess) return e;
    const AxisMap zmap{(long)p->batch * p->ny * n, n, p->ny, p->vol, (long)n, (long)n * p->ny};
    if (nz > 1 || epilogue) e = axis_str_fn(nz, sign)(dst, dst, twz, zmap, epilogue, V, p->partials, p->vol, st);
    return e;
}

static int energy_args(fft3d_plan_t p, const void* a, const void* b, const void* V, const void* d)
{
    if (!p || !a || !b || !V || !d) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)a % 16) || ((uintptr_t)b % 16) || ((uintptr_t)V % 16) || ((uintptr_t)d % 8))
        return FFT3D_E_ALIGNMENT;
    if (p->many || p->real || p->precision != FFT3D_FP32 || p->nx != p->ny || !p->partials)
        return FFT3D_E_UNSUPPORTED;
    return FFT3D_OK;
}

int fft3d_energy_fwd(fft3d_plan_t p, const void* c, const float* V, void* psi, double* E_dev, fft3d_stream_t stream)
{
    const int rc = energy_args(p, c, psi, V, E_dev);
    if (rc != FFT3D_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = energy_transform(p, FFT3D_INVERSE, static_cast<const float2*>(c), static_cast<float2*>(psi), V,
                                    nullptr, 1, st);
    if (e == hipSuccess) e = launch_sum_partials(p->partials, p->n_partials, E_dev, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_energy(fft3d_plan_t p, const void* c, const float* V, void* work, double* E_dev, fft3d_stream_t stream)
{
    const int rc = energy_args(p, c, work, V, E_dev);
    if (rc != FFT3D_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = energy_transform(p, FFT3D_INVERSE, static_cast<const float2*>(c), static_cast<float2*>(work), V,
                                    nullptr, 2, st);
    if (e == hipSuccess) e = launch_sum_partials(p->partials, p->n_partials, E_dev, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

// out = mult * s * forward(V * inverse(c)), s = scale ? scale[0] : 1, in three
// passes: inverse xy planes (c -> out), the fused z kernel (inverse z, V,
// forward z; psi stays on chip), forward xy planes (out -> out).  With
// `cut` and a cutoff on the plan, the passes are the pruned ones (input
// zero outside the sphere, output defined inside it).  E (optional): sum
// V |inverse(c)|^2.
static hipError_t hloc_run(const fft3d_plan_s* p, const float2* c, float2* out, const float* V, double* E,
                           const double* scale, float mult, bool cut, hipStream_t st)
{
    const int n = p->nx, nz = p->nz;
    const bool inv_plan = p->direction == FFT3D_INVERSE;
    const float2* twx_inv = p->d_tw + (inv_plan ? p->tw_x : p->tw_rx);
    const float2* twx_fwd = p->d_tw + (inv_plan ? p->tw_rx : p->tw_x);
    const float2* twz_inv = p->d_tw + (inv_plan ? p->tw_z : p->tw_rz);
    const float2* twz_fwd = p->d_tw + (inv_plan ? p->tw_rz : p->tw_z);
    const AxisMap zmap{(long)p->batch * p->ny * n, n, p->ny, p->vol, (long)n, (long)n * p->ny};
    double* partials = E ? p->partials : nullptr;
    hipError_t e;
    if (cut) {
        const long planes = (long)p->batch * p->n_zlist;
        const int grid = (int)(planes < p->pf_grid ? planes : p->pf_grid);
        e = plane_pruned_fn(n, FFT3D_INVERSE)(c, out, twx_inv, planes, grid, p->d_zlist, p->n_zlist, nz, p->cut_r2,
                                              nullptr, 0, st);
        if (e == hipSuccess)
            e = axis_hloc_fn(nz)(out, twz_inv, twz_fwd, zmap, V, scale, mult, partials, p->vol, p->cut_r2, 1, st);
        if (e == hipSuccess)
            e = plane_ball_fwd_fn(n)(out, out, twx_fwd, planes, grid, p->d_zlist, p->n_zlist, nz, p->cut_r2, nullptr,
                                     0, st);
    } else {
        const long planes = (long)p->batch * nz;
        e = plane_pf_fn(n, FFT3D_INVERSE)(c, out, twx_inv, planes, p->pf_grid, 0, nullptr, nullptr, nz, true, st);
        if (e == hipSuccess)
            e = axis_hloc_fn(nz)(out, twz_inv, twz_fwd, zmap, V, scale, mult, partials, p->vol, 0.0, 0, st);
        if (e == hipSuccess)
            // reads what the fused z kernel just wrote: no streaming
            e = plane_pf_fn(n, FFT3D_FORWARD)(out, out, twx_fwd, planes, p->pf_grid, 0, nullptr, nullptr, nz, false,
                                              st);
    }
    if (e == hipSuccess && E) e = launch_sum_partials(p->partials, p->n_partials, E, st);
    return e;
}

int fft3d_apply_potential(fft3d_plan_t p, const void* c, const float* V, void* out, double* E_dev,
                          const double* scale_dev, fft3d_stream_t stream)
{
    if (!p || !c || !V || !out) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)c % 16) || ((uintptr_t)out % 16) || ((uintptr_t)V % 16) || ((uintptr_t)E_dev % 8) ||
        ((uintptr_t)scale_dev % 8))
        return FFT3D_E_ALIGNMENT;
    if (p->many || p->real || p->precision != FFT3D_FP32 || p->nx != p->ny || !p->partials)
        return FFT3D_E_UNSUPPORTED;
    const hipError_t e = hloc_run(p, static_cast<const float2*>(c), static_cast<float2*>(out), V, E_dev, scale_dev,
                                  1.0f, p->cut_r2 > 0, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_density(fft3d_plan_t p, const void* c, const float* occ, float* rho, void* work, fft3d_stream_t stream)
{
    if (!p || !c || !occ || !rho || !work) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)c % 16) || ((uintptr_t)work % 16) || ((uintptr_t)rho % 4) || ((uintptr_t)occ % 4))
        return FFT3D_E_ALIGNMENT;
    if (p->many || p->real || p->precision != FFT3D_FP32 || p->nx != p->ny || !p->partials)
        return FFT3D_E_UNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = p->nx, nz = p->nz;
    const bool inv_plan = p->direction == FFT3D_INVERSE;
    const float2* twx = p->d_tw + (inv_plan ? p->tw_x : p->tw_rx);
    const float2* twz = p->d_tw + (inv_plan ? p->tw_z : p->tw_rz);
    const float2* src = static_cast<const float2*>(c);
    float2* w = static_cast<float2*>(work);
    hipError_t e;
    const bool cut = p->cut_r2 > 0;
    if (cut) {
        const long planes = (long)p->batch * p->n_zlist;
        const int grid = (int)(planes < p->pf_grid ? planes : p->pf_grid);
        e = plane_pruned_fn(n, FFT3D_INVERSE)(src, w, twx, planes, grid, p->d_zlist, p->n_zlist, nz, p->cut_r2,
                                              nullptr, 0, st);
    } else {
        e = plane_pf_fn(n, FFT3D_INVERSE)(src, w, twx, (long)p->batch * nz, p->pf_grid, 0, nullptr, nullptr, nz, true,
                                          st);
    }
    // the z-lines of one grid: (y, x) pairs, elements along z
    const AxisMap zmap{(long)p->ny * n, n, p->ny, p->vol, (long)n, (long)n * p->ny};
    if (e == hipSuccess)
        e = axis_density_fn(nz)(w, twz, zmap, p->batch, p->vol, occ, rho, cut ? p->cut_r2 : 0.0, cut ? 1 : 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_energy_bwd(fft3d_plan_t p, const void* c_or_psi, int have_psi, const float* V, const double* gE_dev,
                     void* grad_c, fft3d_stream_t stream)
{
    const int rc = energy_args(p, c_or_psi, grad_c, V, gE_dev);
    if (rc != FFT3D_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float2* src = static_cast<const float2*>(c_or_psi);
    float2* g = static_cast<float2*>(grad_c);
    hipError_t e = hipSuccess;
    if (!have_psi)   // from c: the fused operator, 2 gE forward(V inverse(c)), psi never stored
        e = hloc_run(p, src, g, V, nullptr, gE_dev, 2.0f, false, st);
    else
        e = energy_transform(p, FFT3D_FORWARD, src, g, V, gE_dev, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_quantize(int precision, long rows, int row_len, const void* in, void* out, fft3d_stream_t stream)
{
    if ((precision != FFT3D_FP16_SCALED && precision != FFT3D_BF16_SCALED) || rows < 0 || row_len < 1 || !in || !out)
        return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)in % 16) || ((uintptr_t)out % 16)) return FFT3D_E_ALIGNMENT;
    unsigned* pay = static_cast<unsigned*>(out);
    signed char* ex = reinterpret_cast<signed char*>(pay + (size_t)rows * row_len);
    if (launch_quantize(precision, static_cast<const float2*>(in), rows, row_len, pay, ex,
                        reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_dequantize(int precision, long rows, int row_len, const void* in, void* out, fft3d_stream_t stream)
{
    if ((precision != FFT3D_FP16_SCALED && precision != FFT3D_BF16_SCALED) || rows < 0 || row_len < 1 || !in || !out)
        return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)in % 16) || ((uintptr_t)out % 16)) return FFT3D_E_ALIGNMENT;
    const unsigned* pay = static_cast<const unsigned*>(in);
    const signed char* ex = reinterpret_cast<const signed char*>(pay + (size_t)rows * row_len);
    if (launch_dequantize(precision, pay, ex, rows, row_len, static_cast<float2*>(out),
                          reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_stream_copy(const void* src, void* dst, size_t bytes, fft3d_stream_t stream)
{
    if ((bytes && (!src || !dst)) || bytes % 16) return FFT3D_E_INVALID_ARG;
    if (((uintptr_t)src % 16) || ((uintptr_t)dst % 16)) return FFT3D_E_ALIGNMENT;
    if (launch_stream_copy(src, dst, (long)(bytes / 16), reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

static unsigned* timeouts_ptr(fft3d_plan_t p)
{
    if (!p->many && p->fused_xcd) return &reinterpret_cast<XcdCtl*>(p->ctl)->timeouts;
    return &p->ctl->timeouts;
}

int fft3d_plan_check(fft3d_plan_t p)
{
    if (!p) return FFT3D_E_INVALID_ARG;
    if (!p->ctl) return FFT3D_OK;
    unsigned t = 0;
    const hipError_t e1 = hipDeviceSynchronize();
    const hipError_t e2 = e1 == hipSuccess ? hipMemcpy(&t, timeouts_ptr(p), sizeof t, hipMemcpyDeviceToHost) : e1;
    if (e2 != hipSuccess) {
        if (env_flag("FFT3D_LOG"))
            std::fprintf(stderr, "fft3d_plan_check: %s / %s\n", hipGetErrorString(e1), hipGetErrorString(e2));
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    if (t) {
        const unsigned z = 0;
        (void)hipMemcpy(timeouts_ptr(p), &z, sizeof z, hipMemcpyHostToDevice);
        return FFT3D_E_TIMEOUT;
    }
    return FFT3D_OK;
}

int fft3d_plan_set_cutoff(fft3d_plan_t p, double r2)
{
    if (!p) return FFT3D_E_INVALID_ARG;
    if (!(r2 == r2)) return FFT3D_E_INVALID_ARG;   // NaN
    if (p->many || p->real || p->precision != FFT3D_FP32 || p->nx != p->ny) return FFT3D_E_UNSUPPORTED;
    const int nx = p->nx, nz = p->nz;
    if (!plane_pruned_fn(nx, p->direction) || !axis_str_pruned_fn(nz, p->direction)) return FFT3D_E_UNSUPPORTED;
    if (p->dense_passes.empty()) p->dense_passes = p->passes;
    if (r2 <= 0) {
        p->passes = p->dense_passes;
        p->cut_r2 = 0;
        p->n_zlist = 0;
        p->sphere_pts = 0;
        return FFT3D_OK;
    }
    const int ny = p->ny;
    // planes kz whose signed frequency satisfies Gz^2 < r2, in ascending kz;
    // the z pass applies the same test element by element
    std::vector<int> zl;
    for (int k = 0; k < nz; ++k) {
        const int g = signed_freq(k, nz);
        if ((double)(g * g) < r2) zl.push_back(k);
    }
    // packed-sphere rows: the points of row (kz, ky) inside the sphere are
    // kx = 0 .. npos-1 and the last cnt - npos ones, by the same test
    std::vector<SphereRow> rows((size_t)nz * ny);
    long pts = 0;
    for (int kz = 0; kz < nz; ++kz)
        for (int ky = 0; ky < ny; ++ky) {
            const int gz = signed_freq(kz, nz), gy = signed_freq(ky, ny);
            SphereRow r{(int)pts, 0, 0, 0};
            for (int kx = 0; kx < nx; ++kx) {
                const int gx = signed_freq(kx, nx);
                if ((double)(gx * gx + gy * gy + gz * gz) < r2) {
                    ++r.cnt;
                    if (gx >= 0) ++r.npos;
                }
            }
            rows[(size_t)kz * ny + ky] = r;
            pts += r.cnt;
        }
    int* d = nullptr;
    SphereRow* dr = nullptr;
    if (test_fail_alloc() || hipMalloc((void**)&d, sizeof(int) * zl.size()) != hipSuccess ||
        hipMalloc((void**)&dr, sizeof(SphereRow) * rows.size()) != hipSuccess) {
        (void)hipGetLastError();
        if (d) (void)hipFree(d);
        return FFT3D_E_ALLOC;
    }
    if (hipMemcpy(d, zl.data(), sizeof(int) * zl.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dr, rows.data(), sizeof(SphereRow) * rows.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        (void)hipFree(dr);
        return FFT3D_E_LAUNCH;
    }
    if (p->d_zlist) (void)hipFree(p->d_zlist);
    if (p->d_rows) (void)hipFree(p->d_rows);
    p->d_zlist = d;
    p->d_rows = dr;
    p->n_zlist = (int)zl.size();
    p->sphere_pts = pts;
    p->cut_r2 = r2;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        cus = 1;
    }
    const long B = p->batch;
    const bool inv = p->direction == FFT3D_INVERSE;
    // inverse: only the non-zero planes; forward: every plane
    const long planes = inv ? B * p->n_zlist : B * nz;
    const long resident = (long)plane_pf_blocks_per_cu(nx) * cus;
    const AxisMap zmap{B * p->ny * nx, nx, p->ny, p->vol, (long)nx, (long)nx * p->ny};
    p->passes.clear();
    p->passes.push_back({Pass::kPlanePrunedK, nx, planes, {}, p->tw_x, (int)(planes < resident ? planes : resident)});
    if (nz > 1) p->passes.push_back({Pass::kStrPrunedK, nz, 0, zmap, p->tw_z, 0});
    return FFT3D_OK;
}

long long fft3d_plan_sphere_points(fft3d_plan_t p)
{
    if (!p) return FFT3D_E_INVALID_ARG;
    if (p->cut_r2 <= 0) return FFT3D_E_UNSUPPORTED;
    return p->sphere_pts;
}

static int sphere_copy(fft3d_plan_t p, bool pack, const void* src, void* dst, fft3d_stream_t stream)
{
    const int rc = check_ptrs(p, src, dst);
    if (rc != FFT3D_OK) return rc;
    if (p->cut_r2 <= 0 || p->many) return FFT3D_E_UNSUPPORTED;
    if (src == dst) return FFT3D_E_INVALID_ARG;
    const long total = (long)p->batch * p->vol;
    const hipError_t e = launch_sphere_copy(pack, static_cast<const float2*>(src), static_cast<float2*>(dst), p->d_rows,
                                            p->sphere_pts, p->nx, (long)p->nz * p->ny, total,
                                            reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_sphere_pack(fft3d_plan_t p, const void* dense, void* packed, fft3d_stream_t stream)
{
    return sphere_copy(p, true, dense, packed, stream);
}

int fft3d_sphere_unpack(fft3d_plan_t p, const void* packed, void* dense, fft3d_stream_t stream)
{
    return sphere_copy(p, false, packed, dense, stream);
}

int fft3d_exec_packed(fft3d_plan_t p, void* dense, void* packed, fft3d_stream_t stream)
{
    const int rc = check_ptrs(p, dense, packed);
    if (rc != FFT3D_OK) return rc;
    if (p->cut_r2 <= 0 || p->many) return FFT3D_E_UNSUPPORTED;
    if (dense == packed) return FFT3D_E_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float2* d = static_cast<float2*>(dense);
    float2* pk = static_cast<float2*>(packed);
    const int S = p->direction;
    hipError_t e = hipSuccess;
    // the pass list of the cutoff schedule: [plane, z] (z only when nz > 1)
    const Pass& plane = p->passes[0];
    const float2* twp = p->d_tw + plane.tw;
    if (S == FFT3D_INVERSE) {
        e = plane_pruned_fn(plane.n, S)(pk, d, twp, plane.count, plane.grid, p->d_zlist, p->n_zlist, p->nz, p->cut_r2,
                                        p->d_rows, p->sphere_pts, st);
        if (e == hipSuccess && p->passes.size() > 1)
            e = run_pass(p, p->passes[1], d, d, st);
    } else {
        e = run_pass(p, plane, d, d, st);
        if (e == hipSuccess) {
            if (p->passes.size() > 1) {
                const Pass& z = p->passes[1];
                e = axis_str_pruned_fn(z.n, S)(d, pk, p->d_tw + z.tw, z.map, p->cut_r2, p->d_rows, p->sphere_pts, st);
            } else {
                e = launch_sphere_copy(true, d, pk, p->d_rows, p->sphere_pts, p->nx, (long)p->nz * p->ny,
                                       (long)p->batch * p->vol, st);
            }
        }
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_plan_describe(fft3d_plan_t p, char* buf, size_t len)
{
    if (!p) return FFT3D_E_INVALID_ARG;
    if (p->many) return many_describe(p, buf, len);
    if (p->real) {
        const KernelInfo a = real_info(p->nx), b = axis_str_info(p->nz);
        char t[256];
        snprintf(t, sizeof t, "real %s n=%d half=%d threads=%d lds=%d planes=%ld; z n=%d threads=%d lds=%d kernels=%s",
                 p->direction < 0 ? "r2c" : "c2r", p->nx, p->nx / 2 + 1, a.threads, a.lds_bytes,
                 (long)p->batch * p->nz, p->nz, b.threads, b.lds_bytes,
                 p->nz == 1 ? (p->direction < 0 ? "k_plane_r2c" : "k_plane_c2r")
                            : (p->direction < 0 ? "k_plane_r2c,k_axis_str" : "k_axis_str,k_plane_c2r"));
        const std::string d = t;
        if (buf && len) {
            std::strncpy(buf, d.c_str(), len - 1);
            buf[len - 1] = 0;
        }
        return (int)d.size();
    }
    auto radices = [](int n) {
        const Sched sc = make_sched(n);
        std::string s;
        for (int i = 0; i < sc.count; ++i) s += (i ? "x" : "") + std::to_string(sc.r[i]);
        return s;
    };
    std::string d;
    char tmp[256];
    if (p->scheme == kQ16) {
        const KernelInfo k = q16_info(p->nx);
        const Sched sc = make_sched16(p->nx);
        std::string r;
        for (int i = 0; i < sc.count; ++i) r += (i ? "x" : "") + std::to_string(sc.r[i]);
        snprintf(tmp, sizeof tmp, "scaled16 %s n=%d radices=%s(radix-16 on %s) threads=%d lds=%d planes=%ld",
                 p->precision == FFT3D_FP16_SCALED ? "fp16" : "bf16", p->nx, r.c_str(), p->q16_valu ? "VALU" : "MFMA",
                 k.threads, k.lds_bytes,
                 (long)p->batch * p->nz);
        d = tmp;
    } else if (p->scheme == kFused) {
        const KernelInfo k = fused_info(p->nx);
        snprintf(tmp, sizeof tmp, "fused n=%d radices=%s threads=%d lds=%d grids=%d workgroups=%d lag=%d xcd_queues=%d",
                 p->nx, radices(p->nx).c_str(), k.threads, k.lds_bytes, p->batch, p->fused_grid, p->fused_lag,
                 p->fused_xcd);
        d = tmp;
    } else if (p->scheme == kCube) {
        const KernelInfo k = cube_info(p->nx);
        snprintf(tmp, sizeof tmp, "cube n=%d radices=%s threads=%d lds=%d grids=%d", p->nx,
                 radices(p->nx).c_str(), k.threads, k.lds_bytes, p->batch);
        d = tmp;
    } else if (p->scheme == kPlaneZ) {
        const KernelInfo a = plane_info(p->nx), b = axis_str_info(p->nz);
        snprintf(tmp, sizeof tmp, "plane n=%d radices=%s threads=%d lds=%d planes=%ld; z n=%d radices=%s threads=%d lds=%d",
                 p->nx, radices(p->nx).c_str(), a.threads, a.lds_bytes, (long)p->batch * p->nz, p->nz,
                 radices(p->nz).c_str(), b.threads, b.lds_bytes);
        d = tmp;
    } else {
        const KernelInfo a = axis_row_info(p->nx), b = axis_str_info(p->ny), c = axis_str_info(p->nz);
        snprintf(tmp, sizeof tmp, "axes x=%d(%s,t%d) y=%d(%s,t%d) z=%d(%s,t%d)", p->nx, radices(p->nx).c_str(),
                 a.threads, p->ny, radices(p->ny).c_str(), b.threads, p->nz, radices(p->nz).c_str(), c.threads);
        d = tmp;
    }
    d += p->direction < 0 ? " forward" : " inverse";
    if (p->cut_r2 > 0) {
        snprintf(tmp, sizeof tmp, " cutoff_r2=%.17g zplanes=%d sphere_points=%ld", p->cut_r2, p->n_zlist,
                 p->sphere_pts);
        d += tmp;
    }
    d += " kernels=";
    for (size_t i = 0; i < p->passes.size(); ++i) {
        static const char* names[] = {"k_cube",      "k_plane",    "k_plane_pf",     "k_axis_row",
                                      "k_axis_str",  "k_fused",    "k_q16_plane",    "k_q16_slab",
                                      "k_plane_pruned", "k_axis_str_pruned"};
        d += (i ? "," : "") + std::string(names[p->passes[i].kind]);
    }
    if (buf && len) {
        std::strncpy(buf, d.c_str(), len - 1);
        buf[len - 1] = 0;
    }
    return (int)d.size();
}

}  // extern "C"
