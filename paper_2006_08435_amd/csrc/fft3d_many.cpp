// Heterogeneous batches: fft3d_plan_many / fft3d_exec_many, the work-list
// builder and the schedule autotuner with its JSON cache.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <deque>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "plan_internal.hpp"

using namespace fft3d;

namespace {

int device_cus(int dev)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    return cus;
}

// Work list: for every grid its plane items, and its slab items at least
// `lag` list positions after its last plane item.  Grids of the groups
// marked in `skip` (if given) are left out.
std::vector<unsigned> build_items(const std::vector<ManyGrid>& grids, int threads, long lag,
                                  const bool* skip = nullptr)
{
    std::vector<unsigned> out;
    std::deque<std::pair<long, int>> ready;   // (list length when the planes ended, grid)
    auto emit_slabs = [&](int g) {
        const int n = grids[g].n, per = many_per_item(n, threads);
        for (int i = 0; i < n; i += per) out.push_back(many_item((unsigned)g, 1u, (unsigned)i));
    };
    auto flush = [&]() {
        while (!ready.empty() && (long)out.size() - ready.front().first >= lag) {
            emit_slabs(ready.front().second);
            ready.pop_front();
        }
    };
    // largest grids first: their plane-then-slab chains are the longest, and
    // the many short items of the small grids fill the end of the list
    std::vector<int> order(grids.size());
    for (int g = 0; g < (int)grids.size(); ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return grids[a].n > grids[b].n; });
    for (const int g : order) {
        if (skip && skip[grids[g].group]) continue;
        const int n = grids[g].n, per = many_per_item(n, threads);
        for (int i = 0; i < n; i += per) {
            out.push_back(many_item((unsigned)g, 0u, (unsigned)i));
            flush();
        }
        ready.push_back({(long)out.size(), g});
    }
    while (!ready.empty()) {
        emit_slabs(ready.front().second);
        ready.pop_front();
    }
    return out;
}

size_t plan_lds(const ManyPlan& mp, int threads, const bool* skip = nullptr)
{
    size_t m = 0;
    for (int g = 0; g < mp.ngroups; ++g) {
        if (skip && skip[g]) continue;
        const size_t b = many_lds_bytes(mp.n[g], threads);
        m = b > m ? b : m;
    }
    return m;
}

// Apply a (threads, chunk) schedule: occupancy, grid, work list.  threads
// 0 selects the grouped mode (nothing to prepare); threads < 0 the hybrid
// mode with |threads| threads for the persistent part: a group whose plane
// pass alone fills every compute unit (batch * n planes >= the plane
// kernel's resident workgroups) runs its two plain passes, the others share
// one persistent launch.
int apply_schedule(fft3d_plan_s* p, int threads, int chunk)
{
    ManyPlan& mp = p->mp;
    if (threads == 0) {
        mp.threads = 0;
        mp.chunk = 1;
        mp.hybrid = false;
        return FFT3D_OK;
    }
    const bool hybrid = threads < 0;
    const int t = hybrid ? -threads : threads;
    const int cus = device_cus(p->device);
    bool big[kMaxGroups] = {};
    if (hybrid)
        for (int g = 0; g < mp.ngroups; ++g)
            big[g] = (long)mp.batch[g] * mp.n[g] >= (long)plane_pf_blocks_per_cu(mp.n[g]) * cus;
    const bool* skip = hybrid ? big : nullptr;
    const size_t lds = plan_lds(mp, t, skip);
    long nitems = 0;
    int grid = 1;
    if (lds > 0) {   // at least one group runs in the persistent launch
        const int per_cu = many_blocks_per_cu(t, lds);
        if (per_cu < 1) return FFT3D_E_UNSUPPORTED;
        const int resident = per_cu * cus;
        const long lag = (long)resident * chunk + resident;
        std::vector<unsigned> items = build_items(mp.grids, t, lag, skip);
        if ((long)items.size() > mp.items_cap) return FFT3D_E_INVALID_ARG;
        if (hipMemcpy(mp.d_items, items.data(), items.size() * sizeof(unsigned), hipMemcpyHostToDevice) !=
            hipSuccess) {
            (void)hipGetLastError();
            return FFT3D_E_LAUNCH;
        }
        nitems = (long)items.size();
        const long claims = (nitems + chunk - 1) / chunk;
        grid = (int)(claims < resident ? claims : resident);
    }
    mp.nitems = nitems;
    mp.threads = t;
    mp.chunk = chunk;
    mp.lds = lds;
    mp.grid = grid;
    mp.hybrid = hybrid;
    for (int g = 0; g < kMaxGroups; ++g) mp.big[g] = big[g];
    return FFT3D_OK;
}

// Grouped mode: for each group its plane pass and its z pass, as a dense
// plan of that group would launch them (the persistent kernel's alternative
// when the groups are few and large).  only (if given): the groups to run.
hipError_t launch_grouped(const fft3d_plan_s* p, const void* const* in, void* const* out, hipStream_t st,
                          const bool* only = nullptr)
{
    const ManyPlan& mp = p->mp;
    const int cus = device_cus(p->device);
    hipError_t e = hipSuccess;
    for (int g = 0; g < mp.ngroups && e == hipSuccess; ++g) {
        if (only && !only[g]) continue;
        const int n = mp.n[g], kind = mp.kind[g], zl = mp.zlines[g] ? mp.zlines[g] : kAxisLines;
        const long planes = (long)mp.batch[g] * n, resident = (long)plane_pf_blocks_per_cu(n) * cus;
        const int grid = (int)(planes < resident ? planes : resident);
        const float2* tw = p->d_tw + (kind == 2 ? mp.twoff_alt[n] : mp.twoff_host[n]);
        const float2* src = static_cast<const float2*>(in[g]);
        float2* dst = static_cast<float2*>(out[g]);
        if (kind == 0) {
            e = plane_pf_fn(n, p->direction)(src, dst, tw, planes, grid, 0, nullptr, nullptr, n, true, st);
        } else {
            const PlaneVarFn f = plane_variant_fn(n, p->direction, kind);
            e = f ? f(src, dst, tw, planes, grid, true, st) : hipErrorInvalidValue;
        }
        const long vol = (long)n * n * n;
        const AxisMap zmap{(long)mp.batch[g] * n * n, n, n, vol, (long)n, (long)n * n};
        if (e == hipSuccess && n > 1) {
            if (kind == 0 && zl == kAxisLines) {
                e = axis_str_fn(n, p->direction)(dst, dst, tw, zmap, 0, nullptr, nullptr, 0, st);
            } else {
                const AxisVarFn f = axis_variant_fn(n, p->direction, kind, zl);
                e = f ? f(dst, dst, tw, zmap, st) : hipErrorInvalidValue;
            }
        }
    }
    return e;
}

hipError_t run_many(const fft3d_plan_s* p, const void* const* in, void* const* out, hipStream_t st);

ManyArgs make_args(const fft3d_plan_s* p, const void* const* in, void* const* out)
{
    ManyArgs a{};
    for (int g = 0; g < p->mp.ngroups; ++g) {
        a.in[g] = static_cast<const float2*>(in[g]);
        a.out[g] = static_cast<float2*>(out[g]);
    }
    a.grids = p->mp.d_grids;
    a.items = p->mp.d_items;
    a.nitems = p->mp.nitems;
    a.tw = p->d_tw;
    a.tw_off = p->mp.d_twoff;
    a.ctl = p->ctl;
    a.chunk = p->mp.chunk;
    a.ngrids = (int)p->mp.grids.size();
    return a;
}

// ----------------------------------------------------------- tuning cache --

std::string cache_path()
{
    if (const char* e = std::getenv("FFT3D_TUNE_CACHE")) return e;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/fft3d/tune.json";
}

std::string cache_key(const fft3d_plan_s* p)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << "|many|" << p->direction << "|";
    for (int g = 0; g < p->mp.ngroups; ++g) k << (g ? "," : "") << p->mp.n[g] << "x" << p->mp.batch[g];
    return k.str();
}

// The cache file holds one entry per line:
//   "key": {"threads": T, "chunk": K, "ms": t, "radix": "k0,k1,...", "zlines": "l0,l1,..."},
// with one radix order (0 default, 2 alternative) and z-tile width per group.
// Lines that do not parse are ignored (a corrupt file means "no entries");
// an entry without the per-group fields selects the default variants.
std::map<std::string, std::string> cache_read()
{
    std::map<std::string, std::string> m;
    std::ifstream f(cache_path());
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"'), b = a == std::string::npos ? a : line.find('"', a + 1);
        const size_t c = b == std::string::npos ? b : line.find('{', b);
        const size_t d = c == std::string::npos ? c : line.find('}', c);
        if (d == std::string::npos) continue;
        m[line.substr(a + 1, b - a - 1)] = line.substr(c, d - c + 1);
    }
    return m;
}

// Per-group list "a,b,c" of `count` integers each in `ok`; false otherwise.
bool parse_list(const std::string& v, const char* field, int count, int* out, bool (*ok)(int))
{
    const std::string tag = std::string("\"") + field + "\": \"";
    const size_t a = v.find(tag);
    if (a == std::string::npos) return false;
    const size_t b = v.find('"', a + tag.size());
    if (b == std::string::npos) return false;
    std::stringstream ss(v.substr(a + tag.size(), b - a - tag.size()));
    std::string item;
    int k = 0;
    while (std::getline(ss, item, ',')) {
        char* end = nullptr;
        const long x = std::strtol(item.c_str(), &end, 10);
        if (k >= count || end == item.c_str() || *end != 0 || !ok((int)x)) return false;
        out[k++] = (int)x;
    }
    return k == count;
}

bool kind_ok(int k) { return k == 0 || k == 2; }
bool lines_ok(int l) { return l == 32 || l == 64; }

bool cache_lookup(const std::string& key, int ngroups, int& threads, int& chunk, int* kind, int* zlines)
{
    const auto m = cache_read();
    const auto it = m.find(key);
    if (it == m.end()) return false;
    int t = 0, c = 0;
    double ms = 0;
    if (std::sscanf(it->second.c_str(), "{\"threads\": %d, \"chunk\": %d, \"ms\": %lf", &t, &c, &ms) != 3) return false;
    if ((t != 0 && t != 512 && t != 1024 && t != -512 && t != -1024) || c < 1 || c > 64) return false;
    int k[kMaxGroups], l[kMaxGroups];
    if (parse_list(it->second, "radix", ngroups, k, kind_ok) && parse_list(it->second, "zlines", ngroups, l, lines_ok)) {
        for (int g = 0; g < ngroups; ++g) {
            kind[g] = k[g];
            zlines[g] = l[g];
        }
    }
    threads = t;
    chunk = c;
    return true;
}

void cache_store(const std::string& key, const ManyPlan& mp, double ms)
{
    auto m = cache_read();
    std::ostringstream v;
    char head[128];
    std::snprintf(head, sizeof head, "{\"threads\": %d, \"chunk\": %d, \"ms\": %.5f, \"radix\": \"",
                  mp.hybrid ? -mp.threads : mp.threads, mp.chunk, ms);
    v << head;
    for (int g = 0; g < mp.ngroups; ++g) v << (g ? "," : "") << mp.kind[g];
    v << "\", \"zlines\": \"";
    for (int g = 0; g < mp.ngroups; ++g) v << (g ? "," : "") << (mp.zlines[g] ? mp.zlines[g] : kAxisLines);
    v << "\"}";
    m[key] = v.str();
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash), cur;
        std::stringstream ss(dir);
        std::string part;
        while (std::getline(ss, part, '/')) {
            cur += part + "/";
            (void)mkdir(cur.c_str(), 0755);
        }
    }
    std::ofstream f(path + ".tmp");
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) f << "\"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

// Time every candidate on scratch buffers; keep the fastest.  Each candidate
// is timed in kTuneRounds rounds, the candidates interleaved within a round,
// and scored by its fastest round: with one timing per candidate the 16x4
// order won for a 256 x 64^3 group in two of four runs, and the whole batch
// then ran 3% slower than with 8x8 (clock and cache state drift between
// consecutive timings).
constexpr int kTuneRounds = 3;

int tune(fft3d_plan_s* p)
{
    ManyPlan& mp = p->mp;
    std::vector<void*> bufs(mp.ngroups, nullptr);
    int rc = FFT3D_OK;
    for (int g = 0; g < mp.ngroups && rc == FFT3D_OK; ++g) {
        const size_t b = (size_t)mp.batch[g] * mp.n[g] * mp.n[g] * mp.n[g] * sizeof(float2);
        if (hipMalloc(&bufs[g], b) != hipSuccess || hipMemset(bufs[g], 0, b) != hipSuccess) rc = FFT3D_E_ALLOC;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == FFT3D_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = FFT3D_E_LAUNCH;
    auto time_runs = [&](const bool* only, float& ms_out) {
        const void* const* ib = (const void* const*)bufs.data();
        void* const* ob = bufs.data();
        bool ok = true;
        for (int w = 0; w < 2 && ok; ++w)
            ok = (only ? launch_grouped(p, ib, ob, nullptr, only) : run_many(p, ib, ob, nullptr)) == hipSuccess;
        ok = ok && hipEventRecord(e0, nullptr) == hipSuccess;
        for (int r = 0; r < 5 && ok; ++r)
            ok = (only ? launch_grouped(p, ib, ob, nullptr, only) : run_many(p, ib, ob, nullptr)) == hipSuccess;
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) (void)hipGetLastError();
        ms_out = ms / 5;
        return ok;
    };
    // 1. per group: the radix order and z-tile width of its plain passes,
    //    timed on that group alone
    const int cand_k[] = {0, 2}, cand_l[] = {kAxisLines, 32};
    for (int g = 0; g < mp.ngroups && rc == FFT3D_OK; ++g) {
        bool only[kMaxGroups] = {};
        only[g] = true;
        float gms[2][2] = {{1e30f, 1e30f}, {1e30f, 1e30f}};
        for (int round = 0; round < kTuneRounds; ++round)
            for (int ik = 0; ik < 2; ++ik)
                for (int il = 0; il < 2; ++il) {
                    mp.kind[g] = cand_k[ik];
                    mp.zlines[g] = cand_l[il];
                    float ms = 0.f;
                    if (time_runs(only, ms) && ms < gms[ik][il]) gms[ik][il] = ms;
                }
        int bk = 0, bl = 0;
        for (int ik = 0; ik < 2; ++ik)
            for (int il = 0; il < 2; ++il)
                if (gms[ik][il] < gms[bk][bl]) {
                    bk = ik;
                    bl = il;
                }
        mp.kind[g] = cand_k[bk];
        mp.zlines[g] = cand_l[bl];
    }
    // 2. the launch mode: the grouped mode, then the persistent kernel's and
    //    the hybrid mode's (threads, chunk)
    double best = 1e30;
    int bt = mp.threads, bc = mp.chunk;
    const int cand_t[] = {0, 1024, 512, -1024, -512};
    const int cand_c[] = {1, 2, 4, 8};
    float sms[5][4];
    for (auto& row : sms)
        for (float& v : row) v = 1e30f;
    for (int round = 0; round < kTuneRounds && rc == FFT3D_OK; ++round)
        for (int it = 0; it < 5; ++it)
            for (int ic = 0; ic < 4; ++ic) {
                const int t = cand_t[it], c = cand_c[ic];
                if (t == 0 && c != 1) continue;
                if (apply_schedule(p, t, c) != FFT3D_OK) continue;
                float ms = 0.f;
                if (time_runs(nullptr, ms) && ms < sms[it][ic]) sms[it][ic] = ms;
            }
    for (int it = 0; it < 5; ++it)
        for (int ic = 0; ic < 4; ++ic)
            if (sms[it][ic] < best) {
                best = sms[it][ic];
                bt = cand_t[it];
                bc = cand_c[ic];
            }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (rc != FFT3D_OK) return rc;
    rc = apply_schedule(p, bt, bc);
    if (rc == FFT3D_OK) {
        mp.tuned = true;
        mp.tuned_ms = best;
        cache_store(cache_key(p), mp, best);
    }
    return rc;
}

hipError_t run_many(const fft3d_plan_s* p, const void* const* in, void* const* out, hipStream_t st)
{
    if (p->mp.threads == 0) return launch_grouped(p, in, out, st);
    hipError_t e = hipSuccess;
    if (p->mp.hybrid) e = launch_grouped(p, in, out, st, p->mp.big);
    if (e != hipSuccess || p->mp.nitems == 0) return e;
    const ManyArgs a = make_args(p, in, out);
    return launch_many(a, p->direction, p->mp.threads, p->mp.grid, p->mp.lds, st);
}

void free_plan(fft3d_plan_s* p)
{
    if (!p) return;
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->ctl) (void)hipFree(p->ctl);
    if (p->mp.d_grids) (void)hipFree(p->mp.d_grids);
    if (p->mp.d_items) (void)hipFree(p->mp.d_items);
    if (p->mp.d_twoff) (void)hipFree(p->mp.d_twoff);
    delete p;
}

}  // namespace

extern "C" {

fft3d_plan_t fft3d_plan_many(int count, const int* nx, const int* ny, const int* nz, const int* batch, int precision,
                             int direction)
{
    clear_error();
    if (count < 1 || count > kMaxGroups || !nx || !ny || !nz || !batch) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    if (precision != FFT3D_FP32 && precision != FFT3D_FP16_SCALED && precision != FFT3D_BF16_SCALED) {
        set_error(FFT3D_E_INVALID_ARG);
        return nullptr;
    }
    if (direction != FFT3D_FORWARD && direction != FFT3D_INVERSE) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    long total = 0, ngrids = 0;
    for (int g = 0; g < count; ++g) {
        if (nx[g] < 1 || ny[g] < 1 || nz[g] < 1 || batch[g] < 1) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
        if (!size_supported(nx[g]) || !size_supported(ny[g]) || !size_supported(nz[g])) {
            set_error(FFT3D_E_UNSUPPORTED_SIZE);
            return nullptr;
        }
        if (nx[g] != ny[g] || ny[g] != nz[g] || !many_size_ok(nx[g])) { set_error(FFT3D_E_UNSUPPORTED); return nullptr; }
        total += (long)batch[g] * nx[g] * nx[g] * nx[g];
        ngrids += batch[g];
    }
    if (total > (1L << 36) || ngrids > (1L << 23)) { set_error(FFT3D_E_INVALID_ARG); return nullptr; }
    if (precision != FFT3D_FP32) { set_error(FFT3D_E_UNSUPPORTED); return nullptr; }
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        set_error(FFT3D_E_NO_DEVICE);
        return nullptr;
    }
    fft3d_plan_s* p = new (std::nothrow) fft3d_plan_s{};
    if (!p) { set_error(FFT3D_E_ALLOC); return nullptr; }
    p->many = true;
    p->precision = precision;
    p->direction = direction;
    p->device = dev;
    p->batch = (int)ngrids;
    p->nx = p->ny = p->nz = nx[0];
    p->vol = total / (ngrids ? ngrids : 1);
    ManyPlan& mp = p->mp;
    mp.ngroups = count;
    std::vector<float2> tab;
    std::vector<int> twoff(129, 0);
    for (int g = 0; g < count; ++g) {
        mp.n[g] = nx[g];
        mp.batch[g] = batch[g];
        for (int b = 0; b < batch[g]; ++b) mp.grids.push_back({nx[g], g, (long)b * nx[g] * nx[g] * nx[g]});
        bool seen = false;
        for (int h = 0; h < g; ++h) seen = seen || mp.n[h] == nx[g];
        if (!seen) {
            twoff[nx[g]] = (int)tab.size();
            mp.twoff_host[nx[g]] = (int)tab.size();
            const std::vector<float2> t = twiddles(nx[g], direction);
            tab.insert(tab.end(), t.begin(), t.end());
            if (tab.size() % 2) tab.push_back(make_float2(0.f, 0.f));
            // the alternative radix order's table (tuner candidate)
            mp.twoff_alt[nx[g]] = (int)tab.size();
            const std::vector<float2> ta = twiddles(nx[g], direction, 2);
            tab.insert(tab.end(), ta.begin(), ta.end());
            if (tab.size() % 2) tab.push_back(make_float2(0.f, 0.f));
        }
    }
    if (tab.empty()) tab.push_back(make_float2(0.f, 0.f));
    // capacity: one item per plane and slab at the smallest per-item count
    long cap = 0;
    for (const ManyGrid& gd : mp.grids) cap += 2L * gd.n;
    mp.items_cap = cap;
    const size_t cb = sizeof(FusedCtl) + sizeof(unsigned) * (size_t)ngrids;
    bool ok = !env_flag("FFT3D_TEST_FAIL_ALLOC") && hipMalloc((void**)&p->d_tw, tab.size() * sizeof(float2)) == hipSuccess &&
              hipMalloc((void**)&mp.d_grids, mp.grids.size() * sizeof(ManyGrid)) == hipSuccess &&
              hipMalloc((void**)&mp.d_items, cap * sizeof(unsigned)) == hipSuccess &&
              hipMalloc((void**)&mp.d_twoff, twoff.size() * sizeof(int)) == hipSuccess &&
              hipMalloc((void**)&p->ctl, cb) == hipSuccess;
    ok = ok && hipMemcpy(p->d_tw, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(mp.d_grids, mp.grids.data(), mp.grids.size() * sizeof(ManyGrid), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(mp.d_twoff, twoff.data(), twoff.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(p->ctl, 0, cb) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_plan(p);
        set_error(FFT3D_E_ALLOC);
        return nullptr;
    }
    int threads = 1024, chunk = 1;
    for (int g = 0; g < count; ++g) mp.zlines[g] = kAxisLines;
    const bool cached = cache_lookup(cache_key(p), count, threads, chunk, mp.kind, mp.zlines);
    int rc = apply_schedule(p, threads, chunk);
    if (rc == FFT3D_OK && !cached && env_flag("FFT3D_TUNE")) rc = tune(p);
    if (rc != FFT3D_OK) {
        free_plan(p);
        set_error(rc);
        return nullptr;
    }
    mp.tuned = mp.tuned || cached;
    return p;
}

int fft3d_exec_many(fft3d_plan_t p, const void* const* in, void* const* out, fft3d_stream_t stream)
{
    if (!p || !in || !out) return FFT3D_E_INVALID_ARG;
    if (!p->many) return FFT3D_E_INVALID_ARG;
    for (int g = 0; g < p->mp.ngroups; ++g) {
        if (!in[g] || !out[g]) return FFT3D_E_INVALID_ARG;
        if (((uintptr_t)in[g] % 16) || ((uintptr_t)out[g] % 16)) return FFT3D_E_ALIGNMENT;
    }
    if (run_many(p, in, out, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return FFT3D_E_LAUNCH;
    }
    return FFT3D_OK;
}

int fft3d_plan_set_schedule(fft3d_plan_t p, int threads, int chunk)
{
    if (!p || !p->many || (threads != 0 && threads != 512 && threads != 1024 && threads != -512 && threads != -1024) ||
        chunk < 1 || chunk > 64)
        return FFT3D_E_INVALID_ARG;
    const int rc = apply_schedule(p, threads, chunk);
    if (rc == FFT3D_OK) p->mp.tuned = false;   // a forced schedule, not the tuner's
    return rc;
}

int fft3d_plan_set_group_schedule(fft3d_plan_t p, int group, int radix_order, int z_lines)
{
    if (!p || !p->many || group < 0 || group >= p->mp.ngroups || (radix_order != 0 && radix_order != 1) ||
        (z_lines != 32 && z_lines != 64))
        return FFT3D_E_INVALID_ARG;
    p->mp.kind[group] = radix_order ? 2 : 0;
    p->mp.zlines[group] = z_lines;
    p->mp.tuned = false;
    return FFT3D_OK;
}

int fft3d_plan_tune(fft3d_plan_t p)
{
    if (!p || !p->many) return FFT3D_E_INVALID_ARG;
    return tune(p);
}

}  // extern "C"

namespace fft3d {

int many_describe(fft3d_plan_t p, char* buf, size_t len)
{
    std::ostringstream d;
    d << "many groups=";
    for (int g = 0; g < p->mp.ngroups; ++g) d << (g ? "," : "") << p->mp.n[g] << "^3x" << p->mp.batch[g];
    if (p->mp.threads == 0) {
        d << " mode=grouped" << (p->mp.tuned ? " tuned" : " default") << (p->direction < 0 ? " forward" : " inverse")
          << " kernels=k_plane_pf,k_axis_str per group";
    } else if (p->mp.hybrid) {
        d << " mode=hybrid grouped=";
        bool first = true;
        for (int g = 0; g < p->mp.ngroups; ++g)
            if (p->mp.big[g]) {
                d << (first ? "" : ",") << p->mp.n[g] << "^3x" << p->mp.batch[g];
                first = false;
            }
        if (first) d << "none";
        d << " threads=" << p->mp.threads << " chunk=" << p->mp.chunk << " workgroups=" << p->mp.grid
          << " lds=" << p->mp.lds << " items=" << p->mp.nitems << (p->mp.tuned ? " tuned" : " default")
          << (p->direction < 0 ? " forward" : " inverse") << " kernels=k_plane_pf,k_axis_str per big group + k_many";
    } else {
        d << " mode=persistent threads=" << p->mp.threads << " chunk=" << p->mp.chunk << " workgroups=" << p->mp.grid
          << " lds=" << p->mp.lds << " items=" << p->mp.nitems << (p->mp.tuned ? " tuned" : " default")
          << (p->direction < 0 ? " forward" : " inverse") << " kernels=k_many";
    }
    if (p->mp.threads == 0 || p->mp.hybrid) {
        d << " radix=";
        for (int g = 0; g < p->mp.ngroups; ++g) {
            const Sched sc = make_sched_kind(p->mp.n[g], p->mp.kind[g]);
            d << (g ? "," : "");
            for (int i = 0; i < sc.count; ++i) d << (i ? "x" : "") << sc.r[i];
        }
        d << " zlines=";
        for (int g = 0; g < p->mp.ngroups; ++g) d << (g ? "," : "") << (p->mp.zlines[g] ? p->mp.zlines[g] : kAxisLines);
    }
    const std::string s = d.str();
    if (buf && len) {
        std::strncpy(buf, s.c_str(), len - 1);
        buf[len - 1] = 0;
    }
    return (int)s.size();
}

}  // namespace fft3d
