// ptg_tune.hip -- tile-shape autotuner (a6): one table per process of the launch shape
// each kernel class uses, filled by timing every candidate shape on the device.
//
// The drivers (ptg_plan.hip) ask tune_pick() for the shape of the class they are about to
// launch.  A TuneScope on the calling thread can force one candidate (timing) or make the
// drivers stop right before the launch (queries), so the tuner and the queries go through
// the same validation and kernel choice as ptg_fbm_2d / ptg_fbm_3d themselves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "ptg_internal.h"

namespace ptg {

bool TuneKey::operator<(const TuneKey &o) const
{
    return std::tie(kernel, smooth, f16, size_class, ladder) <
           std::tie(o.kernel, o.smooth, o.f16, o.size_class, o.ladder);
}

namespace {

std::mutex g_mu;
std::map<TuneKey, int> g_table;

struct ThreadTune {
    bool active = false, dry = false, picked = false;
    int force = 0, value = 0, dflt = 0;
    TuneKey key{};
};
thread_local ThreadTune t_tune;

int candidates(int kernel, int *out)
{
    switch (kernel) {
    case PTG_TUNE_GENERAL_2D:
        out[0] = 16, out[1] = 32, out[2] = 64, out[3] = 128;
        return 4;
    case PTG_TUNE_STRIP_2D:
    case PTG_TUNE_STRIP_3D:
        out[0] = 1, out[1] = 2, out[2] = 4;
        return 3;
    default:
        return 0;
    }
}

bool is_candidate(int kernel, int v)
{
    int c[PTG_TUNE_MAX_CANDIDATES];
    const int n = candidates(kernel, c);
    for (int i = 0; i < n; ++i)
        if (c[i] == v) return true;
    return false;
}

}  // namespace

int tune_pick(const TuneKey &k, int dflt)
{
    int v = dflt;
    if (t_tune.active && t_tune.force > 0 && is_candidate(k.kernel, t_tune.force)) {
        v = t_tune.force;
    } else {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(k);
        if (it != g_table.end()) v = it->second;
    }
    if (t_tune.active) {
        t_tune.picked = true;
        t_tune.key = k;
        t_tune.value = v;
        t_tune.dflt = dflt;
    }
    return v;
}

bool tune_dry() { return t_tune.active && t_tune.dry; }

TuneScope::TuneScope(bool dry, int force)
{
    t_tune = ThreadTune{};
    t_tune.active = true;
    t_tune.dry = dry;
    t_tune.force = force;
}
TuneScope::~TuneScope() { t_tune = ThreadTune{}; }
bool TuneScope::picked() const { return t_tune.picked; }
TuneKey TuneScope::key() const { return t_tune.key; }
int TuneScope::value() const { return t_tune.value; }
int TuneScope::dflt() const { return t_tune.dflt; }

int size_class(int64_t samples)
{
    int c = 0;
    while (c < 62 && (int64_t(1) << c) < samples) ++c;
    return c;
}

int ladder_class(const double *freq, int octaves)
{
    double fmax = 0.0;
    for (int o = 0; o < octaves; ++o) fmax = std::max(fmax, freq[o]);
    if (!(fmax > 0.0)) return 8;
    const int c = (int)std::floor(std::log2(1.0 / fmax));
    return std::min(std::max(c, 0), 8);
}

}  // namespace ptg

using namespace ptg;

namespace {

// A dense-field call on this thread inside a TuneScope; dims 2 or 3.
struct Call {
    const ptg_params *p;
    int64_t x0, y0, z0, nx, ny, nz, pitch;
    void *out;
    void *stream;
    int run() const
    {
        return p && p->dim == 3 ? ptg_fbm_3d(p, x0, y0, z0, nx, ny, nz, out, stream)
                                : ptg_fbm_2d(p, x0, y0, nx, ny, out, pitch, stream);
    }
};

// The class, current shape and untuned shape of a call (no launch).
int query(const Call &c, int32_t *kernel, int32_t *value, int32_t *dflt = nullptr)
{
    if (!kernel || !value) return fail(PTG_EINVAL, "NULL output pointer");
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return fail(PTG_EINVAL, "extents must be >= 1");
    Call d = c;
    d.out = reinterpret_cast<void *>(uintptr_t(256));  // never dereferenced: no launch in a dry scope
    d.stream = nullptr;
    TuneScope sc(true, 0);
    const int rc = d.run();
    if (rc != PTG_OK) return rc;
    if (!sc.picked()) return fail(PTG_EINVAL, "no kernel class chosen");
    *kernel = sc.key().kernel;
    *value = sc.value();
    if (dflt) *dflt = sc.dflt();
    return PTG_OK;
}

int set(const Call &c, int32_t value)
{
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return fail(PTG_EINVAL, "extents must be >= 1");
    Call d = c;
    d.out = reinterpret_cast<void *>(uintptr_t(256));
    d.stream = nullptr;
    TuneScope sc(true, 0);
    const int rc = d.run();
    if (rc != PTG_OK) return rc;
    if (!sc.picked() || !is_candidate(sc.key().kernel, value))
        return fail(PTG_EINVAL, "%d is not a shape of kernel class %d", value, sc.picked() ? sc.key().kernel : 0);
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[sc.key()] = value;
    return PTG_OK;
}

int tune(const Call &c, int32_t reps, ptg_tune_result *res)
{
    if (!res) return fail(PTG_EINVAL, "res is NULL");
    if (!c.out) return fail(PTG_EINVAL, "out_dev is NULL");
    if (reps <= 0) reps = 5;
    int32_t kernel = 0, current = 0, dflt = 0;
    int rc = query(c, &kernel, &current, &dflt);
    if (rc != PTG_OK) return rc;
    *res = ptg_tune_result{};
    res->kernel = kernel;
    res->default_value = dflt;
    int cand[PTG_TUNE_MAX_CANDIDATES];
    int n = candidates(kernel, cand);
    if (n == 0) {  // nothing to tune: time the one shape
        cand[0] = current;
        n = 1;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(c.stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PTG_EHIP, "hipEventCreate failed");
    }
    int best = 0;
    for (int i = 0; i < n && rc == PTG_OK; ++i) {
        TuneScope sc(false, cand[i]);
        rc = c.run();  // warm-up
        if (rc == PTG_OK && hipEventRecord(e0, s) != hipSuccess) rc = fail(PTG_EHIP, "hipEventRecord failed");
        for (int r = 0; r < reps && rc == PTG_OK; ++r) rc = c.run();
        if (rc == PTG_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(PTG_EHIP, "hipEventRecord failed");
        if (rc == PTG_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(PTG_EHIP, "hipEventSynchronize failed");
        float ms = 0.0f;
        if (rc == PTG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(PTG_EHIP, "event timing failed");
        res->candidates[i] = cand[i];
        res->us[i] = (double)ms * 1000.0 / reps;
        if (res->us[i] < res->us[best]) best = i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PTG_OK) return rc;
    res->n = n;
    res->value = cand[best];
    if (is_candidate(kernel, cand[best])) {
        TuneScope sc(true, 0);
        Call d = c;
        d.out = reinterpret_cast<void *>(uintptr_t(256));
        (void)d.run();
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[sc.key()] = cand[best];
    }
    return PTG_OK;
}

}  // namespace

extern "C" {

int ptg_tune_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out_dev, int64_t row_pitch,
                void *stream, int32_t reps, ptg_tune_result *res)
{
    if (!p || p->dim != 2) return fail(PTG_EINVAL, "ptg_tune_2d needs dim 2 parameters");
    return tune(Call{p, x0, y0, 0, nx, ny, 1, row_pitch, out_dev, stream}, reps, res);
}

int ptg_tune_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out_dev, void *stream, int32_t reps, ptg_tune_result *res)
{
    if (!p || p->dim != 3) return fail(PTG_EINVAL, "ptg_tune_3d needs dim 3 parameters");
    return tune(Call{p, x0, y0, z0, nx, ny, nz, nx, out_dev, stream}, reps, res);
}

int ptg_tune_query_2d(const ptg_params *p, int64_t nx, int64_t ny, int32_t *kernel, int32_t *value)
{
    if (!p || p->dim != 2) return fail(PTG_EINVAL, "needs dim 2 parameters");
    return query(Call{p, 0, 0, 0, nx, ny, 1, nx, nullptr, nullptr}, kernel, value);
}

int ptg_tune_query_3d(const ptg_params *p, int64_t nx, int64_t ny, int64_t nz, int32_t *kernel, int32_t *value)
{
    if (!p || p->dim != 3) return fail(PTG_EINVAL, "needs dim 3 parameters");
    return query(Call{p, 0, 0, 0, nx, ny, nz, nx, nullptr, nullptr}, kernel, value);
}

int ptg_tune_set_2d(const ptg_params *p, int64_t nx, int64_t ny, int32_t value)
{
    if (!p || p->dim != 2) return fail(PTG_EINVAL, "needs dim 2 parameters");
    return set(Call{p, 0, 0, 0, nx, ny, 1, nx, nullptr, nullptr}, value);
}

int ptg_tune_set_3d(const ptg_params *p, int64_t nx, int64_t ny, int64_t nz, int32_t value)
{
    if (!p || p->dim != 3) return fail(PTG_EINVAL, "needs dim 3 parameters");
    return set(Call{p, 0, 0, 0, nx, ny, nz, nx, nullptr, nullptr}, value);
}

void ptg_tune_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

// The device a table belongs to: its architecture name and compute-unit count ("none" when
// no device is visible, e.g. on a build host).
static void device_identity(char *arch, size_t n, int *cus)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::snprintf(arch, n, "%s", prop.gcnArchName);
        for (char *c = arch; *c; ++c)
            if (*c == ' ' || *c == '\n') *c = '_';
        *cus = prop.multiProcessorCount;
    } else {
        (void)hipGetLastError();
        std::snprintf(arch, n, "none");
        *cus = 0;
    }
}

int ptg_tune_save(const char *path)
{
    if (!path) return fail(PTG_EINVAL, "path is NULL");
    char arch[256];
    int cus = 0;
    device_identity(arch, sizeof(arch), &cus);
    std::FILE *f = std::fopen(path, "w");
    if (!f) return fail(PTG_ENOENT, "cannot open %s for writing", path);
    std::fprintf(f, "ptg_tune 1 %s %d\n", arch, cus);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto &kv : g_table)
            std::fprintf(f, "%d %d %d %d %d %d\n", kv.first.kernel, kv.first.smooth, kv.first.f16,
                         kv.first.size_class, kv.first.ladder, kv.second);
    }
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    return ok ? PTG_OK : fail(PTG_ENOENT, "writing %s failed", path);
}

int ptg_tune_load(const char *path, int32_t *loaded)
{
    if (!path) return fail(PTG_EINVAL, "path is NULL");
    if (loaded) *loaded = 0;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return fail(PTG_ENOENT, "cannot open %s", path);
    char arch[256], farch[256];
    int cus = 0, fcus = 0, ver = 0;
    device_identity(arch, sizeof(arch), &cus);
    if (std::fscanf(f, "ptg_tune %d %255s %d", &ver, farch, &fcus) != 3 || ver != 1) {
        std::fclose(f);
        return fail(PTG_EINVAL, "%s is not a tuning table", path);
    }
    // entries of another device are skipped; every entry is validated before any is kept
    std::map<TuneKey, int> rows;
    int k, sm, f16, sc, lad, v, n;
    while ((n = std::fscanf(f, "%d %d %d %d %d %d", &k, &sm, &f16, &sc, &lad, &v)) == 6) {
        if (!is_candidate(k, v) || sm < 0 || sm > 64 || (f16 != 0 && f16 != 1) || sc < 0 || sc > 62 || lad < 0 ||
            lad > 64) {
            std::fclose(f);
            return fail(PTG_EINVAL, "%s: bad entry", path);
        }
        rows[TuneKey{k, sm, f16, sc, lad}] = v;
    }
    const bool clean = n == EOF;
    std::fclose(f);
    if (!clean) return fail(PTG_EINVAL, "%s: malformed entry", path);
    if (std::strcmp(arch, farch) != 0 || cus != fcus) return PTG_OK;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto &kv : rows) g_table[kv.first] = kv.second;
    }
    if (loaded) *loaded = (int32_t)rows.size();
    return PTG_OK;
}

}  // extern "C"
