// Host runtime: errors, device memory, the harmonic table, batch layout and
// launch, HIP graph capture, and the tile autotuner.
#include "runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/stat.h>

namespace mte {

// ---------------------------------------------------------------- errors
static thread_local std::string t_err = "no error";

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? MTE_ENOMEM : MTE_EDEVICE, "%s failed: %s", what,
                hipGetErrorString(e));
}

const char *last_error() { return t_err.c_str(); }

// ---------------------------------------------------------------- memory
// Block sizes: 64 KiB steps below 16 MiB, 2 MiB steps up to 256 MiB, and
// above that four size classes per octave (2^k times 1, 1.25, 1.5, 1.75), so
// that batches of slightly different sizes reuse each other's blocks: a new
// block of many GB costs about 11 ms per GB to allocate and 6 ms per GB to
// free, and a served mix of unrelated requests otherwise kept reallocating.
static size_t round_size(size_t b) {
    if (b >= (size_t(256) << 20)) {
        size_t o = size_t(1) << (63 - __builtin_clzll((unsigned long long)b));   // 2^k <= b
        const size_t q = o / 4;
        return (b + q - 1) / q * q;
    }
    const size_t g = b < (16u << 20) ? (64u << 10) : (2u << 20);
    return (b + g - 1) / g * g;
}

// Released blocks stay cached for reuse up to half of the device's memory
// (a block released past that is freed), and a new block is taken
// only with kDeviceReserve of device memory left beside it (else the cache is
// freed first): the HIP runtime allocates kernels' scratch (spill) memory on
// its own, and a device filled by cached blocks leaves it none, which aborts
// the queue.
constexpr size_t kDeviceReserve = size_t(4) << 30;

void DeviceAllocator::free_cached_locked() {
    for (auto &kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached_ = 0;
}

void *DeviceAllocator::alloc(size_t bytes) {
    bytes = round_size(bytes ? bytes : 1);
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.lower_bound(bytes);
    void *p = nullptr;
    size_t got = bytes;
    if (it != free_.end() && it->first <= bytes + bytes / 4 + (size_t(64) << 20)) {
        p = it->second;
        got = it->first;
        cached_ -= got;
        free_.erase(it);
        live_[p] = got;
        in_use_ += got;
        peak_ = std::max(peak_, in_use_);
        return p;
    }
    size_t dev_free = 0, dev_total = 0;
    if (!free_.empty() && hipMemGetInfo(&dev_free, &dev_total) == hipSuccess && dev_free < bytes + kDeviceReserve)
        free_cached_locked();
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        free_cached_locked();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    live_[p] = got;
    in_use_ += got;
    peak_ = std::max(peak_, in_use_);
    return p;
}

void DeviceAllocator::release(void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    const size_t got = it != live_.end() ? it->second : round_size(bytes ? bytes : 1);
    if (it != live_.end()) live_.erase(it);
    in_use_ -= got;
    if (cache_cap_ == 0) {
        size_t dev_free = 0, dev_total = 0;
        cache_cap_ = hipMemGetInfo(&dev_free, &dev_total) == hipSuccess ? dev_total / 2 : size_t(16) << 30;
    }
    if (cached_ + got > cache_cap_) {
        (void)hipFree(p);
        return;
    }
    cached_ += got;
    free_.emplace(got, p);
}

void DeviceAllocator::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    free_cached_locked();
}

DevBuf::~DevBuf() { reset(); }

void DevBuf::reset() {
    if (p) ctx().alloc.release(p, bytes);
    p = nullptr;
    bytes = 0;
}

int DevBuf::ensure(size_t n) {
    if (n <= bytes && p) return MTE_OK;
    if (p) ctx().alloc.release(p, bytes);
    p = ctx().alloc.alloc(n);
    bytes = p ? n : 0;
    return p ? MTE_OK : fail(MTE_ENOMEM, "device allocation of %zu bytes failed", n);
}

HostBuf::~HostBuf() { reset(); }

void HostBuf::reset() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

int HostBuf::ensure(size_t n) {
    if (n <= bytes && p) return MTE_OK;
    // grow to the next power of two (at least 1 MiB): pinned allocations are
    // slow and freeing one can wait for the device, so a buffer that keeps
    // growing by a little (launch tables, result staging of the request
    // loop's batches) is reallocated only a few times
    size_t want = size_t(1) << 20;
    while (want < n) want <<= 1;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    MTE_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
    bytes = want;
    return MTE_OK;
}

// ---------------------------------------------------------------- context
Ctx &ctx() {
    static Ctx c;
    return c;
}

static int harm_locked(int64_t n);
static std::string default_tune_file();
static void load_tune_file_locked();

static int init_locked(int device, size_t budget) {
    Ctx &c = ctx();
    if (c.inited) {
        if (device != c.device) return fail(MTE_EINVAL, "already initialised on device %d", c.device);
        MTE_HIP(hipSetDevice(c.device));
        if (budget) c.budget = budget;
        return MTE_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(MTE_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) return fail(MTE_EINVAL, "device %d out of range (%d devices)", device, n);
    MTE_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    MTE_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MTE_EDEVICE, "libmte is built for gfx950, device is %s", prop.gcnArchName);
    c.device = device;
    c.n_cu = prop.multiProcessorCount;
    c.arch = prop.gcnArchName;
    if (size_t colon = c.arch.find(':'); colon != std::string::npos) c.arch.resize(colon);
    c.tune_file = default_tune_file();
    load_tune_file_locked();
    size_t fr = 0, tot = 0;
    MTE_HIP(hipMemGetInfo(&fr, &tot));
    c.budget = budget ? budget : (size_t)(0.9 * (double)fr);
    MTE_HIP(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
    MTE_HIP(hipStreamCreateWithFlags(&c.side_stream, hipStreamNonBlocking));
    // set-up work of the allocation-free call: the harmonic table (2^20
    // entries) and the address of its static scratch array on this device
    int rc;
    if ((rc = harm_locked(int64_t(1) << 20))) return rc;
    if ((rc = noalloc_bind(device))) return rc;
    c.inited = true;
    return MTE_OK;
}

int init_device(int device, size_t budget) {
    std::lock_guard<std::mutex> lk(ctx().mu);
    return init_locked(device, budget);
}

int ensure_init() {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.inited) {
        MTE_HIP(hipSetDevice(c.device));
        return MTE_OK;
    }
    return init_locked(0, 0);
}

double harmonic_host(int64_t n) {
    double h = 0.0;
    for (int64_t m = 1; m <= n; ++m) h += 1.0 / (double)m;
    return h;
}

static int harm_locked(int64_t n) {
    Ctx &c = ctx();
    if (c.harm && n <= c.harm_n) return MTE_OK;
    int64_t cap = std::max<int64_t>(n, std::max<int64_t>(2 * c.harm_n, int64_t(1) << 20));
    std::vector<double> h((size_t)cap + 1);
    h[0] = 0.0;
    for (int64_t m = 1; m <= cap; ++m) h[(size_t)m] = h[(size_t)m - 1] + 1.0 / (double)m;
    double *d = nullptr;
    MTE_HIP(hipMalloc(&d, sizeof(double) * h.size()));
    MTE_HIP(hipMemcpy(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
    if (c.harm) c.retired.push_back(c.harm);
    c.harm = d;
    c.harm_n = cap;
    return MTE_OK;
}

int ensure_harm(int64_t n) {
    std::lock_guard<std::mutex> lk(ctx().mu);
    return harm_locked(n);
}

const double *harm_table() { return ctx().harm; }

int shutdown_all() {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.inited) return MTE_OK;
    MTE_HIP(hipDeviceSynchronize());
    for (auto &pe : c.pending_events) {
        if (pe.own_a) (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    c.pending_events.clear();
    for (hipEvent_t e : c.event_pool) (void)hipEventDestroy(e);
    c.event_pool.clear();
    if (c.harm) (void)hipFree(c.harm);
    for (double *p : c.retired) (void)hipFree(p);
    c.retired.clear();
    c.harm = nullptr;
    c.harm_n = 0;
    c.alloc.trim();
    if (c.capture_stream) (void)hipStreamDestroy(c.capture_stream);
    c.capture_stream = nullptr;
    if (c.side_stream) (void)hipStreamDestroy(c.side_stream);
    c.side_stream = nullptr;
    c.tuned.clear();
    c.tune_log.clear();
    c.inited = false;
    c.device = -1;
    return MTE_OK;
}

// ---------------------------------------------------------------- validation
int validate_dims(int dx, int dy, int dz, int64_t n, int k) {
    if (dx < 1 || dx > kMaxDx) return fail(MTE_EINVAL, "dx=%d out of range [1,%d]", dx, kMaxDx);
    if (dy < 1 || dy > kMaxDy) return fail(MTE_EINVAL, "dy=%d out of range [1,%d]", dy, kMaxDy);
    if (dz < 0 || dz > kMaxDz) return fail(MTE_EINVAL, "dz=%d out of range [0,%d]", dz, kMaxDz);
    if (k < 1 || k > kMaxK) return fail(MTE_EINVAL, "k=%d out of range [1,%d]", k, kMaxK);
    if (n < (int64_t)k + 1) return fail(MTE_EINVAL, "N=%lld must be at least k+1", (long long)n);
    if (n > 0x7fffffffLL) return fail(MTE_EINVAL, "N=%lld exceeds 2^31-1", (long long)n);
    return MTE_OK;
}

int validate_theiler(int64_t n, int k, int theiler) {
    if (theiler < 0) return fail(MTE_EINVAL, "Theiler window %d must be >= 0", theiler);
    if (n < (int64_t)k + 1 + 2 * (int64_t)theiler)
        return fail(MTE_EINVAL, "N=%lld leaves fewer than k=%d rows outside a Theiler window of %d", (long long)n,
                    k, theiler);
    return MTE_OK;
}

// Autocorrelation decay time: the shortest lag L >= 1 at which the biased
// autocovariance r(L) = (1/T) sum_t (x_t - mu)(x_{t+L} - mu) drops below
// r(0)/e (max_lag if none does), with float64 sums in time order.
int autocorr_decay_time(const float *x, int64_t T, int max_lag) {
    double mu = 0.0;
    for (int64_t t = 0; t < T; ++t) mu += (double)x[t];
    mu /= (double)T;
    auto r = [&](int64_t lag) {
        double s = 0.0;
        for (int64_t t = 0; t + lag < T; ++t) s += ((double)x[t] - mu) * ((double)x[t + lag] - mu);
        return s / (double)T;
    };
    const double thr = r(0) / 2.718281828459045;
    const int64_t top = std::min<int64_t>(max_lag, T - 1);
    for (int64_t lag = 1; lag <= top; ++lag)
        if (r(lag) < thr) return (int)lag;
    return max_lag;
}

int validate_host_finite(const float *p, int64_t count, const char *name) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i]))
            return fail(MTE_EINVAL, "%s[%lld] is not finite", name, (long long)i);
    return MTE_OK;
}

// z-score of each node over all its samples (replications, then time):
// mean and variance (1/count) as float64 sums in sample order, each value
// (x - mean) / sd in float64 rounded to float32; a constant node becomes 0.
void standardise_host(const float *in, int R, int P, int64_t T, float *out) {
#pragma clang fp contract(off)
    const double count = (double)R * (double)T;
    for (int p = 0; p < P; ++p) {
        double sum = 0.0;
        for (int r = 0; r < R; ++r)
            for (int64_t t = 0; t < T; ++t) sum += (double)in[((int64_t)r * P + p) * T + t];
        const double mean = sum / count;
        double ss = 0.0;
        for (int r = 0; r < R; ++r)
            for (int64_t t = 0; t < T; ++t) {
                const double d = (double)in[((int64_t)r * P + p) * T + t] - mean;
                const double sq = d * d;
                ss += sq;
            }
        const double sd = std::sqrt(ss / count);
        for (int r = 0; r < R; ++r)
            for (int64_t t = 0; t < T; ++t) {
                const int64_t x = ((int64_t)r * P + p) * T + t;
                out[x] = sd > 0.0 ? (float)(((double)in[x] - mean) / sd) : 0.0f;
            }
    }
}

int timing_event(hipEvent_t *e) {
    Ctx &c = ctx();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (!c.event_pool.empty()) {
            *e = c.event_pool.back();
            c.event_pool.pop_back();
            return MTE_OK;
        }
    }
    MTE_HIP(hipEventCreate(e));
    return MTE_OK;
}

void record_timing_pair(int stage, hipEvent_t a, hipEvent_t b, bool own_a) {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    c.pending_events.push_back(Ctx::Pending{stage, a, b, own_a});
}

void record_timing_pairs(const std::vector<Ctx::Pending> &pairs) {
    if (pairs.empty()) return;
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    c.pending_events.insert(c.pending_events.end(), pairs.begin(), pairs.end());
}

// ---------------------------------------------------------------- paths
static int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

int assign_paths(const std::vector<JobSpec> &specs, std::vector<int> *set_of, int *n_sets) {
    const char *fm = std::getenv("MTE_FORCE_MODE");
    const int force = fm && std::strcmp(fm, "brute") == 0 ? 0 : (fm && std::strcmp(fm, "list") == 0 ? 1 : -1);
    set_of->assign(specs.size(), -1);
    // group by (n, dy, dz, Y and Z column pointers)
    std::map<std::vector<uintptr_t>, int> groups;
    std::vector<int64_t> group_est;
    std::vector<int> gid(specs.size(), -1);
    for (size_t j = 0; j < specs.size(); ++j) {
        const JobSpec &sp = specs[j];
        // the list kernels index the transposed X columns with 32-bit
        // element offsets and a column of the build's copy of Y and Z with
        // 32-bit byte offsets, and pack a row's counts kPackBits to a field;
        // without Z the list path needs one X column (its range counts use
        // the sorted column) and N within the in-LDS sort
        if (force == 0 || (int64_t)sp.dx * sp.n * sp.n_est() >= ((int64_t)1 << 31)) continue;
        if (sp.n > kListMaxN) continue;
        if (sp.dz == 0 && (sp.dx != 1 || sp.n > kNoZSortMax)) continue;
        std::vector<uintptr_t> key{(uintptr_t)sp.n, (uintptr_t)sp.dy, (uintptr_t)sp.dz, (uintptr_t)sp.theiler};
        for (int c = 0; c < sp.dy + sp.dz; ++c) key.push_back((uintptr_t)sp.cols[sp.dx + c]);
        auto it = groups.emplace(key, (int)group_est.size()).first;
        if (it->second == (int)group_est.size()) group_est.push_back(0);
        gid[j] = it->second;
        group_est[it->second] += sp.n_est();
    }
    // keep the groups that take the list path and renumber them densely
    std::vector<int> dense(group_est.size(), -1);
    int ns = 0;
    for (size_t g = 0; g < group_est.size(); ++g)
        if (force == 1 || group_est[g] >= kListMinEstimates) dense[g] = ns++;
    for (size_t j = 0; j < specs.size(); ++j)
        if (gid[j] >= 0) (*set_of)[j] = dense[gid[j]];
    *n_sets = ns;
    return MTE_OK;
}

static int solo_kclass(int k) { return k <= 4 ? 4 : (k <= 8 ? 8 : 16); }

// The few-estimate variant for a set of jobs: the right top-k class, the
// smallest column capacities that fit, then the smallest estimate group that
// holds a job's estimates (else the largest); -1 if none fits.
static int solo_variant_for(const std::vector<JobSpec> &specs) {
    int k = 0, dx = 0, dy = 0, dz = 0, e = 0;
    for (const auto &sp : specs) {
        k = std::max(k, sp.k);
        dx = std::max(dx, sp.dx);
        dy = std::max(dy, sp.dy);
        dz = std::max(dz, sp.dz);
        e = std::max(e, sp.n_est());
    }
    // compiled dimensions when every job has one estimate, k <= 4, one X and
    // one Y column and the same dz
    bool fixed = e == 1 && k <= 4 && dx == 1 && dy == 1;
    for (const auto &sp : specs) fixed = fixed && sp.dz == dz;
    int best = -1;
    SoloCfg bc{};
    auto score = [&](const SoloCfg &c) {
        const int gpen = c.g >= e ? c.g - e : 1000 - c.g;
        return std::make_tuple(c.fz < 0, c.dxm, c.dym, c.dzm, gpen);
    };
    for (int v = 0; v < solo_variant_count(); ++v) {
        SoloCfg c;
        solo_variant(v, &c);
        if (c.fz >= 0 ? !(fixed && c.fz == dz) : c.dzm < dz) continue;
        if (c.kmax != solo_kclass(k) || c.dxm < dx || c.dym < dy) continue;
        if (best < 0 || score(c) < score(bc)) {
            best = v;
            bc = c;
        }
    }
    return best;
}

bool takes_solo(const JobSpec &sp) {
    const char *fm = std::getenv("MTE_FORCE_MODE");
    if (fm && std::strcmp(fm, "brute") == 0) return false;
    const bool forced = fm && std::strcmp(fm, "solo") == 0;
    if (!forced && sp.n_est() > kSoloMaxEstimates) return false;
    if (sp.n > kListMaxN) return false;
    return solo_variant_for(std::vector<JobSpec>{sp}) >= 0;
}

// The jobs of the persistent all-pairs kernel (neither list path nor solo).
static std::vector<JobSpec> pair_specs(const std::vector<JobSpec> &specs) {
    std::vector<int> set_of;
    int ns = 0;
    assign_paths(specs, &set_of, &ns);
    std::vector<JobSpec> out;
    for (size_t j = 0; j < specs.size(); ++j)
        if (set_of[j] < 0 && !takes_solo(specs[j])) out.push_back(specs[j]);
    return out;
}

// ---------------------------------------------------------------- tiles
static int kmax_class(int k) { return k <= 4 ? 4 : (k <= 8 ? 8 : 16); }

struct Need {
    int k = 0, dx = 0, dy = 0, dz = 0;
};

static Need need_of(const std::vector<JobSpec> &specs) {
    Need n;
    for (const auto &s : specs) {
        n.k = std::max(n.k, s.k);
        n.dx = std::max(n.dx, s.dx);
        n.dy = std::max(n.dy, s.dy);
        n.dz = std::max(n.dz, s.dz);
    }
    return n;
}

static bool fits(const TileCfg &c, const Need &n) {
    return c.kmax == kmax_class(n.k) && c.dxm >= n.dx && c.dym >= n.dy && c.dzm >= n.dz;
}

int variant_for(const std::vector<JobSpec> &specs, int g_pref) {
    const Need nd = need_of(specs);
    int best = -1;
    TileCfg bc{};
    // smallest column capacities first, then the largest G <= g_pref
    auto score = [&](const TileCfg &t) {
        int gpen = t.g <= g_pref ? (g_pref - t.g) : 100 + t.g;
        return std::make_tuple(t.dxm, t.dym, t.dzm, gpen);
    };
    for (int v = 0; v < kernel_variant_count(); ++v) {
        TileCfg c;
        kernel_variant(v, &c);
        if (!fits(c, nd)) continue;
        if (best < 0 || score(c) < score(bc)) { best = v; bc = c; }
    }
    return best;
}

static std::string shape_key(const std::vector<JobSpec> &specs) {
    int64_t nsum = 0, esum = 0;
    int dxm = 0, dym = 0, dzm = 0, km = 0;
    for (const auto &s : specs) {
        nsum += s.n;
        esum += s.n_est();
        dxm = std::max(dxm, s.dx);
        dym = std::max(dym, s.dy);
        dzm = std::max(dzm, s.dz);
        km = std::max(km, s.k);
    }
    char buf[160];
    snprintf(buf, sizeof buf, "j%zu:n%lld:e%lld:dx%d:dy%d:dz%d:k%d", specs.size(), (long long)nsum,
             (long long)esum, dxm, dym, dzm, km);
    return buf;
}

static int g_pref_for(const std::vector<JobSpec> &specs) {
    int64_t e = 0;
    for (const auto &s : specs) e += s.n_est();
    const double avg = (double)e / (double)std::max<size_t>(1, specs.size());
    return avg >= 16 ? 8 : (avg >= 4 ? 4 : 1);
}

int pair_tiles(const std::vector<JobSpec> &specs, TileChoice *out) {
    Ctx &c = ctx();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.tuned.find("P:" + shape_key(specs));
        if (it != c.tuned.end()) { *out = it->second; return MTE_OK; }
    }
    out->variant = variant_for(specs, g_pref_for(specs));
    out->rs_mult = 1;
    return out->variant < 0 ? fail(MTE_EINVAL, "no compiled tile configuration fits these dimensions") : MTE_OK;
}

// ---------------------------------------------------------------- tuning file
// One choice per line: "mte-tune 3 <arch> <build> <key> <variant> <rs_mult>
// <build_qb> <coop_lanes> <grouped> <scan_step> <perm_cu> <ms>".  Lines of another architecture or
// another build of the library are skipped, so a rebuilt library tunes anew.
static const char *build_id() {
    static std::string id = [] {
        std::string v = __DATE__ "_" __TIME__;
        for (char &ch : v)
            if (ch == ' ' || ch == ':') ch = '-';
        return v;
    }();
    return id.c_str();
}

static std::string default_tune_file() {
    const char *f = std::getenv("MTE_TUNE_FILE");
    if (f) return std::string(f) == "off" ? std::string() : std::string(f);
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
    else if (const char *h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
    else return std::string();
    return dir + "/mte/tune.txt";
}

static void load_tune_file_locked() {
    Ctx &c = ctx();
    if (c.tune_file.empty()) return;
    FILE *f = std::fopen(c.tune_file.c_str(), "r");
    if (!f) return;
    char line[512], arch[128], bid[128], key[256];
    while (std::fgets(line, sizeof line, f)) {
        TileChoice tc;
        double ms = 0.0;
        int ver = 0;
        if (std::sscanf(line, "mte-tune %d %127s %127s %255s %d %d %d %d %d %d %d %lf", &ver, arch, bid, key,
                        &tc.variant, &tc.rs_mult, &tc.build_qb, &tc.coop_lanes, &tc.grouped, &tc.scan_step, &tc.perm_cu,
                        &ms) != 12)
            continue;
        if (ver != 3 || c.arch != arch || std::strcmp(bid, build_id()) != 0) continue;
        c.tuned[key] = tc;
        c.tune_log.push_back(Ctx::TuneNote{key, tc, ms, 1});
    }
    std::fclose(f);
}

static void save_tune_locked(const std::string &key, const TileChoice &tc, double ms) {
    Ctx &c = ctx();
    c.tuned[key] = tc;
    c.tune_log.push_back(Ctx::TuneNote{key, tc, ms, 0});
    if (c.tune_file.empty()) return;
    // create the directories of the path, then append one line
    for (size_t pos = c.tune_file.find('/', 1); pos != std::string::npos; pos = c.tune_file.find('/', pos + 1))
        (void)mkdir(c.tune_file.substr(0, pos).c_str(), 0755);
    FILE *f = std::fopen(c.tune_file.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "mte-tune 3 %s %s %s %d %d %d %d %d %d %d %.4f\n", c.arch.c_str(), build_id(), key.c_str(),
                 tc.variant, tc.rs_mult, tc.build_qb, tc.coop_lanes, tc.grouped, tc.scan_step, tc.perm_cu, ms);
    std::fclose(f);
}

// Blocks per CU (4 waves each) of the permutation that runs beside the build
// (MTE_PERMUTE_BLOCKS_PER_CU overrides; 0 = uncapped).  The build's waves
// have the higher issue priority and the build is submitted first, so the cap
// only sets how many wave slots the permutation holds as the build's blocks
// retire: at N = 10^4 with 201 estimates, 2 per CU gave 0.686-0.692 ms per
// test against 0.701 ms with 3 and 0.72-0.73 ms with 6 or uncapped (submitted
// after the permutation, the build had been best with 3).  Other boxes had the
// permutation outlast the build at 2, so the tuner also tries one more.
constexpr int kPermuteBlocksPerCu = 2;

// ---------------------------------------------------------------- tuning
constexpr double kTuneMargin = 0.97;   // a candidate must be 3% faster to replace the best
// Wall time one shape's tuning may take (MTE_TUNE_BUDGET_MS overrides): the
// candidates are timed in order of how far they are from the default, and
// the search stops when the budget is spent.  A shape whose launch takes
// tens of milliseconds then keeps the default or a choice one knob away,
// instead of spending seconds on the full candidate set.
constexpr int kTuneBudgetMs = 400;

static double tune_budget_s() { return env_int("MTE_TUNE_BUDGET_MS", kTuneBudgetMs) * 1e-3; }

static double wall_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static bool tuning_on() {
    const char *v = std::getenv("MTE_TUNE");
    return !(v && *v == '0');
}

// Time per launch of `specs` with choice `tc`: after a warm-up launch, two
// rounds of four launches back to back (so that the gaps of one launch's
// submission count as little as in a stream of calls), the faster round;
// negative when the launch cannot be made.
static double time_launch(const std::vector<JobSpec> &specs, const TileChoice &tc, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
    constexpr int kBack = 4;
    Batch b;
    if (b.prepare(specs, tc, s) != MTE_OK) return -1.0;
    if (b.enqueue_quiet(s) != MTE_OK) return -1.0;
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, s);
        for (int q = 0; q < kBack; ++q)
            if (b.enqueue_quiet(s) != MTE_OK) return -1.0;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, (double)ms / kBack);
    }
    if (b.check_error(s) != MTE_OK) return -1.0;
    return best;
}

// The list knobs a job shape is tuned for: launches of one job or of several.
static std::string list_key(const JobSpec &sp, bool several) {
    char buf[200];
    snprintf(buf, sizeof buf, "L:n%d:dx%d:dy%d:dz%d:k%d:e%d:w%d:r%d:%s", sp.n, sp.dx, sp.dy, sp.dz, sp.k, sp.n_est(),
             sp.theiler, sp.reps, several ? "many" : "one");
    return buf;
}

static int tune_pairs(const std::vector<JobSpec> &specs, hipStream_t s, int mode, TileChoice *out) {
    Ctx &c = ctx();
    // test hooks: MTE_FORCE_VARIANT (tile configuration index, used when it
    // fits) and MTE_FORCE_SPLIT (0 = one reference split, m = m times the
    // heuristic split count)
    const int fv = env_int("MTE_FORCE_VARIANT", -1), fs = env_int("MTE_FORCE_SPLIT", -1);
    if (fv >= 0 || fs >= 0) {
        out->variant = variant_for(specs, g_pref_for(specs));
        out->rs_mult = fs >= 0 ? fs : 1;
        TileCfg fc;
        if (fv >= 0 && kernel_variant(fv, &fc) && fits(fc, need_of(specs))) out->variant = fv;
        if (out->variant < 0) return fail(MTE_EINVAL, "no compiled tile configuration fits these dimensions");
        return MTE_OK;
    }
    const std::string key = "P:" + shape_key(specs);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.tuned.find(key);
        if (it != c.tuned.end()) {
            out->variant = it->second.variant;
            out->rs_mult = it->second.rs_mult;
            return MTE_OK;
        }
    }
    TileChoice heur;
    heur.variant = variant_for(specs, g_pref_for(specs));
    heur.rs_mult = 1;
    if (heur.variant < 0) return fail(MTE_EINVAL, "no compiled tile configuration fits these dimensions");
    out->variant = heur.variant;
    out->rs_mult = 1;
    if (mode != kTuneBatch || !tuning_on()) return MTE_OK;
    // candidate set: every fitting variant with the exact k class, and split
    // multipliers 0 (one split), 1, 2
    std::vector<TileChoice> cand;
    const Need nd = need_of(specs);
    TileCfg hc;
    kernel_variant(heur.variant, &hc);
    for (int v = 0; v < kernel_variant_count(); ++v) {
        TileCfg t;
        kernel_variant(v, &t);
        if (!fits(t, nd) || t.dxm != hc.dxm || t.dym != hc.dym || t.dzm > hc.dzm) continue;
        for (int m : {0, 1, 2}) {
            TileChoice tc;
            tc.variant = v;
            tc.rs_mult = m;
            cand.push_back(tc);
        }
    }
    hipEvent_t e0, e1;
    MTE_HIP(hipEventCreate(&e0));
    MTE_HIP(hipEventCreate(&e1));
    // the heuristic choice stands unless a candidate is kTuneMargin faster,
    // so that near ties resolve the same way from one run to the next
    TileChoice best = heur;
    const double t_end = wall_s() + tune_budget_s();
    double best_ms = time_launch(specs, heur, s, e0, e1);
    if (best_ms < 0.0) best_ms = 1e30;
    for (const auto &tc : cand) {
        if (wall_s() > t_end) break;
        const double ms = time_launch(specs, tc, s, e0, e1);
        if (ms >= 0.0 && ms < best_ms * kTuneMargin) {
            best_ms = ms;
            best = tc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        save_tune_locked(key, best, best_ms);
    }
    out->variant = best.variant;
    out->rs_mult = best.rs_mult;
    return MTE_OK;
}

// List knobs: the compiled-dimension build's rows per block (2, 4), the
// scan's cooperative-finish threshold (2, 4, 8), its entries per step (8, 4)
// and, for launches of one job, the estimate-group lane order (on, off).
static int tune_lists(const std::vector<JobSpec> &lists, hipStream_t s, int mode, TileChoice *out) {
    Ctx &c = ctx();
    const bool several = lists.size() > 1;
    const JobSpec &rep = lists.front();
    const std::string key = list_key(rep, several);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.tuned.find(key);
        if (it != c.tuned.end()) {
            out->build_qb = it->second.build_qb;
            out->coop_lanes = it->second.coop_lanes;
            out->grouped = it->second.grouped;
            out->scan_step = it->second.scan_step;
            out->perm_cu = it->second.perm_cu;
            return MTE_OK;
        }
    }
    if (mode == kTuneNone || !tuning_on()) return MTE_OK;
    int64_t pairs = 0;
    for (const auto &sp : lists) pairs += (int64_t)sp.n * sp.n_est();
    if (mode == kTuneShape && pairs < kTuneMinPairs) return MTE_OK;
    // the launch timed: the batch itself, or one job of its first shape (two
    // copies of it for a launch of several jobs, so that the probe takes the
    // several-job scan, whose registers and lane order differ; the copies
    // write the same values to the same outputs)
    const std::vector<JobSpec> probe =
        mode == kTuneBatch ? lists : (several ? std::vector<JobSpec>{rep, rep} : std::vector<JobSpec>{rep});
    const bool lean = rep.dy == 1 && rep.dz >= 1 && rep.dz <= kBuildFixedDz && rep.n < 65536;
    std::vector<TileChoice> cand;
    std::vector<int> away;   // knobs that differ from the default
    const int step0 = several ? 4 : 8, qb0 = lean ? 2 : 0, grp0 = several ? 0 : 1;
    for (int qb : lean ? std::vector<int>{2, 4} : std::vector<int>{0})
        for (int coop : {4, 2, 8})
            for (int grp : several ? std::vector<int>{0} : std::vector<int>{1, 0})
                for (int step : {step0, 12 - step0})
                    for (int pcu : {kPermuteBlocksPerCu, kPermuteBlocksPerCu + 1}) {
                        TileChoice tc = *out;
                        tc.build_qb = qb;
                        tc.coop_lanes = coop;
                        tc.grouped = grp;
                        tc.scan_step = step;
                        tc.perm_cu = pcu;
                        cand.push_back(tc);
                        away.push_back((qb != qb0) + (coop != 4) + (grp != grp0) + (step != step0) +
                                       (pcu != kPermuteBlocksPerCu));
                    }
    // the default first, then one knob away, two, ... (stable within a distance)
    std::vector<size_t> order(cand.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return away[a] < away[b]; });
    hipEvent_t e0, e1;
    MTE_HIP(hipEventCreate(&e0));
    MTE_HIP(hipEventCreate(&e1));
    // the first candidate is the default (2 build rows, 4 lanes, the grouped
    // order and 8-entry steps for one job, 4-entry steps for several);
    // another replaces the best so far only when it is kTuneMargin faster
    double best_ms = 1e30;
    TileChoice best = cand[order.front()];
    const double t_end = wall_s() + tune_budget_s();
    for (size_t oi = 0; oi < order.size(); ++oi) {
        if (oi > 0 && wall_s() > t_end) break;
        const TileChoice &tc = cand[order[oi]];
        const double ms = time_launch(probe, tc, s, e0, e1);
        if (ms >= 0.0 && ms < best_ms * (best_ms < 1e30 ? kTuneMargin : 1.0)) {
            best_ms = ms;
            best = tc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TileChoice rec;
    rec.build_qb = best.build_qb;
    rec.coop_lanes = best.coop_lanes;
    rec.grouped = best.grouped;
    rec.scan_step = best.scan_step;
    rec.perm_cu = best.perm_cu;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        save_tune_locked(key, rec, best_ms);
    }
    out->build_qb = rec.build_qb;
    out->coop_lanes = rec.coop_lanes;
    out->grouped = rec.grouped;
    out->scan_step = rec.scan_step;
    out->perm_cu = rec.perm_cu;
    return MTE_OK;
}

int choose_tiles(const std::vector<JobSpec> &all_specs, hipStream_t s, int mode, TileChoice *out) {
    *out = TileChoice{};
    int rc;
    // the jobs of the all-pairs kernel have a tile choice
    const std::vector<JobSpec> specs = pair_specs(all_specs);
    if (!specs.empty() && (rc = tune_pairs(specs, s, mode, out))) return rc;
    // the list path's jobs have the list knobs
    std::vector<int> set_of;
    int n_sets = 0;
    assign_paths(all_specs, &set_of, &n_sets);
    std::vector<JobSpec> lists;
    for (size_t j = 0; j < all_specs.size(); ++j)
        if (set_of[j] >= 0) lists.push_back(all_specs[j]);
    if (!lists.empty() && (rc = tune_lists(lists, s, mode, out))) return rc;
    return MTE_OK;
}

// ---------------------------------------------------------------- batch
static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Batch::~Batch() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (fork_) (void)hipEventDestroy(fork_);
    if (join_) (void)hipEventDestroy(join_);
}

size_t Batch::device_bytes() const {
    return tables_.bytes + scratch_.bytes + sync_.bytes + ltables_.bytes + lscratch_.bytes + lcounters_.bytes +
           stables_.bytes + sscratch_.bytes;
}

static int check_spec(const JobSpec &sp) {
    if (sp.n_est() < 1) return fail(MTE_EINVAL, "job without estimates");
    if (sp.n < sp.k + 1) return fail(MTE_EINVAL, "N < k+1");
    if (validate_theiler(sp.n, sp.k, sp.theiler)) return MTE_EINVAL;
    if (sp.k < 1 || sp.k > kMaxK || sp.dx < 1 || sp.dx > kMaxDx || sp.dy < 1 || sp.dy > kMaxDy || sp.dz < 0 ||
        sp.dz > kMaxDz)
        return fail(MTE_EINVAL, "job dimensions out of range");
    for (int cc = 0; cc < sp.dx + sp.dy + sp.dz; ++cc)
        if (!sp.cols[cc]) return fail(MTE_EINVAL, "null column pointer");
    if (!sp.out) return fail(MTE_EINVAL, "null output pointer");
    if (sp.reps < 1 || sp.n % sp.reps) return fail(MTE_EINVAL, "N=%d is not a multiple of R=%d", sp.n, sp.reps);
    if (sp.reps > 1 && sp.theiler) return fail(MTE_EINVAL, "the Theiler window needs a single replication");
    if (sp.rep_shuffle && sp.reps < 2) return fail(MTE_EINVAL, "a replication shuffle needs R >= 2");
    return MTE_OK;
}

int Batch::prepare(const std::vector<JobSpec> &specs, const TileChoice &tc, hipStream_t s, size_t *measure) {
    if (specs.empty()) return fail(MTE_EINVAL, "empty batch");
    int rc;
    int64_t nmax = 0;
    for (const auto &sp : specs) {
        if ((rc = check_spec(sp))) return rc;
        nmax = std::max<int64_t>(nmax, sp.n);
    }
    if (measure) *measure = 0;
    else if ((rc = ensure_harm(nmax))) return rc;
    std::vector<int> set_of;
    int n_sets = 0;
    assign_paths(specs, &set_of, &n_sets);
    std::vector<JobSpec> pairs, lists, solo;
    std::vector<int> lset;
    for (size_t j = 0; j < specs.size(); ++j) {
        if (set_of[j] >= 0) {
            lists.push_back(specs[j]);
            lset.push_back(set_of[j]);
        } else if (takes_solo(specs[j])) {
            solo.push_back(specs[j]);
        } else {
            pairs.push_back(specs[j]);
        }
    }
    n_est_total_ = 0;
    for (const auto &sp : specs) n_est_total_ += sp.n_est();
    n_jobs_ = 0;
    variant_ = -1;
    if (!pairs.empty() && (rc = prepare_pairs(pairs, tc, s, measure))) return rc;
    n_ljobs_ = 0;
    if (!lists.empty() && (rc = prepare_lists(lists, lset, n_sets, tc, s, measure))) return rc;
    n_sjobs_ = 0;
    if (!solo.empty() && (rc = prepare_solo(solo, s, measure))) return rc;
    return MTE_OK;
}

// List capacities per row.  The Z list must hold every row with d_z below a
// radius taken in the joint space, so the capacity it needs grows with the
// dimensions outside Z: with e = dx + dy - dz, on the 10-node VAR at
// N = 10^4 the 99th percentile of n_z is about 1000 for e = 0, 2000-3700
// for e = 1 and 4700-6700 for e >= 2 (n_yz about a third to half of that),
// and a pair beyond the capacity is redone over all rows, some 800 times the
// cost of a list scan.  MTE_LIST_CAP="m1,m2" overrides (tests use it to force
// the all-rows redo).
// The lists of one set are kept within kListSetBytes (capacities halved until
// they fit, down to 1024 and 2048).
constexpr double kListSetBytes = 4.0 * (1 << 30);

static void list_caps(int dx, int dy, int dz, int n, int *m1, int *m2) {
    const double cap_bytes = kListSetBytes;
    if (dz == 0) {
        // no Z list; list 1 holds every row when it fits (an incomplete list
        // leaves the surrogates whose permuted x is an outlier undecided)
        *m1 = (int)std::max<double>(1024.0, std::min<double>(n - 1.0, cap_bytes / ((double)n * sizeof(LEnt))));
        *m2 = 0;
    } else {
        const int e = dx + dy - dz;
        *m1 = e >= 2 ? 8192 : e == 1 ? 4096 : e == 0 ? 2048 : 1024;
        while (*m1 > 1024 && (double)n * (std::min(n - 1, *m1) * (double)sizeof(LEnt) +
                                          std::min(n - 1, 2 * *m1) * (double)sizeof(LEnt2)) > cap_bytes)
            *m1 /= 2;
        *m2 = 2 * *m1;
    }
    const char *v = std::getenv("MTE_LIST_CAP");
    if (v && *v) {
        int a = 0, b = 0;
        if (std::sscanf(v, "%d,%d", &a, &b) == 2 && a >= 1 && b >= 1) {
            *m1 = a;
            *m2 = dz == 0 ? 0 : b;
        }
    }
}

constexpr int kUnitsPerXcd = 4;   // fewest scan units per XCD for the XCD-dealt order

int Batch::prepare_lists(const std::vector<JobSpec> &specs, const std::vector<int> &set_of, int n_sets,
                         const TileChoice &tc, hipStream_t s, size_t *measure) {
    Ctx &c = ctx();
    n_ljobs_ = (int)specs.size();
    std::vector<Job> jobs(n_ljobs_);
    std::vector<ListSet> sets(n_sets);
    std::vector<int> set_rep(n_sets, -1);
    std::vector<int64_t> lane_off(n_ljobs_ + 1, 0), est_off(n_ljobs_ + 1, 0), blk_off(n_ljobs_ + 1, 0),
        row_off(n_sets + 1, 0), build_off(n_sets + 1, 0);
    int kmax = 0, dxm = 0;
    int64_t n_keys = 0;
    for (int j = 0; j < n_ljobs_; ++j) {
        const JobSpec &sp = specs[j];
        if (set_rep[set_of[j]] < 0) set_rep[set_of[j]] = j;
        lane_off[j + 1] = lane_off[j] + (int64_t)sp.n * sp.n_est();
        est_off[j + 1] = est_off[j] + sp.n_est();
        blk_off[j + 1] = blk_off[j] + (int64_t)sp.n_est() * permute_blocks(sp.n, sp.reps);
        kmax = std::max(kmax, sp.k);
        dxm = std::max(dxm, sp.dx);
        n_keys += sp.n_est();
    }
    // a launch of several jobs: the scan's units of (job, 64-estimate group),
    // dealt to the XCDs in turn, when there are at least kUnitsPerXcd per XCD
    // (fewer leave XCDs idle and tie each unit to one XCD's CUs: a served
    // batch of two or three requests has six to nine); MTE_GROUPED_MANY=0:
    // job-major lanes in the hardware order always
    int64_t n_units_all = 0;
    for (int j = 0; j < n_ljobs_; ++j) n_units_all += std::max(1, specs[j].n_est() / 64);
    const bool units = n_ljobs_ > 1 && n_units_all >= (int64_t)kUnitsPerXcd * kXcds &&
                       env_int("MTE_GROUPED_MANY", 1) != 0;
    std::vector<int64_t> unit_info, unit_blocks, xcd_off;
    int unit_t = 0;
    int64_t scan_blocks = 0;
    if (units) {
        for (int j = 0; j < n_ljobs_; ++j) {
            const JobSpec &sp = specs[j];
            const int ng = std::max(1, sp.n_est() / 64);
            for (int grp = 0; grp < ng; ++grp) {
                const int eg = grp == ng - 1 ? sp.n_est() - 64 * grp : 64;
                unit_info.push_back((int64_t)j << 32 | grp);
                unit_blocks.push_back(((int64_t)sp.n * eg + kBlock - 1) / kBlock);
            }
        }
        const int nu = (int)unit_info.size();
        unit_t = (nu + kXcds - 1) / kXcds;
        xcd_off.assign((size_t)kXcds * (unit_t + 1), 0);
        for (int x = 0; x < kXcds; ++x) {
            int64_t acc = 0;
            for (int t = 0; t < unit_t; ++t) {
                xcd_off[(size_t)x * (unit_t + 1) + t] = acc;
                const int u = x + t * kXcds;
                if (u < nu) acc += unit_blocks[u];
            }
            xcd_off[(size_t)x * (unit_t + 1) + unit_t] = acc;
            scan_blocks = std::max(scan_blocks, acc);
        }
        scan_blocks *= kXcds;
    }
    // scratch layout: per set its lists and Y,Z copy; per job xt, xp, the
    // packed counts and the chunk sums; then the queue
    size_t bytes = 0;
    int nmax_set = 0;
    std::vector<size_t> o_l1(n_sets), o_l2(n_sets), o_len(n_sets), o_bound(n_sets), o_zy(n_sets),
        o_order(n_sets, 0), o_rank(n_sets, 0);
    std::vector<int> set_dx(n_sets, 0);
    for (int j = 0; j < n_ljobs_; ++j) set_dx[set_of[j]] = std::max(set_dx[set_of[j]], specs[j].dx);
    // sets with one Z column and one Y column are counted by ranks of z
    // (MTE_RANK_COUNTS=0 keeps them on the Z list, for comparison)
    const char *rk_env = std::getenv("MTE_RANK_COUNTS");
    const bool rank_on = !(rk_env && *rk_env == '0');
    std::vector<char> ranked(n_sets, 0);
    int rank_sets = 0, max_rank_n = 0;
    for (int t = 0; t < n_sets; ++t) {
        const JobSpec &sp = specs[set_rep[t]];
        ranked[t] = rank_on && sp.dz == 1 && sp.dy == 1 && sp.n <= kRankMaxN;
        if (ranked[t]) {
            ++rank_sets;
            max_rank_n = std::max(max_rank_n, sp.n);
        }
    }
    for (int t = 0; t < n_sets; ++t) {
        const JobSpec &sp = specs[set_rep[t]];
        ListSet &S = sets[t];
        std::memset(&S, 0, sizeof S);
        int cap1 = 0, cap2 = 0;
        list_caps(set_dx[t], sp.dy, sp.dz, sp.n, &cap1, &cap2);
        if (ranked[t]) cap2 = kRankListCap;
        for (int cc = 0; cc < sp.dy + sp.dz; ++cc) S.cols[cc] = sp.cols[sp.dx + cc];
        S.n = sp.n;
        S.dy = sp.dy;
        S.dz = sp.dz;
        S.theiler = sp.theiler;
        S.m1 = std::min(sp.n - 1, cap1);
        S.m2 = std::min(sp.n - 1, cap2);
        S.s1 = S.m1 + kListPad;
        S.s2 = S.m2 + kListPad;
        row_off[t + 1] = row_off[t] + sp.n;
        nmax_set = std::max(nmax_set, sp.n);
        // kListPad spare entries after each array: the scan loads one step
        // ahead, up to kListPad entries past the last row's sentinels
        o_l1[t] = bytes;
        bytes = align_up(bytes + sizeof(LEnt) * ((size_t)sp.n * S.s1 + kListPad), 256);
        o_l2[t] = bytes;
        bytes = align_up(bytes + sizeof(LEnt2) * ((size_t)sp.n * S.s2 + kListPad), 256);
        o_len[t] = bytes;
        bytes = align_up(bytes + sizeof(int32_t) * 2 * (size_t)sp.n, 256);
        o_bound[t] = bytes;
        bytes = align_up(bytes + sizeof(float) * 2 * (size_t)sp.n, 256);
        o_zy[t] = bytes;
        bytes = align_up(bytes + sizeof(float) * (size_t)(sp.dy + sp.dz) * sp.n, 256);
        // a launch of several jobs scans rows grouped by Morton cell of their
        // Z,Y point: rows with close points share list entries, so their
        // permuted-X gathers meet in L2
        if (n_ljobs_ > 1 && sp.n <= kNoZSortMax) {
            o_order[t] = bytes;
            bytes = align_up(bytes + sizeof(int32_t) * (size_t)sp.n, 256);
        }
        // rank arrays: zs, zord, zrank, yr (n words each)
        if (ranked[t]) {
            o_rank[t] = bytes;
            bytes = align_up(bytes + 4 * sizeof(float) * (size_t)sp.n, 256);
        }
    }
    struct Off { size_t xt, xp, pk, xs, chunk, xr, er; };
    std::vector<Off> offs(n_ljobs_);
    std::vector<int64_t> rank_off(n_ljobs_ + 1, 0);
    for (int j = 0; j < n_ljobs_; ++j) {
        const JobSpec &sp = specs[j];
        const size_t pairs = (size_t)sp.n * sp.n_est();
        offs[j].xt = bytes;
        bytes = align_up(bytes + sizeof(float) * pairs * sp.dx, 256);
        offs[j].xp = bytes;
        bytes = align_up(bytes + sizeof(float) * pairs * sp.dx, 256);
        rank_off[j + 1] = rank_off[j];
        if (ranked[set_of[j]]) {
            offs[j].xr = bytes;
            bytes = align_up(bytes + sizeof(float) * pairs * sp.dx, 256);
            offs[j].er = bytes;
            bytes = align_up(bytes + sizeof(float) * pairs, 256);
            rank_off[j + 1] += (int64_t)sp.n_est() * ((sp.n + 63) / 64);
        }
        offs[j].xs = bytes;
        if (sp.dz == 0) bytes = align_up(bytes + sizeof(float) * (size_t)sp.n, 256);
        offs[j].pk = bytes;
        bytes = align_up(bytes + sizeof(uint64_t) * pairs, 256);
        offs[j].chunk = bytes;
        bytes = align_up(bytes + sizeof(double) * (size_t)sp.n_est() * ((sp.n + kChunk - 1) / kChunk), 256);
    }
    const size_t o_failq = bytes;
    bytes = align_up(bytes + sizeof(uint64_t) * (size_t)lane_off[n_ljobs_], 256);
    // tables: jobs, sets, keys, offsets
    const size_t t_jobs = align_up(sizeof(Job) * n_ljobs_, 256);
    const size_t t_sets = align_up(sizeof(ListSet) * n_sets, 256);
    const size_t t_keys = align_up(sizeof(EstKey) * (size_t)n_keys, 256);
    const size_t t_offs = align_up(sizeof(int64_t) * (5 * (size_t)(n_ljobs_ + 1) + 2 * ((size_t)n_sets + 1) +
                                                      xcd_off.size() + unit_info.size()),
                                   256);
    const size_t tbytes = t_jobs + t_sets + t_keys + t_offs;
    if (measure) {
        *measure += bytes + sizeof(uint32_t) * kListCounterWords + tbytes;
        return MTE_OK;
    }
    int rc;
    if ((rc = lscratch_.ensure(bytes))) return rc;
    if ((rc = lcounters_.ensure(sizeof(uint32_t) * kListCounterWords))) return rc;
    uint8_t *sb = lscratch_.as<uint8_t>();
    for (int t = 0; t < n_sets; ++t) {
        ListSet &S = sets[t];
        S.l1 = reinterpret_cast<LEnt *>(sb + o_l1[t]);
        S.l2 = reinterpret_cast<LEnt2 *>(sb + o_l2[t]);
        S.len = reinterpret_cast<int32_t *>(sb + o_len[t]);
        S.bound = reinterpret_cast<float *>(sb + o_bound[t]);
        S.zy = reinterpret_cast<float *>(sb + o_zy[t]);
        S.order = o_order[t] ? reinterpret_cast<int32_t *>(sb + o_order[t]) : nullptr;
        if (ranked[t]) {
            const size_t nb = sizeof(float) * (size_t)S.n;
            S.zs = reinterpret_cast<float *>(sb + o_rank[t]);
            S.zord = reinterpret_cast<int32_t *>(sb + o_rank[t] + nb);
            S.zrank = reinterpret_cast<int32_t *>(sb + o_rank[t] + 2 * nb);
            S.yr = reinterpret_cast<float *>(sb + o_rank[t] + 3 * nb);
        }
    }
    // build blocks: kBuildRows rows each with packed 16-bit histograms when
    // every set has N <= 2^16, one row each with 32-bit histograms otherwise;
    // the compiled-dimension form when every set has the same dz <=
    // kBuildFixedDz, one Y column and N < 2^16 (kLeanRows rows per block)
    const bool pack = nmax_set <= 65536;
    int build_dz = 0, build_kind = 0;
    {
        const char *bk = std::getenv("MTE_BUILD_KIND");
        const int want = bk && *bk ? std::atoi(bk) : 1;
        bool fixed = pack && want == 1;
        for (int t = 0; t < n_sets; ++t) {
            const JobSpec &sp = specs[set_rep[t]];
            fixed = fixed && sp.dz == specs[set_rep[0]].dz && sp.dy == 1 && sp.n < 65536;
        }
        const int dz0 = specs[set_rep[0]].dz;
        if (fixed && dz0 >= 1 && dz0 <= kBuildFixedDz) {
            build_dz = dz0;
            build_kind = 1;
        }
    }
    const char *bq = std::getenv("MTE_BUILD_QB");
    const int lean_qb = bq && *bq ? std::atoi(bq) : (tc.build_qb == 4 ? 4 : kLeanRows);
    const int qb = build_kind == 1 ? lean_qb : (pack ? kBuildRows : 1);
    for (int t = 0; t < n_sets; ++t) build_off[t + 1] = build_off[t] + (row_off[t + 1] - row_off[t] + qb - 1) / qb;
    if ((rc = ltables_.ensure(tbytes))) return rc;
    static thread_local HostBuf *staging = new HostBuf;
    if ((rc = staging->ensure(tbytes))) return rc;
    uint8_t *tb = ltables_.as<uint8_t>();
    uint8_t *hs = static_cast<uint8_t *>(staging->p);
    EstKey *keys_dev = reinterpret_cast<EstKey *>(tb + t_jobs + t_sets);
    EstKey *keys_host = reinterpret_cast<EstKey *>(hs + t_jobs + t_sets);
    int64_t kpos = 0;
    for (int j = 0; j < n_ljobs_; ++j) {
        const JobSpec &sp = specs[j];
        Job &J = jobs[j];
        std::memset(&J, 0, sizeof J);
        for (int cc = 0; cc < sp.dx + sp.dy + sp.dz; ++cc) J.cols[cc] = sp.cols[cc];
        J.n = sp.n; J.dx = sp.dx; J.dy = sp.dy; J.dz = sp.dz; J.k = sp.k;
        J.n_est = sp.n_est();
        J.rs = 1;
        J.set = set_of[j];
        J.theiler = sp.theiler;
        J.reps = sp.reps;
        J.rep_shuffle = sp.rep_shuffle;
        J.xt = reinterpret_cast<float *>(sb + offs[j].xt);
        J.xp = reinterpret_cast<float *>(sb + offs[j].xp);
        J.xs = sp.dz == 0 ? reinterpret_cast<float *>(sb + offs[j].xs) : nullptr;
        J.eps = sp.diag_eps;
        J.cnt = sp.diag_cnt;
        J.pk = reinterpret_cast<uint64_t *>(sb + offs[j].pk);
        if (ranked[set_of[j]]) {
            J.zrank = sets[set_of[j]].zrank;
            J.xr = reinterpret_cast<float *>(sb + offs[j].xr);
            J.er = reinterpret_cast<float *>(sb + offs[j].er);
        }
        J.chunk = reinterpret_cast<double *>(sb + offs[j].chunk);
        J.out = sp.out;
        J.keys = keys_dev + kpos;
        std::memcpy(keys_host + kpos, sp.keys.data(), sizeof(EstKey) * J.n_est);
        kpos += J.n_est;
    }
    std::memcpy(hs, jobs.data(), sizeof(Job) * n_ljobs_);
    std::memcpy(hs + t_jobs, sets.data(), sizeof(ListSet) * n_sets);
    int64_t *oh = reinterpret_cast<int64_t *>(hs + t_jobs + t_sets + t_keys);
    int64_t *od = reinterpret_cast<int64_t *>(tb + t_jobs + t_sets + t_keys);
    const size_t nj1 = (size_t)n_ljobs_ + 1;
    std::memcpy(oh, lane_off.data(), sizeof(int64_t) * nj1);
    std::memcpy(oh + nj1, est_off.data(), sizeof(int64_t) * nj1);
    std::memcpy(oh + 2 * nj1, blk_off.data(), sizeof(int64_t) * nj1);
    std::memcpy(oh + 3 * nj1, row_off.data(), sizeof(int64_t) * (n_sets + 1));
    std::memcpy(oh + 3 * nj1 + (n_sets + 1), build_off.data(), sizeof(int64_t) * (n_sets + 1));
    std::memcpy(oh + 3 * nj1 + 2 * (n_sets + 1), rank_off.data(), sizeof(int64_t) * nj1);
    const size_t o_units = 4 * nj1 + 2 * ((size_t)n_sets + 1);
    if (!xcd_off.empty()) std::memcpy(oh + o_units, xcd_off.data(), sizeof(int64_t) * xcd_off.size());
    if (!unit_info.empty())
        std::memcpy(oh + o_units + xcd_off.size(), unit_info.data(), sizeof(int64_t) * unit_info.size());
    ljobs_dev_ = reinterpret_cast<Job *>(tb);
    lblk_off_ = od + 2 * nj1;
    lpermute_blocks_ = blk_off[n_ljobs_];
    ListLaunch &L = ll_;
    L.jobs = ljobs_dev_;
    L.sets = reinterpret_cast<const ListSet *>(tb + t_jobs);
    L.lane_off = od;
    L.est_off = od + nj1;
    L.row_off = od + 3 * nj1;
    L.build_off = od + 3 * nj1 + (n_sets + 1);
    L.build_blocks = build_off[n_sets];
    L.build_qb = qb;
    L.build_pack = pack ? 1 : 0;
    L.build_dz = build_dz;
    L.build_kind = build_kind;
    L.stats = 0;
    L.n_jobs = n_ljobs_;
    L.n_sets = n_sets;
    L.lanes = lane_off[n_ljobs_];
    L.rows = row_off[n_sets];
    L.ests = est_off[n_ljobs_];
    L.failq = reinterpret_cast<uint64_t *>(sb + o_failq);
    L.counters = lcounters_.as<uint32_t>();
    L.kmax = kmax <= 4 ? 4 : (kmax <= 8 ? 8 : 16);
    L.dxm = dxm <= 1 ? 1 : kMaxDx;
    L.fb_grid = std::max(1, 2 * c.n_cu);
    L.max_chunks = 0;
    for (const JobSpec &sp : specs) L.max_chunks = std::max(L.max_chunks, (sp.n + kChunk - 1) / kChunk);
    L.sortx = 0;
    for (const JobSpec &sp : specs) L.sortx |= sp.dz == 0;
    L.coop_lanes = env_int("MTE_COOP_LANES", tc.coop_lanes > 0 ? tc.coop_lanes : kCoopLanes);
    L.grouped = units ? 2 : (n_ljobs_ == 1 && env_int("MTE_GROUPED", tc.grouped != 0 ? 1 : 0) != 0 ? 1 : 0);
    L.xcd_off = units ? od + o_units : nullptr;
    L.unit_info = units ? od + o_units + xcd_off.size() : nullptr;
    L.unit_t = unit_t;
    L.n_units = (int)unit_info.size();
    L.scan_blocks = scan_blocks;
    L.scan_step = env_int("MTE_SCAN_STEP", tc.scan_step > 0 ? tc.scan_step : (n_ljobs_ == 1 ? 8 : 4)) == 4 ? 4 : 8;
    perm_cu_ = std::max(0, env_int("MTE_PERMUTE_BLOCKS_PER_CU", tc.perm_cu > 0 ? tc.perm_cu : kPermuteBlocksPerCu));
    L.rank_sets = rank_sets;
    L.max_rank_n = max_rank_n;
    L.rank_off = od + 3 * nj1 + 2 * (n_sets + 1);
    L.rank_waves = rank_off[n_ljobs_];
    if (L.lanes >= ((int64_t)1 << 40) || n_ljobs_ >= (1 << 23)) return fail(MTE_EINVAL, "batch too large");
    n_est_pairs_ = L.lanes;
    MTE_HIP(hipMemcpyAsync(tb, hs, tbytes, hipMemcpyHostToDevice, s));
    MTE_HIP(hipStreamSynchronize(s));
    return MTE_OK;
}

int plan_pairs(const std::vector<JobSpec> &specs, const TileChoice &tc, PairPlan *plan) {
    Ctx &c = ctx();
    TileCfg cfg;
    if (!kernel_variant(tc.variant, &cfg)) return fail(MTE_EINVAL, "bad tile variant");
    PairPlan &P = *plan;
    const int n_jobs = (int)specs.size();
    for (const auto &sp : specs)
        if (sp.k > cfg.kmax || sp.dx > cfg.dxm || sp.dy > cfg.dym || sp.dz > cfg.dzm)
            return fail(MTE_EINVAL, "job does not fit the tile configuration");
    const int qt = kWaves * 64 * cfg.qp;
    const int bpc = variant_blocks_per_cu(tc.variant);
    const int64_t slots = (int64_t)c.n_cu * bpc;
    int64_t base_items = 0;
    for (const auto &sp : specs)
        base_items += (int64_t)((sp.n_est() + cfg.g - 1) / cfg.g) * ((sp.n + qt - 1) / qt);
    int64_t rs_base = 1;
    if (tc.rs_mult > 0 && base_items < 3 * slots) rs_base = (3 * slots + base_items - 1) / base_items;
    if (tc.rs_mult > 1) rs_base *= tc.rs_mult;

    P.jobs.assign(n_jobs, Job{});
    P.a_off.assign(n_jobs + 1, 0);
    P.b_off.assign(n_jobs + 1, 0);
    P.blk_off.assign(n_jobs + 1, 0);
    P.offs.assign(n_jobs, PairPlan::Off{});
    P.scratch_bytes = 0;
    P.sync_words = 2;   // queue head + error flag
    P.n_keys = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const JobSpec &sp = specs[j];
        Job &J = P.jobs[j];
        std::memset(&J, 0, sizeof J);
        for (int cc = 0; cc < sp.dx + sp.dy + sp.dz; ++cc) J.cols[cc] = sp.cols[cc];
        J.n = sp.n; J.dx = sp.dx; J.dy = sp.dy; J.dz = sp.dz; J.k = sp.k;
        J.theiler = sp.theiler;
        J.reps = sp.reps;
        J.rep_shuffle = sp.rep_shuffle;
        J.n_est = sp.n_est();
        J.n_tiles = (sp.n + qt - 1) / qt;
        J.n_groups = (J.n_est + cfg.g - 1) / cfg.g;
        int64_t rs = rs_base;
        const int64_t max_rs = std::max<int64_t>(1, sp.n / 256);
        rs = std::min(rs, max_rs);
        int64_t split_len = ((sp.n + rs - 1) / rs + 63) / 64 * 64;
        rs = (sp.n + split_len - 1) / split_len;
        J.rs = (int)rs;
        J.split_len = (int)split_len;
        const int64_t items = (int64_t)J.n_groups * J.n_tiles * J.rs;
        P.a_off[j + 1] = P.a_off[j] + items;
        P.b_off[j + 1] = P.b_off[j] + (J.rs > 1 ? items : 0);
        P.blk_off[j + 1] = P.blk_off[j] + (int64_t)J.n_est * permute_blocks(sp.n, sp.reps);
        J.a_off = P.a_off[j];
        J.b_off = P.b_off[j];
        const int64_t nch = (sp.n + kChunk - 1) / kChunk;
        PairPlan::Off &o = P.offs[j];
        size_t &sb = P.scratch_bytes;
        o.xp = sb;
        sb = align_up(sb + sizeof(float) * (size_t)J.n_est * sp.dx * sp.n, 256);
        o.chunk = sb;
        sb = align_up(sb + sizeof(double) * (size_t)J.n_est * nch, 256);
        if (J.rs > 1) {
            o.part = sb;
            sb = align_up(sb + sizeof(float) * (size_t)J.rs * J.n_est * sp.n * cfg.kmax, 256);
            o.eps = sb;
            sb = align_up(sb + sizeof(float) * (size_t)J.n_est * sp.n, 256);
            o.cnt = sb;
            sb = align_up(sb + sizeof(int32_t) * (size_t)J.rs * J.n_est * 3 * sp.n, 256);
        }
        o.sync = P.sync_words;
        P.sync_words += sync_words(J.n_groups, J.n_tiles);
        P.sync_words = (P.sync_words + 63) / 64 * 64;
        J.out = sp.out;
        J.diag_eps = sp.diag_eps;
        J.diag_cnt = sp.diag_cnt;
        P.n_keys += J.n_est;
    }
    P.li.items_a = P.a_off[n_jobs];
    P.li.items_b = P.b_off[n_jobs];
    const int64_t total = P.li.items_a + P.li.items_b;
    if (total >= (int64_t)0x7fffffff) return fail(MTE_EINVAL, "batch too large");
    P.li.grid = (int)std::max<int64_t>(1, std::min<int64_t>(total, slots));
    P.permute_blocks = P.blk_off[n_jobs];
    P.tbl_jobs = align_up(sizeof(Job) * n_jobs, 256);
    P.tbl_keys = align_up(sizeof(EstKey) * (size_t)P.n_keys, 256);
    P.tbl_offs = align_up(sizeof(int64_t) * 3 * (n_jobs + 1), 256);
    return MTE_OK;
}

void bind_pairs(PairPlan &P, uint8_t *scratch, uint32_t *sync, EstKey *keys_dev) {
    int64_t kpos = 0;
    for (size_t j = 0; j < P.jobs.size(); ++j) {
        Job &J = P.jobs[j];
        const PairPlan::Off &o = P.offs[j];
        J.xp = reinterpret_cast<float *>(scratch + o.xp);
        J.chunk = reinterpret_cast<double *>(scratch + o.chunk);
        if (J.rs > 1) {
            J.part = reinterpret_cast<float *>(scratch + o.part);
            J.eps = reinterpret_cast<float *>(scratch + o.eps);
            J.cnt = reinterpret_cast<int32_t *>(scratch + o.cnt);
        }
        J.sync = sync + o.sync;
        J.keys = keys_dev + kpos;
        kpos += J.n_est;
    }
}

int Batch::prepare_pairs(const std::vector<JobSpec> &specs, const TileChoice &tc, hipStream_t s, size_t *measure) {
    PairPlan P;
    int rc;
    if ((rc = plan_pairs(specs, tc, &P))) return rc;
    if (measure) {
        *measure += std::max<size_t>(P.scratch_bytes, 256) + sizeof(uint32_t) * (size_t)P.sync_words + P.tbl_jobs +
                    P.tbl_keys + P.tbl_offs;
        return MTE_OK;
    }
    variant_ = tc.variant;
    n_jobs_ = (int)specs.size();
    li_ = P.li;
    permute_blocks_ = P.permute_blocks;
    sync_total_ = P.sync_words;
    if ((rc = scratch_.ensure(std::max<size_t>(P.scratch_bytes, 256)))) return rc;
    if ((rc = sync_.ensure(sizeof(uint32_t) * (size_t)sync_total_))) return rc;
    work_ = sync_.as<uint32_t>();
    const size_t tbl_bytes = P.tbl_jobs + P.tbl_keys + P.tbl_offs;
    if ((rc = tables_.ensure(tbl_bytes))) return rc;
    // pinned staging, reused by this thread (the copy below completes before
    // prepare returns)
    // (never freed, so no HIP call runs in thread-exit destructors)
    static thread_local HostBuf *staging = new HostBuf;
    if ((rc = staging->ensure(tbl_bytes))) return rc;
    uint8_t *tb = tables_.as<uint8_t>();
    uint8_t *hs = static_cast<uint8_t *>(staging->p);
    bind_pairs(P, scratch_.as<uint8_t>(), work_, reinterpret_cast<EstKey *>(tb + P.tbl_jobs));
    EstKey *keys_host = reinterpret_cast<EstKey *>(hs + P.tbl_jobs);
    int64_t kpos = 0;
    for (const JobSpec &sp : specs) {
        std::memcpy(keys_host + kpos, sp.keys.data(), sizeof(EstKey) * sp.n_est());
        kpos += sp.n_est();
    }
    std::memcpy(hs, P.jobs.data(), sizeof(Job) * n_jobs_);
    int64_t *offs_host = reinterpret_cast<int64_t *>(hs + P.tbl_jobs + P.tbl_keys);
    std::memcpy(offs_host, P.a_off.data(), sizeof(int64_t) * (n_jobs_ + 1));
    std::memcpy(offs_host + (n_jobs_ + 1), P.b_off.data(), sizeof(int64_t) * (n_jobs_ + 1));
    std::memcpy(offs_host + 2 * (n_jobs_ + 1), P.blk_off.data(), sizeof(int64_t) * (n_jobs_ + 1));
    jobs_dev_ = reinterpret_cast<Job *>(tb);
    a_off_ = reinterpret_cast<int64_t *>(tb + P.tbl_jobs + P.tbl_keys);
    b_off_ = a_off_ + (n_jobs_ + 1);
    blk_off_ = b_off_ + (n_jobs_ + 1);
    MTE_HIP(hipMemcpyAsync(tb, hs, tbl_bytes, hipMemcpyHostToDevice, s));
    // the staging buffer must not be rewritten before the copy has run
    MTE_HIP(hipStreamSynchronize(s));
    return MTE_OK;
}

// Few-estimate jobs: per job the permuted X (estimate-major), the packed
// counts and the chunk sums of the list path's reduction; tables: jobs, keys,
// and the prefix sums of waves, permute blocks and estimates.
int Batch::prepare_solo(const std::vector<JobSpec> &specs, hipStream_t s, size_t *measure) {
    const int v = solo_variant_for(specs);
    if (v < 0) return fail(MTE_EINVAL, "no compiled few-estimate configuration fits these dimensions");
    SoloCfg cfg;
    solo_variant(v, &cfg);
    const int nj = (int)specs.size();
    std::vector<int64_t> wave_off(nj + 1, 0), blk_off(nj + 1, 0), est_off(nj + 1, 0);
    struct Off { size_t xp, pk, chunk; };
    std::vector<Off> offs(nj);
    size_t bytes = 0;
    int64_t n_keys = 0;
    int max_chunks = 0;
    // a job whose estimates are all the identity (no surrogates) reads its X
    // columns in place and needs no permutation
    auto all_ident = [](const JobSpec &sp) {
        for (const EstKey &kk : sp.keys)
            if (!kk.ident) return false;
        return true;
    };
    for (int j = 0; j < nj; ++j) {
        const JobSpec &sp = specs[j];
        const int E = sp.n_est(), groups = (E + cfg.g - 1) / cfg.g, nch = (sp.n + kChunk - 1) / kChunk;
        const bool ident = all_ident(sp);
        wave_off[j + 1] = wave_off[j] + (int64_t)groups * ((sp.n + cfg.qp - 1) / cfg.qp);
        blk_off[j + 1] = blk_off[j] + (ident ? 0 : (int64_t)E * permute_blocks(sp.n, sp.reps));
        est_off[j + 1] = est_off[j] + E;
        offs[j].xp = ident ? SIZE_MAX : bytes;
        if (!ident) bytes = align_up(bytes + sizeof(float) * (size_t)E * sp.dx * sp.n, 256);
        offs[j].pk = bytes;
        bytes = align_up(bytes + sizeof(uint64_t) * (size_t)E * sp.n, 256);
        offs[j].chunk = bytes;
        bytes = align_up(bytes + sizeof(double) * (size_t)E * nch, 256);
        n_keys += E;
        max_chunks = std::max(max_chunks, nch);
    }
    const size_t t_jobs = align_up(sizeof(Job) * nj, 256);
    const size_t t_keys = align_up(sizeof(EstKey) * (size_t)n_keys, 256);
    const size_t t_offs = align_up(sizeof(int64_t) * 3 * (size_t)(nj + 1), 256);
    const size_t tbytes = t_jobs + t_keys + t_offs;
    if (measure) {
        *measure += std::max<size_t>(bytes, 256) + tbytes;
        return MTE_OK;
    }
    int rc;
    if ((rc = sscratch_.ensure(std::max<size_t>(bytes, 256)))) return rc;
    if ((rc = stables_.ensure(tbytes))) return rc;
    static thread_local HostBuf *staging = new HostBuf;
    if ((rc = staging->ensure(tbytes))) return rc;
    uint8_t *sb = sscratch_.as<uint8_t>(), *tb = stables_.as<uint8_t>();
    uint8_t *hs = static_cast<uint8_t *>(staging->p);
    EstKey *keys_dev = reinterpret_cast<EstKey *>(tb + t_jobs);
    EstKey *keys_host = reinterpret_cast<EstKey *>(hs + t_jobs);
    std::vector<Job> jobs(nj);
    int64_t kpos = 0;
    for (int j = 0; j < nj; ++j) {
        const JobSpec &sp = specs[j];
        Job &J = jobs[j];
        std::memset(&J, 0, sizeof J);
        for (int cc = 0; cc < sp.dx + sp.dy + sp.dz; ++cc) J.cols[cc] = sp.cols[cc];
        J.n = sp.n; J.dx = sp.dx; J.dy = sp.dy; J.dz = sp.dz; J.k = sp.k;
        J.n_est = sp.n_est();
        J.rs = 1;
        J.theiler = sp.theiler;
        J.reps = sp.reps;
        J.rep_shuffle = sp.rep_shuffle;
        J.xp = offs[j].xp == SIZE_MAX ? nullptr : reinterpret_cast<float *>(sb + offs[j].xp);
        J.pk = reinterpret_cast<uint64_t *>(sb + offs[j].pk);
        J.chunk = reinterpret_cast<double *>(sb + offs[j].chunk);
        J.out = sp.out;
        J.diag_eps = sp.diag_eps;
        J.diag_cnt = sp.diag_cnt;
        J.keys = keys_dev + kpos;
        std::memcpy(keys_host + kpos, sp.keys.data(), sizeof(EstKey) * J.n_est);
        kpos += J.n_est;
    }
    std::memcpy(hs, jobs.data(), sizeof(Job) * nj);
    int64_t *oh = reinterpret_cast<int64_t *>(hs + t_jobs + t_keys);
    int64_t *od = reinterpret_cast<int64_t *>(tb + t_jobs + t_keys);
    const size_t nj1 = (size_t)nj + 1;
    std::memcpy(oh, wave_off.data(), sizeof(int64_t) * nj1);
    std::memcpy(oh + nj1, blk_off.data(), sizeof(int64_t) * nj1);
    std::memcpy(oh + 2 * nj1, est_off.data(), sizeof(int64_t) * nj1);
    n_sjobs_ = nj;
    svariant_ = v;
    sjobs_dev_ = reinterpret_cast<Job *>(tb);
    s_wave_off_ = od;
    s_blk_off_ = od + nj1;
    s_total_waves_ = wave_off[nj];
    s_permute_blocks_ = blk_off[nj];
    std::memset(&sl_, 0, sizeof sl_);
    sl_.jobs = sjobs_dev_;
    sl_.est_off = od + 2 * nj1;
    sl_.n_jobs = nj;
    sl_.ests = est_off[nj];
    sl_.max_chunks = max_chunks;
    MTE_HIP(hipMemcpyAsync(tb, hs, tbytes, hipMemcpyHostToDevice, s));
    MTE_HIP(hipStreamSynchronize(s));
    return MTE_OK;
}


// Launch sequence: the all-pairs part (reset, permute, main kernel), then
// the list part (reset, Y,Z copy; permute into xt on the side stream beside
// the build and the X sort, which read only the unpermuted columns; joined
// before the scan; then scan, fallback, reduce).
int Batch::launch_all(hipStream_t s, bool timed) {
    // timed: a stage's events bracket its kernels; a stage that follows
    // another on the same stream starts at that one's end event (each
    // recorded event is a queue packet, a few microseconds of device time)
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool own_a = true;
    struct Pairs {
        std::vector<Ctx::Pending> v;
        ~Pairs() { record_timing_pairs(v); }
    } pairs;
    auto begin = [&](hipStream_t st) -> int {
        if (!timed) return MTE_OK;
        int rc;
        if ((rc = timing_event(&ev[0])) || (rc = timing_event(&ev[1]))) return rc;
        own_a = true;
        MTE_HIP(hipEventRecord(ev[0], st));
        return MTE_OK;
    };
    auto begin_after = [&]() -> int {   // right after end() on the same stream
        if (!timed) return MTE_OK;
        ev[0] = ev[1];
        own_a = false;
        return timing_event(&ev[1]);
    };
    auto end = [&](int stage, hipStream_t st) -> int {
        if (!timed) return MTE_OK;
        MTE_HIP(hipEventRecord(ev[1], st));
        pairs.v.push_back(Ctx::Pending{stage, ev[0], ev[1], own_a});
        return MTE_OK;
    };
    int rc;
    if (n_jobs_ > 0) {
        if (launch_reset(sync_.as<uint32_t>(), sync_total_, s)) return hip_fail(hipGetLastError(), "reset launch");
        if ((rc = begin(s))) return rc;
        if (launch_permute(jobs_dev_, n_jobs_, permute_blocks_, blk_off_, s))
            return hip_fail(hipGetLastError(), "permute launch");
        if ((rc = end(kStagePermute, s))) return rc;
        if ((rc = begin(s))) return rc;
        if (launch_main(variant_, jobs_dev_, n_jobs_, a_off_, b_off_, li_, work_, harm_table(), s))
            return hip_fail(hipGetLastError(), "main kernel launch");
        if ((rc = end(kStageAllPairs, s))) return rc;
    }
    if (n_sjobs_ > 0) {
        if (s_permute_blocks_ > 0) {
            if ((rc = begin(s))) return rc;
            if (launch_permute(sjobs_dev_, n_sjobs_, s_permute_blocks_, s_blk_off_, s))
                return hip_fail(hipGetLastError(), "permute launch");
            if ((rc = end(kStagePermute, s))) return rc;
        }
        if ((rc = begin(s))) return rc;
        if (launch_solo(svariant_, sjobs_dev_, n_sjobs_, s_wave_off_, s_total_waves_, s))
            return hip_fail(hipGetLastError(), "few-estimate kernel launch");
        if ((rc = end(kStageAllPairs, s))) return rc;
        if ((rc = begin(s))) return rc;
        if (launch_list_reduce(sl_, harm_table(), s)) return hip_fail(hipGetLastError(), "reduce launch");
        if ((rc = end(kStageReduce, s))) return rc;
    }
    if (n_ljobs_ > 0) {
        const hipStream_t side = ctx().side_stream;
        if (!fork_) MTE_HIP(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
        if (!join_) MTE_HIP(hipEventCreateWithFlags(&join_, hipEventDisableTiming));
        // the Y,Z copy also clears the counters
        if (launch_list_zy(ll_, s)) return hip_fail(hipGetLastError(), "Y,Z copy launch");
        // the build is submitted first: the side stream's launches (ranks,
        // permutation, row order) then do not delay its start.  The side
        // stream forks at the build's start event when timed
        ll_.stats = ctx().list_stats ? 1 : 0;
        if ((rc = begin(s))) return rc;
        const hipEvent_t fork = timed ? ev[0] : fork_;
        if (!timed) MTE_HIP(hipEventRecord(fork_, s));
        if (launch_list_build(ll_, s)) return hip_fail(hipGetLastError(), "list build launch");
        if (ll_.sortx && launch_list_sortx(ll_, s)) return hip_fail(hipGetLastError(), "X sort launch");
        if ((rc = end(kStageBuild, s))) return rc;
        MTE_HIP(hipStreamWaitEvent(side, fork, 0));
        // the ranks of the one-Z-column sets come first: the permutation
        // writes those sets' jobs' X in rank order
        if (launch_list_rank_sort(ll_, side)) return hip_fail(hipGetLastError(), "rank launch");
        if ((rc = begin(side))) return rc;
        // capped only while the permutation is the smaller part: a launch of
        // many estimates over few list sets has more permutation than build
        const int64_t pgrid = perm_cu_ > 0 && lpermute_blocks_ <= ll_.build_blocks ? (int64_t)perm_cu_ * ctx().n_cu : 0;
        if (launch_permute(ljobs_dev_, n_ljobs_, lpermute_blocks_, lblk_off_, side, pgrid))
            return hip_fail(hipGetLastError(), "permute launch");
        if ((rc = end(kStagePermute, side))) return rc;
        // the scan's row order (launches of several jobs) is needed by the
        // scan only, so it waits on the side stream too
        if (launch_list_order(ll_, side)) return hip_fail(hipGetLastError(), "row order launch");
        // timed with no row-order kernel (one job), the permutation's end
        // event is the join
        const bool join_at_end = timed && ll_.n_jobs <= 1;
        if (!join_at_end) MTE_HIP(hipEventRecord(join_, side));
        MTE_HIP(hipStreamWaitEvent(s, join_at_end ? ev[1] : join_, 0));
        if ((rc = begin(s))) return rc;
        if (launch_list_scan(ll_, s)) return hip_fail(hipGetLastError(), "list scan launch");
        if (launch_list_rank_count(ll_, s)) return hip_fail(hipGetLastError(), "rank count launch");
        if ((rc = end(kStageScan, s))) return rc;
        if ((rc = begin_after())) return rc;
        if (launch_list_fallback(ll_, s)) return hip_fail(hipGetLastError(), "list fallback launch");
        if ((rc = end(kStageFallback, s))) return rc;
        if ((rc = begin_after())) return rc;
        if (launch_list_reduce(ll_, harm_table(), s)) return hip_fail(hipGetLastError(), "list reduce launch");
        if ((rc = end(kStageReduce, s))) return rc;
    }
    return MTE_OK;
}

int Batch::launch_direct(hipStream_t s) { return launch_all(s, ctx().timing); }

int Batch::capture() {
    Ctx &c = ctx();
    hipStream_t cs = c.capture_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        graph_failed_ = true;
        return MTE_OK;
    }
    bool ok = launch_all(cs, false) == MTE_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (!ok || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        graph_failed_ = true;
        return MTE_OK;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        graph_failed_ = true;
        return MTE_OK;
    }
    graph_ = g;
    exec_ = x;
    return MTE_OK;
}

int Batch::enqueue(hipStream_t s, bool use_graph) {
    if (use_graph && !ctx().timing && !graph_failed_) {
        if (!exec_) {
            int rc = capture();
            if (rc) return rc;
        }
        if (exec_) {
            MTE_HIP(hipGraphLaunch(exec_, s));
            return MTE_OK;
        }
    }
    return launch_direct(s);
}

int Batch::enqueue_quiet(hipStream_t s) {
    quiet_ = true;
    return launch_all(s, false);
}

int Batch::check_error(hipStream_t s) {
    uint32_t flag = 0;
    static thread_local std::vector<uint32_t> words(kListCounterWords);
    if (n_jobs_ > 0) MTE_HIP(hipMemcpyAsync(&flag, work_ + 1, sizeof flag, hipMemcpyDeviceToHost, s));
    if (n_ljobs_ > 0)
        MTE_HIP(hipMemcpyAsync(words.data(), lcounters_.as<uint32_t>(), sizeof(uint32_t) * kListCounterWords,
                               hipMemcpyDeviceToHost, s));
    MTE_HIP(hipStreamSynchronize(s));
    if (n_ljobs_ > 0 && !quiet_) {
        uint64_t seen[2] = {0, 0};
        for (int slot = 0; slot < kListStatSlots; ++slot) {
            uint64_t v[2];
            std::memcpy(v, words.data() + kListStatWord + slot * kListStatStride, sizeof v);
            seen[0] += v[0];
            seen[1] += v[1];
        }
        Ctx &c = ctx();
        std::lock_guard<std::mutex> lk(c.mu);
        c.list_pairs += n_est_pairs_;
        c.list_undecided += words[0];
        for (int t = 0; t < 2; ++t) c.list_seen[t] += (int64_t)seen[t];
    }
    if (flag) return fail(MTE_EDEVICE, "a kernel exceeded its bounded wait");
    return MTE_OK;
}

int run_blocking(const std::vector<JobSpec> &specs, hipStream_t s) {
    TileChoice tc;
    int rc = choose_tiles(specs, s, kTuneShape, &tc);
    if (rc) return rc;
    Batch b;
    if ((rc = b.prepare(specs, tc, s))) return rc;
    if ((rc = b.enqueue(s, false))) return rc;
    return b.check_error(s);
}

}  // namespace mte
