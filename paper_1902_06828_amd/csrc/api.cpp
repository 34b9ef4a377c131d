// C ABI entry points: estimator calls (host and device buffers), the
// surrogate permutation, kernel timing, init and shutdown.
#include <algorithm>
#include <cstring>
#include <list>
#include <tuple>

#include "runtime.h"

namespace mte {

const char *last_error();
int init_device(int device, size_t budget);
int shutdown_all();
int serve_shutdown();

// ---------------------------------------------------------------- permutation
static constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t surrogate_key(uint64_t seed, uint32_t cand, uint32_t s) {
    return mix64(mix64(seed + kGolden) ^ (((uint64_t)cand << 32) | (uint64_t)s));
}

static int n_rounds(int64_t n) {
    int bits = 0;
    for (uint64_t v = (uint64_t)(n - 1); v; v >>= 1) ++bits;
    return std::max(24, 6 * bits);
}

void permutation_host(uint64_t h, int64_t n, uint32_t *out) {
    const int rounds = n_rounds(n);
    std::vector<uint64_t> rk(rounds);
    std::vector<uint32_t> kk(rounds);
    for (int r = 0; r < rounds; ++r) {
        rk[r] = mix64(h + (uint64_t)(r + 1) * kGolden);
        kk[r] = (uint32_t)(((rk[r] >> 32) * (uint64_t)n) >> 32);
    }
    const uint32_t un = (uint32_t)n;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t x = (uint32_t)i;
        for (int r = 0; r < rounds; ++r) {
            const uint32_t k = kk[r];
            const uint32_t xp = x <= k ? k - x : k - x + un;
            const uint32_t hi = std::max(x, xp);
            if (mix64((uint64_t)hi ^ rk[r]) >> 63) x = xp;
        }
        out[i] = x;
    }
}

void replication_source_rows_host(uint64_t h, int64_t n, int reps, int rep_shuffle, uint32_t *out) {
    const int64_t nr = n / reps;
    if (rep_shuffle) {
        std::vector<uint32_t> sigma((size_t)reps);
        permutation_host(h, reps, sigma.data());
        for (int r = 0; r < reps; ++r)
            for (int64_t t = 0; t < nr; ++t) out[r * nr + t] = (uint32_t)(sigma[(size_t)r] * nr + t);
        return;
    }
    if (reps == 1) {
        permutation_host(h, n, out);
        return;
    }
    for (int r = 0; r < reps; ++r) {
        permutation_host(mix64(h ^ ((uint64_t)(r + 1) * kGolden)), nr, out + r * nr);
        for (int64_t t = 0; t < nr; ++t) out[r * nr + t] += (uint32_t)(r * nr);
    }
}

// Replication shuffle when R! >= S (at least S distinct orderings), else
// within-replication shuffle.
int shuffle_mode(int reps, int S) {
    if (reps < 2) return MTE_SHUFFLE_WITHIN;
    double f = 1.0;
    for (int r = 2; r <= reps && f < (double)S; ++r) f *= r;
    return f >= (double)S ? MTE_SHUFFLE_REPLICATIONS : MTE_SHUFFLE_WITHIN;
}

// ---------------------------------------------------------------- helpers
static thread_local hipStream_t t_stream = nullptr;

static int thread_stream(hipStream_t *s) {
    if (!t_stream) MTE_HIP(hipStreamCreateWithFlags(&t_stream, hipStreamNonBlocking));
    *s = t_stream;
    return MTE_OK;
}

static void fill_keys(JobSpec &sp, int S, uint64_t seed, uint32_t cand) {
    sp.keys.resize((size_t)S + 1);
    sp.keys[0] = EstKey{0, 1, 0};
    for (int s = 0; s < S; ++s) sp.keys[(size_t)s + 1] = EstKey{surrogate_key(seed, cand, (uint32_t)s), 0, 0};
}

// Host-buffer estimate with S surrogates; optional diagnostics.
static int host_estimate(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
                         int64_t N, int k, int theiler, int S, uint64_t seed, uint32_t cand,
                         double *cmi_out, float *eps_out, int32_t *nxz, int32_t *nyz, int32_t *nz,
                         int reps = 1, int rep_shuffle = 0) {
    int rc;
    if ((rc = validate_dims(dx, dy, dz, N, k))) return rc;
    if ((rc = validate_theiler(N, k, theiler))) return rc;
    if (S < 0) return fail(MTE_EINVAL, "S=%d must be >= 0", S);
    if (!X || !Y || (dz > 0 && !Z) || !cmi_out) return fail(MTE_EINVAL, "null pointer argument");
    if (dz == 0 && Z) return fail(MTE_EINVAL, "Z must be NULL when dz == 0");
    if ((rc = validate_host_finite(X, (int64_t)dx * N, "X"))) return rc;
    if ((rc = validate_host_finite(Y, (int64_t)dy * N, "Y"))) return rc;
    if (dz && (rc = validate_host_finite(Z, (int64_t)dz * N, "Z"))) return rc;
    if ((rc = ensure_init())) return rc;
    hipStream_t s;
    if ((rc = thread_stream(&s))) return rc;
    const int64_t E = (int64_t)S + 1;
    const bool diag = eps_out != nullptr;
    DevBuf in, out, deps, dcnt;
    const size_t nin = (size_t)(dx + dy + dz) * (size_t)N;
    if ((rc = in.ensure(sizeof(float) * nin))) return rc;
    if ((rc = out.ensure(sizeof(double) * (size_t)E))) return rc;
    if (diag) {
        if ((rc = deps.ensure(sizeof(float) * (size_t)E * N))) return rc;
        if ((rc = dcnt.ensure(sizeof(int32_t) * 3 * (size_t)E * N))) return rc;
    }
    float *d = in.as<float>();
    MTE_HIP(hipMemcpyAsync(d, X, sizeof(float) * dx * N, hipMemcpyHostToDevice, s));
    MTE_HIP(hipMemcpyAsync(d + (size_t)dx * N, Y, sizeof(float) * dy * N, hipMemcpyHostToDevice, s));
    if (dz) MTE_HIP(hipMemcpyAsync(d + (size_t)(dx + dy) * N, Z, sizeof(float) * dz * N, hipMemcpyHostToDevice, s));
    JobSpec sp;
    for (int c = 0; c < dx + dy + dz; ++c) sp.cols[c] = d + (size_t)c * N;
    sp.n = (int)N; sp.dx = dx; sp.dy = dy; sp.dz = dz; sp.k = k; sp.theiler = theiler;
    sp.reps = reps;
    sp.rep_shuffle = rep_shuffle;
    fill_keys(sp, S, seed, cand);
    sp.out = out.as<double>();
    if (diag) {
        sp.diag_eps = deps.as<float>();
        sp.diag_cnt = dcnt.as<int32_t>();
    }
    std::vector<JobSpec> specs{sp};
    if ((rc = run_blocking(specs, s))) return rc;
    std::vector<double> res((size_t)E);
    MTE_HIP(hipMemcpyAsync(res.data(), sp.out, sizeof(double) * E, hipMemcpyDeviceToHost, s));
    std::vector<int32_t> cnt;
    if (diag) {
        cnt.resize((size_t)3 * E * N);
        MTE_HIP(hipMemcpyAsync(eps_out, sp.diag_eps, sizeof(float) * E * N, hipMemcpyDeviceToHost, s));
        MTE_HIP(hipMemcpyAsync(cnt.data(), sp.diag_cnt, sizeof(int32_t) * 3 * E * N, hipMemcpyDeviceToHost, s));
    }
    MTE_HIP(hipStreamSynchronize(s));
    std::memcpy(cmi_out, res.data(), sizeof(double) * E);
    if (diag) {
        for (int64_t e = 0; e < E; ++e) {
            std::memcpy(nxz + e * N, cnt.data() + (e * 3 + 0) * N, sizeof(int32_t) * N);
            std::memcpy(nyz + e * N, cnt.data() + (e * 3 + 1) * N, sizeof(int32_t) * N);
            std::memcpy(nz + e * N, cnt.data() + (e * 3 + 2) * N, sizeof(int32_t) * N);
        }
    }
    return MTE_OK;
}

// ---------------------------------------------------------------- device-call cache
struct DevKey {
    const float *x, *y, *z;
    int dx, dy, dz;
    int64_t n, ld;
    int k, theiler, S;
    uint64_t seed;
    uint32_t cand;
    double *out;
    bool operator==(const DevKey &o) const {
        return std::tie(x, y, z, dx, dy, dz, n, ld, k, theiler, S, seed, cand, out) ==
               std::tie(o.x, o.y, o.z, o.dx, o.dy, o.dz, o.n, o.ld, o.k, o.theiler, o.S, o.seed, o.cand,
                        o.out);
    }
};

struct DevEntry {
    DevKey key;
    std::unique_ptr<Batch> batch;
};

static std::mutex g_dev_mu;
// most recent first; never destroyed, so no HIP call runs during static
// destruction at exit (mte_shutdown clears it).  Bounded in entries and in
// the device memory the cached launches hold.
static std::list<DevEntry> &g_dev_cache = *new std::list<DevEntry>;
static size_t g_dev_bytes = 0;
static constexpr size_t kDevCacheMax = 512;
static constexpr size_t kDevCacheBytes = (size_t)16 << 30;

static int dev_estimate(const float *dX, int dx, const float *dY, int dy, const float *dZ, int dz,
                        int64_t N, int64_t ld, int k, int theiler, int S, uint64_t seed, uint32_t cand,
                        double *d_out, void *stream) {
    int rc;
    if ((rc = validate_dims(dx, dy, dz, N, k))) return rc;
    if ((rc = validate_theiler(N, k, theiler))) return rc;
    if (S < 0) return fail(MTE_EINVAL, "S=%d must be >= 0", S);
    if (!dX || !dY || (dz > 0 && !dZ) || !d_out) return fail(MTE_EINVAL, "null pointer argument");
    if (ld < N) return fail(MTE_EINVAL, "ld=%lld < N", (long long)ld);
    if ((rc = ensure_init())) return rc;
    hipStream_t s = (hipStream_t)stream;
    DevKey key{dX, dY, dZ, dx, dy, dz, N, ld, k, theiler, S, seed, cand, d_out};
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto it = g_dev_cache.begin(); it != g_dev_cache.end(); ++it) {
        if (it->key == key) {
            g_dev_cache.splice(g_dev_cache.begin(), g_dev_cache, it);
            return g_dev_cache.front().batch->enqueue(s, true);
        }
    }
    JobSpec sp;
    for (int c = 0; c < dx; ++c) sp.cols[c] = dX + (size_t)c * ld;
    for (int c = 0; c < dy; ++c) sp.cols[dx + c] = dY + (size_t)c * ld;
    for (int c = 0; c < dz; ++c) sp.cols[dx + dy + c] = dZ + (size_t)c * ld;
    sp.n = (int)N; sp.dx = dx; sp.dy = dy; sp.dz = dz; sp.k = k; sp.theiler = theiler;
    fill_keys(sp, S, seed, cand);
    sp.out = d_out;
    std::vector<JobSpec> specs{sp};
    TileChoice tc;
    if ((rc = choose_tiles(specs, s, kTuneBatch, &tc))) return rc;
    auto b = std::make_unique<Batch>();
    if ((rc = b->prepare(specs, tc, s))) return rc;
    g_dev_bytes += b->device_bytes();
    g_dev_cache.push_front(DevEntry{key, std::move(b)});
    if (g_dev_cache.size() > kDevCacheMax || (g_dev_bytes > kDevCacheBytes && g_dev_cache.size() > 1)) {
        // the evicted launches may still be queued on some stream
        MTE_HIP(hipDeviceSynchronize());
        while (g_dev_cache.size() > 1 && (g_dev_cache.size() > kDevCacheMax || g_dev_bytes > kDevCacheBytes)) {
            g_dev_bytes -= g_dev_cache.back().batch->device_bytes();
            g_dev_cache.pop_back();
        }
    }
    return g_dev_cache.front().batch->enqueue(s, true);
}

void clear_dev_cache() {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_dev_cache.clear();
    g_dev_bytes = 0;
}

}  // namespace mte

using namespace mte;

extern "C" {

const char *mte_last_error(void) { return mte::last_error(); }

int mte_abi_version(void) { return 7; }

int mte_init(int device, size_t hbm_budget_bytes) { return init_device(device, hbm_budget_bytes); }

int mte_shutdown(void) {
    serve_shutdown();
    clear_dev_cache();
    return shutdown_all();
}

int cmi_ksg(const float *X, int dx, const float *Y, int dy, const float *Z, int dz, int64_t N, int k,
            double *cmi_out) {
    return host_estimate(X, dx, Y, dy, Z, dz, N, k, 0, 0, 0, 0, cmi_out, nullptr, nullptr, nullptr, nullptr);
}

int cmi_ksg_surrogates(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
                       int64_t N, int k, int S, uint64_t seed, double *cmi_out, double *surr_out) {
    if (S < 1) return fail(MTE_EINVAL, "S=%d must be >= 1", S);
    if (!surr_out || !cmi_out) return fail(MTE_EINVAL, "null output pointer");
    std::vector<double> all((size_t)S + 1);
    int rc = host_estimate(X, dx, Y, dy, Z, dz, N, k, 0, S, seed, 0, all.data(), nullptr, nullptr,
                           nullptr, nullptr);
    if (rc) return rc;
    *cmi_out = all[0];
    std::memcpy(surr_out, all.data() + 1, sizeof(double) * S);
    return MTE_OK;
}

int cmi_ksg_diag(const float *X, int dx, const float *Y, int dy, const float *Z, int dz, int64_t N,
                 int k, int S, uint64_t seed, uint32_t cand, double *cmi_out, float *eps_out,
                 int32_t *nxz_out, int32_t *nyz_out, int32_t *nz_out) {
    return cmi_ksg_diag_ex(X, dx, Y, dy, Z, dz, N, k, 0, S, seed, cand, cmi_out, eps_out, nxz_out, nyz_out,
                           nz_out);
}

int cmi_ksg_diag_ex(const float *X, int dx, const float *Y, int dy, const float *Z, int dz, int64_t N,
                    int k, int theiler, int S, uint64_t seed, uint32_t cand, double *cmi_out,
                    float *eps_out, int32_t *nxz_out, int32_t *nyz_out, int32_t *nz_out) {
    if (!eps_out || !nxz_out || !nyz_out || !nz_out) return fail(MTE_EINVAL, "null output pointer");
    return host_estimate(X, dx, Y, dy, Z, dz, N, k, theiler, S, seed, cand, cmi_out, eps_out, nxz_out,
                         nyz_out, nz_out);
}

int cmi_ksg_dev(const float *dX, int dx, const float *dY, int dy, const float *dZ, int dz, int64_t N,
                int64_t ld, int k, double *d_out, void *stream) {
    return dev_estimate(dX, dx, dY, dy, dZ, dz, N, ld, k, 0, 0, 0, 0, d_out, stream);
}

int cmi_ksg_surrogates_dev(const float *dX, int dx, const float *dY, int dy, const float *dZ, int dz,
                           int64_t N, int64_t ld, int k, int S, uint64_t seed, uint32_t cand,
                           double *d_out, void *stream) {
    return dev_estimate(dX, dx, dY, dy, dZ, dz, N, ld, k, 0, S, seed, cand, d_out, stream);
}

int cmi_ksg_surrogates_dev_ex(const float *dX, int dx, const float *dY, int dy, const float *dZ, int dz,
                              int64_t N, int64_t ld, int k, int theiler, int S, uint64_t seed,
                              uint32_t cand, double *d_out, void *stream) {
    return dev_estimate(dX, dx, dY, dy, dZ, dz, N, ld, k, theiler, S, seed, cand, d_out, stream);
}

int mte_autocorr_decay_time(const float *x, int64_t T, int max_lag, int *act_out) {
    if (!x || !act_out) return fail(MTE_EINVAL, "null pointer argument");
    if (T < 2 || max_lag < 1) return fail(MTE_EINVAL, "need T >= 2 and max_lag >= 1");
    int rc;
    if ((rc = validate_host_finite(x, T, "x"))) return rc;
    *act_out = autocorr_decay_time(x, T, max_lag);
    return MTE_OK;
}

int mte_permutation(uint64_t seed, uint32_t cand, uint32_t s, int64_t N, uint32_t *out) {
    if (N < 1 || N > 0x7fffffffLL) return fail(MTE_EINVAL, "N=%lld out of range", (long long)N);
    if (!out) return fail(MTE_EINVAL, "null output pointer");
    permutation_host(surrogate_key(seed, cand, s), N, out);
    return MTE_OK;
}

int mte_standardise(const float *in, int R, int P, int64_t T, float *out) {
    if (!in || !out || R < 1 || P < 1 || T < 1) return fail(MTE_EINVAL, "bad arguments");
    int rc;
    if ((rc = validate_host_finite(in, (int64_t)R * P * T, "data"))) return rc;
    standardise_host(in, R, P, T, out);
    return MTE_OK;
}

int mte_shuffle_mode(int R, int S, int *mode_out) {
    if (!mode_out || R < 1 || S < 1) return fail(MTE_EINVAL, "bad arguments");
    *mode_out = shuffle_mode(R, S);
    return MTE_OK;
}

int mte_permutation_rep(uint64_t seed, uint32_t cand, uint32_t s, int64_t N, int R, int mode, uint32_t *out) {
    if (N < 1 || N > 0x7fffffffLL) return fail(MTE_EINVAL, "N=%lld out of range", (long long)N);
    if (!out) return fail(MTE_EINVAL, "null output pointer");
    if (R < 1 || N % R) return fail(MTE_EINVAL, "N=%lld is not a multiple of R=%d", (long long)N, R);
    if (mode != MTE_SHUFFLE_WITHIN && mode != MTE_SHUFFLE_REPLICATIONS) return fail(MTE_EINVAL, "bad mode %d", mode);
    if (mode == MTE_SHUFFLE_REPLICATIONS && R < 2) return fail(MTE_EINVAL, "a replication shuffle needs R >= 2");
    replication_source_rows_host(surrogate_key(seed, cand, s), N, R, mode == MTE_SHUFFLE_REPLICATIONS, out);
    return MTE_OK;
}

int cmi_ksg_surrogates_rep(const float *X, int dx, const float *Y, int dy, const float *Z, int dz, int64_t N,
                           int R, int k, int S, uint64_t seed, uint32_t cand, int mode, double *cmi_out,
                           double *surr_out) {
    if (S < 1) return fail(MTE_EINVAL, "S=%d must be >= 1", S);
    if (!surr_out || !cmi_out) return fail(MTE_EINVAL, "null output pointer");
    if (R < 1 || N % R) return fail(MTE_EINVAL, "N=%lld is not a multiple of R=%d", (long long)N, R);
    if (mode == MTE_SHUFFLE_AUTO) mode = shuffle_mode(R, S);
    if (mode != MTE_SHUFFLE_WITHIN && mode != MTE_SHUFFLE_REPLICATIONS) return fail(MTE_EINVAL, "bad mode %d", mode);
    if (mode == MTE_SHUFFLE_REPLICATIONS && R < 2) return fail(MTE_EINVAL, "a replication shuffle needs R >= 2");
    std::vector<double> all((size_t)S + 1);
    int rc = host_estimate(X, dx, Y, dy, Z, dz, N, k, 0, S, seed, cand, all.data(), nullptr, nullptr, nullptr,
                           nullptr, R, mode == MTE_SHUFFLE_REPLICATIONS);
    if (rc) return rc;
    *cmi_out = all[0];
    std::memcpy(surr_out, all.data() + 1, sizeof(double) * S);
    return MTE_OK;
}

int mte_tile_configs(int32_t *cfg_out, int capacity, int *count_out) {
    if (!count_out || (capacity > 0 && !cfg_out)) return fail(MTE_EINVAL, "null argument");
    const int n = kernel_variant_count();
    for (int i = 0; i < n && i < capacity; ++i) {
        TileCfg c;
        kernel_variant(i, &c);
        const int32_t v[6] = {c.kmax, c.g, c.qp, c.dzm, c.dym, c.dxm};
        std::memcpy(cfg_out + 6 * i, v, sizeof v);
    }
    *count_out = n;
    return MTE_OK;
}

int mte_tune_report(char *buf, size_t cap, size_t *len_out) {
    if (!len_out || (cap && !buf)) return fail(MTE_EINVAL, "null pointer argument");
    std::string text;
    {
        Ctx &c = ctx();
        std::lock_guard<std::mutex> lk(c.mu);
        char line[512];
        for (const auto &t : c.tune_log) {
            snprintf(line, sizeof line,
                     "%s variant=%d split=%d build_rows=%d coop_lanes=%d grouped=%d scan_step=%d perm_cu=%d ms=%.4f "
                     "from=%s\n",
                     t.key.c_str(), t.tc.variant, t.tc.rs_mult, t.tc.build_qb, t.tc.coop_lanes, t.tc.grouped,
                     t.tc.scan_step, t.tc.perm_cu, t.ms, t.from_disk ? "file" : "tuned");
            text += line;
        }
    }
    *len_out = text.size();
    if (cap) {
        const size_t m = std::min(cap - 1, text.size());
        std::memcpy(buf, text.data(), m);
        buf[m] = '\0';
    }
    return MTE_OK;
}

int mte_kernel_timing(int enable) {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    c.timing = enable != 0;
    return MTE_OK;
}

int mte_kernel_timing_stage(int stage, int64_t *launches_out, double *total_ms_out, int reset) {
    if (stage < 0 || stage >= kStages) return fail(MTE_EINVAL, "stage %d out of range", stage);
    Ctx &c = ctx();
    std::vector<Ctx::Pending> ev;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        ev.swap(c.pending_events);
    }
    double add[kStages] = {};
    int64_t cnt[kStages] = {};
    for (auto &pe : ev) {
        MTE_HIP(hipEventSynchronize(pe.b));
        float ms = 0.f;
        MTE_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
        add[pe.stage] += ms;
        cnt[pe.stage] += 1;
    }
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto &pe : ev) {
        if (pe.own_a) c.event_pool.push_back(pe.a);
        c.event_pool.push_back(pe.b);
    }
    for (int t = 0; t < kStages; ++t) {
        c.timed_ms[t] += add[t];
        c.timed_launches[t] += cnt[t];
    }
    if (launches_out) *launches_out = c.timed_launches[stage];
    if (total_ms_out) *total_ms_out = c.timed_ms[stage];
    if (reset) {
        c.timed_ms[stage] = 0.0;
        c.timed_launches[stage] = 0;
    }
    return MTE_OK;
}

int mte_kernel_timing_read(int64_t *launches_out, double *total_ms_out, int reset) {
    return mte_kernel_timing_stage(kStageAllPairs, launches_out, total_ms_out, reset);
}

int mte_list_stats_enable(int enable) {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    c.list_stats = enable != 0;
    return MTE_OK;
}

int mte_list_stats(int64_t *pairs_out, int64_t *undecided_out, int64_t *entries_out, int reset) {
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    if (pairs_out) *pairs_out = c.list_pairs;
    if (undecided_out) *undecided_out = c.list_undecided;
    if (entries_out)
        for (int t = 0; t < 2; ++t) entries_out[t] = c.list_seen[t];
    if (reset) {
        c.list_pairs = c.list_undecided = 0;
        for (int t = 0; t < 2; ++t) c.list_seen[t] = 0;
    }
    return MTE_OK;
}

}  // extern "C"
