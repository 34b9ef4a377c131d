// Network-level inference: the greedy source selection of every target
// (through the request loop, targets running concurrently), the
// Benjamini-Hochberg correction over the targets' omnibus p-values, the
// inferred adjacency, and link statistics against a known structure.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "greedy.h"
#include "runtime.h"

namespace mte {

const char *last_error();
int select_sources_served(int32_t sid, int P, int64_t T, int target, const int32_t *candidates,
                          int n_candidates, int max_lag_sources, double alpha, const mte_opts *opts,
                          mte_result *out);

// Benjamini-Hochberg step-up at level q: sort ascending (stable), find the
// largest rank r with p_(r) <= q * (r/m), keep ranks 1..r.
static void fdr_bh(const double *p, int m, double q, uint8_t *keep) {
    std::vector<int> order((size_t)m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p[a] < p[b]; });
    int last = -1;
    for (int r = 0; r < m; ++r)
        if (p[order[(size_t)r]] <= q * ((double)(r + 1) / (double)m)) last = r;
    std::memset(keep, 0, (size_t)m);
    for (int r = 0; r <= last; ++r) keep[order[(size_t)r]] = 1;
}

}  // namespace mte

using namespace mte;

extern "C" {

int mte_fdr_bh(const double *p, int m, double q, uint8_t *keep_out) {
    if (!p || !keep_out || m < 1) return fail(MTE_EINVAL, "bad arguments");
    if (!(q > 0.0 && q < 1.0)) return fail(MTE_EINVAL, "q must be in (0,1)");
    for (int i = 0; i < m; ++i)
        if (!(p[i] >= 0.0 && p[i] <= 1.0)) return fail(MTE_EINVAL, "p[%d] is not a probability", i);
    fdr_bh(p, m, q, keep_out);
    return MTE_OK;
}

int mte_link_metrics(const uint8_t *inferred, const uint8_t *truth, int P, int64_t *counts_out,
                     double *rates_out) {
    if (!inferred || !truth || !counts_out || !rates_out || P < 1) return fail(MTE_EINVAL, "bad arguments");
    int64_t tp = 0, fp = 0, tn = 0, fn = 0;
    for (int s = 0; s < P; ++s)
        for (int t = 0; t < P; ++t) {
            if (s == t) continue;
            const bool a = inferred[(size_t)s * P + t] != 0, b = truth[(size_t)s * P + t] != 0;
            tp += a && b;
            fp += a && !b;
            tn += !a && !b;
            fn += !a && b;
        }
    counts_out[0] = tp;
    counts_out[1] = fp;
    counts_out[2] = tn;
    counts_out[3] = fn;
    auto div = [](int64_t x, int64_t y) { return y ? (double)x / (double)y : std::nan(""); };
    rates_out[0] = div(tp, tp + fp);   // precision
    rates_out[1] = div(tp, tp + fn);   // recall
    rates_out[2] = div(tn, tn + fp);   // specificity
    rates_out[3] = div(fp, fp + tn);   // false positive rate
    return MTE_OK;
}

int mte_infer_network(const float *data, int P, int64_t T, int max_lag_sources, double alpha, double alpha_fdr,
                      const mte_opts *opts, int n_threads, uint8_t *adj_out, mte_target_summary *targets_out) {
    if (!data || !adj_out || !targets_out) return fail(MTE_EINVAL, "null argument");
    if (P < 2) return fail(MTE_EINVAL, "need at least two processes");
    if (alpha_fdr > 0.0 && !(alpha_fdr < 1.0)) return fail(MTE_EINVAL, "alpha_fdr must be in (0,1) or <= 0");
    mte_opts base;
    base.k = 4;
    base.S = 200;
    base.max_lag_target = 5;
    base.seed = 0;
    base.theiler = 0;
    base.estimator = MTE_ESTIMATOR_KSG;
    base.replications = 1;
    base.standardise = 1;
    if (opts) base = *opts;
    // One replication: every target's search goes through the request loop
    // (concurrent targets share batches).  Several: the embedding of all
    // replications is gathered once and each target runs direct launches.
    const int R = base.replications;
    if (R < 1) return fail(MTE_EINVAL, "replications=%d must be >= 1", R);
    const int l_m = std::max(max_lag_sources, base.max_lag_target);
    int32_t sid = -1;
    DevBuf series, emb;
    Columns cols;
    int rc;
    std::vector<float> z;
    if (base.standardise) {
        if ((rc = validate_host_finite(data, (int64_t)R * P * T, "data"))) return rc;
        z.resize((size_t)R * P * T);
        standardise_host(data, R, P, T, z.data());
        data = z.data();
        base.standardise = 0;        // the targets' searches use the z-scored copy
    }
    if (R == 1) {
        if ((rc = mte_series_register(data, P, T, &sid))) return rc;
    } else {
        if (T <= l_m) return fail(MTE_EINVAL, "T=%lld too short", (long long)T);
        if ((int64_t)R * (T - l_m) > 0x7fffffffLL) return fail(MTE_EINVAL, "R*(T-L) exceeds 2^31-1 rows");
        if ((rc = ensure_init())) return rc;
        hipStream_t s;
        MTE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        rc = resident_columns(data, P, T, l_m, R, s, &series, &emb, &cols);
        (void)hipStreamDestroy(s);
        if (rc) return rc;
    }
    if (n_threads <= 0) n_threads = std::min(P, 16);
    n_threads = std::min(n_threads, P);

    struct Out {
        std::vector<mte_var> tp, src;
        mte_result res;
        int rc = MTE_OK;
        std::string err;
    };
    std::vector<Out> outs((size_t)P);
    std::atomic<int> next{0};
    auto worker = [&]() {
        for (;;) {
            const int t = next.fetch_add(1);
            if (t >= P) return;
            Out &o = outs[(size_t)t];
            std::vector<int32_t> cands;
            for (int j = 0; j < P; ++j)
                if (j != t) cands.push_back(j);
            o.tp.assign((size_t)std::max(1, base.max_lag_target), mte_var{});
            o.src.assign((size_t)std::max(1, (P - 1) * max_lag_sources), mte_var{});
            std::memset(&o.res, 0, sizeof o.res);
            o.res.target_past = o.tp.data();
            o.res.sources = o.src.data();
            mte_opts mo = base;
            mo.seed = base.seed + (uint64_t)t;
            if (R == 1) {
                o.rc = select_sources_served(sid, P, T, t, cands.data(), (int)cands.size(), max_lag_sources,
                                             alpha, &mo, &o.res);
            } else {
                o.rc = greedy_check(P, T, t, cands.data(), (int)cands.size(), max_lag_sources, alpha, mo, &o.res);
                if (!o.rc)
                    o.rc = select_sources_columns(cols, t, cands.data(), (int)cands.size(), max_lag_sources, alpha,
                                                  mo, &o.res);
            }
            if (o.rc) o.err = last_error();
        }
    };
    std::vector<std::thread> pool;
    for (int i = 0; i < n_threads; ++i) pool.emplace_back(worker);
    for (auto &th : pool) th.join();
    if (sid >= 0) (void)mte_series_release(sid);
    for (int t = 0; t < P; ++t)
        if (outs[(size_t)t].rc) return fail(outs[(size_t)t].rc, "target %d: %s", t, outs[(size_t)t].err.c_str());

    std::vector<double> pv((size_t)P);
    for (int t = 0; t < P; ++t) pv[(size_t)t] = outs[(size_t)t].res.omnibus_p;
    std::vector<uint8_t> keep((size_t)P, 1);
    if (alpha_fdr > 0.0) fdr_bh(pv.data(), P, alpha_fdr, keep.data());
    std::memset(adj_out, 0, (size_t)P * P);
    for (int t = 0; t < P; ++t) {
        const mte_result &r = outs[(size_t)t].res;
        mte_target_summary &ts = targets_out[t];
        ts.n_target_past = r.n_target_past;
        ts.n_sources = r.n_sources;
        ts.n_sources_tested = r.n_sources_tested;
        ts.omnibus_te = r.omnibus_te;
        ts.omnibus_p = r.omnibus_p;
        ts.significant = r.significant;
        ts.fdr_kept = keep[(size_t)t];
        ts.n_estimates = r.n_estimates;
        if (r.significant && keep[(size_t)t])
            for (int i = 0; i < r.n_sources; ++i) adj_out[(size_t)r.sources[i].node * P + t] = 1;
    }
    return MTE_OK;
}

}  // extern "C"
