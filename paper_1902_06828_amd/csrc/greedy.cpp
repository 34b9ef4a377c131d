// Significance tests and the four-step greedy source selection for one target
// (Inference algorithm and Statistical tests sections of the paper).
//
// Readings of the paper fixed here (the same ones the oracle uses):
//  * embedding rows t = L..T-1, L = max(l_target, l_sources), N = T - L;
//    variable (node, lag) is series[node][t - lag];
//  * candidate order: target lags ascending; sources in the given order with
//    lags ascending; removing a variable keeps the order of the rest; ties in
//    the maximum or minimum go to the first candidate in that order;
//  * surrogate keys: a running candidate-test counter (one per candidate per
//    round, then one for the omnibus test) is the `cand` of pi_{seed,cand,s};
//  * alpha is used for the maximum, minimum and omnibus tests; p counts the
//    surrogate statistics strictly larger than the observed one, and a test
//    is significant iff p < alpha (S*alpha > 1 is required);
//  * step 3 removes the minimising variable while its minimum-statistic test
//    is not significant; an empty X^S skips the omnibus test (p = 1).
#include <algorithm>
#include <chrono>
#include <map>
#include <cstring>

#include "gauss.h"
#include "greedy.h"
#include "runtime.h"

namespace mte {

int stat_max(const double *real, const double *surr, int n, int S, double alpha, int *idx,
             double *p, int *sig) {
    if (n < 1 || S < 1) return fail(MTE_EINVAL, "need n >= 1 and S >= 1");
    if (!(S * alpha > 1.0)) return fail(MTE_EINVAL, "S*alpha must exceed 1 (S=%d, alpha=%g)", S, alpha);
    int j = 0;
    for (int c = 1; c < n; ++c)
        if (real[c] > real[j]) j = c;
    int larger = 0;
    for (int s = 0; s < S; ++s) {
        double m = surr[s];
        for (int c = 1; c < n; ++c) m = std::max(m, surr[(size_t)c * S + s]);
        larger += m > real[j];
    }
    *idx = j;
    *p = (double)larger / (double)S;
    *sig = *p < alpha;
    return MTE_OK;
}

int stat_min(const double *real, const double *surr, int n, int S, double alpha, int *idx,
             double *p, int *sig) {
    if (n < 1 || S < 1) return fail(MTE_EINVAL, "need n >= 1 and S >= 1");
    if (!(S * alpha > 1.0)) return fail(MTE_EINVAL, "S*alpha must exceed 1 (S=%d, alpha=%g)", S, alpha);
    int j = 0;
    for (int c = 1; c < n; ++c)
        if (real[c] < real[j]) j = c;
    int larger = 0;
    for (int s = 0; s < S; ++s) {
        double m = surr[s];
        for (int c = 1; c < n; ++c) m = std::min(m, surr[(size_t)c * S + s]);
        larger += m > real[j];
    }
    *idx = j;
    *p = (double)larger / (double)S;
    *sig = *p < alpha;
    return MTE_OK;
}

int stat_omnibus(double real, const double *surr, int S, double alpha, double *p, int *sig) {
    if (S < 1) return fail(MTE_EINVAL, "need S >= 1");
    if (!(S * alpha > 1.0)) return fail(MTE_EINVAL, "S*alpha must exceed 1 (S=%d, alpha=%g)", S, alpha);
    int larger = 0;
    for (int s = 0; s < S; ++s) larger += surr[s] > real;
    *p = (double)larger / (double)S;
    *sig = *p < alpha;
    return MTE_OK;
}

// ---------------------------------------------------------------- greedy
struct Var {
    int node, lag;
    bool operator==(const Var &o) const { return node == o.node && lag == o.lag; }
};

// One test round: candidate j has X = xs[j] (one or more variables, rows
// shuffled jointly in surrogates), Y = target present, Z = zs[j].
struct Round {
    std::vector<std::vector<Var>> xs, zs;
};

// Executes rounds; `tid0` is the first candidate-test counter of the round.
class RoundExec {
public:
    virtual ~RoundExec() = default;
    // real[n], surr[n][S]
    virtual int run(const Round &r, uint32_t tid0, std::vector<double> *real,
                    std::vector<double> *surr) = 0;
    // true: no surrogates; the tests use the chi^2 null with `rows` samples
    virtual bool analytic() const { return false; }
    virtual int64_t rows() const { return 0; }
    double gpu_seconds = 0.0;
};

static int build_embedding(const float *dev_data, int R, int P, int64_t T, int l_m, hipStream_t s, DevBuf *buf,
                           Columns *c) {
    const int64_t nr = T - l_m, N = (int64_t)R * nr;
    if (N > 0x7fffffffLL) return fail(MTE_EINVAL, "R*(T-L) exceeds 2^31-1 rows");
    int rc;
    if ((rc = buf->ensure(sizeof(float) * (size_t)P * (l_m + 1) * N))) return rc;
    float *e = buf->as<float>();
    for (int node = 0; node < P; ++node)
        for (int lag = 0; lag <= l_m; ++lag)
            MTE_HIP(hipMemcpy2DAsync(e + ((size_t)node * (l_m + 1) + lag) * N, sizeof(float) * nr,
                                     dev_data + (size_t)node * T + (l_m - lag), sizeof(float) * (size_t)P * T,
                                     sizeof(float) * nr, R, hipMemcpyDeviceToDevice, s));
    MTE_HIP(hipStreamSynchronize(s));
    c->series = dev_data;
    c->T = T;
    c->l_m = l_m;
    c->emb = e;
    c->N = N;
    c->reps = R;
    return MTE_OK;
}

// Direct executor: every round is one batched launch.
class DirectExec : public RoundExec {
public:
    DirectExec(const Columns &cols, int64_t N, int target, int k, int S, uint64_t seed, int theiler)
        : c_(cols), N_(N), target_(target), k_(k), S_(S), w_(theiler), seed_(seed),
          rep_shuffle_(cols.reps > 1 && shuffle_mode(cols.reps, S) == MTE_SHUFFLE_REPLICATIONS) {}
    int run(const Round &r, uint32_t tid0, std::vector<double> *real, std::vector<double> *surr) override {
        const int n = (int)r.xs.size();
        const int E = S_ + 1;
        int rc;
        if ((rc = out_.ensure(sizeof(double) * (size_t)n * E))) return rc;
        std::vector<JobSpec> specs((size_t)n);
        for (int j = 0; j < n; ++j) {
            JobSpec &sp = specs[(size_t)j];
            int c = 0;
            for (const Var &v : r.xs[j]) sp.cols[c++] = col(v);
            sp.cols[c++] = col(Var{target_, 0});
            for (const Var &v : r.zs[j]) sp.cols[c++] = col(v);
            sp.n = (int)N_;
            sp.dx = (int)r.xs[j].size();
            sp.dy = 1;
            sp.dz = (int)r.zs[j].size();
            sp.k = k_;
            sp.theiler = w_;
            sp.reps = c_.reps;
            sp.rep_shuffle = rep_shuffle_;
            sp.keys.resize((size_t)E);
            sp.keys[0] = EstKey{0, 1, 0};
            for (int s = 0; s < S_; ++s)
                sp.keys[(size_t)s + 1] = EstKey{surrogate_key(seed_, tid0 + (uint32_t)j, (uint32_t)s), 0, 0};
            sp.out = out_.as<double>() + (size_t)j * E;
        }
        hipStream_t s;
        if ((rc = stream(&s))) return rc;
        auto t0 = std::chrono::steady_clock::now();
        if ((rc = run_blocking(specs, s))) return rc;
        std::vector<double> all((size_t)n * E);
        MTE_HIP(hipMemcpyAsync(all.data(), out_.p, sizeof(double) * all.size(), hipMemcpyDeviceToHost, s));
        MTE_HIP(hipStreamSynchronize(s));
        gpu_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        real->assign((size_t)n, 0.0);
        surr->assign((size_t)n * S_, 0.0);
        for (int j = 0; j < n; ++j) {
            (*real)[(size_t)j] = all[(size_t)j * E];
            std::memcpy(surr->data() + (size_t)j * S_, all.data() + (size_t)j * E + 1, sizeof(double) * S_);
        }
        return MTE_OK;
    }
    ~DirectExec() override {
        if (s_) (void)hipStreamDestroy(s_);
    }
private:
    const float *col(const Var &v) const { return c_.col(v.node, v.lag); }
    int stream(hipStream_t *s) {
        if (!s_) MTE_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
        *s = s_;
        return MTE_OK;
    }
    Columns c_;
    int64_t N_;
    int target_, k_, S_, w_;
    uint64_t seed_;
    int rep_shuffle_;
    DevBuf out_;
    hipStream_t s_ = nullptr;
};

// Served executor: every candidate test is one request of the request loop.
class ServedExec : public RoundExec {
public:
    ServedExec(int32_t sid, int l_m, int64_t N, int target, int k, int S, uint64_t seed, int theiler)
        : sid_(sid), lm_(l_m), N_(N), target_(target), k_(k), S_(S), w_(theiler), seed_(seed) {}
    int run(const Round &r, uint32_t tid0, std::vector<double> *real, std::vector<double> *surr) override {
        const int n = (int)r.xs.size();
        std::vector<uint64_t> tickets((size_t)n);
        auto t0 = std::chrono::steady_clock::now();
        for (int j = 0; j < n; ++j) {
            std::vector<int32_t> nodes, lags;
            for (const Var &v : r.xs[j]) { nodes.push_back(v.node); lags.push_back(v.lag); }
            nodes.push_back(target_);
            lags.push_back(0);
            for (const Var &v : r.zs[j]) { nodes.push_back(v.node); lags.push_back(v.lag); }
            mte_request q;
            std::memset(&q, 0, sizeof q);
            q.sid = sid_;
            q.dx = (int)r.xs[j].size();
            q.dy = 1;
            q.dz = (int)r.zs[j].size();
            q.nodes = nodes.data();
            q.lags = lags.data();
            q.t0 = lm_;
            q.N = N_;
            q.k = k_;
            q.S = S_;
            q.seed = seed_;
            q.cand = tid0 + (uint32_t)j;
            q.theiler = w_;
            int rc = mte_submit(&q, &tickets[(size_t)j]);
            if (rc) {
                // retire the requests already queued before returning
                std::vector<double> junk((size_t)S_ + 1);
                for (int t = 0; t < j; ++t) (void)mte_wait(tickets[(size_t)t], junk.data(), junk.data() + 1, -1.0);
                return rc;
            }
        }
        real->assign((size_t)n, 0.0);
        surr->assign((size_t)n * S_, 0.0);
        int first_err = MTE_OK;
        for (int j = 0; j < n; ++j) {
            int rc = mte_wait(tickets[(size_t)j], &(*real)[(size_t)j], surr->data() + (size_t)j * S_, -1.0);
            if (rc && !first_err) first_err = rc;
        }
        gpu_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return first_err;
    }
private:
    int32_t sid_;
    int lm_;
    int64_t N_;
    int target_, k_, S_, w_;
    uint64_t seed_;
};

// Gaussian executor: one float64 covariance matrix of every variable the
// search can touch (target present, target lags 1..l_t, each candidate with
// lags 1..l_s), computed once; each round is one launch of the estimate
// kernel over index sets into that matrix.  No surrogates.
class GaussExec : public RoundExec {
public:
    GaussExec(const Columns &cols, int64_t N, int target, const int32_t *cands, int n_cands, int l_s, int l_t)
        : c_(cols), N_(N), target_(target), ls_(l_s), lt_(l_t) {
        for (int i = 0; i < n_cands; ++i) slot_[cands[i]] = i;
        cols_.push_back(col(Var{target, 0}));
        for (int l = 1; l <= l_t; ++l) cols_.push_back(col(Var{target, l}));
        for (int i = 0; i < n_cands; ++i)
            for (int l = 1; l <= l_s; ++l) cols_.push_back(col(Var{cands[i], l}));
    }
    bool analytic() const override { return true; }
    int64_t rows() const override { return N_; }
    int run(const Round &r, uint32_t, std::vector<double> *real, std::vector<double> *surr) override {
        int rc;
        hipStream_t s;
        if ((rc = stream(&s))) return rc;
        auto t0 = std::chrono::steady_clock::now();
        if (!have_cov_) {
            if ((int)cols_.size() > kGaussMaxD)
                return fail(MTE_EINVAL, "%zu variables exceed the %d-column covariance limit", cols_.size(),
                            kGaussMaxD);
            if ((rc = gauss_covariance(cols_, N_, s, &work_, &cov_))) return rc;
            have_cov_ = true;
        }
        const int n = (int)r.xs.size();
        std::vector<GaussJob> jobs((size_t)n);
        std::vector<int32_t> idx;
        for (int j = 0; j < n; ++j) {
            jobs[(size_t)j] = GaussJob{(int32_t)r.xs[j].size(), 1, (int32_t)r.zs[j].size(), (int32_t)idx.size()};
            for (const Var &v : r.zs[j]) idx.push_back(index(v));
            for (const Var &v : r.xs[j]) idx.push_back(index(v));
            idx.push_back(0);
        }
        if ((rc = gauss_estimates(cov_.as<double>(), (int)cols_.size(), jobs, idx, s, &wj_, real))) return rc;
        gpu_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        surr->clear();
        return MTE_OK;
    }
    ~GaussExec() override {
        if (s_) (void)hipStreamDestroy(s_);
    }
private:
    const float *col(const Var &v) const { return c_.col(v.node, v.lag); }
    int index(const Var &v) const {
        if (v.node == target_) return v.lag;
        return 1 + lt_ + slot_.at(v.node) * ls_ + (v.lag - 1);
    }
    int stream(hipStream_t *s) {
        if (!s_) MTE_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
        *s = s_;
        return MTE_OK;
    }
    Columns c_;
    int64_t N_;
    int target_, ls_, lt_;
    std::map<int, int> slot_;
    std::vector<const float *> cols_;
    bool have_cov_ = false;
    DevBuf work_, cov_, wj_;
    hipStream_t s_ = nullptr;
};

// The three tests of a round: surrogate-based, or with the analytic null.
static int test_max(const RoundExec &ex, const std::vector<double> &real, const std::vector<double> &surr, int S,
                    double alpha, int *j, double *p, int *sig) {
    if (!ex.analytic()) return stat_max(real.data(), surr.data(), (int)real.size(), S, alpha, j, p, sig);
    const int n = (int)real.size();
    *j = (int)(std::max_element(real.begin(), real.end()) - real.begin());
    *p = p_max_analytic(real[(size_t)*j], n, ex.rows());
    *sig = *p < alpha;
    return MTE_OK;
}

static int test_min(const RoundExec &ex, const std::vector<double> &real, const std::vector<double> &surr, int S,
                    double alpha, int *j, double *p, int *sig) {
    if (!ex.analytic()) return stat_min(real.data(), surr.data(), (int)real.size(), S, alpha, j, p, sig);
    const int n = (int)real.size();
    *j = (int)(std::min_element(real.begin(), real.end()) - real.begin());
    *p = p_min_analytic(real[(size_t)*j], n, ex.rows());
    *sig = *p < alpha;
    return MTE_OK;
}

static int greedy(RoundExec &ex, int target, const int32_t *cands, int n_cands, int l_s, int l_t,
                  double alpha, int S, mte_result *out) {
    if (ex.analytic()) S = 0;
    uint32_t tid = 0;
    int64_t n_est = 0;
    std::vector<double> real, surr;
    int rc;
    // Step 1: target past
    std::vector<Var> ycand, ysel;
    std::vector<std::pair<double, double>> ystat;
    for (int l = 1; l <= l_t; ++l) ycand.push_back(Var{target, l});
    while (!ycand.empty()) {
        Round r;
        for (const Var &c : ycand) { r.xs.push_back({c}); r.zs.push_back(ysel); }
        if ((rc = ex.run(r, tid, &real, &surr))) return rc;
        tid += (uint32_t)ycand.size();
        n_est += (int64_t)ycand.size() * (S + 1);
        int j, sig;
        double p;
        if ((rc = test_max(ex, real, surr, S, alpha, &j, &p, &sig))) return rc;
        if (!sig) break;
        ysel.push_back(ycand[(size_t)j]);
        ystat.emplace_back(real[(size_t)j], p);
        ycand.erase(ycand.begin() + j);
    }
    // Step 2: sources past
    std::vector<Var> xcand, xsel;
    std::vector<std::pair<double, double>> xstat;
    for (int i = 0; i < n_cands; ++i)
        for (int l = 1; l <= l_s; ++l) xcand.push_back(Var{cands[i], l});
    while (!xcand.empty()) {
        if ((int)(ysel.size() + xsel.size()) + 1 > kMaxDz)
            return fail(MTE_EINVAL, "conditioning set would exceed %d variables", kMaxDz);
        std::vector<Var> cond = ysel;
        cond.insert(cond.end(), xsel.begin(), xsel.end());
        Round r;
        for (const Var &c : xcand) { r.xs.push_back({c}); r.zs.push_back(cond); }
        if ((rc = ex.run(r, tid, &real, &surr))) return rc;
        tid += (uint32_t)xcand.size();
        n_est += (int64_t)xcand.size() * (S + 1);
        int j, sig;
        double p;
        if ((rc = test_max(ex, real, surr, S, alpha, &j, &p, &sig))) return rc;
        if (!sig) break;
        xsel.push_back(xcand[(size_t)j]);
        xstat.emplace_back(real[(size_t)j], p);
        xcand.erase(xcand.begin() + j);
    }
    // Step 3: pruning
    while (!xsel.empty()) {
        Round r;
        for (size_t c = 0; c < xsel.size(); ++c) {
            std::vector<Var> cond = ysel;
            for (size_t o = 0; o < xsel.size(); ++o)
                if (o != c) cond.push_back(xsel[o]);
            r.xs.push_back({xsel[c]});
            r.zs.push_back(cond);
        }
        if ((rc = ex.run(r, tid, &real, &surr))) return rc;
        tid += (uint32_t)xsel.size();
        n_est += (int64_t)xsel.size() * (S + 1);
        int j, sig;
        double p;
        if ((rc = test_min(ex, real, surr, S, alpha, &j, &p, &sig))) return rc;
        if (sig) break;
        xsel.erase(xsel.begin() + j);
        xstat.erase(xstat.begin() + j);
    }
    // Step 4: omnibus
    double omni = 0.0, omni_p = 1.0;
    int omni_sig = 0;
    if (!xsel.empty()) {
        if ((int)xsel.size() > kMaxDx)
            return fail(MTE_EINVAL, "%zu selected sources exceed the %d-column limit", xsel.size(), kMaxDx);
        Round r;
        r.xs.push_back(xsel);
        r.zs.push_back(ysel);
        if ((rc = ex.run(r, tid, &real, &surr))) return rc;
        tid += 1;
        n_est += S + 1;
        omni = real[0];
        if (ex.analytic()) {
            omni_p = chi2_sf(2.0 * (double)ex.rows() * omni, (int)xsel.size());
            omni_sig = omni_p < alpha;
        } else if ((rc = stat_omnibus(omni, surr.data(), S, alpha, &omni_p, &omni_sig))) {
            return rc;
        }
    }
    out->n_target_past = (int)ysel.size();
    for (size_t i = 0; i < ysel.size(); ++i)
        out->target_past[i] = mte_var{ysel[i].node, ysel[i].lag, ystat[i].first, ystat[i].second};
    out->n_sources_tested = (int)xsel.size();
    for (size_t i = 0; i < xsel.size(); ++i)
        out->sources[i] = mte_var{xsel[i].node, xsel[i].lag, xstat[i].first, xstat[i].second};
    out->n_sources = omni_sig ? (int)xsel.size() : 0;
    out->omnibus_te = omni;
    out->omnibus_p = omni_p;
    out->significant = omni_sig;
    out->n_estimates = n_est;
    out->gpu_seconds = ex.gpu_seconds;
    return MTE_OK;
}

static int check_greedy_args(int P, int64_t T, int target, const int32_t *cands, int n_cands, int l_s,
                             double alpha, const mte_opts &o, mte_result *out) {
    if (!out || !cands || n_cands < 0) return fail(MTE_EINVAL, "null argument");
    if (P < 1 || target < 0 || target >= P) return fail(MTE_EINVAL, "target %d out of range", target);
    if (l_s < 1 || o.max_lag_target < 1) return fail(MTE_EINVAL, "maximum lags must be >= 1");
    if (o.estimator != MTE_ESTIMATOR_KSG && o.estimator != MTE_ESTIMATOR_GAUSS)
        return fail(MTE_EINVAL, "unknown estimator %d", o.estimator);
    const bool gauss = o.estimator == MTE_ESTIMATOR_GAUSS;
    if (!gauss && (o.k < 1 || o.k > kMaxK)) return fail(MTE_EINVAL, "k=%d out of range", o.k);
    if (!gauss && (o.S < 1 || !(o.S * alpha > 1.0))) return fail(MTE_EINVAL, "S*alpha must exceed 1");
    if (gauss && o.theiler != 0) return fail(MTE_EINVAL, "the Theiler window applies to the KSG estimator only");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(MTE_EINVAL, "alpha must be in (0,1)");
    for (int i = 0; i < n_cands; ++i) {
        if (cands[i] < 0 || cands[i] >= P) return fail(MTE_EINVAL, "candidate %d out of range", cands[i]);
        if (cands[i] == target) return fail(MTE_EINVAL, "the target is among the candidates");
        for (int j = 0; j < i; ++j)
            if (cands[j] == cands[i]) return fail(MTE_EINVAL, "duplicate candidate %d", cands[i]);
    }
    const int l_m = std::max(l_s, o.max_lag_target);
    const int R = o.replications;
    if (R < 1) return fail(MTE_EINVAL, "replications=%d must be >= 1", R);
    if (R > 1 && o.theiler) return fail(MTE_EINVAL, "the Theiler window needs a single replication");
    if (T <= (int64_t)l_m + (gauss ? 1 : o.k)) return fail(MTE_EINVAL, "T=%lld too short", (long long)T);
    if (!gauss) {
        int rc = validate_theiler(T - l_m, o.k, o.theiler);
        if (rc) return rc;
    }
    if ((int64_t)R * (T - l_m) > 0x7fffffffLL) return fail(MTE_EINVAL, "R*(T-L) exceeds 2^31-1 rows");
    if (!out->target_past || (n_cands > 0 && !out->sources))
        return fail(MTE_EINVAL, "result arrays must be allocated by the caller");
    return MTE_OK;
}

static mte_opts opts_or_default(const mte_opts *o) {
    mte_opts d;
    d.k = 4;
    d.S = 200;
    d.max_lag_target = 5;
    d.seed = 0;
    d.theiler = 0;
    d.estimator = MTE_ESTIMATOR_KSG;
    d.replications = 1;
    d.standardise = 1;
    return o ? *o : d;
}

int series_pin(int32_t sid, const float **dev, int *P, int64_t *T);
void series_unpin(int32_t sid);
int series_standardised(int32_t sid, int32_t *std_sid);

// Greedy search of one target over resident columns (arguments checked).
int select_sources_columns(const Columns &c, int target, const int32_t *candidates, int n_candidates,
                           int max_lag_sources, double alpha, const mte_opts &o, mte_result *out) {
    const int64_t N = (int64_t)c.reps * (c.T - c.l_m);
    if (o.estimator == MTE_ESTIMATOR_GAUSS) {
        GaussExec ex(c, N, target, candidates, n_candidates, max_lag_sources, o.max_lag_target);
        return greedy(ex, target, candidates, n_candidates, max_lag_sources, o.max_lag_target, alpha, o.S, out);
    }
    DirectExec ex(c, N, target, o.k, o.S, o.seed, o.theiler);
    return greedy(ex, target, candidates, n_candidates, max_lag_sources, o.max_lag_target, alpha, o.S, out);
}

int select_sources_served(int32_t sid, int P, int64_t T, int target, const int32_t *candidates,
                          int n_candidates, int max_lag_sources, double alpha, const mte_opts *opts,
                          mte_result *out) {
    const mte_opts o = opts_or_default(opts);
    int rc = check_greedy_args(P, T, target, candidates, n_candidates, max_lag_sources, alpha, o, out);
    if (rc) return rc;
    if (o.replications != 1)
        return fail(MTE_EINVAL, "a registered series has one replication (use mte_select_sources or "
                                "mte_infer_network for replications)");
    if (o.standardise && (rc = series_standardised(sid, &sid))) return rc;
    const int l_m = std::max(max_lag_sources, o.max_lag_target);
    if (o.estimator == MTE_ESTIMATOR_GAUSS) {
        const float *dev;
        int P2;
        int64_t T2;
        if ((rc = series_pin(sid, &dev, &P2, &T2))) return rc;
        Columns c;
        c.series = dev;
        c.T = T;
        c.l_m = l_m;
        rc = select_sources_columns(c, target, candidates, n_candidates, max_lag_sources, alpha, o, out);
        series_unpin(sid);
        return rc;
    }
    ServedExec ex(sid, l_m, T - l_m, target, o.k, o.S, o.seed, o.theiler);
    return greedy(ex, target, candidates, n_candidates, max_lag_sources, o.max_lag_target, alpha, o.S, out);
}

// Device copy of a host series [R][P][T] (R = o.replications) and its
// columns; with R > 1 the embedding of every (node, lag <= l_m) is gathered.
int resident_columns(const float *data, int P, int64_t T, int l_m, int R, hipStream_t s, DevBuf *series,
                     DevBuf *emb, Columns *c) {
    int rc;
    const size_t count = (size_t)R * P * T;
    if ((rc = validate_host_finite(data, (int64_t)count, "data"))) return rc;
    if ((rc = series->ensure(sizeof(float) * count))) return rc;
    MTE_HIP(hipMemcpyAsync(series->p, data, sizeof(float) * count, hipMemcpyHostToDevice, s));
    MTE_HIP(hipStreamSynchronize(s));
    if (R > 1) return build_embedding(series->as<float>(), R, P, T, l_m, s, emb, c);
    c->series = series->as<float>();
    c->T = T;
    c->l_m = l_m;
    c->emb = nullptr;
    c->N = T - l_m;
    c->reps = 1;
    return MTE_OK;
}

int greedy_check(int P, int64_t T, int target, const int32_t *cands, int n_cands, int l_s, double alpha,
                 const mte_opts &o, mte_result *out) {
    return check_greedy_args(P, T, target, cands, n_cands, l_s, alpha, o, out);
}

mte_opts greedy_opts(const mte_opts *o) { return opts_or_default(o); }

}  // namespace mte

using namespace mte;

extern "C" {

int mte_max_statistic(const double *real, const double *surr, int n, int S, double alpha,
                      int *index_out, double *p_out, int *significant_out) {
    if (!real || !surr || !index_out || !p_out || !significant_out) return fail(MTE_EINVAL, "null argument");
    return stat_max(real, surr, n, S, alpha, index_out, p_out, significant_out);
}

int mte_min_statistic(const double *real, const double *surr, int n, int S, double alpha,
                      int *index_out, double *p_out, int *significant_out) {
    if (!real || !surr || !index_out || !p_out || !significant_out) return fail(MTE_EINVAL, "null argument");
    return stat_min(real, surr, n, S, alpha, index_out, p_out, significant_out);
}

int mte_omnibus(double real, const double *surr, int S, double alpha, double *p_out, int *significant_out) {
    if (!surr || !p_out || !significant_out) return fail(MTE_EINVAL, "null argument");
    return stat_omnibus(real, surr, S, alpha, p_out, significant_out);
}

int mte_select_sources(const float *data, int P, int64_t T, int target, const int32_t *candidates,
                       int n_candidates, int max_lag_sources, double alpha, const mte_opts *opts,
                       mte_result *out) {
    const mte_opts o = opts_or_default(opts);
    int rc = check_greedy_args(P, T, target, candidates, n_candidates, max_lag_sources, alpha, o, out);
    if (rc) return rc;
    if (!data) return fail(MTE_EINVAL, "null data");
    if ((rc = ensure_init())) return rc;
    const int l_m = std::max(max_lag_sources, o.max_lag_target);
    std::vector<float> z;
    if (o.standardise) {
        if ((rc = validate_host_finite(data, (int64_t)o.replications * P * T, "data"))) return rc;
        z.resize((size_t)o.replications * P * T);
        standardise_host(data, o.replications, P, T, z.data());
        data = z.data();
    }
    hipStream_t s;
    MTE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    DevBuf series, emb;
    Columns c;
    rc = resident_columns(data, P, T, l_m, o.replications, s, &series, &emb, &c);
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    return select_sources_columns(c, target, candidates, n_candidates, max_lag_sources, alpha, o, out);
}

}  // extern "C"
