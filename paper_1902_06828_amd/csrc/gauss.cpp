// Host side of the Gaussian estimator: workspace, launches, the chi-squared
// survival function of the analytic null, and the C ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gauss.h"
#include "runtime.h"

namespace mte {

// One launch, bracketed by HIP events on its stream when kernel timing is on.
template <class F>
static int timed_launch(int stage, hipStream_t s, F launch) {
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = ctx().timing;
    if (timed) {
        int rc;
        if ((rc = timing_event(&ev[0])) || (rc = timing_event(&ev[1]))) return rc;
        MTE_HIP(hipEventRecord(ev[0], s));
    }
    if (launch()) return hip_fail(hipGetLastError(), "Gaussian estimator launch");
    if (timed) {
        MTE_HIP(hipEventRecord(ev[1], s));
        record_timing_pair(stage, ev[0], ev[1]);
    }
    return MTE_OK;
}

// P(chi^2_dof > x) = Q(dof/2, x/2), the regularised upper incomplete gamma
// function, for integer dof (h = x/2):
//   dof = 2m:    Q = e^{-h} sum_{i=0}^{m-1} h^i / i!
//   dof = 2m+1:  Q = erfc(sqrt h) + e^{-h} sum_{i=1}^{m} h^{i-1/2} / Gamma(i+1/2)
// (the finite series of the incomplete gamma function at integer and
// half-integer order).  The sums run in log space (log-sum-exp), so large h
// underflows to 0 only where the true value does.
double chi2_sf(double x, int dof) {
    if (dof < 1) return std::nan("");
    if (!(x > 0.0)) return 1.0;
    const double h = 0.5 * x, lh = std::log(h);
    const bool odd = dof & 1;
    const int m = dof / 2;
    const int first = odd ? 1 : 0, last = odd ? m : m - 1;
    double series = 0.0;
    if (last >= first) {
        std::vector<double> lt;
        for (int i = first; i <= last; ++i)
            lt.push_back(odd ? (i - 0.5) * lh - std::lgamma(i + 0.5) : i * lh - std::lgamma(i + 1.0));
        const double top = *std::max_element(lt.begin(), lt.end());
        double s = 0.0;
        for (double v : lt) s += std::exp(v - top);
        series = std::exp(-h + top + std::log(s));
    }
    return odd ? std::erfc(std::sqrt(h)) + series : series;
}

// Maximum statistic over n candidates, each 2 N I ~ chi^2(1) and independent
// under the null: P(max > observed) = 1 - (1 - sf)^n.
double p_max_analytic(double i_max, int n, int64_t N) {
    const double sf = chi2_sf(2.0 * (double)N * i_max, 1);
    if (sf >= 1.0) return 1.0;
    return -std::expm1((double)n * std::log1p(-sf));
}

// Minimum statistic: P(min > observed) = sf^n.
double p_min_analytic(double i_min, int n, int64_t N) {
    return std::pow(chi2_sf(2.0 * (double)N * i_min, 1), (double)n);
}

int gauss_covariance(const std::vector<const float *> &cols_dev, int64_t n, hipStream_t s, DevBuf *work,
                     DevBuf *cov) {
    const int D = (int)cols_dev.size();
    if (D < 1 || D > kGaussMaxD) return fail(MTE_EINVAL, "covariance of %d columns (1..%d)", D, kGaussMaxD);
    if (n < 2 || n > 0x7fffffffLL) return fail(MTE_EINVAL, "N=%lld out of range", (long long)n);
    const GaussChunks ch = gauss_chunks(n);
    const size_t ptr_bytes = (sizeof(void *) * (size_t)D + 255) / 256 * 256;
    const size_t mean_bytes = sizeof(double) * (size_t)(ch.count + 1) * D;
    const size_t part_bytes = sizeof(double) * (size_t)ch.count * D * D;
    int rc;
    if ((rc = work->ensure(ptr_bytes + mean_bytes + part_bytes))) return rc;
    if ((rc = cov->ensure(sizeof(double) * (size_t)D * D))) return rc;
    char *w = work->as<char>();
    MTE_HIP(hipMemcpyAsync(w, cols_dev.data(), sizeof(void *) * (size_t)D, hipMemcpyHostToDevice, s));
    GaussCov a;
    a.cols = reinterpret_cast<const float *const *>(w);
    a.D = D;
    a.n = (int)n;
    a.chunk_rows = ch.rows;
    a.n_chunks = ch.count;
    a.tile = 64;
    a.n_tiles = (D + a.tile - 1) / a.tile;
    a.part_mean = reinterpret_cast<double *>(w + ptr_bytes);
    a.mean = a.part_mean + (size_t)ch.count * D;
    a.part = reinterpret_cast<double *>(w + ptr_bytes + mean_bytes);
    a.cov = cov->as<double>();
    if (launch_gauss_colsum(a, s)) return hip_fail(hipGetLastError(), "column-sum launch");
    int rc2;
    if ((rc2 = timed_launch(kStageGaussGram, s, [&] { return launch_gauss_gram(a, s); }))) return rc2;
    if (launch_gauss_cov_reduce(a, s)) return hip_fail(hipGetLastError(), "covariance reduce launch");
    MTE_HIP(hipStreamSynchronize(s));
    return MTE_OK;
}

int gauss_estimates(const double *cov_dev, int D, const std::vector<GaussJob> &jobs,
                    const std::vector<int32_t> &idx, hipStream_t s, DevBuf *work, std::vector<double> *out) {
    const int n = (int)jobs.size();
    out->assign((size_t)n, 0.0);
    if (n == 0) return MTE_OK;
    for (const GaussJob &j : jobs) {
        if (j.dx < 1 || j.dy < 1 || j.dz < 0 || j.dx + j.dy + j.dz > kGaussMaxVars)
            return fail(MTE_EINVAL, "estimate of (%d, %d, %d) variables (dx, dy >= 1, total <= %d)", j.dx, j.dy,
                        j.dz, kGaussMaxVars);
        if (j.off < 0 || (size_t)j.off + j.dx + j.dy + j.dz > idx.size()) return fail(MTE_EINVAL, "bad index list");
    }
    for (int32_t v : idx)
        if (v < 0 || v >= D) return fail(MTE_EINVAL, "variable index %d outside the %d covariance columns", v, D);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t jb = al(sizeof(GaussJob) * (size_t)n), ib = al(sizeof(int32_t) * idx.size());
    const size_t ob = al(sizeof(double) * (size_t)n), sb = al(sizeof(int32_t) * (size_t)n);
    int rc;
    if ((rc = work->ensure(jb + ib + ob + sb))) return rc;
    char *w = work->as<char>();
    MTE_HIP(hipMemcpyAsync(w, jobs.data(), sizeof(GaussJob) * (size_t)n, hipMemcpyHostToDevice, s));
    MTE_HIP(hipMemcpyAsync(w + jb, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice, s));
    GaussJobs a;
    a.cov = cov_dev;
    a.D = D;
    a.jobs = reinterpret_cast<const GaussJob *>(w);
    a.idx = reinterpret_cast<const int32_t *>(w + jb);
    a.out = reinterpret_cast<double *>(w + jb + ib);
    a.status = reinterpret_cast<int32_t *>(w + jb + ib + ob);
    a.n_jobs = n;
    if ((rc = timed_launch(kStageGaussCmi, s, [&] { return launch_gauss_cmi(a, s); }))) return rc;
    std::vector<int32_t> st((size_t)n);
    MTE_HIP(hipMemcpyAsync(out->data(), a.out, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s));
    MTE_HIP(hipMemcpyAsync(st.data(), a.status, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    MTE_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < n; ++j)
        if (st[(size_t)j])
            return fail(MTE_EINVAL, "estimate %d: covariance submatrix is not positive definite "
                                    "(constant or collinear variables, or N too small)", j);
    return MTE_OK;
}

}  // namespace mte

using namespace mte;

namespace {

thread_local hipStream_t t_gstream = nullptr;

int gauss_stream(void *given, hipStream_t *s) {
    if (given) {
        *s = (hipStream_t)given;
        return MTE_OK;
    }
    if (!t_gstream) MTE_HIP(hipStreamCreateWithFlags(&t_gstream, hipStreamNonBlocking));
    *s = t_gstream;
    return MTE_OK;
}

}  // namespace

extern "C" {

int mte_chi2_sf(double x, int dof, double *out) {
    if (!out) return fail(MTE_EINVAL, "null output");
    if (dof < 1) return fail(MTE_EINVAL, "dof=%d must be >= 1", dof);
    if (std::isnan(x)) return fail(MTE_EINVAL, "x is NaN");
    *out = chi2_sf(x, dof);
    return MTE_OK;
}

int cmi_gauss(const float *X, int dx, const float *Y, int dy, const float *Z, int dz, int64_t N, double *cmi_out,
              double *p_out) {
    if (!X || !Y || (dz > 0 && !Z) || !cmi_out) return fail(MTE_EINVAL, "null pointer argument");
    if (dz == 0 && Z) return fail(MTE_EINVAL, "Z must be NULL when dz == 0");
    if (dx < 1 || dy < 1 || dz < 0 || dx + dy + dz > kGaussMaxVars)
        return fail(MTE_EINVAL, "dx=%d, dy=%d, dz=%d: need dx, dy >= 1 and dx+dy+dz <= %d", dx, dy, dz,
                    kGaussMaxVars);
    if (N < 2 || N > 0x7fffffffLL) return fail(MTE_EINVAL, "N=%lld out of range", (long long)N);
    int rc;
    if ((rc = validate_host_finite(X, (int64_t)dx * N, "X"))) return rc;
    if ((rc = validate_host_finite(Y, (int64_t)dy * N, "Y"))) return rc;
    if (dz && (rc = validate_host_finite(Z, (int64_t)dz * N, "Z"))) return rc;
    if ((rc = ensure_init())) return rc;
    hipStream_t s;
    if ((rc = gauss_stream(nullptr, &s))) return rc;
    const int D = dx + dy + dz;
    DevBuf in, work, cov, wj;
    if ((rc = in.ensure(sizeof(float) * (size_t)D * N))) return rc;
    float *d = in.as<float>();
    MTE_HIP(hipMemcpyAsync(d, X, sizeof(float) * dx * N, hipMemcpyHostToDevice, s));
    MTE_HIP(hipMemcpyAsync(d + (size_t)dx * N, Y, sizeof(float) * dy * N, hipMemcpyHostToDevice, s));
    if (dz) MTE_HIP(hipMemcpyAsync(d + (size_t)(dx + dy) * N, Z, sizeof(float) * dz * N, hipMemcpyHostToDevice, s));
    std::vector<const float *> cols((size_t)D);
    for (int c = 0; c < D; ++c) cols[(size_t)c] = d + (size_t)c * N;
    if ((rc = gauss_covariance(cols, N, s, &work, &cov))) return rc;
    // column order X, Y, Z; the estimate wants Z, X, Y
    std::vector<int32_t> idx;
    for (int c = 0; c < dz; ++c) idx.push_back(dx + dy + c);
    for (int c = 0; c < dx; ++c) idx.push_back(c);
    for (int c = 0; c < dy; ++c) idx.push_back(dx + c);
    std::vector<GaussJob> jobs{GaussJob{dx, dy, dz, 0}};
    std::vector<double> out;
    if ((rc = gauss_estimates(cov.as<double>(), D, jobs, idx, s, &wj, &out))) return rc;
    *cmi_out = out[0];
    if (p_out) *p_out = chi2_sf(2.0 * (double)N * out[0], dx * dy);
    return MTE_OK;
}

int mte_gauss_covariance_dev(const float *dV, int D, int64_t N, int64_t ld, double *d_cov, void *stream) {
    if (!dV || !d_cov) return fail(MTE_EINVAL, "null pointer argument");
    if (D < 1 || D > kGaussMaxD) return fail(MTE_EINVAL, "D=%d out of range 1..%d", D, kGaussMaxD);
    if (N < 2 || N > 0x7fffffffLL || ld < N) return fail(MTE_EINVAL, "N=%lld or ld=%lld out of range",
                                                       (long long)N, (long long)ld);
    int rc;
    if ((rc = ensure_init())) return rc;
    hipStream_t s;
    if ((rc = gauss_stream(stream, &s))) return rc;
    std::vector<const float *> cols((size_t)D);
    for (int c = 0; c < D; ++c) cols[(size_t)c] = dV + (size_t)c * ld;
    DevBuf work, cov;
    if ((rc = gauss_covariance(cols, N, s, &work, &cov))) return rc;
    MTE_HIP(hipMemcpyAsync(d_cov, cov.p, sizeof(double) * (size_t)D * D, hipMemcpyDeviceToDevice, s));
    MTE_HIP(hipStreamSynchronize(s));
    return MTE_OK;
}

int mte_gauss_cmi_sets(const double *d_cov, int D, int n_sets, const int32_t *dims, const int32_t *idx,
                       double *cmi_out, void *stream) {
    if (!d_cov || !dims || !idx || !cmi_out || n_sets < 0) return fail(MTE_EINVAL, "null pointer argument");
    if (D < 1 || D > kGaussMaxD) return fail(MTE_EINVAL, "D=%d out of range 1..%d", D, kGaussMaxD);
    int rc;
    if ((rc = ensure_init())) return rc;
    hipStream_t s;
    if ((rc = gauss_stream(stream, &s))) return rc;
    std::vector<GaussJob> jobs((size_t)n_sets);
    std::vector<int32_t> order;
    size_t at = 0;
    for (int j = 0; j < n_sets; ++j) {
        const int dx = dims[3 * j], dy = dims[3 * j + 1], dz = dims[3 * j + 2];
        if (dx < 1 || dy < 1 || dz < 0 || dx + dy + dz > kGaussMaxVars)
            return fail(MTE_EINVAL, "set %d: dx=%d, dy=%d, dz=%d", j, dx, dy, dz);
        jobs[(size_t)j] = GaussJob{dx, dy, dz, (int32_t)order.size()};
        // caller order X, Y, Z -> kernel order Z, X, Y
        for (int c = 0; c < dz; ++c) order.push_back(idx[at + dx + dy + c]);
        for (int c = 0; c < dx; ++c) order.push_back(idx[at + c]);
        for (int c = 0; c < dy; ++c) order.push_back(idx[at + dx + c]);
        at += (size_t)(dx + dy + dz);
    }
    DevBuf work;
    std::vector<double> out;
    if ((rc = gauss_estimates(d_cov, D, jobs, order, s, &work, &out))) return rc;
    if (n_sets) std::memcpy(cmi_out, out.data(), sizeof(double) * (size_t)n_sets);
    return MTE_OK;
}

}  // extern "C"
