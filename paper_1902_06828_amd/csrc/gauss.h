// Gaussian (linear) estimator of I(X;Y|Z) and its analytic null: device
// launch descriptions and host helpers (VAR section, where the paper uses this
// estimator; Maximum statistic test section, where it notes the analytic null).
//
//   Sigma = (1/N) sum_t (v_t - mean)(v_t - mean)^T      float64, two passes
//   I     = 1/2 [ln det Sigma_{Y|Z} - ln det Sigma_{Y|XZ}]
//         = 1/2 [ln det Sigma_XZ + ln det Sigma_YZ - ln det Sigma_Z - ln det Sigma_XYZ]
//   2 N I ~ chi^2(dx * dy) under independence.
//
// Every estimate of a greedy search is a function of one covariance matrix
// of all the variables it can touch (each candidate's sets are principal
// submatrices), so the N-dependent work is one fp64 Gram product per target
// and every estimate after that is two small Cholesky factorisations.
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace mte {

constexpr int kGaussMaxD = 512;        // columns of one covariance matrix
constexpr int kGaussMaxVars = 64;      // dx + dy + dz of one estimate
constexpr int kGaussRowStage = 32;     // rows staged in LDS per step
constexpr int kGaussMaxChunks = 256;

// Row chunking of the covariance reductions.  It depends on N only, so a
// covariance entry is the same bits whatever the other columns of the matrix.
struct GaussChunks {
    int rows, count;
};
GaussChunks gauss_chunks(int64_t n);

struct GaussCov {
    const float *const *cols;   // device array of D column pointers, N floats each
    int D, n, chunk_rows, n_chunks;
    int tile, n_tiles;          // Gram tile side (64), tiles per side
    double *part_mean;          // [n_chunks][D]
    double *mean;               // [D]
    double *part;               // [n_chunks][D][D]
    double *cov;                // [D][D], symmetric
};

// One estimate: the index lists (into the covariance matrix) of Z, X, Y.
struct GaussJob {
    int32_t dx, dy, dz, off;    // off: first index in GaussJobs::idx (Z, then X, then Y)
};

struct GaussJobs {
    const double *cov;
    int D;
    const GaussJob *jobs;
    const int32_t *idx;
    double *out;                // I per job (nats)
    int32_t *status;            // 0, or 1 if a covariance submatrix is not positive definite
    int n_jobs;
};

int launch_gauss_colsum(const GaussCov &a, hipStream_t s);
int launch_gauss_gram(const GaussCov &a, hipStream_t s);
int launch_gauss_cov_reduce(const GaussCov &a, hipStream_t s);
int launch_gauss_cmi(const GaussJobs &a, hipStream_t s);

// Chi-squared survival function P(chi^2_dof > x) for integer dof >= 1.
double chi2_sf(double x, int dof);
// Analytic tests over n candidates with N rows (dof 1 per candidate).
double p_max_analytic(double i_max, int n, int64_t N);
double p_min_analytic(double i_min, int n, int64_t N);

// Device covariance of D device columns of N rows (blocking on `s`), kept in
// `cov` (D*D doubles); `work` is resized as needed.
struct DevBuf;
int gauss_covariance(const std::vector<const float *> &cols_dev, int64_t n, hipStream_t s,
                     DevBuf *work, DevBuf *cov);
// I for each job against a device covariance (blocking on `s`).
int gauss_estimates(const double *cov_dev, int D, const std::vector<GaussJob> &jobs,
                    const std::vector<int32_t> &idx, hipStream_t s, DevBuf *work,
                    std::vector<double> *out);

}  // namespace mte
