/*
 * mte.h -- C ABI of libmte.so, the MI355X (gfx950) library for the hot path of
 * greedy multivariate transfer-entropy network inference: the KSG nearest-
 * neighbour estimator of conditional mutual information (CMI), its permutation
 * surrogates, the maximum/minimum-statistic and omnibus tests, the four-step
 * greedy source selection for one target, and a continuous-batching request
 * loop.
 *
 * Paper: Novelli, Wollstadt, Mediano, Wibral, Lizier, "Large-scale directed
 * network inference with multivariate transfer entropy and hierarchical
 * statistical testing" (arXiv:1902.06828).
 *
 * Conventions for every call
 *   - Return value: MTE_OK (0) or a negative mte_status.  Outputs are written
 *     only when MTE_OK is returned.  mte_last_error() gives a message for the
 *     last failing call on the calling thread.
 *   - Sample matrices are column-major ("structure of arrays"): column c of a
 *     d-column matrix with N rows is V[c*ld + i], i < N (ld = N for the host
 *     calls).  Values are IEEE binary32 and must be finite (MTE_EINVAL
 *     otherwise, checked for host inputs).
 *   - N is the number of embedded samples (rows) of one estimate; the paper's
 *     N (number of processes) is called P here and its T (series length) T.
 *   - Host pointers are owned by the caller and not retained after return.
 *     Device pointers (the *_dev calls) must stay valid until the work queued
 *     on `stream` has finished.  `stream` is a hipStream_t (NULL = the null
 *     stream).
 *   - The library runs on one GPU, chosen by mte_init (device 0 if the first
 *     call is made without mte_init).  Calls are thread-safe.
 */
#ifndef MTE_H
#define MTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MTE_OK = 0,
    MTE_EINVAL = -1,   /* an argument is out of range or inconsistent */
    MTE_ENOMEM = -2,   /* device memory (or the HBM budget) is exhausted */
    MTE_EDEVICE = -3,  /* no usable GPU, a HIP call failed, or a kernel reported an error */
    MTE_ETIMEOUT = -4, /* mte_wait ran out of time; the request is still pending */
    MTE_EBUSY = -5,    /* the object is in use (e.g. a series with pending requests) */
    MTE_ECANCELED = -6 /* the request's series was cancelled (mte_serve_cancel) */
} mte_status;

/* Message for the last failing call on this thread (never NULL). */
const char *mte_last_error(void);

/* ABI version; changes whenever a declaration in this header changes. */
int mte_abi_version(void);

/*
 * Select the GPU and the HBM budget that the request loop may use for
 * per-request scratch memory (0 = 90% of the free memory at init).
 * Idempotent for the same device; MTE_EINVAL for another device while
 * initialised.  Without a GPU: MTE_EDEVICE.
 */
int mte_init(int device, size_t hbm_budget_bytes);

/* Drain the request loop, free every device allocation, release the GPU. */
int mte_shutdown(void);

/* --------------------------------------------------------------------------
 * KSG estimator of I(X;Y|Z), in nats (estimator named by citation in the CLM
 * section: Kraskov's I^(1) with k neighbours and its CMI extension).
 *   eps_i  = k-th smallest max-norm distance from row i to the other rows in
 *            the joint (X,Y,Z) space, distances |fl32(a_i - a_j)|;
 *   counts = strict (< eps_i) neighbour counts in the (X,Z), (Y,Z) and Z
 *            subspaces (N-1 for Z when dz = 0);
 *   with a Theiler window w (the *_ex calls, mte_opts, mte_request), the rows
 *   j with |i - j| <= w are left out of row i's neighbours and counts (the
 *   dynamic correlation exclusion of the section on autocorrelation in real
 *   data); w = 0 leaves out row i only, and without Z n_z is the number of
 *   rows outside the window.  Needs N >= k + 1 + 2w;
 *   I      = psi(k) - mean_i[psi(n_xz+1) + psi(n_yz+1) - psi(n_z+1)].
 * The value may be negative (Statistical tests section).  eps and counts are
 * exact; the mean is a float64 sum in a fixed order that does not depend on
 * batching, so the plain, batched and served forms return identical bits.
 * Limits: 1 <= dx <= 16; 1 <= dy <= 8; 0 <= dz <= 31; 1 <= k <= 16;
 * k+1 <= N <= 2^31-1; Z must be NULL iff dz == 0.
 * ------------------------------------------------------------------------ */

/* One estimate from host buffers (blocking). */
int cmi_ksg(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
            int64_t N, int k, double *cmi_out);

/*
 * One estimate plus S permutation surrogates, all computed in one batched
 * launch (blocking).  Surrogate s (0-based) keeps Y and Z and replaces the
 * rows of X jointly: row i takes row pi_{seed,0,s}(i) (see mte_permutation).
 * surr_out has S entries.  S >= 1.
 */
int cmi_ksg_surrogates(const float *X, int dx, const float *Y, int dy, const float *Z,
                       int dz, int64_t N, int k, int S, uint64_t seed, double *cmi_out,
                       double *surr_out);

/*
 * Diagnostic form of cmi_ksg_surrogates for parity checks: same kernel, plus
 * the per-row radius and counts of every estimate (estimate 0 = unpermuted,
 * estimate 1+s = surrogate s, keyed with candidate index `cand`).  Host
 * arrays: cmi_out [1+S]; eps_out, nxz_out, nyz_out, nz_out [1+S][N].  S >= 0.
 */
int cmi_ksg_diag(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
                 int64_t N, int k, int S, uint64_t seed, uint32_t cand, double *cmi_out,
                 float *eps_out, int32_t *nxz_out, int32_t *nyz_out, int32_t *nz_out);
/* cmi_ksg_diag with a Theiler window w = theiler >= 0 (cmi_ksg_diag is w = 0). */
int cmi_ksg_diag_ex(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
                    int64_t N, int k, int theiler, int S, uint64_t seed, uint32_t cand,
                    double *cmi_out, float *eps_out, int32_t *nxz_out, int32_t *nyz_out,
                    int32_t *nz_out);

/*
 * Device-resident forms (asynchronous on `stream`, no host synchronisation).
 * dX, dY, dZ are device matrices with leading dimension ld >= N; d_out is a
 * device array of 1+S doubles (estimate first, then the surrogates; S may be
 * 0 in cmi_ksg_surrogates_dev, and cmi_ksg_dev is the S = 0 case).
 * Repeated calls with the same shapes and pointers replay a captured HIP
 * graph.  Scratch memory is owned by the library and reused.
 */
int cmi_ksg_dev(const float *dX, int dx, const float *dY, int dy, const float *dZ, int dz,
                int64_t N, int64_t ld, int k, double *d_out, void *stream);
int cmi_ksg_surrogates_dev(const float *dX, int dx, const float *dY, int dy, const float *dZ,
                           int dz, int64_t N, int64_t ld, int k, int S, uint64_t seed,
                           uint32_t cand, double *d_out, void *stream);
/* cmi_ksg_surrogates_dev with a Theiler window w = theiler >= 0. */
int cmi_ksg_surrogates_dev_ex(const float *dX, int dx, const float *dY, int dy, const float *dZ,
                              int dz, int64_t N, int64_t ld, int k, int theiler, int S,
                              uint64_t seed, uint32_t cand, double *d_out, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimate and S surrogates of cmi_ksg_surrogates_dev, same arguments and
 * results (bit for bit), with every scratch word in one static device array
 * of MTE_NOALLOC_SCRATCH_BYTES that each GPU holds from the library's load
 * until the process ends.  The call allocates nothing: no hipMalloc, no
 * host staging, no library allocator; it enqueues a setup kernel and the
 * all-pairs kernels on `stream` and returns.
 *   - mte_init must have been called (it builds the harmonic table and binds
 *     the array's device address); otherwise MTE_EINVAL.
 *   - N <= 2^20 (the harmonic table of mte_init).
 *   - The scratch needed, about 4*dx*N*(1+S) bytes of permuted X plus
 *     8*(1+S)*ceil(N/64) of chunk sums and small tables, must fit
 *     MTE_NOALLOC_SCRATCH_BYTES; otherwise MTE_EINVAL with the size in the
 *     message.  (N = 10^4, 1+S = 201, dx = 1 takes 8.3 MB.)
 *   - All calls on one GPU share the array and keep the last call's
 *     contents; calls that overlap in time on one GPU (different streams,
 *     or threads) race and give wrong results.  Serialise them.
 */
#define MTE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cmi_ksg_surrogates_dev_noalloc(const float *dX, int dx, const float *dY, int dy,
                                   const float *dZ, int dz, int64_t N, int64_t ld, int k, int S,
                                   uint64_t seed, uint32_t cand, double *d_out, void *stream);

/*
 * Autocorrelation decay time of a series x[T] (host), the heuristic the
 * paper uses to size the Theiler window (section on autocorrelation in real
 * data): the shortest lag L >= 1 at which the autocorrelation function has
 * dropped below 1/e of its zero-lag value, r(L) < r(0)/e, with
 * r(L) = (1/T) sum_{t<T-L} (x_t - mean)(x_{t+L} - mean) summed in float64 in
 * time order; max_lag if no lag up to max_lag qualifies.  T >= 2,
 * max_lag >= 1, x finite (MTE_EINVAL otherwise).
 */
int mte_autocorr_decay_time(const float *x, int64_t T, int max_lag, int *act_out);

/* --------------------------------------------------------------------------
 * Gaussian (linear) estimator of I(X;Y|Z), in nats: the estimator the paper
 * uses for its VAR processes (VAR section) and compares with KSG on coupled
 * logistic maps (Estimators section); its null distribution is analytic
 * (Maximum statistic test section).
 *   Sigma  = (1/N) sum_t (v_t - mean)(v_t - mean)^T, float64, two passes
 *            (means first); every entry is the same bits in any matrix that
 *            holds both of its columns;
 *   I      = 1/2 [ln det Sigma_XZ + ln det Sigma_YZ - ln det Sigma_Z
 *                 - ln det Sigma_XYZ]
 *          = 1/2 [ln det Sigma_{Y|Z} - ln det Sigma_{Y|XZ}] (Schur complements,
 *            from Cholesky factorisations of the (Z,Y) and (Z,X,Y) blocks);
 *   null   2 N I ~ chi^2 with dx*dy degrees of freedom.
 * Limits: dx, dy >= 1, dz >= 0, dx+dy+dz <= 64; 2 <= N <= 2^31-1.
 * MTE_EINVAL if a covariance block is not positive definite (a constant or
 * collinear variable, or N too small for the dimension).
 * ------------------------------------------------------------------------ */

/* One estimate from host column-major buffers X[dx][N], Y[dy][N], Z[dz][N]
 * (Z NULL iff dz == 0), blocking.  p_out (may be NULL) receives the analytic
 * p-value sf_{dx*dy}(2 N I). */
int cmi_gauss(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
              int64_t N, double *cmi_out, double *p_out);

/* Covariance matrix of D device columns dV + c*ld (c < D, N rows each) into
 * the device array d_cov[D][D] (row-major, symmetric).  1 <= D <= 512,
 * ld >= N.  Runs on `stream` and returns when it has finished (the partial
 * sums use library-owned scratch of about min(256, N/256) * D * D doubles). */
int mte_gauss_covariance_dev(const float *dV, int D, int64_t N, int64_t ld, double *d_cov,
                             void *stream);

/* I for n_sets index sets against a device covariance d_cov[D][D] (from
 * mte_gauss_covariance_dev): dims[3*j..] = (dx, dy, dz) of set j and idx
 * holds, set after set, its X, Y and Z column indices (0 <= index < D).
 * Host arrays; cmi_out[n_sets] on the host; returns when finished. */
int mte_gauss_cmi_sets(const double *d_cov, int D, int n_sets, const int32_t *dims,
                       const int32_t *idx, double *cmi_out, void *stream);

/* Chi-squared survival function P(chi^2_dof > x) for integer dof >= 1 (the
 * finite incomplete-gamma series for integer and half-integer order). */
int mte_chi2_sf(double x, int dof, double *out);

/*
 * The surrogate permutation pi_{seed,cand,s} of {0..N-1} (host computation of
 * the same definition the kernels use): a swap-or-not shuffle (Hoang, Morris,
 * Rogaway 2012) with max(24, 6*ceil(log2 N)) rounds keyed by SplitMix64.
 * out has N entries.  1 <= N <= 2^31-1.
 */
int mte_permutation(uint64_t seed, uint32_t cand, uint32_t s, int64_t N, uint32_t *out);

/* --------------------------------------------------------------------------
 * Replications (trials).  With R replications of the same experiment the
 * rows of an estimate are the embedded rows of every replication, one
 * replication after the other: row i = r*n_r + t, N = R*n_r.  The Maximum
 * statistic test section prefers surrogates that shuffle the order of the
 * candidate's replications (the other variables keep theirs) and falls back to
 * shuffling the embedded samples within each trial when the replications allow
 * too few permutations:
 *   MTE_SHUFFLE_REPLICATIONS  row (r, t) of surrogate s takes row
 *                             (sigma(r), t), sigma = pi_{seed,cand,s} over R;
 *   MTE_SHUFFLE_WITHIN        row (r, t) takes (r, pi_r(t)), pi_r the
 *                             swap-or-not permutation of {0..n_r-1} keyed by
 *                             h_r = mix64(h ^ ((r+1)*0x9E3779B97F4A7C15)) with
 *                             h the key hash of (seed, cand, s) (R = 1: keyed
 *                             by h itself, i.e. pi_{seed,cand,s} over N);
 *   MTE_SHUFFLE_AUTO          REPLICATIONS when R! >= S, else WITHIN.
 * The Theiler window is defined for one replication only (theiler must be 0
 * when R > 1).
 * ------------------------------------------------------------------------ */
#define MTE_SHUFFLE_AUTO (-1)
#define MTE_SHUFFLE_WITHIN 0
#define MTE_SHUFFLE_REPLICATIONS 1

/* The mode MTE_SHUFFLE_AUTO picks for R replications and S surrogates. */
int mte_shuffle_mode(int R, int S, int *mode_out);

/* Per-node z-score applied by the greedy search and network inference when
 * mte_opts.standardise is set (the paper is silent on normalisation; KSG's
 * max-norm is not scale invariant, so every node is put on one scale): for
 * each node, over all its R*T samples in order (replications, then time),
 * mean and variance (1/(R*T)) as float64 sums in that order, and each value
 * (x - mean)/sd computed in float64 and rounded to float32; a constant node
 * becomes all zeros.  in, out: host [R][P][T] (may be the same array). */
int mte_standardise(const float *in, int R, int P, int64_t T, float *out);

/* Source rows of surrogate s (host computation of the kernels' definition):
 * out[i] = the candidate row that row i takes.  N a multiple of R; mode
 * WITHIN or REPLICATIONS (REPLICATIONS needs R >= 2). */
int mte_permutation_rep(uint64_t seed, uint32_t cand, uint32_t s, int64_t N, int R, int mode,
                        uint32_t *out);

/* cmi_ksg_surrogates over R replications (X, Y, Z [d][N] host buffers with
 * the rows of replication r at r*N/R..), surrogate keys pi_{seed,cand,s}
 * and the given shuffle mode (MTE_SHUFFLE_AUTO allowed). */
int cmi_ksg_surrogates_rep(const float *X, int dx, const float *Y, int dy, const float *Z,
                           int dz, int64_t N, int R, int k, int S, uint64_t seed, uint32_t cand,
                           int mode, double *cmi_out, double *surr_out);

/* --------------------------------------------------------------------------
 * Significance tests over CMI estimates (Statistical tests section, Table 1).
 * real[n] are the candidates' estimates, surr[n][S] their surrogates
 * (row-major).  S*alpha must exceed 1 (Maximum statistic test, item a).
 *   max: I* = max_j real[j] (first on ties); p = #{s: max_j surr[j][s] > I*}/S
 *   min: I  = min_j real[j] (first on ties); p = #{s: min_j surr[j][s] > I}/S
 *   omnibus: p = #{s: surr[s] > real}/S
 * significant = (p < alpha).
 * ------------------------------------------------------------------------ */
int mte_max_statistic(const double *real, const double *surr, int n, int S, double alpha,
                      int *index_out, double *p_out, int *significant_out);
int mte_min_statistic(const double *real, const double *surr, int n, int S, double alpha,
                      int *index_out, double *p_out, int *significant_out);
int mte_omnibus(double real, const double *surr, int S, double alpha, double *p_out,
                int *significant_out);

/* --------------------------------------------------------------------------
 * Greedy source selection for one target (Inference algorithm section,
 * steps 1-4).  data: host float32 [P][T] row-major (one series per process),
 * or [R][P][T] with mte_opts.replications = R > 1 (rows of replication r
 * follow those of r-1; see Replications above).
 * Embedding rows t = L..T-1 with L = max(max_lag_target, max_lag_sources);
 * variable (node, lag) is data[node][t-lag].  Candidates: target lags
 * 1..max_lag_target, then each candidate source (given order) with lags
 * 1..max_lag_sources.  Every candidate test of a greedy iteration (all
 * candidates and their S surrogates) runs as one batched launch; the tests
 * run on the host.  Surrogate keys: a running candidate-test counter t
 * (starting at 0, one per candidate per iteration in candidate order, then
 * one for the omnibus test) gives pi_{seed,t,s}.
 * ------------------------------------------------------------------------ */
typedef struct {
    int k;              /* neighbours (default 4) */
    int S;              /* surrogates per candidate test (default 200) */
    int max_lag_target; /* target-past candidate lags 1..max_lag_target (default 5) */
    uint64_t seed;      /* surrogate key seed (default 0) */
    int theiler;        /* Theiler window of every estimate (default 0; KSG only) */
    int estimator;      /* MTE_ESTIMATOR_KSG (default) or MTE_ESTIMATOR_GAUSS */
    int replications;   /* R >= 1 (default 1): data holds R replications [R][P][T], T per
                           replication; the rows of all replications are pooled
                           (N = R*(T-L)) and the surrogates follow MTE_SHUFFLE_AUTO;
                           needs theiler = 0 when R > 1 (not for the _sid form) */
    int standardise;    /* 1 (default): z-score each node series once before embedding
                           (mte_standardise); 0: use the data as given */
} mte_opts;

/* Estimators of the greedy search.  KSG: every test is a surrogate test
 * with S permutation surrogates (k, S, seed, theiler apply).  GAUSS: the
 * Gaussian estimator (cmi_gauss) with its analytic null, no surrogates (k, S
 * and seed are ignored; theiler must be 0): with n candidates in a round and
 * N rows, the maximum-statistic p is 1 - (1 - sf_1(2 N I_max))^n, the
 * minimum-statistic p is sf_1(2 N I_min)^n, and the omnibus p is
 * sf_{|X^S|}(2 N T) (sf_d: chi^2 survival function with d degrees of freedom),
 * the candidates' statistics being treated as independent, as in the
 * family-wise error correction of the Maximum statistic test section.
 * n_estimates counts one estimate per candidate test. */
#define MTE_ESTIMATOR_KSG 0
#define MTE_ESTIMATOR_GAUSS 1

typedef struct {
    int32_t node, lag;  /* process index and lag in samples */
    double cmi;         /* estimate of the test that selected it */
    double p;           /* p-value of that test */
} mte_var;

typedef struct {
    /* caller-allocated arrays and their capacities */
    mte_var *target_past;  /* capacity >= max_lag_target */
    mte_var *sources;      /* capacity >= n_candidates * max_lag_sources */
    /* results */
    int n_target_past;
    int n_sources;         /* accepted sources (0 unless the omnibus test passed) */
    int n_sources_tested;  /* selected sources before the omnibus test */
    double omnibus_te;     /* collective TE I(X^S; Y_t | Y^S); 0 if X^S is empty */
    double omnibus_p;      /* 1 if X^S is empty */
    int significant;       /* omnibus test passed */
    int64_t n_estimates;   /* CMI estimates computed (real and surrogate) */
    double gpu_seconds;    /* wall time spent waiting for the GPU */
} mte_result;

/* opts may be NULL (defaults).  alpha is used for all three tests.
 * MTE_EINVAL if S*alpha <= 1, the target is among the candidates, a node is
 * out of range, T <= L + k, or a capacity is missing. */
int mte_select_sources(const float *data, int P, int64_t T, int target,
                       const int32_t *candidates, int n_candidates, int max_lag_sources,
                       double alpha, const mte_opts *opts, mte_result *out);

/* The same greedy selection over a series registered with
 * mte_series_register; every candidate test goes through the request loop
 * below as one request, so concurrent calls (one per target) are batched
 * together on the GPU.  Same arguments and results as mte_select_sources. */
int mte_select_sources_sid(int32_t sid, int target, const int32_t *candidates, int n_candidates,
                           int max_lag_sources, double alpha, const mte_opts *opts,
                           mte_result *out);

/* --------------------------------------------------------------------------
 * Network level (Combining across multiple targets; Validation sections).
 * ------------------------------------------------------------------------ */

/* Benjamini-Hochberg step-up at level q over p[m] (FDR correction of the
 * targets' omnibus p-values): keep_out[i] = 1 for the rejected nulls, i.e.
 * the ranks 1..r of the ascending order (stable for ties) where r is the
 * largest rank with p_(r) <= q*r/m.  0 < q < 1, p in [0,1]. */
int mte_fdr_bh(const double *p, int m, double q, uint8_t *keep_out);

typedef struct {
    int n_target_past;     /* selected target-past variables */
    int n_sources;         /* accepted source variables (0 unless the omnibus test passed) */
    int n_sources_tested;  /* selected source variables before the omnibus test */
    double omnibus_te;     /* collective TE of the selected sources (0 if none) */
    double omnibus_p;      /* omnibus p-value (1 if no source was selected) */
    int significant;       /* omnibus test passed (p < alpha) */
    int fdr_kept;          /* kept by the FDR correction (1 when it is off) */
    int64_t n_estimates;   /* CMI estimates computed for this target */
} mte_target_summary;

/*
 * Network inference over data [P][T] (host, row-major): the greedy source
 * selection (mte_select_sources) of every target t with all other processes
 * as candidate sources, run concurrently through the request loop on
 * n_threads host threads (<= 0: min(P, 16)); target t uses surrogate seed
 * opts->seed + t.  Then, if alpha_fdr > 0, the Benjamini-Hochberg correction
 * at level alpha_fdr over the P omnibus p-values.  adj_out [P][P] (caller
 * array): adj[s][t] = 1 iff some past variable of s is an accepted source of
 * t, t's omnibus test passed and (if on) the correction kept t.  targets_out
 * [P] (caller array).  opts may be NULL (defaults).  Errors as
 * mte_select_sources; the first failing target's error is returned.
 */
int mte_infer_network(const float *data, int P, int64_t T, int max_lag_sources, double alpha,
                      double alpha_fdr, const mte_opts *opts, int n_threads, uint8_t *adj_out,
                      mte_target_summary *targets_out);

/*
 * Link statistics of an inferred adjacency against a known one, over the
 * P*(P-1) ordered pairs of distinct processes (Validation section):
 * counts_out = {TP, FP, TN, FN}; rates_out = {precision TP/(TP+FP), recall
 * TP/(TP+FN), specificity TN/(TN+FP), false positive rate FP/(FP+TN)} (NaN
 * for an empty denominator).
 */
int mte_link_metrics(const uint8_t *inferred, const uint8_t *truth, int P, int64_t *counts_out,
                     double *rates_out);

/* --------------------------------------------------------------------------
 * Request loop (continuous batching).  Series registered once stay resident
 * in HBM; each request is one candidate test (1 + S estimates of
 * I(X;Y|Z) over lag-shifted windows of a resident series); requests are
 * admitted while the in-flight limit and the HBM budget allow, batched with
 * whatever else is pending, and run concurrently with earlier batches.
 * At most three batches are in flight, each on its own stream; the
 * environment variable MTE_SERVE_SLOTS=1|2|3, read when the loop starts,
 * lowers that limit (1 runs the batches one after another, for attributing
 * time to kernels); results do not depend on it.  A batch of several
 * requests is halved while it needs more than 16 GiB of device memory
 * (MTE_BATCH_BYTES_MAX, in bytes, read once, overrides); a single request
 * above that still runs alone if it fits the HBM budget.
 * ------------------------------------------------------------------------ */

/* Upload data [P][T] (host, row-major) and keep it resident.  *sid_out >= 0. */
int mte_series_register(const float *data, int P, int64_t T, int32_t *sid_out);

/* Free a series; MTE_EBUSY while requests on it are pending. */
int mte_series_release(int32_t sid);

typedef struct {
    int32_t sid;              /* registered series */
    int dx, dy, dz;           /* column counts (same limits as cmi_ksg) */
    const int32_t *nodes;     /* dx+dy+dz process indices: X columns, Y, then Z */
    const int32_t *lags;      /* matching lags (>= 0) */
    int64_t t0;               /* first embedded time index; rows t0..t0+N-1 */
    int64_t N;                /* rows; needs t0-lag >= 0 and t0+N-1-lag < T */
    int k;                    /* neighbours */
    int S;                    /* surrogates (>= 0) */
    uint64_t seed;            /* surrogate keys pi_{seed,cand,s} */
    uint32_t cand;
    int theiler;              /* Theiler window (>= 0) */
} mte_request;

/* Queue a request without blocking; copies nodes and lags.  A request whose
 * launch alone would exceed the HBM budget finishes with MTE_ENOMEM (reported
 * by mte_wait); one that needs memory held by batches in flight waits at the
 * queue front until they retire.  MTE_ECANCELED on a cancelled series. */
int mte_submit(const mte_request *req, uint64_t *ticket_out);

/* Cancel a series (the paper's run-time section runs one search per target
 * concurrently; this stops all of them on one series): its queued requests
 * finish with MTE_ECANCELED, new requests on it and on its z-scored copy are
 * refused with MTE_ECANCELED, and batches already on the GPU complete.  A
 * greedy search on it returns MTE_ECANCELED.  mte_series_release frees it. */
int mte_serve_cancel(int32_t sid);

/* Wait for a request: cmi_out gets the estimate, surr_out (may be NULL) the S
 * surrogates.  timeout_s < 0 waits forever.  MTE_ETIMEOUT leaves the ticket
 * valid; any other return retires it. */
int mte_wait(uint64_t ticket, double *cmi_out, double *surr_out, double timeout_s);

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t batches;          /* launches made by the loop */
    int64_t estimates;        /* CMI estimates completed */
    double p50_latency_s, p99_latency_s, mean_batch_requests;
    int64_t peak_bytes_in_use;
    int64_t budget_bytes;
    int64_t waited;           /* requests admitted after waiting at the queue front for memory */
    /* Phases of a completed request's latency (seconds): queued = submit to
     * the start of the admission that launched it (waits for a free slot or
     * for memory included), host = that admission (sizing, preparing and
     * enqueueing its batch), device = launch to the retirement that found the
     * batch done (its kernels, kernels of other batches sharing the GPU, the
     * result copy and the loop's polling).  p50/p99 of each phase on its own: */
    double queue_p50_s, queue_p99_s, host_p50_s, host_p99_s, device_p50_s, device_p99_s;
    /* The requests whose latency is at or above p99_latency_s: their count,
     * mean phases, mean N and mean requests per batch. */
    double tail_queue_s, tail_host_s, tail_device_s, tail_mean_n, tail_mean_batch_requests;
    int64_t tail_requests;
} mte_serve_stats;

/* Statistics since the last reset (reset = 1 clears them after reading). */
int mte_serve_get_stats(mte_serve_stats *out, int reset);

/* --------------------------------------------------------------------------
 * Compiled tile configurations of the KSG kernel.  cfg_out receives up to
 * `capacity` rows of 6 int32: top-k capacity, estimates per lane, queries per
 * lane, Z, Y and X column capacities; *count_out is the total number.  The
 * environment variables MTE_FORCE_VARIANT=<row index> and MTE_FORCE_SPLIT=<m>
 * (0: one reference split; m: m times the default number of splits) force a
 * configuration for testing; results do not depend on either.
 * ------------------------------------------------------------------------ */
int mte_tile_configs(int32_t *cfg_out, int capacity, int *count_out);

/* --------------------------------------------------------------------------
 * Tuned launch choices.  The autotuner times candidate launch choices on a
 * shape's first call and keeps the fastest; none of them changes a result.
 *   all-pairs kernel: tile configuration (a row of mte_tile_configs) and
 *     reference-split multiplier, per batch shape ("P:" keys), tuned by the
 *     device calls (cmi_ksg_surrogates_dev);
 *   list path: rows per block of the compiled-dimension build (2, 4), the
 *     scan's cooperative-finish threshold (2, 4, 8 lanes) and entries per
 *     step (4, 8), the blocks per CU of the permutation beside the build
 *     (2, 3) and, for launches of one job, the estimate-group lane
 *     order, per job shape ("L:" keys:
 *     N, dims, k, estimates, Theiler window, replications, one job or
 *     several), tuned by the device calls on the batch itself and by the host
 *     calls and greedy rounds on one job of the shape when the batch holds at
 *     least 2^20 (row, estimate) pairs; the request loop only looks them up.
 * Choices persist in a text file, MTE_TUNE_FILE or else
 * $XDG_CACHE_HOME/mte/tune.txt or $HOME/.cache/mte/tune.txt ("off": none),
 * keyed by the GPU architecture and the library build; MTE_TUNE=0 turns
 * tuning off.
 * mte_tune_report writes the choices made or read in this process, one per
 * line: "<key> variant=<v> split=<m> build_rows=<q> coop_lanes=<c>
 * grouped=<g> scan_step=<s> perm_cu=<p> ms=<t> from=<tuned|file>" (0 / -1: the default).  It writes at
 * most cap - 1 bytes and a NUL to buf (buf may be NULL when cap is 0) and
 * the full length to *len_out, so a second call with a larger buffer gets
 * everything.
 * ------------------------------------------------------------------------ */
int mte_tune_report(char *buf, size_t cap, size_t *len_out);

/* --------------------------------------------------------------------------
 * Kernel timing: when enabled, launches are made directly (no graph replay)
 * and HIP events are recorded around every kernel launch of the stages
 * below, on the stream the kernel runs on (the list path's permutation runs
 * on a library stream beside the build, so those two stages overlap); the
 * elapsed times are accumulated per stage (reading waits for the recorded
 * events).  In a list-path launch of several jobs, the kernel that orders
 * the rows for the scan follows the permutation on that stream and falls in
 * no stage.  mte_kernel_timing_read reads stage MTE_STAGE_ALL_PAIRS.
 * reset = 1 clears the stage after reading.
 *   MTE_STAGE_ALL_PAIRS  all-pairs KSG kernel (jobs the list path does not
 *                        take: fewer than 8 estimates per (Y,Z) sample, no Z
 *                        with several X columns or N > 16384, or N > 2^21)
 *   MTE_STAGE_BUILD      neighbour-list build, once per (Y,Z) sample
 *   MTE_STAGE_SCAN       per (row, estimate) k-NN radius and counts over the lists
 *   MTE_STAGE_FALLBACK   all-rows redo of the pairs the lists cannot decide
 *   MTE_STAGE_REDUCE     fixed-order digamma sums of the list path
 *   MTE_STAGE_PERMUTE    surrogate permutation of the X columns (both paths)
 *   MTE_STAGE_GAUSS_GRAM float64 centered Gram product of the Gaussian estimator
 *   MTE_STAGE_GAUSS_CMI  Cholesky estimates of the Gaussian estimator
 * ------------------------------------------------------------------------ */
enum {
    MTE_STAGE_ALL_PAIRS = 0,
    MTE_STAGE_BUILD = 1,
    MTE_STAGE_SCAN = 2,
    MTE_STAGE_FALLBACK = 3,
    MTE_STAGE_REDUCE = 4,
    MTE_STAGE_PERMUTE = 5,
    MTE_STAGE_GAUSS_GRAM = 6,
    MTE_STAGE_GAUSS_CMI = 7
};
int mte_kernel_timing(int enable);
int mte_kernel_timing_read(int64_t *launches_out, double *total_ms_out, int reset);
int mte_kernel_timing_stage(int stage, int64_t *launches_out, double *total_ms_out, int reset);

/* --------------------------------------------------------------------------
 * Neighbour-list path statistics over the launches whose completion the
 * library has checked (the host-pointer calls, the greedy driver and the
 * request loop): (row, estimate) pairs computed on the list path, how many of
 * them the lists could not decide and were redone over all rows, and (if
 * entries_out is not NULL) entries_out[0..1] = list entries read by the
 * k-NN scan of the (Y,Z) lists and by the count scan of the Z lists; the
 * entry counts are only taken by launches made while
 * mte_list_stats_enable(1) is in effect (directly launched or captured), as
 * they cost atomics in the scan kernel.  reset = 1 clears them.
 * ------------------------------------------------------------------------ */
int mte_list_stats_enable(int enable);
int mte_list_stats(int64_t *pairs_out, int64_t *undecided_out, int64_t *entries_out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* MTE_H */
