// Auxiliary kernels of the KSG launch (queue/counter reset, surrogate
// permutation of the X columns) and the launch helpers; the main kernel's
// device code is in ksg_device.h and its instantiations in kernels_k*.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include <vector>

#include "engine.h"
#include "ksg_device.h"

namespace mte {

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t dmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Swap-or-not rounds for a domain of n: max(24, 6*ceil(log2 n)).
__device__ __forceinline__ int n_rounds_dev(int64_t n) {
    int bits = 0;
    for (uint64_t v = (uint64_t)(n - 1); v; v >>= 1) ++bits;
    const int r = 6 * bits;
    return r < 24 ? 24 : r;
}

// ------------------------------------------------------------------ permute
// xp[e][c][i] = X_c[src_e(i)] (and, for the list path, also xt[c][i][e]) for
// every job, estimate and row.  Rows are R = J.reps replications of nr = n/R rows
// (R = 1: one block of all rows).  One thread block per (job, estimate,
// replication, 1024-row chunk of the replication); the block derives one
// swap-or-not key schedule in LDS:
//   replication shuffle (rep_shuffle): row (r, t) takes (sigma(r), t), sigma
//     the permutation of {0..R-1} keyed by the estimate's hash h;
//   within-replication shuffle: row (r, t) takes (r, pi_r(t)), pi_r the
//     permutation of {0..nr-1} keyed by h for R = 1 and by
//     mix64(h ^ (r+1) G) for R > 1.
__device__ __forceinline__ uint32_t swap_or_not(uint32_t x, uint32_t n, int rounds, const uint64_t *rk,
                                                const uint32_t *kk) {
    for (int r = 0; r < rounds; ++r) {
        const uint32_t k = kk[r];
        const uint32_t xp = (x <= k) ? (k - x) : (k - x + n);
        const uint32_t hi = x > xp ? x : xp;
        if (dmix64((uint64_t)hi ^ rk[r]) >> 63) x = xp;
    }
    return x;
}

__global__ __launch_bounds__(256) void permute_kernel(const Job *__restrict__ jobs, int n_jobs,
                                                     const int64_t *__restrict__ blk_off, int64_t total) {
    __shared__ uint64_t s_rk[192];
    __shared__ uint32_t s_k[192];
    __shared__ int s_job;
    __shared__ uint32_t s_src_rep;
    // a grid smaller than the work takes the blocks' items in turn
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    if (threadIdx.x == 0) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (blk_off[mid] <= b) lo = mid; else hi = mid - 1;
        }
        s_job = lo;
    }
    __syncthreads();
    const Job &J = jobs[s_job];
    const int64_t local = b - blk_off[s_job];
    const int reps = J.reps;
    const int nr = J.n / reps;
    const int cpr = (nr + 1023) / 1024;
    const int e = (int)(local / ((int64_t)reps * cpr));
    const int rem = (int)(local % ((int64_t)reps * cpr));
    const int rep = rem / cpr;
    const int c0 = (rem % cpr) * 1024;
    const EstKey key = J.keys[e];
    // key schedule: domain dn, hash hh
    const uint32_t dn = J.rep_shuffle ? (uint32_t)reps : (uint32_t)nr;
    const uint64_t hh = (J.rep_shuffle || reps == 1) ? key.h : dmix64(key.h ^ ((uint64_t)(rep + 1) * kGolden));
    const int rounds = n_rounds_dev(dn);
    if (!key.ident) {
        for (int r = threadIdx.x; r < rounds; r += blockDim.x) {
            uint64_t rk = dmix64(hh + (uint64_t)(r + 1) * kGolden);
            s_rk[r] = rk;
            s_k[r] = (uint32_t)(((rk >> 32) * (uint64_t)dn) >> 32);
        }
    }
    __syncthreads();
    if (J.rep_shuffle && threadIdx.x == 0)
        s_src_rep = key.ident ? (uint32_t)rep : swap_or_not((uint32_t)rep, dn, rounds, s_rk, s_k);
    __syncthreads();
    const int64_t base = (int64_t)rep * nr;
    for (int ii = threadIdx.x; ii < 1024; ii += blockDim.x) {
        const int t = c0 + ii;
        if (t >= nr) break;
        const int64_t i = base + t;
        int64_t x;
        if (key.ident)
            x = i;
        else if (J.rep_shuffle)
            x = (int64_t)s_src_rep * nr + t;
        else
            x = base + swap_or_not((uint32_t)t, dn, rounds, s_rk, s_k);
        const int64_t ri = J.xr ? (int64_t)min(max(J.zrank[i], 0), J.n - 1) : 0;
        for (int c = 0; c < J.dx; ++c) {
            const float v = J.cols[c][x];
            if (J.xt) J.xt[((int64_t)c * J.n + i) * J.n_est + e] = v;
            J.xp[((int64_t)e * J.dx + c) * J.n + i] = v;
            if (J.xr) J.xr[((int64_t)e * J.dx + c) * J.n + ri] = v;
        }
    }
    __syncthreads();   // the next item rewrites the key schedule
    }
}

__global__ void reset_kernel(uint32_t *__restrict__ w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0u;
}

}  // namespace

// ------------------------------------------------------------------ variants
// Compiled in kernels_k4.hip, kernels_k8.hip and kernels_k16.hip (one top-k
// capacity each, built in parallel).
const dev::VariantEntry *variants_k4(int *n);
const dev::VariantEntry *variants_k8(int *n);
const dev::VariantEntry *variants_k16(int *n);

namespace {
struct Registry {
    std::vector<dev::VariantEntry> v;
    Registry() {
        int n = 0;
        const dev::VariantEntry *p = variants_k4(&n);
        v.insert(v.end(), p, p + n);
        p = variants_k8(&n);
        v.insert(v.end(), p, p + n);
        p = variants_k16(&n);
        v.insert(v.end(), p, p + n);
    }
};
const Registry &registry() {
    static Registry r;
    return r;
}
}  // namespace

int kernel_variant_count() { return (int)registry().v.size(); }

bool kernel_variant(int i, TileCfg *cfg) {
    if (i < 0 || i >= kernel_variant_count()) return false;
    *cfg = registry().v[i].cfg;
    return true;
}

int variant_blocks_per_cu(int v) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, registry().v[v].fn, kBlock, 0) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

int launch_reset(uint32_t *words, int64_t n_words, void *stream) {
    if (n_words <= 0) return 0;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, words,
                       n_words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_permute(const Job *jobs_dev, int n_jobs, int64_t total_blocks, const int64_t *blk_off,
                   void *stream, int64_t max_grid) {
    if (total_blocks <= 0) return 0;
    const int64_t grid = max_grid > 0 && max_grid < total_blocks ? max_grid : total_blocks;
    hipLaunchKernelGGL(permute_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, jobs_dev,
                       n_jobs, blk_off, total_blocks);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_main(int v, const Job *jobs_dev, int n_jobs, const int64_t *a_off, const int64_t *b_off,
                const LaunchInfo &li, uint32_t *work, const double *harm, void *stream) {
    void *args[] = {(void *)&jobs_dev, (void *)&n_jobs, (void *)&a_off, (void *)&b_off,
                    (void *)&li.items_a, (void *)&li.items_b, (void *)&work, (void *)&harm};
    hipError_t e = hipLaunchKernel(registry().v[v].fn, dim3(li.grid), dim3(kBlock), args, 0,
                                   (hipStream_t)stream);
    return e == hipSuccess ? 0 : -1;
}

}  // namespace mte
