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
// replication, 1024-row chunk of the replication), keyed by the estimate's
// swap-or-not schedule:
//   replication shuffle (rep_shuffle): row (r, t) takes (sigma(r), t), sigma
//     the permutation of {0..R-1} keyed by the estimate's hash h;
//   within-replication shuffle: row (r, t) takes (r, pi_r(t)), pi_r the
//     permutation of {0..nr-1} keyed by h for R = 1 and by
//     mix64(h ^ (r+1) G) for R > 1.
//
// A round r of the schedule for domain n: round key rk = mix64(hh + (r+1) G),
// K = ((rk >> 32) n) >> 32; x pairs with x' = (K - x) mod n and takes x' when
// the top bit of mix64(max(x, x') ^ rk) is set.  The schedule is the same for
// every row of a block, so the round keys are computed in scalar registers once
// per round and applied to four rows per thread.  max(x, x') < 2^32, so the
// high word of max(x, x') ^ rk is rk's, and the first xor-shift and the high
// half of the first product's cross terms are scalar too; of the last
// product only the top bit is needed (the final xor-shift keeps it).
constexpr uint32_t kMixC1Lo = 0x1CE4E5B9u, kMixC1Hi = 0xBF58476Du;
constexpr uint32_t kMixC2Lo = 0x133111EBu, kMixC2Hi = 0x94D049BBu;

struct SonRound {
    uint32_t k, rk_lo, rk_hi, cross;   // cross = (rk_hi ^ rk_hi >> 30) * C1 low word
};

__device__ __forceinline__ SonRound son_round_key(uint64_t hh, int r, uint32_t n) {
    const uint64_t rk = dmix64(hh + (uint64_t)(r + 1) * kGolden);
    SonRound s;
    s.k = (uint32_t)(((rk >> 32) * (uint64_t)n) >> 32);
    s.rk_lo = (uint32_t)rk;
    s.rk_hi = (uint32_t)(rk >> 32);
    s.cross = (s.rk_hi ^ (s.rk_hi >> 30)) * kMixC1Lo;
    return s;
}

__device__ __forceinline__ uint32_t son_step(uint32_t x, uint32_t n, const SonRound &s) {
    const uint32_t xp = (x <= s.k) ? (s.k - x) : (s.k - x + n);
    const uint32_t m = x > xp ? x : xp;
    // z = (rk_hi : m ^ rk_lo);  z ^= z >> 30
    uint32_t lo = m ^ s.rk_lo;
    lo ^= __builtin_amdgcn_alignbit(s.rk_hi, lo, 30);
    // z *= C1 (mod 2^64)
    const uint64_t p = (uint64_t)lo * kMixC1Lo;
    uint32_t nl = (uint32_t)p;
    uint32_t nh = (uint32_t)(p >> 32) + lo * kMixC1Hi + s.cross;
    // z ^= z >> 27
    nl ^= __builtin_amdgcn_alignbit(nh, nl, 27);
    nh ^= nh >> 27;
    // top bit of z * C2
    const uint32_t top = (uint32_t)(((uint64_t)nl * kMixC2Lo) >> 32) + nl * kMixC2Hi + nh * kMixC2Lo;
    return (int32_t)top < 0 ? xp : x;
}

// The whole permutation of one index (wave-uniform arguments: scalar code).
__device__ __forceinline__ uint32_t swap_or_not(uint32_t x, uint32_t n, int rounds, uint64_t hh) {
    for (int r = 0; r < rounds; ++r) x = son_step(x, n, son_round_key(hh, r, n));
    return x;
}

constexpr int kPermRows = 1024;                        // rows per block
constexpr int kPermThreads = 256;
constexpr int kPermPer = kPermRows / kPermThreads;     // rows per thread

__global__ __launch_bounds__(kPermThreads) void permute_kernel(const Job *__restrict__ jobs, int n_jobs,
                                                              const int64_t *__restrict__ blk_off, int64_t total,
                                                              int64_t grid) {
    // a grid smaller than the work takes the blocks' items in turn; the
    // indices come straight from the hardware registers (the group index is
    // a scalar value, so everything derived from it stays wave-uniform)
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    for (int64_t b = (int64_t)__builtin_amdgcn_workgroup_id_x(); b < total; b += grid) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (blk_off[mid] <= b) lo = mid; else hi = mid - 1;
        }
        const int job = __builtin_amdgcn_readfirstlane(lo);
        const Job &J = jobs[job];
        const int64_t local = b - blk_off[job];
        const int reps = J.reps;
        const int nr = J.n / reps;
        const int cpr = (nr + kPermRows - 1) / kPermRows;
        const int e = (int)(local / ((int64_t)reps * cpr));
        const int rem = (int)(local % ((int64_t)reps * cpr));
        const int rep = rem / cpr;
        const int c0 = (rem % cpr) * kPermRows;
        const EstKey key = J.keys[e];
        // key schedule: domain dn, hash hh
        const uint32_t dn = J.rep_shuffle ? (uint32_t)reps : (uint32_t)nr;
        const uint64_t hh = (J.rep_shuffle || reps == 1) ? key.h : dmix64(key.h ^ ((uint64_t)(rep + 1) * kGolden));
        const int rounds = n_rounds_dev(dn);
        // the divisions above leave these uniform values in vector registers;
        // read back into scalar ones, the round keys are computed by the
        // scalar unit
        const uint64_t hs = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(hh >> 32)) << 32) |
                            (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)hh);
        const uint32_t dns = (uint32_t)__builtin_amdgcn_readfirstlane((int)dn);
        const int rs = __builtin_amdgcn_readfirstlane(rounds);
        const int64_t base = (int64_t)rep * nr;
        uint32_t src[kPermPer];
#pragma unroll
        for (int q = 0; q < kPermPer; ++q) src[q] = (uint32_t)min(c0 + tid + q * kPermThreads, nr - 1);
        // source row of row base + t: xbase + src
        int64_t xbase = base;
        if (key.ident) {
        } else if (J.rep_shuffle) {
            xbase = (int64_t)swap_or_not((uint32_t)rep, dns, rs, hs) * nr;
        } else {
            for (int r = 0; r < rs; ++r) {
                const SonRound s = son_round_key(hs, r, dns);
#pragma unroll
                for (int q = 0; q < kPermPer; ++q) src[q] = son_step(src[q], dns, s);
            }
        }
#pragma unroll
        for (int q = 0; q < kPermPer; ++q) {
            const int t = c0 + tid + q * kPermThreads;
            if (t >= nr) break;
            const int64_t i = base + t;
            const int64_t x = xbase + (int64_t)src[q];
            const int64_t ri = J.xr ? (int64_t)min(max(J.zrank[i], 0), J.n - 1) : 0;
            for (int c = 0; c < J.dx; ++c) {
                const float v = J.cols[c][x];
                if (J.xt) J.xt[((int64_t)c * J.n + i) * J.n_est + e] = v;
                J.xp[((int64_t)e * J.dx + c) * J.n + i] = v;
                if (J.xr) J.xr[((int64_t)e * J.dx + c) * J.n + ri] = v;
            }
        }
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
    hipLaunchKernelGGL(permute_kernel, dim3((unsigned)grid), dim3(kPermThreads), 0, (hipStream_t)stream, jobs_dev,
                       n_jobs, blk_off, total_blocks, grid);
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
