// Allocation-free form of the batched device-resident estimate.
//
// Every word of scratch memory its kernels use (the job record, the
// surrogate keys, the work-item and permute-block offsets, the permuted X
// columns, the 64-row chunk sums, the partial top-k lists of split reference
// ranges and the counter words) lives in one static device array, so a call
// allocates nothing.  The estimate runs on the all-pairs kernel with the same
// tile rules as the other entry points; its radii and counts are exact and
// its sums fixed in order, so its results equal theirs bit for bit.
//
// The array's name is a host-side stand-in in host code: its device address
// is taken once per device with hipGetSymbolAddress at initialisation and
// only that address reaches kernels.
#include <hip/hip_runtime.h>

#include <cstring>

#include "runtime.h"

// Held on every GPU the library runs on, from the code object's load until
// the process ends.  Calls that overlap on one GPU share it and race.
static __device__ __align__(256) unsigned char scratch[MTE_NOALLOC_SCRATCH_BYTES];

namespace mte {

namespace {

constexpr int kMaxDevices = 64;
// device address of `scratch` per device (set under the context lock)
void *g_scratch[kMaxDevices] = {};

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea and Flood 2014), as in the
// surrogate keys of the other entry points.
__device__ __forceinline__ uint64_t smix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The launch tables in scratch: thread 0 writes the job record and the three
// offset arrays ([0, items_a], [0, items_b], [0, blocks]); estimate 0 gets
// the identity key and estimate 1 + s the key of surrogate s of (seed, cand).
__global__ __launch_bounds__(256) void noalloc_setup_kernel(const Job job, Job *__restrict__ jobs,
                                                            EstKey *__restrict__ keys, int64_t *__restrict__ offs,
                                                            int64_t items_a, int64_t items_b, int64_t blocks,
                                                            uint64_t seed, uint32_t cand, int n_est) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t == 0) {
        *jobs = job;
        offs[0] = 0;
        offs[1] = items_a;
        offs[2] = 0;
        offs[3] = items_b;
        offs[4] = 0;
        offs[5] = blocks;
    }
    const uint64_t base = smix64(seed + kGolden);
    for (int e = t; e < n_est; e += (int)(gridDim.x * blockDim.x)) {
        EstKey k;
        k.h = e == 0 ? 0 : smix64(base ^ (((uint64_t)cand << 32) | (uint64_t)(uint32_t)(e - 1)));
        k.ident = e == 0 ? 1u : 0u;
        k.pad = 0;
        keys[e] = k;
    }
}

}  // namespace

int noalloc_bind(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(MTE_EINVAL, "device %d out of range", device);
    if (g_scratch[device]) return MTE_OK;
    void *p = nullptr;
    MTE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[device] = p;
    return MTE_OK;
}

}  // namespace mte

using namespace mte;

extern "C" int cmi_ksg_surrogates_dev_noalloc(const float *dX, int dx, const float *dY, int dy, const float *dZ,
                                              int dz, int64_t N, int64_t ld, int k, int S, uint64_t seed,
                                              uint32_t cand, double *d_out, void *stream) {
    int rc;
    if ((rc = validate_dims(dx, dy, dz, N, k))) return rc;
    if (S < 0) return fail(MTE_EINVAL, "S=%d must be >= 0", S);
    if (!dX || !dY || (dz > 0 && !dZ) || !d_out) return fail(MTE_EINVAL, "null pointer argument");
    if (dz == 0 && dZ) return fail(MTE_EINVAL, "dZ must be NULL when dz == 0");
    if (ld < N) return fail(MTE_EINVAL, "ld=%lld < N", (long long)ld);
    // the permuted X columns alone, before anything is sized on the host
    const size_t xp_bytes = sizeof(float) * (size_t)dx * (size_t)N * ((size_t)S + 1);
    if (xp_bytes > MTE_NOALLOC_SCRATCH_BYTES)
        return fail(MTE_EINVAL,
                    "N=%lld with %lld estimates and dx=%d needs at least %zu bytes of scratch; the "
                    "allocation-free call holds %zu",
                    (long long)N, (long long)S + 1, dx, xp_bytes, (size_t)MTE_NOALLOC_SCRATCH_BYTES);
    Ctx &c = ctx();
    int device;
    uint8_t *base;
    const double *harm;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (!c.inited)
            return fail(MTE_EINVAL, "cmi_ksg_surrogates_dev_noalloc needs the library initialised by mte_init");
        device = c.device;
        base = static_cast<uint8_t *>(g_scratch[device]);
        harm = c.harm;
        if (N > c.harm_n)
            return fail(MTE_EINVAL, "N=%lld exceeds the harmonic table built at mte_init (%lld rows)", (long long)N,
                        (long long)c.harm_n);
    }
    if (!base) return fail(MTE_EDEVICE, "no scratch address for device %d", device);
    MTE_HIP(hipSetDevice(device));

    std::vector<JobSpec> specs(1);
    JobSpec &sp = specs[0];
    for (int cc = 0; cc < dx; ++cc) sp.cols[cc] = dX + (size_t)cc * ld;
    for (int cc = 0; cc < dy; ++cc) sp.cols[dx + cc] = dY + (size_t)cc * ld;
    for (int cc = 0; cc < dz; ++cc) sp.cols[dx + dy + cc] = dZ + (size_t)cc * ld;
    sp.n = (int)N;
    sp.dx = dx;
    sp.dy = dy;
    sp.dz = dz;
    sp.k = k;
    sp.keys.resize((size_t)S + 1);   // the count only: the setup kernel writes the keys
    sp.out = d_out;
    TileChoice tc;
    if ((rc = pair_tiles(specs, &tc))) return rc;
    PairPlan P;
    auto bytes_of = [](const PairPlan &q) {
        return q.tbl_jobs + q.tbl_keys + q.tbl_offs + q.scratch_bytes + sizeof(uint32_t) * (size_t)q.sync_words;
    };
    if ((rc = plan_pairs(specs, tc, &P))) return rc;
    if (bytes_of(P) > MTE_NOALLOC_SCRATCH_BYTES && tc.rs_mult != 0) {
        // split reference ranges keep partial top-k lists: one range needs none
        tc.rs_mult = 0;
        if ((rc = plan_pairs(specs, tc, &P))) return rc;
    }
    const size_t need = bytes_of(P);
    if (need > MTE_NOALLOC_SCRATCH_BYTES)
        return fail(MTE_EINVAL,
                    "N=%lld with %d estimates and dx=%d needs %zu bytes of scratch; the allocation-free call "
                    "holds %zu",
                    (long long)N, S + 1, dx, need, (size_t)MTE_NOALLOC_SCRATCH_BYTES);
    // scratch layout: job record, keys, offsets, then the kernels' scratch,
    // then the counter words (every part a multiple of 256 bytes)
    Job *jobs_dev = reinterpret_cast<Job *>(base);
    EstKey *keys_dev = reinterpret_cast<EstKey *>(base + P.tbl_jobs);
    int64_t *offs_dev = reinterpret_cast<int64_t *>(base + P.tbl_jobs + P.tbl_keys);
    uint8_t *work_area = base + P.tbl_jobs + P.tbl_keys + P.tbl_offs;
    uint32_t *sync = reinterpret_cast<uint32_t *>(work_area + P.scratch_bytes);
    bind_pairs(P, work_area, sync, keys_dev);
    hipStream_t s = (hipStream_t)stream;
    const int n_est = S + 1;
    const int setup_grid = std::min(64, (n_est + 255) / 256);
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(setup_grid), dim3(256), 0, s, P.jobs[0], jobs_dev, keys_dev,
                       offs_dev, P.li.items_a, P.li.items_b, P.permute_blocks, seed, cand, n_est);
    MTE_HIP(hipGetLastError());
    if (launch_reset(sync, P.sync_words, s)) return hip_fail(hipGetLastError(), "reset launch");
    if (launch_permute(jobs_dev, 1, P.permute_blocks, offs_dev + 4, s))
        return hip_fail(hipGetLastError(), "permute launch");
    if (launch_main(tc.variant, jobs_dev, 1, offs_dev, offs_dev + 2, P.li, sync, harm, s))
        return hip_fail(hipGetLastError(), "main kernel launch");
    return MTE_OK;
}
