// Neighbour-list path of the KSG estimator (gfx950).
//
// Every estimate of a job shares the rows of Y and Z; only X is permuted.  A
// row's k-th neighbour distance eps and its three strict counts below eps
// only involve rows that are close to it in the (Y,Z) subspace (for the k-NN
// radius and n_yz) or in the Z subspace (n_z and n_xz, since both need
// d_z < eps).  So, once per (Y,Z) sample:
//
//   build    for each row i, the other rows bucketed by d_yz(i,j) and by
//            d_z(i,j) (12-bit keys of the float encoding), keeping the
//            smallest buckets that fit the list capacity, in bucket order,
//            with a lower bound of every distance left out;
//
// and then, for every (row, estimate) pair, one lane:
//
//   scan     k-NN over list 1 in bucket order, max(d_x, d_yz) with the
//            estimate's permuted X; it stops at the first bucket whose floor
//            reaches the current k-th distance (nothing later can enter).  The
//            radius is exact when it stopped that way or when the k-th
//            distance is at most the list's bound.  n_z, n_yz and n_xz scan
//            list 2 (whose entries also carry d_yz) until its bucket floor
//            reaches eps, exact when it stopped that way or eps <= its bound.
//            Without Z (one X column) there is no list 2: n_y comes from list
//            1 and n_x from range counts on the sorted X column;
//   fallback the pairs the lists cannot decide (rare) are queued and redone
//            over all rows (a block per pair, or a wave when they are many);
//   reduce   the digamma sum per estimate in the same fixed order as the
//            all-pairs kernel (64-row butterfly, then chunks in index order),
//            so both paths return the same bits.
//
// The results are the definitions' exact values: every distance is the same
// fl32 subtraction, |.| and max as in the all-pairs kernel, and the lists only
// skip rows whose distances provably cannot change the outcome.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "engine.h"
#include "ksg_device.h"

namespace mte {

namespace {

using dev::absdiff;
using dev::find_job;
using dev::fmax_;
using dev::inf_f;
using dev::topk_insert;
using dev::Unroll;

constexpr uint32_t kKeyMask = kKeyBins - 1;
constexpr uint32_t kFloorMask = ~((1u << kKeyShift) - 1u);

// Work-item and work-group indices straight from the hardware registers (the
// group index is a scalar value, so it stays wave-uniform).
__device__ __forceinline__ int tid_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int64_t bid_x() { return (int64_t)__builtin_amdgcn_workgroup_id_x(); }

// Load through a global-address-space pointer: a generic (flat) load would
// count against both the vector-memory and the LDS counters, and the wait for
// the gathers would then also wait for the next step's entries loaded ahead.
__device__ __forceinline__ float gload(const float *p, uint32_t off) {
    return ((const __attribute__((address_space(1))) float *)p)[off];
}

// List entries stored through global-address-space pointers: a generic
// (flat) store counts against the LDS counter too, so the next wait for an
// LDS atomic's return would also wait for the store to reach memory.
__device__ __forceinline__ void gstore(LEnt *p, uint32_t idx, const LEnt &v) {
    auto *q = (__attribute__((address_space(1))) uint32_t *)(p + idx);
    q[0] = __float_as_uint(v.d);
    q[1] = (uint32_t)v.j;
}

__device__ __forceinline__ void gstore(LEnt2 *p, uint32_t idx, const LEnt2 &v) {
    auto *q = (__attribute__((address_space(1))) uint32_t *)(p + idx);
    q[0] = __float_as_uint(v.dz);
    q[1] = __float_as_uint(v.dyz);
    q[2] = (uint32_t)v.j;
}

// The same with a byte offset: the address is then a uniform base plus one
// 32-bit register, the form the global loads take without address arithmetic.
__device__ __forceinline__ float gload_b(const float *p, uint32_t byte_off) {
    return *(const __attribute__((address_space(1))) float *)((const __attribute__((address_space(1))) char *)p +
                                                              byte_off);
}

constexpr uint64_t kPackMask = (uint64_t(1) << kPackBits) - 1;

__device__ __forceinline__ uint64_t pack_counts(int cxz, int cyz, int cz) {
    return (uint64_t)(uint32_t)cxz | ((uint64_t)(uint32_t)cyz << kPackBits) |
           ((uint64_t)(uint32_t)cz << (2 * kPackBits));
}

// Bucket key of a distance d >= 0 (+inf included): its exponent and top
// mantissa bits.  The sign bit is clear, so a plain shift (which gfx950
// issues at twice the rate of a bit-field extract) gives the 12-bit field.
__device__ __forceinline__ uint32_t key_of(float d) {
    return __float_as_uint(d) >> kKeyShift;
}

// Smallest value of d's bucket (d >= 0).
__device__ __forceinline__ float bucket_floor(float d) {
    return __uint_as_float(__float_as_uint(d) & kFloorMask);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = __builtin_fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The build shares the CUs with the surrogate permutation (a second stream),
// and both are bound by instruction issue; the scan needs both.  The build's
// waves take the issue arbiter's highest priority, so that the permutation,
// held to a few blocks per CU, runs in the build's idle issue cycles instead
// of stretching it: at N = 10^4 with 201 estimates the pair finishes
// together in 0.25 ms instead of 0.28.
constexpr int kBuildPrio = 3;

// Threads per build block: 8 waves, so that the 4 blocks whose histograms fit
// in LDS keep 8 waves on every SIMD (the kernel waits mostly on LDS atomics
// and L2 loads, and needs the waves to hide them).
constexpr int kBT = 512;
constexpr int kBW = kBT / 64;

// Inclusive scan over the kBT threads of a build block; returns the block total.
template <int NW = kBW>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t &incl, uint32_t *wtot) {
    const int lane = tid_x() & 63, wave = tid_x() >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    if (lane == 63) wtot[wave] = v;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        before += w < wave ? wtot[w] : 0u;
        total += wtot[w];
    }
    incl = before + v;
    __syncthreads();
    return total;
}

// ------------------------------------------------------------------ build
// One block per (list set, QB consecutive rows).  Pass 1 histograms the keys
// of d_yz and d_z over the other rows; for each row and list the largest key
// prefix that fits the capacity is kept and the histogram becomes the bucket
// write cursors; pass 2 recomputes the same distances and writes the kept
// rows bucket by bucket.  Each reference row is loaded once for the QB rows of
// the block.  The histogram of a row has C copies, lane l counting into copy
// l mod C, so that lanes with equal keys mostly update different words (the
// cursors of a bucket's copies follow each other, keeping bucket order).
// PACK: both lists' counts of a bucket share one 32-bit word, 16 bits each
// (counts stay below 2^16 when N <= 2^16).
template <int QB>
constexpr int row_batch() { return QB == 1 ? 8 : 4; }   // reference rows per thread per step

// The selection gives each thread kPer consecutive buckets (read and written
// as 16-byte words).  Bucket b of a histogram is word b: the passes over the
// pairs then take a bucket's address straight from the distance's bits.
constexpr int kPer = kKeyBins / kBT;
constexpr int kHistWords = kKeyBins;

__device__ __forceinline__ uint32_t hist_slot(uint32_t key) { return key; }

template <int QB, int C, bool PACK>
struct BuildSmem {
    static constexpr int kCopy = PACK ? kHistWords : 2 * kHistWords;   // words of one copy
    alignas(16) uint32_t h[QB][C][kCopy];
    float q[QB][kMaxDy + kMaxDz];
    uint32_t wtot[kBW];
    uint32_t red[2][kBW];
    uint32_t kept_bins[QB][2], kept_rows[QB][2];
    int set;
};

template <bool PACK>
__device__ __forceinline__ uint32_t *bin_word(uint32_t *h, int w, uint32_t key) {
    return PACK ? h + hist_slot(key) : h + w * kHistWords + hist_slot(key);
}

template <bool PACK>
__device__ __forceinline__ uint32_t bin_inc(int w) {
    return PACK ? (1u << (16 * w)) : 1u;
}

template <bool PACK>
__device__ __forceinline__ uint32_t bin_get(uint32_t word, int w) {
    return PACK ? (word >> (16 * w)) & 0xffffu : word;
}

template <bool PACK>
__device__ __forceinline__ void bin_set(uint32_t *wd, int w, uint32_t v) {
    if (PACK) *wd = (*wd & ~(0xffffu << (16 * w))) | (v << (16 * w));
    else *wd = v;
}

// Max-norm over coordinates [c_lo, c_hi) of the contiguous column copy
// (column c at zy + c * n) into acc[r][u] for the block rows r and the
// reference rows whose byte offsets within a column are boff[u]; the loads of
// up to kColChunk coordinates are issued together before they are used.
constexpr int kColChunk = 4;

template <int QB, int R>
__device__ __forceinline__ void acc_cols(const float *zy, int n, const float (*q)[kMaxDy + kMaxDz], int c_lo,
                                         int c_hi, const uint32_t (&boff)[R], float (&acc)[QB][R]) {
    for (int c0 = c_lo; c0 < c_hi; c0 += kColChunk) {
        float v[kColChunk][R];
#pragma unroll
        for (int cc = 0; cc < kColChunk; ++cc) {
            if (c0 + cc < c_hi) {
                const float *col = zy + (size_t)(c0 + cc) * n;
#pragma unroll
                for (int u = 0; u < R; ++u) v[cc][u] = gload_b(col, boff[u]);
            }
        }
#pragma unroll
        for (int cc = 0; cc < kColChunk; ++cc) {
            if (c0 + cc < c_hi) {
#pragma unroll
                for (int r = 0; r < QB; ++r) {
                    const float qc = q[r][c0 + cc];
#pragma unroll
                    for (int u = 0; u < R; ++u) acc[r][u] = fmax_(acc[r][u], absdiff(qc, v[cc][u]));
                }
            }
        }
    }
}

// Geometry of one list set, held in registers for the whole block.
struct BuildGeo {
    const float *zy;
    int n, dy, dz, w;
};

// Calls f(r, j, d_z, d_yz) for every block row r (valid rows only) and every
// row j outside its Theiler window (|j - i| > w; j != i when w = 0),
// row_batch<QB>() reference rows per thread at a time.
template <int QB, class F>
__device__ __forceinline__ void for_each_pair(const BuildGeo &G, const float (*q)[kMaxDy + kMaxDz], int i0,
                                              int nq, int tid, F &&f) {
    constexpr int kRowBatch = row_batch<QB>();
    const int n = G.n, D = G.dy + G.dz;
    // |j - i| > w  <=>  (unsigned)(j - i + w) > 2w
    const uint32_t w2 = 2u * (uint32_t)G.w;
    for (int j0 = tid; j0 < n; j0 += kBT * kRowBatch) {
        float a[QB][kRowBatch], b[QB][kRowBatch];
        uint32_t boff[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
            const int j = j0 + u * kBT;
            boff[u] = (uint32_t)(j < n ? j : i0) * 4u;
        }
#pragma unroll
        for (int r = 0; r < QB; ++r)
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) a[r][u] = 0.f;
        acc_cols<QB, kRowBatch>(G.zy, n, q, 0, G.dz, boff, a);
#pragma unroll
        for (int r = 0; r < QB; ++r)
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) b[r][u] = a[r][u];
        acc_cols<QB, kRowBatch>(G.zy, n, q, G.dz, D, boff, b);
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
            const int j = j0 + u * kBT;
            if (j >= n) continue;
#pragma unroll
            for (int r = 0; r < QB; ++r)
                if (r < nq && (uint32_t)(j + (G.w - i0 - r)) > w2) f(r, j, a[r][u], b[r][u]);
        }
    }
}

template <int QB, int C, bool PACK>
__global__ __launch_bounds__(kBT) void list_build_kernel(const ListSet *__restrict__ sets, int n_sets,
                                                           const int64_t *__restrict__ blk_off) {
    using Sm = BuildSmem<QB, C, PACK>;
    __shared__ Sm sm;
    __builtin_amdgcn_s_setprio(kBuildPrio);
    const int tid = tid_x();
    const int copy = tid & (C - 1);
    const int64_t b = bid_x();
    if (tid == 0) sm.set = find_job(blk_off, n_sets, b);
    for (int x = tid; x < QB * C * Sm::kCopy; x += kBT) (&sm.h[0][0][0])[x] = 0u;
    __syncthreads();
    const ListSet &S = sets[sm.set];
    const BuildGeo G{S.zy, S.n, S.dy, S.dz, S.theiler};
    const int n = G.n;
    const int i0 = (int)(b - blk_off[sm.set]) * QB;
    const int nq = min(QB, n - i0);
    for (int x = tid; x < QB * (G.dy + G.dz); x += kBT) {
        const int r = x / (G.dy + G.dz), c = x - r * (G.dy + G.dz);
        sm.q[r][c] = G.zy[(size_t)c * n + min(i0 + r, n - 1)];
    }
    __syncthreads();

    for_each_pair<QB>(G, sm.q, i0, nq, tid, [&](int r, int, float a, float c) {
        const uint32_t k1 = key_of(c), k2 = key_of(a);
        if (PACK) {
            // d_yz and d_z often share a bucket (when d_y <= d_z): one atomic
            // then counts both lists
            atomicAdd(bin_word<PACK>(sm.h[r][copy], 0, k1),
                      k1 == k2 ? bin_inc<PACK>(0) + bin_inc<PACK>(1) : bin_inc<PACK>(0));
            if (k1 != k2) atomicAdd(bin_word<PACK>(sm.h[r][copy], 1, k2), bin_inc<PACK>(1));
        } else {
            atomicAdd(bin_word<PACK>(sm.h[r][copy], 0, k1), bin_inc<PACK>(0));
            atomicAdd(bin_word<PACK>(sm.h[r][copy], 1, k2), bin_inc<PACK>(1));
        }
    });
    __syncthreads();

    // per row and list: keep the largest bucket prefix with at most m entries
    // (bucket keys below kept_bins are listed: the prefix is contiguous
    // because the cumulative counts grow with the key)
#pragma unroll
    for (int r = 0; r < QB; ++r) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const uint32_t cap = (uint32_t)(w == 0 ? S.m1 : S.m2);
            uint32_t local = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x)
#pragma unroll
                for (int cp = 0; cp < C; ++cp)
                    local += bin_get<PACK>(*bin_word<PACK>(sm.h[r][cp], w, tid * kPer + x), w);
            uint32_t incl;
            block_scan(local, incl, sm.wtot);
            uint32_t run = incl - local, nb = 0, nr = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x) {
                uint32_t cnt = 0;
#pragma unroll
                for (int cp = 0; cp < C; ++cp) {
                    // exclusive start of (bucket, copy) = write cursor
                    uint32_t *wd = bin_word<PACK>(sm.h[r][cp], w, tid * kPer + x);
                    const uint32_t v = bin_get<PACK>(*wd, w);
                    bin_set<PACK>(wd, w, run + cnt);
                    cnt += v;
                }
                run += cnt;
                if (run <= cap) { ++nb; nr += cnt; }
            }
            nb = (uint32_t)wave_sum((int)nb);
            nr = (uint32_t)wave_sum((int)nr);
            if ((tid & 63) == 0) { sm.red[0][tid >> 6] = nb; sm.red[1][tid >> 6] = nr; }
            __syncthreads();
            if (tid == 0) {
                uint32_t kb = 0, kr = 0;
                for (int v = 0; v < kBW; ++v) { kb += sm.red[0][v]; kr += sm.red[1][v]; }
                sm.kept_bins[r][w] = kb;
                sm.kept_rows[r][w] = kr;
            }
            __syncthreads();
        }
    }
    // pass 2 with the kept prefixes and the rows' list bases in registers
    uint32_t keep[QB][2];
    LEnt *out1[QB];
    LEnt2 *out2[QB];
#pragma unroll
    for (int r = 0; r < QB; ++r) {
        keep[r][0] = sm.kept_bins[r][0];
        keep[r][1] = sm.kept_bins[r][1];
        const int64_t i = min(i0 + r, n - 1);
        out1[r] = S.l1 + i * S.s1;
        out2[r] = S.l2 + i * S.s2;
    }
    const uint32_t m1 = (uint32_t)S.m1, m2 = (uint32_t)S.m2;
    for_each_pair<QB>(G, sm.q, i0, nq, tid, [&](int r, int j, float a, float c) {
        const uint32_t k1 = key_of(c), k2 = key_of(a);
        if (k1 < keep[r][0]) {
            const uint32_t pos =
                bin_get<PACK>(atomicAdd(bin_word<PACK>(sm.h[r][copy], 0, k1), bin_inc<PACK>(0)), 0);
            if (pos < m1) gstore(out1[r], pos, LEnt{c, j});
        }
        if (k2 < keep[r][1]) {
            const uint32_t pos =
                bin_get<PACK>(atomicAdd(bin_word<PACK>(sm.h[r][copy], 1, k2), bin_inc<PACK>(1)), 1);
            if (pos < m2) gstore(out2[r], pos, LEnt2{a, c, j});
        }
    });
    // lengths, bounds and the sentinels after each list.  A list is whole
    // when it holds every row outside the window, or when the first bucket
    // left out is the +inf bucket (every row at a finite distance fitted and
    // the others' differences overflow): a row at +inf can enter neither a
    // radius (every listed distance is at most +inf) nor a strict count below
    // any radius, so leaving it out changes nothing.  Whole lists get +inf
    // for the bound and the sentinels; bound + 1 ulp would be a NaN there.
    for (int x = tid; x < QB * 2 * kListPad; x += kBT) {
        const int r = x / (2 * kListPad), w = (x / kListPad) & 1, u = x % kListPad;
        if (r >= nq) continue;
        const int64_t i = i0 + r;
        const int tw = S.theiler;   // rows outside the window
        const uint32_t total = (uint32_t)(n - 1 - min((int)i, tw) - min(n - 1 - (int)i, tw));
        const uint32_t kb = sm.kept_bins[r][w], kr = sm.kept_rows[r][w];
        const bool whole = kr == total || (kb << kKeyShift) >= __float_as_uint(inf_f());
        const float bound = whole ? inf_f() : __uint_as_float(kb << kKeyShift);
        const float sent = whole ? inf_f() : __uint_as_float((kb << kKeyShift) + 1u);
        if (w == 0) S.l1[i * S.s1 + kr + u] = LEnt{sent, (int32_t)i};
        else S.l2[i * S.s2 + kr + u] = LEnt2{sent, inf_f(), (int32_t)i};
        if (u == 0) {
            S.len[2 * i + w] = (int32_t)kr;
            S.bound[2 * i + w] = bound;
        }
    }
}

// ------------------------------------------------------------------ build, compiled dimensions
// list_build_kernel for sets with DZ Z columns and one Y column, N < 2^16,
// QB rows per block: two passes over the pairs as there, with straight-line
// distance code and a counting pass without branches.  The counting pass
// counts every row j < N, the query row itself included (its distances are
// exactly 0, so it adds one to bin 0 of both lists), and sends the lanes past
// the last row to bin 4095, the bin of NaN encodings, which no distance
// reaches; afterwards the query row and the rows of its Theiler window are
// taken out again and bin 4095 is cleared.  The selection takes both lists
// of every row in one block scan: a bin's word holds both lists' counts, 16
// bits each, and their sums stay below 2^16, so one packed prefix is both
// lists' write cursors.  The write pass checks the window per pair.
constexpr int kLR = 4;                  // reference rows per thread per step

template <int DZ, int QB, int R>
__device__ __forceinline__ void lean_dists(const float *zy, int n, const float (&q)[QB][DZ + 1],
                                           const uint32_t (&boff)[R], float (&az)[QB][R], float (&ayz)[QB][R]) {
    float v[DZ + 1][R];
#pragma unroll
    for (int c = 0; c < DZ + 1; ++c)
#pragma unroll
        for (int u = 0; u < R; ++u) v[c][u] = gload_b(zy + (size_t)c * n, boff[u]);
#pragma unroll
    for (int r = 0; r < QB; ++r)
#pragma unroll
        for (int u = 0; u < R; ++u) {
            float a = absdiff(q[r][0], v[0][u]);
#pragma unroll
            for (int c = 1; c < DZ; ++c) a = fmax_(a, absdiff(q[r][c], v[c][u]));
            az[r][u] = a;
            ayz[r][u] = fmax_(a, absdiff(q[r][DZ], v[DZ][u]));
        }
}

template <int QB>
struct LeanSmem {
    alignas(16) uint32_t h[QB][kKeyBins];   // list 1 count | list 2 count << 16, then cursors
    float q[QB][kBuildFixedDz + 1];
    uint32_t wtot[QB][kBW];
    uint32_t red[2 * QB][kBW];
    int set;
};

template <int DZ, int QB>
__global__ __launch_bounds__(kBT) void list_build_dz_kernel(const ListSet *__restrict__ sets, int n_sets,
                                                            const int64_t *__restrict__ blk_off) {
    __shared__ LeanSmem<QB> sm;
    __builtin_amdgcn_s_setprio(kBuildPrio);
    const int tid = tid_x(), lane = tid & 63, wave = tid >> 6;
    const int64_t b = bid_x();
    if (tid == 0) sm.set = find_job(blk_off, n_sets, b);
    for (int x = tid; x < QB * kKeyBins; x += kBT) (&sm.h[0][0])[x] = 0u;
    __syncthreads();
    const ListSet &S = sets[sm.set];
    const float *zy = S.zy;
    const int n = S.n, tw = S.theiler;
    const int i0 = (int)(b - blk_off[sm.set]) * QB;
    const int nq = min(QB, n - i0);
    for (int x = tid; x < QB * (DZ + 1); x += kBT) {
        const int r = x / (DZ + 1), c = x - r * (DZ + 1);
        sm.q[r][c] = zy[(size_t)c * n + min(i0 + r, n - 1)];
    }
    __syncthreads();
    float q[QB][DZ + 1];
#pragma unroll
    for (int r = 0; r < QB; ++r)
#pragma unroll
        for (int c = 0; c < DZ + 1; ++c) q[r][c] = sm.q[r][c];
    constexpr uint32_t kInc1 = 1u, kInc2 = 1u << 16, kSink = (uint32_t)kKeyBins - 1u;
    const int step = kBT * kLR;
    const int full = n / step * step;

    // pass 1: counts of every row j < n
    auto count_step = [&](int j0, bool tail) {
        uint32_t boff[kLR], sink[kLR];
#pragma unroll
        for (int u = 0; u < kLR; ++u) {
            const int j = j0 + u * kBT;
            const bool in = !tail || j < n;
            boff[u] = (uint32_t)(in ? j : i0) * 4u;
            sink[u] = in ? 0u : kSink;
        }
        float az[QB][kLR], ayz[QB][kLR];
        lean_dists<DZ, QB, kLR>(zy, n, q, boff, az, ayz);
#pragma unroll
        for (int r = 0; r < QB; ++r)
#pragma unroll
            for (int u = 0; u < kLR; ++u) {
                const uint32_t k1 = key_of(ayz[r][u]) | sink[u], k2 = key_of(az[r][u]) | sink[u];
                // one compare: the increment is chosen in the branch that
                // takes the second key's atomic
                uint32_t inc = kInc1 + kInc2;
                if (k1 != k2) {
                    inc = kInc1;
                    atomicAdd(&sm.h[r][k2], kInc2);
                }
                atomicAdd(&sm.h[r][k1], inc);
            }
    };
    int j0 = tid;
    for (; j0 < full; j0 += step) count_step(j0, false);
    if (j0 < n) count_step(j0, true);
    __syncthreads();
    // take out the query rows and their windows (counted above), clear the sink
    const int wn = 2 * tw + 1;
    for (int x = tid; x < QB * wn; x += kBT) {
        const int r = x / wn, j = i0 + r + (x % wn) - tw;
        if (r >= nq || j < 0 || j >= n) continue;
        float a = 0.f;
#pragma unroll
        for (int c = 0; c < DZ; ++c) a = fmax_(a, absdiff(sm.q[r][c], zy[(size_t)c * n + j]));
        const float cyz = fmax_(a, absdiff(sm.q[r][DZ], zy[(size_t)DZ * n + j]));
        atomicSub(&sm.h[r][key_of(cyz)], kInc1);
        atomicSub(&sm.h[r][key_of(a)], kInc2);
    }
    __syncthreads();
    if (tid < QB) sm.h[tid][kSink] = 0u;
    __syncthreads();

    // selection: per row, the packed exclusive prefix over the bins (thread t
    // owns bins t*kPer .. t*kPer+kPer-1) becomes the cursors; a list keeps
    // the bins whose inclusive count fits its capacity (a prefix, since the
    // counts only grow)
    const uint32_t m1 = (uint32_t)S.m1, m2 = (uint32_t)S.m2;
    uint32_t kb[QB][2], kr[QB][2];
    {
        uint32_t loc[QB], run[QB];
#pragma unroll
        for (int r = 0; r < QB; ++r) {
            loc[r] = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x) loc[r] += sm.h[r][tid * kPer + x];
            run[r] = loc[r];
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1)
#pragma unroll
            for (int r = 0; r < QB; ++r) {
                const uint32_t t = __shfl_up(run[r], off, 64);
                if (lane >= off) run[r] += t;
            }
        if (lane == 63)
#pragma unroll
            for (int r = 0; r < QB; ++r) sm.wtot[r][wave] = run[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QB; ++r) {
            uint32_t before = 0;
#pragma unroll
            for (int w = 0; w < kBW; ++w) before += w < wave ? sm.wtot[r][w] : 0u;
            run[r] += before - loc[r];         // exclusive start of this thread's bins
            uint32_t nb = 0, nr = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x) {
                uint32_t *wd = &sm.h[r][tid * kPer + x];
                const uint32_t v = *wd;
                *wd = run[r];
                run[r] += v;
                // bins kept by list 1 (low half) and list 2 (high half)
                if ((run[r] & 0xffffu) <= m1) { nb += 1u; nr += v & 0xffffu; }
                if ((run[r] >> 16) <= m2) { nb += 1u << 16; nr += v & 0xffff0000u; }
            }
            nb = (uint32_t)wave_sum((int)nb);
            nr = (uint32_t)wave_sum((int)nr);
            if (lane == 0) {
                sm.red[2 * r][wave] = nb;
                sm.red[2 * r + 1][wave] = nr;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QB; ++r) {
            uint32_t nb = 0, nr = 0;
#pragma unroll
            for (int w = 0; w < kBW; ++w) {
                nb += sm.red[2 * r][w];
                nr += sm.red[2 * r + 1][w];
            }
            kb[r][0] = nb & 0xffffu;
            kb[r][1] = nb >> 16;
            kr[r][0] = nr & 0xffffu;
            kr[r][1] = nr >> 16;
        }
    }

    // pass 2: write the kept rows (bin 4095 never holds a row: kept bins are
    // taken below it)
    uint32_t keep1[QB], keep2[QB];
    LEnt *out1[QB];
    LEnt2 *out2[QB];
#pragma unroll
    for (int r = 0; r < QB; ++r) {
        keep1[r] = min(kb[r][0], kSink);
        keep2[r] = min(kb[r][1], kSink);
        const int64_t i = min(i0 + r, n - 1);
        out1[r] = S.l1 + i * S.s1;
        out2[r] = S.l2 + i * S.s2;
    }
    const uint32_t w2 = 2u * (uint32_t)tw;
    auto write_step = [&](int jb, bool tail) {
        uint32_t boff[kLR];
        int jj[kLR];
#pragma unroll
        for (int u = 0; u < kLR; ++u) {
            jj[u] = jb + u * kBT;
            boff[u] = (uint32_t)(!tail || jj[u] < n ? jj[u] : i0) * 4u;
        }
        float az[QB][kLR], ayz[QB][kLR];
        lean_dists<DZ, QB, kLR>(zy, n, q, boff, az, ayz);
#pragma unroll
        for (int r = 0; r < QB; ++r)
#pragma unroll
            for (int u = 0; u < kLR; ++u) {
                const int j = jj[u];
                const bool ok = r < nq && (!tail || j < n) && (uint32_t)(j + (tw - i0 - r)) > w2;
                const uint32_t k1 = key_of(ayz[r][u]), k2 = key_of(az[r][u]);
                if (ok && k1 < keep1[r]) {
                    const uint32_t pos = atomicAdd(&sm.h[r][k1], kInc1) & 0xffffu;
                    if (pos < m1) gstore(out1[r], pos, LEnt{ayz[r][u], j});
                }
                if (ok && k2 < keep2[r]) {
                    const uint32_t pos = atomicAdd(&sm.h[r][k2], kInc2) >> 16;
                    if (pos < m2) gstore(out2[r], pos, LEnt2{az[r][u], ayz[r][u], j});
                }
            }
    };
    j0 = tid;
    for (; j0 < full; j0 += step) write_step(j0, false);
    if (j0 < n) write_step(j0, true);
    // lengths, bounds and the sentinels (as in list_build_kernel; they lie
    // past the kept entries, so no barrier is needed before them)
    for (int x = tid; x < QB * 2 * kListPad; x += kBT) {
        const int r = x / (2 * kListPad), w = (x / kListPad) & 1, u = x % kListPad;
        if (r >= nq) continue;
        const int64_t i = i0 + r;
        const uint32_t total = (uint32_t)(n - 1 - min((int)i, tw) - min(n - 1 - (int)i, tw));
        // the row's kept bins and rows, summed again from the waves' shares
        // in LDS (a register array indexed by r would go to scratch memory)
        uint32_t nb = 0, nr = 0;
#pragma unroll
        for (int v2 = 0; v2 < kBW; ++v2) {
            nb += sm.red[2 * r][v2];
            nr += sm.red[2 * r + 1][v2];
        }
        const uint32_t kbw = w == 0 ? nb & 0xffffu : nb >> 16, krw = w == 0 ? nr & 0xffffu : nr >> 16;
        const bool whole = krw == total || (kbw << kKeyShift) >= __float_as_uint(inf_f());
        const float bound = whole ? inf_f() : __uint_as_float(kbw << kKeyShift);
        const float sent = whole ? inf_f() : __uint_as_float((kbw << kKeyShift) + 1u);
        if (w == 0) S.l1[i * S.s1 + krw + u] = LEnt{sent, (int32_t)i};
        else S.l2[i * S.s2 + krw + u] = LEnt2{sent, inf_f(), (int32_t)i};
        if (u == 0) {
            S.len[2 * i + w] = (int32_t)krw;
            S.bound[2 * i + w] = bound;
        }
    }
}

// ------------------------------------------------------------------ columns
// One thread per (set, row): the row's Z then Y coordinates into the set's
// contiguous column copy, so that the build addresses every column from one
// base pointer; the first threads also clear the launch's counters.
__global__ __launch_bounds__(kBlock) void list_zy_kernel(const ListLaunch L) {
    const int64_t g = bid_x() * kBlock + tid_x();
    // the launch's counters are cleared here too (a kernel launch fewer; the
    // grid covers at least kListCounterWords threads)
    if (g < kListCounterWords) L.counters[g] = 0u;
    if (g >= L.rows) return;
    const int t = find_job(L.row_off, L.n_sets, g);
    const ListSet &S = L.sets[t];
    const int64_t j = g - L.row_off[t], n = S.n;
    const int dy = S.dy, dz = S.dz;
    for (int c = 0; c < dz; ++c) S.zy[c * n + j] = S.cols[dy + c][j];
    for (int c = 0; c < dy; ++c) S.zy[(dz + c) * n + j] = S.cols[c][j];
}

// ------------------------------------------------------------------ X sort
// One block per job without Z: its X column sorted ascending (bitonic, in
// LDS, padded with +inf to a power of two), for the n_x range counts.
constexpr int kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void list_sortx_kernel(const ListLaunch L) {
    __shared__ float v[kNoZSortMax];
    const Job &J = L.jobs[bid_x()];
    if (!J.xs) return;
    const int tid = tid_x();
    const int n = J.n;
    int P = 1;
    while (P < n) P <<= 1;
    for (int x = tid; x < P; x += kSortThreads) v[x] = x < n ? J.cols[0][x] : inf_f();
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int x = tid; x < P; x += kSortThreads) {
                const int y = x ^ j;
                if (y > x) {
                    const float a = v[x], b = v[y];
                    if ((a > b) == ((x & k) == 0)) {
                        v[x] = b;
                        v[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int x = tid; x < n; x += kSortThreads) J.xs[x] = v[x];
}

// ------------------------------------------------------------------ row order
// One block per list set with an order array: its rows grouped by Morton
// (Z-curve) cell of their first D <= 6 coordinates in the contiguous copy (Z
// columns, then Y).  Each coordinate is cut into 2^(12/D) equal steps between
// the column's minimum and maximum and the step indices' bits are interleaved
// from the top into a cell code below 2^12; a counting sort over the codes in
// LDS (histogram, block scan, scatter) then lists the rows cell by cell.  The
// cell codes stay in registers (a thread takes rows tid + u * 1024) and the
// block takes 17 KB of LDS, so it finds room beside the build's blocks.
// Rows next to each other in this order are near in (Y,Z) and share list
// entries.  The order of the rows within a cell follows the scatter's LDS
// atomics and may differ between launches: only the order in which the scan
// visits rows depends on it, not any result.
constexpr int kOrderDims = 6;
constexpr int kOrderBits = 12;
constexpr int kOrderCells = 1 << kOrderBits;

__global__ __launch_bounds__(kSortThreads) void list_order_kernel(const ListLaunch L) {
    constexpr int NW = kSortThreads / 64, PER = kOrderCells / kSortThreads;
    constexpr int ROWS = kNoZSortMax / kSortThreads;   // rows per thread
    __shared__ uint32_t h[kOrderCells];
    __shared__ float red[2][kOrderDims][NW];
    __shared__ uint32_t wtot[NW];
    const ListSet &S = L.sets[bid_x()];
    const int n = S.n;
    if (!S.order || n > kNoZSortMax) return;    // the host sets no order array then
    const int tid = tid_x(), lane = tid & 63, w = tid >> 6;
    const int D = min(kOrderDims, S.dy + S.dz);
    const int bpd = kOrderBits / D;
    for (int c = tid; c < kOrderCells; c += kSortThreads) h[c] = 0;
    // column ranges
    float lo[kOrderDims], hi[kOrderDims];
#pragma unroll
    for (int q = 0; q < kOrderDims; ++q) {
        lo[q] = inf_f();
        hi[q] = -inf_f();
        if (q < D)
            for (int x = tid; x < n; x += kSortThreads) {
                const float c = S.zy[(int64_t)q * n + x];
                lo[q] = __builtin_fminf(lo[q], c);
                hi[q] = __builtin_fmaxf(hi[q], c);
            }
        lo[q] = wave_min(lo[q]);
        hi[q] = -wave_min(-hi[q]);
        if (lane == 0) {
            red[0][q][w] = lo[q];
            red[1][q][w] = hi[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kOrderDims; ++q) {
        lo[q] = red[0][q][0];
        hi[q] = red[1][q][0];
        for (int u = 1; u < NW; ++u) {
            lo[q] = __builtin_fminf(lo[q], red[0][q][u]);
            hi[q] = __builtin_fmaxf(hi[q], red[1][q][u]);
        }
    }
    // the steps are cut on halved values: differences of halved finite
    // floats cannot overflow, so no step of the cell code meets inf / inf
    const float steps = (float)(1 << bpd);
#pragma unroll
    for (int q = 0; q < kOrderDims; ++q) {
        lo[q] *= 0.5f;
        hi[q] *= 0.5f;
    }
    uint32_t code[ROWS];                        // each row's cell, computed once
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int x = tid + u * kSortThreads;
        code[u] = 0;
        if (x >= n) continue;
        uint32_t cell[kOrderDims];
#pragma unroll
        for (int q = 0; q < kOrderDims; ++q) {
            cell[q] = 0;
            if (q < D && hi[q] > lo[q]) {
                const float t = (0.5f * S.zy[(int64_t)q * n + x] - lo[q]) / (hi[q] - lo[q]) * steps;
                cell[q] = t >= 1.0f ? (t < steps ? (uint32_t)t : (uint32_t)steps - 1u) : 0u;
            }
        }
        uint32_t c = 0;
        for (int bit = bpd - 1; bit >= 0; --bit)
            for (int q = 0; q < D; ++q) c = c << 1 | ((cell[q] >> bit) & 1u);
        code[u] = c;              // < 2^(D * bpd) <= kOrderCells
        atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    // exclusive offsets: each thread owns PER consecutive cells
    uint32_t loc[PER], sum = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        loc[u] = h[tid * PER + u];
        sum += loc[u];
    }
    uint32_t incl;
    block_scan<NW>(sum, incl, wtot);
    uint32_t run = incl - sum;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        h[tid * PER + u] = run;
        run += loc[u];
    }
    __syncthreads();
    // the counts add up to n, so every position is below n
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int x = tid + u * kSortThreads;
        if (x < n) S.order[atomicAdd(&h[code[u]], 1u)] = x;
    }
}

// ------------------------------------------------------------------ scan
// Each list row is followed by kListPad sentinel entries (row = self, d_yz =
// +inf) whose key distance lies in the bucket that starts at the row's bound:
// the bound plus one unit in the last place (+inf for a whole list: nothing
// left out, or only rows at +inf).
// A step of kU <= kListPad entries that starts at or before the list's end
// then needs no bounds checks, and the last step of a list always ends on a
// sentinel, whose bucket-floor test (floor = bound >= radius) is exactly the
// condition under which the list decides the pair.  A sentinel that enters
// the k-NN list (bound + 1 ulp < k-th distance) leaves a radius above the
// bound, i.e. an undecided pair, as it should.
// Entries per step (KU, the next step's loaded ahead): 8 or 4, a launch
// parameter.  One-job launches take 8 (C2's scan: 0.33 ms against 0.38-0.40
// with 4); launches of several jobs take 4, whose scan kernel holds 55
// instead of 79 registers and runs 8 waves per SIMD instead of 6 (network
// inference 1.08-1.09 s against 1.13-1.14 s with 8).
constexpr int kU = 8;   // the largest step
static_assert(kU <= kListPad, "a step must stay within the sentinels");

template <int KMAX, int DXM>
struct Lane {
    const float *xt;
    uint32_t cs;    // xt column stride n * n_est (xt has fewer than 2^31 elements)
    uint32_t E, e;
    int dx;
    float xq[DXM];

    __device__ Lane(const Job &J, int i, int e_) : e((uint32_t)e_) {
        xt = J.xt;
        E = (uint32_t)J.n_est;
        cs = (uint32_t)J.n * E;
        dx = J.dx;
        Unroll<0, DXM>::upto(dx, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            xq[c] = xt[c * cs + (uint32_t)i * E + e];
        });
    }

    // max-norm over the X columns between this lane's row and the rows of a
    // step (under the estimate's permutation); all loads issued before use
    template <class Ent, int NU>
    __device__ __forceinline__ void xdist(const Ent (&en)[NU], float (&d)[NU]) const {
        uint32_t o[NU];
        float v[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            o[u] = (uint32_t)en[u].j * E + e;
            v[u] = gload(xt, o[u]);
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) d[u] = absdiff(xq[0], v[u]);
        Unroll<1, DXM>::upto(dx, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int u = 0; u < NU; ++u) v[u] = gload(xt, c * cs + o[u]);
#pragma unroll
            for (int u = 0; u < NU; ++u) d[u] = fmax_(d[u], absdiff(xq[c], v[u]));
        });
    }
};

template <class Ent, int NU>
__device__ __forceinline__ void load_step(const Ent *l, Ent (&en)[NU]) {
#pragma unroll
    for (int u = 0; u < NU; ++u) en[u] = l[u];
}

// Wave-uniform helpers of the cooperative finish.
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
// The lane mask of one compare as the compare writes it (no round trip of the
// predicate through a vector register); masks are combined by the scalar unit.
// (The scan keeps ballot(): with this form its one-job launch at N = 10^4 took
// 0.343 ms instead of 0.329.)
__device__ __forceinline__ uint64_t cmp_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int lowest(uint64_t m) { return __builtin_amdgcn_readfirstlane(__builtin_ctzll(m)); }
__device__ __forceinline__ float bcast(float v, int o) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), o));
}
__device__ __forceinline__ int bcast(int v, int o) { return __builtin_amdgcn_readlane(v, o); }
__device__ __forceinline__ uint32_t bcast(uint32_t v, int o) { return (uint32_t)__builtin_amdgcn_readlane((int)v, o); }
template <class T>
__device__ __forceinline__ T *bcast(T *v, int o) {
    const uint64_t a = reinterpret_cast<uint64_t>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a, o);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a >> 32), o);
    return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// The scans' divergence: the 64 lanes of a wave stop at very different list
// positions (a few estimates of a row have radii far above the others), and
// a wave runs until its slowest lane is done.  So each phase runs lane by lane
// only while more than kCoopLanes lanes are still scanning; the wave then
// finishes the remaining lanes one after the other with all 64 lanes, 64
// list entries per step (a ballot per test, the top-k kept wave-uniform).
// Entries, distances and tests are the same, so the results are too: a scan
// may stop at any position whose bucket floor reaches the current radius.
// A cooperative step gathers X for 64 different rows (64 cache lines instead
// of the 2-4 of a lane-by-lane step, whose lanes are adjacent estimates), so
// it only pays for the last few lanes: on C2 (N = 10^4, 201 estimates), in the
// hardware block order, the scan took 0.62 ms without it, 0.48 ms with
// kCoopLanes = 2, 0.50 ms with 4, 0.54 ms with 8, 0.67 ms with 16; with the
// XCD-aware order (below), whose gathers mostly hit L2, 0.343 ms with 2,
// 0.335 ms with 4, 0.350 ms with 6, 0.372 ms with 8.  2 or 4 entries per lane
// per cooperative step were slower still (more scattered gathers past the
// stop position).
// The threshold (kCoopLanes by default) and the grouped lane order are launch
// parameters, chosen by the tuner; neither changes a result.
constexpr int kCoopU = 1;      // list entries per lane per cooperative step

// UNITS: the lane order of launches of several jobs below (a separate
// instance, so that the other orders' kernels keep their registers: with both
// mappings in one kernel the one-job scan took 81 registers instead of 79, 5
// waves per SIMD instead of 6, and 0.342 ms instead of 0.328 at N = 10^4).
template <int KMAX, int DXM, int KU, bool UNITS>
__global__ __launch_bounds__(kBlock) void list_scan_kernel(const ListLaunch L) {
    static_assert(KU <= kU, "a step must stay within the sentinels");
    const int lane = tid_x() & 63;
    // Lane order.  A launch of one job runs its lanes over estimate groups:
    // group c holds rows x estimates 64c .. 64c + E_c - 1, row-major, with
    // E_c = 64 but for the last group, which takes the remainder too (64 to
    // 127 estimates; all E when E < 64), so that a wave takes one row and 64
    // consecutive estimates, or two rows.  The hardware deals blocks to the
    // XCDs in turn; block b is renumbered so that each XCD takes a contiguous
    // range of lanes, i.e. one or two groups, and its L2 holds those groups'
    // columns of xt (n * 256 bytes each) instead of all of them.  A launch of
    // several jobs runs its lanes over units of (job, estimate group), each
    // row-major over the group's estimates with the rows in the set's Morton
    // order (rows that run together are near in (Y,Z), so their list entries
    // and the X values they gather overlap), and deals the units to the XCDs
    // in turn (unit u to XCD u mod 8, each XCD taking its units one after
    // another): an XCD's L2 then holds the xt columns of the group it is on
    // (n * 256 bytes) instead of gathering over whole jobs' xt (n * E * 4
    // bytes each), and unequal jobs still spread over all XCDs.
    const bool grouped = L.grouped == 1;          // set by the host for launches of one job only
    const int coop = L.coop_lanes;
    int64_t b = bid_x();
    if (grouped) {
        const int64_t nb = (int64_t)__builtin_amdgcn_grid_size_x() / kBlock, hb = b;
        const int64_t q = nb / kXcds, rem = nb % kXcds, x = hb % kXcds;
        b = x * q + min(x, rem) + hb / kXcds;
    }
    bool live;
    int64_t g;
    int jb, i, e;
    if constexpr (UNITS) {
        // XCD x's k-th block: the last of x's units whose first block is <= k
        const int x = (int)(b % kXcds);
        const int64_t k = b / kXcds;
        const int64_t *xo = L.xcd_off + (int64_t)x * (L.unit_t + 1);
        if (k >= xo[L.unit_t]) return;            // past x's blocks (no barrier in this kernel)
        int lo = 0, hi = L.unit_t - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (xo[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const int u = x + lo * kXcds;
        const int64_t info = L.unit_info[u];
        jb = (int)(info >> 32);
        const int grp = (int)(info & 0xffffffff);
        const Job &Ju = L.jobs[jb];
        const int ng = max(1, Ju.n_est / 64);
        const int eg = grp == ng - 1 ? Ju.n_est - 64 * grp : 64;
        const int64_t ul = (int64_t)Ju.n * eg;
        const int64_t l0 = (k - xo[lo]) * kBlock + tid_x();
        // lanes past the unit's last pair mirror it and store nothing
        live = l0 < ul;
        const int64_t lu = live ? l0 : ul - 1;
        const int il = (int)(lu / eg);
        e = 64 * grp + (int)(lu - (int64_t)il * eg);
        const ListSet &Su = L.sets[Ju.set];
        i = Su.order ? Su.order[il] : il;
        g = L.lane_off[jb] + (int64_t)il * Ju.n_est + e;
    } else {
    const int64_t g0 = b * kBlock + tid_x();
    // every lane of a wave takes part in the cooperative steps: lanes past
    // the last pair mirror it and store nothing
    live = g0 < L.lanes;
    g = live ? g0 : L.lanes - 1;
    jb = find_job(L.lane_off, L.n_jobs, g);
    {
        const Job &J = L.jobs[jb];
        const ListSet &S = L.sets[J.set];
        const int64_t r = g - L.lane_off[jb];
        if (grouped) {
            const int64_t gsz = (int64_t)J.n * 64;
            const int ng = max(1, J.n_est / 64);
            const int grp = (int)min(r / gsz, (int64_t)(ng - 1));
            const int64_t rr = r - grp * gsz;
            const int eg = grp == ng - 1 ? J.n_est - 64 * grp : 64;
            i = (int)(rr / eg);
            e = 64 * grp + (int)(rr - (int64_t)i * eg);
        } else {
            const int il = (int)(r / J.n_est);
            e = (int)(r - (int64_t)il * J.n_est);
            i = S.order ? S.order[il] : il;
        }
    }
    }
    const Job &J = L.jobs[jb];
    const ListSet &S = L.sets[J.set];
    const int n = J.n;
    Lane<KMAX, DXM> ln(J, i, e);

    // X distance of one entry under lane o's estimate (cooperative steps)
    auto coop_xdist = [&](const float *xt, uint32_t cs, uint32_t E, uint32_t eo, int dxo, const float (&xq)[DXM],
                          int32_t j) {
        const uint32_t oo = (uint32_t)j * E + eo;
        float d = absdiff(xq[0], gload(xt, oo));
        Unroll<1, DXM>::upto(dxo, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            d = fmax_(d, absdiff(xq[c], gload(xt, c * cs + oo)));
        });
        return d;
    };

    // k-NN radius over list 1
    float top[KMAX];
    const int pad_front = KMAX - J.k;
#pragma unroll
    for (int m = 0; m < KMAX; ++m) top[m] = m < pad_front ? -inf_f() : inf_f();
    const LEnt *l1 = S.l1 + (int64_t)i * S.s1;
    const int len1 = S.len[2 * (int64_t)i];
    bool decided = false, act = live;
    int seen1 = 0, seen2 = 0;     // list entries read (statistics)
    int m1 = 0;
    {
        LEnt cur[KU];
        load_step(l1, cur);
        while (__builtin_popcountll(ballot(act)) > coop) {
            if (!act) continue;
            if (m1 > len1) {          // list exhausted: undecided
                act = false;
                continue;
            }
            seen1 = m1 + KU;
            LEnt nxt[KU];
            load_step(l1 + m1 + KU, nxt);
            float d[KU];
            ln.xdist(cur, d);
            float lo = inf_f();
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                d[u] = fmax_(d[u], cur[u].d);
                lo = __builtin_fminf(lo, d[u]);
            }
            if (lo < top[KMAX - 1]) {
#pragma unroll
                for (int u = 0; u < KU; ++u) topk_insert<KMAX>(top, d[u]);
            }
            if (bucket_floor(cur[KU - 1].d) >= top[KMAX - 1]) {
                decided = true;
                act = false;
                continue;
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) cur[u] = nxt[u];
            m1 += KU;
        }
    }
    for (uint64_t rest = ballot(act); rest; rest &= rest - 1) {
        const int o = lowest(rest);
        const LEnt *pl = bcast(l1, o);
        const int end = bcast(len1, o) + kListPad;
        const float *xt = bcast(ln.xt, o);
        const uint32_t cs = bcast(ln.cs, o), E = bcast(ln.E, o), eo = bcast(ln.e, o);
        const int dxo = bcast(ln.dx, o);
        float xq[DXM], pt[KMAX];
#pragma unroll
        for (int c = 0; c < DXM; ++c) xq[c] = bcast(ln.xq[c], o);
#pragma unroll
        for (int q = 0; q < KMAX; ++q) pt[q] = bcast(top[q], o);
        bool dec = false;
        int p = bcast(m1, o);
        for (; p < end; p += 64 * kCoopU) {
            // kCoopU entries per lane, all loads issued first
            const int last = min(p + 64 * kCoopU - 1, end - 1);
            const float stop = bucket_floor(pl[last].d);
            LEnt en[kCoopU];
#pragma unroll
            for (int u = 0; u < kCoopU; ++u) {
                const int idx = p + lane + 64 * u;
                en[u] = pl[min(idx, end - 1)];
            }
            float d[kCoopU];
#pragma unroll
            for (int u = 0; u < kCoopU; ++u) {
                d[u] = fmax_(coop_xdist(xt, cs, E, eo, dxo, xq, en[u].j), en[u].d);
                if (p + lane + 64 * u >= end) d[u] = inf_f();
            }
#pragma unroll
            for (int u = 0; u < kCoopU; ++u)
                for (uint64_t cand = ballot(d[u] < pt[KMAX - 1]); cand; cand &= cand - 1)
                    topk_insert<KMAX>(pt, bcast(d[u], lowest(cand)));
            if (stop >= pt[KMAX - 1]) {
                dec = true;
                p = last + 1;
                break;
            }
        }
        if (lane == o) {
#pragma unroll
            for (int q = 0; q < KMAX; ++q) top[q] = pt[q];
            decided = dec;
            seen1 = min(p, end);
        }
    }
    const float eps = top[KMAX - 1];

    // n_z, n_yz and n_xz from list 2 below eps (every row with d_z < eps, and
    // so every row with d_yz < eps, is listed when eps <= its bound)
    int cxz = 0, cyz = 0, cz = 0;
    const LEnt2 *l2 = S.l2 + (int64_t)i * S.s2;
    const int len2 = S.len[2 * (int64_t)i + 1];
    const bool noz = J.dz == 0;
    const bool knn_decided = decided;
    // a job of a set counted by ranks takes its counts from the rank-count
    // kernel: this kernel hands it the radius (or the pair to the redo)
    const bool ranked = J.er != nullptr;
    act = live && decided && !noz && !ranked;
    decided = ranked && knn_decided;
    int m2 = 0;
    {
        LEnt2 cur[KU];
        load_step(l2, cur);
        while (__builtin_popcountll(ballot(act)) > coop) {
            if (!act) continue;
            if (m2 > len2) {
                act = false;
                continue;
            }
            seen2 = m2 + KU;
            LEnt2 nxt[KU];
            load_step(l2 + m2 + KU, nxt);
            float dx[KU];
            ln.xdist(cur, dx);
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                cz += cur[u].dz < eps;
                cyz += cur[u].dyz < eps;
                cxz += fmax_(dx[u], cur[u].dz) < eps;
            }
            if (bucket_floor(cur[KU - 1].dz) >= eps) {
                decided = true;
                act = false;
                continue;
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) cur[u] = nxt[u];
            m2 += KU;
        }
    }
    for (uint64_t rest = ballot(act); rest; rest &= rest - 1) {
        const int o = lowest(rest);
        const LEnt2 *pl = bcast(l2, o);
        const int end = bcast(len2, o) + kListPad;
        const float *xt = bcast(ln.xt, o);
        const uint32_t cs = bcast(ln.cs, o), E = bcast(ln.E, o), eo = bcast(ln.e, o);
        const int dxo = bcast(ln.dx, o);
        const float pe = bcast(eps, o);
        float xq[DXM];
#pragma unroll
        for (int c = 0; c < DXM; ++c) xq[c] = bcast(ln.xq[c], o);
        int qz = 0, qyz = 0, qxz = 0;
        bool dec = false;
        int p = bcast(m2, o);
        for (; p < end; p += 64 * kCoopU) {
            const int last = min(p + 64 * kCoopU - 1, end - 1);
            const float stop = bucket_floor(pl[last].dz);
            LEnt2 en[kCoopU];
#pragma unroll
            for (int u = 0; u < kCoopU; ++u) en[u] = pl[min(p + lane + 64 * u, end - 1)];
            float dxv[kCoopU];
#pragma unroll
            for (int u = 0; u < kCoopU; ++u) dxv[u] = coop_xdist(xt, cs, E, eo, dxo, xq, en[u].j);
#pragma unroll
            for (int u = 0; u < kCoopU; ++u) {
                const bool in = p + lane + 64 * u < end;
                qz += __builtin_popcountll(ballot(in && en[u].dz < pe));
                qyz += __builtin_popcountll(ballot(in && en[u].dyz < pe));
                qxz += __builtin_popcountll(ballot(in && fmax_(dxv[u], en[u].dz) < pe));
            }
            if (stop >= pe) {
                dec = true;
                p = last + 1;
                break;
            }
        }
        if (lane == o) {
            cz += qz;
            cyz += qyz;
            cxz += qxz;
            decided = dec;
            seen2 = min(p, end);
        }
    }
    if (noz && live && knn_decided) {
        // Without Z: n_z is the number of rows outside the window; n_y comes
        // from list 1 (its d is d_y, and every row with d_y < eps precedes the
        // k-NN stop); n_x counts the rows j != i with |x_j - x_i| < eps.  The
        // permuted values x_j run over the job's X column, so that count is
        // the range of the sorted column around x_i: the s with
        // -eps < fl(xs[s] - x_i) < eps (fl(. - x_i) is monotone), less row i
        // itself and the rows of its Theiler window.
        const int w = J.theiler;
        cz = n - 1 - min(i, w) - min(n - 1 - i, w);
        for (int m = 0;; ++m) {
            const float d = l1[m].d;
            if (bucket_floor(d) >= eps) break;
            cyz += d < eps;
        }
        const float x = ln.xq[0];
        const float *xs = J.xs;
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (gload(xs, mid) - x > -eps) hi = mid; else lo = mid + 1;
        }
        const int first = lo;
        hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (gload(xs, mid) - x >= eps) hi = mid; else lo = mid + 1;
        }
        cxz = lo - first - (0.f < eps ? 1 : 0);
        for (int j = max(0, i - w); j <= min(n - 1, i + w); ++j)
            if (j != i && absdiff(x, gload(ln.xt, (uint32_t)j * ln.E + ln.e)) < eps) --cxz;
        decided = true;
    }
    if (live) {
        if (ranked) {
            J.er[(int64_t)e * n + i] = decided ? eps : -1.0f;
        }
        if (!decided) {
            const uint32_t pos = atomicAdd(&L.counters[0], 1u);
            L.failq[pos] = ((uint64_t)jb << 40) | ((uint64_t)i * J.n_est + e);
        } else if (!ranked) {
            J.pk[(int64_t)e * n + i] = pack_counts(cxz, cyz, cz);
            if (J.eps) J.eps[(int64_t)e * n + i] = eps;
            if (J.cnt) {
                J.cnt[((int64_t)e * 3 + 0) * n + i] = cxz;
                J.cnt[((int64_t)e * 3 + 1) * n + i] = cyz;
                J.cnt[((int64_t)e * 3 + 2) * n + i] = cz;
            }
        }
        if (L.stats) {
            const int slot = (int)((g >> 6) & (kListStatSlots - 1));
            unsigned long long *st =
                reinterpret_cast<unsigned long long *>(L.counters + kListStatWord + slot * kListStatStride);
            atomicAdd(&st[0], (unsigned long long)seen1);
            atomicAdd(&st[1], (unsigned long long)seen2);
        }
    }
}

// ------------------------------------------------------------------ ranks
// Sets with one Z column: the rows ranked by z (ties by row index).  A block
// takes 64 rows; its four waves count, for those rows, the rows before them
// in a quarter of the set each (z staged in LDS), and the four partial
// ranks are added.
constexpr int kRankThreads = 256;
constexpr int kRankRows = 64;

__global__ __launch_bounds__(kRankThreads) void list_rank_sort_kernel(const ListLaunch L) {
    const ListSet &S = L.sets[__builtin_amdgcn_workgroup_id_y()];
    if (!S.zs) return;
    const int n = S.n;
    const int i0 = (int)bid_x() * kRankRows;
    if (i0 >= n) return;
    const int tid = tid_x(), lane = tid & 63, part = tid >> 6;
    const float *z = S.cols[S.dy];
    __shared__ float t[kRankThreads];
    __shared__ int partial[kRankThreads / 64][kRankRows];
    const int i = i0 + lane;
    const float zi = i < n ? z[i] : 0.f;
    const int span = (n + 3) / 4;
    const int j_lo = part * span, j_hi = min(n, j_lo + span);
    int r = 0;
    // every thread takes part in the staging, so the loop bounds are
    // those of the longest part
    for (int j0 = 0; j0 < span; j0 += 64) {
        __syncthreads();
        const int jj = j_lo + j0 + lane;
        t[tid] = jj < j_hi ? z[jj] : 0.f;
        __syncthreads();
        const int m = min(64, j_hi - (j_lo + j0));
        for (int u = 0; u < m; ++u) {
            const float v = t[part * 64 + u];
            const int j = j_lo + j0 + u;
            r += (v < zi) | ((v == zi) & (j < i));
        }
    }
    partial[part][lane] = r;
    __syncthreads();
    if (part == 0 && i < n) {
        const int rank = partial[0][lane] + partial[1][lane] + partial[2][lane] + partial[3][lane];
        S.zrank[i] = rank;
        S.zord[rank] = i;
        S.zs[rank] = zi;
        S.yr[rank] = S.cols[0][i];
    }
}

// Counts of the pairs of a set with one Z column.  The rows within the
// radius of row i in z are the ranks [lo, hi) with fl(zs[r] - z_i) > -eps
// and fl(zs[r] - z_i) < eps (two binary searches), so n_z = hi - lo, and
// n_yz, n_xz are the rows of that range within eps in y, in x: a wave takes
// 64 pairs (64 ranks, one estimate), finds their ranges lane by lane, then
// counts each pair in turn with all lanes, 64 ranks per step (coalesced
// loads of y and of the estimate's permuted x in rank order, ballot counts).
// The pair's own row and the rows of its Theiler window are taken out
// afterwards.  Same tests as the definition, so the same counts, and every
// pair is decided.
template <int DXM>
__global__ __launch_bounds__(kRankThreads) void list_rank_count_kernel(const ListLaunch L) {
    const int lane = tid_x() & 63;
    const int64_t w = (int64_t)bid_x() * (kRankThreads / 64) +
                      (int)__builtin_amdgcn_readfirstlane((uint32_t)tid_x() >> 6);
    if (w >= L.rank_waves) return;
    const int jb = find_job(L.rank_off, L.n_jobs, w);
    const Job &J = L.jobs[jb];
    const ListSet &S = L.sets[J.set];
    const int n = J.n, dx = J.dx;
    const int nt = (n + 63) / 64;
    const int64_t loc = w - L.rank_off[jb];
    const int e = (int)(loc / nt);
    const int r = (int)(loc - (int64_t)e * nt) * 64 + lane;
    const int rr = min(r, n - 1);
    // (ranks and rows are clamped to the set: inputs that are not finite,
    // which device calls do not check, leave a wrong result, never a fault)
    const int i = min(max(S.zord[rr], 0), n - 1);
    const float eps = J.er[(int64_t)e * n + i];
    const bool ok = r < n && eps >= 0.f;      // -1: the pair is in the redo queue
    const float *zs = S.zs, *yr = S.yr;
    const float *xr = J.xr + (int64_t)e * dx * n;
    const float zq = zs[rr], yq = yr[rr];
    float xq[DXM];
#pragma unroll
    for (int c = 0; c < DXM; ++c) xq[c] = c < dx ? xr[(int64_t)c * n + rr] : 0.f;
    int lo = 0, hi = n;
    {
        int a = 0, b = n;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (zs[m] - zq > -eps) b = m; else a = m + 1;
        }
        lo = a;
        b = n;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (zs[m] - zq >= eps) b = m; else a = m + 1;
        }
        hi = a;
    }
    int mx = 0, my = 0, mz = 0;
    int64_t ent = 0;
    for (uint64_t todo = ballot(ok); todo; todo &= todo - 1) {
        const int o = lowest(todo);
        const int plo = bcast(lo, o), phi = bcast(hi, o), pi = bcast(i, o);
        const float pe = bcast(eps, o), py = bcast(yq, o);
        float px[DXM];
#pragma unroll
        for (int c = 0; c < DXM; ++c) px[c] = bcast(xq[c], o);
        int cx = 0, cy = 0;
        // kRankU steps per iteration, their loads issued together (a pair's
        // steps would otherwise wait for their loads one after another): the
        // network-inference workload ran 3% faster than with one step per
        // iteration; buffer loads over the range (no clamp, a lane mask
        // instead) were 6% slower than either
        constexpr int kRankU = DXM == 1 ? 4 : 1;
        for (int q = plo; q < phi; q += 64 * kRankU) {
            bool in[kRankU];
            uint32_t bo[kRankU];
            float y[kRankU], x0[kRankU];
#pragma unroll
            for (int u = 0; u < kRankU; ++u) {
                const int m = q + 64 * u + lane;
                in[u] = m < phi;
                // byte offsets from the wave-uniform bases: the loads take
                // no 64-bit address arithmetic
                bo[u] = (uint32_t)(in[u] ? m : phi - 1) * 4u;
                y[u] = gload_b(yr, bo[u]);
                x0[u] = gload_b(xr, bo[u]);
            }
#pragma unroll
            for (int u = 0; u < kRankU; ++u) {
                float d = absdiff(x0[u], px[0]);
                Unroll<1, DXM>::upto(dx, [&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    d = fmax_(d, absdiff(gload_b(xr + (int64_t)c * n, bo[u]), px[c]));
                });
                // the masks of single compares, combined by the scalar unit
                const uint64_t inm = cmp_mask(in[u]);
                cy += __builtin_popcountll(inm & cmp_mask(absdiff(y[u], py) < pe));
                cx += __builtin_popcountll(inm & cmp_mask(d < pe));
            }
        }
        int cz = phi - plo;
        // without a Theiler window only the pair's own row is taken out: it
        // is in the range and within eps in y and x exactly when eps > 0
        // (its differences are all 0), else the range is empty
        const int w0 = max(0, pi - J.theiler), w1 = min(n - 1, pi + J.theiler);
        if (J.theiler == 0) {
            const int own = pe > 0.f ? 1 : 0;
            cz -= own;
            cy -= own;
            cx -= own;
        } else
        for (int j = w0 + lane; j - lane <= w1; j += 64) {
            const bool inw = j <= w1;
            const int rj = min(max(S.zrank[inw ? j : w1], 0), n - 1);
            const bool inr = inw && rj >= plo && rj < phi;
            float d = absdiff(xr[rj], px[0]);
            Unroll<1, DXM>::upto(dx, [&](auto cc) {
                constexpr int c = decltype(cc)::value;
                d = fmax_(d, absdiff(xr[(int64_t)c * n + rj], px[c]));
            });
            cz -= __builtin_popcountll(ballot(inr));
            cy -= __builtin_popcountll(ballot(inr && absdiff(yr[rj], py) < pe));
            cx -= __builtin_popcountll(ballot(inr && d < pe));
        }
        ent += phi - plo;
        if (lane == o) {
            mx = cx;
            my = cy;
            mz = cz;
        }
    }
    if (ok) {
        J.pk[(int64_t)e * n + i] = pack_counts(mx, my, mz);
        if (J.eps) J.eps[(int64_t)e * n + i] = eps;
        if (J.cnt) {
            J.cnt[((int64_t)e * 3 + 0) * n + i] = mx;
            J.cnt[((int64_t)e * 3 + 1) * n + i] = my;
            J.cnt[((int64_t)e * 3 + 2) * n + i] = mz;
        }
    }
    if (L.stats && lane == 0) {
        const int slot = (int)(w & (kListStatSlots - 1));
        unsigned long long *st =
            reinterpret_cast<unsigned long long *>(L.counters + kListStatWord + slot * kListStatStride);
        atomicAdd(&st[1], (unsigned long long)ent);
    }
}

// ------------------------------------------------------------------ fallback
// The undecided (row, estimate) pairs, over every other row as in the
// definition: each thread keeps the KMAX smallest distances of its rows, k
// pops of the minimum give the radius, then the threads count and a sum adds
// the counts.  Two shapes, chosen from the queue length (a scalar, so the
// choice is uniform): a few pairs (the usual case, e.g. 244 of 2 million on
// C2) take a whole 1024-thread block each, which keeps the latency of a pair
// short; many pairs (lists short for the data) take one wave each, with no
// block synchronisation, for throughput.
constexpr int kFbBatch = 12;
constexpr int kFbThreads = 1024;
constexpr int kFbWaves = kFbThreads / 64;
constexpr uint32_t kFbBlockModeMax = 2048;   // queue length up to which a pair gets a block

struct FbPair {
    const Job *J;
    int i, e, n, dx, dy, dz;
};

__device__ __forceinline__ FbPair fb_pair(const ListLaunch &L, uint32_t it) {
    const uint64_t item = L.failq[it];
    const int jb = (int)(item >> 40);
    const int64_t r = (int64_t)(item & ((1ull << 40) - 1));
    FbPair p;
    p.J = &L.jobs[jb];
    const int E = p.J->n_est;
    p.i = (int)(r / E);
    p.e = (int)(r - (int64_t)p.i * E);
    p.n = p.J->n;
    p.dx = p.J->dx;
    p.dy = p.J->dy;
    p.dz = p.J->dz;
    return p;
}

// distances of rows j0, j0 + step, ... (kFbBatch of them; rows inside row i's
// Theiler window and rows past the end get +inf in every subspace)
__device__ __forceinline__ void fb_dists(const FbPair &p, int j0, int step, float (&ax)[kFbBatch],
                                         float (&ay)[kFbBatch], float (&az)[kFbBatch]) {
    const Job &J = *p.J;
    int jj[kFbBatch];
#pragma unroll
    for (int u = 0; u < kFbBatch; ++u) {
        const int j = j0 + u * step;
        jj[u] = j < p.n ? j : p.i;
        ax[u] = ay[u] = az[u] = 0.f;
    }
    for (int c = 0; c < p.dx; ++c) {
        // the estimate-major copy: consecutive rows are adjacent words (in the
        // transposed one they are n_est words apart, a page apart in big launches)
        const float *xe = J.xp + ((int64_t)p.e * p.dx + c) * p.n;
        const float q = gload(xe, (uint32_t)p.i);
        float v[kFbBatch];
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) v[u] = gload(xe, (uint32_t)jj[u]);
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) ax[u] = fmax_(ax[u], absdiff(q, v[u]));
    }
    const float *const *yc = J.cols + p.dx;
    for (int c = 0; c < p.dy; ++c) {
        const float q = gload(yc[c], (uint32_t)p.i);
        float v[kFbBatch];
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) v[u] = gload(yc[c], (uint32_t)jj[u]);
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) ay[u] = fmax_(ay[u], absdiff(q, v[u]));
    }
    const float *const *zc = J.cols + p.dx + p.dy;
    for (int c = 0; c < p.dz; ++c) {
        const float q = gload(zc[c], (uint32_t)p.i);
        float v[kFbBatch];
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) v[u] = gload(zc[c], (uint32_t)jj[u]);
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) az[u] = fmax_(az[u], absdiff(q, v[u]));
    }
#pragma unroll
    for (int u = 0; u < kFbBatch; ++u)
        if (abs(jj[u] - p.i) <= J.theiler) ax[u] = ay[u] = az[u] = inf_f();
}

// top-k of this thread's rows j0, j0 + step, ..., and the counts below eps
template <int KMAX>
__device__ __forceinline__ void fb_topk(const FbPair &p, int j0, int step, float (&top)[KMAX]) {
#pragma unroll
    for (int m = 0; m < KMAX; ++m) top[m] = inf_f();
    for (int j = j0; j < p.n; j += step * kFbBatch) {
        float ax[kFbBatch], ay[kFbBatch], az[kFbBatch];
        fb_dists(p, j, step, ax, ay, az);
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) topk_insert<KMAX>(top, fmax_(fmax_(ax[u], ay[u]), az[u]));
    }
}

__device__ __forceinline__ void fb_counts(const FbPair &p, int j0, int step, float eps, int (&c3)[3]) {
    c3[0] = c3[1] = c3[2] = 0;
    for (int j = j0; j < p.n; j += step * kFbBatch) {
        float ax[kFbBatch], ay[kFbBatch], az[kFbBatch];
        fb_dists(p, j, step, ax, ay, az);
#pragma unroll
        for (int u = 0; u < kFbBatch; ++u) {
            c3[0] += fmax_(ax[u], az[u]) < eps;
            c3[1] += fmax_(ay[u], az[u]) < eps;
            c3[2] += az[u] < eps;
        }
    }
}

__device__ __forceinline__ void fb_store(const FbPair &p, float eps, int (&c3)[3]) {
    const Job &J = *p.J;
    const int n = p.n, i = p.i, e = p.e;
    if (p.dz == 0) c3[2] = n - 1 - min(i, J.theiler) - min(n - 1 - i, J.theiler);
    J.pk[(int64_t)e * n + i] = pack_counts(c3[0], c3[1], c3[2]);
    if (J.eps) J.eps[(int64_t)e * n + i] = eps;
    if (J.cnt)
        for (int t = 0; t < 3; ++t) J.cnt[((int64_t)e * 3 + t) * n + i] = c3[t];
}

// k pops of the wave-wide minimum of the threads' sorted lists; the last
// popped value is the wave's k-th smallest
template <int KMAX>
__device__ __forceinline__ float wave_kth(float (&top)[KMAX], int k, float *popped) {
    const int lane = tid_x() & 63;
    float mn = inf_f();
    for (int t = 0; t < k; ++t) {
        mn = wave_min(top[0]);
        const uint64_t bal = __ballot(top[0] == mn);
        if (lane == __builtin_ctzll(bal)) {
#pragma unroll
            for (int m = 0; m < KMAX - 1; ++m) top[m] = top[m + 1];
            top[KMAX - 1] = inf_f();
        }
        if (popped && lane == 0) popped[t] = mn;
    }
    return mn;
}

template <int KMAX>
__global__ __launch_bounds__(kFbThreads) void list_fallback_kernel(const ListLaunch L) {
    __shared__ float wtop[kFbWaves][KMAX];
    __shared__ int wcnt[kFbWaves][3];
    __shared__ float s_eps;
    const int tid = tid_x();
    const int lane = tid & 63;
    // The item count, the wave index and the block index are scalar values,
    // so the item loops and everything derived from an item are uniform and
    // all lanes stay together through the cross-lane steps below.
    const uint32_t total = __builtin_amdgcn_readfirstlane(__atomic_load_n(&L.counters[0], __ATOMIC_RELAXED));
    const int wave = (int)__builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
    if (total <= kFbBlockModeMax) {
        for (uint32_t it = (uint32_t)bid_x(); it < total; it += (uint32_t)L.fb_grid) {
            const FbPair p = fb_pair(L, it);
            float top[KMAX];
            fb_topk<KMAX>(p, tid, kFbThreads, top);
            wave_kth<KMAX>(top, p.J->k, wtop[wave]);
            __syncthreads();
            if (tid == 0) {
                int pos[kFbWaves] = {};
                float kth = inf_f();
                for (int t = 0; t < p.J->k; ++t) {
                    int best = 0;
                    float bv = inf_f();
                    for (int w = 0; w < kFbWaves; ++w)
                        if (pos[w] < p.J->k && wtop[w][pos[w]] < bv) { bv = wtop[w][pos[w]]; best = w; }
                    ++pos[best];
                    kth = bv;
                }
                s_eps = kth;
            }
            __syncthreads();
            const float eps = s_eps;
            int c3[3];
            fb_counts(p, tid, kFbThreads, eps, c3);
            for (int t = 0; t < 3; ++t) c3[t] = wave_sum(c3[t]);
            if (lane == 0) { wcnt[wave][0] = c3[0]; wcnt[wave][1] = c3[1]; wcnt[wave][2] = c3[2]; }
            __syncthreads();
            if (tid == 0) {
                int s3[3] = {0, 0, 0};
                for (int w = 0; w < kFbWaves; ++w)
                    for (int t = 0; t < 3; ++t) s3[t] += wcnt[w][t];
                fb_store(p, eps, s3);
            }
            __syncthreads();
        }
    } else {
        const uint32_t first = (uint32_t)bid_x() * kFbWaves + (uint32_t)wave;
        const uint32_t n_waves = (uint32_t)L.fb_grid * kFbWaves;
        for (uint32_t it = first; it < total; it += n_waves) {
            const FbPair p = fb_pair(L, it);
            float top[KMAX];
            fb_topk<KMAX>(p, lane, 64, top);
            const float eps = wave_kth<KMAX>(top, p.J->k, nullptr);
            int c3[3];
            fb_counts(p, lane, 64, eps, c3);
            for (int t = 0; t < 3; ++t) c3[t] = wave_sum(c3[t]);
            if (lane == 0) fb_store(p, eps, c3);
        }
    }
}

// ------------------------------------------------------------------ reduce
// (H[n_xz] + H[n_yz]) - H[n_z] per row, summed in the all-pairs kernel's order
// so that both paths return the same bits: a 64-row butterfly per chunk, then
// the chunk sums added in index order.  Phase 1: one wave per (estimate,
// chunk), blocks of kWaves chunks of one estimate, sums stored [chunk][estimate];
// phase 2: one thread per estimate adds its chunk sums.
__global__ __launch_bounds__(kBlock) void list_chunk_kernel(const ListLaunch L, const double *__restrict__ harm) {
    const int64_t g = bid_x();
    const int jb = find_job(L.est_off, L.n_jobs, g);
    const Job &J = L.jobs[jb];
    const int e = (int)(g - L.est_off[jb]);
    const int n = J.n, lane = tid_x() & 63;
    const int wave = (int)__builtin_amdgcn_readfirstlane((uint32_t)tid_x() >> 6);
    const int c = (int)__builtin_amdgcn_workgroup_id_y() * kWaves + wave;
    const int nch = (n + kChunk - 1) / kChunk;
    if (c >= nch) return;
    const int i = c * kChunk + lane;
    double v = 0.0;
    if (i < n) {
        const uint64_t w = J.pk[(int64_t)e * n + i];
        v = (harm[w & kPackMask] + harm[(w >> kPackBits) & kPackMask]) - harm[w >> (2 * kPackBits)];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    if (lane == 0) J.chunk[(int64_t)c * J.n_est + e] = v;
}

__global__ __launch_bounds__(kBlock) void list_reduce_kernel(const ListLaunch L, const double *__restrict__ harm) {
    const int64_t g = bid_x() * kBlock + tid_x();
    if (g >= L.ests) return;
    const int jb = find_job(L.est_off, L.n_jobs, g);
    const Job &J = L.jobs[jb];
    const int e = (int)(g - L.est_off[jb]);
    const int n = J.n;
    const int nch = (n + kChunk - 1) / kChunk;
    // chunk sums are [chunk][estimate], so the threads of a wave (consecutive
    // estimates) load adjacent words; added in index order, the loads of 16
    // chunk sums issued before their adds
    const double *part = J.chunk + e;
    const int64_t st = J.n_est;
    constexpr int kU = 16;
    double acc = 0.0;
    int c = 0;
    for (; c + kU <= nch; c += kU) {
        double v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = part[(c + u) * st];
#pragma unroll
        for (int u = 0; u < kU; ++u) acc += v[u];
    }
    for (; c < nch; ++c) acc += part[c * st];
    J.out[e] = harm[J.k - 1] - acc / (double)n;
}

template <int KMAX, int DXM>
void *scan_fn(int step, bool units) {
    if (units)
        return step == 4 ? reinterpret_cast<void *>(&list_scan_kernel<KMAX, DXM, 4, true>)
                         : reinterpret_cast<void *>(&list_scan_kernel<KMAX, DXM, 8, true>);
    return step == 4 ? reinterpret_cast<void *>(&list_scan_kernel<KMAX, DXM, 4, false>)
                     : reinterpret_cast<void *>(&list_scan_kernel<KMAX, DXM, 8, false>);
}

}  // namespace

int launch_list_zy(const ListLaunch &L, void *stream) {
    const int64_t threads = L.rows > kListCounterWords ? L.rows : (int64_t)kListCounterWords;
    hipLaunchKernelGGL(list_zy_kernel, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, L);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_order(const ListLaunch &L, void *stream) {
    if (L.n_jobs <= 1) return 0;
    hipLaunchKernelGGL(list_order_kernel, dim3((unsigned)L.n_sets), dim3(kSortThreads), 0, (hipStream_t)stream, L);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int QB, int... D>
void *lean_fn(int dz, std::integer_sequence<int, D...>) {
    void *fns[] = {nullptr, reinterpret_cast<void *>(&list_build_dz_kernel<D + 1, QB>)...};
    return dz >= 0 && dz <= (int)sizeof...(D) ? fns[dz] : nullptr;
}

int launch_list_build(const ListLaunch &L, void *stream) {
    if (L.build_blocks <= 0) return 0;
    if (L.build_kind == 1) {
        void *fn = L.build_qb == 4 ? lean_fn<4>(L.build_dz, std::make_integer_sequence<int, kBuildFixedDz>{})
                                   : lean_fn<kBuildRows>(L.build_dz, std::make_integer_sequence<int, kBuildFixedDz>{});
        if (!fn) return -1;
        const ListSet *sets = L.sets;
        int n_sets = L.n_sets;
        const int64_t *off = L.build_off;
        void *args[] = {(void *)&sets, (void *)&n_sets, (void *)&off};
        return hipLaunchKernel(fn, dim3((unsigned)L.build_blocks), dim3(kBT), args, 0, (hipStream_t)stream) ==
                       hipSuccess
                   ? 0
                   : -1;
    }
    const dim3 grid((unsigned)L.build_blocks), block(kBT);
    if (L.build_pack && L.build_qb == kBuildRows)
        hipLaunchKernelGGL((list_build_kernel<kBuildRows, kBuildCopies, true>), grid, block, 0,
                           (hipStream_t)stream, L.sets, L.n_sets, L.build_off);
    else if (!L.build_pack && L.build_qb == 1)
        hipLaunchKernelGGL((list_build_kernel<1, 1, false>), grid, block, 0, (hipStream_t)stream, L.sets,
                           L.n_sets, L.build_off);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_scan(const ListLaunch &L, void *stream) {
    if (L.lanes <= 0) return 0;
    const int64_t blocks = L.grouped == 2 ? L.scan_blocks : (L.lanes + kBlock - 1) / kBlock;
    void *fn = nullptr;
    const bool wide = L.dxm > 1;
    const int st = L.scan_step;
    const bool un = L.grouped == 2;
    if (L.kmax == 4) fn = wide ? scan_fn<4, kMaxDx>(st, un) : scan_fn<4, 1>(st, un);
    else if (L.kmax == 8) fn = wide ? scan_fn<8, kMaxDx>(st, un) : scan_fn<8, 1>(st, un);
    else if (L.kmax == 16) fn = wide ? scan_fn<16, kMaxDx>(st, un) : scan_fn<16, 1>(st, un);
    else return -1;
    ListLaunch arg = L;
    void *args[] = {(void *)&arg};
    return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(kBlock), args, 0, (hipStream_t)stream) == hipSuccess
               ? 0
               : -1;
}

int launch_list_rank_sort(const ListLaunch &L, void *stream) {
    if (L.rank_sets <= 0) return 0;
    const dim3 grid((unsigned)((L.max_rank_n + kRankRows - 1) / kRankRows), (unsigned)L.n_sets);
    hipLaunchKernelGGL(list_rank_sort_kernel, grid, dim3(kRankThreads), 0, (hipStream_t)stream, L);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_rank_count(const ListLaunch &L, void *stream) {
    if (L.rank_waves <= 0) return 0;
    const int64_t blocks = (L.rank_waves + kRankThreads / 64 - 1) / (kRankThreads / 64);
    if (L.dxm > 1)
        hipLaunchKernelGGL(list_rank_count_kernel<kMaxDx>, dim3((unsigned)blocks), dim3(kRankThreads), 0,
                           (hipStream_t)stream, L);
    else
        hipLaunchKernelGGL(list_rank_count_kernel<1>, dim3((unsigned)blocks), dim3(kRankThreads), 0,
                           (hipStream_t)stream, L);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_fallback(const ListLaunch &L, void *stream) {
    if (L.lanes <= 0) return 0;
    const dim3 grid((unsigned)L.fb_grid), block(kFbThreads);
    if (L.kmax == 4) hipLaunchKernelGGL(list_fallback_kernel<4>, grid, block, 0, (hipStream_t)stream, L);
    else if (L.kmax == 8) hipLaunchKernelGGL(list_fallback_kernel<8>, grid, block, 0, (hipStream_t)stream, L);
    else if (L.kmax == 16) hipLaunchKernelGGL(list_fallback_kernel<16>, grid, block, 0, (hipStream_t)stream, L);
    else return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_sortx(const ListLaunch &L, void *stream) {
    if (L.n_jobs <= 0) return 0;
    hipLaunchKernelGGL(list_sortx_kernel, dim3((unsigned)L.n_jobs), dim3(kSortThreads), 0, (hipStream_t)stream, L);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_list_reduce(const ListLaunch &L, const double *harm, void *stream) {
    if (L.ests <= 0 || L.max_chunks <= 0) return 0;
    const dim3 grid1((unsigned)L.ests, (unsigned)((L.max_chunks + kWaves - 1) / kWaves));
    hipLaunchKernelGGL(list_chunk_kernel, grid1, dim3(kBlock), 0, (hipStream_t)stream, L, harm);
    hipLaunchKernelGGL(list_reduce_kernel, dim3((unsigned)((L.ests + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, L, harm);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mte
