// All-pairs KSG estimate for jobs with few estimates (gfx950).
//
// A job with one to a few estimates has too little work per query row for the
// persistent kernel's register blocks: at N = 10^4 and one estimate its items
// cover the chip only when the reference rows are split, and the split radii
// and counts are then merged serially.  Here one wave takes QP consecutive
// query rows and G estimates (their coordinates are wave-uniform) and its 64
// lanes stride over the reference rows, so no step crosses waves:
//   pass 1  each lane keeps the KMAX smallest joint distances of its rows for
//           every (query, estimate); the k-th smallest of the wave's lists is
//           k pops of the wave-wide minimum (with multiplicity, as in the
//           definition);
//   pass 2  each lane counts its rows strictly below the radius in the (X,Z),
//           (Y,Z) and Z subspaces; wave sums give the counts.
// The counts go out as the per-row packed word of the list path, whose
// fixed-order reduction kernels give the digamma sums; the results are the
// same bits as on every other path.  Pairs inside the Theiler window
// (|i - j| <= w, the row itself when w = 0) are left out.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "engine.h"
#include "ksg_device.h"

namespace mte {

namespace {

using dev::absdiff;
using dev::count_lt;
using dev::find_job;
using dev::fmax_;
using dev::inf_f;
using dev::topk_insert;
using dev::Unroll;

constexpr int kSoloBlock = 256;   // 4 waves, one (job, group, query tile) each
constexpr int kSoloU = 2;         // reference rows per lane per step (4 held more registers: slower)

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

// Row j (0 <= j < n) of a column: a uniform base plus a 32-bit byte offset,
// the form a global load takes with no 64-bit address arithmetic (an int
// index is sign-extended and added in 64 bits per load).
__device__ __forceinline__ float lload(const float *p, int j) {
    using gchar = const __attribute__((address_space(1))) char;
    return *(const __attribute__((address_space(1))) float *)((gchar *)p + (uint32_t)j * 4u);
}

// Wave-uniform values moved to scalar registers (the compiler cannot prove a
// load uniform when the kernel also stores to global memory).
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ const float *uni(const float *p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    return reinterpret_cast<const float *>(((uint64_t)hi << 32) | lo);
}

// Calls f(integral_constant<c>) for the columns c < lim: all FZ of them when
// FZ >= 0 (compiled dimensions: straight-line code, so the max chains fuse
// into three-operand maxima), else through the run-time guard chain.
template <int FZ, int CAP, class F>
__device__ __forceinline__ void cols(int lim, F &&f) {
    if constexpr (FZ >= 0) {
        (void)lim;
        Unroll<0, (FZ < CAP ? FZ : CAP)>::upto(FZ, f);
    } else {
        Unroll<0, CAP>::upto(lim, f);
    }
}

// FZ >= 0: compiled dimensions, FZ Z columns, one Y and one X column.
template <int KMAX, int G, int QP, int DZM, int DYM, int DXM, int FZ>
__global__ __launch_bounds__(kSoloBlock) void ksg_solo_kernel(const Job *__restrict__ jobs, int n_jobs,
                                                              const int64_t *__restrict__ wave_off,
                                                              int64_t total_waves) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wv = (int64_t)blockIdx.x * (kSoloBlock / 64) +
                       (int64_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wv >= total_waves) return;
    const int jb = find_job(wave_off, n_jobs, wv);
    const Job &J = jobs[jb];
    const int64_t local = wv - wave_off[jb];
    const int n = J.n, nqt = (n + QP - 1) / QP;
    const int g = (int)(local / nqt), i0 = (int)(local - (int64_t)g * nqt) * QP;
    const int e0 = g * G, gc = min(G, J.n_est - e0);
    const int dx = FZ >= 0 ? 1 : J.dx, dy = FZ >= 0 ? 1 : J.dy, dz = FZ >= 0 ? FZ : J.dz, w = J.theiler, k = J.k;
    // the columns, the estimates' permuted X columns and the tile's query
    // coordinates, all wave-uniform
    const float *zcol[DZM], *ycol[DYM], *xe[G][DXM];
    cols<FZ, DZM>(dz, [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        zcol[c] = uni(J.cols[dx + dy + c]);
    });
    cols<(FZ >= 0 ? 1 : -1), DYM>(dy, [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        ycol[c] = uni(J.cols[dx + c]);
    });
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        const int e = e0 + min(gg, gc - 1);
        cols<(FZ >= 0 ? 1 : -1), DXM>(dx, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            // a job whose estimates are all the identity reads X in place
            xe[gg][c] = uni(J.xp ? J.xp + ((int64_t)e * dx + c) * n : J.cols[c]);
        });
    }
    float qz[QP][DZM], qy[QP][DYM], qx[G][QP][DXM];
#pragma unroll
    for (int q = 0; q < QP; ++q) {
        const int i = min(i0 + q, n - 1);
        cols<FZ, DZM>(dz, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            qz[q][c] = uni(zcol[c][i]);
        });
        cols<(FZ >= 0 ? 1 : -1), DYM>(dy, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            qy[q][c] = uni(ycol[c][i]);
        });
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
            cols<(FZ >= 0 ? 1 : -1), DXM>(dx, [&](auto cc) {
                constexpr int c = decltype(cc)::value;
                qx[gg][q][c] = uni(xe[gg][c][i]);
            });
    }

    // d_z, d_yz of the tile's rows against this lane's rows j[u] (+inf for
    // rows past the end and inside a row's window), then the X part per estimate
    // a step needs the mask only when its rows reach past the end or into
    // the window of one of the tile's rows (a wave-uniform test)
    auto edge = [&](int j0) { return j0 + 64 * kSoloU > n || (j0 + 64 * kSoloU > i0 - w && j0 <= i0 + QP - 1 + w); };
    auto dists = [&](const int (&jj)[kSoloU], bool masked, float (&az)[QP][kSoloU], float (&ayz)[QP][kSoloU],
                     float (&ad)[G][QP][kSoloU]) {
        int jl[kSoloU];
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) jl[u] = jj[u] < n ? jj[u] : n - 1;
        float rz[DZM][kSoloU], ry[DYM][kSoloU], rx[G][DXM][kSoloU];
        cols<FZ, DZM>(dz, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int u = 0; u < kSoloU; ++u) rz[c][u] = lload(zcol[c], jl[u]);
        });
        cols<(FZ >= 0 ? 1 : -1), DYM>(dy, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int u = 0; u < kSoloU; ++u) ry[c][u] = lload(ycol[c], jl[u]);
        });
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
            cols<(FZ >= 0 ? 1 : -1), DXM>(dx, [&](auto cc) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) rx[gg][c][u] = lload(xe[gg][c], jl[u]);
            });
#pragma unroll
        for (int q = 0; q < QP; ++q)
#pragma unroll
            for (int u = 0; u < kSoloU; ++u) {
                float a = 0.f;
                cols<FZ, DZM>(dz, [&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    a = fmax_(a, absdiff(qz[q][c], rz[c][u]));
                });
                float b = a;
                cols<(FZ >= 0 ? 1 : -1), DYM>(dy, [&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    b = fmax_(b, absdiff(qy[q][c], ry[c][u]));
                });
                // |j - i| <= w  <=>  (unsigned)(j - i + w) <= 2w; j >= n: out
                const bool kill =
                    masked && (jj[u] >= n || (uint32_t)(jj[u] - (i0 + q) + w) <= 2u * (uint32_t)w);
                az[q][u] = kill ? inf_f() : a;
                ayz[q][u] = kill ? inf_f() : b;
            }
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) {
                    float d = 0.f;
                    cols<(FZ >= 0 ? 1 : -1), DXM>(dx, [&](auto cc) {
                        constexpr int c = decltype(cc)::value;
                        d = fmax_(d, absdiff(qx[gg][q][c], rx[gg][c][u]));
                    });
                    ad[gg][q][u] = d;
                }
    };

    // pass 1: each lane's KMAX smallest joint distances per (estimate, query)
    float top[G][QP][KMAX];
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
        for (int q = 0; q < QP; ++q)
#pragma unroll
            for (int m = 0; m < KMAX; ++m) top[gg][q][m] = inf_f();
    for (int j0 = 0; j0 < n; j0 += 64 * kSoloU) {
        int jj[kSoloU];
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) jj[u] = j0 + u * 64 + lane;
        float az[QP][kSoloU], ayz[QP][kSoloU], ad[G][QP][kSoloU];
        if (edge(j0)) dists(jj, true, az, ayz, ad);
        else dists(jj, false, az, ayz, ad);
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                float d[kSoloU], lo = inf_f();
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) {
                    d[u] = fmax_(ad[gg][q][u], ayz[q][u]);
                    lo = __builtin_fminf(lo, d[u]);
                }
                if (lo < top[gg][q][KMAX - 1]) {
#pragma unroll
                    for (int u = 0; u < kSoloU; ++u) topk_insert<KMAX>(top[gg][q], d[u]);
                }
            }
    }
    // radii: the k-th smallest of the wave's lists, k pops of the wave minimum
    float eps[G][QP];
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
        for (int q = 0; q < QP; ++q) {
            float mn = inf_f();
            for (int t = 0; t < k; ++t) {
                mn = wave_min(top[gg][q][0]);
                const uint64_t b = __ballot(top[gg][q][0] == mn);
                if (lane == __builtin_ctzll(b)) {
#pragma unroll
                    for (int m = 0; m < KMAX - 1; ++m) top[gg][q][m] = top[gg][q][m + 1];
                    top[gg][q][KMAX - 1] = inf_f();
                }
            }
            eps[gg][q] = mn;
        }

    // pass 2: strict counts below the radii
    int cxz[G][QP], cyz[G][QP], cz[G][QP];
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
        for (int q = 0; q < QP; ++q) cxz[gg][q] = cyz[gg][q] = cz[gg][q] = 0;
    for (int j0 = 0; j0 < n; j0 += 64 * kSoloU) {
        int jj[kSoloU];
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) jj[u] = j0 + u * 64 + lane;
        float az[QP][kSoloU], ayz[QP][kSoloU], ad[G][QP][kSoloU];
        if (edge(j0)) dists(jj, true, az, ayz, ad);
        else dists(jj, false, az, ayz, ad);
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) {
                    count_lt(cz[gg][q], az[q][u], eps[gg][q]);
                    count_lt(cyz[gg][q], ayz[q][u], eps[gg][q]);
                    count_lt(cxz[gg][q], fmax_(ad[gg][q][u], az[q][u]), eps[gg][q]);
                }
    }
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
        for (int q = 0; q < QP; ++q) {
            const int i = i0 + q;
            int a = wave_sum(cxz[gg][q]), b = wave_sum(cyz[gg][q]), c = wave_sum(cz[gg][q]);
            // without Z every row outside the window counts in n_z
            if (dz == 0) c = n - 1 - min(i, w) - min(n - 1 - i, w);
            if (lane == 0 && gg < gc && i < n) {
                const int e = e0 + gg;
                J.pk[(int64_t)e * n + i] = (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)b << kPackBits) |
                                           ((uint64_t)(uint32_t)c << (2 * kPackBits));
                if (J.diag_eps) J.diag_eps[(int64_t)e * n + i] = eps[gg][q];
                if (J.diag_cnt) {
                    J.diag_cnt[((int64_t)e * 3 + 0) * n + i] = a;
                    J.diag_cnt[((int64_t)e * 3 + 1) * n + i] = b;
                    J.diag_cnt[((int64_t)e * 3 + 2) * n + i] = c;
                }
            }
        }
}

struct SoloEntry {
    SoloCfg cfg;
    const void *fn;
};

#define MTE_SOLO(K, Z, Y, X, G, Q) \
    {{K, Z, Y, X, G, Q, -1}, reinterpret_cast<const void *>(&ksg_solo_kernel<K, G, Q, Z, Y, X, -1>)},
#define MTE_SOLO_K(K)                                                                                     \
    MTE_SOLO(K, 8, 1, 1, 1, 4) MTE_SOLO(K, 8, 1, 1, 4, 1) MTE_SOLO(K, 8, 1, 1, 8, 1)                      \
        MTE_SOLO(K, 32, 1, 1, 1, 2) MTE_SOLO(K, 32, 1, 1, 8, 1) MTE_SOLO(K, 32, 8, 16, 1, 1)
// compiled dimensions: k <= 4, one estimate, dz = FZ, one Y and one X column
#define MTE_SOLO_F(FZ) \
    {{4, (FZ > 0 ? FZ : 1), 1, 1, 1, 4, FZ}, \
     reinterpret_cast<const void *>(&ksg_solo_kernel<4, 1, 4, (FZ > 0 ? FZ : 1), 1, 1, FZ>)},

const SoloEntry kSolo[] = {MTE_SOLO_K(4) MTE_SOLO_K(8) MTE_SOLO_K(16) MTE_SOLO_F(0) MTE_SOLO_F(1) MTE_SOLO_F(2)
                           MTE_SOLO_F(3) MTE_SOLO_F(4) MTE_SOLO_F(5) MTE_SOLO_F(6) MTE_SOLO_F(7) MTE_SOLO_F(8)
                           MTE_SOLO_F(9) MTE_SOLO_F(10) MTE_SOLO_F(11) MTE_SOLO_F(12)};

}  // namespace

int solo_variant_count() { return (int)(sizeof(kSolo) / sizeof(kSolo[0])); }

bool solo_variant(int i, SoloCfg *cfg) {
    if (i < 0 || i >= solo_variant_count()) return false;
    *cfg = kSolo[i].cfg;
    return true;
}

int launch_solo(int v, const Job *jobs_dev, int n_jobs, const int64_t *wave_off, int64_t total_waves,
                void *stream) {
    if (total_waves <= 0) return 0;
    if (v < 0 || v >= solo_variant_count()) return -1;
    const int64_t blocks = (total_waves + kSoloBlock / 64 - 1) / (kSoloBlock / 64);
    void *args[] = {(void *)&jobs_dev, (void *)&n_jobs, (void *)&wave_off, (void *)&total_waves};
    return hipLaunchKernel(kSolo[v].fn, dim3((unsigned)blocks), dim3(kSoloBlock), args, 0, (hipStream_t)stream) ==
                   hipSuccess
               ? 0
               : -1;
}

}  // namespace mte
