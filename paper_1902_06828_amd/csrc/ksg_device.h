// Device code of the KSG conditional-mutual-information kernel (gfx950).
//
// The estimator (named by citation in the paper's CLM section) needs, for
// every estimate and every row i, the k-th smallest max-norm distance eps_i to
// the other rows in the joint (X,Y,Z) space and three strict neighbour counts
// below eps_i in the (X,Z), (Y,Z) and Z subspaces; the CMI is then a digamma
// sum over the counts.  Max-norm distances are maxima of |fl32(a-b)|: there is
// no multiply-add, so this is FP32 VALU work (sub, max with the |.| source
// modifier, med3/min for the top-k, compare + carry-add for the counts), not a
// dense contraction for the matrix cores.
//
// Structure (one persistent launch per batch of jobs, see engine.h):
//  * block = 4 wave64; each lane owns QP query rows and up to G estimates, a
//    register block of QP x G (row, estimate) pairs;
//  * reference rows stream through LDS in tiles (coalesced column loads); all
//    lanes read the same reference, so LDS reads are broadcasts;
//  * the Y,Z part of a pair's distance is the same for every estimate of a job
//    (only X is permuted) and is computed once per pair per lane for all the
//    lane's estimates;
//  * the top-k is a sorted register list updated with med3, entered only when
//    some lane has a new neighbour among the 8 references of a step;
//  * counts are exact int32; the digamma sum uses a float64 harmonic table and
//    a fixed-order reduction (64-row butterfly, then chunks in index order), so
//    results do not depend on tiling, splitting or batching.
// Column counts are runtime values below compile-time capacities; the guards
// are wave-uniform branches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "engine.h"

namespace mte {
namespace dev {

constexpr int kSteps = 8;                    // references per inner step
constexpr int kTileBytes = 32768;            // LDS bytes of one reference tile
constexpr uint32_t kSpinLimit = 1u << 26;    // bounded wait (seconds)

__device__ __forceinline__ float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float fmin_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float absdiff(float a, float b) { return __builtin_fabsf(a - b); }
__device__ __forceinline__ float inf_f() { return __builtin_inff(); }

// c += (a < b): the compare writes VCC and the carry-in add consumes it right
// away.  Written as one ALU-only asm pair because the compiler otherwise
// hoists all compares of a step and spills their 64-bit masks.
__device__ __forceinline__ void count_lt(int &c, float a, float b) {
    asm("v_cmp_lt_f32_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, 0, %0, vcc"
        : "+v"(c)
        : "v"(a), "v"(b)
        : "vcc");
}

// Insert d into the ascending list t[0..K-1], dropping the largest entry.
template <int K>
__device__ __forceinline__ void topk_insert(float (&t)[K], float d) {
#pragma unroll
    for (int m = K - 1; m >= 1; --m) t[m] = __builtin_amdgcn_fmed3f(t[m - 1], d, t[m]);
    t[0] = fmin_(t[0], d);
}

// Calls f(integral_constant<I>) for I = FIRST .. min(lim, N)-1 as a straight
// chain of wave-uniform early exits, so every register index stays static.
template <int I, int N>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void upto(int lim, F &&f) {
        if constexpr (I < N) {
            if (I >= lim) return;
            f(std::integral_constant<int, I>{});
            Unroll<I + 1, N>::upto(lim, f);
        }
    }
};

__device__ __forceinline__ void lds8(const float *p, float (&v)[kSteps]) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

template <int KMAX, int G, int QP, int DZM, int DYM, int DXM>
struct Tile {
    static constexpr int QT = kWaves * 64 * QP;           // query rows per item
    static constexpr int COLS = DZM + DYM + G * DXM;
    static constexpr int RT0 = (kTileBytes / (COLS * 4)) / 64 * 64;
    static constexpr int RT = RT0 > 512 ? 512 : (RT0 < 64 ? 64 : RT0);
};

template <int KMAX, int G, int QP, int DZM, int DYM, int DXM>
struct Smem {
    float rz[DZM][Tile<KMAX, G, QP, DZM, DYM, DXM>::RT];
    float ry[DYM][Tile<KMAX, G, QP, DZM, DYM, DXM>::RT];
    float rx[G][DXM][Tile<KMAX, G, QP, DZM, DYM, DXM>::RT];
    const float *col[kMaxCols];
    double red[G * 64];                    // chunk sums staged by the final reduction
    int item;
    int flag;
};

__device__ __forceinline__ int find_job(const int64_t *off, int n_jobs, int64_t x) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int KMAX, int G, int QP, int DZM, int DYM, int DXM>
struct Worker {
    using T = Tile<KMAX, G, QP, DZM, DYM, DXM>;
    using S = Smem<KMAX, G, QP, DZM, DYM, DXM>;
    static constexpr int RT = T::RT;
    static constexpr int QT = T::QT;

    const Job &J;
    S &sm;
    const double *__restrict__ harm;
    uint32_t *__restrict__ err;
    int g, t, gc, dx, dy, dz, n, w, lane, wave, tid;

    __device__ Worker(const Job &j, S &s, const double *h, uint32_t *e, int g_, int t_)
        : J(j), sm(s), harm(h), err(e), g(g_), t(t_) {
        n = J.n;
        dx = J.dx;
        dz = J.dz;
        dy = J.dy;
        w = J.theiler;
        gc = min(G, J.n_est - g * G);
        tid = threadIdx.x;
        lane = tid & 63;
        wave = tid >> 6;
    }

    __device__ __forceinline__ int qrow(int q) const {
        return t * QT + wave * 64 * QP + q * 64 + lane;
    }

    __device__ __forceinline__ const float *zcol(int c) const { return sm.col[dx + J.dy + c]; }
    __device__ __forceinline__ const float *ycol(int c) const { return sm.col[dx + c]; }

    __device__ void load_cols() {
        if (tid < kMaxCols) sm.col[tid] = tid < J.dx + J.dy + J.dz ? J.cols[tid] : nullptr;
        __syncthreads();
    }

    __device__ void load_queries(float (&qz)[QP][DZM], float (&qy)[QP][DYM], float (&qx)[G][QP][DXM]) {
#pragma unroll
        for (int q = 0; q < QP; ++q) {
            const int i = min(qrow(q), n - 1);
#pragma unroll
            for (int c = 0; c < DZM; ++c) qz[q][c] = c < dz ? zcol(c)[i] : 0.f;
#pragma unroll
            for (int c = 0; c < DYM; ++c) qy[q][c] = c < dy ? ycol(c)[i] : 0.f;
#pragma unroll
            for (int gg = 0; gg < G; ++gg) {
                const int e = g * G + min(gg, gc - 1);
#pragma unroll
                for (int c = 0; c < DXM; ++c)
                    qx[gg][q][c] = c < dx ? J.xp[((int64_t)e * dx + c) * n + i] : 0.f;
            }
        }
    }

    // Reference rows [base, base+len) into LDS (zeros past len).
    __device__ void load_tile(int base, int len) {
        __syncthreads();
        for (int idx = tid; idx < dz * RT; idx += kBlock) {
            const int c = idx / RT, jj = idx - c * RT;
            sm.rz[c][jj] = jj < len ? zcol(c)[base + jj] : 0.f;
        }
        for (int idx = tid; idx < dy * RT; idx += kBlock) {
            const int c = idx / RT, jj = idx - c * RT;
            sm.ry[c][jj] = jj < len ? ycol(c)[base + jj] : 0.f;
        }
        const int xcols = gc * dx;
        for (int idx = tid; idx < xcols * RT; idx += kBlock) {
            const int gcol = idx / RT, jj = idx - gcol * RT;
            const int gg = gcol / dx, c = gcol - gg * dx;
            sm.rx[gg][c][jj] = jj < len ? J.xp[((int64_t)(g * G + gg) * dx + c) * n + base + jj] : 0.f;
        }
        __syncthreads();
    }

    // Max-norm over the Z columns (HASZ: dz > 0) into az, then over the Y
    // columns on top of it into ayz, for QP queries x kSteps references.
    template <bool HASZ>
    __device__ __forceinline__ void zy_dist(const float (&qz)[QP][DZM], const float (&qy)[QP][DYM], int st,
                                            float (&az)[QP][kSteps], float (&ayz)[QP][kSteps]) {
        float rv[kSteps];
        if (HASZ) {
            lds8(&sm.rz[0][st], rv);
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) az[q][r] = absdiff(qz[q][0], rv[r]);
            Unroll<1, DZM>::upto(dz, [&](auto cc) {
                constexpr int c = decltype(cc)::value;
                float rc[kSteps];
                lds8(&sm.rz[c][st], rc);
#pragma unroll
                for (int q = 0; q < QP; ++q)
#pragma unroll
                    for (int r = 0; r < kSteps; ++r) az[q][r] = fmax_(az[q][r], absdiff(qz[q][c], rc[r]));
            });
            lds8(&sm.ry[0][st], rv);
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) ayz[q][r] = fmax_(az[q][r], absdiff(qy[q][0], rv[r]));
        } else {
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) az[q][r] = 0.f;
            lds8(&sm.ry[0][st], rv);
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) ayz[q][r] = absdiff(qy[q][0], rv[r]);
        }
        Unroll<1, DYM>::upto(dy, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            float rc[kSteps];
            lds8(&sm.ry[c][st], rc);
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) ayz[q][r] = fmax_(ayz[q][r], absdiff(qy[q][c], rc[r]));
        });
    }

    // Pairs inside the Theiler window |i - j| <= w (self pairs when w = 0) and
    // references at or past `hi` get distance +inf.
    template <bool BOTH>
    __device__ __forceinline__ void mask(int j0, int hi, float (&az)[QP][kSteps], float (&ayz)[QP][kSteps]) {
        const int qlo = t * QT;
        const bool diag = j0 < qlo + QT + w && j0 + kSteps + w > qlo;
        const bool pad = j0 + kSteps > hi;
        if (!(diag || pad)) return;
#pragma unroll
        for (int q = 0; q < QP; ++q) {
            const int rel = qrow(q) - j0;
#pragma unroll
            for (int r = 0; r < kSteps; ++r) {
                const bool kill = ((unsigned)(rel - r + w) <= (unsigned)(2 * w)) || (j0 + r >= hi);
                if (BOTH) az[q][r] = kill ? inf_f() : az[q][r];
                ayz[q][r] = kill ? inf_f() : ayz[q][r];
            }
        }
    }

    // X part of the distance for estimate gg: d = max(base, max_c |qx - rx|).
    template <int gg>
    __device__ __forceinline__ void xdist(int st, const float (&qx)[G][QP][DXM],
                                          const float (&base)[QP][kSteps], float (&d)[QP][kSteps]) {
        float xr[kSteps];
        lds8(&sm.rx[gg][0][st], xr);
#pragma unroll
        for (int q = 0; q < QP; ++q)
#pragma unroll
            for (int r = 0; r < kSteps; ++r) d[q][r] = fmax_(base[q][r], absdiff(qx[gg][q][0], xr[r]));
        Unroll<1, DXM>::upto(dx, [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            float xc[kSteps];
            lds8(&sm.rx[gg][c][st], xc);
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int r = 0; r < kSteps; ++r) d[q][r] = fmax_(d[q][r], absdiff(qx[gg][q][c], xc[r]));
        });
    }

    // k-NN pass over references [lo, hi): top[g][q] holds the k smallest
    // distances (ascending, -inf padded in front when k < KMAX).
    template <bool HASZ>
    __device__ void knn(int lo, int hi, const float (&qz)[QP][DZM], const float (&qy)[QP][DYM],
                        const float (&qx)[G][QP][DXM], float (&top)[G][QP][KMAX]) {
        const float ninf = -inf_f();
        const int pad_front = KMAX - J.k;
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q)
#pragma unroll
                for (int m = 0; m < KMAX; ++m) top[gg][q][m] = m < pad_front ? ninf : inf_f();
        for (int base = lo; base < hi; base += RT) {
            const int len = min(RT, hi - base);
            load_tile(base, len);
            for (int st = 0; st < len; st += kSteps) {
                float az[QP][kSteps], ayz[QP][kSteps];
                zy_dist<HASZ>(qz, qy, st, az, ayz);
                mask<false>(base + st, hi, az, ayz);
                Unroll<0, G>::upto(gc, [&](auto gi) {
                    constexpr int gg = decltype(gi)::value;
                    float d[QP][kSteps];
                    xdist<gg>(st, qx, ayz, d);
#pragma unroll
                    for (int q = 0; q < QP; ++q) {
                        const float m = fmin_(fmin_(fmin_(d[q][0], d[q][1]), fmin_(d[q][2], d[q][3])),
                                              fmin_(fmin_(d[q][4], d[q][5]), fmin_(d[q][6], d[q][7])));
                        if (m < top[gg][q][KMAX - 1]) {
#pragma unroll
                            for (int r = 0; r < kSteps; ++r) topk_insert<KMAX>(top[gg][q], d[q][r]);
                        }
                    }
                });
            }
        }
    }

    // Count pass over references [lo, hi).
    template <bool HASZ>
    __device__ void count(int lo, int hi, const float (&qz)[QP][DZM], const float (&qy)[QP][DYM],
                          const float (&qx)[G][QP][DXM], const float (&eps)[G][QP], int (&cxz)[G][QP],
                          int (&cyz)[G][QP], int (&cz)[G][QP]) {
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) cxz[gg][q] = cyz[gg][q] = cz[gg][q] = 0;
        for (int base = lo; base < hi; base += RT) {
            const int len = min(RT, hi - base);
            load_tile(base, len);
            for (int st = 0; st < len; st += kSteps) {
                float az[QP][kSteps], ayz[QP][kSteps];
                zy_dist<HASZ>(qz, qy, st, az, ayz);
                mask<true>(base + st, hi, az, ayz);
                Unroll<0, G>::upto(gc, [&](auto gi) {
                    constexpr int gg = decltype(gi)::value;
                    float dxz[QP][kSteps];
                    xdist<gg>(st, qx, az, dxz);
#pragma unroll
                    for (int q = 0; q < QP; ++q) {
                        const float e = eps[gg][q];
#pragma unroll
                        for (int r = 0; r < kSteps; ++r) {
                            count_lt(cxz[gg][q], dxz[q][r], e);
                            count_lt(cyz[gg][q], ayz[q][r], e);
                            if (HASZ) count_lt(cz[gg][q], az[q][r], e);
                        }
                    }
                });
            }
        }
    }

    __device__ void knn_any(int lo, int hi, const float (&qz)[QP][DZM], const float (&qy)[QP][DYM],
                            const float (&qx)[G][QP][DXM], float (&top)[G][QP][KMAX]) {
        if (dz > 0) knn<true>(lo, hi, qz, qy, qx, top);
        else knn<false>(lo, hi, qz, qy, qx, top);
    }

    __device__ void count_any(int lo, int hi, const float (&qz)[QP][DZM], const float (&qy)[QP][DYM],
                              const float (&qx)[G][QP][DXM], const float (&eps)[G][QP], int (&cxz)[G][QP],
                              int (&cyz)[G][QP], int (&cz)[G][QP]) {
        if (dz > 0) count<true>(lo, hi, qz, qy, qx, eps, cxz, cyz, cz);
        else count<false>(lo, hi, qz, qy, qx, eps, cxz, cyz, cz);
    }

    // Fixed-order partial sums of (H[n_xz] + H[n_yz]) - H[n_z] per 64 rows,
    // then the tile ticket and, for the last tile of the group, the result.
    __device__ void finish(const int (&cxz)[G][QP], const int (&cyz)[G][QP], const int (&cz)[G][QP]) {
        const int nch = (n + kChunk - 1) / kChunk;
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            if (gg >= gc) continue;
            const int e = g * G + gg;
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = qrow(q);
                // without Z, n_z is the number of rows outside the window
                const int nz = dz == 0 ? n - 1 - min(i, w) - min(n - 1 - i, w) : cz[gg][q];
                double v = 0.0;
                if (i < n) {
                    v = (harm[cxz[gg][q]] + harm[cyz[gg][q]]) - harm[nz];
                    if (J.diag_cnt) {
                        J.diag_cnt[((int64_t)e * 3 + 0) * n + i] = cxz[gg][q];
                        J.diag_cnt[((int64_t)e * 3 + 1) * n + i] = cyz[gg][q];
                        J.diag_cnt[((int64_t)e * 3 + 2) * n + i] = nz;
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
                const int ch = (t * QT + wave * 64 * QP + q * 64) / kChunk;
                if (lane == 0 && ch < nch) J.chunk[(int64_t)e * nch + ch] = v;
            }
        }
        __threadfence();
        __syncthreads();
        const int64_t gt = (int64_t)J.n_groups * J.n_tiles;
        if (tid == 0) {
            const uint32_t old = atomicAdd(&J.sync[3 * gt + g], 1u);
            sm.flag = old == (uint32_t)(J.n_tiles - 1);
        }
        __syncthreads();
        if (!sm.flag) return;
        __threadfence();
        // last tile of this group: sum each estimate's chunks in index order
        double acc = 0.0;
        for (int c0 = 0; c0 < nch; c0 += 64) {
            const int m = min(64, nch - c0);
            __syncthreads();
            for (int idx = tid; idx < gc * 64; idx += kBlock) {
                const int gg = idx / 64, c = idx % 64;
                sm.red[idx] = c < m ? __builtin_nontemporal_load(&J.chunk[(int64_t)(g * G + gg) * nch + c0 + c]) : 0.0;
            }
            __syncthreads();
            if (tid < gc)
                for (int c = 0; c < m; ++c) acc += sm.red[tid * 64 + c];
        }
        if (tid < gc) J.out[g * G + tid] = harm[J.k - 1] - acc / (double)n;
    }

    // ---- item bodies
    __device__ void fused() {
        float qz[QP][DZM], qy[QP][DYM], qx[G][QP][DXM];
        load_queries(qz, qy, qx);
        float eps[G][QP];
        {
            float top[G][QP][KMAX];
            knn_any(0, n, qz, qy, qx, top);
#pragma unroll
            for (int gg = 0; gg < G; ++gg)
#pragma unroll
                for (int q = 0; q < QP; ++q) eps[gg][q] = top[gg][q][KMAX - 1];
        }
        if (J.diag_eps) {
#pragma unroll
            for (int gg = 0; gg < G; ++gg)
#pragma unroll
                for (int q = 0; q < QP; ++q)
                    if (gg < gc && qrow(q) < n) J.diag_eps[(int64_t)(g * G + gg) * n + qrow(q)] = eps[gg][q];
        }
        int cxz[G][QP], cyz[G][QP], cz[G][QP];
        count_any(0, n, qz, qy, qx, eps, cxz, cyz, cz);
        finish(cxz, cyz, cz);
    }

    __device__ void knn_split(int r) {
        float qz[QP][DZM], qy[QP][DYM], qx[G][QP][DXM];
        load_queries(qz, qy, qx);
        const int lo = r * J.split_len, hi = min(n, lo + J.split_len);
        float top[G][QP][KMAX];
        knn_any(lo, hi, qz, qy, qx, top);
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = qrow(q);
                if (gg < gc && i < n) {
                    float *p = J.part + (((int64_t)r * J.n_est + g * G + gg) * n + i) * KMAX;
#pragma unroll
                    for (int m = 0; m < KMAX; ++m) p[m] = top[gg][q][m];
                }
            }
        __threadfence();
        __syncthreads();
        const int64_t slot = (int64_t)g * J.n_tiles + t;
        if (tid == 0) sm.flag = atomicAdd(&J.sync[slot], 1u) == (uint32_t)(J.rs - 1);
        __syncthreads();
        if (!sm.flag) return;
        __threadfence();
        // last split of this (group, tile): merge the partial lists into eps
        const float ninf = -inf_f();
        const int pad_front = KMAX - J.k;
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = qrow(q);
                if (gg < gc && i < n) {
                    float m_[KMAX];
#pragma unroll
                    for (int m = 0; m < KMAX; ++m) m_[m] = m < pad_front ? ninf : inf_f();
                    for (int rr = 0; rr < J.rs; ++rr) {
                        const float *p = J.part + (((int64_t)rr * J.n_est + g * G + gg) * n + i) * KMAX;
#pragma unroll
                        for (int m = 0; m < KMAX; ++m)
                            if (m >= pad_front) topk_insert<KMAX>(m_, __builtin_nontemporal_load(&p[m]));
                    }
                    const int64_t o = (int64_t)(g * G + gg) * n + i;
                    J.eps[o] = m_[KMAX - 1];
                    if (J.diag_eps) J.diag_eps[o] = m_[KMAX - 1];
                }
            }
        __threadfence();
        __syncthreads();
        if (tid == 0) atomicExch(&J.sync[(int64_t)J.n_groups * J.n_tiles + slot], 1u);
    }

    __device__ void count_split(int r) {
        const int64_t gt = (int64_t)J.n_groups * J.n_tiles;
        const int64_t slot = (int64_t)g * J.n_tiles + t;
        if (tid == 0) {
            uint32_t spins = 0;
            sm.flag = 1;
            while (__hip_atomic_load(&J.sync[gt + slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                __builtin_amdgcn_s_sleep(8);
                if (++spins > kSpinLimit) {
                    sm.flag = 0;
                    atomicExch(err, 1u);
                    break;
                }
            }
        }
        __syncthreads();
        if (!sm.flag) return;
        __threadfence();
        float qz[QP][DZM], qy[QP][DYM], qx[G][QP][DXM];
        load_queries(qz, qy, qx);
        float eps[G][QP];
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = min(qrow(q), n - 1);
                const int e = g * G + min(gg, gc - 1);
                eps[gg][q] = __builtin_nontemporal_load(&J.eps[(int64_t)e * n + i]);
            }
        const int lo = r * J.split_len, hi = min(n, lo + J.split_len);
        int cxz[G][QP], cyz[G][QP], cz[G][QP];
        count_any(lo, hi, qz, qy, qx, eps, cxz, cyz, cz);
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = qrow(q);
                if (gg < gc && i < n) {
                    int32_t *p = J.cnt + (((int64_t)r * J.n_est + g * G + gg) * 3) * n + i;
                    p[0] = cxz[gg][q];
                    p[n] = cyz[gg][q];
                    p[2 * (int64_t)n] = cz[gg][q];
                }
            }
        __threadfence();
        __syncthreads();
        if (tid == 0) sm.flag = atomicAdd(&J.sync[2 * gt + slot], 1u) == (uint32_t)(J.rs - 1);
        __syncthreads();
        if (!sm.flag) return;
        __threadfence();
        // last split: total counts, then the digamma partial sums
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int i = min(qrow(q), n - 1);
                const int e = g * G + min(gg, gc - 1);
                int a = 0, b = 0, c = 0;
                for (int rr = 0; rr < J.rs; ++rr) {
                    const int32_t *p = J.cnt + (((int64_t)rr * J.n_est + e) * 3) * n + i;
                    a += __builtin_nontemporal_load(&p[0]);
                    b += __builtin_nontemporal_load(&p[n]);
                    c += __builtin_nontemporal_load(&p[2 * (int64_t)n]);
                }
                cxz[gg][q] = a;
                cyz[gg][q] = b;
                cz[gg][q] = c;
            }
        finish(cxz, cyz, cz);
    }
};

template <int KMAX, int G, int QP, int DZM, int DYM, int DXM>
__global__ __launch_bounds__(kBlock) void ksg_kernel(const Job *__restrict__ jobs, int n_jobs,
                                                     const int64_t *__restrict__ a_off,
                                                     const int64_t *__restrict__ b_off,
                                                     int64_t items_a, int64_t items_b,
                                                     uint32_t *__restrict__ work,
                                                     const double *__restrict__ harm) {
    using W = Worker<KMAX, G, QP, DZM, DYM, DXM>;
    __shared__ Smem<KMAX, G, QP, DZM, DYM, DXM> sm;
    const int64_t total = items_a + items_b;
    for (;;) {
        if (threadIdx.x == 0) sm.item = (int)atomicAdd(&work[0], 1u);
        __syncthreads();
        const int64_t it = (uint32_t)sm.item;
        __syncthreads();
        if (it >= total) break;
        int phase, j;
        int64_t local;
        if (it < items_a) {
            phase = 0;
            j = find_job(a_off, n_jobs, it);
            local = it - a_off[j];
        } else {
            phase = 1;
            j = find_job(b_off, n_jobs, it - items_a);
            local = it - items_a - b_off[j];
        }
        const Job &J = jobs[j];
        const int r = (int)(local % J.rs);
        const int t = (int)((local / J.rs) % J.n_tiles);
        const int g = (int)(local / ((int64_t)J.rs * J.n_tiles));
        W w(J, sm, harm, work + 1, g, t);
        w.load_cols();
        if (phase == 1) w.count_split(r);
        else if (J.rs == 1) w.fused();
        else w.knn_split(r);
        __syncthreads();
    }
}

struct VariantEntry {
    TileCfg cfg;
    const void *fn;
};

}  // namespace dev
}  // namespace mte

#define MTE_VARIANT_ENTRY(K, G, Q, Z, Y, X) \
    {{K, G, Q, Z, Y, X}, reinterpret_cast<const void *>(&::mte::dev::ksg_kernel<K, G, Q, Z, Y, X>)},
