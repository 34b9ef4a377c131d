// Gaussian estimator kernels (gfx950): the float64 covariance of a set of
// columns and, from it, I(X;Y|Z) of many (X, Y, Z) index sets.
//
//   colsum   per row chunk and column (one wave), the float64 sum of the
//            chunk's rows (lane-strided partial sums, then a fixed butterfly),
//            then per column the mean of the chunk sums (the same pattern);
//   gram     per row chunk and 64x64 tile of the upper triangle, the centered
//            cross products sum_r (a_r - mean_a)(b_r - mean_b) in float64 on the
//            matrix cores, 4-row groups in order;
//   reduce   per entry, the chunk partials summed in chunk order, / N.
//
// The chunking depends on N only and every entry is one fixed sequence of
// operations on its two columns, so an entry has the same bits in any
// covariance matrix that contains both columns (an estimate from a small
// matrix equals the same estimate taken from a large one).
//
//   cmi      one wave per estimate: Cholesky (outer-product form) of the
//            submatrix ordered (Z, X, Y), then of (Z, Y); the Schur pivots of
//            the Y block give ln det Sigma_{Y|XZ} and ln det Sigma_{Y|Z}.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gauss.h"

namespace mte {

namespace {

constexpr int kThreads = 256;
constexpr int kRB = kGaussRowStage;

__device__ __forceinline__ int tid_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int bid_x() { return (int)__builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ int bid_y() { return (int)__builtin_amdgcn_workgroup_id_y(); }

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per (row chunk, column): lane l keeps four partial sums over the
// rows r0 + l + 64 (4m + u), u = 0..3 (four loads in flight per lane), adds
// them as (s0 + s1) + (s2 + s3), and a fixed butterfly sums the lanes.
__global__ __launch_bounds__(64) void gauss_colsum_kernel(GaussCov a) {
    const int lane = tid_x();
    const int c = bid_x(), col = bid_y();
    const int r0 = c * a.chunk_rows;
    const int r1 = min(a.n, r0 + a.chunk_rows);
    const float *p = a.cols[col];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int r = r0 + lane;
    for (; r + 192 < r1; r += 256) {
        const float v0 = p[r], v1 = p[r + 64], v2 = p[r + 128], v3 = p[r + 192];
        s[0] += (double)v0;
        s[1] += (double)v1;
        s[2] += (double)v2;
        s[3] += (double)v3;
    }
    if (r < r1) s[0] += (double)p[r];
    if (r + 64 < r1) s[1] += (double)p[r + 64];
    if (r + 128 < r1) s[2] += (double)p[r + 128];
    double t = wave_sum_f64((s[0] + s[1]) + (s[2] + s[3]));
    if (lane == 0) a.part_mean[(int64_t)c * a.D + col] = t;
}

// Column means from the chunk sums: one wave per column, lane l adds the
// chunks l, l+64, ... in order, a fixed butterfly adds the lanes.
__global__ __launch_bounds__(64) void gauss_mean_kernel(GaussCov a) {
    const int lane = tid_x(), col = bid_x();
    double s = 0.0;
    for (int h = lane; h < a.n_chunks; h += 64) s += a.part_mean[(int64_t)h * a.D + col];
    s = wave_sum_f64(s);
    if (lane == 0) a.mean[col] = s / (double)a.n;
}

// Upper-triangle tile pair y -> (tp, tq), tp <= tq.
constexpr int kXcds = 8;   // accelerator complex dies (one L2 each) of an MI355X

__device__ __forceinline__ void tile_pair(int y, int n_tiles, int *tp, int *tq) {
    int p = 0;
    while (y >= n_tiles - p) {
        y -= n_tiles - p;
        ++p;
    }
    *tp = p;
    *tq = p + y;
}

// Matrix-core Gram tile.  A block computes one 64x64 tile of the upper
// triangle over its row chunk; wave w computes the 32x32 quarter
// (32 (w & 1), 32 (w >> 1)) as 2x2 blocks of v_mfma_f64_16x16x4f64: for every
// group of 4 rows, D[m][n] += sum_k A[m][k] B[k][n] with A[m][k] the centered
// value of column p0+m at row k and B[k][n] that of column q0+n.  Operand
// layout: lane l supplies row k = l/16 of column l%16; the 4 results of lane
// l are D[l/16 + 4v][l%16], v = 0..3 (checked on the device).  Tiles are
// staged column-major in LDS, 33 doubles per column: the 16 columns one
// operand load touches per row start 66 dwords apart, so each group of 16
// lanes covers the 32 banks once (no bank conflicts in the counters; a
// 34-double stride conflicted), and the staging stores are consecutive.  Every
// entry sees the same sequence of 4-row groups in the same order whatever the
// tile, so its bits do not depend on the other columns.  On gfx950 the fp64
// matrix rate equals the fp64 vector rate (78.6 TFLOP/s); the matrix cores
// need 4x fewer LDS reads per fma than a 4x4 vector register tile.
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void gauss_gram_kernel(GaussCov a) {
    constexpr int T = 64;
    constexpr int LDC = kRB + 1;      // column stride in LDS (doubles)
    __shared__ double mu[2][T];
    __shared__ __align__(16) double As[T][LDC];
    __shared__ __align__(16) double Bs[T][LDC];
    const int tid = tid_x();
    // One block per (row chunk, tile pair), numbered chunk-major.  With
    // several tile pairs, the blocks, which the hardware deals to the XCDs in
    // turn, are renumbered so that each XCD takes a contiguous range, i.e. all
    // tile pairs of its chunks together: they read the same rows of the same
    // columns step by step, so a column tile comes from HBM about once per
    // chunk instead of once per pair.
    const int pairs = a.n_tiles * (a.n_tiles + 1) / 2;
    int b = bid_x();
    if (pairs > 1) {
        const int nb = (int)(__builtin_amdgcn_grid_size_x() / kThreads), hb = b;
        const int q = nb / kXcds, rem = nb % kXcds, x = hb % kXcds;
        b = x * q + min(x, rem) + hb / kXcds;
    }
    const int c = b / pairs;
    int tp, tq;
    tile_pair(b - c * pairs, a.n_tiles, &tp, &tq);
    const int p0 = tp * T, q0 = tq * T;
    const int r0 = c * a.chunk_rows;
    const int r1 = min(a.n, r0 + a.chunk_rows);
    if (tid < 2 * T) {
        const int col = (tid < T ? p0 : q0 - T) + tid;
        mu[tid / T][tid % T] = col < a.D ? a.mean[col] : 0.0;
    }
    const int lane = tid & 63, w = tid >> 6;
    const int pw = (w & 1) * 32, qw = (w >> 1) * 32;
    const int kk = lane >> 4, cc = lane & 15;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    // Staging: element m of this thread is row (tid + 256 m) % 32 of tile
    // column (tid + 256 m) / 32.  The next step's values are loaded into
    // registers while the matrix cores work on the current one.
    constexpr int M = kRB * T / kThreads;
    const int sr = tid % kRB;
    const float *pa[M], *pb[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int col = tid / kRB + m * (kThreads / kRB);
        pa[m] = p0 + col < a.D ? a.cols[p0 + col] : nullptr;
        pb[m] = q0 + col < a.D ? a.cols[q0 + col] : nullptr;
    }
    float na[M], nb[M];
    auto fetch = [&](int rs) {
        const int row = rs + sr;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            na[m] = (pa[m] && row < r1) ? pa[m][row] : 0.0f;
            nb[m] = (pb[m] && row < r1) ? pb[m][row] : 0.0f;
        }
    };
    fetch(r0);
    for (int rs = r0; rs < r1; rs += kRB) {
        __syncthreads();
        const bool in = rs + sr < r1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int col = tid / kRB + m * (kThreads / kRB);
            As[col][sr] = (pa[m] && in) ? (double)na[m] - mu[0][col] : 0.0;
            Bs[col][sr] = (pb[m] && in) ? (double)nb[m] - mu[1][col] : 0.0;
        }
        __syncthreads();
        if (rs + kRB < r1) fetch(rs + kRB);
#pragma unroll
        for (int g = 0; g < kRB / 4; ++g) {
            const int rr = 4 * g + kk;
            const double a0 = As[pw + cc][rr], a1 = As[pw + 16 + cc][rr];
            const double b0 = Bs[qw + cc][rr], b1 = Bs[qw + 16 + cc][rr];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    double *out = a.part + (int64_t)c * a.D * a.D;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = q0 + qw + 16 * j + cc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = p0 + pw + 16 * i + kk + 4 * v;
                if (p < a.D && q < a.D) out[(int64_t)p * a.D + q] = acc[i][j][v];
            }
        }
}

__global__ __launch_bounds__(kThreads) void gauss_cov_reduce_kernel(GaussCov a) {
    const int64_t e = (int64_t)bid_x() * kThreads + tid_x();
    if (e >= (int64_t)a.D * a.D) return;
    const int p = (int)(e / a.D), q = (int)(e % a.D);
    if (p > q) return;
    double s = 0.0;
    for (int h = 0; h < a.n_chunks; ++h) s += a.part[(int64_t)h * a.D * a.D + e];
    s /= (double)a.n;
    a.cov[(int64_t)p * a.D + q] = s;
    a.cov[(int64_t)q * a.D + p] = s;
}

// One wave per estimate.  Outer-product Cholesky: at step k the pivot is
// the Schur complement diagonal d_k, and column j > k (owned by lane j) is
// updated below its diagonal by A[i][j] -= A[i][k] * (A[j][k] / d_k).  Only
// column k (rows >= k) is read at step k and it is not written then, so one
// barrier per step suffices.  ln det of a leading block = sum of ln d_k.
__global__ __launch_bounds__(64) void gauss_cmi_kernel(GaussJobs a) {
    __shared__ double A[kGaussMaxVars][kGaussMaxVars + 1];
    __shared__ int32_t ix[kGaussMaxVars];
    const int lane = tid_x();
    const int jb = bid_x();
    const GaussJob J = a.jobs[jb];
    double ylog[2] = {0.0, 0.0};
    int bad = 0;
    for (int f = 0; f < 2 && !bad; ++f) {
        // f = 0: (Z, X, Y); f = 1: (Z, Y)
        const int m = f == 0 ? J.dz + J.dx + J.dy : J.dz + J.dy;
        const int ybeg = m - J.dy;
        __syncthreads();
        if (lane < m) ix[lane] = a.idx[J.off + ((f == 1 && lane >= J.dz) ? lane + J.dx : lane)];
        __syncthreads();
        if (lane < m) {
            const int64_t cj = ix[lane];
            for (int i = 0; i < m; ++i) A[i][lane] = a.cov[(int64_t)ix[i] * a.D + cj];
        }
        __syncthreads();
        double acc = 0.0;
        for (int k = 0; k < m; ++k) {
            const double d = A[k][k];
            if (!(d > 0.0)) {
                bad = 1;
                break;
            }
            if (k >= ybeg) acc += log(d);
            if (lane > k && lane < m) {
                const double t = A[lane][k] / d;
                for (int i = lane; i < m; ++i) A[i][lane] -= A[i][k] * t;
            }
            __syncthreads();
        }
        ylog[f] = acc;
    }
    if (lane == 0) {
        a.out[jb] = bad ? 0.0 : 0.5 * (ylog[1] - ylog[0]);
        a.status[jb] = bad;
    }
}

}  // namespace

GaussChunks gauss_chunks(int64_t n) {
    int64_t rows = (n + kGaussMaxChunks - 1) / kGaussMaxChunks;
    if (rows < 64) rows = 64;
    rows = (rows + kRB - 1) / kRB * kRB;
    return GaussChunks{(int)rows, (int)((n + rows - 1) / rows)};
}

int launch_gauss_colsum(const GaussCov &a, hipStream_t s) {
    if (a.D < 1 || a.n < 1) return 0;
    hipLaunchKernelGGL(gauss_colsum_kernel, dim3((unsigned)a.n_chunks, (unsigned)a.D), dim3(64), 0, s, a);
    hipLaunchKernelGGL(gauss_mean_kernel, dim3((unsigned)a.D), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gauss_gram(const GaussCov &a, hipStream_t s) {
    if (a.D < 1 || a.n < 1) return 0;
    if (a.tile != 64) return -1;
    const int64_t blocks = (int64_t)a.n_chunks * (a.n_tiles * (a.n_tiles + 1) / 2);
    hipLaunchKernelGGL(gauss_gram_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gauss_cov_reduce(const GaussCov &a, hipStream_t s) {
    if (a.D < 1 || a.n < 1) return 0;
    const int64_t entries = (int64_t)a.D * a.D;
    hipLaunchKernelGGL(gauss_cov_reduce_kernel, dim3((unsigned)((entries + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gauss_cmi(const GaussJobs &a, hipStream_t s) {
    if (a.n_jobs < 1) return 0;
    hipLaunchKernelGGL(gauss_cmi_kernel, dim3((unsigned)a.n_jobs), dim3(64), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mte
