/*
 * Plain C brute-force KSG conditional mutual information.
 * TEST INFRASTRUCTURE ONLY: used by the tests (cross-check of the numpy
 * oracle, sampled parity at full size) and by the benchmark's CPU baseline.
 * The product library never links or calls it.
 *
 * It computes exactly what oracle/ksg.py computes (the estimator the paper
 * cites in its CLM section, written out there), by the same definition:
 *   d(i,j) = max over all columns of |fl32(a_i - a_j)| (subspace maxima for
 *   the counts), eps_i = k-th smallest d(i,j) over the rows j outside row i's
 *   Theiler window |i - j| <= w (w = 0: j != i), strict counts over the same rows
 *   n_xz, n_yz, n_z, and I = psi(k) - mean_i[psi(n_xz+1)+psi(n_yz+1)-psi(n_z+1)]
 *   with psi(m+1) + gamma = H_m, the harmonic number, so that
 *   I = H_{k-1} - (1/N) sum_i (H_{n_xz} + H_{n_yz} - H_{n_z}).
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math, so
 * every float operation is one IEEE binary32 operation).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static float group_dist(const float *cols, int d, long n, long i, long j)
{
    float m = 0.0f;
    for (int c = 0; c < d; ++c) {
        float t = cols[(long)c * n + i] - cols[(long)c * n + j];
        t = fabsf(t);
        if (t > m) m = t;
    }
    return m;
}

/* eps and strict counts for one query i. */
static void one_query(const float *X, int dx, const float *Y, int dy,
                      const float *Z, int dz, long n, int k, long w, long i,
                      float *top, float *eps, int *nxz, int *nyz, int *nz)
{
    for (int m = 0; m < k; ++m) top[m] = INFINITY;
    for (long j = 0; j < n; ++j) {
        if (labs(j - i) <= w) continue;
        float a = group_dist(X, dx, n, i, j);
        float b = group_dist(Y, dy, n, i, j);
        float c = group_dist(Z, dz, n, i, j);
        float d = a > b ? a : b;
        d = d > c ? d : c;
        if (d < top[k - 1]) {           /* insertion into the sorted k smallest */
            int m = k - 1;
            while (m > 0 && top[m - 1] > d) { top[m] = top[m - 1]; --m; }
            top[m] = d;
        }
    }
    float e = top[k - 1];
    int cx = 0, cy = 0, cz = 0, valid = 0;
    for (long j = 0; j < n; ++j) {
        if (labs(j - i) <= w) continue;
        ++valid;
        float a = group_dist(X, dx, n, i, j);
        float b = group_dist(Y, dy, n, i, j);
        float c = group_dist(Z, dz, n, i, j);
        float ac = a > c ? a : c;
        float bc = b > c ? b : c;
        if (ac < e) ++cx;
        if (bc < e) ++cy;
        if (c < e) ++cz;
    }
    if (dz == 0) cz = valid;
    *eps = e; *nxz = cx; *nyz = cy; *nz = cz;
}

/*
 * X, Y, Z: column-major sample matrices [d][n] (Z may be NULL when dz == 0);
 * theiler: Theiler window w >= 0.
 * queries: NULL for all rows (then *cmi_out is written), else nq row indices.
 * Outputs per query: eps, nxz, nyz, nz.  Returns 0, or -1 on bad arguments.
 */
int oracle_ksg(const float *X, int dx, const float *Y, int dy, const float *Z, int dz,
               long n, int k, int theiler, int nthreads, const long *queries, long nq,
               float *eps, int *nxz, int *nyz, int *nz, double *cmi_out)
{
    if (!X || !Y || dx < 1 || dy < 1 || dz < 0 || (dz > 0 && !Z) || k < 1 || theiler < 0 ||
        n < k + 1 + 2 * (long)theiler)
        return -1;
    long total = queries ? nq : n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        float *top = (float *)malloc(sizeof(float) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
        for (long q = 0; q < total; ++q) {
            long i = queries ? queries[q] : q;
            one_query(X, dx, Y, dy, Z, dz, n, k, theiler, i, top, &eps[q], &nxz[q], &nyz[q], &nz[q]);
        }
        free(top);
    }
    if (!queries && cmi_out) {
        double *h = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        h[0] = 0.0;
        for (long m = 1; m <= n; ++m) h[m] = h[m - 1] + 1.0 / (double)m;
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += (h[nxz[i]] + h[nyz[i]]) - h[nz[i]];
        *cmi_out = h[k - 1] - s / (double)n;
        free(h);
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
