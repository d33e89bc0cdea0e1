/*
 * Oracle: direct O(N^2) summation of the extended Gaussian ANOVA kernel
 * product, in plain C with OpenMP, float64 throughout.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code with the HIP path.
 *
 * What it computes (the plain definitions, written out):
 *   kernel   kappa(x_i, x_j) = sum_l eta_l exp(-||x_i^{W_l} - x_j^{W_l}||^2 / ell^2)
 *            (Sec. 3, eq. extended_Gaussian_ANOVA_kernel; the Gaussian uses
 *            sigma^2 in the denominator with no factor 1/2, Sec. 3; the
 *            weighted sum over windows is the combined kernel of Sec. 5)
 *   product  (K alpha)_i = sum_j alpha_j kappa(x_i, x_j)   (Sec. 2, eq. mult_with_K)
 *   shifted  ((K + beta I) alpha)_i = (K alpha)_i + beta alpha_i
 *            (Sec. 2: the regularised normal equation (K + lambda I) alpha = y)
 *   predict  s(z_i) = sum_j alpha_j kappa(z_i, x_j) for new points z_i and the
 *            training points x_j (Sec. 4.2, eq. kernelsum with two node sets;
 *            Sec. 4.3 evaluates the trained model this way)
 * The diagonal term j = i is included (the kernel has no singularity).
 *
 * Summation: for each output row the sum over j is taken in consecutive
 * blocks of 256 terms, and the block sums are added in order; this keeps the
 * oracle's own rounding near 1e-15 relative for N up to a few million.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_BLOCK 256

/* Window description: win_dA[l] in {1,2,3}; win_feat[3*l + t] feature index.
 * kappa(a, b) for two feature vectors a and b. */
static double anova_kernel_pair(const double *a, const double *b,
                                const int32_t *win_feat, const int32_t *win_dA,
                                const double *eta, int32_t P, double inv_ell2)
{
    double k = 0.0;
    for (int32_t l = 0; l < P; ++l) {
        double r2 = 0.0;
        for (int32_t t = 0; t < win_dA[l]; ++t) {
            int32_t f = win_feat[3 * l + t];
            double diff = a[f] - b[f];
            r2 += diff * diff;
        }
        k += eta[l] * exp(-r2 * inv_ell2);
    }
    return k;
}

static double anova_kernel_entry(const double *X, int64_t ldx, int64_t i, int64_t j,
                                 const int32_t *win_feat, const int32_t *win_dA,
                                 const double *eta, int32_t P, double inv_ell2)
{
    return anova_kernel_pair(X + i * ldx, X + j * ldx, win_feat, win_dA, eta, P, inv_ell2);
}

/*
 * out[c*nrows + r] = beta*alpha[c*lda + i] + sum_j kappa(x_i, x_j) alpha[c*lda + j]
 * for i = rows[r] (r < nrows), c < nrhs.  If rows == NULL, rows are 0..N-1.
 * X: N x d row-major with leading dimension ldx.  alpha: column-major, lda.
 * Returns the number of threads used.
 */
int oracle_anova_matvec(const double *X, int64_t N, int64_t ldx,
                        const int32_t *win_feat, const int32_t *win_dA,
                        const double *eta, int32_t P, double ell, double beta,
                        const double *alpha, int32_t nrhs, int64_t lda,
                        const int64_t *rows, int64_t nrows, double *out)
{
    const double inv_ell2 = 1.0 / (ell * ell);
    int nthreads = 1;
    if (rows == NULL) nrows = N;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        double *acc = (double *)malloc(sizeof(double) * (size_t)nrhs * 2);
        double *blk = acc + nrhs;
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            for (int32_t c = 0; c < nrhs; ++c) acc[c] = 0.0;
            for (int64_t j0 = 0; j0 < N; j0 += ORACLE_BLOCK) {
                int64_t j1 = j0 + ORACLE_BLOCK < N ? j0 + ORACLE_BLOCK : N;
                for (int32_t c = 0; c < nrhs; ++c) blk[c] = 0.0;
                for (int64_t j = j0; j < j1; ++j) {
                    double k = anova_kernel_entry(X, ldx, i, j, win_feat, win_dA, eta, P, inv_ell2);
                    for (int32_t c = 0; c < nrhs; ++c) blk[c] += k * alpha[c * lda + j];
                }
                for (int32_t c = 0; c < nrhs; ++c) acc[c] += blk[c];
            }
            for (int32_t c = 0; c < nrhs; ++c)
                out[(int64_t)c * nrows + r] = acc[c] + beta * alpha[c * lda + i];
        }
        free(acc);
    }
    return nthreads;
}

/*
 * Prediction: out[c*nrows + r] = sum_j kappa(z_i, x_j) alpha[c*lda + j] for
 * i = rows[r] (r < nrows; rows == NULL: i = r, nrows = Nz), c < nrhs.
 * Z: Nz x d row-major (ldz), X: N x d row-major (ldx), alpha: N x nrhs
 * column-major (lda).  Blocked summation over j as in the product above.
 * Returns the number of threads used.
 */
int oracle_anova_predict(const double *Z, int64_t Nz, int64_t ldz,
                         const double *X, int64_t N, int64_t ldx,
                         const int32_t *win_feat, const int32_t *win_dA,
                         const double *eta, int32_t P, double ell,
                         const double *alpha, int32_t nrhs, int64_t lda,
                         const int64_t *rows, int64_t nrows, double *out)
{
    const double inv_ell2 = 1.0 / (ell * ell);
    int nthreads = 1;
    if (rows == NULL) nrows = Nz;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        double *acc = (double *)malloc(sizeof(double) * (size_t)nrhs * 2);
        double *blk = acc + nrhs;
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            for (int32_t c = 0; c < nrhs; ++c) acc[c] = 0.0;
            for (int64_t j0 = 0; j0 < N; j0 += ORACLE_BLOCK) {
                int64_t j1 = j0 + ORACLE_BLOCK < N ? j0 + ORACLE_BLOCK : N;
                for (int32_t c = 0; c < nrhs; ++c) blk[c] = 0.0;
                for (int64_t j = j0; j < j1; ++j) {
                    double k = anova_kernel_pair(Z + i * ldz, X + j * ldx, win_feat, win_dA,
                                                 eta, P, inv_ell2);
                    for (int32_t c = 0; c < nrhs; ++c) blk[c] += k * alpha[c * lda + j];
                }
                for (int32_t c = 0; c < nrhs; ++c) acc[c] += blk[c];
            }
            for (int32_t c = 0; c < nrhs; ++c) out[(int64_t)c * nrows + r] = acc[c];
        }
        free(acc);
    }
    (void)Nz;
    return nthreads;
}

/*
 * Dense kernel block: out[a*ncols + b] = kappa(x_{ri[a]}, x_{cj[b]}).
 * Used for small matrices (eigenvalue checks, direct solves, column tests).
 */
void oracle_kernel_block(const double *X, int64_t ldx,
                         const int32_t *win_feat, const int32_t *win_dA,
                         const double *eta, int32_t P, double ell,
                         const int64_t *ri, int64_t nrows, const int64_t *cj, int64_t ncols,
                         double *out)
{
    const double inv_ell2 = 1.0 / (ell * ell);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nrows; ++a)
        for (int64_t b = 0; b < ncols; ++b)
            out[a * ncols + b] = anova_kernel_entry(X, ldx, ri[a], cj[b], win_feat, win_dA,
                                                    eta, P, inv_ell2);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (the host-baseline timing reports a
 * one-thread figure beside the all-threads one). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
