/*
 * ORACLE — test infrastructure only. Nothing in the product library links,
 * loads or calls this file; only tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.
 *
 * Direct FP64 evaluation of the ANOVA Gaussian kernel sum (Section 3, the
 * "extended Gaussian ANOVA kernel" and the component form of K v):
 *
 *   y_j = sum_{l=1..P} eta_l * sum_{i=1..N} exp( -||x_j^{W_l} - x_i^{W_l}||^2 / sigma_l^2 ) * v_i
 *
 * for every requested target row j. Differences are formed explicitly (no
 * |a|^2 + |b|^2 - 2 a.b expansion) and the self term i = j is included.
 * Plain double loops; OpenMP only splits target rows between threads.
 *
 * X: N x d row-major. win: P x 3 feature indices, -1 = unused slot.
 * V: N x R column-major (V[i + r*N]). rows: target indices (NULL = 0..N-1).
 * Y: nrows x R column-major.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

int oracle_anova_direct(const double* X, int64_t N, int32_t d,
                        const int32_t* win, int32_t P,
                        const double* sigma, const double* eta,
                        const double* V, int32_t R,
                        const int64_t* rows, int64_t nrows,
                        double* Y)
{
    if (R < 1 || R > 256) return 1;
    int64_t total = rows ? nrows : N;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t jj = 0; jj < total; ++jj) {
        int64_t j = rows ? rows[jj] : jj;
        double acc[256];
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int l = 0; l < P; ++l) {
            double inv_s2 = 1.0 / (sigma[l] * sigma[l]);
            for (int64_t i = 0; i < N; ++i) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    int f = win[3 * l + a];
                    if (f < 0) continue;
                    double diff = X[j * d + f] - X[i * d + f];
                    s += diff * diff;
                }
                double k = eta[l] * exp(-s * inv_s2);
                for (int r = 0; r < R; ++r) acc[r] += k * V[i + (int64_t)r * N];
            }
        }
        for (int r = 0; r < R; ++r) Y[jj + (int64_t)r * total] = acc[r];
    }
    return 0;
}

/* Kernel columns K[:, p] for the requested source indices p (Section 3 kernel,
 * same definition as above): out is N x ncols column-major. */
int oracle_anova_columns(const double* X, int64_t N, int32_t d,
                         const int32_t* win, int32_t P,
                         const double* sigma, const double* eta,
                         const int64_t* cols, int64_t ncols, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t c = 0; c < ncols; ++c) {
            int64_t p = cols[c];
            double acc = 0.0;
            for (int l = 0; l < P; ++l) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    int f = win[3 * l + a];
                    if (f < 0) continue;
                    double diff = X[i * d + f] - X[p * d + f];
                    s += diff * diff;
                }
                acc += eta[l] * exp(-s / (sigma[l] * sigma[l]));
            }
            out[i + c * N] = acc;
        }
    }
    return 0;
}
