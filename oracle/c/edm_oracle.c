/*
 * CPU oracle for the lower-triangular Euclidean distance map, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the HIP library includes or links
 * this file; it is loaded by the test suite and timed as the CPU baseline.
 *
 * Double-precision loops that restate the definitions:
 *   D_ij = sqrt( sum_k (a_i^k - a_j^k)^2 ),  0 <= j <= i < N
 * (the per-pair function of Sec. IV, Eq. (17)), and its gradient
 *   dL/dx_i = sum_{j<i} g_ij (x_i - x_j)/D_ij - sum_{k>i} g_ki (x_k - x_i)/D_ki
 * with a term taken as 0 where D = 0.  OpenMP splits the outer loop over
 * rows (points); each row is computed exactly as in the serial loop, so the
 * result does not depend on the thread count.  Built -O2 without fast-math.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double pair_dist(const float *X, int64_t ldx, int32_t d, int64_t i, int64_t j)
{
    double s = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = (double)X[i * ldx + k] - (double)X[j * ldx + k];
        s += t * t;
    }
    return sqrt(s);
}

/* Rows rows[0..nrows) of the triangle; row i (i+1 values) goes to
 * out[out_off[r] .. out_off[r] + i]. */
void oracle_edm_rows_f64(const float *X, int64_t N, int32_t d, int64_t ldx,
                         const int64_t *rows, int64_t nrows,
                         const int64_t *out_off, double *out)
{
    (void)N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        double *o = out + out_off[r];
        for (int64_t j = 0; j <= i; ++j)
            o[j] = pair_dist(X, ldx, d, i, j);
    }
}

/* The whole triangle, packed: cell (i, j) at i(i+1)/2 + j. */
void oracle_edm_packed_f64(const float *X, int64_t N, int32_t d, int64_t ldx,
                           double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double *o = out + i * (i + 1) / 2;
        for (int64_t j = 0; j <= i; ++j)
            o[j] = pair_dist(X, ldx, d, i, j);
    }
}

/* Gradient through the EDM; dD is the packed cell gradient (diagonal
 * ignored), dX is N x d row-major (overwritten).  Gather form, one point
 * per iteration. */
void oracle_edm_backward_f64(const float *X, int64_t N, int32_t d, int64_t ldx,
                             const float *dD, double *dX)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        for (int32_t k = 0; k < d; ++k)
            dX[i * d + k] = 0.0;
        for (int64_t j = 0; j < i; ++j) {
            double D = pair_dist(X, ldx, d, i, j);
            if (D > 0.0) {
                double c = (double)dD[i * (i + 1) / 2 + j] / D;
                for (int32_t k = 0; k < d; ++k)
                    dX[i * d + k] += c * ((double)X[i * ldx + k] - (double)X[j * ldx + k]);
            }
        }
        for (int64_t m = i + 1; m < N; ++m) {
            double D = pair_dist(X, ldx, d, m, i);
            if (D > 0.0) {
                double c = (double)dD[m * (m + 1) / 2 + i] / D;
                for (int32_t k = 0; k < d; ++k)
                    dX[i * d + k] -= c * ((double)X[m * ldx + k] - (double)X[i * ldx + k]);
            }
        }
    }
}
