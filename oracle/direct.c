/*
 * CPU oracle: the plain O(N^2) boundary-integral sum in float64.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.
 *
 * It evaluates the quadrature sum of the paper's general integral problem
 * (Sec. II.A, Eq. sum_fmm) for the Laplace kernels used in Sec. II-III:
 *
 *   pot_i   = sum_j  q_j / (4 pi r_ij)  +  m_j . (x_i - y_j) / (4 pi r_ij^3)
 *   field_i = sum_j  q_j (x_i - y_j) / (4 pi r_ij^3)
 *
 * The first term is the single layer; the second is the double layer
 * d/dn_y [1/(4 pi |x-y|)] with the dipole m_j = mu_j n_j (Eq. fk_integral
 * and Eq. kernel with the 1/(4 pi) of Eq. fk_integral_discrete). The field is
 * the kernel of Eq. kernel_pol, i.e. -grad of the single-layer potential.
 * A pair with r_ij < delta contributes nothing (Sec. III.A.1, singularity
 * exclusion); r_ij = 0 is always excluded.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define FOUR_PI 12.566370614359172953850573533118

void oracle_direct_sum(int64_t nt, const double *tx, const double *ty, const double *tz,
                       int64_t ns, const double *sx, const double *sy, const double *sz,
                       const double *q, const double *mx, const double *my, const double *mz,
                       double delta, double *pot, double *fx, double *fy, double *fz)
{
    const double d2 = delta * delta;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double p = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double dx = tx[i] - sx[j];
            double dy = ty[i] - sy[j];
            double dz = tz[i] - sz[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0 || r2 < d2)
                continue;
            double r = sqrt(r2);
            double inv_r = 1.0 / r;
            double inv_r3 = inv_r / r2;
            if (q) {
                p += q[j] * inv_r;
                ex += q[j] * dx * inv_r3;
                ey += q[j] * dy * inv_r3;
                ez += q[j] * dz * inv_r3;
            }
            if (mx)
                p += (mx[j] * dx + my[j] * dy + mz[j] * dz) * inv_r3;
        }
        if (pot)
            pot[i] = p / FOUR_PI;
        if (fx) {
            fx[i] = ex / FOUR_PI;
            fy[i] = ey / FOUR_PI;
            fz[i] = ez / FOUR_PI;
        }
    }
}

/* Number of OpenMP threads the sum above runs on. */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
