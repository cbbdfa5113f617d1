/*
 * Test infrastructure only: part of the FP64 CPU oracle of the bbFMM matvec.
 * Nothing in the product library links or calls this file.
 *
 * The direct kernel summation of eq. (1):
 *     phi_i = sum_j K(x_i, y_j) sigma_j,   for every target i,
 * evaluated pair by pair in double precision.  The oracle uses it twice:
 * as the exact O(N^2) reference (the dense product of eq. (2)) and as the
 * near-field (P2P) step of Section 2.3, where the source set is the union of
 * a leaf's neighbours.
 *
 * Kernels (Section 1 and Section 4):
 *   0   K = 1/|x-y|, with K = 0 where |x-y|^2 == 0 (singular diagonal)
 *   1   K = exp(-|x-y|/a)
 *   2   K = exp(-|x-y|^2/a^2)
 *   3   K = (x_1 - y_1)/|x-y|^3, with K = 0 where |x-y|^2 == 0: the x-component
 *       of a dipole field, skew-symmetric (K(y,x) = -K(x,y)) and homogeneous
 *       of degree -2
 *   100 K = g(u_x) g(u_y) g(u_z), u = (x-y)/a, g(u) = 1 + u/2 - u^2/3 + u^3/5
 *       (a test kernel: degree 3 in each coordinate, not symmetric)
 *
 * Plain loops, no blocking; OpenMP only splits the independent targets.
 */
#include <math.h>
#include <stdint.h>

static double oracle_kernel(int kid, double a, double dx, double dy, double dz)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    switch (kid) {
    case 0:
        return r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    case 1:
        return exp(-sqrt(r2) / a);
    case 2:
        return exp(-r2 / (a * a));
    case 3:
        return r2 > 0.0 ? dx / (r2 * sqrt(r2)) : 0.0;
    case 100: {
        double u[3] = {dx / a, dy / a, dz / a};
        double p = 1.0;
        for (int d = 0; d < 3; ++d)
            p *= 1.0 + u[d] / 2.0 - u[d] * u[d] / 3.0 + u[d] * u[d] * u[d] / 5.0;
        return p;
    }
    default:
        return NAN;
    }
}

/* out[i*r + c] = sum_j K(t_i, s_j) * sigma[j*r + c]   (overwrites out) */
void oracle_direct_sum(int64_t nt, const double *tx, const double *ty,
                       const double *tz, int64_t ns, const double *sx,
                       const double *sy, const double *sz,
                       const double *sigma, int64_t r, int32_t kid,
                       double param, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double *o = out + i * r;
        for (int64_t c = 0; c < r; ++c)
            o[c] = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double k = oracle_kernel(kid, param, tx[i] - sx[j], ty[i] - sy[j],
                                     tz[i] - sz[j]);
            const double *s = sigma + j * r;
            for (int64_t c = 0; c < r; ++c)
                o[c] += k * s[c];
        }
    }
}

/* Kernel values for explicit pairs: out[p] = K(t_p, s_p). */
void oracle_kernel_pairs(int64_t np_, const double *dx, const double *dy,
                         const double *dz, int32_t kid, double param,
                         double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np_; ++p)
        out[p] = oracle_kernel(kid, param, dx[p], dy[p], dz[p]);
}
