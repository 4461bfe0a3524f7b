/*
 * FP64 reference ("oracle") for FDK preprocessing of cone-beam projections:
 * the weighting and row filtering that turn line integrals into the filtered
 * projections a voxel-driven backprojection consumes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests and the benchmark do.  It shares no code
 * with the GPU path.
 *
 * The paper's benchmark data arrive filtered (Sec. "RabbitCT Benchmarking
 * Framework"); the filtering follows the FDK method (Feldkamp, Davis and
 * Kress, 1984) with short-scan weights (Parker, 1982) and the band-limited
 * ramp kernel sampled at the detector pitch (Kak and Slaney, "Principles of
 * Computerized Tomographic Imaging", Ch. 3):
 *   u_i = (i - u0) pu, v_j = (j - v0) pv                      detector mm
 *   cosine weight   c(i, j) = SDD / sqrt(SDD^2 + u_i^2 + v_j^2)
 *   fan angle       g_i     = s atan(u_i / SDD), s = +1 or -1 (orientation)
 *   Parker weight   w(b, g) with d = (R - pi) / 2 for a scan range R:
 *                     sin^2(pi/4 b / (d - g))            0 <= b < 2d - 2g
 *                     1                                  2d - 2g <= b <= pi - 2g
 *                     sin^2(pi/4 (pi + 2d - b) / (d + g)) pi - 2g < b <= pi + 2d
 *                     0                                  otherwise
 *                   (R <= 0: no short-scan weighting, w = 1)
 *   ramp kernel     h(0) = 1/(4 t^2), h(n) = 0 for even n != 0,
 *                   h(n) = -1/(n pi t)^2 for odd n, t = pu SID / SDD
 *   q_k(i, j) = t * dbeta * SID^2 * sum_{i'} h(i - i') p_k(i', j) c(i', j) w(b_k, g_i')
 * The sum is the plain linear convolution over the row (i' = 0 .. W-1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

double oracle_parker_weight(double beta, double gamma, double range)
{
    if (range <= 0.0) return 1.0;
    const double d = 0.5 * (range - M_PI);
    if (beta < 0.0 || beta > M_PI + 2.0 * d) return 0.0;
    if (beta < 2.0 * d - 2.0 * gamma) {
        const double s = sin(M_PI / 4.0 * beta / (d - gamma));
        return s * s;
    }
    if (beta <= M_PI - 2.0 * gamma) return 1.0;
    const double s = sin(M_PI / 4.0 * (M_PI + 2.0 * d - beta) / (d + gamma));
    return s * s;
}

double oracle_ramp_kernel(int64_t n, double tau)
{
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if (n % 2 == 0) return 0.0;
    const double a = (double)n * M_PI * tau;
    return -1.0 / (a * a);
}

void oracle_fdk_filter(int64_t N, int64_t W, int64_t H, double pu, double pv, double u0, double v0,
                       double sdd, double sid, const double *beta, double range, double dbeta,
                       double fan_sign, const double *p, double *q)
{
    const double tau = pu * sid / sdd;
    const double gain = tau * dbeta * sid * sid;
    double *hk = (double *)malloc(sizeof(double) * (size_t)(2 * W - 1));   /* h(n), n = -(W-1) .. W-1 */
    for (int64_t n = -(W - 1); n <= W - 1; ++n) hk[n + W - 1] = oracle_ramp_kernel(n, tau);
#pragma omp parallel
    {
        double *x = (double *)malloc(sizeof(double) * (size_t)W);
#pragma omp for collapse(2) schedule(dynamic, 4)
        for (int64_t k = 0; k < N; ++k) {
            for (int64_t j = 0; j < H; ++j) {
                const double v = ((double)j - v0) * pv;
                const double *row = p + (k * H + j) * W;
                double *out = q + (k * H + j) * W;
                /* weighted row: cosine and short-scan weights */
                for (int64_t ip = 0; ip < W; ++ip) {
                    const double u = ((double)ip - u0) * pu;
                    const double c = sdd / sqrt(sdd * sdd + u * u + v * v);
                    const double g = fan_sign * atan(u / sdd);
                    x[ip] = row[ip] * c * oracle_parker_weight(beta[k], g, range);
                }
                /* linear convolution with the ramp kernel */
                for (int64_t i = 0; i < W; ++i) {
                    double acc = 0.0;
                    for (int64_t ip = 0; ip < W; ++ip) acc += hk[i - ip + W - 1] * x[ip];
                    out[i] = gain * acc;
                }
            }
        }
        free(x);
    }
    free(hk);
}
