/*
 * FP64 reference ("oracle") for voxel-driven FDK cone-beam backprojection and
 * its exact adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU path.
 *
 * What it computes (paper, Sec. "RabbitCT Benchmarking Framework", Listing 1
 * and the prose that follows it):
 *   for every voxel (x, y, z) and projection k
 *     world point   X = O + (x, y, z) * MM                (voxel -> WCS)
 *     (u, v, w)     = A_k (X, 1)                          (forward projection)
 *     (ix, iy)      = (u / w, v / w)                      (dehomogenisation)
 *     val           = bilinear sample of I_k at (ix, iy), zero off the detector
 *     V(x, y, z)   += val / w^2                           (inverse-square weight)
 * with these readings of the listing:
 *   - the integer part is floor(), not truncation toward zero, so the sample is
 *     continuous at ix = 0 and agrees with the zero-padded form the paper uses
 *     in its optimised kernel;
 *   - a tap (i, j) is on the detector iff 0 <= i < W and 0 <= j < H (the row
 *     stride is the width, so the column index is bounded by the width);
 *   - zero is applied per tap (the image is zero-extended);
 *   - A is row-major A[r][c]; the listing's A[r + 3c] is the same matrix;
 *   - division, not a reciprocal; summation over k in ascending order in FP64.
 *
 * The adjoint (forward projector) is the transpose of that linear map: every
 * voxel value x_v, weighted by 1/w^2, is scattered onto the four taps with the
 * same bilinear weights, skipping taps that are off the detector.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Projection of voxel (x, y, z) through row-major A (12 doubles). */
static void project_voxel(const double *A, const double *origin, double voxel,
                          int64_t x, int64_t y, int64_t z,
                          double *ix, double *iy, double *w)
{
    double wx = origin[0] + (double)x * voxel;
    double wy = origin[1] + (double)y * voxel;
    double wz = origin[2] + (double)z * voxel;
    double u = A[0] * wx + A[1] * wy + A[2] * wz + A[3];
    double v = A[4] * wx + A[5] * wy + A[6] * wz + A[7];
    double ww = A[8] * wx + A[9] * wy + A[10] * wz + A[11];
    *ix = u / ww;
    *iy = v / ww;
    *w = ww;
}

static double tap(const double *I, int64_t W, int64_t H, int64_t i, int64_t j)
{
    if (i < 0 || i >= W || j < 0 || j >= H)
        return 0.0;
    return I[j * W + i];
}

/* Bilinear sample with zero extension.  Coordinates far outside the detector
 * are resolved before the integer conversion so that it cannot overflow. */
static double sample(const double *I, int64_t W, int64_t H, double ix, double iy)
{
    if (!(ix > -1.0 && ix < (double)W && iy > -1.0 && iy < (double)H)) {
        if (isnan(ix) || isnan(iy))
            return NAN;
        return 0.0;  /* every tap is off the detector */
    }
    double fx = floor(ix), fy = floor(iy);
    int64_t i0 = (int64_t)fx, j0 = (int64_t)fy;
    double sx = ix - fx, sy = iy - fy;
    double b = (1.0 - sx) * tap(I, W, H, i0, j0) + sx * tap(I, W, H, i0 + 1, j0);
    double t = (1.0 - sx) * tap(I, W, H, i0, j0 + 1) + sx * tap(I, W, H, i0 + 1, j0 + 1);
    return (1.0 - sy) * b + sy * t;
}

/*
 * Backprojection of projections [k_begin, k_end) into the planes
 * [z_begin, z_begin + z_count) of an L^3 grid.
 *   mats  : n_proj * 12 doubles, row-major per projection
 *   proj  : n_proj * H * W doubles, [k][j][i]
 *   vol   : z_count * L * L doubles, index ((z - z_begin) * L + y) * L + x
 *   accumulate = 0 overwrites vol, 1 adds to it.
 * The outermost z-loop is split across threads, as the paper does on CPUs;
 * each voxel still sums its projections in ascending k.
 */
void oracle_backproject(int64_t L, double voxel, const double *origin,
                        int64_t z_begin, int64_t z_count,
                        int64_t n_proj, int64_t W, int64_t H,
                        const double *mats, const double *proj,
                        int64_t k_begin, int64_t k_end,
                        double *vol, int accumulate)
{
    int64_t zz;
#pragma omp parallel for schedule(dynamic, 1)
    for (zz = 0; zz < z_count; ++zz) {
        double *plane = vol + zz * L * L;
        int64_t z = z_begin + zz;
        if (!accumulate)
            memset(plane, 0, (size_t)(L * L) * sizeof(double));
        for (int64_t k = k_begin; k < k_end; ++k) {
            const double *A = mats + 12 * k;
            const double *I = proj + k * H * W;
            for (int64_t y = 0; y < L; ++y) {
                for (int64_t x = 0; x < L; ++x) {
                    double ix, iy, w;
                    project_voxel(A, origin, voxel, x, y, z, &ix, &iy, &w);
                    plane[y * L + x] += sample(I, W, H, ix, iy) / (w * w);
                }
            }
        }
    }
    (void)n_proj;
}

/*
 * Backprojection at an arbitrary list of voxels: out[p] = sum_k val/w^2 for
 * voxel (xyz[3p], xyz[3p+1], xyz[3p+2]).  Used to check large volumes one
 * voxel at a time.
 */
void oracle_backproject_points(int64_t n_points, const int32_t *xyz,
                               double voxel, const double *origin,
                               int64_t n_proj, int64_t W, int64_t H,
                               const double *mats, const double *proj,
                               double *out)
{
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n_points; ++p) {
        double acc = 0.0;
        for (int64_t k = 0; k < n_proj; ++k) {
            double ix, iy, w;
            project_voxel(mats + 12 * k, origin, voxel, xyz[3 * p], xyz[3 * p + 1],
                          xyz[3 * p + 2], &ix, &iy, &w);
            acc += sample(proj + k * H * W, W, H, ix, iy) / (w * w);
        }
        out[p] = acc;
    }
}

/*
 * Exact adjoint of oracle_backproject: for each projection k, scatter every
 * voxel value times 1/w^2 onto the four bilinear taps that lie on the detector.
 *   vol  : z_count * L * L doubles (planes [z_begin, z_begin + z_count))
 *   out  : n_proj * H * W doubles; overwritten unless accumulate.
 * Projections are independent, so they are split across threads; within a
 * projection the scatter is sequential.
 */
void oracle_forwardproject(int64_t L, double voxel, const double *origin,
                           int64_t z_begin, int64_t z_count,
                           int64_t n_proj, int64_t W, int64_t H,
                           const double *mats, const double *vol,
                           double *out, int accumulate)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 1)
    for (k = 0; k < n_proj; ++k) {
        const double *A = mats + 12 * k;
        double *P = out + k * H * W;
        if (!accumulate)
            memset(P, 0, (size_t)(H * W) * sizeof(double));
        for (int64_t zz = 0; zz < z_count; ++zz) {
            for (int64_t y = 0; y < L; ++y) {
                for (int64_t x = 0; x < L; ++x) {
                    double ix, iy, w;
                    project_voxel(A, origin, voxel, x, y, z_begin + zz, &ix, &iy, &w);
                    if (!(ix > -1.0 && ix < (double)W && iy > -1.0 && iy < (double)H))
                        continue;
                    double fx = floor(ix), fy = floor(iy);
                    int64_t i0 = (int64_t)fx, j0 = (int64_t)fy;
                    double sx = ix - fx, sy = iy - fy;
                    double s = vol[(zz * L + y) * L + x] / (w * w);
                    double wt[4] = {(1.0 - sx) * (1.0 - sy), sx * (1.0 - sy),
                                    (1.0 - sx) * sy, sx * sy};
                    int64_t ti[4] = {i0, i0 + 1, i0, i0 + 1};
                    int64_t tj[4] = {j0, j0, j0 + 1, j0 + 1};
                    for (int q = 0; q < 4; ++q)
                        if (ti[q] >= 0 && ti[q] < W && tj[q] >= 0 && tj[q] < H)
                            P[tj[q] * W + ti[q]] += wt[q] * s;
                }
            }
        }
    }
}

/*
 * Number of (voxel, projection) pairs whose sample touches the detector, i.e.
 * the updates a clipping backprojector must perform (the paper counts GUp/s
 * over these "clipped" updates).  Planes [z_begin, z_begin + z_count).
 */
int64_t oracle_supported_updates(int64_t L, double voxel, const double *origin,
                                 int64_t z_begin, int64_t z_count,
                                 int64_t n_proj, int64_t W, int64_t H,
                                 const double *mats)
{
    int64_t total = 0, zz;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (zz = 0; zz < z_count; ++zz) {
        for (int64_t k = 0; k < n_proj; ++k)
            for (int64_t y = 0; y < L; ++y)
                for (int64_t x = 0; x < L; ++x) {
                    double ix, iy, w;
                    project_voxel(mats + 12 * k, origin, voxel, x, y, z_begin + zz,
                                  &ix, &iy, &w);
                    if (ix > -1.0 && ix < (double)W && iy > -1.0 && iy < (double)H)
                        ++total;
                }
    }
    return total;
}
