// gfx950 vector kernels of the iterative solvers (CGLS and SIRT on the
// matched forward/back projector pair) that run between the projector
// launches.  All of them stream HBM once per operand:
//   - reductions (sum of squares, maximum) with a fixed grid of kRedBlocks
//     workgroups and a fixed combination order, so the FP64 results are
//     bit-reproducible for a given size;
//   - a one-workgroup scalar kernel that combines the partials and derives
//     the step lengths (alpha, beta of CGLS) in device memory, so an
//     iteration never waits for the host;
//   - fused element-wise updates that read those step lengths.
// Vectors are FP32; every update is evaluated in FP64 and rounded once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdk_internal.h"

namespace fdk {
namespace {

constexpr int kT = 256;   // threads of every kernel here (4 wavefronts)

// Sum (or max) over the workgroup; the result is valid in thread 0.
template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double* sh)
{
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double u = __shfl_down(v, o, kWave);
        v = MAX ? fmax(v, u) : v + u;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = sh[0];
    if (threadIdx.x == 0)
        for (int w = 1; w < kT / kWave; ++w) t = MAX ? fmax(t, sh[w]) : t + sh[w];
    return t;
}

__global__ void __launch_bounds__(kT) sumsq_kernel(const float* __restrict__ a, int64_t n,
                                                   double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT) {
        const double x = a[i];
        acc = fma(x, x, acc);
    }
    const double t = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kT) max_kernel(const float* __restrict__ a, int64_t n,
                                                 double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    double m = 0.0;   // the reduced arrays are sums of non-negative weights
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT)
        m = fmax(m, (double)a[i]);
    const double t = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Combines the kRedBlocks partials in a fixed order and applies `op`.
__global__ void __launch_bounds__(kT) scalar_kernel(const double* __restrict__ part, double* __restrict__ st,
                                                    double* __restrict__ hist, int op, int slot)
{
    __shared__ double sh[kT / kWave];
    const bool is_max = op == kOpMax;
    double v = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kT) v = is_max ? fmax(v, part[i]) : v + part[i];
    const double t = is_max ? block_reduce<true>(v, sh) : block_reduce<false>(v, sh);
    if (threadIdx.x != 0) return;
    switch (op) {
    case kOpStore:
    case kOpMax:
        st[slot] = t;
        break;
    case kOpAlpha:   // t = ||A d||^2
        st[kStQQ] = t;
        st[kStAlpha] = t > 0.0 ? st[kStGamma] / t : 0.0;
        break;
    case kOpBeta:    // t = ||A^T r||^2 of the new residual
        st[kStBeta] = st[kStGamma] > 0.0 ? t / st[kStGamma] : 0.0;
        st[kStGamma] = t;
        break;
    case kOpHist:
        if (hist) hist[slot] = t;
        break;
    }
}

// x += alpha d over the volume and r -= alpha q over the projections (one
// index space of nv + np elements); the partial sums of the new ||r||^2.
__global__ void __launch_bounds__(kT) cgls_update_kernel(float* __restrict__ x, const float* __restrict__ d,
                                                         int64_t nv, float* __restrict__ r,
                                                         const float* __restrict__ q, int64_t np,
                                                         const double* __restrict__ st,
                                                         double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const double alpha = st[kStAlpha];
    double acc = 0.0;
    const int64_t n = nv + np;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT) {
        if (i < nv) {
            x[i] = (float)fma(alpha, (double)d[i], (double)x[i]);
        } else {
            const int64_t j = i - nv;
            const float rn = (float)fma(-alpha, (double)q[j], (double)r[j]);
            r[j] = rn;
            acc = fma((double)rn, (double)rn, acc);
        }
    }
    const double t = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// d = s + beta d
__global__ void __launch_bounds__(kT) cgls_direction_kernel(float* __restrict__ d, const float* __restrict__ s,
                                                            int64_t n, const double* __restrict__ st)
{
    const double beta = st[kStBeta];
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        d[i] = (float)fma(beta, (double)d[i], (double)s[i]);
}

// e = p - r;  partial sums of ||e||^2;  r = e (or e * w when w is given)
__global__ void __launch_bounds__(kT) residual_kernel(float* __restrict__ r, const float* __restrict__ p,
                                                      const float* __restrict__ w, int64_t n,
                                                      double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT) {
        const double e = (double)p[i] - (double)r[i];
        acc = fma(e, e, acc);
        r[i] = (float)(w ? e * (double)w[i] : e);
    }
    const double t = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += lambda c t, then max(x, 0) when nonneg
__global__ void __launch_bounds__(kT) sirt_update_kernel(float* __restrict__ x, const float* __restrict__ t,
                                                         const float* __restrict__ c, int64_t n, double lambda,
                                                         int nonneg)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        double v = fma(lambda * (double)c[i], (double)t[i], (double)x[i]);
        if (nonneg) v = fmax(v, 0.0);
        x[i] = (float)v;
    }
}

// a = 1 / max(a, floor_rel * st[slot]); all zero when the maximum is zero
__global__ void __launch_bounds__(kT) inv_floor_kernel(float* __restrict__ a, int64_t n,
                                                       const double* __restrict__ st, int slot, double floor_rel)
{
    const double f = floor_rel * st[slot];
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        a[i] = f > 0.0 ? (float)(1.0 / fmax((double)a[i], f)) : 0.0f;
}

// Element-wise kernels: enough workgroups to fill the chip several times over.
unsigned ew_grid(int64_t n)
{
    const int64_t g = (n + kT - 1) / kT;
    return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

}  // namespace

hipError_t launch_sumsq(const float* a, int64_t n, double* part, hipStream_t s)
{
    sumsq_kernel<<<kRedBlocks, kT, 0, s>>>(a, n, part);
    return hipGetLastError();
}

hipError_t launch_max(const float* a, int64_t n, double* part, hipStream_t s)
{
    max_kernel<<<kRedBlocks, kT, 0, s>>>(a, n, part);
    return hipGetLastError();
}

hipError_t launch_scalar(const double* part, double* st, double* hist, int op, int slot, hipStream_t s)
{
    scalar_kernel<<<1, kT, 0, s>>>(part, st, hist, op, slot);
    return hipGetLastError();
}

hipError_t launch_cgls_update(float* x, const float* d, int64_t nv, float* r, const float* q, int64_t np,
                              const double* st, double* part, hipStream_t s)
{
    cgls_update_kernel<<<kRedBlocks, kT, 0, s>>>(x, d, nv, r, q, np, st, part);
    return hipGetLastError();
}

hipError_t launch_cgls_direction(float* d, const float* sv, int64_t n, const double* st, hipStream_t s)
{
    cgls_direction_kernel<<<ew_grid(n), kT, 0, s>>>(d, sv, n, st);
    return hipGetLastError();
}

hipError_t launch_residual(float* r, const float* p, const float* w, int64_t n, double* part, hipStream_t s)
{
    residual_kernel<<<kRedBlocks, kT, 0, s>>>(r, p, w, n, part);
    return hipGetLastError();
}

hipError_t launch_sirt_update(float* x, const float* t, const float* c, int64_t n, double lambda, int nonneg,
                              hipStream_t s)
{
    sirt_update_kernel<<<ew_grid(n), kT, 0, s>>>(x, t, c, n, lambda, nonneg);
    return hipGetLastError();
}

hipError_t launch_inv_floor(float* a, int64_t n, const double* st, int slot, double floor_rel, hipStream_t s)
{
    inv_floor_kernel<<<ew_grid(n), kT, 0, s>>>(a, n, st, slot, floor_rel);
    return hipGetLastError();
}

}  // namespace fdk
