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

#include <initializer_list>

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

// The element loops below take four elements per load (float4) when VEC is
// set (every operand 16-byte aligned), then the remainder one by one.
template <bool VEC>
__global__ void __launch_bounds__(kT) sumsq_kernel(const float* __restrict__ a, int64_t n,
                                                   double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const int64_t t0 = (int64_t)blockIdx.x * kT + threadIdx.x, stride = (int64_t)kRedBlocks * kT;
    double acc = 0.0;
    int64_t done = 0;
    if (VEC) {
        const float4* a4 = reinterpret_cast<const float4*>(a);
        for (int64_t i = t0; i < (n >> 2); i += stride) {
            const float4 v = a4[i];
            acc = fma((double)v.x, (double)v.x, acc);
            acc = fma((double)v.y, (double)v.y, acc);
            acc = fma((double)v.z, (double)v.z, acc);
            acc = fma((double)v.w, (double)v.w, acc);
        }
        done = n & ~(int64_t)3;
    }
    for (int64_t i = done + t0; i < n; i += stride) {
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

// x += alpha d over the volume and r -= alpha q over the projections; the
// partial sums of the new ||r||^2.
__device__ __forceinline__ float axpy1(double a, float y, float x) { return (float)fma(a, (double)y, (double)x); }

template <bool VEC>
__global__ void __launch_bounds__(kT) cgls_update_kernel(float* __restrict__ x, const float* __restrict__ d,
                                                         int64_t nv, float* __restrict__ r,
                                                         const float* __restrict__ q, int64_t np,
                                                         const double* __restrict__ st,
                                                         double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const double alpha = st[kStAlpha];
    const int64_t t0 = (int64_t)blockIdx.x * kT + threadIdx.x, stride = (int64_t)kRedBlocks * kT;
    int64_t done = 0;
    if (VEC) {
        float4* x4 = reinterpret_cast<float4*>(x);
        const float4* d4 = reinterpret_cast<const float4*>(d);
        for (int64_t i = t0; i < (nv >> 2); i += stride) {
            const float4 a = x4[i], b = d4[i];
            x4[i] = make_float4(axpy1(alpha, b.x, a.x), axpy1(alpha, b.y, a.y), axpy1(alpha, b.z, a.z),
                                axpy1(alpha, b.w, a.w));
        }
        done = nv & ~(int64_t)3;
    }
    for (int64_t i = done + t0; i < nv; i += stride) x[i] = axpy1(alpha, d[i], x[i]);
    double acc = 0.0;
    done = 0;
    if (VEC) {
        float4* r4 = reinterpret_cast<float4*>(r);
        const float4* q4 = reinterpret_cast<const float4*>(q);
        for (int64_t i = t0; i < (np >> 2); i += stride) {
            const float4 a = r4[i], b = q4[i];
            const float4 o = make_float4(axpy1(-alpha, b.x, a.x), axpy1(-alpha, b.y, a.y), axpy1(-alpha, b.z, a.z),
                                         axpy1(-alpha, b.w, a.w));
            r4[i] = o;
            acc = fma((double)o.x, (double)o.x, acc);
            acc = fma((double)o.y, (double)o.y, acc);
            acc = fma((double)o.z, (double)o.z, acc);
            acc = fma((double)o.w, (double)o.w, acc);
        }
        done = np & ~(int64_t)3;
    }
    for (int64_t i = done + t0; i < np; i += stride) {
        const float rn = axpy1(-alpha, q[i], r[i]);
        r[i] = rn;
        acc = fma((double)rn, (double)rn, acc);
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
template <bool VEC>
__global__ void __launch_bounds__(kT) residual_kernel(float* __restrict__ r, const float* __restrict__ p,
                                                      const float* __restrict__ w, int64_t n,
                                                      double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const int64_t t0 = (int64_t)blockIdx.x * kT + threadIdx.x, stride = (int64_t)kRedBlocks * kT;
    double acc = 0.0;
    int64_t done = 0;
    auto one = [&](float rv, float pv, float wv) {
        const double e = (double)pv - (double)rv;
        acc = fma(e, e, acc);
        return (float)(w ? e * (double)wv : e);
    };
    if (VEC) {
        float4* r4 = reinterpret_cast<float4*>(r);
        const float4* p4 = reinterpret_cast<const float4*>(p);
        const float4* w4 = reinterpret_cast<const float4*>(w);
        for (int64_t i = t0; i < (n >> 2); i += stride) {
            const float4 a = r4[i], b = p4[i], c = w ? w4[i] : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
            r4[i] = make_float4(one(a.x, b.x, c.x), one(a.y, b.y, c.y), one(a.z, b.z, c.z), one(a.w, b.w, c.w));
        }
        done = n & ~(int64_t)3;
    }
    for (int64_t i = done + t0; i < n; i += stride) r[i] = one(r[i], p[i], w ? w[i] : 1.0f);
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

static bool aligned16(std::initializer_list<const void*> ptrs)
{
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return false;
    return true;
}

hipError_t launch_sumsq(const float* a, int64_t n, double* part, hipStream_t s)
{
    if (aligned16({a}))
        sumsq_kernel<true><<<kRedBlocks, kT, 0, s>>>(a, n, part);
    else
        sumsq_kernel<false><<<kRedBlocks, kT, 0, s>>>(a, n, part);
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
    if (aligned16({x, d, r, q}))
        cgls_update_kernel<true><<<kRedBlocks, kT, 0, s>>>(x, d, nv, r, q, np, st, part);
    else
        cgls_update_kernel<false><<<kRedBlocks, kT, 0, s>>>(x, d, nv, r, q, np, st, part);
    return hipGetLastError();
}

hipError_t launch_cgls_direction(float* d, const float* sv, int64_t n, const double* st, hipStream_t s)
{
    cgls_direction_kernel<<<ew_grid(n), kT, 0, s>>>(d, sv, n, st);
    return hipGetLastError();
}

hipError_t launch_residual(float* r, const float* p, const float* w, int64_t n, double* part, hipStream_t s)
{
    if (aligned16({r, p, w}))
        residual_kernel<true><<<kRedBlocks, kT, 0, s>>>(r, p, w, n, part);
    else
        residual_kernel<false><<<kRedBlocks, kT, 0, s>>>(r, p, w, n, part);
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
