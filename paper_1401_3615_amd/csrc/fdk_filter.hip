// gfx950 kernel of FDK preprocessing: cosine and short-scan (Parker) weights
// and the band-limited ramp filter along detector rows (the filtering that
// precedes the paper's backprojection; its benchmark data arrive filtered,
// Sec. "RabbitCT Benchmarking Framework").
//
// One workgroup filters two rows of one projection at once as the real and
// imaginary parts of one complex sequence: the ramp kernel is real and even,
// so its spectrum is real and multiplying the packed spectrum by it filters
// both rows independently.  The linear convolution is a circular one of
// length M >= 2W - 1 (rows zero-padded), computed as FFT, multiply, inverse
// FFT (the inverse through conjugation: conj(FFT(conj(Z H)))), with radix-4
// Stockham passes in LDS (ping-pong buffers, no bit reversal).  The weights,
// the kernel spectrum (with the output gain and 1/M folded in) and the
// twiddles come from FP64 tables computed on the host.
//
// The arithmetic is FP64 (full rate on gfx950's vector units) and only the
// output is rounded to FP32: the ramp filter amplifies white rounding noise
// of its input by ~|H|max ||x|| / ||y|| (20-30x for projection data), so an
// FP32 pipeline lands near 1e-5 relative error from rounding alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdk_internal.h"

namespace fdk {
namespace {

constexpr int kFilterThreads = 1024;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Forward DFT (length M, power of two >= 4) of buf0 by Stockham passes in
// LDS: radix-4 while four sub-transforms fit, then one radix-2 pass if
// log2(M) is odd.  tw holds exp(-2 pi i t / M) for t < M/4; the powers w^2,
// w^3 are formed by multiplication and the radix-2 twiddles beyond M/4 by a
// quarter turn.  Returns the buffer that holds the result.
__device__ __forceinline__ double2* fft(double2* buf0, double2* buf1, const double2* tw, int M)
{
    double2* in = buf0;
    double2* out = buf1;
    const int q = M >> 2;
    int Ns = 1;
    for (; 4 * Ns <= M; Ns <<= 2) {
        const int tstep = q / Ns;
        for (int j = threadIdx.x; j < q; j += kFilterThreads) {
            const int k = j & (Ns - 1);
            const double2 w = tw[k * tstep];
            const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
            const double2 v0 = in[j];
            const double2 v1 = cmul(in[j + q], w);
            const double2 v2 = cmul(in[j + 2 * q], w2);
            const double2 v3 = cmul(in[j + 3 * q], w3);
            const double2 a0 = make_double2(v0.x + v2.x, v0.y + v2.y), a1 = make_double2(v0.x - v2.x, v0.y - v2.y);
            const double2 a2 = make_double2(v1.x + v3.x, v1.y + v3.y);
            const double2 a3 = make_double2(v1.y - v3.y, v3.x - v1.x);   // -i (v1 - v3)
            const int o = ((j - k) << 2) + k;
            out[o] = make_double2(a0.x + a2.x, a0.y + a2.y);
            out[o + Ns] = make_double2(a1.x + a3.x, a1.y + a3.y);
            out[o + 2 * Ns] = make_double2(a0.x - a2.x, a0.y - a2.y);
            out[o + 3 * Ns] = make_double2(a1.x - a3.x, a1.y - a3.y);
        }
        __syncthreads();
        double2* t = in;
        in = out;
        out = t;
    }
    if (Ns < M) {   // Ns = M / 2: radix-2 pass, twiddle exp(-2 pi i j / M)
        const int h = M >> 1;
        for (int j = threadIdx.x; j < h; j += kFilterThreads) {
            double2 w;
            if (j < q) {
                w = tw[j];
            } else {
                const double2 r = tw[j - q];
                w = make_double2(r.y, -r.x);
            }
            const double2 v0 = in[j];
            const double2 v1 = cmul(in[j + h], w);
            out[j] = make_double2(v0.x + v1.x, v0.y + v1.y);
            out[j + h] = make_double2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
        in = out;
    }
    return in;
}

__global__ __launch_bounds__(kFilterThreads) void filter_kernel(FilterArgs f)
{
    extern __shared__ double2 lds2[];   // 2 M complex buffers + M/4 twiddles
    const int pairs = (f.H + 1) >> 1;
    const int k = (int)(blockIdx.x / pairs);
    const int j0 = 2 * (int)(blockIdx.x - k * pairs), j1 = j0 + 1;
    const bool has1 = j1 < f.H;
    const int M = f.M;
    double2* b0 = lds2;
    double2* b1 = lds2 + M;
    double2* tws = lds2 + 2 * M;
    for (int t = threadIdx.x; t < (M >> 2); t += kFilterThreads) tws[t] = f.tw[t];
    const float* s0 = f.src + ((int64_t)k * f.H + j0) * f.W;
    const float* s1 = s0 + f.W;
    const double* c0 = f.wc + (int64_t)j0 * f.W;
    const double* c1 = c0 + f.W;
    const double* wp = f.wp + (int64_t)k * f.W;
    for (int i = threadIdx.x; i < M; i += kFilterThreads) {
        double x0 = 0.0, x1 = 0.0;
        if (i < f.W) {
            const double w = wp[i];
            x0 = (double)s0[i] * c0[i] * w;
            if (has1) x1 = (double)s1[i] * c1[i] * w;
        }
        b0[i] = make_double2(x0, x1);
    }
    __syncthreads();
    double2* z = fft(b0, b1, tws, M);
    // conj(Z H): H real (kernel even), gain / M folded in
    for (int m = threadIdx.x; m < M; m += kFilterThreads) {
        const double h = f.hs[m];
        const double2 v = z[m];
        z[m] = make_double2(v.x * h, -v.y * h);
    }
    __syncthreads();
    double2* y = fft(z, z == b0 ? b1 : b0, tws, M);
    // inverse = conj of the forward transform of the conjugate
    float* d0 = f.dst + ((int64_t)k * f.H + j0) * f.W;
    float* d1 = d0 + f.W;
    for (int i = threadIdx.x; i < f.W; i += kFilterThreads) {
        const double2 v = y[i];
        d0[i] = (float)v.x;
        if (has1) d1[i] = (float)-v.y;
    }
}

}  // namespace

hipError_t launch_filter(const FilterArgs& f, hipStream_t s)
{
    const int64_t blocks = (int64_t)f.n_proj * ((f.H + 1) / 2);
    const size_t lds = (size_t)(2 * f.M + f.M / 4) * sizeof(double2);
    if (blocks < 1 || blocks > 0x7fffffffLL || f.M < 4 || (f.M & (f.M - 1)) != 0 || lds > 160 * 1024)
        return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&filter_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(filter_kernel, dim3((unsigned)blocks), dim3(kFilterThreads), lds, s, f);
    return hipGetLastError();
}

}  // namespace fdk
