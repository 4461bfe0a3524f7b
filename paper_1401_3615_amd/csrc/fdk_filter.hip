// gfx950 kernel of FDK preprocessing: cosine and short-scan (Parker) weights
// and the band-limited ramp filter along detector rows (the filtering that
// precedes the paper's backprojection; its benchmark data arrive filtered,
// Sec. "RabbitCT Benchmarking Framework").
//
// One workgroup filters two rows of one projection at once as the real and
// imaginary parts of one complex sequence: the ramp kernel is real and even,
// so its spectrum is real and multiplying the packed spectrum by it filters
// both rows independently.  The linear convolution is a circular one of
// length M >= 2W - 1 (rows zero-padded; M = 2^k or 5 * 2^k, the shorter),
// computed in place in one LDS buffer: a decimation-in-frequency FFT (a
// radix-5 stage first when 5 divides M, then a radix-2 stage when the power
// of two left has an odd exponent, then radix-4 stages) leaves the spectrum
// in mixed-radix digit-reversed order, the kernel spectrum is multiplied in
// that order (the host stores it permuted), and the inverse runs the same
// stages in reverse order, each twiddling its inputs before the butterfly,
// on the conjugated data (the inverse of the stage product, up to 1/M and
// conjugation).  From M = 16 on, the passes at the ends and in the middle are
// fused: the input weighting is the first stage (whose legs from M/2 on are
// zero padding), the last forward stage, the spectrum product and the first
// inverse stage run on the four values a thread holds, and the last inverse
// stage writes the W outputs.  One buffer of M complex values plus the
// twiddles is 80 KiB at M = 4096 (two workgroups of 1024 threads per CU) and
// 50 KiB at M = 2560 (three of 640).  The weights, the permuted kernel
// spectrum (with the output gain and 1/M folded in) and the twiddles come
// from FP64 tables computed on the host.
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

constexpr int kFilterThreads = 1024;   // the largest workgroup (FFT sizes 2^k)
static_assert(kFilterThreads == 64 * kFilterWaves, "one per-wave maximum slot per wave");

// FFT sizes: 2^k (k >= 2) or 5 * 2^k (k >= 2, a radix-5 stage first).
__host__ __device__ constexpr bool filter_size_ok(int M)
{
    const int m = M % 5 == 0 ? M / 5 : M;
    return m >= 4 && (m & (m - 1)) == 0;
}

// Threads of a workgroup: 1024 for 2^k, and for 5 * 2^k one per radix-4
// butterfly (M / 4, in whole waves), so that its passes keep every thread
// busy and more workgroups share a CU (640 at M = 2560: three per CU).
__host__ __device__ constexpr int filter_threads(int M)
{
    return M % 5 != 0 ? kFilterThreads : ((M / 4 + 63) / 64 * 64 > kFilterThreads ? kFilterThreads : (M / 4 + 63) / 64 * 64);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(-2 pi i t / M) for t < M / 2 from the quarter table (beyond M / 4 by a
// quarter turn)
__device__ __forceinline__ double2 twiddle_half(const double2* tw, int t, int q)
{
    if (t < q) return tw[t];
    const double2 r = tw[t - q];
    return make_double2(r.y, -r.x);
}

// Radix-4 butterfly of the legs in place: y_r = sum_m x_m (-i)^(r m).
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3)
{
    const double2 a = make_double2(x0.x + x2.x, x0.y + x2.y), b = make_double2(x0.x - x2.x, x0.y - x2.y);
    const double2 c = make_double2(x1.x + x3.x, x1.y + x3.y);
    const double2 d = make_double2(x1.y - x3.y, x3.x - x1.x);   // -i (x1 - x3)
    x0 = make_double2(a.x + c.x, a.y + c.y);
    x1 = make_double2(b.x + d.x, b.y + d.y);
    x2 = make_double2(a.x - c.x, a.y - c.y);
    x3 = make_double2(b.x - d.x, b.y - d.y);
}

// Decimation-in-frequency stages over blocks of Bs = M, M/r1, ...: radix-2
// (when log2 M is odd) then radix-4; a stage's outputs are multiplied by
// exp(-2 pi i r i / Bs) (leg r, index i in the block's first quarter/half).
__device__ __forceinline__ void dif(double2* x, const double2* tw, int M, bool odd)
{
    const int q = M >> 2;
    int Bs = M;
    if (odd) {
        const int h = M >> 1;
        for (int j = threadIdx.x; j < h; j += (int)blockDim.x) {
            const double2 a = x[j], b = x[j + h];
            x[j] = make_double2(a.x + b.x, a.y + b.y);
            x[j + h] = cmul(make_double2(a.x - b.x, a.y - b.y), twiddle_half(tw, j, q));
        }
        __syncthreads();
        Bs = h;
    }
    for (; Bs >= 4; Bs >>= 2) {
        const int L = Bs >> 2, s = M / Bs;
        for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
            const int i = t & (L - 1), b0 = (t - i) << 2;
            double2* p = x + b0 + i;
            double2 x0 = p[0], x1 = p[L], x2 = p[2 * L], x3 = p[3 * L];
            dft4(x0, x1, x2, x3);
            const double2 w = tw[i * s];
            const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
            p[0] = x0;
            p[L] = cmul(x1, w);
            p[2 * L] = cmul(x2, w2);
            p[3 * L] = cmul(x3, w3);
        }
        __syncthreads();
    }
}

// The inverse of the dif() stage product up to a factor M, on conjugated
// data: the stages in reverse order, each multiplying its legs by the same
// twiddles first and then applying the butterfly.
__device__ __forceinline__ void dif_reverse(double2* x, const double2* tw, int M, bool odd)
{
    const int q = M >> 2;
    const int top = odd ? (M >> 1) : M;   // block size of the first radix-4 stage of dif()
    for (int Bs = 4; Bs <= top; Bs <<= 2) {
        const int L = Bs >> 2, s = M / Bs;
        for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
            const int i = t & (L - 1), b0 = (t - i) << 2;
            double2* p = x + b0 + i;
            const double2 w = tw[i * s];
            const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
            double2 x0 = p[0], x1 = cmul(p[L], w), x2 = cmul(p[2 * L], w2), x3 = cmul(p[3 * L], w3);
            dft4(x0, x1, x2, x3);
            p[0] = x0;
            p[L] = x1;
            p[2 * L] = x2;
            p[3 * L] = x3;
        }
        __syncthreads();
    }
    if (odd) {
        const int h = M >> 1;
        for (int j = threadIdx.x; j < h; j += (int)blockDim.x) {
            const double2 a = x[j], b = cmul(x[j + h], twiddle_half(tw, j, q));
            x[j] = make_double2(a.x + b.x, a.y + b.y);
            x[j + h] = make_double2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
}

// exp(-2 pi i t / M) for t < M from the quarter table (a quarter turn per
// quarter of the circle)
__device__ __forceinline__ double2 twiddle_full(const double2* tw, int t, int q)
{
    const int k = t / q;
    const double2 r = tw[t - k * q];
    switch (k) {
    case 0: return r;
    case 1: return make_double2(r.y, -r.x);
    case 2: return make_double2(-r.x, -r.y);
    default: return make_double2(-r.y, r.x);
    }
}

// Radix-5 butterfly: y_r = sum_m x_m exp(-2 pi i r m / 5), from the sums and
// differences of the legs paired around the middle.
__device__ __forceinline__ void dft5(double2 (&x)[5])
{
    constexpr double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;   // cos(2 pi / 5), cos(4 pi / 5)
    constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;    // sin(2 pi / 5), sin(4 pi / 5)
    const double2 t1 = make_double2(x[1].x + x[4].x, x[1].y + x[4].y);
    const double2 t2 = make_double2(x[2].x + x[3].x, x[2].y + x[3].y);
    const double2 t3 = make_double2(x[1].x - x[4].x, x[1].y - x[4].y);
    const double2 t4 = make_double2(x[2].x - x[3].x, x[2].y - x[3].y);
    const double2 a1 = make_double2(x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y);
    const double2 a2 = make_double2(x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y);
    const double2 b1 = make_double2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    const double2 b2 = make_double2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    x[0] = make_double2(x[0].x + t1.x + t2.x, x[0].y + t1.y + t2.y);
    // -i b = (b.y, -b.x)
    x[1] = make_double2(a1.x + b1.y, a1.y - b1.x);
    x[4] = make_double2(a1.x - b1.y, a1.y + b1.x);
    x[2] = make_double2(a2.x + b2.y, a2.y - b2.x);
    x[3] = make_double2(a2.x - b2.y, a2.y + b2.x);
}

// One radix-2 stage of dif() on blocks of Bs (after a radix-5 first stage),
// and its inverse (twiddle first, then the butterfly).
__device__ __forceinline__ void dif_radix2(double2* x, const double2* tw, int M, int Bs, bool reverse)
{
    const int q = M >> 2, L = Bs >> 1, s = M / Bs;
    for (int t = threadIdx.x; t < (M >> 1); t += (int)blockDim.x) {
        const int i = t & (L - 1), b0 = (t - i) << 1;
        double2* p = x + b0 + i;
        const double2 w = twiddle_half(tw, i * s, q);
        const double2 a = p[0];
        if (!reverse) {
            const double2 b = p[L];
            p[0] = make_double2(a.x + b.x, a.y + b.y);
            p[L] = cmul(make_double2(a.x - b.x, a.y - b.y), w);
        } else {
            const double2 b = cmul(p[L], w);
            p[0] = make_double2(a.x + b.x, a.y + b.y);
            p[L] = make_double2(a.x - b.x, a.y - b.y);
        }
    }
    __syncthreads();
}

// Radix-4 stages of dif() for block sizes hi, hi / 4, ..., lo (lo >= 4).
__device__ __forceinline__ void dif_stages(double2* x, const double2* tw, int M, int hi, int lo)
{
    const int q = M >> 2;
    for (int Bs = hi; Bs >= lo; Bs >>= 2) {
        const int L = Bs >> 2, s = M / Bs;
        for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
            const int i = t & (L - 1), b0 = (t - i) << 2;
            double2* p = x + b0 + i;
            double2 x0 = p[0], x1 = p[L], x2 = p[2 * L], x3 = p[3 * L];
            dft4(x0, x1, x2, x3);
            const double2 w = tw[i * s];
            const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
            p[0] = x0;
            p[L] = cmul(x1, w);
            p[2 * L] = cmul(x2, w2);
            p[3 * L] = cmul(x3, w3);
        }
        __syncthreads();
    }
}

// Radix-4 stages of dif_reverse() for block sizes lo, 4 lo, ..., hi.
__device__ __forceinline__ void dif_reverse_stages(double2* x, const double2* tw, int M, int lo, int hi)
{
    const int q = M >> 2;
    for (int Bs = lo; Bs <= hi; Bs <<= 2) {
        const int L = Bs >> 2, s = M / Bs;
        for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
            const int i = t & (L - 1), b0 = (t - i) << 2;
            double2* p = x + b0 + i;
            const double2 w = tw[i * s];
            const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
            double2 x0 = p[0], x1 = cmul(p[L], w), x2 = cmul(p[2 * L], w2), x3 = cmul(p[3 * L], w3);
            dft4(x0, x1, x2, x3);
            p[0] = x0;
            p[L] = x1;
            p[2 * L] = x2;
            p[3 * L] = x3;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kFilterThreads) void filter_kernel(FilterArgs f)
{
    extern __shared__ double2 lds2[];   // M complex values + M/4 twiddles
    const int pairs = (f.H + 1) >> 1;
    const int k = (int)(blockIdx.x / pairs);
    const int j0 = 2 * (int)(blockIdx.x - k * pairs), j1 = j0 + 1;
    const bool has1 = j1 < f.H;
    const int M = f.M;
    const bool odd = (__builtin_ctz(M) & 1) != 0;
    double2* x = lds2;
    double2* tws = lds2 + M;
    for (int t = threadIdx.x; t < (M >> 2); t += (int)blockDim.x) tws[t] = f.tw[t];
    const float* s0 = f.src + ((int64_t)k * f.H + j0) * f.W;
    const float* s1 = s0 + f.W;
    const double* c0 = f.wc + (int64_t)j0 * f.W;
    const double* c1 = c0 + f.W;
    const double* wp = f.wp + (int64_t)k * f.W;
    // weighted input of the two rows at i (zero padding from W on)
    auto in = [&](int i) {
        double x0 = 0.0, x1 = 0.0;
        if (i < f.W) {
            const double w = wp[i];
            x0 = (double)s0[i] * c0[i] * w;
            if (has1) x1 = (double)s1[i] * c1[i] * w;
        }
        return make_double2(x0, x1);
    };
    // the conjugate of the result: row 0 real part, row 1 minus imaginary part
    float* d0 = f.dst + ((int64_t)k * f.H + j0) * f.W;
    float* d1 = d0 + f.W;
    float m = 0.0f;
    auto out = [&](int i, double2 v) {
        const float r0 = (float)v.x, r1 = has1 ? (float)-v.y : 0.0f;
        d0[i] = r0;
        if (has1) d1[i] = r1;
        m = fmaxf(m, fmaxf(fabsf(r0), fabsf(r1)));
    };
    const int q = M >> 2, h = M >> 1;
    const bool five = M % 5 == 0;   // M = 5 * 2^k: a radix-5 stage first
    const int f5 = M / 5;
    if (M < 16 && !five) {
        // tiny transforms: every stage on its own
        for (int i = threadIdx.x; i < M; i += (int)blockDim.x) x[i] = in(i);
        __syncthreads();
        dif(x, tws, M, odd);
        for (int i = threadIdx.x; i < M; i += (int)blockDim.x) {
            const double hv = f.hs[i];
            const double2 v = x[i];
            x[i] = make_double2(v.x * hv, -v.y * hv);
        }
        __syncthreads();
        dif_reverse(x, tws, M, odd);
        for (int i = threadIdx.x; i < f.W; i += (int)blockDim.x) out(i, x[i]);
    } else {
        // first stage fused with the input weighting: the padded input is zero
        // from W <= M / 2 on, so those legs are not read (the twiddles come
        // from the global table: the LDS copy is not synced yet)
        int hi4;   // block size of the first radix-4 stage
        if (five) {
            for (int t = threadIdx.x; t < f5; t += (int)blockDim.x) {
                double2 v[5];
#pragma unroll
                for (int a = 0; a < 5; ++a) v[a] = in(t + a * f5);
                dft5(v);
                x[t] = v[0];
#pragma unroll
                for (int a = 1; a < 5; ++a) x[t + a * f5] = cmul(v[a], twiddle_full(f.tw, a * t, q));
            }
            __syncthreads();
            hi4 = f5;
            if (odd) {
                dif_radix2(x, tws, M, f5, false);
                hi4 = f5 >> 1;
            }
        } else if (odd) {
            for (int j = threadIdx.x; j < h; j += (int)blockDim.x) {
                const double2 a = in(j);
                x[j] = a;
                x[j + h] = cmul(a, twiddle_half(f.tw, j, q));
            }
            __syncthreads();
            hi4 = h;
        } else {
            for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
                const double2 x0 = in(t), x1 = in(t + q);
                const double2 d = make_double2(x1.y, -x1.x);   // -i x1
                const double2 w = f.tw[t];
                const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
                x[t] = make_double2(x0.x + x1.x, x0.y + x1.y);
                x[t + q] = cmul(make_double2(x0.x + d.x, x0.y + d.y), w);
                x[t + 2 * q] = cmul(make_double2(x0.x - x1.x, x0.y - x1.y), w2);
                x[t + 3 * q] = cmul(make_double2(x0.x - d.x, x0.y - d.y), w3);
            }
            __syncthreads();
            hi4 = q;
        }
        dif_stages(x, tws, M, hi4, 16);
        // the last forward stage (blocks of four, unit twiddles), conj(Z H) in
        // the digit-reversed order of the spectrum (hs is stored so) and the
        // first inverse stage, on the four values each thread holds
        for (int t = threadIdx.x; t < q; t += (int)blockDim.x) {
            double2* p = x + 4 * t;
            double2 v[4] = {p[0], p[1], p[2], p[3]};
            dft4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double hv = f.hs[4 * t + r];
                v[r] = make_double2(v[r].x * hv, -v[r].y * hv);
            }
            dft4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r) p[r] = v[r];
        }
        __syncthreads();
        dif_reverse_stages(x, tws, M, 16, hi4);
        // last inverse stage fused with the output: only the first W values
        if (five) {
            if (odd) dif_radix2(x, tws, M, f5, true);
            for (int t = threadIdx.x; t < f5 && t < f.W; t += (int)blockDim.x) {
                double2 v[5];
                v[0] = x[t];
#pragma unroll
                for (int a = 1; a < 5; ++a) v[a] = cmul(x[t + a * f5], twiddle_full(tws, a * t, q));
                dft5(v);
#pragma unroll
                for (int a = 0; a < 5; ++a)
                    if (t + a * f5 < f.W) out(t + a * f5, v[a]);
            }
        } else if (odd) {
            for (int j = threadIdx.x; j < f.W; j += (int)blockDim.x) {
                const double2 a = x[j], b = cmul(x[j + h], twiddle_half(tws, j, q));
                out(j, make_double2(a.x + b.x, a.y + b.y));
            }
        } else {
            for (int t = threadIdx.x; t < q && t < f.W; t += (int)blockDim.x) {
                const double2 w = tws[t];
                const double2 w2 = cmul(w, w), w3 = cmul(w2, w);
                double2 x0 = x[t], x1 = cmul(x[t + q], w), x2 = cmul(x[t + 2 * q], w2), x3 = cmul(x[t + 3 * q], w3);
                dft4(x0, x1, x2, x3);
                out(t, x0);
                if (t + q < f.W) out(t + q, x1);
            }
        }
    }
    if (f.wave_max != nullptr) {
        // the largest magnitude this wave wrote, for the packing pass that
        // follows (one plain store per wave: no barrier, no atomics)
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0)
            f.wave_max[((int64_t)k * pairs + (j0 >> 1)) * kFilterWaves + (threadIdx.x >> 6)] = m;
    }
}

// One workgroup per projection: the largest of its per-wave maxima, as bits
// (non-negative floats order like their bits).
// Slots of waves the filter's workgroups do not have (nw of kFilterWaves
// per row pair are written) are skipped.
__global__ __launch_bounds__(256) void filter_max_kernel(const float* __restrict__ wave_max, int per_proj, int nw,
                                                         unsigned* __restrict__ maxbits)
{
    __shared__ float red[4];
    const float* p = wave_max + (int64_t)blockIdx.x * per_proj;
    float m = 0.0f;
    for (int i = threadIdx.x; i < per_proj; i += 256)
        if (i % kFilterWaves < nw) m = fmaxf(m, p[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) maxbits[blockIdx.x] = __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
}

}  // namespace

hipError_t launch_filter(const FilterArgs& f, hipStream_t s)
{
    const int64_t blocks = (int64_t)f.n_proj * ((f.H + 1) / 2);
    const size_t lds = (size_t)(f.M + f.M / 4) * sizeof(double2);
    if (blocks < 1 || blocks > 0x7fffffffLL || !filter_size_ok(f.M) || 2 * f.W - 1 > f.M || lds > 160 * 1024)
        return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&filter_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(filter_kernel, dim3((unsigned)blocks), dim3(filter_threads(f.M)), lds, s, f);
    return hipGetLastError();
}

hipError_t launch_filter_max(const FilterArgs& f, unsigned* maxbits, hipStream_t s)
{
    if (f.wave_max == nullptr || f.n_proj < 1) return hipErrorInvalidValue;
    const int per = ((f.H + 1) / 2) * kFilterWaves;
    hipLaunchKernelGGL(filter_max_kernel, dim3((unsigned)f.n_proj), dim3(256), 0, s, f.wave_max, per,
                       filter_threads(f.M) / 64, maxbits);
    return hipGetLastError();
}

}  // namespace fdk
