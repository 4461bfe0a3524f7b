// gfx950 kernels around the backprojection: staging of projection stacks
// into the zero-bordered layouts the backprojection samples (the paper's
// zero-padding, Sec. "Implementation"), folding of per-projection FP16/BF16
// scales into the FP64 coefficients, FP16/BF16 packing, and small fill /
// copy-back kernels.  All of them are memory-bound copies.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "fdk_internal.h"

namespace fdk {
namespace {

// ----------------------------------------------------------------- staging
// One padded row of the staged layout.  Pixel (ip, jp) of the padded image
// is the detector pixel (ip - 2, jp - 2), zero outside the detector; the quad
// layout stores the 2x2 block starting at (ip, jp) instead of one pixel.
template <typename E>
__device__ __forceinline__ E padded_px(const E* img, const StageArgs& a, int ip, int jp)
{
    const int i = ip - kPadLo, j = jp - kPadLo;
    return (i >= 0 && i < a.W && j >= 0 && j < a.H) ? img[(int64_t)j * a.W + i] : E(0);
}

__device__ __forceinline__ void stage_row(const StageArgs& a, int64_t local_row)
{
    const int k = (int)(local_row / a.Hp);
    const int jp = (int)(local_row - (int64_t)k * a.Hp);
    const int j = jp - kPadLo;
    const bool row_in = j >= 0 && j < a.H;
    if (a.layout == 1) {
        if (a.esize == 4) {
            const float* img = (const float*)a.src + (int64_t)k * a.H * a.W;
            float4* d = (float4*)(a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * 16);
            for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x)
                d[ip] = make_float4(padded_px(img, a, ip, jp), padded_px(img, a, ip + 1, jp),
                                    padded_px(img, a, ip, jp + 1), padded_px(img, a, ip + 1, jp + 1));
        } else {
            const unsigned short* img = (const unsigned short*)a.src + (int64_t)k * a.H * a.W;
            uint2* d = (uint2*)(a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * 8);
            for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x) {
                const uint32_t t0 = (uint32_t)padded_px(img, a, ip, jp) |
                                    ((uint32_t)padded_px(img, a, ip + 1, jp) << 16);
                const uint32_t t1 = (uint32_t)padded_px(img, a, ip, jp + 1) |
                                    ((uint32_t)padded_px(img, a, ip + 1, jp + 1) << 16);
                d[ip] = make_uint2(t0, t1);
            }
        }
        return;
    }
    if (a.layout == 2) {
        if (a.esize == 4) {
            const float* img = (const float*)a.src + (int64_t)k * a.H * a.W;
            float2* d = (float2*)(a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * 8);
            for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x)
                d[ip] = make_float2(padded_px(img, a, ip, jp), padded_px(img, a, ip + 1, jp));
        } else {
            const unsigned short* img = (const unsigned short*)a.src + (int64_t)k * a.H * a.W;
            uint32_t* d = (uint32_t*)(a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * 4);
            for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x)
                d[ip] = (uint32_t)padded_px(img, a, ip, jp) | ((uint32_t)padded_px(img, a, ip + 1, jp) << 16);
        }
        return;
    }
    unsigned char* drow = a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * a.esize;
    if (a.esize == 4) {
        const float* src = (const float*)a.src + ((int64_t)k * a.H + (row_in ? j : 0)) * a.W;
        float* d = (float*)drow;
        if ((a.W & 1) == 0 && (reinterpret_cast<uintptr_t>(a.src) & 7) == 0) {
            // four staged pixels per store (rows start 32-byte aligned); their
            // sources are two 8-byte aligned pairs (kPadLo = 2), each loaded
            // whole when it lies on the row
            float4* d4 = (float4*)d;
            for (int c = threadIdx.x; c < (a.Wp >> 2); c += blockDim.x) {
                const int i = 4 * c - kPadLo;
                float2 lo = make_float2(0.0f, 0.0f), hi = make_float2(0.0f, 0.0f);
                if (row_in) {   // W even: a pair is wholly on the row or wholly off it
                    if (i >= 0 && i < a.W) lo = *(const float2*)(src + i);
                    if (i + 2 < a.W) hi = *(const float2*)(src + i + 2);
                }
                d4[c] = make_float4(lo.x, lo.y, hi.x, hi.y);
            }
        } else {
            for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x) {
                const int i = ip - kPadLo;
                d[ip] = (row_in && i >= 0 && i < a.W) ? src[i] : 0.0f;
            }
        }
    } else {
        const unsigned short* src =
            (const unsigned short*)a.src + ((int64_t)k * a.H + (row_in ? j : 0)) * a.W;
        unsigned short* d = (unsigned short*)drow;
        for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x) {
            const int i = ip - kPadLo;
            d[ip] = (row_in && i >= 0 && i < a.W) ? src[i] : (unsigned short)0;
        }
    }
}

// Every workgroup stages kRowsPerBlock consecutive padded rows (one row is
// only ~1300 pixels, too little work to amortise a workgroup's launch).
constexpr int kRowsPerBlock = 8;

__global__ __launch_bounds__(256) void stage_kernel(StageArgs a)
{
    const int64_t rows = (int64_t)a.n * a.Hp;
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    for (int64_t row = r0; row < r0 + kRowsPerBlock && row < rows; ++row) stage_row(a, row);
}

// Rows of many stacks, numbered stack after stack (StageArgs::row_begin).
__global__ __launch_bounds__(256) void stage_batched_kernel(const StageArgs* __restrict__ stacks,
                                                            int n_stacks, int64_t total_rows)
{
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    for (int64_t row = r0; row < r0 + kRowsPerBlock && row < total_rows; ++row) {
        int lo = 0, hi = n_stacks - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (stacks[mid].row_begin <= row) lo = mid; else hi = mid - 1;
        }
        const StageArgs a = stacks[lo];
        stage_row(a, row - a.row_begin);
    }
}

// Dequantisation factor s of a projection, folded into its coefficients
// (16 doubles per projection): |s| scales w by 1/sqrt|s|, so the kernel's
// 1/w^2 weight carries |s| while u/w and v/w are untouched, and slot 12 holds
// the sign, +1 or -1, or 0 for s = 0 (the projection then adds nothing and is
// skipped).  Slots 13..15 are zero.
__device__ __forceinline__ double fold_entry(const double* coef64, int p, int c, const float* sp)
{
    const double s = sp != nullptr ? (double)*sp : 1.0;
    if (c == 12) return s > 0.0 ? 1.0 : s < 0.0 ? -1.0 : 0.0;
    if (c > 12) return 0.0;
    const double f = (s > 0.0 || s < 0.0) ? 1.0 / sqrt(fabs(s)) : 1.0;
    return coef64[p * 12 + c] * f;
}

__global__ void fold_kernel(const double* __restrict__ coef64, const float* const* __restrict__ scale_ptrs,
                            double* __restrict__ out, int n_total)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_total * 16) return;
    const int p = t >> 4, c = t & 15;
    out[t] = fold_entry(coef64, p, c, scale_ptrs != nullptr ? scale_ptrs[p] : nullptr);
}

__global__ void fold_single_kernel(const double* __restrict__ coef64, const float* __restrict__ scale,
                                   double* __restrict__ out, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 16) return;
    const int p = t >> 4, c = t & 15;
    out[t] = fold_entry(coef64, p, c, scale != nullptr ? scale + p : nullptr);
}

__global__ void reset_counter_kernel(unsigned* c) { *c = 0u; }

__global__ void fill_kernel(float* __restrict__ p, uint64_t n, float value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// out[k][j][i] (+)= padded[k][j + 2][i + 2]
__global__ __launch_bounds__(256) void unstage_kernel(const float* __restrict__ padded, float* __restrict__ out,
                                                      int W, int H, int Wp, uint64_t stride_elems,
                                                      int accumulate)
{
    const int64_t row = blockIdx.x;           // k * H + j
    const int k = (int)(row / H), j = (int)(row - (int64_t)k * H);
    const float* src = padded + (uint64_t)k * stride_elems + (uint64_t)(j + kPadLo) * Wp + kPadLo;
    float* dst = out + row * W;
    for (int i = threadIdx.x; i < W; i += blockDim.x) {
        const float v = src[i];
        dst[i] = accumulate ? dst[i] + v : v;
    }
}

// ----------------------------------------------------------------- packing
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ src, int64_t per_proj,
                                                     unsigned* __restrict__ maxbits)
{
    const int k = blockIdx.y;
    const float* p = src + (int64_t)k * per_proj;
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_proj;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(p[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        atomicMax(maxbits + k, __float_as_uint(m));   // non-negative floats order like their bits
    }
}

// scale_out: null (a later pass turns maxbits into the scales in place), or
// where block 0 of each projection writes its scale
__global__ __launch_bounds__(256) void convert_kernel(const float* __restrict__ src, int64_t per_proj,
                                                      const unsigned* __restrict__ maxbits, int dtype,
                                                      unsigned short* __restrict__ dst, float* scale_out)
{
    const int k = blockIdx.y;
    const float s = pack_scale(maxbits[k]);
    if (scale_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) scale_out[k] = s;
    const float* p = src + (int64_t)k * per_proj;
    unsigned short* d = dst + (int64_t)k * per_proj;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if ((per_proj & 7) == 0 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0) {
        // eight values per thread: two 16-byte loads, one 16-byte store
        const float4* p4 = reinterpret_cast<const float4*>(p);
        uint4* d8 = reinterpret_cast<uint4*>(d);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (per_proj >> 3); i += stride) {
            const float4 a = p4[2 * i], b = p4[2 * i + 1];
            auto two = [&](float x, float y) {
                return (uint32_t)pack_value(x, s, dtype) | ((uint32_t)pack_value(y, s, dtype) << 16);
            };
            d8[i] = make_uint4(two(a.x, a.y), two(a.z, a.w), two(b.x, b.y), two(b.z, b.w));
        }
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_proj; i += stride)
        d[i] = pack_value(p[i], s, dtype);
}

__global__ void finalize_scale_kernel(unsigned* __restrict__ maxbits, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        const float s = pack_scale(maxbits[k]);
        reinterpret_cast<float*>(maxbits)[k] = s;
    }
}

__global__ void zero_u32_kernel(unsigned* p, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0u;
}

// Row bands of a device-resident stack (out-of-core form): band row r of
// projection k is source row j0[k] + r.  One workgroup per band row.
template <typename U>
__global__ __launch_bounds__(256) void band_gather_kernel(const U* __restrict__ src, U* __restrict__ dst,
                                                          const int32_t* __restrict__ j0, int H, int rows,
                                                          int row_units)
{
    const int64_t row = blockIdx.x;
    const int k = (int)(row / rows), r = (int)(row - (int64_t)k * rows);
    const U* from = src + ((int64_t)k * H + j0[k] + r) * row_units;
    U* to = dst + row * row_units;
    for (int i = threadIdx.x; i < row_units; i += blockDim.x) to[i] = from[i];
}

}  // namespace

hipError_t launch_band_gather(const void* src, void* dst, const int32_t* j0, int n, int H, int rows,
                              int64_t row_bytes, hipStream_t s)
{
    const int64_t blocks = (int64_t)n * rows;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const uintptr_t a = (uintptr_t)src | (uintptr_t)dst | (uintptr_t)row_bytes;
    if (a % 16 == 0)
        band_gather_kernel<uint4><<<(unsigned)blocks, 256, 0, s>>>((const uint4*)src, (uint4*)dst, j0, H, rows,
                                                                   (int)(row_bytes / 16));
    else if (a % 4 == 0)
        band_gather_kernel<uint32_t><<<(unsigned)blocks, 256, 0, s>>>((const uint32_t*)src, (uint32_t*)dst, j0, H,
                                                                      rows, (int)(row_bytes / 4));
    else
        band_gather_kernel<uint16_t><<<(unsigned)blocks, 256, 0, s>>>((const uint16_t*)src, (uint16_t*)dst, j0, H,
                                                                      rows, (int)(row_bytes / 2));
    return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& a, hipStream_t s)
{
    const int64_t rows = (int64_t)a.n * a.Hp;
    hipLaunchKernelGGL(stage_kernel, dim3((unsigned)((rows + kRowsPerBlock - 1) / kRowsPerBlock)), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_stage_batched(const StageArgs* dev_args, int n_stacks, int64_t total_rows, hipStream_t s)
{
    if (n_stacks <= 0 || total_rows <= 0) return hipSuccess;   // nothing to stage
    hipLaunchKernelGGL(stage_batched_kernel,
                       dim3((unsigned)((total_rows + kRowsPerBlock - 1) / kRowsPerBlock)), dim3(256), 0, s,
                       dev_args, n_stacks, total_rows);
    return hipGetLastError();
}

hipError_t launch_fold(const double* coef64, const float* const* scale_ptrs, double* coef32, int n_total,
                       hipStream_t s)
{
    const int threads = n_total * 16;
    hipLaunchKernelGGL(fold_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, coef64, scale_ptrs,
                       coef32, n_total);
    return hipGetLastError();
}

hipError_t launch_fold_single(const double* coef64, const float* scale, double* coef32, int n,
                              hipStream_t s)
{
    const int threads = n * 16;
    hipLaunchKernelGGL(fold_single_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, coef64, scale,
                       coef32, n);
    return hipGetLastError();
}

hipError_t launch_reset_counter(unsigned* counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, uint64_t n, float value, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t launch_unstage_add(const float* padded, float* out, int n, int W, int H, int Wp,
                              uint64_t stride_elems, int accumulate, hipStream_t s)
{
    const int64_t rows = (int64_t)n * H;
    hipLaunchKernelGGL(unstage_kernel, dim3((unsigned)rows), dim3(256), 0, s, padded, out, W, H, Wp,
                       stride_elems, accumulate);
    return hipGetLastError();
}

hipError_t launch_pack_known_max(const float* src, int n, int W, int H, int dtype, void* dst, const unsigned* maxbits,
                                 float* scale, hipStream_t s)
{
    const int64_t per = (int64_t)W * H;
    int bx = (int)((per + 256 * 16 - 1) / (256 * 16));
    if (bx < 1) bx = 1;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(convert_kernel, dim3(bx, n), dim3(256), 0, s, src, per, maxbits, dtype, (unsigned short*)dst,
                       scale);
    return hipGetLastError();
}

hipError_t launch_pack(const float* src, int n, int W, int H, int dtype, void* dst, float* scale,
                       hipStream_t s)
{
    const int64_t per = (int64_t)W * H;
    unsigned* bits = reinterpret_cast<unsigned*>(scale);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, bits, n);
    int bx = (int)((per + 256 * 16 - 1) / (256 * 16));
    if (bx < 1) bx = 1;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(absmax_kernel, dim3(bx, n), dim3(256), 0, s, src, per, bits);
    hipLaunchKernelGGL(convert_kernel, dim3(bx, n), dim3(256), 0, s, src, per, bits, dtype,
                       (unsigned short*)dst, nullptr);
    hipLaunchKernelGGL(finalize_scale_kernel, dim3((n + 255) / 256), dim3(256), 0, s, bits, n);
    return hipGetLastError();
}

}  // namespace fdk
