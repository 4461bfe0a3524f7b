// gfx950 (CDNA4) kernels of the voxel-driven FDK backprojector.
//
// The arithmetic is the paper's backprojection (Sec. "RabbitCT Benchmarking
// Framework", Listing 1): voxel centre -> (u, v, w) by the 3x4 matrix,
// dehomogenise, bilinear sample with zero outside the detector, weight 1/w^2,
// accumulate.  The paper's CPU optimisations reappear in GPU form:
//   * zero-padding (Sec. "Implementation"): projections are staged into a
//     zero border so the four taps need no bounds checks; a clamp of the
//     detector coordinate keeps far-off voxels inside the border;
//   * FMA and reciprocal instead of divide (Sec. "Implementation");
//   * the line-update unit of work: one 64-lane wavefront owns 64 consecutive
//     voxels along x (coalesced volume traffic) and every lane keeps a strip of
//     voxels along y in registers for all projections, so the volume is read
//     and written once per call instead of once per projection;
//   * the paper's compact thread placement, which keeps threads that share a
//     cache on neighbouring voxels: consecutive workgroups are remapped so
//     each of the eight XCDs (each with its own L2) sweeps one contiguous slab
//     of the volume and therefore one band of detector rows.
// Projection taps are fetched with raw buffer loads: 32-bit offsets from a
// per-projection descriptor whose range check returns zero for any address
// past the staged image, so a wrong coordinate can never fault.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "fdk_internal.h"

namespace fdk {
namespace {

// Buffer descriptor word 3 for gfx9-family raw (untyped, stride 0) buffers.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// floor(x) converted to int in one VALU op (the compiler only emits the
// two-op floor + convert form).
__device__ __forceinline__ int cvt_floor(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Byte offset of tap (i0, j0) relative to an anchor: ((j0 * Wp + i0) << log2(esize)) + base.
// (The multiply-add is written out so the compiler cannot re-associate it into
// a full-rate-unfriendly 32-bit multiply of j0 by the byte pitch.)
template <typename T>
__device__ __forceinline__ uint32_t tap_offset(int i0, int j0, int wp, int base)
{
    int t, off;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(t) : "v"(j0), "s"(wp), "v"(i0));
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(off) : "v"(t), "i"(sizeof(T) == 4 ? 2 : 1), "v"(base));
    return (uint32_t)off;
}

// One detector row of the 2x2 tap block: the taps (i0, i0+1) come from one
// load at byte offset `off` (+ `soff`), and row() returns their linear
// interpolation  l + sx (r - l)  in FP32.
template <typename T> struct Taps;

template <> struct Taps<float> {
    static __device__ __forceinline__ float row(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                                float sx)
    {
        // two dword loads at off and off + 4; the compiler fuses them into one
        // buffer_load_dwordx2.  (The 64-bit load builtin is not used: this
        // compiler lowers it to a single dword load whose value fills both lanes.)
        const float a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
        const float b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 4, soff, 0));
        return fmaf(sx, b - a, a);
    }
};

// FP16 taps feed mixed-precision FMAs directly (no separate widening):
// l (1 - sx) + sx r, with both halves of one 32-bit load as operands.
template <> struct Taps<__half> {
    static __device__ __forceinline__ float row(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                                float sx)
    {
        const uint32_t t = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
        const float a = __half2float(__ushort_as_half((unsigned short)(t & 0xffffu)));
        const float b = __half2float(__ushort_as_half((unsigned short)(t >> 16)));
        return fmaf(sx, b, fmaf(-sx, a, a));
    }
};

struct bf16_t { unsigned short bits; };

template <> struct Taps<bf16_t> {
    static __device__ __forceinline__ float row(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                                float sx)
    {
        const uint32_t t = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
        const float a = __uint_as_float(t << 16), b = __uint_as_float(t & 0xffff0000u);
        return fmaf(sx, b - a, a);
    }
};

// Workgroup -> tile remap: hardware hands consecutive workgroups to the 8
// XCDs round-robin; this bijection gives XCD j the contiguous tile range
// [j*q + min(j, r), ...) so its L2 serves one slab of the volume.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    constexpr int kXcd = 8;
    const int q = nblocks / kXcd, r = nblocks % kXcd;
    const int xcd = bid % kXcd, j = bid / kXcd;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
}

struct TilePos {
    int x, y0, zl;
    double xd, yd, zd;   // centred voxel indices of the strip start
};

template <int S, int NW>
__device__ __forceinline__ TilePos tile_pos(const TileArgs& a, int tile)
{
    TilePos p;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int tx = tile % a.tiles_x;
    const int t2 = tile / a.tiles_x;
    const int ty = t2 % a.tiles_y;
    const int tz = t2 / a.tiles_y;
    p.x = tx * kWave + lane;
    p.y0 = ty * S;
    p.zl = tz * NW + wave;
    p.xd = (double)(p.x - a.ctr);
    p.yd = (double)(p.y0 - a.ctr);
    p.zd = (double)(a.z_begin + p.zl - a.ctr);
    return p;
}

// Per lane and projection: detector coordinates of the strip start in FP64,
// split into an integer anchor pixel (au, av) and FP32 remainders that are
// stepped along the strip.  u/w then only has to resolve a few pixels in
// FP32 instead of the detector half-width, which is what keeps the sampling
// position accurate to ~1e-5 px at 1248x960.
struct Strip {
    float ub, vb, wb;          // u - au w, v - av w, w at the strip start
    float du, dv, dw;          // steps per voxel along y
    float lox, hix, loy, hiy;  // clamp range of the remainders (detector border, minus anchor)
    int base;                  // byte offset of the anchor pixel in a staged image
};

template <int ES>
__device__ __forceinline__ Strip strip_setup(const double* c, const TilePos& p, const TileArgs& a, int wp)
{
    const double ub = fma(p.xd, c[0], fma(p.yd, c[1], fma(p.zd, c[2], c[3])));
    const double vb = fma(p.xd, c[4], fma(p.yd, c[5], fma(p.zd, c[6], c[7])));
    const double wb = fma(p.xd, c[8], fma(p.yd, c[9], fma(p.zd, c[10], c[11])));
    const float wf = (float)wb;
    const float rf = __builtin_amdgcn_rcpf(wf);
    // any integer near u/w will do; clamping keeps the integer math bounded
    const float fau = fminf(fmaxf(rintf((float)ub * rf), a.lo_x), a.hi_x);
    const float fav = fminf(fmaxf(rintf((float)vb * rf), a.lo_y), a.hi_y);
    const double dau = (double)fau, dav = (double)fav;
    Strip st;
    st.ub = (float)fma(-dau, wb, ub);
    st.vb = (float)fma(-dav, wb, vb);
    st.wb = wf;
    st.du = (float)fma(-dau, c[9], c[1]);
    st.dv = (float)fma(-dav, c[9], c[5]);
    st.dw = (float)c[9];
    st.lox = a.lo_x - fau;
    st.hix = a.hi_x - fau;
    st.loy = a.lo_y - fav;
    st.hiy = a.hi_y - fav;
    st.base = ((__mul24((int)fav, wp) + (int)fau) << (ES == 4 ? 2 : 1)) + (int)a.centre_bytes;
    return st;
}

// The 12 FP64 coefficients of projection k (16 are stored per projection).
struct Coef {
    double c[12];
};

__device__ __forceinline__ Coef load_coef(const double* tab, int k)
{
    Coef r;
    const double* t = tab + 16 * k;
#pragma unroll
    for (int i = 0; i < 12; ++i) r.c[i] = t[i];
    return r;
}

// Backprojection of all projections into one tile: 64 x-columns x S y-rows
// per wavefront, NW wavefronts stacked along z.
template <typename T, int S, int NW>
__device__ __forceinline__ void bp_tile(const TileArgs& a, int tile)
{
    constexpr int ES = sizeof(T);
    const TilePos p = tile_pos<S, NW>(a, tile);
    float acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0f;
    const unsigned char* img = a.proj;
    const uint32_t row = a.row_bytes;
    const int wp = (int)(a.row_bytes / ES);
    // coefficients of projection k+1 are fetched while projection k is processed
    Coef next = load_coef(a.coef, 0);
    for (int k = 0; k < a.n_proj; ++k, img += a.proj_stride) {
        const Coef cur = next;
        if (k + 1 < a.n_proj) next = load_coef(a.coef, k + 1);
        const Strip st = strip_setup<ES>(cur.c, p, a, wp);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, a.proj_bytes);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float u = fmaf((float)s, st.du, st.ub);
            const float v = fmaf((float)s, st.dv, st.vb);
            const float w = fmaf((float)s, st.dw, st.wb);
            const float r = __builtin_amdgcn_rcpf(w);
            const float dx = __builtin_amdgcn_fmed3f(u * r, st.lox, st.hix);
            const float dy = __builtin_amdgcn_fmed3f(v * r, st.loy, st.hiy);
            const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
            const uint32_t off = tap_offset<T>(cvt_floor(dx), cvt_floor(dy), wp, st.base);
            const float top = Taps<T>::row(rs, off, 0, sx);
            const float bot = Taps<T>::row(rs, off, row, sx);
            const float val = fmaf(sy, bot - top, top);
            acc[s] = fmaf(val, r * r, acc[s]);
        }
    }
    if (p.x < a.L && p.zl < a.z_count) {
        float* out = a.vol + ((int64_t)p.zl * a.L + p.y0) * a.L + p.x;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (p.y0 + s < a.L) {
                float v = acc[s] * a.out_scale;
                if (a.accumulate) v += out[(int64_t)s * a.L];
                out[(int64_t)s * a.L] = v;
            }
        }
    }
}

// Register budget: longer strips keep more taps in flight, so they are allowed
// more VGPRs (fewer resident waves per SIMD).
template <int S>
constexpr int waves_per_eu() { return S <= 4 ? 8 : S <= 8 ? 6 : S <= 16 ? 4 : 3; }

template <typename T, int S, int NW>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu<S>(), waves_per_eu<S>()))) void bp_kernel(TileArgs a)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    bp_tile<T, S, NW>(a, tile);
}

// Persistent backprojection over many scans: every workgroup pulls
// (scan, tile) items from a queue until it is empty.  Items are ordered by
// decreasing cost (projection count) on the host, so the tail is made of the
// cheapest tiles.
template <int S, int NW>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu<S>(), waves_per_eu<S>()))) void bp_batched_kernel(const TileArgs* __restrict__ scans,
                                                                const int32_t* __restrict__ item_begin,
                                                                int n_scans, unsigned* counter,
                                                                int total_items)
{
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= total_items) break;
        int lo = 0, hi = n_scans - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_begin[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const TileArgs a = scans[lo];
        const int tile = item - item_begin[lo];
        if (a.dtype == 1)
            bp_tile<__half, S, NW>(a, tile);
        else if (a.dtype == 2)
            bp_tile<bf16_t, S, NW>(a, tile);
        else
            bp_tile<float, S, NW>(a, tile);
    }
}

// Forward projection (adjoint): every voxel scatters value/w^2 onto its four
// bilinear taps in a zero-bordered FP32 accumulation image per projection,
// with the same strip coordinates as the backprojection.  Voxels whose sample
// does not touch the detector issue no atomics.
template <int S, int NW>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu<S>(), waves_per_eu<S>()))) void fp_kernel(TileArgs a)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const TilePos p = tile_pos<S, NW>(a, tile);
    float xv[S];
    const bool col_ok = p.x < a.L && p.zl < a.z_count;
    const float* in = a.vol + ((int64_t)p.zl * a.L + p.y0) * a.L + p.x;
#pragma unroll
    for (int s = 0; s < S; ++s)
        xv[s] = (col_ok && p.y0 + s < a.L) ? in[(int64_t)s * a.L] * a.out_scale : 0.0f;
    const unsigned char* img = a.proj;
    const int row = (int)a.row_bytes;
    const int wp = row / 4;
    Coef next = load_coef(a.coef, 0);
    for (int k = 0; k < a.n_proj; ++k, img += a.proj_stride) {
        const Coef cur = next;
        if (k + 1 < a.n_proj) next = load_coef(a.coef, k + 1);
        const Strip st = strip_setup<4>(cur.c, p, a, wp);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, a.proj_bytes);
        // a sample touches the detector iff the remainder lies strictly inside
        // (border + 1) on both axes
        const float in_lox = st.lox + 1.0f, in_hix = st.hix - 1.0f;
        const float in_loy = st.loy + 1.0f, in_hiy = st.hiy - 1.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float u = fmaf((float)s, st.du, st.ub);
            const float v = fmaf((float)s, st.dv, st.vb);
            const float w = fmaf((float)s, st.dw, st.wb);
            const float r = __builtin_amdgcn_rcpf(w);
            const float dx = u * r, dy = v * r;
            const bool hit = dx > in_lox && dx < in_hix && dy > in_loy && dy < in_hiy;
            if (hit && xv[s] != 0.0f) {
                const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
                const int off = (int)tap_offset<float>(cvt_floor(dx), cvt_floor(dy), wp, st.base);
                const float val = xv[s] * (r * r);
                const float b = val * sy, t = val - b;   // row weights times value
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(t - t * sx, rs, off, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(t * sx, rs, off + 4, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(b - b * sx, rs, off, row, 0);
                __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(b * sx, rs, off + 4, row, 0);
            }
        }
    }
}

// ----------------------------------------------------------------- staging
__device__ __forceinline__ void stage_row(const StageArgs& a, int64_t local_row)
{
    const int k = (int)(local_row / a.Hp);
    const int jp = (int)(local_row - (int64_t)k * a.Hp);
    const int j = jp - kPadLo;
    const bool row_in = j >= 0 && j < a.H;
    unsigned char* drow = a.dst + (uint64_t)k * a.proj_stride + (uint64_t)jp * a.Wp * a.esize;
    if (a.esize == 4) {
        const float* src = (const float*)a.src + ((int64_t)k * a.H + (row_in ? j : 0)) * a.W;
        float* d = (float*)drow;
        for (int ip = threadIdx.x; ip < a.Wp; ip += blockDim.x) {
            const int i = ip - kPadLo;
            d[ip] = (row_in && i >= 0 && i < a.W) ? src[i] : 0.0f;
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

__global__ __launch_bounds__(256) void stage_kernel(StageArgs a)
{
    stage_row(a, (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(256) void stage_batched_kernel(const StageArgs* __restrict__ stacks,
                                                            int n_stacks)
{
    const int64_t row = (int64_t)blockIdx.x;
    int lo = 0, hi = n_stacks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (stacks[mid].row_begin <= row) lo = mid; else hi = mid - 1;
    }
    const StageArgs a = stacks[lo];
    stage_row(a, row - a.row_begin);
}

// out[p][0..11] = coef64[p][0..11] / sqrt(scale_p) in FP64 (16 doubles per
// projection): folding the dequantisation factor into the matrix scales w by
// 1/sqrt(s), so the kernel's 1/w^2 weight carries s while u/w and v/w are
// untouched.
__global__ void fold_kernel(const double* __restrict__ coef64, const float* const* __restrict__ scale_ptrs,
                            double* __restrict__ out, int n_total)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_total * 16) return;
    const int p = t >> 4, c = t & 15;
    if (c >= 12) { out[t] = 0.0; return; }
    double f = 1.0;
    if (scale_ptrs != nullptr && scale_ptrs[p] != nullptr) f = 1.0 / sqrt((double)*scale_ptrs[p]);
    out[t] = coef64[p * 12 + c] * f;
}

__global__ void fold_single_kernel(const double* __restrict__ coef64, const float* __restrict__ scale,
                                   double* __restrict__ out, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 16) return;
    const int p = t >> 4, c = t & 15;
    if (c >= 12) { out[t] = 0.0; return; }
    const double f = scale != nullptr ? 1.0 / sqrt((double)scale[p]) : 1.0;
    out[t] = coef64[p * 12 + c] * f;
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

__device__ __forceinline__ float pack_scale(unsigned maxbits)
{
    const float m = __uint_as_float(maxbits);
    return m > 0.0f ? m * 0x1p-14f : 1.0f;
}

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void convert_kernel(const float* __restrict__ src, int64_t per_proj,
                                                      const unsigned* __restrict__ maxbits, int dtype,
                                                      unsigned short* __restrict__ dst)
{
    const int k = blockIdx.y;
    const float s = pack_scale(maxbits[k]);
    const float* p = src + (int64_t)k * per_proj;
    unsigned short* d = dst + (int64_t)k * per_proj;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_proj;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float q = p[i] / s;
        d[i] = dtype == 1 ? __half_as_ushort(__float2half_rn(q)) : f32_to_bf16_rne(q);
    }
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

// ----------------------------------------------------------------- dispatch
template <int S, int NW>
hipError_t bp_dispatch_t(const TileArgs& a, int nblocks, hipStream_t st)
{
    dim3 grid(nblocks), block(kWave * NW);
    if (a.dtype == 1)
        hipLaunchKernelGGL((bp_kernel<__half, S, NW>), grid, block, 0, st, a);
    else if (a.dtype == 2)
        hipLaunchKernelGGL((bp_kernel<bf16_t, S, NW>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((bp_kernel<float, S, NW>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int S, int NW>
hipError_t fp_dispatch_t(const TileArgs& a, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((fp_kernel<S, NW>), dim3(nblocks), dim3(kWave * NW), 0, st, a);
    return hipGetLastError();
}

template <int S, int NW>
hipError_t batched_dispatch_t(const TileArgs* scans, const int32_t* ib, int n, unsigned* c, int total,
                              int grid, hipStream_t st)
{
    hipLaunchKernelGGL((bp_batched_kernel<S, NW>), dim3(grid), dim3(kWave * NW), 0, st, scans, ib, n, c,
                       total);
    return hipGetLastError();
}

template <int S, int NW>
int batched_occupancy_t()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched_kernel<S, NW>, kWave * NW, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

#define FDK_TILE_TABLE(X) \
    X(2, 1) X(2, 2) X(2, 4) X(4, 1) X(4, 2) X(4, 4) X(8, 1) X(8, 2) X(8, 4) X(16, 1) X(16, 2) X(16, 4) \
    X(32, 1) X(32, 2) X(32, 4)

}  // namespace

int supported_tile(int strip, int waves)
{
#define X(S, W) if (strip == S && waves == W) return 1;
    FDK_TILE_TABLE(X)
#undef X
    return 0;
}

static int tile_blocks(const TileArgs& a) { return a.tiles_x * a.tiles_y * a.tiles_z; }

hipError_t launch_bp(const TileArgs& a, int strip, int waves, hipStream_t s)
{
    const int nb = tile_blocks(a);
#define X(S, W) if (strip == S && waves == W) return bp_dispatch_t<S, W>(a, nb, s);
    FDK_TILE_TABLE(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_fp(const TileArgs& a, int strip, int waves, hipStream_t s)
{
    const int nb = tile_blocks(a);
#define X(S, W) if (strip == S && waves == W) return fp_dispatch_t<S, W>(a, nb, s);
    FDK_TILE_TABLE(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_bp_batched(const TileArgs* scans, const int32_t* item_begin, int n_scans,
                             unsigned* counter, int total_items, int grid, int strip, int waves,
                             hipStream_t s)
{
#define X(S, W) \
    if (strip == S && waves == W) return batched_dispatch_t<S, W>(scans, item_begin, n_scans, counter, total_items, grid, s);
    FDK_TILE_TABLE(X)
#undef X
    return hipErrorInvalidValue;
}

int batched_blocks_per_cu(int strip, int waves)
{
#define X(S, W) if (strip == S && waves == W) return batched_occupancy_t<S, W>();
    FDK_TILE_TABLE(X)
#undef X
    return 0;
}

hipError_t launch_stage(const StageArgs& a, hipStream_t s)
{
    const int64_t rows = (int64_t)a.n * a.Hp;
    hipLaunchKernelGGL(stage_kernel, dim3((unsigned)rows), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stage_batched(const StageArgs* dev_args, int n_stacks, int64_t total_rows, hipStream_t s)
{
    hipLaunchKernelGGL(stage_batched_kernel, dim3((unsigned)total_rows), dim3(256), 0, s, dev_args,
                       n_stacks);
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
                       (unsigned short*)dst);
    hipLaunchKernelGGL(finalize_scale_kernel, dim3((n + 255) / 256), dim3(256), 0, s, bits, n);
    return hipGetLastError();
}

}  // namespace fdk
