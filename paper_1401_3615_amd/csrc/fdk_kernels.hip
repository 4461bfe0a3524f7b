// gfx950 (CDNA4) kernels of the voxel-driven FDK backprojector and its
// adjoint.
//
// The arithmetic is the paper's backprojection (Sec. "RabbitCT Benchmarking
// Framework", Listing 1): voxel centre -> (u, v, w) by the 3x4 matrix,
// dehomogenise, bilinear sample with zero outside the detector, weight 1/w^2,
// accumulate.  The paper's CPU optimisations reappear in GPU form:
//   * zero-padding (Sec. "Implementation"): projections are staged into a
//     zero border so the four taps need no bounds checks; a clamp of the
//     detector coordinate keeps far-off voxels inside the border;
//   * FMA and reciprocal instead of divide (Sec. "Implementation"), and one
//     reciprocal per strip where w does not change along it;
//   * the clipping mask (Sec. "Implementation"), per wavefront (ballot) and
//     per tile and projection (window prepass);
//   * the line-update unit of work becomes a 64-lane wavefront owning an 8x8
//     patch of (x, y) columns, every lane a strip of voxels along z kept in
//     registers for all projections, so the volume is written once per call;
//   * the paper's compact thread placement becomes a blocked tile order and
//     an XCD-aware block remap: the workgroups resident on one XCD (one L2)
//     cover a compact box of the volume and, with per-tile rotation of the
//     projection order, work on the same projection at the same time.
// Projection taps are fetched from LDS windows or with raw buffer loads:
// 32-bit offsets from a per-projection descriptor whose range check returns
// zero for any address past the staged image, so a wrong coordinate can never
// fault.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "fdk_internal.h"

#include <algorithm>
#include <map>
#include <type_traits>

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

// Byte offset of staged pixel (i0, j0) relative to an anchor:
// ((j0 * Wp + i0) << SHIFT) + base, SHIFT = log2(bytes per staged pixel).
// (The multiply-add is written out so the compiler cannot re-associate it into
// a quarter-rate 32-bit multiply of j0 by the byte pitch.)
template <int SHIFT>
__device__ __forceinline__ uint32_t tap_offset(int i0, int j0, int wp, int base)
{
    int t, off;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(t) : "v"(j0), "s"(wp), "v"(i0));
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(off) : "v"(t), "i"(SHIFT), "v"(base));
    return (uint32_t)off;
}

// Byte offset of column i0 relative to an anchor: (i0 << 2) + base.
__device__ __forceinline__ int col_offset(int i0, int base)
{
    int off;
    asm("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(off) : "v"(i0), "v"(base));
    return off;
}

// Byte offset of row j0 in rows ROWB bytes apart: j0 * ROWB + col, one VALU op.
template <int ROWB>
__device__ __forceinline__ uint32_t row_offset(int j0, int col)
{
    int off;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(off) : "v"(j0), "s"(ROWB), "v"(col));
    return (uint32_t)off;
}

// j0 * rowb + col, one VALU op (|j0|, rowb < 2^23, rowb in a register).
__device__ __forceinline__ uint32_t row_offset_dyn(int j0, int rowb, int col)
{
    int off;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(off) : "v"(j0), "s"(rowb), "v"(col));
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

// The bilinear sample at fraction (sx, sy) inside the 2x2 tap block whose
// first tap sits at byte offset `off`.  Three staged layouts:
//   plain (LAY 0): the detector image itself, one (unaligned) load per tap row;
//   quad  (LAY 1): every staged pixel holds its whole 2x2 block
//                  (I[j][i], I[j][i+1], I[j+1][i], I[j+1][i+1]), so one aligned
//                  load per sample fetches all four taps;
//   pair  (LAY 2): every staged pixel holds (I[j][i], I[j][i+1]), one aligned
//                  load per tap row.
template <typename T, int LAY> struct Sampler;

template <typename T> struct Sampler<T, 0> {
    static constexpr int kShift = sizeof(T) == 4 ? 2 : 1;
    static __device__ __forceinline__ float sample(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t row,
                                                   float sx, float sy)
    {
        const float top = Taps<T>::row(r, off, 0, sx);
        const float bot = Taps<T>::row(r, off, row, sx);
        return fmaf(sy, bot - top, top);
    }
};

template <> struct Sampler<float, 1> {
    static constexpr int kShift = 4;
    static __device__ __forceinline__ float sample(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t,
                                                   float sx, float sy)
    {
        // four adjacent dword loads, fused by the compiler into one dwordx4
        const float a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
        const float b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 4, 0, 0));
        const float c = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 8, 0, 0));
        const float d = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 12, 0, 0));
        const float top = fmaf(sx, b - a, a);
        const float bot = fmaf(sx, d - c, c);
        return fmaf(sy, bot - top, top);
    }
};

template <> struct Sampler<__half, 1> {
    static constexpr int kShift = 3;
    static __device__ __forceinline__ float sample(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t,
                                                   float sx, float sy)
    {
        const uint32_t t0 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        const uint32_t t1 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4, 0, 0);
        const float a = __half2float(__ushort_as_half((unsigned short)(t0 & 0xffffu)));
        const float b = __half2float(__ushort_as_half((unsigned short)(t0 >> 16)));
        const float c = __half2float(__ushort_as_half((unsigned short)(t1 & 0xffffu)));
        const float d = __half2float(__ushort_as_half((unsigned short)(t1 >> 16)));
        const float top = fmaf(sx, b, fmaf(-sx, a, a));
        const float bot = fmaf(sx, d, fmaf(-sx, c, c));
        return fmaf(sy, bot - top, top);
    }
};

template <> struct Sampler<bf16_t, 1> {
    static constexpr int kShift = 3;
    static __device__ __forceinline__ float sample(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t,
                                                   float sx, float sy)
    {
        const uint32_t t0 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        const uint32_t t1 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4, 0, 0);
        const float a = __uint_as_float(t0 << 16), b = __uint_as_float(t0 & 0xffff0000u);
        const float c = __uint_as_float(t1 << 16), d = __uint_as_float(t1 & 0xffff0000u);
        const float top = fmaf(sx, b - a, a);
        const float bot = fmaf(sx, d - c, c);
        return fmaf(sy, bot - top, top);
    }
};

// The pair layout reads the same bytes per tap row as the plain layout, but
// every load is aligned to its own size.
template <typename T> struct Sampler<T, 2> {
    static constexpr int kShift = sizeof(T) == 4 ? 3 : 2;
    static __device__ __forceinline__ float sample(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t row,
                                                   float sx, float sy)
    {
        const float top = Taps<T>::row(r, off, 0, sx);
        const float bot = Taps<T>::row(r, off, row, sx);
        return fmaf(sy, bot - top, top);
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

// Thread -> voxel mapping.  A wavefront owns an 8 x 8 patch of (x, y) columns
// and every lane a strip of S voxels along z.  The 64 voxels of one strip
// step lie in one plane, so their projections fall onto the same one or two
// detector rows within a few tens of pixels: each tap load of the wavefront
// touches only a handful of cache lines.  A workgroup holds NW patches
// (1 x 1, 2 x 1 or 2 x 2).
template <int NW> struct Patch {
    static constexpr int kBX = NW >= 16 ? 4 : NW >= 2 ? 2 : 1;
    static constexpr int kBY = NW / kBX;
};

// Tile order: tiles are numbered block by block, blocks of 8 x 8 x 4 tiles
// (x fastest inside a block, then y, then z; blocks likewise), edge blocks
// partial.  Consecutive tiles -- the ones an XCD holds at the same time --
// then form a compact box of the volume, whose projection footprint is a few
// hundred kilobytes instead of a band across the whole detector.
constexpr int kBlkX = 8, kBlkY = 8, kBlkZ = 4;

__device__ __forceinline__ void tile_coords(const TileArgs& a, int tile, int& tx, int& ty, int& tz)
{
    const int plane = a.tiles_x * a.tiles_y;
    const int kz = tile / (plane * kBlkZ);              // z block (all but the last are full)
    int t = tile - kz * plane * kBlkZ;
    const int wz = min(kBlkZ, a.tiles_z - kz * kBlkZ);
    const int jy = t / (a.tiles_x * kBlkY * wz);        // y block row inside the z block
    t -= jy * a.tiles_x * kBlkY * wz;
    const int wy = min(kBlkY, a.tiles_y - jy * kBlkY);
    const int ix = t / (kBlkX * wy * wz);               // x block inside the row
    t -= ix * kBlkX * wy * wz;
    const int wx = min(kBlkX, a.tiles_x - ix * kBlkX);
    const int lx = t % wx, t2 = t / wx;
    tx = ix * kBlkX + lx;
    ty = jy * kBlkY + t2 % wy;
    tz = kz * kBlkZ + t2 / wy;
}

struct TilePos {
    int x, y, z0;          // column and first plane (buffer-local) of the lane's strip
    double xd, yd, zd;     // centred voxel indices of the strip's anchor voxel
};

template <int S, int NW>
__device__ __forceinline__ TilePos tile_pos(const TileArgs& a, int tile)
{
    TilePos p;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    int tx, ty, tz;
    tile_coords(a, tile, tx, ty, tz);
    p.x = (tx * Patch<NW>::kBX + wave % Patch<NW>::kBX) * 8 + (lane & 7);
    p.y = (ty * Patch<NW>::kBY + wave / Patch<NW>::kBX) * 8 + (lane >> 3);
    p.z0 = tz * S;
    p.xd = (double)(p.x - a.ctr);
    p.yd = (double)(p.y - a.ctr);
    p.zd = (double)(a.z_begin + p.z0 + S / 2 - a.ctr);
    return p;
}

// Per lane and projection: detector coordinates of the strip's middle voxel
// in FP64, split into an integer anchor pixel (au, av) and FP32 remainders
// that are stepped along the strip.  u/w then only has to resolve a few
// pixels in FP32 instead of the detector half-width, which is what keeps the
// sampling position accurate to ~1e-5 px at 1248x960.
struct Strip {
    float ub, vb, wb;          // u - au w, v - av w, w at the anchor voxel
    float du, dv, dw;          // steps per voxel along z
    float fau, fav;            // anchor pixel (au, av), centred detector coordinates
    float lox, hix, loy, hiy;  // clamp range of the remainders (detector border, minus anchor)
    int base;                  // byte offset of the anchor pixel in a staged image
};

template <int SHIFT>
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
    st.du = (float)fma(-dau, c[10], c[2]);
    st.dv = (float)fma(-dav, c[10], c[6]);
    st.dw = (float)c[10];
    st.fau = fau;
    st.fav = fav;
    st.lox = a.lo_x - fau;
    st.hix = a.hi_x - fau;
    st.loy = a.lo_y - fav;
    st.hiy = a.hi_y - fav;
    st.base = ((__mul24((int)fav, wp) + (int)fau) << SHIFT) + (int)a.centre_bytes;
    return st;
}

// Clipping (the paper's clipping mask, per wavefront): does the lane's strip
// touch the detector?  The strip projects onto the segment between its first
// and last voxel (w > 0), so if that segment's bounding box misses the
// support (-1, W) x (-1, H), every tap of every voxel is zero.  A 0.01 px
// margin keeps the test conservative under FP32 rounding.
template <int S>
__device__ __forceinline__ bool strip_touches(const Strip& st)
{
    constexpr float t0 = (float)(-(S / 2)), t1 = (float)(S - 1 - S / 2);
    const float r0 = __builtin_amdgcn_rcpf(fmaf(t0, st.dw, st.wb));
    const float r1 = __builtin_amdgcn_rcpf(fmaf(t1, st.dw, st.wb));
    const float x0 = fmaf(t0, st.du, st.ub) * r0, y0 = fmaf(t0, st.dv, st.vb) * r0;
    const float x1 = fmaf(t1, st.du, st.ub) * r1, y1 = fmaf(t1, st.dv, st.vb) * r1;
    constexpr float m = 0.99f;   // support edge is border + 1, minus the margin
    return fmaxf(x0, x1) > st.lox + m && fminf(x0, x1) < st.hix - m &&
           fmaxf(y0, y1) > st.loy + m && fminf(y0, y1) < st.hiy - m;
}

// Sample coordinates along a strip.  In general 1/w is taken per voxel.  When
// w does not change along z (the projection's depth axis is perpendicular to
// the z axis, dw = 0 exactly, as for a circular orbit about z), 1/w is one
// reciprocal per strip and the remainders u/w, v/w step linearly: two FMAs per
// voxel instead of a reciprocal and two multiplies.  The choice is made per
// projection (uniform), around the strip loop.
template <bool CONSTW>
struct Walk {
    float ax, bx, ay, by, aw, bw, r2;
    // sgn: +1 or -1, the sign of the weight where it is one per strip (CONSTW)
    __device__ __forceinline__ explicit Walk(const Strip& st, float sgn = 1.0f)
    {
        if (CONSTW) {
            const float r = __builtin_amdgcn_rcpf(st.wb);
            ax = st.ub * r;
            bx = st.du * r;
            ay = st.vb * r;
            by = st.dv * r;
            r2 = r * r * sgn;
            aw = bw = 0.0f;
        } else {
            ax = st.ub;
            bx = st.du;
            ay = st.vb;
            by = st.dv;
            aw = st.wb;
            bw = st.dw;
            r2 = 0.0f;
        }
    }
    // remainders (dx, dy) and weight 1/w^2 of the voxel at offset t from the anchor
    __device__ __forceinline__ void at(float t, float& dx, float& dy, float& wgt) const
    {
        if (CONSTW) {
            dx = fmaf(t, bx, ax);
            dy = fmaf(t, by, ay);
            wgt = r2;
        } else {
            const float r = __builtin_amdgcn_rcpf(fmaf(t, bw, aw));
            dx = fmaf(t, bx, ax) * r;
            dy = fmaf(t, by, ay) * r;
            wgt = r * r;
        }
    }
};

// Runs body(std::true_type) when projection c has w constant along z, else
// body(std::false_type); the condition is uniform per projection.
template <typename F>
__device__ __forceinline__ void with_walk(const double* c, F&& body)
{
    if (c[10] == 0.0) body(std::true_type{});
    else body(std::false_type{});
}

// The 12 FP64 coefficients of projection k and the sign of its
// dequantisation factor (c[12]: +1, -1 or 0; 16 doubles are stored per
// projection).
struct Coef {
    double c[13];
};

// Coefficients of projection k, read through the scalar cache (the table is
// written before the launch and only read during it).
__device__ __forceinline__ Coef load_coef(const double* tab, int k)
{
    using DC = const __attribute__((address_space(4))) double;
    Coef r;
    DC* t = (DC*)(tab + 16 * k);
#pragma unroll
    for (int i = 0; i < 13; ++i) r.c[i] = t[i];
    return r;
}

// A projection with a negative dequantisation factor is subtracted.  Where
// the weight is one value per strip (w constant along z) its sign is folded
// into that weight; elsewhere the accumulators are negated before and after
// the projection's samples are added, under a uniform branch (volatile, so
// the compiler cannot turn it into sign flips executed for every projection).
template <int S>
__device__ __forceinline__ void negate_acc(float (&acc)[S])
{
#pragma unroll
    for (int s = 0; s < S; ++s) asm volatile("v_xor_b32 %0, 0x80000000, %0" : "+v"(acc[s]));
}

// Projection order of a tile.  Workgroups start one after another as slots
// free up, so with every tile starting at k = 0 the resident workgroups would
// be spread over all projections and share nothing in L2.  Tile t instead
// starts at k0 = t N / D (mod N), D = the number of workgroups resident at once
// on one XCD (or on the device, for the persistent kernel): a workgroup that
// starts later starts further on, and all resident workgroups then work on
// about the same projection, whose footprint they share in L2.  The sum over k
// is the same; only its FP32 rounding order depends on the tile.
struct ProjOrder {
    int k;                      // current projection
    const unsigned char* img;   // its staged image
    __device__ __forceinline__ ProjOrder(const TileArgs& a, int tile, int rot_div)
    {
        k = rot_div > 0 ? (int)(((int64_t)tile * a.n_proj / rot_div) % a.n_proj) : 0;
        img = a.proj + (uint64_t)k * a.proj_stride;
    }
    __device__ __forceinline__ void advance(const TileArgs& a)
    {
        ++k;
        img += a.proj_stride;
        if (k == a.n_proj) {
            k = 0;
            img = a.proj;
        }
    }
};

// Backprojection of all projections into one tile: NW patches of 8 x 8
// columns, S planes deep.
template <typename T, int LAY, int S, int NW>
__device__ __forceinline__ void bp_tile(const TileArgs& a, int tile, int rot_div)
{
    using Smp = Sampler<T, LAY>;
    const TilePos p = tile_pos<S, NW>(a, tile);
    float acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0f;
    const uint32_t row = a.row_bytes;
    const int wp = (int)(a.row_bytes >> Smp::kShift);
    ProjOrder po(a, tile, rot_div);
    // coefficients of the next projection are fetched while this one is processed
    Coef next = load_coef(a.coef, po.k);
    for (int n = 0; n < a.n_proj; ++n) {
        const Coef cur = next;
        const unsigned char* img = po.img;
        po.advance(a);
        if (n + 1 < a.n_proj) next = load_coef(a.coef, po.k);
        if (cur.c[12] == 0.0) continue;   // zero dequantisation factor
        const Strip st = strip_setup<Smp::kShift>(cur.c, p, a, wp);
        if (__builtin_amdgcn_ballot_w64(strip_touches<S>(st)) == 0) continue;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, a.proj_bytes);
        const bool neg = cur.c[12] < 0.0;
        with_walk(cur.c, [&](auto cw) {
            constexpr bool CW = decltype(cw)::value;
            if (!CW && neg) negate_acc(acc);
            const Walk<CW> wk(st, neg ? -1.0f : 1.0f);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                constexpr int kMid = S / 2;
                float ux, uy, wgt;
                wk.at((float)(s - kMid), ux, uy, wgt);
                const float dx = __builtin_amdgcn_fmed3f(ux, st.lox, st.hix);
                const float dy = __builtin_amdgcn_fmed3f(uy, st.loy, st.hiy);
                const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
                const uint32_t off = tap_offset<Smp::kShift>(cvt_floor(dx), cvt_floor(dy), wp, st.base);
                const float val = Smp::sample(rs, off, row, sx, sy);
                acc[s] = fmaf(val, wgt, acc[s]);
            }
            if (!CW && neg) negate_acc(acc);
        });
    }
    if (p.x < a.L && p.y < a.L) {
        const int64_t plane = (int64_t)a.L * a.L;
        float* out = a.vol + ((int64_t)p.z0 * a.L + p.y) * a.L + p.x;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (p.z0 + s < a.z_count) {
                float v = acc[s] * a.out_scale;
                if (a.accumulate) v += out[s * plane];
                out[s * plane] = v;
            }
        }
    }
}

template <int LAY, int S, int NW>
__device__ __forceinline__ void bp_tile_lay(const TileArgs& a, int tile, int rot_div)
{
    if (a.dtype == 1) bp_tile<__half, LAY, S, NW>(a, tile, rot_div);
    else if (a.dtype == 2) bp_tile<bf16_t, LAY, S, NW>(a, tile, rot_div);
    else bp_tile<float, LAY, S, NW>(a, tile, rot_div);
}

template <int S, int NW>
__device__ __forceinline__ void bp_tile_any(const TileArgs& a, int tile, int rot_div)
{
    if (a.layout == 1) bp_tile_lay<1, S, NW>(a, tile, rot_div);
    else if (a.layout == 2) bp_tile_lay<2, S, NW>(a, tile, rot_div);
    else bp_tile_lay<0, S, NW>(a, tile, rot_div);
}

// Register budget: longer strips keep more taps in flight, so they are allowed
// more VGPRs (fewer resident waves per SIMD).
template <int S>
constexpr int waves_per_eu() { return S <= 4 ? 8 : S <= 8 ? 6 : S <= 16 ? 4 : 3; }

template <typename T, int LAY, int S, int NW>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(waves_per_eu<S>(), waves_per_eu<S>()))) void bp_kernel(TileArgs a)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    bp_tile<T, LAY, S, NW>(a, tile, a.rot_div);
}

// ----------------------------------------------------------------- LDS tiles
// Window prepass: for every (tile, projection) the staged-pixel window that
// holds all taps of the tile's voxels, from the projections of the tile's
// eight corner voxels in FP64 (w > 0 on the box, so the projected box lies in
// the hull of its corners), widened by one pixel against FP32 rounding in the
// kernel.  A tile whose footprint misses the detector gets an empty window:
// the paper's clipping mask at tile granularity.
__global__ void window_kernel(TileArgs a, int strip, int bx, int by, int pitch, Win* __restrict__ out,
                              Anc* __restrict__ anc)
{
    const int64_t n_tiles = (int64_t)a.tiles_x * a.tiles_y * a.tiles_z;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles * a.n_proj) return;
    const int tile = (int)(t / a.n_proj), k = (int)(t - (int64_t)tile * a.n_proj);
    int tx, ty, tz;
    tile_coords(a, tile, tx, ty, tz);
    const int x0 = tx * 8 * bx, x1 = min(x0 + 8 * bx, a.L) - 1;
    const int y0 = ty * 8 * by, y1 = min(y0 + 8 * by, a.L) - 1;
    const int z0 = tz * strip, z1 = min(z0 + strip, a.z_count) - 1;
    const double* c = a.coef + 16 * k;
    double ilo = 1e300, ihi = -1e300, jlo = 1e300, jhi = -1e300;
    for (int q = 0; q < 8; ++q) {
        const double X = (double)(((q & 1) ? x1 : x0) - a.ctr);
        const double Y = (double)(((q & 2) ? y1 : y0) - a.ctr);
        const double Z = (double)(a.z_begin + ((q & 4) ? z1 : z0) - a.ctr);
        const double u = c[0] * X + c[1] * Y + c[2] * Z + c[3];
        const double v = c[4] * X + c[5] * Y + c[6] * Z + c[7];
        const double w = c[8] * X + c[9] * Y + c[10] * Z + c[11];
        const double ix = u / w, iy = v / w;
        ilo = fmin(ilo, ix); ihi = fmax(ihi, ix);
        jlo = fmin(jlo, iy); jhi = fmax(jhi, iy);
    }
    Win wv;
    // support of a sample, centred coordinates: (-1 - cu, W - cu) = (lo + 1, hi - 1)
    // (a projection whose dequantisation factor is zero adds nothing: empty window)
    const bool off = !(ihi > a.lo_x + 0.99 && ilo < a.hi_x - 0.99 && jhi > a.lo_y + 0.99 && jlo < a.hi_y - 0.99) ||
                     c[12] == 0.0;
    if (off || !(ilo == ilo) || !(jlo == jlo)) {
        wv.i0 = 1; wv.i1 = 0; wv.j0 = 1; wv.j1 = 0;
    } else {
        const double cil = fmin(fmax(floor(ilo) - 1.0, (double)a.lo_x), (double)a.hi_x + 1.0);
        const double cih = fmin(fmax(floor(ihi) + 2.0, (double)a.lo_x), (double)a.hi_x + 1.0);
        const double cjl = fmin(fmax(floor(jlo) - 1.0, (double)a.lo_y), (double)a.hi_y + 1.0);
        const double cjh = fmin(fmax(floor(jhi) + 2.0, (double)a.lo_y), (double)a.hi_y + 1.0);
        wv.i0 = (int16_t)((int)cil + a.cu + kPadLo);
        wv.i1 = (int16_t)((int)cih + a.cu + kPadLo);
        wv.j0 = (int16_t)((int)cjl + a.cv + kPadLo);
        wv.j1 = (int16_t)((int)cjh + a.cv + kPadLo);
    }
    out[t] = wv;
    if (anc == nullptr) return;   // launches that anchor every lane themselves
    Anc r = {};
    if (wv.i0 <= wv.i1) {
        // reference voxel: the tile's centre column (x0 + 4 bx, y0 + 4 by) at the
        // middle of its strip, as each lane's strip is anchored at its middle
        const double X = (double)(x0 + 4 * bx - a.ctr), Y = (double)(y0 + 4 * by - a.ctr);
        const double Z = (double)(a.z_begin + z0 + strip / 2 - a.ctr);
        const double u = fma(X, c[0], fma(Y, c[1], fma(Z, c[2], c[3])));
        const double v = fma(X, c[4], fma(Y, c[5], fma(Z, c[6], c[7])));
        const double w = fma(X, c[8], fma(Y, c[9], fma(Z, c[10], c[11])));
        // any integer near u/w will do; clamping keeps the integer math bounded
        const double fau = fmin(fmax(rint(u / w), (double)a.lo_x), (double)a.hi_x);
        const double fav = fmin(fmax(rint(v / w), (double)a.lo_y), (double)a.hi_y);
        r.ub = (float)fma(-fau, w, u);
        r.vb = (float)fma(-fav, w, v);
        r.wb = (float)w;
        r.ux = (float)fma(-fau, c[8], c[0]);
        r.vx = (float)fma(-fav, c[8], c[4]);
        r.wx = (float)c[8];
        r.uy = (float)fma(-fau, c[9], c[1]);
        r.vy = (float)fma(-fav, c[9], c[5]);
        r.wy = (float)c[9];
        r.du = (float)fma(-fau, c[10], c[2]);
        r.dv = (float)fma(-fav, c[10], c[6]);
        r.dw = (float)c[10];
        // anchor in window (staged-pixel) coordinates; the clamp range keeps
        // both tap columns and rows inside the window held in LDS
        const int ax = (int)fau + a.cu + kPadLo, ay = (int)fav + a.cv + kPadLo;
        const int c_lo = wv.i0 & ~3, c_hi = wv.i1 | 3;
        r.lox = (float)(c_lo - ax);
        r.hix = (float)(c_hi - 1 - ax);
        r.loy = (float)(wv.j0 - ay);
        r.hiy = (float)(wv.j1 - 1 - ay);
        r.base = ((ay - wv.j0) * pitch + (ax - c_lo)) * 4;
        r.neg = c[12] < 0.0 ? 1 : 0;
    }
    anc[t] = r;
}

// Staged pixels of one LDS chunk (4 consecutive pixels of a row, 16-byte
// aligned in the staged image): `load` returns the stored bits (Raw), `widen`
// turns them into FP32.  The two are kept apart so that a chunk prefetched
// into registers is converted only when it is stored to LDS, long after its
// load has landed (converting at once would make the wave wait for it).
template <typename T> struct Chunk;
template <> struct Chunk<float> {
    using Raw = float4;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t px)
    {
        const uint32_t o = px * 4;
        return make_float4(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0)),
                           __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, 0)),
                           __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o + 8, 0, 0)),
                           __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o + 12, 0, 0)));
    }
    static __device__ __forceinline__ float4 widen(const Raw& v) { return v; }
};
template <> struct Chunk<__half> {
    using Raw = uint2;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t px)
    {
        const uint32_t o = px * 2;
        return make_uint2((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0),
                          (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, 0));
    }
    static __device__ __forceinline__ float4 widen(const Raw& v)
    {
        return make_float4(__half2float(__ushort_as_half((unsigned short)(v.x & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(v.x >> 16))),
                           __half2float(__ushort_as_half((unsigned short)(v.y & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(v.y >> 16))));
    }
};
template <> struct Chunk<bf16_t> {
    using Raw = uint2;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t px)
    {
        const uint32_t o = px * 2;
        return make_uint2((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0),
                          (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, 0));
    }
    static __device__ __forceinline__ float4 widen(const Raw& v)
    {
        return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                           __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    }
};

// Backprojection with the projection footprint of the workgroup staged in
// LDS: per projection the tile's window is copied from the staged image with
// aligned 16-byte loads (all threads), and the four taps of every voxel are
// then read from LDS, which keeps the scattered gathers off the vector-memory
// path.
//
// The LDS window of a workgroup has rows of a fixed pitch (a compile-time
// constant, so the second tap row of a sample is an immediate offset of the
// same LDS read) and at most lds_rows<S>() rows.  Both are sized for the
// footprints of the target geometry: 0.5 mm voxels seen at up to 2.1x
// magnification on a 0.308 mm detector, i.e. up to 80 x 63 pixels for a
// 16 x 16 x 16 tile (16, 36 and 116 rows for 4, 8 and 32 planes; 44 pixels
// wide for 8-column tiles).  A larger window is gathered from the staged
// image instead.  The caps, not the largest possible window, set how many
// workgroups share a CU: for the 16 x 16 x 16 tile, 21 KiB each, seven fit in
// its 160 KiB (registers then allow six).  Rows 84 floats apart put
// vertically adjacent taps 20 banks apart.
template <int NW> constexpr int lds_pitch() { return NW == 1 ? 52 : 84; }
template <int S> constexpr int lds_rows() { return S >= 32 ? 120 : S >= 16 ? 64 : S >= 8 ? 40 : S >= 4 ? 24 : 16; }
template <int S, int NW> constexpr int lds_cap() { return lds_rows<S>() * lds_pitch<NW>(); }

// Occupancy of the LDS kernels: the workgroups whose windows fit a CU's
// 160 KiB, as waves per SIMD, capped by what the tile body's registers allow
// without spilling (from the compiled register counts): the column walk
// (CWM 3) over a staged image needs the fewest, the per-voxel walks, the
// bounds-checked fills of unpadded images (RAWOK) and the per-lane anchors
// (CWM 2) more; 16-bit windows hold half the prefetched bits (the FP16/BF16
// column walk at 16 planes fits seven waves; FP32 six), and the per-voxel
// walks on staged images fit six with one sample per group.
template <int S, int NW, int CWM, bool RAWOK, bool HALF>
constexpr int lds_vgpr_waves()
{
    if (S <= 4) return CWM == 2 || NW < 4 ? 6 : 8;
    if (CWM == 2) return S <= 8 ? 4 : 3;
    const bool lean = CWM == 3 && !RAWOK;
    if (S <= 8) return lean ? 7 : 5;
    if (S <= 16) return lean ? (HALF ? 7 : 6) : !RAWOK ? 6 : 4;
    return lean || HALF ? 4 : 3;
}
template <int S, int NW, int CWM, bool RAWOK, bool HALF>
constexpr int lds_waves_per_eu()
{
    constexpr int per_cu = (160 * 1024) / (lds_cap<S, NW>() * 4);
    constexpr int w = per_cu * NW / 4;
    constexpr int v = lds_vgpr_waves<S, NW, CWM, RAWOK, HALF>();
    return w < 1 ? 1 : (w < v ? w : v);
}

// The persistent batched kernel holds every sampling path (gathers from the
// three staged layouts, LDS windows of the three dtypes, each with the
// column walk and the per-voxel walk): its own budget, from the compiled
// register counts (32-plane strips need more than three waves allow).
template <int S> constexpr int batched_waves_per_eu() { return S <= 2 ? 5 : S <= 8 ? 4 : S <= 16 ? 3 : 2; }

// The window of one projection as the LDS tile holds it: 4-pixel chunks
// [c_lo, c_hi] x [j0, j1] of the staged image, in rows `pitch` pixels apart.
// It fits when its rows are at most `pitch` pixels and at most cap / pitch
// rows (every row's chunks are copied side by side by the workgroup's
// threads, of which there are more than chunks in a row).
struct LdsWin {
    int c_lo, c_hi, j0, j1, tw, th, nc, total;   // total = chunks = nc * th
    bool empty, fits;
    __device__ __forceinline__ LdsWin(Win w, int pitch, int cap)
    {
        empty = w.i0 > w.i1;
        c_lo = w.i0 & ~3;
        c_hi = w.i1 | 3;
        j0 = w.j0;
        j1 = w.j1;
        tw = c_hi - c_lo + 1;
        th = j1 - j0 + 1;
        nc = tw >> 2;
        total = empty ? 0 : nc * th;
        fits = !empty && tw <= pitch && th * pitch <= cap;
    }
};

// How the threads of a workgroup copy a window: a row of the LDS window has
// kCols = pitch / 4 chunk slots, and thread t always takes slot t mod kCols
// of rows r0 = t / kCols, r0 + kRows, r0 + 2 kRows, ... (kRows = threads /
// kCols rows per pass; the threads past kRows * kCols copy nothing, as do the
// slots past the window's own width).  The split is fixed per thread, so the
// only per-projection set-up is the first chunk's source pixel.  The first
// kPre chunks of a thread are prefetched into registers while the previous
// projection is sampled; rows past them are loaded after the barrier.
constexpr int kPre = 5;

template <int NW> struct FillSplit {
    static constexpr int kCols = lds_pitch<NW>() / 4;
    static constexpr int kRows = kWave * NW / kCols;
};

template <typename T>
struct Fill {
    typename Chunk<T>::Raw v[kPre];   // chunk i: row r0 + i * kRows of this thread's slot
    uint32_t px0;                     // first chunk's source pixel
    bool on;                          // the slot lies inside the window
};

// Unpadded source images (RAW): window pixel (ip, jp) is image pixel
// (ip - kPadLo, jp - kPadLo); a window that reaches past the image (edge) is
// loaded pixel by pixel, with the pixels off the image set to zero.
struct RawImg {
    int W, H;
};

__device__ __forceinline__ bool raw_edge(const LdsWin& w, const RawImg& im)
{
    return w.c_lo < kPadLo || w.c_hi - kPadLo >= im.W || w.j0 < kPadLo || w.j1 - kPadLo >= im.H;
}

// Chunk (r, cc) of a window: `px` is its first pixel in the source image
// (staged, or the caller's image for RAW scans, which are FP32).
template <typename T, bool RAWOK>
__device__ __forceinline__ typename Chunk<T>::Raw window_chunk(__amdgpu_buffer_rsrc_t rs, const LdsWin& w, int wp,
                                                               int r, int cc, uint32_t px, const RawImg& im,
                                                               bool raw, bool edge)
{
    if constexpr (RAWOK) {
        static_assert(std::is_same<T, float>::value, "unstaged images are FP32");
        if (raw && edge) {
            // a window reaching past the image: each pixel on its own (adjacent
            // b32 loads are merged into one multi-dword load, which the buffer
            // range check drops whole when it starts before the image, in-image
            // pixels included); a pixel off the image is read at the end of
            // the image's range, which the range check returns as zero
            const int j = w.j0 + r - kPadLo, i = w.c_lo - kPadLo + 4 * cc;
            const bool row = (unsigned)j < (unsigned)im.H;
            const uint32_t end = (uint32_t)__mul24(im.W, im.H) * 4u;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = row && (unsigned)(i + e) < (unsigned)im.W;
                const uint32_t o = ok ? (uint32_t)(__mul24(j, wp) + i + e) * 4u : end;
                v[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0));
            }
            return make_float4(v[0], v[1], v[2], v[3]);
        }
    }
    return Chunk<T>::load(rs, px);
}

template <typename T, int NW, bool RAWOK = false>
__device__ __forceinline__ void window_prefetch(Fill<T>& f, const LdsWin& w, __amdgpu_buffer_rsrc_t rs, int wp,
                                                int r0, int cc, const RawImg& im = RawImg{0, 0}, bool raw = false)
{
    using FS = FillSplit<NW>;
    const bool edge = RAWOK && raw && raw_edge(w, im);
    const int sh = RAWOK && raw ? kPadLo : 0;
    f.on = cc < w.nc;
    f.px0 = (uint32_t)(__mul24(w.j0 + r0 - sh, wp) + w.c_lo - sh + 4 * cc);
    // uniform step, kept opaque so that each chunk's offset is one add
    const uint32_t dpx = (uint32_t)__builtin_amdgcn_readfirstlane(__mul24(FS::kRows, wp));
#pragma unroll
    for (int i = 0; i < kPre; ++i)
        if (f.on && r0 + i * FS::kRows < w.th)
            f.v[i] = window_chunk<T, RAWOK>(rs, w, wp, r0 + i * FS::kRows, cc, f.px0 + (uint32_t)i * dpx, im, raw,
                                            edge);
}

template <typename T, int NW, bool RAWOK = false>
__device__ __forceinline__ void window_store(float* lds, const Fill<T>& f, const LdsWin& w, __amdgpu_buffer_rsrc_t rs,
                                             int wp, int r0, int cc, const RawImg& im = RawImg{0, 0},
                                             bool raw = false)
{
    using FS = FillSplit<NW>;
    constexpr int P = lds_pitch<NW>();
    if (!f.on) return;
    const int lo0 = r0 * P + 4 * cc;
#pragma unroll
    for (int i = 0; i < kPre; ++i)
        if (r0 + i * FS::kRows < w.th)
            *reinterpret_cast<float4*>(&lds[lo0 + i * FS::kRows * P]) = Chunk<T>::widen(f.v[i]);
    // rows past the prefetched ones, loaded and stored here
    int r = r0 + kPre * FS::kRows;
    if (r >= w.th) return;
    const bool edge = RAWOK && raw && raw_edge(w, im);
    const uint32_t dpx = (uint32_t)__builtin_amdgcn_readfirstlane(__mul24(FS::kRows, wp));
    uint32_t px = f.px0 + (uint32_t)kPre * dpx;
    int lo = lo0 + kPre * FS::kRows * P;
    for (; r < w.th; r += FS::kRows, px += dpx, lo += FS::kRows * P)
        *reinterpret_cast<float4*>(&lds[lo]) = Chunk<T>::widen(window_chunk<T, RAWOK>(rs, w, wp, r, cc, px, im, raw, edge));
}

// Window of (tile, projection) from the table written by window_kernel, read
// through the scalar cache (the table does not change during the launch).
__device__ __forceinline__ Win load_win(const Win* p)
{
    using U64C = const __attribute__((address_space(4))) uint64_t;
    return __builtin_bit_cast(Win, *(U64C*)p);
}

// Sampling set-up of (tile, projection) from the table written by
// window_kernel, read through the scalar cache like the windows.
__device__ __forceinline__ Anc load_anc(const Anc* p)
{
    using FC = const __attribute__((address_space(4))) uint32_t;
    struct Words {
        uint32_t v[20];
    } r;
    FC* q = (FC*)p;
#pragma unroll
    for (int i = 0; i < 20; ++i) r.v[i] = q[i];
    return __builtin_bit_cast(Anc, r);
}

// Wait for every vector-memory load of this wave (vmcnt = 0, other counters
// left alone).
__device__ __forceinline__ void wait_vm_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// One tile of the LDS backprojection; `lds` is the workgroup's 32 KiB tile.
// CWM: 3 every projection has u and w constant along z (the column walk), 1
// w constant (one 1/w per strip), 0 none is assumed to, all three from the
// tile anchors; 2 per-lane anchors from the coefficients, the walk decided
// per projection (for launches without an anchor table).
// Bilinear sample of an unpadded FP32 image at (anchor + (dx, dy)), zero off
// the detector; out of line (see the caller).
__device__ __attribute__((noinline)) float raw_sample(const unsigned char* img, uint32_t bytes, float dx, float dy,
                                                      int ia, int ja, int W, int H)
{
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, bytes);
    const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
    const int i0 = cvt_floor(dx) + ia, j0 = cvt_floor(dy) + ja;
    float tap[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + (q & 1), j = j0 + (q >> 1);
        const float v =
            __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)(j * W + i) * 4u, 0, 0));
        tap[q] = (unsigned)i < (unsigned)W && (unsigned)j < (unsigned)H ? v : 0.0f;
    }
    const float top = fmaf(sx, tap[1] - tap[0], tap[0]);
    const float bot = fmaf(sx, tap[3] - tap[2], tap[2]);
    return fmaf(sy, bot - top, top);
}

// RAWOK: the launch may hold scans whose images are unpadded (a.raw); their
// windows are filled with bounds checks and their oversized windows gathered
// with per-tap checks.
template <typename T, int S, int NW, int CWM, bool RAWOK = false>
__device__ __forceinline__ void bp_lds_tile(const TileArgs& a, int tile, int rot_div, float* lds)
{
    const TilePos p = tile_pos<S, NW>(a, tile);
    const bool raw = RAWOK && a.raw != 0;
    // image size from the clamp range of the centred coordinates (hi = size + 1 - centre)
    const RawImg im{(int)a.hi_x + a.cu - 1, (int)a.hi_y + a.cv - 1};
    float acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0f;
    const uint32_t row = a.row_bytes;
    const int wp = (int)(a.row_bytes / sizeof(T));
    const Win* wins = a.win + (int64_t)tile * a.n_proj;
    const Anc* ancs = CWM == 2 ? nullptr : a.anc + (int64_t)tile * a.n_proj;
    // the lane's column relative to the tile's reference voxel (its centre column)
    constexpr int kTX = 8 * Patch<NW>::kBX, kTY = 8 * Patch<NW>::kBY;
    const float lx = (float)(p.x % kTX - kTX / 2), ly = (float)(p.y % kTY - kTY / 2);
    ProjOrder po(a, tile, rot_div);
    // software pipeline: the window of the projection after this one is
    // loaded into registers while this one is sampled from LDS
    Fill<T> pre;
    constexpr int P = lds_pitch<NW>(), CAP = lds_cap<S, NW>();
    // this thread's chunk slot in every window copy (a thread past the last
    // full pass gets a slot past every window)
    const int fr0 = (int)threadIdx.x / FillSplit<NW>::kCols;
    const int fcc = fr0 < FillSplit<NW>::kRows ? (int)threadIdx.x % FillSplit<NW>::kCols : FillSplit<NW>::kCols;
    LdsWin wv(load_win(wins + po.k), P, CAP);
    bool big = false;
    if (wv.fits) window_prefetch<T, NW, RAWOK>(pre, wv, make_rsrc(po.img, a.proj_bytes), wp, fr0, fcc, im, raw);
    for (int n = 0; n < a.n_proj; ++n) {
        // this projection's set-up, loaded ahead of the window store so that
        // its latency passes behind the barriers: the tile's anchor record,
        // or (per-lane anchors) the projection's coefficients
        Anc an;
        Coef cur;
        if constexpr (CWM == 2) cur = load_coef(a.coef, po.k);
        else an = load_anc(ancs + po.k);
        const unsigned char* img = po.img;
        po.advance(a);
        const bool more = n + 1 < a.n_proj;
        const LdsWin wn(more ? load_win(wins + po.k) : Win{1, 0, 1, 0}, P, CAP);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, a.proj_bytes);
        const __amdgpu_buffer_rsrc_t rs_next = make_rsrc(po.img, a.proj_bytes);
        if (wv.fits) {
            __syncthreads();                                // previous projection's reads are done
            window_store<T, NW, RAWOK>(lds, pre, wv, rs, wp, fr0, fcc, im, raw);
            __syncthreads();
        }
        // every chunk of this window is in LDS by now; an unconditional wait
        // here tells the compiler so, and the next window's loads below are
        // then issued back to back (after the chunk loads and stores under
        // per-thread branches it would otherwise wait for each load before
        // reusing its registers for the next)
        wait_vm_loads();
        if (wn.fits) window_prefetch<T, NW, RAWOK>(pre, wn, rs_next, wp, fr0, fcc, im, raw);
        if (wv.fits) {
            Strip st;
            float lox, hix, loy, hiy;
            int base;
            if constexpr (CWM == 2) {
                // per-lane anchor at the strip's middle voxel; clamp so both
                // tap columns and rows stay inside the window held in LDS
                st = strip_setup<2>(cur.c, p, a, wp);
                const float ax = st.fau + (float)(a.cu + kPadLo), ay = st.fav + (float)(a.cv + kPadLo);
                lox = (float)wv.c_lo - ax;
                hix = (float)(wv.c_hi - 1) - ax;
                loy = (float)wv.j0 - ay;
                hiy = (float)(wv.j1 - 1) - ay;
                base = (((int)ay - wv.j0) * P + ((int)ax - wv.c_lo)) * 4;
            } else {
                // the tile's anchor, clamp range and LDS offset are shared by
                // all lanes; each lane adds its column's offset
                st.ub = fmaf(lx, an.ux, fmaf(ly, an.uy, an.ub));
                st.vb = fmaf(lx, an.vx, fmaf(ly, an.vy, an.vb));
                st.wb = fmaf(lx, an.wx, fmaf(ly, an.wy, an.wb));
                st.du = an.du;
                st.dv = an.dv;
                st.dw = an.dw;
                lox = an.lox;
                hix = an.hix;
                loy = an.loy;
                hiy = an.hiy;
                base = an.base;
            }
            // the four taps of a sample at LDS byte offset `off`: two reads of
            // two floats each, the second row at the immediate offset P
            auto taps = [&](uint32_t off, float& t00, float& t01, float& t10, float& t11) {
                const float* q = reinterpret_cast<const float*>(reinterpret_cast<const char*>(lds) + off);
                t00 = q[0];
                t01 = q[1];
                t10 = q[P];
                t11 = q[P + 1];
            };
            // kGrp samples at a time: their positions first, then all their
            // LDS reads, then the interpolations, so that a wave has the reads
            // of several samples in flight instead of waiting for each
            // sample's taps in turn: four when reading unpadded images in place
            // (four waves per SIMD); one on staged images, whose kernels then
            // fit six waves (the tilted 512^3 x 496 walk: 37.2 -> 32.9 ms)
            constexpr int kGrp = RAWOK ? (S < 4 ? S : 4) : 1;
            constexpr int kMid = S / 2;
            const bool neg = CWM == 2 ? cur.c[12] < 0.0 : an.neg != 0;
            const float sgn = neg ? -1.0f : 1.0f;
            auto sample = [&](auto cw) {
                constexpr bool CW = decltype(cw)::value;
                if (!CW && neg) negate_acc(acc);
                const Walk<CW> wk(st, sgn);
#pragma unroll
                for (int g = 0; g < S; g += kGrp) {
                    uint32_t off[kGrp];
                    float sx[kGrp], sy[kGrp], wgt[kGrp];
#pragma unroll
                    for (int j = 0; j < kGrp; ++j) {
                        float ux, uy;
                        wk.at((float)(g + j - kMid), ux, uy, wgt[j]);
                        const float dx = __builtin_amdgcn_fmed3f(ux, lox, hix);
                        const float dy = __builtin_amdgcn_fmed3f(uy, loy, hiy);
                        sx[j] = __builtin_amdgcn_fractf(dx);
                        sy[j] = __builtin_amdgcn_fractf(dy);
                        off[j] = tap_offset<2>(cvt_floor(dx), cvt_floor(dy), P, base);
                    }
                    float t00[kGrp], t01[kGrp], t10[kGrp], t11[kGrp];
#pragma unroll
                    for (int j = 0; j < kGrp; ++j) taps(off[j], t00[j], t01[j], t10[j], t11[j]);
#pragma unroll
                    for (int j = 0; j < kGrp; ++j) {
                        const float top = fmaf(sx[j], t01[j] - t00[j], t00[j]);
                        const float bot = fmaf(sx[j], t11[j] - t10[j], t10[j]);
                        const float val = fmaf(sy[j], bot - top, top);
                        acc[g + j] = fmaf(val, wgt[j], acc[g + j]);
                    }
                }
                if (!CW && neg) negate_acc(acc);
            };
            // u and w do not change along z (CWM 3): the lane's detector
            // column, its fraction and 1/w hold for the whole strip, and only
            // the row is stepped from voxel to voxel.  Samples per group: two
            // on staged images, whose kernels run six or seven waves per SIMD
            // (25.8 ms against 26.2 with four at 512^3 x 496), four when
            // reading unpadded images in place at four waves (the persistent
            // kernel: 11.6 ms against 12.0 with two for the 16 scans)
            auto sample_column = [&]() {
                constexpr int kColGrp = S < (RAWOK ? 4 : 2) ? S : (RAWOK ? 4 : 2);
                const float r = __builtin_amdgcn_rcpf(st.wb);
                const float dx = __builtin_amdgcn_fmed3f(st.ub * r, lox, hix);
                const float sx = __builtin_amdgcn_fractf(dx);
                const int col = col_offset(cvt_floor(dx), base);
                const float ay = st.vb * r, by = st.dv * r, r2 = r * r * sgn;
#pragma unroll
                for (int g = 0; g < S; g += kColGrp) {
                    uint32_t off[kColGrp];
                    float sy[kColGrp];
#pragma unroll
                    for (int j = 0; j < kColGrp; ++j) {
                        const float dy = __builtin_amdgcn_fmed3f(fmaf((float)(g + j - kMid), by, ay), loy, hiy);
                        sy[j] = __builtin_amdgcn_fractf(dy);
                        off[j] = row_offset<4 * P>(cvt_floor(dy), col);
                    }
                    float t00[kColGrp], t01[kColGrp], t10[kColGrp], t11[kColGrp];
#pragma unroll
                    for (int j = 0; j < kColGrp; ++j) taps(off[j], t00[j], t01[j], t10[j], t11[j]);
#pragma unroll
                    for (int j = 0; j < kColGrp; ++j) {
                        const float top = fmaf(sx, t01[j] - t00[j], t00[j]);
                        const float bot = fmaf(sx, t11[j] - t10[j], t10[j]);
                        const float val = fmaf(sy[j], bot - top, top);
                        acc[g + j] = fmaf(val, r2, acc[g + j]);
                    }
                }
            };
            if constexpr (CWM == 2) {
                with_walk(cur.c, sample);
            } else if constexpr (CWM == 3) {
                sample_column();
            } else {
                sample(std::integral_constant<bool, CWM == 1>{});
            }
        }
        big |= !wv.fits && !wv.empty;
        wv = wn;
    }
    if (big) {
        // projections whose window is larger than the LDS tile: gather from
        // the staged images (kept out of the main loop, which then has a
        // single sampling path)
        for (int k = 0; k < a.n_proj; ++k) {
            const LdsWin w(load_win(wins + k), P, CAP);
            if (w.fits || w.empty) continue;
            const Coef cur = load_coef(a.coef, k);
            const bool neg = cur.c[12] < 0.0;
            if (neg) negate_acc(acc);
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.proj + (uint64_t)k * a.proj_stride, a.proj_bytes);
            const Strip st = strip_setup<Sampler<T, 0>::kShift>(cur.c, p, a, wp);
            if (RAWOK && raw) {
                // unpadded image: every tap checked against the detector (an
                // out-of-line call per sample keeps this rare path's loads out of
                // the registers of the main loop)
                const unsigned char* img = a.proj + (uint64_t)k * a.proj_stride;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    constexpr int kMid = S / 2;
                    const float t = (float)(s - kMid);
                    const float w = fmaf(t, st.dw, st.wb);
                    const float r = __builtin_amdgcn_rcpf(w);
                    const float dx = __builtin_amdgcn_fmed3f(fmaf(t, st.du, st.ub) * r, st.lox, st.hix);
                    const float dy = __builtin_amdgcn_fmed3f(fmaf(t, st.dv, st.vb) * r, st.loy, st.hiy);
                    acc[s] = fmaf(raw_sample(img, a.proj_bytes, dx, dy, (int)st.fau + a.cu, (int)st.fav + a.cv, im.W,
                                             im.H),
                                  r * r, acc[s]);
                }
                if (neg) negate_acc(acc);
                continue;
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                constexpr int kMid = S / 2;
                const float t = (float)(s - kMid);
                const float u = fmaf(t, st.du, st.ub);
                const float v = fmaf(t, st.dv, st.vb);
                const float w = fmaf(t, st.dw, st.wb);
                const float r = __builtin_amdgcn_rcpf(w);
                const float dx = __builtin_amdgcn_fmed3f(u * r, st.lox, st.hix);
                const float dy = __builtin_amdgcn_fmed3f(v * r, st.loy, st.hiy);
                const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
                const uint32_t off = tap_offset<Sampler<T, 0>::kShift>(cvt_floor(dx), cvt_floor(dy), wp, st.base);
                const float val = Sampler<T, 0>::sample(rs, off, row, sx, sy);
                acc[s] = fmaf(val, r * r, acc[s]);
            }
            if (neg) negate_acc(acc);
        }
    }
    if (p.x < a.L && p.y < a.L) {
        const int64_t plane = (int64_t)a.L * a.L;
        float* out = a.vol + ((int64_t)p.z0 * a.L + p.y) * a.L + p.x;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (p.z0 + s < a.z_count) {
                float v = acc[s] * a.out_scale;
                if (a.accumulate) v += out[s * plane];
                out[s * plane] = v;
            }
        }
    }
}

// One LDS tile of a scan in the persistent kernel, from the scan's tile
// anchors: the column walk when its orbit keeps u and w constant along z (a
// circular orbit about z, a.const_w == 2), otherwise the per-voxel walk.
// (Two bodies per storage type: with a third, the constant-w walk, the
// persistent kernel's registers spill at 32-plane strips.)
template <typename T, int S, int NW, bool RAWOK>
__device__ __forceinline__ void lds_tile_by_walk(const TileArgs& a, int tile, int rot_div, float* lds)
{
    if (a.const_w == 2) bp_lds_tile<T, S, NW, 3, RAWOK>(a, tile, rot_div, lds);
    else bp_lds_tile<T, S, NW, 0, RAWOK>(a, tile, rot_div, lds);
}

template <typename T, int S, int NW, int CWM, bool RAWOK = false>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(lds_waves_per_eu<S, NW, CWM, RAWOK, sizeof(T) == 2>(),
                                       lds_waves_per_eu<S, NW, CWM, RAWOK, sizeof(T) == 2>()))) void bp_lds_kernel(TileArgs a)
{
    __shared__ __attribute__((aligned(16))) float lds[lds_cap<S, NW>()];
    bp_lds_tile<T, S, NW, CWM, RAWOK>(a, xcd_remap(blockIdx.x, gridDim.x), a.rot_div, lds);
}

// Persistent backprojection over many scans: every workgroup pulls
// (scan, tile) items from a queue until it is empty.  Items are ordered by
// decreasing cost (projection count) on the host, so the tail is made of the
// cheapest tiles.  CIRC: every scan is FP32, sampled from LDS windows, on a
// circular orbit about z; the kernel then holds only the column walk and
// runs at that body's occupancy.
template <int S, int NW, bool CIRC>
constexpr int batched_waves()
{
    // 32-plane strips: the queue loop's registers on top of the column walk's
    // need more than three waves allow
    return CIRC ? (S >= 32 && NW >= 4 ? 2 : lds_waves_per_eu<S, NW, 3, true, false>()) : batched_waves_per_eu<S>();
}
template <int S, int NW, bool CIRC = false>
__global__ __launch_bounds__(kWave * NW)
    __attribute__((amdgpu_waves_per_eu(batched_waves<S, NW, CIRC>(), batched_waves<S, NW, CIRC>()))) void bp_batched_kernel(const TileArgs* __restrict__ scans,
                                                                const int32_t* __restrict__ item_begin,
                                                                int n_scans, unsigned* counter,
                                                                int total_items)
{
    __shared__ int s_item;
    __shared__ __attribute__((aligned(16))) float lds[lds_cap<S, NW>()];
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
        if constexpr (CIRC) {
            bp_lds_tile<float, S, NW, 3, true>(a, tile, (int)gridDim.x, lds);
        } else if (a.layout == 3) {
            if (a.dtype == 1) lds_tile_by_walk<__half, S, NW, false>(a, tile, (int)gridDim.x, lds);
            else if (a.dtype == 2) lds_tile_by_walk<bf16_t, S, NW, false>(a, tile, (int)gridDim.x, lds);
            else lds_tile_by_walk<float, S, NW, true>(a, tile, (int)gridDim.x, lds);
        } else {
            bp_tile_any<S, NW>(a, tile, (int)gridDim.x);
        }
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
    const bool col_ok = p.x < a.L && p.y < a.L;
    const int64_t plane = (int64_t)a.L * a.L;
    const float* in = a.vol + ((int64_t)p.z0 * a.L + p.y) * a.L + p.x;
#pragma unroll
    for (int s = 0; s < S; ++s)
        xv[s] = (col_ok && p.z0 + s < a.z_count) ? in[s * plane] * a.out_scale : 0.0f;
    const unsigned char* img = a.proj;
    const int row = (int)a.row_bytes;
    const int wp = row / 4;
    Coef next = load_coef(a.coef, 0);
    for (int k = 0; k < a.n_proj; ++k, img += a.proj_stride) {
        const Coef cur = next;
        if (k + 1 < a.n_proj) next = load_coef(a.coef, k + 1);
        const Strip st = strip_setup<2>(cur.c, p, a, wp);
        if (__builtin_amdgcn_ballot_w64(strip_touches<S>(st)) == 0) continue;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(img, a.proj_bytes);
        // a sample touches the detector iff the remainder lies strictly inside
        // (border + 1) on both axes
        const float in_lox = st.lox + 1.0f, in_hix = st.hix - 1.0f;
        const float in_loy = st.loy + 1.0f, in_hiy = st.hiy - 1.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            constexpr int kMid = S / 2;
            const float t = (float)(s - kMid);
            const float u = fmaf(t, st.du, st.ub);
            const float v = fmaf(t, st.dv, st.vb);
            const float w = fmaf(t, st.dw, st.wb);
            const float r = __builtin_amdgcn_rcpf(w);
            const float dx = u * r, dy = v * r;
            const bool hit = dx > in_lox && dx < in_hix && dy > in_loy && dy < in_hiy;
            if (hit && xv[s] != 0.0f) {
                const float sx = __builtin_amdgcn_fractf(dx), sy = __builtin_amdgcn_fractf(dy);
                const int off = (int)tap_offset<2>(cvt_floor(dx), cvt_floor(dy), wp, st.base);
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

// ----------------------------------------------------------------- adjoint by detector tiles
// The forward projector as a gather over detector tiles: workgroup (tile, g)
// owns the pixels [i0, i1) x [j0, j1) of the P projections g P .. g P + P - 1,
// one FP64 LDS accumulation tile each, and writes them once: no global
// atomics.  (LDS FP64 adds also run about ten times faster than FP32 ones.)
// Its threads walk the (x, y) voxel columns.  Along a column u/w and v/w are
// monotonic in z (w > 0 on the processed planes), so the planes whose samples
// can put a tap into the tile's rows form one interval per projection, found
// from the column's two end planes and the crossing planes in closed form;
// a column whose u/w range over that interval misses the tile's columns is
// skipped for that projection.  Each voxel value in the union of the P
// intervals is read once and scattered into all P tiles: value/w^2 times each
// bilinear weight, for the taps that fall inside the tile, sampled exactly as
// the backprojection samples (FP64 anchor at the interval's middle plane,
// FP32 remainders).  The interval test runs in FP32 with a 0.05 px margin,
// which far exceeds its rounding error, so it can only admit planes that add
// nothing, never drop one that adds something.
constexpr int kBandThreads = 1024;
constexpr float kBandMargin = 0.05f;

struct BandCol {
    float za, zb;   // plane interval (centred), za > zb if empty
};

// Planes z in [zlo, zhi] (centred indices) whose sample can have a tap in the
// detector rows/columns [tlo, thi) x [slo, shi), for the column with FP32
// affine parts (u0, v0, w0) and z-coefficients (uz, vz, wz).
__device__ __forceinline__ BandCol band_interval(float u0, float v0, float w0, float uz, float vz, float wz,
                                                 float zlo, float zhi, float tlo, float thi, float slo,
                                                 float shi)
{
    BandCol r;
    const float ya = fmaf(zlo, vz, v0) * __builtin_amdgcn_rcpf(fmaf(zlo, wz, w0));
    const float yb = fmaf(zhi, vz, v0) * __builtin_amdgcn_rcpf(fmaf(zhi, wz, w0));
    const float lo = tlo - 1.0f - kBandMargin, hi = thi + kBandMargin;   // v/w in [lo, hi]
    r.za = zlo;
    r.zb = zhi;
    if (fmaxf(ya, yb) < lo || fminf(ya, yb) > hi) {
        r.za = 1.0f;
        r.zb = 0.0f;
        return r;
    }
    const bool inc = yb >= ya;
    const float sd = fabsf(vz) + fmaxf(fabsf(lo), fabsf(hi)) * fabsf(wz);
    // entry crossing (v/w = lo when increasing, hi when decreasing) inside the slab
    const float t_in = inc ? lo : hi, t_out = inc ? hi : lo;
    if (inc ? ya < lo : ya > hi) {
        const float d = fmaf(-t_in, wz, vz);
        if (fabsf(d) > 1e-4f * sd) r.za = fmaxf(zlo, ceilf(fmaf(t_in, w0, -v0) / d - 1e-3f));
    }
    if (inc ? yb > hi : yb < lo) {
        const float d = fmaf(-t_out, wz, vz);
        if (fabsf(d) > 1e-4f * sd) r.zb = fminf(zhi, floorf(fmaf(t_out, w0, -v0) / d + 1e-3f));
    }
    if (r.za <= r.zb) {
        const float xa = fmaf(r.za, uz, u0) * __builtin_amdgcn_rcpf(fmaf(r.za, wz, w0));
        const float xb = fmaf(r.zb, uz, u0) * __builtin_amdgcn_rcpf(fmaf(r.zb, wz, w0));
        if (fmaxf(xa, xb) < slo - 1.0f - kBandMargin || fminf(xa, xb) > shi + kBandMargin) {
            r.za = 1.0f;
            r.zb = 0.0f;
        }
    }
    return r;
}

// CW: w does not change along z for any projection (one 1/w per column and
// projection; the remainders step linearly).  CU (with CW): u does not change
// either (a circular orbit about z), so a column's detector column, its
// fraction and clamped tile column hold for all its planes.
template <int P, bool CW, bool CU = false>
__global__ __launch_bounds__(kBandThreads) void fp_band_kernel(BandArgs b)
{
    // P tiles of FP64 accumulators, each th x tw pixels inside a border of
    // kBandBorder pixels that absorbs the taps falling just off the tile
    extern __shared__ double lds[];
    const int groups = (b.n_proj + P - 1) / P;
    // group-minor order: concurrently resident workgroups share the planes of
    // one band of detector rows
    const int tile = (int)(blockIdx.x / groups), g = (int)(blockIdx.x - tile * groups);
    const int k0 = g * P, np = min(P, b.n_proj - k0);
    const int tu = tile % b.tiles_u, tv = tile / b.tiles_u;
    const int i0 = tu * b.tw, i1 = min(i0 + b.tw, b.W);
    const int j0 = tv * b.th, j1 = min(j0 + b.th, b.H);
    const int tw = i1 - i0, th = j1 - j0;
    // pitch (odd, so the FP64 accumulators of one column in neighbouring rows
    // fall on different LDS banks) and size of one tile
    const int tp = (tw + 2 * kBandBorder) | 1, tsz = tp * (th + 2 * kBandBorder);
    for (int e = threadIdx.x; e < P * tsz; e += kBandThreads) lds[e] = 0.0;
    __syncthreads();
    const double* coef = b.coef + 16 * k0;
    // the tile in centred detector coordinates
    const float slo = (float)(i0 - b.cu), shi = (float)(i1 - b.cu);
    const float tlo = (float)(j0 - b.cv), thi = (float)(j1 - b.cv);
    const int64_t plane = (int64_t)b.L * b.L;
    const float zlo = (float)(b.z_begin - b.ctr), zhi = (float)(b.z_begin + b.z_count - 1 - b.ctr);
    // the workgroup walks 32 x 32 blocks of columns, each wavefront a 16 x 4
    // patch of them with its long side along the volume axis that moves the
    // samples across detector columns (judged from the first projection of
    // the group at the volume centre): the 64 lanes fall on >= 16 distinct
    // columns, at most 4 deep along the ray, which keeps same-address LDS
    // atomics low
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int pa = (wave & 1) * 16 + (lane & 15), pb = (wave >> 1) * 4 + (lane >> 4);
    const bool along_x = fabs(coef[0] * coef[11] - coef[3] * coef[8]) >= fabs(coef[1] * coef[11] - coef[3] * coef[9]);
    const int px = along_x ? pa : pb, py = along_x ? pb : pa;
    const int nbx = (b.L + 31) >> 5, nblk = nbx * nbx;
    // Block pruning: a 32 x 32 block of columns whose eight corner voxels (all
    // planes of the launch) project, for every projection of the group, to a
    // box that misses the tile cannot put a tap into it (w > 0 on the box, so
    // the projected box lies in the hull of its corners).  The waves test 64
    // blocks at a time, one per lane, and walk only the blocks that can hit.
    auto block_hits = [&](int blk) {
        const int by = blk / nbx, bx = blk - by * nbx;
        const float xa = (float)(bx * 32 - b.ctr), xb = (float)(min(bx * 32 + 31, b.L - 1) - b.ctr);
        const float ya = (float)(by * 32 - b.ctr), yb = (float)(min(by * 32 + 31, b.L - 1) - b.ctr);
        constexpr float m = 1.5f;   // pixels, far above the FP32 rounding of the corner projections
        bool hit = false;
        for (int p = 0; p < np; ++p) {
            const double* c = coef + 16 * p;
            float c32[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) c32[i] = (float)c[i];
            float ulo = 3.0e38f, uhi = -3.0e38f, vlo = 3.0e38f, vhi = -3.0e38f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float X = (q & 1) ? xb : xa, Y = (q & 2) ? yb : ya, Z = (q & 4) ? zhi : zlo;
                const float u = fmaf(X, c32[0], fmaf(Y, c32[1], fmaf(Z, c32[2], c32[3])));
                const float v = fmaf(X, c32[4], fmaf(Y, c32[5], fmaf(Z, c32[6], c32[7])));
                const float r = __builtin_amdgcn_rcpf(fmaf(X, c32[8], fmaf(Y, c32[9], fmaf(Z, c32[10], c32[11]))));
                ulo = fminf(ulo, u * r);
                uhi = fmaxf(uhi, u * r);
                vlo = fminf(vlo, v * r);
                vhi = fmaxf(vhi, v * r);
            }
            hit = hit || (uhi > slo - 1.0f - m && ulo < shi + m && vhi > tlo - 1.0f - m && vlo < thi + m);
        }
        return hit;
    };
    for (int c0 = 0; c0 < nblk; c0 += kWave) {
        uint64_t todo = __builtin_amdgcn_ballot_w64(c0 + lane < nblk && block_hits(c0 + lane));
        while (todo != 0) {
            const int blk = c0 + (int)__builtin_ctzll(todo);
            todo &= todo - 1;
            const int by = blk / nbx;
            const int x = (blk - by * nbx) * 32 + px, y = by * 32 + py;
            if (x >= b.L || y >= b.L) continue;
            const float xf = (float)(x - b.ctr), yf = (float)(y - b.ctr);
            BandCol iv[P];
            float za = zhi + 1.0f, zb = zlo - 1.0f;
    #pragma unroll
            for (int p = 0; p < P; ++p) {
                iv[p].za = 1.0f;
                iv[p].zb = 0.0f;
                if (p < np) {
                    const double* c = coef + 16 * p;
                    const float u0 = fmaf(xf, (float)c[0], fmaf(yf, (float)c[1], (float)c[3]));
                    const float v0 = fmaf(xf, (float)c[4], fmaf(yf, (float)c[5], (float)c[7]));
                    const float w0 = fmaf(xf, (float)c[8], fmaf(yf, (float)c[9], (float)c[11]));
                    iv[p] = band_interval(u0, v0, w0, (float)c[2], (float)c[6], (float)c[10], zlo, zhi, tlo, thi, slo,
                                          shi);
                    if (iv[p].za <= iv[p].zb) {
                        za = fminf(za, iv[p].za);
                        zb = fmaxf(zb, iv[p].zb);
                    }
                }
            }
            if (za > zb) continue;
            const int zl_a = (int)za + b.ctr - b.z_begin, zl_b = (int)zb + b.ctr - b.z_begin;
            const int zmid = (zl_a + zl_b) >> 1;
            const double xd = (double)(x - b.ctr), yd = (double)(y - b.ctr);
            const double zd = (double)(b.z_begin + zmid - b.ctr);
            // per projection: FP64 anchor at the middle plane, FP32 remainders
            float sub[P], svb[P], swb[P], sdu[P], sdv[P];
            int oi[P], oj[P];
            float rlo[P], rhi[P];
            int rcol[P];
            double csx[P], comsx[P];   // CU: the column's fraction sx and 1 - sx
            int ccol[P];               // CU: byte offset of its clamped tile column (row 0 of the border)
    #pragma unroll
            for (int p = 0; p < P; ++p) {
                const double* c = coef + 16 * p;
                const bool on = p < np && iv[p].za <= iv[p].zb;
                const double ub = fma(xd, c[0], fma(yd, c[1], fma(zd, c[2], c[3])));
                const double vb = fma(xd, c[4], fma(yd, c[5], fma(zd, c[6], c[7])));
                const double wb = fma(xd, c[8], fma(yd, c[9], fma(zd, c[10], c[11])));
                const float wf = (float)wb;
                const float rf = __builtin_amdgcn_rcpf(wf);
                const float fau = fminf(fmaxf(rintf((float)ub * rf), -1.0e6f), 1.0e6f);
                const float fav = fminf(fmaxf(rintf((float)vb * rf), -1.0e6f), 1.0e6f);
                sub[p] = (float)fma(-(double)fau, wb, ub);
                svb[p] = (float)fma(-(double)fav, wb, vb);
                swb[p] = wf;
                sdu[p] = (float)fma(-(double)fau, c[10], c[2]);
                sdv[p] = (float)fma(-(double)fav, c[10], c[6]);
                if (CW) {   // u/w and v/w themselves step linearly; swb holds out_scale / w^2
                    sub[p] *= rf;
                    svb[p] *= rf;
                    sdu[p] *= rf;
                    sdv[p] *= rf;
                    swb[p] = rf * rf * b.out_scale;
                }
                // tap (i, j) relative to the tile; an inactive projection gets a
                // row offset that keeps every tap outside
                oi[p] = (int)fau + b.cu - i0;
                oj[p] = on ? (int)fav + b.cv - j0 : -(1 << 28);
                if (CU) {
                    const float dx = __builtin_amdgcn_fmed3f(sub[p], -2.0e6f, 2.0e6f);
                    const float fx = __builtin_amdgcn_fractf(dx);
                    csx[p] = (double)fx;
                    comsx[p] = 1.0 - (double)fx;
                    ccol[p] = (p * tsz + min(max(oi[p] + cvt_floor(dx), -kBandBorder), tw) + kBandBorder) * 8;
                }
                // the row of a sample is clamped into [-rb, th + kBandBorder - rb]
                // (rb = its anchor row from the first border row), and rb is
                // added in the byte offset: a tap pair off the tile lands in the
                // border, where both taps stay (the border is never written
                // back); an inactive projection sends every tap to border row 0
                const int rb = on ? oj[p] + kBandBorder : 0;
                rlo[p] = on ? (float)-rb : 0.0f;
                rhi[p] = on ? (float)(th + kBandBorder - rb) + 0.5f : 0.5f;
                rcol[p] = rb * tp * 8;
            }
            // voxel values four planes per step, the next four in flight while the
            // current ones are scattered (the loads are unconditional, past the
            // interval from its last plane, so the waits for them can be partial)
            const float* in = b.vol + (int64_t)y * b.L + x;
            // t: plane offset from the anchor plane
            auto scatter = [&](float t, float val0) {
                const float vs = CW ? val0 : val0 * b.out_scale;   // CW: the scale is in swb
    #pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double* c = coef + 16 * p;
                    float ux, uy, wgt;
                    if (CW) {
                        ux = fmaf(t, sdu[p], sub[p]);
                        uy = fmaf(t, sdv[p], svb[p]);
                        wgt = swb[p];
                    } else {
                        const float r = __builtin_amdgcn_rcpf(fmaf(t, (float)c[10], swb[p]));
                        ux = fmaf(t, sdu[p], sub[p]) * r;
                        uy = fmaf(t, sdv[p], svb[p]) * r;
                        wgt = r * r;
                    }
                    const float dy = __builtin_amdgcn_fmed3f(uy, rlo[p], rhi[p]);
                    const float sy = __builtin_amdgcn_fractf(dy);
                    double sx, omsx;
                    int col;
                    if (CU) {
                        sx = csx[p];
                        omsx = comsx[p];
                        col = ccol[p];
                    } else {
                        const float dx = __builtin_amdgcn_fmed3f(ux, -2.0e6f, 2.0e6f);
                        const float fx = __builtin_amdgcn_fractf(dx);
                        sx = (double)fx;
                        omsx = 1.0 - sx;
                        col = (p * tsz + min(max(oi[p] + cvt_floor(dx), -kBandBorder), tw) + kBandBorder) * 8;
                    }
                    // the four bilinear weights times the value, in FP64
                    const double val = (double)(vs * wgt);
                    const double bw = val * (double)sy, tv = val - bw;
                    char* base = reinterpret_cast<char*>(lds);
                    const uint32_t off = row_offset_dyn(cvt_floor(dy), tp * 8, col + rcol[p]);
                    double* tl = reinterpret_cast<double*>(base + off);
                    double* bl = reinterpret_cast<double*>(base + off + tp * 8);
                    __hip_atomic_fetch_add(tl, tv * omsx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(tl + 1, tv * sx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(bl, bw * omsx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(bl + 1, bw * sx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            };
            const float* pz = in + (int64_t)zl_a * plane;   // first plane of the current step
            const float* plast = in + (int64_t)zl_b * plane;
            float cur[4], nxt[4];
    #pragma unroll
            for (int j = 0; j < 4; ++j) cur[j] = *(zl_a + j <= zl_b ? pz + j * plane : plast);
            for (int z4 = zl_a; z4 <= zl_b; z4 += 4) {
                pz += 4 * plane;
    #pragma unroll
                for (int j = 0; j < 4; ++j) nxt[j] = *(z4 + 4 + j <= zl_b ? pz + j * plane : plast);
                const float tz = (float)(z4 - zmid);
    #pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (z4 + j <= zl_b && cur[j] != 0.0f) scatter(tz + (float)j, cur[j]);
    #pragma unroll
                for (int j = 0; j < 4; ++j) cur[j] = nxt[j];
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
        float* out = b.out + ((int64_t)(k0 + p) * b.H + j0) * b.W + i0;
        const double* src = lds + p * tsz + kBandBorder * tp + kBandBorder;
        for (int e = threadIdx.x; e < tw * th; e += kBandThreads) {
            const int r = e / tw, cl = e - r * tw;
            float* d = out + (int64_t)r * b.W + cl;
            const double v = src[r * tp + cl];
            *d = b.accumulate ? (float)(v + (double)*d) : (float)v;
        }
    }
}

// ----------------------------------------------------------------- dispatch
// Workgroups of `kernel` resident at once on one XCD (eight XCDs share the
// device's CUs); cached per kernel.  Callers hold the library lock.
int resident_per_xcd(const void* kernel, int threads)
{
    static std::map<const void*, int> cache;
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
        return 0;   // no rotation
    const int r = std::max(1, cus / 8) * std::max(1, per_cu);
    cache[kernel] = r;
    return r;
}

template <typename K>
void launch_rotated(K kernel, TileArgs a, dim3 grid, dim3 block, hipStream_t st)
{
    a.rot_div = resident_per_xcd(reinterpret_cast<const void*>(kernel), (int)block.x);
    hipLaunchKernelGGL(kernel, grid, block, 0, st, a);
}

template <int LAY, int S, int NW>
void bp_dispatch_q(const TileArgs& a, dim3 grid, dim3 block, hipStream_t st)
{
    if (a.dtype == 1)
        launch_rotated(bp_kernel<__half, LAY, S, NW>, a, grid, block, st);
    else if (a.dtype == 2)
        launch_rotated(bp_kernel<bf16_t, LAY, S, NW>, a, grid, block, st);
    else
        launch_rotated(bp_kernel<float, LAY, S, NW>, a, grid, block, st);
}

template <int S, int NW>
hipError_t bp_dispatch_t(const TileArgs& a, int nblocks, hipStream_t st)
{
    dim3 grid(nblocks), block(kWave * NW);
    if (a.layout == 3) {
        // the walk: 3 u and w constant along z, 1 w constant, 0 neither
        auto by_walk = [&](auto k3, auto k1, auto k0) {
            if (a.const_w == 2) launch_rotated(k3, a, grid, block, st);
            else if (a.const_w == 1) launch_rotated(k1, a, grid, block, st);
            else launch_rotated(k0, a, grid, block, st);
        };
        if (a.dtype == 1)
            by_walk(bp_lds_kernel<__half, S, NW, 3>, bp_lds_kernel<__half, S, NW, 1>, bp_lds_kernel<__half, S, NW, 0>);
        else if (a.dtype == 2)
            by_walk(bp_lds_kernel<bf16_t, S, NW, 3>, bp_lds_kernel<bf16_t, S, NW, 1>,
                    bp_lds_kernel<bf16_t, S, NW, 0>);
        else if (a.raw)
            by_walk(bp_lds_kernel<float, S, NW, 3, true>, bp_lds_kernel<float, S, NW, 1, true>,
                    bp_lds_kernel<float, S, NW, 0, true>);
        else
            by_walk(bp_lds_kernel<float, S, NW, 3>, bp_lds_kernel<float, S, NW, 1>, bp_lds_kernel<float, S, NW, 0>);
        return hipGetLastError();
    }
    if (a.layout == 1)
        bp_dispatch_q<1, S, NW>(a, grid, block, st);
    else if (a.layout == 2)
        bp_dispatch_q<2, S, NW>(a, grid, block, st);
    else
        bp_dispatch_q<0, S, NW>(a, grid, block, st);
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
                              int grid, bool circ, hipStream_t st)
{
    if (circ)
        hipLaunchKernelGGL((bp_batched_kernel<S, NW, true>), dim3(grid), dim3(kWave * NW), 0, st, scans, ib, n,
                           c, total);
    else
        hipLaunchKernelGGL((bp_batched_kernel<S, NW, false>), dim3(grid), dim3(kWave * NW), 0, st, scans, ib, n,
                           c, total);
    return hipGetLastError();
}

template <int S, int NW>
int batched_occupancy_t(bool circ)
{
    int nb = 0;
    const hipError_t e =
        circ ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched_kernel<S, NW, true>, kWave * NW, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched_kernel<S, NW, false>, kWave * NW, 0);
    return e == hipSuccess ? nb : 0;
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

hipError_t launch_bp_lanes(const TileArgs& a, hipStream_t s)
{
    launch_rotated(bp_lds_kernel<float, 16, 4, 2, true>, a, dim3(tile_blocks(a)), dim3(kWave * 4), s);
    return hipGetLastError();
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
                             unsigned* counter, int total_items, int grid, int strip, int waves, int circular,
                             hipStream_t s)
{
#define X(S, W)                                                                                              \
    if (strip == S && waves == W)                                                                            \
        return batched_dispatch_t<S, W>(scans, item_begin, n_scans, counter, total_items, grid, circular != 0, s);
    FDK_TILE_TABLE(X)
#undef X
    return hipErrorInvalidValue;
}

int batched_blocks_per_cu(int strip, int waves, int circular)
{
#define X(S, W) if (strip == S && waves == W) return batched_occupancy_t<S, W>(circular != 0);
    FDK_TILE_TABLE(X)
#undef X
    return 0;
}

hipError_t launch_window(const TileArgs& a, int strip, int waves, Win* out, Anc* anc, hipStream_t s)
{
    const int bx = waves >= 16 ? 4 : waves >= 2 ? 2 : 1, by = waves / bx;   // as Patch<NW>
    const int64_t n = (int64_t)a.tiles_x * a.tiles_y * a.tiles_z * a.n_proj;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int pitch = waves == 1 ? lds_pitch<1>() : lds_pitch<4>();
    hipLaunchKernelGGL(window_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, strip, bx, by, pitch, out, anc);
    return hipGetLastError();
}

int supported_band_group(int p) { return p == 1 || p == 2 || p == 4 || p == 8; }

template <int P, bool CW, bool CU = false>
static hipError_t launch_band(const BandArgs& b, hipStream_t s)
{
    const int groups = (b.n_proj + P - 1) / P;
    const int64_t blocks = (int64_t)b.tiles_u * b.tiles_v * groups;
    const size_t lds = (size_t)P * ((b.tw + 2 * kBandBorder) | 1) * (b.th + 2 * kBandBorder) * sizeof(double);
    if (blocks > 0x7fffffffLL || lds > (size_t)kBandCap * sizeof(double)) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fp_band_kernel<P, CW, CU>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kBandCap * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((fp_band_kernel<P, CW, CU>), dim3((unsigned)blocks), dim3(kBandThreads), lds, s, b);
    return hipGetLastError();
}

hipError_t launch_fp_band(const BandArgs& b, int group, hipStream_t s)
{
    const int cw = b.const_w;   // 2: u and w constant along z, 1: w, 0: neither
    switch (group) {
    case 1: return cw == 2 ? launch_band<1, true, true>(b, s) : cw ? launch_band<1, true>(b, s) : launch_band<1, false>(b, s);
    case 2: return cw == 2 ? launch_band<2, true, true>(b, s) : cw ? launch_band<2, true>(b, s) : launch_band<2, false>(b, s);
    case 4: return cw == 2 ? launch_band<4, true, true>(b, s) : cw ? launch_band<4, true>(b, s) : launch_band<4, false>(b, s);
    case 8: return cw == 2 ? launch_band<8, true, true>(b, s) : cw ? launch_band<8, true>(b, s) : launch_band<8, false>(b, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fdk
