// Internal interface between the host layer (fdk_api.cpp) and the gfx950
// kernels (fdk_kernels.hip).  Not installed; the public ABI is include/fdk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace fdk {

// Zero border around every staged projection: two columns/rows before the
// detector and three after.  A detector coordinate clamped to [-2, W+1] then
// always addresses a 2x2 tap block inside the staged image, and every tap that
// lies off the detector reads a stored zero (the paper's zero-padding).
constexpr int kPadLo = 2;
constexpr int kPadHi = 3;
constexpr int kWave = 64;

// Window of staged (zero-bordered) pixels that one workgroup tile needs from
// one projection, inclusive bounds; i0 > i1 means every tap is off the
// detector and the projection is skipped for that tile (clipping).
struct Win {
    int16_t i0, i1, j0, j1;
};

// Per (tile, projection) sampling set-up of the LDS backprojection, computed
// by the window prepass in FP64 and rounded once: the remainders u - au w,
// v - av w and w at the tile's reference voxel (its centre column, at the
// middle of its strip of planes) for an integer anchor pixel (au, av) near
// that voxel's projection, their steps per voxel along x, y and z, and, in
// the tile's window, the clamp range of the remainders and the byte offset
// of the anchor pixel.  A lane then only adds its column's offset from the
// reference voxel in FP32; its remainders stay a few tens of pixels times w.
// The sign of the projection's dequantisation factor rides along (its
// magnitude is folded into w; a zero factor gives an empty window).
struct Anc {
    float ub, vb, wb;
    float ux, vx, wx;
    float uy, vy, wy;
    float du, dv, dw;
    float lox, hix, loy, hiy;
    int32_t base;
    int32_t neg;       // 1: the projection's dequantisation factor is negative
    int32_t pad[2];
};
static_assert(sizeof(Anc) == 80, "anchor records are 20 dwords");

// Per-scan arguments of the backprojection / forward-projection tile body.
// Coordinates inside the kernels are centred: the voxel index is offset by
// `ctr` on every axis and the detector column/row by (cu, cv) = (W/2, H/2),
// both integers, so floor() and the fraction are unchanged while the FP32
// magnitudes of u, v, x, y, z halve.
struct TileArgs {
    const unsigned char* proj;   // staged padded projections (or adjoint accumulation buffer)
    const double* coef;          // n_proj x 16 doubles: rows u, v, w of the composed matrix
                                 // (1/sqrt|s| of the dequantisation factor s folded in), then
                                 // sign(s) in {+1, -1, 0}
    float* vol;                  // volume buffer (planes z_begin .. z_begin + z_count)
    uint64_t proj_stride;        // bytes between consecutive staged projections
    int32_t n_proj;
    int32_t L;
    int32_t z_begin;
    int32_t z_count;
    int32_t ctr;                 // voxel index centre offset
    uint32_t row_bytes;          // staged row pitch in bytes
    uint32_t centre_bytes;       // byte offset of detector pixel (cu, cv) in a staged image
    uint32_t proj_bytes;         // bytes of one staged image (buffer range limit)
    float lo_x, hi_x, lo_y, hi_y;  // clamp range of centred coordinates ([-2, W+1] - cu ...)
    float out_scale;             // power-of-two renormalisation of the 1/w^2 weight
    int32_t accumulate;
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t dtype;               // fdk_dtype of the staged images
    int32_t layout;              // 0 plain, 1 quad, 2 pair (global gathers), 3 LDS tiles
    const Win* win;              // layout 3: n_tiles x n_proj windows
    const Anc* anc;              // layout 3: n_tiles x n_proj sampling set-ups (order of win)
    int32_t cu, cv;              // integer detector centre (W/2, H/2)
    int32_t rot_div;             // projection-order rotation divisor (0: every tile starts at k = 0)
    int32_t const_w;             // 1: w does not depend on z for any projection of the launch,
                                 // 2: neither u nor w does
    int32_t raw;                 // 1: proj holds the caller's FP32 images unpadded (row pitch W,
                                 //    W even; LDS layout only), windows read with bounds checks
};

// Forward projection by detector-tile ownership: one workgroup per
// (detector tile, group of projections) accumulates every voxel's
// contribution to its tiles in LDS and writes them once.
struct BandArgs {
    const double* coef;          // n_proj x 16 doubles (centred composition, power-of-two scaled)
    const float* vol;            // planes z_begin .. z_begin + z_count
    float* out;                  // n_proj x H x W
    int32_t n_proj, L, z_begin, z_count, ctr;
    int32_t W, H, cu, cv;
    int32_t tw, th, tiles_u, tiles_v;
    float out_scale;
    int32_t accumulate;
    int32_t const_w;             // 1: w does not depend on z for any projection, 2: neither u nor w
};

// group = projections per workgroup (1, 2, 4 or 8); P (tw + 2 kBandBorder)
// (th + 2 kBandBorder) <= kBandCap
hipError_t launch_fp_band(const BandArgs& b, int group, hipStream_t s);
int supported_band_group(int group);
constexpr int kBandCap = 20480;   // FP64 accumulators of one workgroup's detector tiles (160 KiB of LDS)
constexpr int kBandBorder = 2;    // border pixels around each tile that absorb off-tile taps

// FP16/BF16 storage of projections: scale = max|p| / 2^14 (1 for an
// all-zero projection), from the bits of max|p| (non-negative floats order
// like their bits); stored value = round_to_nearest_even(p / scale).
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

// dtype 1: FP16, 2: BF16
__device__ __forceinline__ unsigned short pack_value(float p, float scale, int dtype)
{
    const float q = p / scale;
    return dtype == 1 ? __half_as_ushort(__float2half_rn(q)) : f32_to_bf16_rne(q);
}

// FDK preprocessing: weights and ramp filtering of every row (fdk_filter.hip).
struct FilterArgs {
    const float* src;            // n_proj x H x W line integrals
    float* dst;                  // n_proj x H x W filtered (FP32)
    const double* wc;            // H x W cosine weights
    const double* wp;            // n_proj x W short-scan weights
    const double* hs;            // M: real spectrum of the circular ramp kernel x gain / M, in the
                                 // order the in-place FFT leaves the spectrum
    const double2* tw;           // M / 4 twiddles exp(-2 pi i t / M)
    int32_t n_proj, W, H, M;     // M: 2^k or 5 * 2^k >= 2 W - 1, 1.25 M FP64 complex fit 80 KiB of LDS
    float* wave_max;             // or null: max |dst| of each wave's share of a row pair, at
                                 // ((k * pairs) + pair) * kFilterWaves + wave, pairs = (H + 1) / 2
};
constexpr int kFilterWaves = 16;   // waves per filter workgroup
hipError_t launch_filter(const FilterArgs& f, hipStream_t s);
// maxbits[k] = bits of the largest wave_max entry of projection k (k < f.n_proj)
hipError_t launch_filter_max(const FilterArgs& f, unsigned* maxbits, hipStream_t s);

// Iterative solvers (fdk_iter.hip).  Reductions write one FP64 partial per
// workgroup of a fixed grid of kRedBlocks; scalar_kernel combines them and
// applies an op to the solver state `st` (slots kSt*).
constexpr int kRedBlocks = 1024;
enum { kStGamma = 0, kStAlpha = 1, kStBeta = 2, kStQQ = 3, kStRowMax = 4, kStColMax = 5, kStSlots = 8 };
enum { kOpStore = 0, kOpAlpha = 1, kOpBeta = 2, kOpHist = 3, kOpMax = 4 };
hipError_t launch_sumsq(const float* a, int64_t n, double* part, hipStream_t s);
hipError_t launch_max(const float* a, int64_t n, double* part, hipStream_t s);
hipError_t launch_scalar(const double* part, double* st, double* hist, int op, int slot, hipStream_t s);
hipError_t launch_cgls_update(float* x, const float* d, int64_t nv, float* r, const float* q, int64_t np,
                              const double* st, double* part, hipStream_t s);
hipError_t launch_cgls_direction(float* d, const float* sv, int64_t n, const double* st, hipStream_t s);
hipError_t launch_residual(float* r, const float* p, const float* w, int64_t n, double* part, hipStream_t s);
hipError_t launch_sirt_update(float* x, const float* t, const float* c, int64_t n, double lambda, int nonneg,
                              hipStream_t s);
hipError_t launch_inv_floor(float* a, int64_t n, const double* st, int slot, double floor_rel, hipStream_t s);

// One projection stack to stage into the padded layout.
struct StageArgs {
    const void* src;             // [n][H][W] elements of esize bytes
    unsigned char* dst;          // staged images, proj_stride apart
    uint64_t proj_stride;        // bytes
    int32_t n, W, H, Wp, Hp;
    int32_t esize;               // 2 or 4 (bytes of one source pixel)
    int32_t layout;              // 0: plain, 1: quad (2x2 block per staged pixel)
    int64_t row_begin;           // first global row index of this stack (batched staging)
};

// Launch wrappers (fdk_kernels.hip).  All return the launch's hipError_t.
hipError_t launch_stage(const StageArgs& a, hipStream_t s);
hipError_t launch_stage_batched(const StageArgs* dev_args, int n_stacks, int64_t total_rows,
                                hipStream_t s);
hipError_t launch_fold(const double* coef64, const float* const* scale_ptrs, double* out,
                       int n_total, hipStream_t s);
hipError_t launch_fold_single(const double* coef64, const float* scale, double* out, int n,
                              hipStream_t s);
hipError_t launch_bp(const TileArgs& a, int strip, int waves, hipStream_t s);
// The LDS backprojection of the caller's unpadded FP32 images with per-lane
// anchors (no sampling set-up table), tile 16 planes x 4 waves; a.win holds
// the windows of that tile shape.
hipError_t launch_bp_lanes(const TileArgs& a, hipStream_t s);
hipError_t launch_fp(const TileArgs& a, int strip, int waves, hipStream_t s);
// circular: every scan is FP32, sampled from LDS windows, with const_w == 2
// (the persistent kernel that holds only the column walk)
hipError_t launch_bp_batched(const TileArgs* dev_scans, const int32_t* dev_item_begin, int n_scans,
                             unsigned* dev_counter, int total_items, int grid, int strip, int waves,
                             int circular, hipStream_t s);
hipError_t launch_reset_counter(unsigned* counter, hipStream_t s);
hipError_t launch_fill(float* p, uint64_t n, float value, hipStream_t s);
// rows [j0[k], j0[k] + rows) of each of n device images of H rows of row_bytes
// (even) bytes, packed into n x rows rows
hipError_t launch_band_gather(const void* src, void* dst, const int32_t* j0, int n, int H, int rows,
                              int64_t row_bytes, hipStream_t s);
hipError_t launch_unstage_add(const float* padded, float* out, int n, int W, int H, int Wp,
                              uint64_t stride_elems, int accumulate, hipStream_t s);
hipError_t launch_pack(const float* src, int n, int W, int H, int dtype, void* dst, float* scale,
                       hipStream_t s);
// FP16/BF16 packing of n projections whose max |src| bits are known (maxbits):
// dst and scale as fdk_pack_projections
hipError_t launch_pack_known_max(const float* src, int n, int W, int H, int dtype, void* dst, const unsigned* maxbits,
                                 float* scale, hipStream_t s);
// Windows (out) and sampling set-ups (anc, n_tiles x n_proj each; null: none,
// for launches whose lanes anchor themselves from the coefficients) of an LDS
// launch with the given tile shape.
hipError_t launch_window(const TileArgs& a, int strip, int waves, Win* out, Anc* anc, hipStream_t s);
int supported_tile(int strip, int waves);
int batched_blocks_per_cu(int strip, int waves, int circular);

}  // namespace fdk
