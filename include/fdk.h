/*
 * fdk.h -- C ABI of the MI355X (gfx950) voxel-driven FDK backprojection library.
 *
 * The operation (Hofmann et al., "Performance Engineering for a Medical Imaging
 * Application on the Intel Xeon Phi Accelerator", Sec. "RabbitCT Benchmarking
 * Framework", Listing 1 and the text after it):
 *
 *   for every voxel (x, y, z) of an L^3 grid and every projection k:
 *     X          = O + (x, y, z) * MM           voxel centre in world coordinates (mm)
 *     (u, v, w)  = A_k (X, 1)                   3x4 projection matrix of projection k
 *     val        = bilinear sample of I_k at (u/w, v/w), zero off the detector
 *     V(x, y, z) += val / w^2                   inverse-square weight
 *
 * with floor() for the integer part of the detector coordinates, a tap (i, j)
 * on the detector iff 0 <= i < width and 0 <= j < height, pixel (i, j) centred
 * on integer coordinates, and zero applied per tap.
 *
 * Layouts (all row-major, C order):
 *   volume      float32, index ((z - z_begin) * L + y) * L + x  (x fastest)
 *   projections [n_proj][height][width], column index (u) fastest
 *   matrices    float64, 12 per projection, A[r][c] at r * 4 + c.  (The paper's
 *               listing indexes the same matrix column-major, A[r + 3c].)
 *
 * Ownership and concurrency:
 *   - the caller owns every buffer; the library never frees or retains them;
 *   - host arrays (matrices, descriptors) are read before the call returns;
 *   - device pointers belong to the current HIP device;
 *   - work is enqueued on the given HIP stream (NULL = the null stream) and
 *     the call returns without waiting for it; results are valid once the
 *     stream has been synchronised.  The host does wait in these cases only:
 *       . a workspace buffer grows (the first call needing a larger one):
 *         freeing the old buffer synchronises the device;
 *       . a projector call whose geometry is not among the 64 most recently
 *         used ones recycles the oldest coefficient table: the host waits
 *         for the queued work that last read it (usually long finished);
 *       . fdk_backproject_batched with descriptors not in its graph cache
 *         uploads its tables and builds the graph (waits for the stream;
 *         evicting one of the 4 cached graphs, or growing its staging
 *         buffer, synchronises the device);
 *       . fdk_filter_projections with a geometry not among the 4 most
 *         recent ones uploads its tables (waits for the stream; evicting
 *         one synchronises the device);
 *       . fdk_backproject_streamed: pageable host memory is copied
 *         synchronously by the runtime; with a device stack the host waits
 *         until the previous streamed call has read its band table;
 *       . fdk_cgls / fdk_sirt as the projectors, plus their own workspace;
 *       . fdk_release_workspace and fdk_profile_read.
 *   - the library keeps one device workspace per device (projection staging,
 *     coefficient tables, counters).  Calls issued on different streams of one
 *     device are ordered by the library (a call on a new stream first waits for
 *     the previous stream's work to finish) so they never share workspace
 *     concurrently.
 *
 * Errors: every argument is validated on the host before anything is
 * enqueued; on error nothing is enqueued, outputs are untouched, the status is
 * returned and fdk_last_error() (thread-local) holds a description.
 */
#ifndef FDK_H
#define FDK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDK_ABI_VERSION 1

typedef enum fdk_status {
    FDK_OK = 0,
    FDK_E_INVALID_ARG = -1,  /* null pointer, bad size, non-finite geometry, overflow */
    FDK_E_GEOMETRY = -2,     /* w <= 0 at a corner voxel of the processed region */
    FDK_E_UNSUPPORTED = -3,  /* unknown dtype, device is not gfx950 */
    FDK_E_NOMEM = -4,        /* workspace allocation failed */
    FDK_E_DEVICE = -5        /* a HIP runtime call failed */
} fdk_status;

typedef enum fdk_dtype {
    FDK_F32 = 0,   /* IEEE binary32 */
    FDK_F16 = 1,   /* IEEE binary16 */
    FDK_BF16 = 2   /* bfloat16 */
} fdk_dtype;

/* Tuning slots besides the three projection dtypes (fdk_set_tile and the
 * tuning table): the forward projector, and the tile shape of the batched
 * persistent launch. */
#define FDK_TUNE_ADJOINT 3
#define FDK_TUNE_BATCHED 4

/* The volume grid (paper: edge L, voxel pitch MM, origin O).  The buffer
 * passed with it holds the planes [z_begin, z_begin + z_count), which lets a
 * large volume be processed as z-slabs. */
typedef struct fdk_volume {
    int32_t L;             /* voxels per edge, 1 .. 32768 */
    int32_t z_begin;       /* first plane held by the buffer, 0 <= z_begin < L */
    int32_t z_count;       /* planes held, 1 <= z_count <= L - z_begin */
    int32_t reserved;      /* must be 0 */
    double voxel_mm;       /* voxel pitch MM > 0 */
    double origin_mm[3];   /* world position (mm) of the centre of voxel (0, 0, 0) */
} fdk_volume;

/* A projection stack: one 3x4 matrix and one width x height image per
 * projection.  With a scale array, projection k contributes scale[k] times
 * its stored values (for FDK_F16 / FDK_BF16 data packed by
 * fdk_pack_projections, the stored value is p / scale[k], so the product is
 * p again).  Any finite factor is exact up to rounding: a zero factor adds
 * nothing, a negative one subtracts the projection; a non-finite factor gives
 * unspecified values in the voxels that projection reaches.  The factors are
 * read on the device, by the call's own work on its stream.
 * fdk_forwardproject uses only n_proj, width, height and mats. */
typedef struct fdk_projections {
    int32_t n_proj;        /* N >= 1 */
    int32_t width;         /* W >= 1, row length (u, fastest) */
    int32_t height;        /* H >= 1, rows (v) */
    int32_t dtype;         /* fdk_dtype of data */
    const double* mats;    /* HOST, n_proj * 12 float64, row-major per projection */
    const void* data;      /* DEVICE, [n_proj][height][width] of dtype */
    const float* scale;    /* DEVICE, n_proj float32 factors (finite, any sign), or NULL for 1 */
} fdk_projections;

/* One scan of a batch. */
typedef struct fdk_scan {
    fdk_volume vol;
    fdk_projections proj;
    float* volume;         /* DEVICE output, z_count * L * L float32 */
} fdk_scan;

/*
 * Backprojection (the paper's Listing 1, all projections in one call):
 * volume[v] = (accumulate ? volume[v] : 0) + sum_k val_k(v) / w_k(v)^2.
 * Defined by: Sec. "RabbitCT Benchmarking Framework", Listing 1; the paper's
 * zero-padding and clipping optimisations (Sec. "Implementation") change only
 * how it is computed.
 *   vol        grid description (host)
 *   proj       projection stack (host struct; data and scale on the device)
 *   volume     DEVICE, z_count * L * L float32, written (or added to)
 *   accumulate 0: overwrite, 1: add to the existing contents
 *   stream     hipStream_t or NULL
 * FDK_E_GEOMETRY if w <= 0 at any corner voxel of the processed planes for any
 * projection (w is affine in the voxel position, so this covers the region).
 */
fdk_status fdk_backproject(const fdk_volume* vol, const fdk_projections* proj,
                           float* volume, int accumulate, void* stream);

/*
 * fdk_backproject for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, computed without any allocation.  Its working memory (the
 * coefficient tables and the LDS window table of one z-chunk) is a 32 MiB
 * array in the library's device code, one copy per device, held until the
 * process ends; the call allocates nothing, neither on the device nor through
 * a library.  FP32 projections only, read in place.
 *   vol, proj, volume, accumulate, stream  as for fdk_backproject
 * Limits (FDK_E_INVALID_ARG beyond them, nothing enqueued): n_proj <= 4096;
 * ceil(L/16)^2 * n_proj * 8 bytes <= 31 MiB (one window table entry per
 * 16x16x16 tile and projection, for 16 planes: L = 512 allows 4000
 * projections); width * height * 4 < 4 GiB.  FDK_E_UNSUPPORTED for FP16/BF16
 * data.  The matrices are copied from the host by the call (from pageable
 * memory, so the host may wait for the stream).  Every call on one device
 * shares that device's array and leaves its contents behind; the library
 * orders its own calls (a call on a new stream first waits for the previous
 * call's work), and calls made around that ordering, e.g. from two processes
 * sharing the library's code object or work captured into graphs that are
 * replayed concurrently, would race on it.
 */
fdk_status fdk_backproject_noalloc(const fdk_volume* vol, const fdk_projections* proj, float* volume,
                                   int accumulate, void* stream);

/*
 * Voxel-driven forward projection, the exact adjoint B^T of fdk_backproject
 * (the transpose of the linear map of Listing 1): for every voxel v and
 * projection k the value volume[v] / w^2 is scattered onto the four bilinear
 * taps that lie on the detector, with the bilinear weights of the sample the
 * backprojection would take there.
 *   vol        grid description (host)
 *   volume     DEVICE, z_count * L * L float32 input
 *   geom       n_proj, width, height, mats (data, dtype, scale are ignored)
 *   proj_out   DEVICE, n_proj * height * width float32, written (or added to)
 *   accumulate 0: overwrite, 1: add
 *   stream     hipStream_t or NULL
 * With the default tiling each detector pixel is summed in FP64 in LDS and
 * rounded to FP32 once; the order of the FP64 additions varies from run to
 * run, so results are reproducible to FP64 rounding before that final
 * rounding.  Layout 0 accumulates with FP32 atomics in global memory.
 * FDK_E_GEOMETRY as for fdk_backproject.
 */
fdk_status fdk_forwardproject(const fdk_volume* vol, const float* volume,
                              const fdk_projections* geom, float* proj_out,
                              int accumulate, void* stream);

/*
 * Many independent backprojections (scans of uneven size, each with its own
 * grid, projections, matrices and output) in one persistent launch that pulls
 * (scan, tile) work items from a queue.  The launch sequence is captured once
 * into a HIP graph, cached by the content of the descriptors (pointers, sizes,
 * matrices, scales), and replayed on later calls with the same content.
 * Same per-scan semantics and errors as fdk_backproject; a failing scan's
 * index is reported by fdk_last_error().
 *   scans      HOST array of n_scans descriptors
 *   n_scans    1 .. 4096
 */
fdk_status fdk_backproject_batched(const fdk_scan* scans, int32_t n_scans,
                                   int accumulate, void* stream);

/*
 * Projection storage conversion (FP32 -> FP16 or BF16) with a per-projection
 * scale: scale_out[k] = max_ij |src[k][j][i]| / 2^14 (1 if the projection is
 * all zero), dst[k][j][i] = round_to_nearest_even(src / scale_out[k]).
 *   src        DEVICE, n_proj * height * width float32
 *   dtype      FDK_F16 or FDK_BF16
 *   dst        DEVICE, n_proj * height * width 16-bit values
 *   scale_out  DEVICE, n_proj float32
 */
fdk_status fdk_pack_projections(const float* src, int32_t n_proj, int32_t width,
                                int32_t height, int32_t dtype, void* dst,
                                float* scale_out, void* stream);

/* Geometry of FDK preprocessing (the filtering that turns line integrals
 * into the projections fdk_backproject consumes). */
typedef struct fdk_filter_geometry {
    int32_t n_proj, width, height;  /* N, W (1 .. 2048), H */
    int32_t reserved;               /* must be 0 */
    double pixel_u_mm, pixel_v_mm;  /* detector pitch along u (rows) and v (columns) */
    double u0, v0;                  /* principal point, pixels */
    double sdd_mm, sid_mm;          /* source-detector and source-isocentre distances */
    const double* angles_rad;       /* HOST, n_proj gantry angles from the scan start */
    double scan_range_rad;          /* short-scan range R (Parker weights); <= 0: no weighting */
    double dbeta_rad;               /* angular step folded into the output scale */
    double fan_sign;                /* +1 or -1: fan angle = fan_sign * atan(u / SDD) */
} fdk_filter_geometry;

/*
 * FDK preprocessing of a stack of line integrals, one projection per image
 * (Feldkamp-Davis-Kress weighting and filtering; the paper's benchmark data
 * arrive already filtered, Sec. "RabbitCT Benchmarking Framework"):
 *   u = (i - u0) pixel_u, v = (j - v0) pixel_v, t = pixel_u SID / SDD
 *   x_k(i, j) = src_k(i, j) SDD / sqrt(SDD^2 + u^2 + v^2) * parker(beta_k, fan_sign atan(u / SDD))
 *   dst_k(i, j) = t dbeta SID^2 sum_i' h(i - i') x_k(i', j)
 * with the band-limited ramp kernel h(0) = 1/(4 t^2), h(odd n) = -1/(n pi t)^2,
 * h(even n != 0) = 0 (Kak and Slaney) and Parker's short-scan weights for
 * R = pi + 2 d (Parker 1982); the convolution is the linear one along each
 * row.  dtype FDK_F32 writes float32 to dst; FDK_F16 / FDK_BF16 write the
 * packed form of fdk_pack_projections (scale_out required, DEVICE n_proj
 * floats).  Weights, FFT and convolution run in FP64; only the output is
 * rounded.
 *   g          host geometry (angles copied before return)
 *   src        DEVICE, n_proj * height * width float32
 *   dst        DEVICE, n_proj * height * width of dtype
 * Limits: width 1 .. 2048 (one row pair's FP64 spectrum of the circular
 * length, at most 4096, is held in LDS), n_proj * height * width <= 2^40;
 * FDK_E_INVALID_ARG beyond them, nothing enqueued.
 * FDK_E_GEOMETRY if R > 0 and d = (R - pi) / 2 is smaller than the largest
 * fan angle of the detector (the short scan does not cover every ray).
 */
fdk_status fdk_filter_projections(const fdk_filter_geometry* g, const float* src, void* dst,
                                  int32_t dtype, float* scale_out, void* stream);

/*
 * Out-of-core backprojection, for stacks and volumes that should not (or
 * cannot) be resident on the device: the paper's outlook to very large
 * detectors (Sec. "Conclusion and Outlook").  The volume is processed in
 * z-slabs of `slab_planes` planes; for each slab and projection only the
 * band of detector rows the slab can reach is copied to the device (from
 * the slab's corner voxels, exact for w > 0, widened by two rows), on a
 * library copy stream, while the previous slab is backprojected on
 * `stream`.  The band's first row is folded into the matrix in FP64
 * (v' = v - j0 w), so each slab is an ordinary fdk_backproject call on a
 * band-high detector; results equal fdk_backproject on the whole stack up
 * to FP32 rounding.
 *   vol          grid (planes z_begin .. z_begin + z_count)
 *   proj         n_proj, width, height, mats, dtype, scale as for
 *                fdk_backproject; data may be HOST or DEVICE memory (page-locked
 *                host memory lets the copies overlap the kernels; pageable
 *                memory is copied synchronously by the runtime)
 *   volume       DEVICE z_count * L * L float32, or HOST memory with
 *                FDK_STREAM_HOST_VOLUME (each slab is computed into one of two
 *                device slab buffers and copied back on a second copy stream;
 *                with accumulate the slab is first copied in)
 *   slab_planes  >= 1 planes per slab (the last slab may be thinner)
 * Device memory held until fdk_release_workspace: two band stacks of
 * n_proj * (largest band) * width elements, and with FDK_STREAM_HOST_VOLUME
 * two slabs of slab_planes * L * L float32.  The call returns once all work
 * is enqueued; `stream` completes when the volume (host or device) is
 * written.  The host buffers must stay valid until then.  Errors as for
 * fdk_backproject; every slab is validated before anything is enqueued.
 */
#define FDK_STREAM_HOST_VOLUME 1
fdk_status fdk_backproject_streamed(const fdk_volume* vol, const fdk_projections* proj, float* volume,
                                    int32_t slab_planes, int32_t flags, int accumulate, void* stream);

/* The slab plan fdk_backproject_streamed would use (host only, no device
 * work): *n_slabs slabs; band_rows[s] (HOST, n_slabs entries, or NULL) rows
 * copied per projection for slab s; first_rows[s * n_proj + k] (HOST, or NULL)
 * the first detector row of projection k's band.  Call with NULL arrays to
 * get n_slabs = ceil(z_count / slab_planes). */
fdk_status fdk_streamed_plan(const fdk_volume* vol, const fdk_projections* proj, int32_t slab_planes,
                             int32_t* n_slabs, int32_t* band_rows, int32_t* first_rows);

/*
 * Iterative reconstruction on the matched projector pair: the system A x = p
 * with A = fdk_forwardproject (volume -> projections, the transpose of the
 * backprojection of Listing 1) and A^T = fdk_backproject.  Each iteration
 * costs one forward projection, one backprojection and a few passes over
 * the vectors; step lengths are computed on the device (no host round trip
 * inside a call).  Vectors are FP32, reductions and scalars FP64.
 *   vol        grid of the unknown volume (planes z_begin .. z_begin + z_count)
 *   proj       measured projections p: FP32 only (FDK_E_UNSUPPORTED otherwise),
 *              DEVICE data, scale ignored
 *   volume     DEVICE, z_count * L * L float32: the start x0 when requested,
 *              else overwritten; the result x_n on return
 *   n_iter     >= 0 iterations
 *   history    DEVICE doubles or NULL (see each solver); FDK_E_INVALID_ARG if
 *              it is not device memory
 * The library holds four solver vectors (two of the projection stack's size,
 * two of the volume's) until fdk_release_workspace.  Buffers must not
 * overlap.  Errors as for the projectors; on a validation error nothing is
 * enqueued and `volume` is untouched.
 *
 * CGLS (conjugate gradients on the normal equations, Hestenes & Stiefel
 * 1952, in the residual form of Bjorck 1996): x_k minimises ||A x - p|| over
 * x0 + span{A^T r0, (A^T A) A^T r0, ...} (k vectors), r0 = p - A x0.
 * history[k] = ||r_k||^2 as carried by the recursion, k = 0 .. n_iter
 * (n_iter + 1 values).  use_x0: 0 starts from x0 = 0.
 */
fdk_status fdk_cgls(const fdk_volume* vol, const fdk_projections* proj, float* volume, int32_t n_iter,
                    int use_x0, double* history, void* stream);

/*
 * SIRT (simultaneous iterative reconstruction, Gilbert 1972, with row and
 * column normalisation):  x <- x + lambda C A^T R (p - A x), then max(x, 0)
 * with FDK_SIRT_NONNEG.  R and C invert the row sums A 1 and column sums
 * A^T 1, each floored at 1e-3 times its largest entry: 1 / max(s, 1e-3 max s)
 * (rows and columns with a zero sum contribute nothing either way).
 * history[k] = ||p - A x_k||^2 for k = 0 .. n_iter - 1, the residual each
 * update starts from (n_iter values).  lambda finite and > 0.
 */
#define FDK_SIRT_USE_X0 1   /* start from the contents of `volume` (else 0) */
#define FDK_SIRT_NONNEG 2   /* clamp every iterate at 0 */
fdk_status fdk_sirt(const fdk_volume* vol, const fdk_projections* proj, float* volume, int32_t n_iter,
                    double lambda, int32_t flags, double* history, void* stream);

/* Tile shape and staged layout of the backprojection kernel: a 64-wide
 * wavefront owns an 8 x 8 patch of (x, y) columns and each lane a strip of
 * `strip` voxels along z; a workgroup holds `waves` patches (1 x 1, 2 x 1 or
 * 2 x 2); strip in {2, 4, 8, 16, 32}, waves in {1, 2, 4}.  layout 0 stages each
 * projection as a zero-bordered image; layout 1 stores with every staged
 * pixel its whole 2x2 bilinear block (four times the staging memory, one load
 * per sample); layout 2 stores with every pixel its right neighbour (twice the
 * memory, aligned row loads); layout 3 (the built-in choice for every dtype)
 * copies each workgroup's projection window into LDS and reads the taps there
 * (a window of more than 8192 pixels, or wider than 4 pixels per thread of
 * the workgroup, is gathered from the staged image instead).  The `dtype` argument selects a
 * tuning slot: FDK_F32, FDK_F16, FDK_BF16 (backprojection by projection
 * dtype), FDK_TUNE_BATCHED (strip and waves of fdk_backproject_batched, and
 * the layout of its FP32 scans; FP16/BF16 scans keep the layout of their own
 * slot) or FDK_TUNE_ADJOINT (the forward projector).  For the forward
 * projector, layout 4 (the default) gives each workgroup a detector tile of
 * `strip` rows (1 <= strip, (strip + 4) * 5 * waves <= 20480) by
 * min(width, 20480 / ((strip + 4) * waves) - 4) pixels (one fewer where the
 * row pitch, rounded up to an odd number of accumulators, would not fit) in
 * `waves` projections (1, 2, 4 or 8), accumulated in FP64 in LDS inside a
 * two-pixel border and written once; layout 0 scatters
 * every voxel straight to global memory with float atomics (tile shapes as for
 * the backprojection).
 * fdk_set_tile pins the choice for a dtype (strip = waves = 0 restores the
 * automatic choice from the tuning table); fdk_get_tile reports what a call
 * with this grid and dtype would use. */
fdk_status fdk_set_tile(int32_t dtype, int32_t strip, int32_t waves, int32_t layout);
fdk_status fdk_get_tile(const fdk_volume* vol, int32_t dtype, int32_t* strip, int32_t* waves,
                        int32_t* layout);

/* Tuning table: entries (dtype, size class) -> tile shape and layout, as
 * written by the autotuner.  fdk_load_tuning reads a file of lines
 * "dtype class strip waves layout" ('#' starts a comment); size class =
 * floor(log2(L)).  A file for another library ABI version or device is
 * rejected (its first line must read "fdk-tuning <FDK_ABI_VERSION> gfx950").
 * Returns the number of entries read or a negative fdk_status.
 * fdk_set_tuning_entry sets one entry; strip = waves = 0 removes it.  The
 * environment variable FDK_TUNING_FILE names a file loaded on first use.
 * FP32 stacks sampled through LDS windows (layout 3) are read in place, with
 * bounds-checked window loads, instead of being staged, by
 * fdk_backproject_batched and by fdk_backproject when the grid has fewer
 * than one voxel per eight projection pixels (staging would cost more than
 * the slightly slower loads); FDK_STAGE_FP32=1 in the environment (read on
 * first use) stages them in every case. */
int32_t fdk_load_tuning(const char* path);
fdk_status fdk_set_tuning_entry(int32_t dtype, int32_t size_class, int32_t strip, int32_t waves,
                                int32_t layout);

/* Matrix normalisation (host only): rescales each row-major 3x4 matrix of
 * mats (HOST, n_proj * 12 doubles, in place) by s = +-1 / ||A[2][0:3]|| so
 * that w becomes the signed distance along the principal ray (in the units of
 * the world coordinates, mm) and w > 0 at the world origin, the isocentre.
 * u/w and v/w are unchanged; the 1/w^2 weight then depends on the
 * geometry only through distances (Sec. "RabbitCT Benchmarking Framework":
 * w approximates the distance to the source).  FDK_E_INVALID_ARG for NULL,
 * n_proj < 1, non-finite entries, a zero third row or w = 0 at the origin. */
fdk_status fdk_normalize_matrices(double* mats, int32_t n_proj);

/* Host-side check of a call's arguments: the validation fdk_backproject
 * performs, without touching the GPU. */
fdk_status fdk_validate(const fdk_volume* vol, const fdk_projections* proj,
                        int need_data);

/* Kernel timing for measurement: while enabled, every kernel launch of the
 * library is bracketed by HIP events on its stream.  fdk_profile_read waits for
 * the recorded events and returns, for one kernel kind ("stage", "fold",
 * "window", "bp", "fp", "fill", "unstage", "pack", "batched", "filter"), the
 * number of launches and their
 * summed duration in milliseconds since the last fdk_profile_enable call
 * (which clears the records). */
fdk_status fdk_profile_enable(int enable);
fdk_status fdk_profile_read(const char* kernel, int64_t* launches, double* total_ms);

/* Releases the calling thread's current-device workspace and cached graphs
 * (waits for the device first). */
fdk_status fdk_release_workspace(void);

const char* fdk_status_string(fdk_status status);
const char* fdk_last_error(void);   /* thread-local, "" if none */
int32_t fdk_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDK_H */
