// Host layer of the FDK backprojection library: argument validation, FP64
// matrix composition, workspace management, tile selection, launches, and the
// HIP-graph cache of the batched form.  Implements include/fdk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdk.h"
#include "fdk_internal.h"

using namespace fdk;

namespace {

thread_local std::string g_last_error;

fdk_status fail(fdk_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FDK_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr int kMaxL = 32768;
constexpr int kMaxScans = 4096;

int esize_of(int dtype) { return dtype == FDK_F32 ? 4 : 2; }

// Staged row length in pixels: detector plus zero border, rounded up to 8
// pixels so that every row starts 16-byte aligned.
int staged_pitch(int W) { return (W + kPadLo + kPadHi + 7) & ~7; }

// ------------------------------------------------------------------ validation
fdk_status check_volume(const fdk_volume* v)
{
    if (v == nullptr) return fail(FDK_E_INVALID_ARG, "volume descriptor is NULL");
    if (v->L < 1 || v->L > kMaxL) return fail(FDK_E_INVALID_ARG, "L=%d outside [1, %d]", v->L, kMaxL);
    if (v->z_begin < 0 || v->z_begin >= v->L)
        return fail(FDK_E_INVALID_ARG, "z_begin=%d outside [0, L)", v->z_begin);
    if (v->z_count < 1 || v->z_count > v->L - v->z_begin)
        return fail(FDK_E_INVALID_ARG, "z_count=%d outside [1, L - z_begin]", v->z_count);
    if (v->reserved != 0) return fail(FDK_E_INVALID_ARG, "reserved field must be 0");
    if (!std::isfinite(v->voxel_mm) || !(v->voxel_mm > 0.0))
        return fail(FDK_E_INVALID_ARG, "voxel_mm must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(v->origin_mm[a])) return fail(FDK_E_INVALID_ARG, "origin_mm is not finite");
    return FDK_OK;
}

fdk_status check_proj(const fdk_projections* p, bool need_data)
{
    if (p == nullptr) return fail(FDK_E_INVALID_ARG, "projection descriptor is NULL");
    if (p->n_proj < 1) return fail(FDK_E_INVALID_ARG, "n_proj=%d < 1", p->n_proj);
    if (p->width < 1 || p->height < 1)
        return fail(FDK_E_INVALID_ARG, "detector %dx%d has an empty axis", p->width, p->height);
    if (p->mats == nullptr) return fail(FDK_E_INVALID_ARG, "mats is NULL");
    if (need_data) {
        if (p->dtype != FDK_F32 && p->dtype != FDK_F16 && p->dtype != FDK_BF16)
            return fail(FDK_E_UNSUPPORTED, "unknown dtype %d", p->dtype);
        if (p->data == nullptr) return fail(FDK_E_INVALID_ARG, "projection data is NULL");
    }
    const int es = need_data ? esize_of(p->dtype) : 4;
    const int64_t wp = (int64_t)staged_pitch(p->width);
    const int64_t hp = (int64_t)p->height + kPadLo + kPadHi;
    // staged image offsets are signed 32-bit, row pitch a 24-bit multiplier
    if (wp * hp * es >= (int64_t(1) << 31) || wp >= (int64_t(1) << 23) || hp >= (int64_t(1) << 23))
        return fail(FDK_E_INVALID_ARG, "detector %dx%d too large", p->width, p->height);
    if ((int64_t)p->n_proj * wp * hp * es > (int64_t(1) << 46))
        return fail(FDK_E_INVALID_ARG, "projection stack too large");
    for (int64_t i = 0; i < (int64_t)p->n_proj * 12; ++i)
        if (!std::isfinite(p->mats[i])) return fail(FDK_E_INVALID_ARG, "matrix %lld has a non-finite entry", (long long)(i / 12));
    return FDK_OK;
}

// w > 0 at the eight corner voxel centres of the processed planes, for every
// projection.  w is affine in the voxel position, so this covers the region.
fdk_status check_geometry(const fdk_volume* v, const fdk_projections* p)
{
    const double xs[2] = {0.0, (double)(v->L - 1)};
    const double zs[2] = {(double)v->z_begin, (double)(v->z_begin + v->z_count - 1)};
    for (int k = 0; k < p->n_proj; ++k) {
        const double* A = p->mats + 12 * k;
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 0; cy < 2; ++cy)
                for (int cz = 0; cz < 2; ++cz) {
                    const double X = v->origin_mm[0] + xs[cx] * v->voxel_mm;
                    const double Y = v->origin_mm[1] + xs[cy] * v->voxel_mm;
                    const double Z = v->origin_mm[2] + zs[cz] * v->voxel_mm;
                    const double w = A[8] * X + A[9] * Y + A[10] * Z + A[11];
                    if (!(w > 0.0))
                        return fail(FDK_E_GEOMETRY,
                                    "projection %d: w=%g <= 0 at corner voxel (%d,%d,%d)", k, w,
                                    cx ? v->L - 1 : 0, cy ? v->L - 1 : 0,
                                    cz ? v->z_begin + v->z_count - 1 : v->z_begin);
                }
    }
    return FDK_OK;
}

// ------------------------------------------------------------------ composition
// Per projection, the FP64 matrix that maps centred voxel indices
// (x - c, y - c, z - c, 1), c = L/2, to centred detector coordinates
// (u - cu w, v - cv w, w), cu = W/2, cv = H/2, scaled by one power of two 2^e
// chosen so w is O(1).  The kernel's weight is then 2^-2e / w^2 and the
// result is multiplied by out_scale = 2^2e.
struct Composed {
    std::vector<double> coef;  // n_proj * 12
    float out_scale;
    int const_w;               // 1: w independent of z for every projection (coefficient exactly 0),
                               // 2: u and w both (a circular orbit about the z axis)
};

// Writes n_proj * 12 doubles to `coef` (no allocation).
void compose_into(const fdk_volume* v, const fdk_projections* p, double* coef, float* out_scale, int* const_w)
{
    const int N = p->n_proj;
    const int ctr = v->L / 2;
    const double cu = (double)(p->width / 2), cv = (double)(p->height / 2);
    double wsum = 0.0;
    for (int k = 0; k < N; ++k) {
        const double* A = p->mats + 12 * k;
        double M[3][4];
        for (int r = 0; r < 3; ++r) {
            double t = A[r * 4 + 3];
            for (int a = 0; a < 3; ++a) {
                M[r][a] = A[r * 4 + a] * v->voxel_mm;
                t += A[r * 4 + a] * (v->origin_mm[a] + ctr * v->voxel_mm);
            }
            M[r][3] = t;
        }
        for (int a = 0; a < 4; ++a) {
            M[0][a] -= cu * M[2][a];
            M[1][a] -= cv * M[2][a];
        }
        for (int r = 0; r < 3; ++r)
            for (int a = 0; a < 4; ++a) coef[(size_t)k * 12 + r * 4 + a] = M[r][a];
        wsum += std::fabs(M[2][3]);
    }
    const double wmean = wsum / N;
    const int e = (wmean > 0.0 && std::isfinite(wmean)) ? -(int)std::lround(std::log2(wmean)) : 0;
    const double s = std::ldexp(1.0, e);
    for (size_t i = 0; i < (size_t)N * 12; ++i) coef[i] *= s;
    *out_scale = (float)std::ldexp(1.0, 2 * e);
    bool cw = true, cz = true;
    for (int k = 0; k < N; ++k) {
        cw = cw && coef[(size_t)k * 12 + 10] == 0.0;
        cz = cz && coef[(size_t)k * 12 + 2] == 0.0;
    }
    *const_w = cw ? (cz ? 2 : 1) : 0;
}

Composed compose(const fdk_volume* v, const fdk_projections* p)
{
    Composed c;
    c.coef.resize((size_t)p->n_proj * 12);
    compose_into(v, p, c.coef.data(), &c.out_scale, &c.const_w);
    return c;
}

// ------------------------------------------------------------------ kernel timing
// When enabled, every launch is bracketed by a pair of HIP events on the
// launch's stream; fdk_profile_read sums the elapsed times per kernel kind.
struct ProfRecord {
    const char* kind;
    hipEvent_t start, end;
};

struct Profiler {
    bool on = false;
    std::vector<ProfRecord> records;
    std::vector<hipEvent_t> pool;
};

Profiler g_prof;
constexpr size_t kProfMax = 1 << 16;

hipEvent_t prof_event()
{
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// RAII bracket: records the start event now and the end event at scope exit.
struct ProfScope {
    const char* kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* k, hipStream_t st) : kind(k), s(st)
    {
        if (!g_prof.on || g_prof.records.size() >= kProfMax) return;
        a = prof_event();
        b = prof_event();
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (a && b) {
            (void)hipEventRecord(b, s);
            g_prof.records.push_back({kind, a, b});
        }
    }
};

// ------------------------------------------------------------------ tiles
struct TileShape { int strip, waves, layout; };

// Tuning slots: FDK_F32, FDK_F16, FDK_BF16 for the backprojection, and one for
// the adjoint (forward projection).
constexpr int kAdjointSlot = FDK_TUNE_ADJOINT;
constexpr int kBatchedSlot = FDK_TUNE_BATCHED;
constexpr int kSlots = 5;

struct Tuning {
    std::map<std::pair<int, int>, TileShape> table;  // (dtype, size class) -> shape
    TileShape forced[kSlots] = {};   // by slot: FP32, FP16, BF16, adjoint, batched
    bool env_loaded = false;
    bool stage_fp32 = false;         // FDK_STAGE_FP32=1: stage FP32 stacks for the LDS kernels too
};

int size_class(int L)
{
    int c = 0;
    while ((1 << (c + 1)) <= L) ++c;
    return c;
}

// Built-in choice when no tuning entry applies: four 8x8 patches per
// workgroup and the longest strip (fewer per-projection set-ups per voxel)
// that still gives ~4 workgroups per CU on a 256-CU device, sampling the tile
// footprint from LDS for every storage type (FP16/BF16 windows are widened
// to FP32 in LDS; at 512^3 x 496 this is 37 ms against 46 ms for gathers of
// whole 2x2 blocks, and the staged stack is a quarter of the quad layout's).
// The adjoint (tuning slot 3) accumulates detector tiles in LDS: (rows,
// projections per workgroup, layout 4); the columns are as many as the LDS
// holds.  Measured at 496 x 1248x960: 36 rows x 2 projections (251 columns)
// 87.5 ms at 512^3 against 91.0 for 60 x 1; at 256^3 60 x 1 (316 columns)
// 14.9 ms against 15.1.
TileShape default_adjoint_tile(int L)
{
    return L >= 384 ? TileShape{36, 2, 4} : TileShape{60, 1, 4};
}

TileShape default_tile(int L, int dtype)
{
    (void)dtype;
    const int layout = 3;
    const int64_t want = 1024;
    for (int strip : {16, 8, 4}) {
        const int64_t tiles = (int64_t)((L + 15) / 16) * ((L + 15) / 16) * ((L + strip - 1) / strip);
        if (tiles >= want) return {strip, 4, layout};
    }
    return {2, 4, layout};
}

// ------------------------------------------------------------------ device state
struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

hipError_t ensure(DevBuf& b, size_t bytes)
{
    if (b.n >= bytes && b.p != nullptr) return hipSuccess;
    if (b.p != nullptr) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.n = want;
    return hipSuccess;
}

void release(DevBuf& b)
{
    if (b.p != nullptr) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

// Pinned host memory (uploads from it run asynchronously).
struct HostBuf {
    void* p = nullptr;
    size_t n = 0;
};

hipError_t ensure_host(HostBuf& b, size_t bytes)
{
    if (b.n >= bytes && b.p != nullptr) return hipSuccess;
    if (b.p != nullptr) {
        hipError_t e = hipHostFree(b.p);
        b.p = nullptr;
        b.n = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&b.p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.n = want;
    return hipSuccess;
}

void release_host(HostBuf& b)
{
    if (b.p != nullptr) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

// Composed coefficients of one geometry (one slab, or every slab of an
// out-of-core call, 12 doubles per projection each), uploaded from a pinned
// host copy without waiting; `used` is recorded after the last kernel that
// reads the device table, so an entry is recycled only once that has run.
struct CoefSlab {
    const double* dev;   // n_proj * 12 doubles
    float out_scale;
    int const_w;
};

struct CoefEntry {
    std::string key;
    DevBuf buf;
    HostBuf host;
    hipEvent_t used = nullptr;
    std::vector<float> out_scale;   // per slab
    std::vector<int> const_w;       // per slab
    size_t slab_doubles = 0;        // doubles per slab in buf
    CoefSlab slab(size_t i) const
    {
        return CoefSlab{static_cast<const double*>(buf.p) + i * slab_doubles, out_scale[i], const_w[i]};
    }
};

void release_coef(CoefEntry& c)
{
    release(c.buf);
    release_host(c.host);
    if (c.used) (void)hipEventDestroy(c.used);
    c.used = nullptr;
}

struct BatchEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
    DevBuf tiles, item_begin, stage, scale_ptrs, coef64, coef_dev, counter, windows;
};

void release_entry(BatchEntry& b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
    for (DevBuf* x : {&b.tiles, &b.item_begin, &b.stage, &b.scale_ptrs, &b.coef64, &b.coef_dev, &b.counter,
                      &b.windows})
        release(*x);
}

// FDK preprocessing tables of one geometry (FP64 on the host, FP32 on the device).
struct FilterEntry {
    std::string key;
    int M = 0;
    DevBuf hs, tw, wc, wp;
};

struct DeviceState {
    bool init = false;
    bool arch_ok = false;
    unsigned char* scratch = nullptr;   // this device's copy of the allocation-free scratch array
    int num_cus = 0;
    std::string arch;
    DevBuf staged, coef_dev, adjoint, windows;
    std::list<CoefEntry> coef_cache;   // most recent first
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    hipEvent_t done = nullptr;
    // batched form
    DevBuf batch_staged;
    std::list<BatchEntry> batch_cache;
    hipStream_t capture_stream = nullptr;
    // preprocessing
    std::list<FilterEntry> filter_cache;   // most recent first
    DevBuf filter_ws, filter_max;
    // iterative solvers: two projection-sized and two volume-sized vectors,
    // reduction partials and the solver's scalar state
    DevBuf it_p0, it_p1, it_v0, it_v1, it_part, it_st;
    // out-of-core form: double-buffered row-band stacks and volume slabs,
    // a host-to-device and a device-to-host copy stream, and the events that
    // order the buffers between the streams (kept across calls)
    DevBuf band[2], slab[2], band_j0;
    HostBuf band_j0_host;   // pinned source of the band_j0 upload
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t band_ready[2] = {}, band_free[2] = {}, slab_done[2] = {}, slab_free[2] = {};
    hipEvent_t call_start = nullptr, j0_read = nullptr;
    bool j0_pending = false;
    bool band_used[2] = {false, false}, slab_used[2] = {false, false};
};

// Scratch memory of fdk_backproject_noalloc, one copy per device, held until
// the process ends: the folded coefficient table, the composed one, and the
// window table of one z-chunk.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (DeviceState::scratch).
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kNoAllocMaxProj = 4096;
constexpr size_t kScratchFolded = 0;                                         // n_proj x 16 doubles
constexpr size_t kScratchComposed = (size_t)kNoAllocMaxProj * 16 * 8;        // n_proj x 12 doubles
constexpr size_t kScratchWin = kScratchComposed + (size_t)kNoAllocMaxProj * 12 * 8;   // windows
static_assert(kScratchWin % 256 == 0, "window table offset");
static __device__ __align__(256) unsigned char g_scratch[kScratchBytes];
// host source of the coefficient upload (guarded by g_mu)
double g_noalloc_coef[kNoAllocMaxProj * 12];

// Recursive: the iterative solvers call the projector entry points while holding it.
std::recursive_mutex g_mu;
std::map<int, DeviceState> g_dev;
Tuning g_tune;

constexpr size_t kCoefCacheMax = 64;
constexpr size_t kBatchCacheMax = 4;

fdk_status device_state(DeviceState** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceState& d = g_dev[dev];
    if (!d.init) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        d.arch = prop.gcnArchName;
        d.arch_ok = d.arch.rfind("gfx950", 0) == 0;
        d.num_cus = prop.multiProcessorCount;
        HIP_TRY(hipEventCreateWithFlags(&d.done, hipEventDisableTiming));
        if (d.arch_ok) {
            // the device address of this device's copy of the scratch array (the
            // array's name in host code is only a stand-in for the symbol)
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_scratch));
            if (e != hipSuccess)
                return fail(FDK_E_DEVICE, "scratch array of device %d: %s", dev, hipGetErrorString(e));
            d.scratch = static_cast<unsigned char*>(p);
        }
        d.init = true;
    }
    if (!d.arch_ok)
        return fail(FDK_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev,
                    d.arch.c_str());
    *out = &d;
    return FDK_OK;
}

// Calls on a new stream wait for the previous call's work (shared workspace).
fdk_status begin_call(DeviceState& d, hipStream_t s)
{
    if (d.have_last && d.last_stream != s) HIP_TRY(hipStreamWaitEvent(s, d.done, 0));
    return FDK_OK;
}

fdk_status end_call(DeviceState& d, hipStream_t s)
{
    HIP_TRY(hipEventRecord(d.done, s));
    d.last_stream = s;
    d.have_last = true;
    return FDK_OK;
}

std::string coef_key(const fdk_volume* v, const fdk_projections* p)
{
    std::string k;
    auto put = [&k](const void* x, size_t n) { k.append(static_cast<const char*>(x), n); };
    put(&v->L, sizeof(int32_t));
    put(&v->voxel_mm, sizeof(double));
    put(v->origin_mm, 3 * sizeof(double));
    put(&p->n_proj, sizeof(int32_t));
    put(&p->width, sizeof(int32_t));
    put(&p->height, sizeof(int32_t));
    put(p->mats, (size_t)p->n_proj * 12 * sizeof(double));
    return k;
}

// Device copy of the composed FP64 coefficients of one or more slabs, cached
// by content.  A miss composes into the entry's pinned host buffer and
// uploads asynchronously on `s`; no host wait unless the least recently used
// entry, recycled for it, is still being read by queued work (then the host
// waits for that work), or a buffer has to grow (hipFree and hipHostFree
// synchronise the device).  The caller records `used` after its fold kernel.
fdk_status coef_lookup(DeviceState& d, const std::string& key, hipStream_t s,
                       const std::vector<std::pair<const fdk_volume*, const fdk_projections*>>& slabs,
                       CoefEntry** out)
{
    for (auto it = d.coef_cache.begin(); it != d.coef_cache.end(); ++it) {
        if (it->key == key) {
            d.coef_cache.splice(d.coef_cache.begin(), d.coef_cache, it);
            *out = &d.coef_cache.front();
            return FDK_OK;
        }
    }
    std::vector<Composed> cs;
    cs.reserve(slabs.size());
    size_t per = 0;
    for (const auto& sl : slabs) {
        cs.push_back(compose(sl.first, sl.second));
        for (double x : cs.back().coef)
            if (!std::isfinite((float)x))
                return fail(FDK_E_INVALID_ARG, "composed projection matrix exceeds FP32 range");
        per = std::max(per, cs.back().coef.size());
    }
    CoefEntry e;
    if (d.coef_cache.size() >= kCoefCacheMax) {
        e = std::move(d.coef_cache.back());
        d.coef_cache.pop_back();
        if (e.used) HIP_TRY(hipEventSynchronize(e.used));
    }
    if (e.used == nullptr) HIP_TRY(hipEventCreateWithFlags(&e.used, hipEventDisableTiming));
    const size_t bytes = per * cs.size() * sizeof(double);
    hipError_t err = ensure(e.buf, bytes);
    if (err == hipSuccess) err = ensure_host(e.host, bytes);
    if (err != hipSuccess) {
        release_coef(e);
        return fail(FDK_E_NOMEM, "coefficient table allocation failed: %s", hipGetErrorString(err));
    }
    e.key = key;
    e.slab_doubles = per;
    e.out_scale.clear();
    e.const_w.clear();
    double* h = static_cast<double*>(e.host.p);
    for (size_t i = 0; i < cs.size(); ++i) {
        std::copy(cs[i].coef.begin(), cs[i].coef.end(), h + i * per);
        e.out_scale.push_back(cs[i].out_scale);
        e.const_w.push_back(cs[i].const_w);
    }
    err = hipMemcpyAsync(e.buf.p, e.host.p, bytes, hipMemcpyHostToDevice, s);
    // until the table has been read, recycling this entry must wait for the upload
    if (err == hipSuccess) err = hipEventRecord(e.used, s);
    if (err != hipSuccess) {
        release_coef(e);
        return fail(FDK_E_DEVICE, "coefficient upload failed: %s", hipGetErrorString(err));
    }
    d.coef_cache.push_front(std::move(e));
    *out = &d.coef_cache.front();
    return FDK_OK;
}

fdk_status coef_table(DeviceState& d, const fdk_volume* v, const fdk_projections* p, hipStream_t s,
                      CoefEntry** out)
{
    return coef_lookup(d, coef_key(v, p), s, {{v, p}}, out);
}

// Bytes of one staged pixel: the source element (plain), its 2x2 block (quad)
// or its pair of row taps (pair).
int pixel_bytes(int esize, int layout) { return layout == 1 ? 4 * esize : layout == 2 ? 2 * esize : esize; }
// Layout 3 (LDS tiles) reads the plain staged image.
int staged_layout(int layout) { return layout == 3 ? 0 : layout; }

// The quad layout multiplies the staged image by four; images whose quad form
// would not fit 31-bit offsets use the plain layout.
TileShape fit_layout(TileShape t, const fdk_projections* p, int esize)
{
    const int64_t px = (int64_t)staged_pitch(p->width) * (p->height + kPadLo + kPadHi);
    if (t.layout != 0 && px * pixel_bytes(esize, t.layout) >= (int64_t(1) << 31)) t.layout = 0;
    return t;
}

TileShape pick_tile(int L, int dtype)
{
    const TileShape f = g_tune.forced[dtype];
    if (f.strip > 0) return f;
    auto it = g_tune.table.find({dtype, size_class(L)});
    if (it != g_tune.table.end()) return it->second;
    if (dtype == kAdjointSlot) return default_adjoint_tile(L);
    return default_tile(L, dtype == kBatchedSlot ? FDK_F32 : dtype);
}

bool valid_shape(int slot, TileShape t)
{
    if (slot == kAdjointSlot) {
        if (t.layout == 4)   // at least one column per tile
            return t.strip >= 1 && (int64_t)(t.strip + 2 * kBandBorder) * (1 + 2 * kBandBorder) * t.waves <= kBandCap &&
                   supported_band_group(t.waves);
        return t.layout == 0 && supported_tile(t.strip, t.waves) != 0;
    }
    return t.layout >= 0 && t.layout <= 3 && supported_tile(t.strip, t.waves) != 0;
}

void load_env_tuning();


TileArgs make_args(const fdk_volume* v, const fdk_projections* p, int esize, TileShape t,
                   const unsigned char* staged, const double* coef_dev, float* vol, float out_scale,
                   int accumulate, int dtype)
{
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    const int W = p->width, H = p->height;
    const int Wp = staged_pitch(W), Hp = H + kPadLo + kPadHi;
    const int cu = W / 2, cv = H / 2;
    esize = pixel_bytes(esize, staged_layout(t.layout));
    a.layout = t.layout;
    a.proj = staged;
    a.coef = coef_dev;
    a.vol = vol;
    const uint64_t img = (uint64_t)Wp * Hp * esize;
    a.proj_stride = (img + 255) & ~uint64_t(255);
    a.n_proj = p->n_proj;
    a.L = v->L;
    a.z_begin = v->z_begin;
    a.z_count = v->z_count;
    a.ctr = v->L / 2;
    a.row_bytes = (uint32_t)(Wp * esize);
    a.centre_bytes = (uint32_t)((cv + kPadLo) * Wp * esize + (cu + kPadLo) * esize);
    a.proj_bytes = (uint32_t)img;
    a.lo_x = (float)(-kPadLo - cu);
    a.hi_x = (float)(W - 1 + kPadLo - cu);
    a.lo_y = (float)(-kPadLo - cv);
    a.hi_y = (float)(H - 1 + kPadLo - cv);
    a.out_scale = out_scale;
    a.accumulate = accumulate ? 1 : 0;
    // a workgroup covers (8 bx) x (8 by) columns and `strip` planes
    const int bx = t.waves >= 16 ? 4 : t.waves >= 2 ? 2 : 1, by = t.waves / bx;
    a.tiles_x = (v->L + 8 * bx - 1) / (8 * bx);
    a.tiles_y = (v->L + 8 * by - 1) / (8 * by);
    a.tiles_z = (v->z_count + t.strip - 1) / t.strip;
    a.dtype = dtype;
    a.cu = cu;
    a.cv = cv;
    a.win = nullptr;
    a.anc = nullptr;
    a.rot_div = 0;
    a.const_w = 0;
    a.raw = 0;
    return a;
}

// A window table of n entries and its sampling set-ups share one allocation:
// the windows, then (at a 256-byte boundary) the set-ups.
size_t anc_offset(uint64_t n) { return (size_t)((n * sizeof(Win) + 255) / 256 * 256); }
size_t window_table_bytes(uint64_t n) { return anc_offset(n) + (size_t)n * sizeof(Anc); }
// the anchor records of a batch's window table of n entries
Anc* batch_anchors(BatchEntry& b, uint64_t n)
{
    return reinterpret_cast<Anc*>(static_cast<unsigned char*>(b.windows.p) + anc_offset(n));
}

fdk_status check_grid(const TileArgs& a)
{
    const int64_t nb = (int64_t)a.tiles_x * a.tiles_y * a.tiles_z;
    if (nb > 0x7fffffffLL) return fail(FDK_E_INVALID_ARG, "volume too large for one launch");
    return FDK_OK;
}

uint64_t staged_bytes(const fdk_projections* p, int esize, int layout)
{
    esize = pixel_bytes(esize, staged_layout(layout));
    const uint64_t img = (uint64_t)staged_pitch(p->width) * (p->height + kPadLo + kPadHi) * esize;
    return (uint64_t)p->n_proj * ((img + 255) & ~uint64_t(255));
}

StageArgs make_stage(const fdk_projections* p, int esize, int layout, unsigned char* dst, int64_t row_begin)
{
    StageArgs s;
    layout = staged_layout(layout);
    s.layout = layout;
    s.src = p->data;
    s.dst = dst;
    s.n = p->n_proj;
    s.W = p->width;
    s.H = p->height;
    s.Wp = staged_pitch(p->width);
    s.Hp = p->height + kPadLo + kPadHi;
    s.esize = esize;
    const uint64_t img = (uint64_t)s.Wp * s.Hp * pixel_bytes(esize, layout);
    s.proj_stride = (img + 255) & ~uint64_t(255);
    s.row_begin = row_begin;
    return s;
}

void load_env_tuning()
{
    if (g_tune.env_loaded) return;
    g_tune.env_loaded = true;
    const char* path = std::getenv("FDK_TUNING_FILE");
    if (path != nullptr && *path) (void)fdk_load_tuning(path);
    const char* stage = std::getenv("FDK_STAGE_FP32");
    g_tune.stage_fp32 = stage != nullptr && std::strcmp(stage, "1") == 0;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int32_t fdk_abi_version(void) { return FDK_ABI_VERSION; }

const char* fdk_status_string(fdk_status st)
{
    switch (st) {
    case FDK_OK: return "FDK_OK";
    case FDK_E_INVALID_ARG: return "FDK_E_INVALID_ARG";
    case FDK_E_GEOMETRY: return "FDK_E_GEOMETRY";
    case FDK_E_UNSUPPORTED: return "FDK_E_UNSUPPORTED";
    case FDK_E_NOMEM: return "FDK_E_NOMEM";
    case FDK_E_DEVICE: return "FDK_E_DEVICE";
    }
    return "FDK_E_UNKNOWN";
}

const char* fdk_last_error(void) { return g_last_error.c_str(); }

fdk_status fdk_normalize_matrices(double* mats, int32_t n_proj)
{
    g_last_error.clear();
    if (mats == nullptr) return fail(FDK_E_INVALID_ARG, "mats is NULL");
    if (n_proj < 1) return fail(FDK_E_INVALID_ARG, "n_proj=%d < 1", n_proj);
    for (int64_t i = 0; i < (int64_t)n_proj * 12; ++i)
        if (!std::isfinite(mats[i])) return fail(FDK_E_INVALID_ARG, "matrix %lld has a non-finite entry", (long long)(i / 12));
    for (int k = 0; k < n_proj; ++k) {
        const double* A = mats + 12 * (size_t)k;
        const double n = std::sqrt(A[8] * A[8] + A[9] * A[9] + A[10] * A[10]);
        if (!(n > 0.0)) return fail(FDK_E_INVALID_ARG, "matrix %d: third row has no direction", k);
        if (A[11] == 0.0) return fail(FDK_E_INVALID_ARG, "matrix %d: w = 0 at the origin", k);
    }
    for (int k = 0; k < n_proj; ++k) {
        double* A = mats + 12 * (size_t)k;
        const double n = std::sqrt(A[8] * A[8] + A[9] * A[9] + A[10] * A[10]);
        const double s = (A[11] > 0.0 ? 1.0 : -1.0) / n;
        for (int i = 0; i < 12; ++i) A[i] *= s;
    }
    return FDK_OK;
}

fdk_status fdk_validate(const fdk_volume* vol, const fdk_projections* proj, int need_data)
{
    g_last_error.clear();
    fdk_status st = check_volume(vol);
    if (st != FDK_OK) return st;
    st = check_proj(proj, need_data != 0);
    if (st != FDK_OK) return st;
    return check_geometry(vol, proj);
}

}  // extern "C": host helpers below have C++ linkage

namespace {

// The backprojection of one (slab of a) volume.  `pre`: the slab's composed
// coefficients from a table the caller owns (out-of-core calls compose all
// their slabs at once), or null to look them up by geometry.  `used`: where
// the caller wants an event recorded once the coefficients have been read.
fdk_status backproject_impl(const fdk_volume* vol, const fdk_projections* proj, float* volume, int accumulate,
                            hipStream_t s, const CoefSlab* pre, hipEvent_t used)
{
    fdk_status st;
    const int es = esize_of(proj->dtype);
    const TileShape t = fit_layout(pick_tile(vol->L, proj->dtype), proj, es);
    TileArgs probe = make_args(vol, proj, es, t, nullptr, nullptr, volume, 1.0f, accumulate, proj->dtype);
    if ((st = check_grid(probe)) != FDK_OK) return st;

    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    // FP32 stacks sampled from LDS windows can be read in place (bounds-checked
    // window loads, ~2.5% slower per sample than from the zero-bordered
    // staged copy): done when staging would be the larger cost, i.e. when the
    // grid is small against the stack (below 1/8 of a voxel per pixel);
    // every other stack is staged
    const bool raw = proj->dtype == FDK_F32 && t.layout == 3 && !g_tune.stage_fp32 &&
                     (double)vol->z_count * vol->L * vol->L * 8.0 <
                         (double)proj->n_proj * proj->width * proj->height;
    hipError_t e = hipSuccess;
    if (!raw) {
        e = ensure(d->staged, staged_bytes(proj, es, t.layout));
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "staging workspace: %s", hipGetErrorString(e));
    }
    e = ensure(d->coef_dev, (size_t)proj->n_proj * 16 * sizeof(double));
    if (e != hipSuccess) return fail(FDK_E_NOMEM, "coefficient workspace: %s", hipGetErrorString(e));
    CoefSlab cf;
    CoefEntry* ce = nullptr;
    if (pre != nullptr) {
        cf = *pre;
    } else {
        if ((st = coef_table(*d, vol, proj, s, &ce)) != FDK_OK) return st;
        cf = ce->slab(0);
    }

    if (!raw) {
        StageArgs sa = make_stage(proj, es, t.layout, static_cast<unsigned char*>(d->staged.p), 0);
        ProfScope ps("stage", s);
        HIP_TRY(launch_stage(sa, s));
    }
    {
        ProfScope ps("fold", s);
        HIP_TRY(launch_fold_single(cf.dev, proj->scale, static_cast<double*>(d->coef_dev.p), proj->n_proj, s));
    }
    if (ce != nullptr) HIP_TRY(hipEventRecord(ce->used, s));
    if (used != nullptr) HIP_TRY(hipEventRecord(used, s));
    TileArgs a = make_args(vol, proj, es, t, static_cast<unsigned char*>(d->staged.p),
                           static_cast<double*>(d->coef_dev.p), volume, cf.out_scale, accumulate, proj->dtype);
    a.const_w = cf.const_w;
    if (raw) {   // the caller's unpadded images, row pitch W
        const uint64_t img = (uint64_t)proj->width * proj->height * 4;
        a.proj = static_cast<const unsigned char*>(proj->data);
        a.proj_stride = img;
        a.proj_bytes = (uint32_t)img;
        a.row_bytes = (uint32_t)proj->width * 4;
        a.raw = 1;
    }
    if (t.layout == 3) {
        const uint64_t nwin = (uint64_t)a.tiles_x * a.tiles_y * a.tiles_z * proj->n_proj;
        e = ensure(d->windows, window_table_bytes(nwin));
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "window table: %s", hipGetErrorString(e));
        Win* win = static_cast<Win*>(d->windows.p);
        Anc* anc = reinterpret_cast<Anc*>(static_cast<unsigned char*>(d->windows.p) + anc_offset(nwin));
        a.win = win;
        a.anc = anc;
        ProfScope ps("window", s);
        HIP_TRY(launch_window(a, t.strip, t.waves, win, anc, s));
    }
    {
        ProfScope ps("bp", s);
        HIP_TRY(launch_bp(a, t.strip, t.waves, s));
    }
    return end_call(*d, s);
}

}  // namespace

extern "C" {

fdk_status fdk_backproject(const fdk_volume* vol, const fdk_projections* proj, float* volume,
                           int accumulate, void* stream)
{
    fdk_status st = fdk_validate(vol, proj, 1);
    if (st != FDK_OK) return st;
    if (volume == nullptr) return fail(FDK_E_INVALID_ARG, "volume buffer is NULL");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    return backproject_impl(vol, proj, volume, accumulate, static_cast<hipStream_t>(stream), nullptr, nullptr);
}

fdk_status fdk_backproject_noalloc(const fdk_volume* vol, const fdk_projections* proj, float* volume,
                                   int accumulate, void* stream)
{
    fdk_status st = fdk_validate(vol, proj, 1);
    if (st != FDK_OK) return st;
    if (volume == nullptr) return fail(FDK_E_INVALID_ARG, "volume buffer is NULL");
    if (proj->dtype != FDK_F32)
        return fail(FDK_E_UNSUPPORTED, "the allocation-free backprojection reads FP32 projections only");
    if (proj->n_proj > kNoAllocMaxProj)
        return fail(FDK_E_INVALID_ARG, "n_proj=%d exceeds the allocation-free maximum of %d", proj->n_proj,
                    kNoAllocMaxProj);
    if ((uint64_t)proj->width * proj->height * 4 > 0xffffffffull)
        return fail(FDK_E_INVALID_ARG, "projection of %dx%d pixels exceeds 4 GiB", proj->width, proj->height);
    // one tile shape: 16 x 16 columns, 16 planes deep; z-chunks of whole tile
    // layers whose window tables fit the scratch
    constexpr int kStrip = 16, kWaves = 4, kSide = 16;
    const uint64_t tiles_xy = (uint64_t)((vol->L + kSide - 1) / kSide) * ((vol->L + kSide - 1) / kSide);
    const uint64_t layer_bytes = tiles_xy * (uint64_t)proj->n_proj * sizeof(Win);
    const uint64_t budget = kScratchBytes - kScratchWin;
    if (layer_bytes > budget)
        return fail(FDK_E_INVALID_ARG,
                    "grid of %d^2 columns x %d projections needs %llu bytes of window table per 16 planes; the "
                    "allocation-free scratch holds %llu", vol->L, proj->n_proj, (unsigned long long)layer_bytes,
                    (unsigned long long)budget);
    const int chunk_planes = (int)std::min<uint64_t>(budget / layer_bytes, 1u << 20) * kStrip;
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    float out_scale = 1.0f;
    int const_w = 0;
    compose_into(vol, proj, g_noalloc_coef, &out_scale, &const_w);
    for (int i = 0; i < proj->n_proj * 12; ++i)
        if (!std::isfinite((float)g_noalloc_coef[i]))
            return fail(FDK_E_INVALID_ARG, "composed projection matrix exceeds FP32 range");
    double* folded = reinterpret_cast<double*>(d->scratch + kScratchFolded);
    double* composed = reinterpret_cast<double*>(d->scratch + kScratchComposed);
    Win* win = reinterpret_cast<Win*>(d->scratch + kScratchWin);
    // from pageable memory: the runtime has read the source when the call returns
    HIP_TRY(hipMemcpyAsync(composed, g_noalloc_coef, (size_t)proj->n_proj * 12 * sizeof(double),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fold_single(composed, proj->scale, folded, proj->n_proj, s));
    const TileShape t{kStrip, kWaves, 3};
    const size_t plane = (size_t)vol->L * vol->L;
    for (int z0 = 0; z0 < vol->z_count; z0 += chunk_planes) {
        fdk_volume cv = *vol;
        cv.z_begin = vol->z_begin + z0;
        cv.z_count = std::min(chunk_planes, vol->z_count - z0);
        TileArgs a = make_args(&cv, proj, 4, t, nullptr, folded, volume + (size_t)z0 * plane, out_scale, accumulate,
                               FDK_F32);
        // the caller's unpadded images, row pitch W, sampled through LDS windows
        const uint64_t img = (uint64_t)proj->width * proj->height * 4;
        a.proj = static_cast<const unsigned char*>(proj->data);
        a.proj_stride = img;
        a.proj_bytes = (uint32_t)img;
        a.row_bytes = (uint32_t)proj->width * 4;
        a.raw = 1;
        a.const_w = const_w;
        a.win = win;
        a.anc = nullptr;
        HIP_TRY(launch_window(a, kStrip, kWaves, win, nullptr, s));
        HIP_TRY(launch_bp_lanes(a, s));
    }
    return end_call(*d, s);
}

// Forward projection by detector-tile ownership: each workgroup owns t.strip
// detector rows (as many columns as fit its LDS) of t.waves projections and
// writes them once, straight into the caller's stack.
static fdk_status forwardproject_tiles(const fdk_volume* vol, const float* volume, const fdk_projections* geom,
                                float* proj_out, int accumulate, void* stream, TileShape t)
{
    fdk_status st;
    BandArgs b{};
    b.th = std::min(t.strip, geom->height);
    b.tw = std::min(geom->width, kBandCap / ((b.th + 2 * kBandBorder) * t.waves) - 2 * kBandBorder);
    // the kernel rounds the tile pitch up to an odd number of accumulators
    if ((int64_t)((b.tw + 2 * kBandBorder) | 1) * (b.th + 2 * kBandBorder) * t.waves > kBandCap) b.tw -= 1;
    b.tiles_u = (geom->width + b.tw - 1) / b.tw;
    b.tiles_v = (geom->height + b.th - 1) / b.th;
    if ((int64_t)b.tiles_u * b.tiles_v * ((geom->n_proj + t.waves - 1) / t.waves) > 0x7fffffffLL)
        return fail(FDK_E_INVALID_ARG, "detector tile grid too large");
    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    hipError_t e = ensure(d->coef_dev, (size_t)geom->n_proj * 16 * sizeof(double));
    if (e != hipSuccess) return fail(FDK_E_NOMEM, "coefficient workspace: %s", hipGetErrorString(e));
    CoefEntry* ce = nullptr;
    if ((st = coef_table(*d, vol, geom, s, &ce)) != FDK_OK) return st;
    const CoefSlab cf = ce->slab(0);
    {
        ProfScope ps("fold", s);
        HIP_TRY(launch_fold_single(cf.dev, nullptr, static_cast<double*>(d->coef_dev.p), geom->n_proj, s));
    }
    HIP_TRY(hipEventRecord(ce->used, s));
    const float out_scale = cf.out_scale;
    b.const_w = cf.const_w;
    b.coef = static_cast<const double*>(d->coef_dev.p);
    b.vol = volume;
    b.out = proj_out;
    b.n_proj = geom->n_proj;
    b.L = vol->L;
    b.z_begin = vol->z_begin;
    b.z_count = vol->z_count;
    b.ctr = vol->L / 2;
    b.W = geom->width;
    b.H = geom->height;
    b.cu = geom->width / 2;
    b.cv = geom->height / 2;
    b.out_scale = out_scale;
    b.accumulate = accumulate;
    {
        ProfScope ps("fp", s);
        HIP_TRY(launch_fp_band(b, t.waves, s));
    }
    return end_call(*d, s);
}

fdk_status fdk_forwardproject(const fdk_volume* vol, const float* volume, const fdk_projections* geom,
                              float* proj_out, int accumulate, void* stream)
{
    fdk_status st = fdk_validate(vol, geom, 0);
    if (st != FDK_OK) return st;
    if (volume == nullptr) return fail(FDK_E_INVALID_ARG, "volume buffer is NULL");
    if (proj_out == nullptr) return fail(FDK_E_INVALID_ARG, "projection output is NULL");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    const TileShape t = pick_tile(vol->L, kAdjointSlot);
    if (t.layout == 4) return forwardproject_tiles(vol, volume, geom, proj_out, accumulate, stream, t);
    TileArgs probe = make_args(vol, geom, 4, t, nullptr, nullptr, nullptr, 1.0f, 0, FDK_F32);
    if ((st = check_grid(probe)) != FDK_OK) return st;

    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    const uint64_t bytes = staged_bytes(geom, 4, 0);
    hipError_t e = ensure(d->adjoint, bytes);
    if (e != hipSuccess) return fail(FDK_E_NOMEM, "adjoint workspace: %s", hipGetErrorString(e));
    e = ensure(d->coef_dev, (size_t)geom->n_proj * 16 * sizeof(double));
    if (e != hipSuccess) return fail(FDK_E_NOMEM, "coefficient workspace: %s", hipGetErrorString(e));
    CoefEntry* ce = nullptr;
    if ((st = coef_table(*d, vol, geom, s, &ce)) != FDK_OK) return st;
    const CoefSlab cf = ce->slab(0);
    const float out_scale = cf.out_scale;

    {
        ProfScope ps("fill", s);
        HIP_TRY(launch_fill(static_cast<float*>(d->adjoint.p), bytes / 4, 0.0f, s));
    }
    {
        ProfScope ps("fold", s);
        HIP_TRY(launch_fold_single(cf.dev, nullptr, static_cast<double*>(d->coef_dev.p), geom->n_proj, s));
    }
    HIP_TRY(hipEventRecord(ce->used, s));
    TileArgs a = make_args(vol, geom, 4, t, static_cast<unsigned char*>(d->adjoint.p),
                           static_cast<double*>(d->coef_dev.p), const_cast<float*>(volume), out_scale, 0,
                           FDK_F32);
    {
        ProfScope ps("fp", s);
        HIP_TRY(launch_fp(a, t.strip, t.waves, s));
    }
    const int Wp = staged_pitch(geom->width);
    {
        ProfScope ps("unstage", s);
        HIP_TRY(launch_unstage_add(static_cast<const float*>(d->adjoint.p), proj_out, geom->n_proj, geom->width,
                                   geom->height, Wp, a.proj_stride / 4, accumulate, s));
    }
    return end_call(*d, s);
}

// ------------------------------------------------------------------ FDK preprocessing
}  // extern "C": host helpers below have C++ linkage

namespace {

constexpr int kMaxFilterWidth = 2048;   // FFT size 4096: 1.25 x 4096 FP64 complex = 80 KiB of LDS
constexpr size_t kFilterCacheMax = 2;

double ramp_tap(int64_t n, double tau)
{
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if (n % 2 == 0) return 0.0;
    const double a = (double)n * M_PI * tau;
    return -1.0 / (a * a);
}

double parker(double beta, double gamma, double range)
{
    if (range <= 0.0) return 1.0;
    const double d = 0.5 * (range - M_PI);
    if (beta < 0.0 || beta > M_PI + 2.0 * d) return 0.0;
    if (beta < 2.0 * d - 2.0 * gamma) {
        const double s = std::sin(M_PI / 4.0 * beta / (d - gamma));
        return s * s;
    }
    if (beta <= M_PI - 2.0 * gamma) return 1.0;
    const double s = std::sin(M_PI / 4.0 * (M_PI + 2.0 * d - beta) / (d + gamma));
    return s * s;
}

// Circular length of the row filter: the shortest 2^k or 5 * 2^k (k >= 2)
// of at least 2 W - 1 (1248-pixel rows: 2560 instead of 4096).
int filter_size(int W)
{
    int M = 4;
    while (M < 2 * W - 1) M <<= 1;
    int M5 = 20;
    while (M5 < 2 * W - 1) M5 <<= 1;
    return std::min(M, M5);
}

fdk_status check_filter(const fdk_filter_geometry* g)
{
    if (g == nullptr) return fail(FDK_E_INVALID_ARG, "filter geometry is NULL");
    if (g->reserved != 0) return fail(FDK_E_INVALID_ARG, "reserved field must be 0");
    if (g->n_proj < 1 || g->height < 1 || g->width < 1 || g->width > kMaxFilterWidth)
        return fail(FDK_E_INVALID_ARG, "n_proj=%d width=%d height=%d (width 1 .. %d)", g->n_proj, g->width,
                    g->height, kMaxFilterWidth);
    if ((int64_t)g->n_proj * g->height * g->width > (int64_t(1) << 40))
        return fail(FDK_E_INVALID_ARG, "projection stack too large");
    const double v[] = {g->pixel_u_mm, g->pixel_v_mm, g->u0, g->v0, g->sdd_mm, g->sid_mm, g->scan_range_rad,
                        g->dbeta_rad};
    for (double x : v)
        if (!std::isfinite(x)) return fail(FDK_E_INVALID_ARG, "non-finite filter geometry");
    if (g->pixel_u_mm <= 0.0 || g->pixel_v_mm <= 0.0 || g->sdd_mm <= 0.0 || g->sid_mm <= 0.0)
        return fail(FDK_E_INVALID_ARG, "pixel pitch and distances must be positive");
    if (g->fan_sign != 1.0 && g->fan_sign != -1.0) return fail(FDK_E_INVALID_ARG, "fan_sign must be +1 or -1");
    if (g->angles_rad == nullptr) return fail(FDK_E_INVALID_ARG, "angles_rad is NULL");
    for (int k = 0; k < g->n_proj; ++k)
        if (!std::isfinite(g->angles_rad[k])) return fail(FDK_E_INVALID_ARG, "angle %d is not finite", k);
    if (g->scan_range_rad > 0.0) {
        double gmax = 0.0;
        for (int i : {0, g->width - 1})
            gmax = std::max(gmax, std::fabs(std::atan(((double)i - g->u0) * g->pixel_u_mm / g->sdd_mm)));
        if (0.5 * (g->scan_range_rad - M_PI) < gmax)
            return fail(FDK_E_GEOMETRY, "scan range %.4f rad too short for Parker weights (fan half-angle %.4f)",
                        g->scan_range_rad, gmax);
    }
    return FDK_OK;
}

std::string filter_key(const fdk_filter_geometry* g)
{
    std::string key;
    auto put = [&key](const void* x, size_t n) { key.append(static_cast<const char*>(x), n); };
    put(g, offsetof(fdk_filter_geometry, angles_rad));
    put(&g->scan_range_rad, 3 * sizeof(double));
    put(g->angles_rad, (size_t)g->n_proj * sizeof(double));
    return key;
}

// Tables of one geometry: kernel spectrum (gain / M folded in), twiddles,
// cosine weights (H x W) and short-scan weights (N x W), all from FP64.
// Frequency held at each position after the in-place decimation-in-frequency
// FFT of length M (a radix-2 stage first when log2 M is odd, then radix-4):
// a stage of radix r over blocks of n leaves sub-spectrum d (frequencies
// d + r k) in the d-th block of n / r, so p = d (n / r) + p' holds
// d + r f'(p').
std::vector<int> dif_order(int M)
{
    // the kernel's stages: radix 5 first when 5 divides M, then radix 2 when
    // the power of two left has an odd exponent, then radix 4
    std::vector<int> radix;
    int m = M;
    if (m % 5 == 0) {
        radix.push_back(5);
        m /= 5;
    }
    int lg = 0;
    while ((1 << lg) < m) ++lg;
    if (lg & 1) radix.push_back(2);
    for (int i = 0; i < lg / 2; ++i) radix.push_back(4);
    std::vector<int> order(M);
    for (int p = 0; p < M; ++p) {
        int n = M, rest = p, f = 0, mult = 1;
        for (int r : radix) {
            const int sub = n / r, d = rest / sub;
            f += d * mult;
            mult *= r;
            rest -= d * sub;
            n = sub;
        }
        order[p] = f;
    }
    return order;
}

fdk_status filter_tables(DeviceState& d, const fdk_filter_geometry* g, hipStream_t s, FilterEntry** out)
{
    std::string key = filter_key(g);
    for (auto it = d.filter_cache.begin(); it != d.filter_cache.end(); ++it) {
        if (it->key == key) {
            d.filter_cache.splice(d.filter_cache.begin(), d.filter_cache, it);
            *out = &d.filter_cache.front();
            return FDK_OK;
        }
    }
    const int W = g->width, H = g->height, N = g->n_proj, M = filter_size(W);
    const double tau = g->pixel_u_mm * g->sid_mm / g->sdd_mm;
    const double gain = tau * g->dbeta_rad * g->sid_mm * g->sid_mm / (double)M;
    // spectrum of the circular kernel: h even and zero for |n| >= W, so
    // H[m] = h(0) + 2 sum_{n = 1 .. W-1} h(n) cos(2 pi m n / M)
    std::vector<double> cosv(M);
    for (int t = 0; t < M; ++t) cosv[t] = std::cos(2.0 * M_PI * (double)t / (double)M);
    std::vector<double> hs(M), wc((size_t)H * W), wp((size_t)N * W);
    std::vector<double> tw((size_t)M / 2);   // M/4 complex
    // the kernel works on the spectrum in the order its in-place decimation-
    // in-frequency FFT leaves it: position p holds frequency dif_order(p)
    const std::vector<int> order = dif_order(M);
    for (int p = 0; p < M; ++p) {
        const int m = order[p];
        double acc = ramp_tap(0, tau);
        for (int n = 1; n < W; n += 2) acc += 2.0 * ramp_tap(n, tau) * cosv[(int)(((int64_t)m * n) % M)];
        hs[p] = acc * gain;
    }
    for (int t = 0; t < M / 4; ++t) {
        tw[2 * t] = cosv[t];
        tw[2 * t + 1] = -std::sin(2.0 * M_PI * (double)t / (double)M);
    }
    for (int j = 0; j < H; ++j) {
        const double v = ((double)j - g->v0) * g->pixel_v_mm;
        for (int i = 0; i < W; ++i) {
            const double u = ((double)i - g->u0) * g->pixel_u_mm;
            wc[(size_t)j * W + i] = g->sdd_mm / std::sqrt(g->sdd_mm * g->sdd_mm + u * u + v * v);
        }
    }
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < W; ++i) {
            const double u = ((double)i - g->u0) * g->pixel_u_mm;
            wp[(size_t)k * W + i] = parker(g->angles_rad[k], g->fan_sign * std::atan(u / g->sdd_mm), g->scan_range_rad);
        }
    if (d.filter_cache.size() >= kFilterCacheMax) {
        HIP_TRY(hipDeviceSynchronize());
        FilterEntry& b = d.filter_cache.back();
        release(b.hs); release(b.tw); release(b.wc); release(b.wp);
        d.filter_cache.pop_back();
    }
    FilterEntry f;
    f.key = std::move(key);
    f.M = M;
    const size_t dsz = sizeof(double);
    hipError_t e = ensure(f.hs, hs.size() * dsz);
    if (e == hipSuccess) e = ensure(f.tw, tw.size() * dsz);
    if (e == hipSuccess) e = ensure(f.wc, wc.size() * dsz);
    if (e == hipSuccess) e = ensure(f.wp, wp.size() * dsz);
    if (e == hipSuccess) e = hipMemcpyAsync(f.hs.p, hs.data(), hs.size() * dsz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f.tw.p, tw.data(), tw.size() * dsz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f.wc.p, wc.data(), wc.size() * dsz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f.wp.p, wp.data(), wp.size() * dsz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release(f.hs); release(f.tw); release(f.wc); release(f.wp);
        return fail(FDK_E_NOMEM, "filter tables: %s", hipGetErrorString(e));
    }
    d.filter_cache.push_front(std::move(f));
    *out = &d.filter_cache.front();
    return FDK_OK;
}

}  // namespace

extern "C" {

fdk_status fdk_filter_projections(const fdk_filter_geometry* g, const float* src, void* dst, int32_t dtype,
                                  float* scale_out, void* stream)
{
    g_last_error.clear();
    fdk_status st = check_filter(g);
    if (st != FDK_OK) return st;
    if (src == nullptr || dst == nullptr) return fail(FDK_E_INVALID_ARG, "NULL projection pointer");
    if (dtype != FDK_F32 && dtype != FDK_F16 && dtype != FDK_BF16) return fail(FDK_E_UNSUPPORTED, "dtype %d", dtype);
    if (dtype != FDK_F32 && scale_out == nullptr) return fail(FDK_E_INVALID_ARG, "scale_out is NULL");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    FilterEntry* f = nullptr;
    if ((st = filter_tables(*d, g, s, &f)) != FDK_OK) return st;
    FilterArgs a;
    a.src = src;
    a.dst = static_cast<float*>(dst);
    a.wc = static_cast<const double*>(f->wc.p);
    a.wp = static_cast<const double*>(f->wp.p);
    a.hs = static_cast<const double*>(f->hs.p);
    a.tw = static_cast<const double2*>(f->tw.p);
    a.n_proj = g->n_proj;
    a.W = g->width;
    a.H = g->height;
    a.M = f->M;
    a.wave_max = nullptr;
    if (dtype == FDK_F32) {
        ProfScope ps("filter", s);
        HIP_TRY(launch_filter(a, s));
        return end_call(*d, s);
    }
    // FP16/BF16 output: the stack is filtered into an FP32 workspace, each
    // wave recording the largest magnitude it wrote; one small kernel takes
    // the maximum per projection and one pass packs the stack.  (Filtering in
    // chunks through a ring that stays in the memory-side cache measured
    // slower: the chunk boundaries cost more than the cached re-read saves.)
    const int64_t per = (int64_t)g->height * g->width;
    const int64_t wave_per = (int64_t)((g->height + 1) / 2) * kFilterWaves;
    hipError_t e = ensure(d->filter_ws, (size_t)g->n_proj * per * sizeof(float));
    if (e == hipSuccess)
        e = ensure(d->filter_max, (size_t)g->n_proj * (wave_per * sizeof(float) + sizeof(unsigned)));
    if (e != hipSuccess) return fail(FDK_E_NOMEM, "filter workspace: %s", hipGetErrorString(e));
    float* wave_max = static_cast<float*>(d->filter_max.p);
    unsigned* maxbits = reinterpret_cast<unsigned*>(wave_max + (size_t)g->n_proj * wave_per);
    a.dst = static_cast<float*>(d->filter_ws.p);
    a.wave_max = wave_max;
    {
        ProfScope ps("filter", s);
        HIP_TRY(launch_filter(a, s));
        HIP_TRY(launch_filter_max(a, maxbits, s));
    }
    {
        ProfScope ps("pack", s);
        HIP_TRY(launch_pack_known_max(a.dst, g->n_proj, g->width, g->height, dtype, dst, maxbits, scale_out, s));
    }
    return end_call(*d, s);
}

// ------------------------------------------------------------------ iterative solvers
// CGLS and SIRT for A x = p with A = fdk_forwardproject and A^T =
// fdk_backproject.  Each iteration is a forward and a backprojection (the
// projector entry points, called with the library lock held) plus the vector
// kernels of fdk_iter.hip; step lengths stay in device memory.
}  // extern "C": host helpers below have C++ linkage

namespace {

// SIRT weights: 1 / max(sum, kSirtFloor * largest sum)
constexpr double kSirtFloor = 1e-3;

struct IterSetup {
    DeviceState* d = nullptr;
    hipStream_t s = nullptr;
    int64_t nv = 0, np = 0;
    float *p0 = nullptr, *p1 = nullptr, *v0 = nullptr, *v1 = nullptr;
    double *part = nullptr, *st = nullptr;
};

fdk_status iter_setup(const fdk_volume* vol, const fdk_projections* proj, float* volume, int32_t n_iter,
                      const double* history, void* stream, IterSetup& it)
{
    fdk_status st = fdk_validate(vol, proj, 1);
    if (st != FDK_OK) return st;
    if (proj->dtype != FDK_F32) return fail(FDK_E_UNSUPPORTED, "iterative solvers take FP32 projections");
    if (volume == nullptr) return fail(FDK_E_INVALID_ARG, "volume buffer is NULL");
    if (n_iter < 0) return fail(FDK_E_INVALID_ARG, "n_iter=%d < 0", n_iter);
    if (history != nullptr) {   // written by a kernel: it must be device (or managed) memory
        hipPointerAttribute_t attr{};
        const bool ok = hipPointerGetAttributes(&attr, history) == hipSuccess &&
                        (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
        (void)hipGetLastError();
        if (!ok) return fail(FDK_E_INVALID_ARG, "history is not device memory");
    }
    if ((st = device_state(&it.d)) != FDK_OK) return st;
    it.s = static_cast<hipStream_t>(stream);
    it.nv = (int64_t)vol->z_count * vol->L * vol->L;
    it.np = (int64_t)proj->n_proj * proj->height * proj->width;
    DeviceState& d = *it.d;
    const size_t pb = (size_t)it.np * 4, vb = (size_t)it.nv * 4;
    for (auto [b, bytes] : {std::pair<DevBuf*, size_t>{&d.it_p0, pb}, {&d.it_p1, pb}, {&d.it_v0, vb},
                            {&d.it_v1, vb}, {&d.it_part, kRedBlocks * sizeof(double)},
                            {&d.it_st, kStSlots * sizeof(double)}}) {
        hipError_t e = ensure(*b, bytes);
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "solver workspace: %s", hipGetErrorString(e));
    }
    it.p0 = static_cast<float*>(d.it_p0.p);
    it.p1 = static_cast<float*>(d.it_p1.p);
    it.v0 = static_cast<float*>(d.it_v0.p);
    it.v1 = static_cast<float*>(d.it_v1.p);
    it.part = static_cast<double*>(d.it_part.p);
    it.st = static_cast<double*>(d.it_st.p);
    return begin_call(d, it.s);
}

// A^T applied to a projection-sized workspace vector.
fdk_status apply_bp(const fdk_volume* vol, const fdk_projections* proj, const float* src, float* dst,
                    hipStream_t s)
{
    fdk_projections q = *proj;
    q.data = src;
    q.dtype = FDK_F32;
    q.scale = nullptr;
    return fdk_backproject(vol, &q, dst, 0, s);
}

}  // namespace

extern "C" {

fdk_status fdk_cgls(const fdk_volume* vol, const fdk_projections* proj, float* volume, int32_t n_iter,
                    int use_x0, double* history, void* stream)
{
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    IterSetup it;
    fdk_status st = iter_setup(vol, proj, volume, n_iter, history, stream, it);
    if (st != FDK_OK) return st;
    const float* p = static_cast<const float*>(proj->data);
    float *r = it.p0, *q = it.p1, *sv = it.v0, *dv = it.v1;
    hipStream_t s = it.s;
    // r0 = p - A x0 (x0 = 0: r0 = p); the caller's volume is not written
    // before the first update, so a failing projector call leaves it intact.
    if (use_x0) {
        if ((st = fdk_forwardproject(vol, volume, proj, r, 0, s)) != FDK_OK) return st;
        ProfScope ps("iter", s);
        HIP_TRY(launch_residual(r, p, nullptr, it.np, it.part, s));
    } else {
        HIP_TRY(hipMemcpyAsync(r, p, it.np * 4, hipMemcpyDeviceToDevice, s));
        ProfScope ps("iter", s);
        HIP_TRY(launch_sumsq(r, it.np, it.part, s));
    }
    HIP_TRY(launch_scalar(it.part, it.st, history, kOpHist, 0, s));
    if ((st = apply_bp(vol, proj, r, sv, s)) != FDK_OK) return st;      // s0 = A^T r0
    {
        ProfScope ps("iter", s);
        HIP_TRY(launch_sumsq(sv, it.nv, it.part, s));
        HIP_TRY(launch_scalar(it.part, it.st, nullptr, kOpStore, kStGamma, s));
        HIP_TRY(hipMemcpyAsync(dv, sv, it.nv * 4, hipMemcpyDeviceToDevice, s));   // d0 = s0
        if (!use_x0) HIP_TRY(launch_fill(volume, (uint64_t)it.nv, 0.0f, s));
    }
    for (int k = 1; k <= n_iter; ++k) {
        if ((st = fdk_forwardproject(vol, dv, proj, q, 0, s)) != FDK_OK) return st;   // q = A d
        {
            ProfScope ps("iter", s);
            HIP_TRY(launch_sumsq(q, it.np, it.part, s));
            HIP_TRY(launch_scalar(it.part, it.st, nullptr, kOpAlpha, 0, s));
            HIP_TRY(launch_cgls_update(volume, dv, it.nv, r, q, it.np, it.st, it.part, s));
            HIP_TRY(launch_scalar(it.part, it.st, history, kOpHist, k, s));
        }
        if ((st = apply_bp(vol, proj, r, sv, s)) != FDK_OK) return st;  // s = A^T r
        ProfScope ps("iter", s);
        HIP_TRY(launch_sumsq(sv, it.nv, it.part, s));
        HIP_TRY(launch_scalar(it.part, it.st, nullptr, kOpBeta, 0, s));
        HIP_TRY(launch_cgls_direction(dv, sv, it.nv, it.st, s));
    }
    return end_call(*it.d, s);
}

fdk_status fdk_sirt(const fdk_volume* vol, const fdk_projections* proj, float* volume, int32_t n_iter,
                    double lambda, int32_t flags, double* history, void* stream)
{
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    if (!std::isfinite(lambda) || !(lambda > 0.0))
        return fail(FDK_E_INVALID_ARG, "lambda must be finite and > 0");
    if (flags & ~(FDK_SIRT_USE_X0 | FDK_SIRT_NONNEG)) return fail(FDK_E_INVALID_ARG, "unknown flags 0x%x", flags);
    IterSetup it;
    fdk_status st = iter_setup(vol, proj, volume, n_iter, history, stream, it);
    if (st != FDK_OK) return st;
    const float* p = static_cast<const float*>(proj->data);
    float *r = it.p0, *rw = it.p1, *t = it.v0, *cw = it.v1;
    hipStream_t s = it.s;
    // row sums A 1 -> rw, column sums A^T 1 -> cw, each inverted with the floor
    {
        ProfScope ps("iter", s);
        HIP_TRY(launch_fill(t, (uint64_t)it.nv, 1.0f, s));
        HIP_TRY(launch_fill(r, (uint64_t)it.np, 1.0f, s));
    }
    if ((st = fdk_forwardproject(vol, t, proj, rw, 0, s)) != FDK_OK) return st;
    if ((st = apply_bp(vol, proj, r, cw, s)) != FDK_OK) return st;
    {
        ProfScope ps("iter", s);
        HIP_TRY(launch_max(rw, it.np, it.part, s));
        HIP_TRY(launch_scalar(it.part, it.st, nullptr, kOpMax, kStRowMax, s));
        HIP_TRY(launch_inv_floor(rw, it.np, it.st, kStRowMax, kSirtFloor, s));
        HIP_TRY(launch_max(cw, it.nv, it.part, s));
        HIP_TRY(launch_scalar(it.part, it.st, nullptr, kOpMax, kStColMax, s));
        HIP_TRY(launch_inv_floor(cw, it.nv, it.st, kStColMax, kSirtFloor, s));
        if (!(flags & FDK_SIRT_USE_X0)) HIP_TRY(launch_fill(volume, (uint64_t)it.nv, 0.0f, s));
    }
    for (int k = 0; k < n_iter; ++k) {
        if ((st = fdk_forwardproject(vol, volume, proj, r, 0, s)) != FDK_OK) return st;   // A x
        {
            ProfScope ps("iter", s);
            HIP_TRY(launch_residual(r, p, rw, it.np, it.part, s));   // R (p - A x)
            HIP_TRY(launch_scalar(it.part, it.st, history, kOpHist, k, s));
        }
        if ((st = apply_bp(vol, proj, r, t, s)) != FDK_OK) return st;
        ProfScope ps("iter", s);
        HIP_TRY(launch_sirt_update(volume, t, cw, it.nv, lambda, (flags & FDK_SIRT_NONNEG) ? 1 : 0, s));
    }
    return end_call(*it.d, s);
}

// ------------------------------------------------------------------ out-of-core form
}  // extern "C": host helpers below have C++ linkage

namespace {

// Rows of the detector that the voxel centres of planes [z0, z0 + nz) can
// reach in projection k, widened by two rows on each side for the FP32
// rounding of the kernel's coordinates.  v/w is linear-fractional with w > 0
// over the box, so its extremes lie at the box's corners.  Returns false if
// the box projects entirely above or below the detector (then *below says
// which side).
bool band_rows(const fdk_volume* v, const double* A, int H, int z0, int nz, int* lo, int* hi, bool* below)
{
    double mn = 1e300, mx = -1e300;
    for (int c = 0; c < 8; ++c) {
        const double X = v->origin_mm[0] + ((c & 1) ? v->L - 1 : 0) * v->voxel_mm;
        const double Y = v->origin_mm[1] + ((c & 2) ? v->L - 1 : 0) * v->voxel_mm;
        const double Z = v->origin_mm[2] + ((c & 4) ? z0 + nz - 1 : z0) * v->voxel_mm;
        const double iy = (A[4] * X + A[5] * Y + A[6] * Z + A[7]) / (A[8] * X + A[9] * Y + A[10] * Z + A[11]);
        mn = std::min(mn, iy);
        mx = std::max(mx, iy);
    }
    const double l = std::floor(mn) - 2.0, h = std::floor(mx) + 3.0;
    *below = l > (double)(H - 1);
    if (h < 0.0 || l > (double)(H - 1)) return false;
    *lo = (int)std::max(l, 0.0);
    *hi = (int)std::min(h, (double)(H - 1));
    return true;
}

struct SlabPlan {
    int z0, nz, rows;
    std::vector<int> j0;         // first detector row of each projection's band
    std::vector<double> mats;    // matrices with the row offset folded in: v' = v - j0 w
};

std::vector<SlabPlan> plan_slabs(const fdk_volume* v, const fdk_projections* p, int slab_planes)
{
    std::vector<SlabPlan> plan;
    const int N = p->n_proj, H = p->height;
    for (int z0 = v->z_begin; z0 < v->z_begin + v->z_count; z0 += slab_planes) {
        SlabPlan sp;
        sp.z0 = z0;
        sp.nz = std::min(slab_planes, v->z_begin + v->z_count - z0);
        std::vector<int> lo(N), hi(N);
        std::vector<char> hit(N), below(N);
        sp.rows = 1;
        for (int k = 0; k < N; ++k) {
            bool b = false;
            hit[k] = band_rows(v, p->mats + 12 * k, H, sp.z0, sp.nz, &lo[k], &hi[k], &b);
            below[k] = b;
            if (hit[k]) sp.rows = std::max(sp.rows, hi[k] - lo[k] + 1);
        }
        sp.j0.resize(N);
        sp.mats.assign(p->mats, p->mats + 12 * (size_t)N);
        for (int k = 0; k < N; ++k) {
            // a band that misses the detector is placed on the side the box lies on,
            // so every tap stays off the band as it is off the detector
            int j = hit[k] ? std::min(lo[k], H - sp.rows) : (below[k] ? H - sp.rows : 0);
            sp.j0[k] = j;
            double* A = sp.mats.data() + 12 * (size_t)k;
            for (int c = 0; c < 4; ++c) A[4 + c] -= (double)j * A[8 + c];
        }
        plan.push_back(std::move(sp));
    }
    return plan;
}

fdk_status stream_init(DeviceState& d)
{
    if (d.h2d == nullptr) {
        HIP_TRY(hipStreamCreateWithFlags(&d.h2d, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&d.d2h, hipStreamNonBlocking));
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(hipEventCreateWithFlags(&d.band_ready[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&d.band_free[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&d.slab_done[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&d.slab_free[b], hipEventDisableTiming));
        }
        HIP_TRY(hipEventCreateWithFlags(&d.call_start, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&d.j0_read, hipEventDisableTiming));
    }
    return FDK_OK;
}

}  // namespace

extern "C" {

fdk_status fdk_backproject_streamed(const fdk_volume* vol, const fdk_projections* proj, float* volume,
                                    int32_t slab_planes, int32_t flags, int accumulate, void* stream)
{
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    fdk_status st = fdk_validate(vol, proj, 1);
    if (st != FDK_OK) return st;
    if (volume == nullptr) return fail(FDK_E_INVALID_ARG, "volume buffer is NULL");
    if (slab_planes < 1) return fail(FDK_E_INVALID_ARG, "slab_planes=%d < 1", slab_planes);
    if (flags & ~FDK_STREAM_HOST_VOLUME) return fail(FDK_E_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool host_vol = (flags & FDK_STREAM_HOST_VOLUME) != 0;
    DeviceState* d = nullptr;
    if ((st = device_state(&d)) != FDK_OK) return st;
    if ((st = stream_init(*d)) != FDK_OK) return st;
    hipStream_t cs = static_cast<hipStream_t>(stream);

    const std::vector<SlabPlan> plan = plan_slabs(vol, proj, slab_planes);
    const int N = proj->n_proj, W = proj->width, H = proj->height;
    const size_t es = (size_t)esize_of(proj->dtype);
    const size_t plane = (size_t)vol->L * vol->L;
    int max_rows = 1;
    for (const SlabPlan& sp : plan) max_rows = std::max(max_rows, sp.rows);
    // every slab's geometry is validated before anything is enqueued
    for (const SlabPlan& sp : plan) {
        fdk_volume sv = *vol;
        sv.z_begin = sp.z0;
        sv.z_count = sp.nz;
        fdk_projections bp = *proj;
        bp.height = sp.rows;
        bp.mats = sp.mats.data();
        if ((st = fdk_validate(&sv, &bp, 1)) != FDK_OK) return st;
    }
    for (int b = 0; b < 2; ++b) {
        // buffers about to be reallocated must be idle
        if (d->band[b].n < (size_t)N * max_rows * W * es ||
            (host_vol && d->slab[b].n < (size_t)slab_planes * plane * 4))
            HIP_TRY(hipDeviceSynchronize());
        hipError_t e = ensure(d->band[b], (size_t)N * max_rows * W * es);
        if (e == hipSuccess && host_vol) e = ensure(d->slab[b], (size_t)slab_planes * plane * 4);
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "streaming buffers: %s", hipGetErrorString(e));
    }
    // every slab's coefficients composed and uploaded at once (one cache entry)
    CoefEntry* ce = nullptr;
    {
        std::string key = coef_key(vol, proj);
        key.append("streamed", 8);
        key.append(reinterpret_cast<const char*>(&vol->z_begin), 2 * sizeof(int32_t));
        key.append(reinterpret_cast<const char*>(&slab_planes), sizeof(int32_t));
        std::vector<fdk_volume> svs(plan.size());
        std::vector<fdk_projections> bps(plan.size());
        std::vector<std::pair<const fdk_volume*, const fdk_projections*>> slabs;
        for (size_t i = 0; i < plan.size(); ++i) {
            svs[i] = *vol;
            svs[i].z_begin = plan[i].z0;
            svs[i].z_count = plan[i].nz;
            bps[i] = *proj;
            bps[i].height = plan[i].rows;
            bps[i].mats = plan[i].mats.data();
            slabs.emplace_back(&svs[i], &bps[i]);
        }
        if ((st = coef_lookup(*d, key, cs, slabs, &ce)) != FDK_OK) return st;
    }
    // the library's copy stream starts with the work the caller enqueued
    // before this call (the stack may be written by it)
    HIP_TRY(hipEventRecord(d->call_start, cs));
    HIP_TRY(hipStreamWaitEvent(d->h2d, d->call_start, 0));
    const unsigned char* src = static_cast<const unsigned char*>(proj->data);
    unsigned char* hvol = reinterpret_cast<unsigned char*>(volume);
    // a stack in device memory is gathered by one kernel per slab (the band
    // offsets in a device table); host memory goes through one DMA copy per band
    bool dev_src = false;
    {
        hipPointerAttribute_t attr{};
        if (hipPointerGetAttributes(&attr, proj->data) == hipSuccess) dev_src = attr.type == hipMemoryTypeDevice;
        (void)hipGetLastError();
    }
    if (dev_src) {
        std::vector<int32_t> j0s;
        j0s.reserve(plan.size() * (size_t)N);
        for (const SlabPlan& sp : plan) j0s.insert(j0s.end(), sp.j0.begin(), sp.j0.end());
        // the pinned source of the previous upload may still be unread, and a
        // table that must grow may still be read by earlier gathers
        if (d->j0_pending) HIP_TRY(hipEventSynchronize(d->j0_read));
        const size_t jb = j0s.size() * sizeof(int32_t);
        if (d->band_j0.n < jb) HIP_TRY(hipStreamSynchronize(d->h2d));
        hipError_t e = ensure(d->band_j0, jb);
        if (e == hipSuccess) e = ensure_host(d->band_j0_host, jb);
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "band table: %s", hipGetErrorString(e));
        std::memcpy(d->band_j0_host.p, j0s.data(), jb);
        // ordered after the earlier gathers on the same stream
        HIP_TRY(hipMemcpyAsync(d->band_j0.p, d->band_j0_host.p, jb, hipMemcpyHostToDevice, d->h2d));
        HIP_TRY(hipEventRecord(d->j0_read, d->h2d));
        d->j0_pending = true;
    }

    auto enqueue_in = [&](size_t s) -> fdk_status {
        const SlabPlan& sp = plan[s];
        const int b = (int)(s & 1);
        if (d->band_used[b]) HIP_TRY(hipStreamWaitEvent(d->h2d, d->band_free[b], 0));
        unsigned char* dst = static_cast<unsigned char*>(d->band[b].p);
        const size_t chunk = (size_t)sp.rows * W * es;
        if (dev_src) {
            HIP_TRY(launch_band_gather(src, dst, static_cast<const int32_t*>(d->band_j0.p) + s * (size_t)N, N, H,
                                       sp.rows, (int64_t)W * (int64_t)es, d->h2d));
        } else {
            for (int k = 0; k < N; ++k)
                HIP_TRY(hipMemcpyAsync(dst + (size_t)k * chunk, src + ((size_t)k * H + sp.j0[k]) * W * es, chunk,
                                       hipMemcpyDefault, d->h2d));
        }
        if (host_vol && accumulate) {
            if (d->slab_used[b]) HIP_TRY(hipStreamWaitEvent(d->h2d, d->slab_free[b], 0));
            HIP_TRY(hipMemcpyAsync(d->slab[b].p, hvol + (size_t)(sp.z0 - vol->z_begin) * plane * 4,
                                   (size_t)sp.nz * plane * 4, hipMemcpyDefault, d->h2d));
        }
        HIP_TRY(hipEventRecord(d->band_ready[b], d->h2d));
        return FDK_OK;
    };

    if ((st = enqueue_in(0)) != FDK_OK) return st;
    for (size_t s = 0; s < plan.size(); ++s) {
        if (s + 1 < plan.size() && (st = enqueue_in(s + 1)) != FDK_OK) return st;
        const SlabPlan& sp = plan[s];
        const int b = (int)(s & 1);
        HIP_TRY(hipStreamWaitEvent(cs, d->band_ready[b], 0));
        if (host_vol && !accumulate && d->slab_used[b]) HIP_TRY(hipStreamWaitEvent(cs, d->slab_free[b], 0));
        fdk_volume sv = *vol;
        sv.z_begin = sp.z0;
        sv.z_count = sp.nz;
        fdk_projections bp = *proj;
        bp.height = sp.rows;
        bp.mats = sp.mats.data();
        bp.data = d->band[b].p;
        float* out = host_vol ? static_cast<float*>(d->slab[b].p)
                              : volume + (size_t)(sp.z0 - vol->z_begin) * plane;
        const CoefSlab cf = ce->slab(s);
        if ((st = backproject_impl(&sv, &bp, out, accumulate, cs, &cf,
                                   s + 1 == plan.size() ? ce->used : nullptr)) != FDK_OK)
            return st;
        HIP_TRY(hipEventRecord(d->band_free[b], cs));
        d->band_used[b] = true;
        if (host_vol) {
            HIP_TRY(hipEventRecord(d->slab_done[b], cs));
            HIP_TRY(hipStreamWaitEvent(d->d2h, d->slab_done[b], 0));
            HIP_TRY(hipMemcpyAsync(hvol + (size_t)(sp.z0 - vol->z_begin) * plane * 4, d->slab[b].p,
                                   (size_t)sp.nz * plane * 4, hipMemcpyDefault, d->d2h));
            HIP_TRY(hipEventRecord(d->slab_free[b], d->d2h));
            d->slab_used[b] = true;
        }
    }
    // the caller's stream completes only when the volume is in place
    if (host_vol)
        for (int b = 0; b < 2; ++b)
            if (d->slab_used[b]) HIP_TRY(hipStreamWaitEvent(cs, d->slab_free[b], 0));
    return FDK_OK;
}

fdk_status fdk_streamed_plan(const fdk_volume* vol, const fdk_projections* proj, int32_t slab_planes,
                             int32_t* n_slabs, int32_t* band_rows, int32_t* first_rows)
{
    fdk_status st = fdk_validate(vol, proj, 0);
    if (st != FDK_OK) return st;
    if (slab_planes < 1) return fail(FDK_E_INVALID_ARG, "slab_planes=%d < 1", slab_planes);
    if (n_slabs == nullptr) return fail(FDK_E_INVALID_ARG, "n_slabs is NULL");
    const std::vector<SlabPlan> plan = plan_slabs(vol, proj, slab_planes);
    *n_slabs = (int32_t)plan.size();
    for (size_t s = 0; s < plan.size(); ++s) {
        if (band_rows) band_rows[s] = plan[s].rows;
        if (first_rows)
            std::copy(plan[s].j0.begin(), plan[s].j0.end(), first_rows + s * (size_t)proj->n_proj);
    }
    return FDK_OK;
}

fdk_status fdk_pack_projections(const float* src, int32_t n_proj, int32_t width, int32_t height,
                                int32_t dtype, void* dst, float* scale_out, void* stream)
{
    g_last_error.clear();
    if (src == nullptr || dst == nullptr || scale_out == nullptr)
        return fail(FDK_E_INVALID_ARG, "NULL pointer");
    if (n_proj < 1 || width < 1 || height < 1) return fail(FDK_E_INVALID_ARG, "empty projection stack");
    if (n_proj > 65535) return fail(FDK_E_INVALID_ARG, "n_proj=%d > 65535", n_proj);
    if (dtype != FDK_F16 && dtype != FDK_BF16) return fail(FDK_E_UNSUPPORTED, "pack dtype must be F16 or BF16");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    DeviceState* d = nullptr;
    fdk_status st = device_state(&d);
    if (st != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ProfScope ps("pack", s);
    HIP_TRY(launch_pack(src, n_proj, width, height, dtype, dst, scale_out, s));
    return FDK_OK;
}

fdk_status fdk_backproject_batched(const fdk_scan* scans, int32_t n_scans, int accumulate, void* stream)
{
    g_last_error.clear();
    if (scans == nullptr) return fail(FDK_E_INVALID_ARG, "scans is NULL");
    if (n_scans < 1 || n_scans > kMaxScans)
        return fail(FDK_E_INVALID_ARG, "n_scans=%d outside [1, %d]", n_scans, kMaxScans);
    int maxL = 0;
    for (int i = 0; i < n_scans; ++i) {
        fdk_status st = fdk_validate(&scans[i].vol, &scans[i].proj, 1);
        if (st != FDK_OK) {
            std::string m = g_last_error;
            return fail(st, "scan %d: %s", i, m.c_str());
        }
        if (scans[i].volume == nullptr) return fail(FDK_E_INVALID_ARG, "scan %d: volume buffer is NULL", i);
        maxL = std::max(maxL, scans[i].vol.L);
    }
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    // one tile shape (strip, waves) for the whole batch, from the batched slot;
    // FP32 scans take its layout, FP16/BF16 scans the layout of their own slot
    const TileShape t = pick_tile(maxL, kBatchedSlot);
    auto scan_layout = [&](const fdk_projections* p) {
        TileShape ts = t;
        if (p->dtype != FDK_F32) ts.layout = pick_tile(maxL, p->dtype).layout;
        return fit_layout(ts, p, esize_of(p->dtype)).layout;
    };
    DeviceState* d = nullptr;
    fdk_status st = device_state(&d);
    if (st != FDK_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // cache key: every descriptor field, the matrices, the tile shape and accumulate
    std::string key;
    auto put = [&key](const void* x, size_t n) { key.append(static_cast<const char*>(x), n); };
    put(&t, sizeof(t));
    put(&accumulate, sizeof(int));
    for (int i = 0; i < n_scans; ++i) {
        const fdk_scan& sc = scans[i];
        const int lay = scan_layout(&sc.proj);
        put(&lay, sizeof(int));
        put(&sc.vol, sizeof(fdk_volume));
        put(&sc.proj.n_proj, 4 * sizeof(int32_t));
        put(&sc.proj.data, sizeof(void*));
        put(&sc.proj.scale, sizeof(void*));
        put(&sc.volume, sizeof(void*));
        put(sc.proj.mats, (size_t)sc.proj.n_proj * 12 * sizeof(double));
    }

    // order: most expensive tiles (most projections) first
    std::vector<int> order(n_scans);
    for (int i = 0; i < n_scans; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return scans[a].proj.n_proj > scans[b].proj.n_proj; });
    // FP32 scans that sample from LDS read their windows straight from the
    // caller's images (bounds-checked loads); the others are staged
    auto is_raw = [&](const fdk_projections* p) {
        return p->dtype == FDK_F32 && scan_layout(p) == 3 && !g_tune.stage_fp32;
    };
    uint64_t stage_total = 0;
    std::vector<uint64_t> stage_off(n_scans);
    for (int j = 0; j < n_scans; ++j) {
        const int i = order[j];
        stage_off[j] = stage_total;
        const int es_i = esize_of(scans[i].proj.dtype);
        if (!is_raw(&scans[i].proj)) stage_total += staged_bytes(&scans[i].proj, es_i, scan_layout(&scans[i].proj));
    }

    if ((st = begin_call(*d, s)) != FDK_OK) return st;
    if (d->batch_staged.n < stage_total) {
        // growing the staging buffer invalidates every captured graph
        HIP_TRY(hipDeviceSynchronize());
        for (BatchEntry& b : d->batch_cache) {
            release_entry(b);
        }
        d->batch_cache.clear();
        hipError_t e = ensure(d->batch_staged, stage_total);
        if (e != hipSuccess) return fail(FDK_E_NOMEM, "batched staging workspace: %s", hipGetErrorString(e));
    }

    BatchEntry* hit = nullptr;
    for (auto it = d->batch_cache.begin(); it != d->batch_cache.end(); ++it) {
        if (it->key == key) {
            d->batch_cache.splice(d->batch_cache.begin(), d->batch_cache, it);
            hit = &d->batch_cache.front();
            break;
        }
    }
    if (hit == nullptr) {
        if (d->batch_cache.size() >= kBatchCacheMax) {
            HIP_TRY(hipDeviceSynchronize());
            BatchEntry& b = d->batch_cache.back();
            release_entry(b);
            d->batch_cache.pop_back();
        }
        // host tables
        int total_proj = 0;
        for (int i = 0; i < n_scans; ++i) total_proj += scans[i].proj.n_proj;
        std::vector<double> coef64;
        coef64.reserve((size_t)total_proj * 12);
        std::vector<const float*> scale_ptrs;
        scale_ptrs.reserve(total_proj);
        std::vector<TileArgs> tiles(n_scans);
        std::vector<StageArgs> stages;
        stages.reserve(n_scans);
        std::vector<int32_t> item_begin(n_scans + 1);
        std::vector<float> out_scales(n_scans);
        std::vector<int> const_ws(n_scans);
        std::vector<int> proj_begin(n_scans);
        std::vector<int64_t> win_off(n_scans);   // window table offset (layout 3) or -1
        uint64_t win_total = 0;
        int64_t rows = 0;
        int64_t items = 0;
        for (int j = 0; j < n_scans; ++j) {
            const fdk_scan& sc = scans[order[j]];
            Composed c = compose(&sc.vol, &sc.proj);
            for (double x : c.coef)
                if (!std::isfinite((float)x))
                    return fail(FDK_E_INVALID_ARG, "scan %d: composed matrix exceeds FP32 range", order[j]);
            proj_begin[j] = (int)(coef64.size() / 12);
            coef64.insert(coef64.end(), c.coef.begin(), c.coef.end());
            for (int k = 0; k < sc.proj.n_proj; ++k)
                scale_ptrs.push_back(sc.proj.scale ? sc.proj.scale + k : nullptr);
            out_scales[j] = c.out_scale;
            const_ws[j] = c.const_w;
            const int es = esize_of(sc.proj.dtype);
            TileShape ts = t;
            ts.layout = scan_layout(&sc.proj);
            if (!is_raw(&sc.proj)) {
                stages.push_back(make_stage(&sc.proj, es, ts.layout,
                                            static_cast<unsigned char*>(d->batch_staged.p) + stage_off[j], rows));
                rows += (int64_t)sc.proj.n_proj * stages.back().Hp;
            }
            item_begin[j] = (int32_t)items;
            TileArgs probe = make_args(&sc.vol, &sc.proj, es, ts, nullptr, nullptr, nullptr, 1.0f, 0, sc.proj.dtype);
            const int64_t n_tiles = (int64_t)probe.tiles_x * probe.tiles_y * probe.tiles_z;
            win_off[j] = ts.layout == 3 ? win_total : -1;
            if (ts.layout == 3) win_total += (uint64_t)n_tiles * sc.proj.n_proj;
            items += n_tiles;
            if (items > 0x7fffffffLL) return fail(FDK_E_INVALID_ARG, "batch too large for one launch");
        }
        item_begin[n_scans] = (int32_t)items;
        if (rows > 0x7fffffffLL) return fail(FDK_E_INVALID_ARG, "batch has too many projection rows");

        BatchEntry b;
        b.key = key;
        hipError_t e = hipSuccess;
        auto alloc = [&](DevBuf& buf, size_t n) { if (e == hipSuccess) e = ensure(buf, n); };
        alloc(b.tiles, n_scans * sizeof(TileArgs));
        alloc(b.item_begin, (n_scans + 1) * sizeof(int32_t));
        alloc(b.stage, std::max<size_t>(1, stages.size()) * sizeof(StageArgs));
        alloc(b.scale_ptrs, (size_t)total_proj * sizeof(float*));
        alloc(b.coef64, coef64.size() * sizeof(double));
        alloc(b.coef_dev, (size_t)total_proj * 16 * sizeof(double));
        alloc(b.counter, sizeof(unsigned));
        if (win_total > 0) alloc(b.windows, window_table_bytes(win_total));
        if (e != hipSuccess) {
            release_entry(b);
            return fail(FDK_E_NOMEM, "batched tables: %s", hipGetErrorString(e));
        }
        for (int j = 0; j < n_scans; ++j) {
            const fdk_scan& sc = scans[order[j]];
            TileShape ts = t;
            ts.layout = scan_layout(&sc.proj);
            tiles[j] = make_args(&sc.vol, &sc.proj, esize_of(sc.proj.dtype), ts,
                                 static_cast<unsigned char*>(d->batch_staged.p) + stage_off[j],
                                 static_cast<double*>(b.coef_dev.p) + (size_t)proj_begin[j] * 16, sc.volume,
                                 out_scales[j], accumulate, sc.proj.dtype);
            // LDS scans: the windows and the tile anchors of every (tile,
            // projection); circular orbits (u and w constant along z) take
            // the column walk
            tiles[j].const_w = const_ws[j];
            if (win_off[j] >= 0) {
                tiles[j].win = static_cast<const Win*>(b.windows.p) + win_off[j];
                tiles[j].anc = batch_anchors(b, win_total) + win_off[j];
            }
            if (is_raw(&sc.proj)) {   // the caller's unpadded images, row pitch W
                const uint64_t img = (uint64_t)sc.proj.width * sc.proj.height * 4;
                tiles[j].proj = static_cast<const unsigned char*>(sc.proj.data);
                tiles[j].proj_stride = img;
                tiles[j].proj_bytes = (uint32_t)img;
                tiles[j].row_bytes = (uint32_t)sc.proj.width * 4;
                tiles[j].raw = 1;
            }
        }
        auto up = [&](DevBuf& buf, const void* src, size_t n) {
            if (e == hipSuccess) e = hipMemcpyAsync(buf.p, src, n, hipMemcpyHostToDevice, s);
        };
        up(b.tiles, tiles.data(), tiles.size() * sizeof(TileArgs));
        up(b.item_begin, item_begin.data(), item_begin.size() * sizeof(int32_t));
        if (!stages.empty()) up(b.stage, stages.data(), stages.size() * sizeof(StageArgs));
        up(b.scale_ptrs, scale_ptrs.data(), scale_ptrs.size() * sizeof(float*));
        up(b.coef64, coef64.data(), coef64.size() * sizeof(double));
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && d->capture_stream == nullptr)
            e = hipStreamCreateWithFlags(&d->capture_stream, hipStreamNonBlocking);
        // capture: stage every stack, fold the scales, reset the queue, run the persistent kernel
        // (its column-walk-only form when every scan is an FP32 LDS scan on a circular orbit)
        int circular = 1;
        for (int j = 0; j < n_scans; ++j)
            circular &= (int)(tiles[j].dtype == FDK_F32 && tiles[j].layout == 3 && const_ws[j] == 2);
        hipGraph_t graph = nullptr;
        const int per_cu = batched_blocks_per_cu(t.strip, t.waves, circular);
        int grid = std::max(1, d->num_cus * std::max(1, per_cu));
        if ((int64_t)grid > items) grid = (int)items;
        if (e == hipSuccess) e = hipStreamBeginCapture(d->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e1 = launch_stage_batched(static_cast<const StageArgs*>(b.stage.p), (int)stages.size(), rows,
                                                 d->capture_stream);
            hipError_t e2 = launch_fold(static_cast<const double*>(b.coef64.p),
                                        static_cast<const float* const*>(b.scale_ptrs.p),
                                        static_cast<double*>(b.coef_dev.p), total_proj, d->capture_stream);
            // window tables of the scans that sample from LDS (needs the folded coefficients)
            hipError_t ew = hipSuccess;
            for (int j = 0; j < n_scans && ew == hipSuccess; ++j)
                if (win_off[j] >= 0)
                    ew = launch_window(tiles[j], t.strip, t.waves, static_cast<Win*>(b.windows.p) + win_off[j],
                                       batch_anchors(b, win_total) + win_off[j], d->capture_stream);
            if (e2 == hipSuccess) e2 = ew;
            hipError_t e3 = launch_reset_counter(static_cast<unsigned*>(b.counter.p), d->capture_stream);
            hipError_t e4 = launch_bp_batched(static_cast<const TileArgs*>(b.tiles.p),
                                              static_cast<const int32_t*>(b.item_begin.p), n_scans,
                                              static_cast<unsigned*>(b.counter.p), (int)items, grid,
                                              t.strip, t.waves, circular, d->capture_stream);
            hipError_t ec = hipStreamEndCapture(d->capture_stream, &graph);
            e = e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3 != hipSuccess ? e3 : e4 != hipSuccess ? e4 : ec;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
        if (graph != nullptr) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            release_entry(b);
            return fail(FDK_E_DEVICE, "batched graph build failed: %s", hipGetErrorString(e));
        }
        d->batch_cache.push_front(std::move(b));
        hit = &d->batch_cache.front();
    }
    {
        ProfScope ps("batched", s);
        HIP_TRY(hipGraphLaunch(hit->exec, s));
    }
    return end_call(*d, s);
}

fdk_status fdk_set_tile(int32_t dtype, int32_t strip, int32_t waves, int32_t layout)
{
    g_last_error.clear();
    if (dtype < 0 || dtype >= kSlots) return fail(FDK_E_UNSUPPORTED, "unknown tuning slot %d", dtype);
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    if (strip == 0 && waves == 0) {
        g_tune.forced[dtype] = {0, 0, 0};
        return FDK_OK;
    }
    const TileShape t{strip, waves, layout};
    if (!valid_shape(dtype, t))
        return fail(FDK_E_INVALID_ARG, "tile %dx%d layout %d not compiled for slot %d", strip, waves, layout, dtype);
    g_tune.forced[dtype] = t;
    return FDK_OK;
}

fdk_status fdk_get_tile(const fdk_volume* vol, int32_t dtype, int32_t* strip, int32_t* waves,
                        int32_t* layout)
{
    g_last_error.clear();
    fdk_status st = check_volume(vol);
    if (st != FDK_OK) return st;
    if (dtype < 0 || dtype >= kSlots) return fail(FDK_E_UNSUPPORTED, "unknown tuning slot %d", dtype);
    if (strip == nullptr || waves == nullptr || layout == nullptr) return fail(FDK_E_INVALID_ARG, "NULL output");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    load_env_tuning();
    const TileShape t = pick_tile(vol->L, dtype);
    *strip = t.strip;
    *waves = t.waves;
    *layout = t.layout;
    return FDK_OK;
}

fdk_status fdk_set_tuning_entry(int32_t dtype, int32_t size_class, int32_t strip, int32_t waves,
                                int32_t layout)
{
    g_last_error.clear();
    if (dtype < 0 || dtype >= kSlots) return fail(FDK_E_UNSUPPORTED, "unknown tuning slot %d", dtype);
    if (size_class < 0 || size_class > 15) return fail(FDK_E_INVALID_ARG, "size class %d", size_class);
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    if (strip == 0 && waves == 0) {
        g_tune.table.erase({dtype, size_class});
        return FDK_OK;
    }
    const TileShape t{strip, waves, layout};
    if (!valid_shape(dtype, t))
        return fail(FDK_E_INVALID_ARG, "tile %dx%d layout %d not compiled for slot %d", strip, waves, layout, dtype);
    g_tune.table[{dtype, size_class}] = t;
    return FDK_OK;
}

int32_t fdk_load_tuning(const char* path)
{
    g_last_error.clear();
    if (path == nullptr) return fail(FDK_E_INVALID_ARG, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return fail(FDK_E_INVALID_ARG, "cannot open %s", path);
    char line[256];
    int n = 0;
    bool header = false;
    std::vector<std::pair<std::pair<int, int>, TileShape>> entries;
    while (std::fgets(line, sizeof(line), f)) {
        char* hash = std::strchr(line, '#');
        if (hash) *hash = 0;
        char tag[64], arch[64];
        int ver = 0;
        if (!header) {
            if (std::sscanf(line, "%63s %d %63s", tag, &ver, arch) == 3) {
                if (std::strcmp(tag, "fdk-tuning") != 0 || ver != FDK_ABI_VERSION || std::strcmp(arch, "gfx950") != 0) {
                    std::fclose(f);
                    return fail(FDK_E_INVALID_ARG, "%s: tuning file is for another version or arch", path);
                }
                header = true;
            }
            continue;
        }
        int dt, cls, s, w, lay;
        if (std::sscanf(line, "%d %d %d %d %d", &dt, &cls, &s, &w, &lay) == 5) {
            if (dt < 0 || dt >= kSlots || cls < 0 || cls > 15 || !valid_shape(dt, TileShape{s, w, lay})) {
                std::fclose(f);
                return fail(FDK_E_INVALID_ARG, "%s: bad entry '%d %d %d %d %d'", path, dt, cls, s, w, lay);
            }
            entries.push_back({{dt, cls}, {s, w, lay}});
            ++n;
        }
    }
    std::fclose(f);
    if (!header) return fail(FDK_E_INVALID_ARG, "%s: missing 'fdk-tuning' header", path);
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    for (auto& e : entries) g_tune.table[e.first] = e.second;
    return n;
}

fdk_status fdk_release_workspace(void)
{
    g_last_error.clear();
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) return FDK_OK;
    DeviceState& d = it->second;
    HIP_TRY(hipDeviceSynchronize());
    release(d.staged);
    release(d.coef_dev);
    release(d.adjoint);
    release(d.windows);
    for (CoefEntry& c : d.coef_cache) release_coef(c);
    d.coef_cache.clear();
    for (BatchEntry& b : d.batch_cache) {
        release_entry(b);
    }
    d.batch_cache.clear();
    release(d.batch_staged);
    for (FilterEntry& f : d.filter_cache) {
        release(f.hs); release(f.tw); release(f.wc); release(f.wp);
    }
    d.filter_cache.clear();
    release(d.filter_ws);
    release(d.filter_max);
    for (DevBuf* b : {&d.it_p0, &d.it_p1, &d.it_v0, &d.it_v1, &d.it_part, &d.it_st}) release(*b);
    for (int b = 0; b < 2; ++b) {
        release(d.band[b]);
        release(d.slab[b]);
        d.band_used[b] = d.slab_used[b] = false;
    }
    release(d.band_j0);
    release_host(d.band_j0_host);
    d.j0_pending = false;
    d.have_last = false;
    return FDK_OK;
}

fdk_status fdk_profile_enable(int enable)
{
    g_last_error.clear();
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    for (ProfRecord& r : g_prof.records) {
        (void)hipEventSynchronize(r.end);
        g_prof.pool.push_back(r.start);
        g_prof.pool.push_back(r.end);
    }
    g_prof.records.clear();
    g_prof.on = enable != 0;
    return FDK_OK;
}

fdk_status fdk_profile_read(const char* kernel, int64_t* launches, double* total_ms)
{
    g_last_error.clear();
    if (kernel == nullptr || launches == nullptr || total_ms == nullptr)
        return fail(FDK_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::recursive_mutex> lock(g_mu);
    int64_t n = 0;
    double ms = 0.0;
    for (ProfRecord& r : g_prof.records) {
        if (std::strcmp(r.kind, kernel) != 0) continue;
        HIP_TRY(hipEventSynchronize(r.end));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, r.start, r.end));
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return FDK_OK;
}

}  // extern "C"
