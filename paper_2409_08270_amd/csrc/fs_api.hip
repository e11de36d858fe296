// C ABI of the library (include/flashsplat.h): context, argument validation,
// workspace, the four calls of the splat-and-accumulate path and the batched
// multi-scene solve captured into a hipGraph.
//
// All calls share one planning step: the views of the call (of one scene for
// the single-scene calls, of many for a batch) are laid out in small device
// tables (ViewDev, SceneDev, projection tasks, sort segments) that the kernels
// index; see fs_internal.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fs_internal.h"

using namespace fs;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

constexpr int kStaging = 8;
constexpr int kQueueWord = 8;  // word of the context's npairs_dev block used as the persistent launch's counter

}  // namespace

struct fs_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    unsigned long long *status_dev = nullptr;
    unsigned long long *status_host = nullptr;  // pinned, kStatusWords
    uint32_t *npairs_dev = nullptr;
    uint32_t *npairs_host = nullptr;            // pinned
    // per-call tables
    DevBuf views, scenes, tasks, dsegs, psegs, lsegs;
    // per-call workspace (grow-only)
    DevBuf dkeys, dvals, dkeys2, dvals2, counts, offsets;
    DevBuf pk_alt, pv_alt, sort_ws, scan_ws;
    DevBuf items, items_k, items_k2, items_v2, items_ws;
    DevBuf fix;                // FS_RED_DET: the call's fixed-point totals
    DevBuf memb;               // fs_render_masks: object membership bytes
    uint64_t items_tiles = 0;  // tile count the XCD-run table in `items` was built for
    Staging stage[kStaging];
    int stage_next = 0;
    hipEvent_t acc_ev[2] = {nullptr, nullptr};  // around the last compositing launch
    bool acc_timed = false;
    // fs_accumulate_noalloc: this device's copy of the static scratch array, and
    // pinned host room for the call's tables (reused once its last copy is done)
    unsigned char *scratch = nullptr;
    void *na_host = nullptr;
    hipEvent_t na_ev = nullptr;
    bool na_pending = false;
    char last_error[512] = {0};  // fixed size: reporting an error allocates nothing
};

namespace {

int set_err(fs_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->last_error, sizeof(ctx->last_error), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHECK(ctx, expr)                                                                      \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess)                                                                    \
            return set_err((ctx), FS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));    \
    } while (0)

#define RCHECK(expr)            \
    do {                        \
        int _rc = (expr);       \
        if (_rc) return _rc;    \
    } while (0)

int alloc_buf(fs_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (b.p) {
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));  // the stream may still use the old buffer
        HIPCHECK(ctx, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return set_err(ctx, FS_ERR_ALLOC, "device allocation of %zu bytes failed", bytes);
    }
    b.cap = bytes;
    return FS_OK;
}

int ensure(fs_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap && b.p) return FS_OK;
    return alloc_buf(ctx, b, bytes + bytes / 4 + 4096);
}

void free_buf(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Copies host bytes to a device buffer asynchronously through a ring of
// pinned staging buffers (a slot is reused only after its copy completed).
int upload(fs_ctx *ctx, DevBuf &dst, const void *src, size_t bytes)
{
    RCHECK(ensure(ctx, dst, bytes));
    if (bytes == 0) return FS_OK;
    Staging &st = ctx->stage[ctx->stage_next];
    ctx->stage_next = (ctx->stage_next + 1) % kStaging;
    if (st.pending) {
        HIPCHECK(ctx, hipEventSynchronize(st.ev));
        st.pending = false;
    }
    if (bytes > st.cap) {
        if (st.host) HIPCHECK(ctx, hipHostFree(st.host));
        st.host = nullptr;
        st.cap = 0;
        size_t want = bytes + 4096;
        if (hipHostMalloc(&st.host, want, hipHostMallocDefault) != hipSuccess)
            return set_err(ctx, FS_ERR_ALLOC, "pinned allocation of %zu bytes failed", want);
        st.cap = want;
    }
    memcpy(st.host, src, bytes);
    HIPCHECK(ctx, hipMemcpyAsync(dst.p, st.host, bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipEventRecord(st.ev, ctx->stream));
    st.pending = true;
    return FS_OK;
}

template <class T>
int upload_vec(fs_ctx *ctx, DevBuf &dst, const std::vector<T> &v)
{
    return upload(ctx, dst, v.data(), v.size() * sizeof(T));
}

bool finite_f(float x) { return isfinite(x); }

int check_params(fs_ctx *ctx, const fs_params *p, bool for_accum)
{
    if (!p) return set_err(ctx, FS_ERR_ARG, "params is NULL");
    if (p->tile_w <= 0 || p->tile_h <= 0 || p->tile_w > 4096 || p->tile_h > 4096)
        return set_err(ctx, FS_ERR_ARG, "tile size %dx%d out of range", p->tile_w, p->tile_h);
    if (for_accum && !(p->tile_w * p->tile_h == 256 && (p->tile_w == 8 || p->tile_w == 16 || p->tile_w == 32)))
        return set_err(ctx, FS_ERR_ARG, "fs_accumulate needs a 256-pixel tile of width 8, 16 or 32 (got %dx%d)",
                       p->tile_w, p->tile_h);
    if (!finite_f(p->sigma_k) || p->sigma_k <= 0.f) return set_err(ctx, FS_ERR_ARG, "sigma_k must be > 0");
    if (!finite_f(p->lowpass) || p->lowpass < 0.f) return set_err(ctx, FS_ERR_ARG, "lowpass must be >= 0");
    if (!finite_f(p->znear)) return set_err(ctx, FS_ERR_ARG, "znear must be finite");
    if (!finite_f(p->guard) || p->guard <= 0.f) return set_err(ctx, FS_ERR_ARG, "guard must be > 0");
    if (!finite_f(p->alpha_min) || !finite_f(p->alpha_max) || p->alpha_min < 0.f || p->alpha_max > 1.f ||
        p->alpha_min > p->alpha_max)
        return set_err(ctx, FS_ERR_ARG, "need 0 <= alpha_min <= alpha_max <= 1");
    if (!finite_f(p->t_min) || p->t_min < 0.f || p->t_min >= 1.f) return set_err(ctx, FS_ERR_ARG, "need 0 <= t_min < 1");
    if (!finite_f(p->fp64_cond) || p->fp64_cond < 1.f) return set_err(ctx, FS_ERR_ARG, "fp64_cond must be >= 1");
    if (p->tile_order < 0 || p->tile_order > 2) return set_err(ctx, FS_ERR_ARG, "tile_order must be 0, 1 or 2");
    if (p->count_ops != 0 && p->count_ops != 1) return set_err(ctx, FS_ERR_ARG, "count_ops must be 0 or 1");
    if (p->persistent != 0 && p->persistent != 1) return set_err(ctx, FS_ERR_ARG, "persistent must be 0 or 1");
    if (!(p->lds_batch == 0 || p->lds_batch == 32 || p->lds_batch == 64 || p->lds_batch == 128 || p->lds_batch == 256))
        return set_err(ctx, FS_ERR_ARG, "lds_batch must be 0, 32, 64, 128 or 256");
    return FS_OK;
}

int check_cams(fs_ctx *ctx, const fs_camera *cams, int32_t n_views)
{
    if (n_views < 0) return set_err(ctx, FS_ERR_ARG, "n_views < 0");
    if (n_views > 0 && !cams) return set_err(ctx, FS_ERR_ARG, "cams is NULL");
    for (int v = 0; v < n_views; ++v) {
        const fs_camera &c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 65535 || c.height > 65535)
            return set_err(ctx, FS_ERR_ARG, "view %d: size %dx%d out of range", v, c.width, c.height);
        for (int i = 0; i < 9; ++i)
            if (!finite_f(c.R[i])) return set_err(ctx, FS_ERR_ARG, "view %d: non-finite rotation", v);
        for (int i = 0; i < 3; ++i)
            if (!finite_f(c.t[i])) return set_err(ctx, FS_ERR_ARG, "view %d: non-finite translation", v);
        if (!finite_f(c.fx) || !finite_f(c.fy) || !(c.fx > 0.f) || !(c.fy > 0.f) || !finite_f(c.cx) || !finite_f(c.cy))
            return set_err(ctx, FS_ERR_ARG, "view %d: bad intrinsics", v);
    }
    return FS_OK;
}

int check_gauss(fs_ctx *ctx, const fs_gaussians *g)
{
    if (!g) return set_err(ctx, FS_ERR_ARG, "Gaussians are NULL");
    if (g->n < 0 || g->n >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "Gaussian count %lld out of range", (long long)g->n);
    if (g->n > 0 && (!g->mx || !g->my || !g->mz || !g->qw || !g->qx || !g->qy || !g->qz || !g->sx || !g->sy ||
                     !g->sz || !g->opacity))
        return set_err(ctx, FS_ERR_ARG, "Gaussian array is NULL");
    return FS_OK;
}

int check_proj(fs_ctx *ctx, const fs_proj *pr)
{
    if (!pr) return set_err(ctx, FS_ERR_ARG, "proj is NULL");
    if (pr->n < 0 || pr->n_views < 0) return set_err(ctx, FS_ERR_ARG, "proj sizes negative");
    if (pr->n >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "too many Gaussians (%lld)", (long long)pr->n);
    if ((int64_t)pr->n * pr->n_views >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "n * n_views too large for one call");
    if (pr->n > 0 && pr->n_views > 0 && (!pr->rec || !pr->rect || !pr->ntiles || !pr->flags))
        return set_err(ctx, FS_ERR_ARG, "proj has NULL planes");
    return FS_OK;
}

int bits_for(uint64_t count)
{
    int b = 1;
    while (b < 32 && (1ull << b) < count) ++b;
    return b;
}

ProjParams proj_params(const fs_params *p)
{
    ProjParams q;
    q.tile_w = p->tile_w;
    q.tile_h = p->tile_h;
    q.sigma_k = p->sigma_k;
    q.lowpass = p->lowpass;
    q.znear = p->znear;
    q.guard = p->guard;
    q.fp64_cond = p->fp64_cond;
    q.fp64_conic = p->fp64_conic;
    q.cshift = 0;
    return q;
}

AccParams acc_params(const fs_params *p, int32_t reduction)
{
    AccParams ap;
    const double LOG2E = 1.4426950408889634;
    ap.cut2 = (float)(-0.5 * (double)p->sigma_k * (double)p->sigma_k * LOG2E);
    ap.alpha_min = p->alpha_min;
    ap.alpha_max = p->alpha_max;
    ap.t_min = p->t_min;
    ap.lmin = p->alpha_min > 0.0f ? (float)std::log2((double)p->alpha_min) : -INFINITY;
    ap.tile_w = p->tile_w;
    ap.tile_h = p->tile_h;
    ap.reduction = reduction;
    ap.count = p->count_ops ? 1 : 0;
    ap.batch = p->lds_batch ? p->lds_batch : 256;
    ap.persistent = p->persistent;
    return ap;
}

GaussPtrs gauss_ptrs(const fs_gaussians *g)
{
    GaussPtrs gp{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (g) gp = GaussPtrs{g->mx, g->my, g->mz, g->qw, g->qx, g->qy, g->qz, g->sx, g->sy, g->sz, g->opacity};
    return gp;
}

// ---- planning -------------------------------------------------------------
// Host tables for a run of views (one call, or one chunk of a batch).
struct Plan {
    std::vector<ViewDev> views;
    std::vector<ProjTask> tasks;
    std::vector<SegDev> dsegs;     // depth sort: one segment per view
    uint32_t proj_blocks = 0;
    uint32_t dblocks = 0;
    uint64_t elems = 0;
    uint64_t tiles = 0;
    uint64_t pixels = 0;
};

// Device description of one view: camera, tile grid, and where its tiles,
// mask, projection plane and pixel state start.
ViewDev make_view(const fs_camera &c, const fs_params *p, uint32_t scene, int64_t n, uint64_t tile_base,
                  uint64_t mask_off, uint64_t elem_off, uint64_t pix_off)
{
    ViewDev d;
    memcpy(d.R, c.R, sizeof(d.R));
    memcpy(d.t, c.t, sizeof(d.t));
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.W = c.width; d.H = c.height;
    d.tiles_x = (c.width + p->tile_w - 1) / p->tile_w;
    d.tiles_y = (c.height + p->tile_h - 1) / p->tile_h;
    d.tile_base = (uint32_t)tile_base;
    d.scene = scene;
    d.mask_off = mask_off;
    d.elem_off = elem_off;
    d.pix_off = pix_off;
    d.n = (uint32_t)n;
    d.pad = 0;
    {
        // binary32, in the projection's operation order (the same value for every element)
#pragma clang fp contract(off)
        d.limx = p->guard * ((0.5f * (float)c.width) / c.fx);
        d.limy = p->guard * ((0.5f * (float)c.height) / c.fy);
    }
    return d;
}

// Appends views [v0, v1) of a scene with n Gaussians; mask_off0 is the mask
// offset of view v0 within the scene's masks.
void plan_add(Plan &pl, const fs_params *p, uint32_t scene, int64_t n, const fs_camera *cams, int v0, int v1,
              uint64_t mask_off0)
{
    uint64_t moff = mask_off0;
    const int first = (int)pl.views.size();
    for (int v = v0; v < v1; ++v) {
        const fs_camera &c = cams[v];
        const ViewDev d = make_view(c, p, scene, n, pl.tiles, moff, pl.elems, pl.pixels);
        pl.views.push_back(d);
        SegDev sg;
        sg.off = pl.elems;
        sg.len = (uint32_t)n;
        sg.blk0 = pl.dblocks;
        sg.alen = (uint32_t)n;
        sg.kbase = 0;
        pl.dsegs.push_back(sg);
        pl.dblocks += (uint32_t)((n + kSortTile - 1) / kSortTile);
        pl.elems += (uint64_t)n;
        pl.tiles += (uint64_t)d.tiles_x * d.tiles_y;
        pl.pixels += (uint64_t)c.width * c.height;
        moff += (uint64_t)c.width * c.height;
    }
    const uint32_t bpv = (uint32_t)((n + 255) / 256);
    for (int v = first; v < (int)pl.views.size(); v += kProjViews) {
        ProjTask t;
        t.blk0 = pl.proj_blocks;
        t.scene = scene;
        t.v0 = (uint32_t)v;
        t.nv = (uint32_t)std::min<int>(kProjViews, (int)pl.views.size() - v);
        pl.tasks.push_back(t);
        pl.proj_blocks += bpv;
    }
}

SceneDev scene_dev(const fs_gaussians *g, int64_t n, const uint8_t *masks, float *A_hi, float *A_lo, int32_t E)
{
    SceneDev s;
    s.g = gauss_ptrs(g);
    s.masks = masks;
    s.A_hi = A_hi;
    s.A_lo = A_lo;
    s.A_fix = nullptr;
    s.n = (uint32_t)n;
    s.E = E;
    return s;
}

// XCD-run work order (tile_order 2). Workgroups are handed to the chip's 8
// XCDs round-robin by index and every XCD has its own L2: the table maps
// workgroup b to tile (b % 8) * run + b / 8, so XCD x composites one
// contiguous run of tiles.
constexpr int kXcds = 8;

int build_xcd_items(fs_ctx *ctx, uint64_t n_tiles)
{
    if (ctx->items_tiles == n_tiles && ctx->items.p) return FS_OK;
    std::vector<uint32_t> it((size_t)n_tiles);
    const uint64_t base = n_tiles / kXcds, rem = n_tiles % kXcds;
    uint64_t start[kXcds];
    uint64_t acc = 0;
    for (int x = 0; x < kXcds; ++x) {
        start[x] = acc;
        acc += base + ((uint64_t)x < rem ? 1 : 0);
    }
    for (uint64_t b = 0; b < n_tiles; ++b) it[b] = (uint32_t)(start[b % kXcds] + b / kXcds);
    ctx->items_tiles = 0;
    RCHECK(upload(ctx, ctx->items, it.data(), it.size() * sizeof(uint32_t)));
    ctx->items_tiles = n_tiles;
    return FS_OK;
}

// Longest-list-first work order (tile_order 0) of `n_tiles` tiles into
// `items`, from their ranges; `lseg` is one segment covering all tiles.
int enqueue_lpt(fs_ctx *ctx, hipStream_t s, const uint32_t *ranges, uint64_t n_tiles, const SegDev *lseg,
                uint32_t *items, uint32_t *k, uint32_t *k2, uint32_t *v2, void *ws)
{
    HIPCHECK(ctx, launch_tile_keys(s, ranges, (int64_t)n_tiles, k, items));
    const uint32_t blocks = (uint32_t)((n_tiles + kSortTile - 1) / kSortTile);
    HIPCHECK(ctx, radix_sort(s, k, items, k2, v2, lseg, 1, blocks, 16, ws, nullptr, 1));
    return FS_OK;
}

// ---- static scratch of fs_accumulate_noalloc -------------------------------
// Layout: the call's tables (scene, work-order sort segment, views), copied
// from the host in one transfer (the persistent launch's work counter sits
// in the segment's block; the launch clears it after that copy), then four
// tile-index arrays for the longest-list-first order and the radix sort's
// workspace.
constexpr size_t kNaAlign = 256;
constexpr size_t na_round(size_t b) { return (b + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr size_t kNaSceneOff = 0;
constexpr size_t kNaSegOff = kNaSceneOff + na_round(sizeof(SceneDev));
constexpr size_t kNaQueueOff = kNaSegOff + kNaAlign / 2;  // the persistent launch's work counter (device-written)
constexpr size_t kNaViewsOff = kNaSegOff + na_round(sizeof(SegDev));
constexpr size_t kNaTableBytes = kNaViewsOff + na_round((size_t)FS_NOALLOC_MAX_VIEWS * sizeof(ViewDev));
constexpr size_t kNaItemBytes = na_round((size_t)FS_NOALLOC_MAX_TILES * 4);
constexpr size_t kNaItemsOff = kNaTableBytes;
constexpr size_t kNaWsOff = kNaItemsOff + 4 * kNaItemBytes;
constexpr size_t kNaWsBytes = (size_t)1 << 20;
constexpr size_t kNaBytes = kNaWsOff + kNaWsBytes;
constexpr int kNaMaxDevices = 64;

}  // namespace

// One copy per GPU, held until the process ends. Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

std::mutex g_na_mu;
unsigned char *g_na_ptr[kNaMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (the caller has made `device` current).
int scratch_address(fs_ctx *ctx, int device, unsigned char **out)
{
    if (device < 0 || device >= kNaMaxDevices) return set_err(ctx, FS_ERR_ARG, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_err(ctx, FS_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_na_ptr[device] = (unsigned char *)ptr;
    }
    *out = g_na_ptr[device];
    return FS_OK;
}

__global__ void k_xcd_items(uint32_t *items, uint32_t n_tiles)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_tiles) return;
    const uint32_t base = n_tiles / kXcds, rem = n_tiles % kXcds, x = b % kXcds;
    items[b] = x * base + min(x, rem) + b / kXcds;
}

// FS_RED_DET: pixels per call (per scene in a batch); see to_fix's range
constexpr uint64_t kFixMaxPixels = (uint64_t)1 << 29;

// Arguments of fs_accumulate and fs_accumulate_noalloc; resolves FS_RED_AUTO.
int check_accumulate(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                     const uint8_t *masks, int32_t n_classes, const fs_params *p, const float *A_hi,
                     const float *A_lo, int32_t *reduction)
{
    RCHECK(check_params(ctx, p, true));
    RCHECK(check_proj(ctx, proj));
    if (!bins || !bins->ranges) return set_err(ctx, FS_ERR_ARG, "bins is NULL");
    RCHECK(check_cams(ctx, cams, proj->n_views));
    if (n_classes < 2 || n_classes > 256) return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, 256]", n_classes);
    int32_t r = *reduction;
    if (r < FS_RED_AUTO || r > FS_RED_DET) return set_err(ctx, FS_ERR_ARG, "unknown reduction %d", r);
    if (r == FS_RED_AUTO) r = A_lo ? FS_RED_LDS2SUM : FS_RED_LDS;
    if (r == FS_RED_LDS2SUM && !A_lo) return set_err(ctx, FS_ERR_ARG, "FS_RED_LDS2SUM needs A_lo");
    if (proj->n > 0 && proj->n_views > 0 && (!masks || !A_hi)) return set_err(ctx, FS_ERR_ARG, "masks or A_hi is NULL");
    if (r == FS_RED_DET) {
        // every pixel adds at most 1 in total, so the fixed-point totals stay below 2^29 * 2^34
        uint64_t px = 0;
        for (int v = 0; v < proj->n_views; ++v) px += (uint64_t)cams[v].width * (uint64_t)cams[v].height;
        if (px > kFixMaxPixels)
            return set_err(ctx, FS_ERR_ARG, "FS_RED_DET: %llu pixels in one call, at most %llu",
                           (unsigned long long)px, (unsigned long long)kFixMaxPixels);
    }
    *reduction = r;
    return FS_OK;
}

}  // namespace

extern "C" {

const char *fs_version(void) { return "flashsplat-gfx950 0.2"; }

const char *fs_error_string(int code)
{
    switch (code) {
    case FS_OK: return "ok";
    case FS_ERR_ARG: return "invalid argument";
    case FS_ERR_ALLOC: return "allocation failed";
    case FS_ERR_HIP: return "HIP runtime error";
    case FS_ERR_CAPACITY: return "output capacity too small";
    case FS_ERR_DEVICE: return "error latched on the device";
    case FS_ERR_STATE: return "invalid state";
    default: return "unknown error";
    }
}

void fs_params_default(fs_params *p)
{
    if (!p) return;
    p->tile_w = 16;
    p->tile_h = 16;
    p->sigma_k = 3.0f;
    p->lowpass = 0.3f;
    p->znear = 0.2f;
    p->guard = 1.3f;
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->t_min = 1e-4f;
    p->fp64_cond = 64.0f;
    p->fp64_conic = 1;
    p->tile_order = 0;
    p->count_ops = 1;
    p->persistent = 0;
    p->lds_batch = 0;
}

void fs_params_exact(fs_params *p)
{
    if (!p) return;
    fs_params_default(p);
    p->alpha_min = 0.0f;
    p->alpha_max = 1.0f;
    p->t_min = 0.0f;
}

int fs_ctx_create(fs_ctx **out, void *stream)
{
    if (!out) return FS_ERR_ARG;
    *out = nullptr;
    fs_ctx *ctx = new (std::nothrow) fs_ctx();
    if (!ctx) return FS_ERR_ALLOC;
    ctx->stream = (hipStream_t)stream;
    int rc = FS_OK;
    if (hipGetDevice(&ctx->device) != hipSuccess) rc = FS_ERR_HIP;
    if (!rc && hipMalloc((void **)&ctx->status_dev, kStatusWords * sizeof(unsigned long long)) != hipSuccess) rc = FS_ERR_ALLOC;
    if (!rc && hipMalloc((void **)&ctx->npairs_dev, 64) != hipSuccess) rc = FS_ERR_ALLOC;
    if (!rc && hipHostMalloc((void **)&ctx->status_host, kStatusWords * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        rc = FS_ERR_ALLOC;
    if (!rc && hipHostMalloc((void **)&ctx->npairs_host, 64, hipHostMallocDefault) != hipSuccess) rc = FS_ERR_ALLOC;
    for (int i = 0; !rc && i < kStaging; ++i)
        if (hipEventCreateWithFlags(&ctx->stage[i].ev, hipEventDisableTiming) != hipSuccess) rc = FS_ERR_HIP;
    for (int i = 0; !rc && i < 2; ++i)
        if (hipEventCreate(&ctx->acc_ev[i]) != hipSuccess) rc = FS_ERR_HIP;
    // fs_accumulate_noalloc's set-up: this device's scratch address, pinned table room
    if (!rc) rc = scratch_address(ctx, ctx->device, &ctx->scratch);
    if (!rc && hipHostMalloc(&ctx->na_host, kNaTableBytes, hipHostMallocDefault) != hipSuccess) rc = FS_ERR_ALLOC;
    if (!rc && hipEventCreateWithFlags(&ctx->na_ev, hipEventDisableTiming) != hipSuccess) rc = FS_ERR_HIP;
    if (!rc && launch_fill_u32(ctx->stream, (uint32_t *)ctx->status_dev, 0u, kStatusWords * 2) != hipSuccess) rc = FS_ERR_HIP;
    if (!rc && launch_fill_u32(ctx->stream, ctx->npairs_dev, 0u, 16) != hipSuccess) rc = FS_ERR_HIP;
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = FS_ERR_HIP;
    if (rc) {
        fs_ctx_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return FS_OK;
}

int fs_ctx_set_stream(fs_ctx *ctx, void *stream)
{
    if (!ctx) return FS_ERR_ARG;
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stream = (hipStream_t)stream;
    return FS_OK;
}

int fs_ctx_destroy(fs_ctx *ctx)
{
    if (!ctx) return FS_ERR_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    DevBuf *bufs[] = {&ctx->views, &ctx->scenes, &ctx->tasks, &ctx->dsegs, &ctx->psegs, &ctx->lsegs,
                      &ctx->dkeys, &ctx->dvals, &ctx->dkeys2, &ctx->dvals2, &ctx->counts, &ctx->offsets,
                      &ctx->pk_alt, &ctx->pv_alt, &ctx->sort_ws, &ctx->scan_ws, &ctx->items, &ctx->items_k,
                      &ctx->items_k2, &ctx->items_v2, &ctx->items_ws, &ctx->fix, &ctx->memb};
    for (DevBuf *b : bufs) free_buf(*b);
    for (int i = 0; i < kStaging; ++i) {
        if (ctx->stage[i].host) (void)hipHostFree(ctx->stage[i].host);
        if (ctx->stage[i].ev) (void)hipEventDestroy(ctx->stage[i].ev);
    }
    for (int i = 0; i < 2; ++i)
        if (ctx->acc_ev[i]) (void)hipEventDestroy(ctx->acc_ev[i]);
    if (ctx->na_ev) (void)hipEventDestroy(ctx->na_ev);
    if (ctx->na_host) (void)hipHostFree(ctx->na_host);
    if (ctx->status_dev) (void)hipFree(ctx->status_dev);
    if (ctx->npairs_dev) (void)hipFree(ctx->npairs_dev);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    if (ctx->npairs_host) (void)hipHostFree(ctx->npairs_host);
    delete ctx;
    return FS_OK;
}

const char *fs_ctx_last_error(fs_ctx *ctx) { return ctx ? ctx->last_error : ""; }

int fs_status_get(fs_ctx *ctx, fs_status *out, int32_t clear)
{
    if (!ctx || !out) return set_err(ctx, FS_ERR_ARG, "NULL argument");
    HIPCHECK(ctx, hipMemcpyAsync(ctx->status_host, ctx->status_dev, kStatusWords * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long h[ST_COUNT];
    for (int c = 0; c < ST_COUNT; ++c) {
        unsigned long long acc = 0;
        for (int l = 0; l < kStatusLanes; ++l) acc += ctx->status_host[c * kStatusLanes + l];
        h[c] = acc;
    }
    h[ST_FLAGS] = ctx->status_host[ST_FLAGS * kStatusLanes];
    out->flags = (uint32_t)h[ST_FLAGS];
    out->bad_labels = (int64_t)h[ST_BAD_LABELS];
    out->invalid_gauss = (int64_t)h[ST_INVALID];
    out->fp64_splats = (int64_t)h[ST_FP64];
    out->pairs_dropped = (int64_t)h[ST_DROPPED];
    out->blends = (int64_t)h[ST_BLENDS];
    out->evaluated = (int64_t)h[ST_EVALS];
    out->wave_steps = (int64_t)h[ST_WSTEPS];
    out->wave_steps_max = (int64_t)h[ST_WSTEPS_MAX];
    out->unseen = (int64_t)h[ST_UNSEEN];
    out->multi_member = (int64_t)h[ST_MULTI];
    out->low_margin = (int64_t)h[ST_LOWMARGIN];
    out->pairs_emitted = (int64_t)h[ST_PAIRS];
    out->entries_staged = (int64_t)h[ST_STAGED];
    if (clear) HIPCHECK(ctx, launch_fill_u32(ctx->stream, (uint32_t *)ctx->status_dev, 0u, kStatusWords * 2));
    const uint32_t errbits = FS_DEV_BAD_LABEL | FS_DEV_PAIR_OVERFLOW | FS_DEV_INVALID_GAUSS;
    if (out->flags & errbits) return set_err(ctx, FS_ERR_DEVICE, "device status flags 0x%x", out->flags);
    return FS_OK;
}

int fs_project(fs_ctx *ctx, const fs_gaussians *g, const fs_camera *cams, int32_t n_views, const fs_params *p,
               const fs_proj *out)
{
    if (!ctx) return FS_ERR_ARG;
    if (!out) return set_err(ctx, FS_ERR_ARG, "NULL argument");
    RCHECK(check_params(ctx, p, false));
    RCHECK(check_cams(ctx, cams, n_views));
    RCHECK(check_proj(ctx, out));
    RCHECK(check_gauss(ctx, g));
    if (out->n != g->n || out->n_views != n_views)
        return set_err(ctx, FS_ERR_ARG, "proj sized for n=%lld, views=%d; need n=%lld, views=%d", (long long)out->n,
                       out->n_views, (long long)g->n, n_views);
    if (g->n == 0 || n_views == 0) return FS_OK;
    Plan pl;
    plan_add(pl, p, 0, g->n, cams, 0, n_views, 0);
    std::vector<SceneDev> sc{scene_dev(g, g->n, nullptr, nullptr, nullptr, 2)};
    RCHECK(upload_vec(ctx, ctx->views, pl.views));
    RCHECK(upload_vec(ctx, ctx->scenes, sc));
    RCHECK(upload_vec(ctx, ctx->tasks, pl.tasks));
    HIPCHECK(ctx, launch_project(ctx->stream, (const ProjTask *)ctx->tasks.p, (int32_t)pl.tasks.size(), pl.proj_blocks,
                                 (const SceneDev *)ctx->scenes.p, (const ViewDev *)ctx->views.p, proj_params(p),
                                 out->rec, out->rect, out->ntiles, out->flags, nullptr, nullptr, nullptr,
                                 ctx->status_dev));
    return FS_OK;
}

int fs_bin_sort(fs_ctx *ctx, const fs_proj *proj, const fs_camera *cams, const fs_params *p, const fs_bins *out,
                int64_t *n_pairs)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_params(ctx, p, false));
    RCHECK(check_proj(ctx, proj));
    if (!out) return set_err(ctx, FS_ERR_ARG, "bins is NULL");
    RCHECK(check_cams(ctx, cams, proj->n_views));
    if (out->capacity < 0 || out->capacity >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "bad bins capacity");
    if (!out->ranges || (out->capacity > 0 && (!out->vals || !out->tiles)))
        return set_err(ctx, FS_ERR_ARG, "bins has NULL arrays");
    const int64_t n = proj->n;
    const int32_t V = proj->n_views;
    Plan pl;
    plan_add(pl, p, 0, n, cams, 0, V, 0);
    if (pl.tiles >= 0xFFFFFFFFull) return set_err(ctx, FS_ERR_ARG, "too many tiles in one call");
    hipStream_t s = ctx->stream;
    HIPCHECK(ctx, launch_fill_u32(s, out->ranges, 0u, (int64_t)pl.tiles * 2));
    const int64_t total = (int64_t)pl.elems;
    if (total == 0) {
        if (n_pairs) *n_pairs = 0;
        HIPCHECK(ctx, launch_fill_u32(s, ctx->npairs_dev, 0u, 1));
        return FS_OK;
    }
    RCHECK(upload_vec(ctx, ctx->views, pl.views));
    RCHECK(upload_vec(ctx, ctx->dsegs, pl.dsegs));
    const size_t tb = (size_t)total * 4;
    RCHECK(ensure(ctx, ctx->dkeys, tb));
    RCHECK(ensure(ctx, ctx->dvals, tb));
    RCHECK(ensure(ctx, ctx->dkeys2, tb));
    RCHECK(ensure(ctx, ctx->dvals2, tb));
    RCHECK(ensure(ctx, ctx->counts, tb));
    RCHECK(ensure(ctx, ctx->offsets, tb));
    RCHECK(ensure(ctx, ctx->sort_ws, radix_ws_bytes(pl.dblocks)));
    RCHECK(ensure(ctx, ctx->scan_ws, scan_ws_bytes(total)));
    uint32_t *dk = (uint32_t *)ctx->dkeys.p, *dv = (uint32_t *)ctx->dvals.p;
    const ViewDev *views = (const ViewDev *)ctx->views.p;
    // depth order of each view's emitting Gaussians (4 passes: result back in dk/dv)
    HIPCHECK(ctx, launch_depth_keys(s, proj->rec, proj->ntiles, proj->flags, views, V, total, dk, dv));
    HIPCHECK(ctx, radix_sort(s, dk, dv, (uint32_t *)ctx->dkeys2.p, (uint32_t *)ctx->dvals2.p,
                             (const SegDev *)ctx->dsegs.p, V, pl.dblocks, 32, ctx->sort_ws.p, nullptr, 1));
    HIPCHECK(ctx, launch_gather_counts(s, dk, dv, proj->ntiles, views, V, total, (uint32_t *)ctx->counts.p));
    HIPCHECK(ctx, scan_exclusive(s, (const uint32_t *)ctx->counts.p, (uint32_t *)ctx->offsets.p, total, ctx->npairs_dev,
                                 ctx->scan_ws.p));
    int64_t sort_len = out->capacity;
    if (n_pairs) {
        HIPCHECK(ctx, hipMemcpyAsync(ctx->npairs_host, ctx->npairs_dev, 4, hipMemcpyDeviceToHost, s));
        HIPCHECK(ctx, hipStreamSynchronize(s));
        const int64_t np = (int64_t)ctx->npairs_host[0];
        *n_pairs = np;
        if (np > out->capacity)
            return set_err(ctx, FS_ERR_CAPACITY, "%lld tile pairs exceed capacity %lld", (long long)np,
                           (long long)out->capacity);
        sort_len = np;
    }
    if (sort_len == 0) return FS_OK;
    // stable sort of the pairs by tile id; the emit target is chosen so that
    // the final pass lands in the caller's buffers
    const int passes = (bits_for(pl.tiles) + 7) / 8;
    RCHECK(ensure(ctx, ctx->pk_alt, (size_t)sort_len * 4));
    RCHECK(ensure(ctx, ctx->pv_alt, (size_t)sort_len * 4));
    const int32_t ptpb = radix_tiles_per_block((uint64_t)sort_len);
    const uint32_t pblocks = (uint32_t)((sort_len + (int64_t)kSortTile * ptpb - 1) / ((int64_t)kSortTile * ptpb));
    RCHECK(ensure(ctx, ctx->sort_ws, radix_ws_bytes(pblocks)));
    std::vector<SegDev> ps{SegDev{0, (uint32_t)sort_len, 0, (uint32_t)sort_len, 0}};
    RCHECK(upload_vec(ctx, ctx->psegs, ps));
    uint32_t *k0, *v0, *k1, *v1;
    if (passes % 2 == 0) {
        k0 = out->tiles; v0 = out->vals; k1 = (uint32_t *)ctx->pk_alt.p; v1 = (uint32_t *)ctx->pv_alt.p;
    } else {
        k0 = (uint32_t *)ctx->pk_alt.p; v0 = (uint32_t *)ctx->pv_alt.p; k1 = out->tiles; v1 = out->vals;
    }
    HIPCHECK(ctx, launch_emit(s, dk, dv, (const uint32_t *)ctx->offsets.p, (const uint32_t *)ctx->counts.p, proj->rec,
                              proj->rect, p->fp64_conic ? nullptr : proj->flags, views, V, total,
                              (uint32_t)out->capacity, p->tile_w, p->tile_h,
                              p->sigma_k, nullptr, k0, v0, ctx->status_dev));
    // without a host count, the device count caps the sort (entries past it are never read)
    HIPCHECK(ctx, radix_sort(s, k0, v0, k1, v1, (const SegDev *)ctx->psegs.p, 1, pblocks, passes * 8, ctx->sort_ws.p,
                             n_pairs ? nullptr : ctx->npairs_dev, ptpb));
    HIPCHECK(ctx, launch_ranges(s, out->tiles, ctx->npairs_dev, (uint32_t)out->capacity, sort_len, out->ranges));
    return FS_OK;
}

int fs_accumulate(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams, const uint8_t *masks,
                  int32_t n_classes, const fs_params *p, float *A_hi, float *A_lo, int32_t reduction,
                  const fs_pixel_out *pix)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_accumulate(ctx, proj, bins, cams, masks, n_classes, p, A_hi, A_lo, &reduction));
    const int32_t V = proj->n_views;
    if (proj->n == 0 || V == 0) return FS_OK;
    Plan pl;
    plan_add(pl, p, 0, proj->n, cams, 0, V, 0);
    std::vector<SceneDev> sc{scene_dev(nullptr, proj->n, masks, A_hi, A_lo, n_classes)};
    const int64_t n_fix = proj->n * (int64_t)n_classes;
    if (reduction == FS_RED_DET) {
        RCHECK(ensure(ctx, ctx->fix, (size_t)n_fix * 8));
        HIPCHECK(ctx, launch_fill_u32(ctx->stream, (uint32_t *)ctx->fix.p, 0u, 2 * n_fix));
        sc[0].A_fix = (unsigned long long *)ctx->fix.p;
    }
    RCHECK(upload_vec(ctx, ctx->views, pl.views));
    RCHECK(upload_vec(ctx, ctx->scenes, sc));
    const uint32_t *items = nullptr;
    if (p->tile_order == 0) {
        const size_t tb = (size_t)pl.tiles * 4;
        const uint32_t lblocks = (uint32_t)((pl.tiles + kSortTile - 1) / kSortTile);
        RCHECK(ensure(ctx, ctx->items, tb));
        RCHECK(ensure(ctx, ctx->items_k, tb));
        RCHECK(ensure(ctx, ctx->items_k2, tb));
        RCHECK(ensure(ctx, ctx->items_v2, tb));
        RCHECK(ensure(ctx, ctx->items_ws, radix_ws_bytes(lblocks)));
        std::vector<SegDev> ls{SegDev{0, (uint32_t)pl.tiles, 0, (uint32_t)pl.tiles, 0}};
        RCHECK(upload_vec(ctx, ctx->lsegs, ls));
        ctx->items_tiles = 0;  // the XCD-run table (tile_order 2) shares the buffer
        RCHECK(enqueue_lpt(ctx, ctx->stream, bins->ranges, pl.tiles, (const SegDev *)ctx->lsegs.p,
                           (uint32_t *)ctx->items.p, (uint32_t *)ctx->items_k.p, (uint32_t *)ctx->items_k2.p,
                           (uint32_t *)ctx->items_v2.p, ctx->items_ws.p));
        items = (const uint32_t *)ctx->items.p;
    } else if (p->tile_order == 2) {
        RCHECK(build_xcd_items(ctx, pl.tiles));
        items = (const uint32_t *)ctx->items.p;
    }
    // events around the compositing launch alone (not under stream capture)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHECK(ctx, hipStreamIsCapturing(ctx->stream, &cap));
    const bool timed = cap == hipStreamCaptureStatusNone;
    if (timed) HIPCHECK(ctx, hipEventRecord(ctx->acc_ev[0], ctx->stream));
    HIPCHECK(ctx, launch_accumulate(ctx->stream, proj->rec, bins->vals, bins->ranges, (const ViewDev *)ctx->views.p, V,
                                    (const SceneDev *)ctx->scenes.p, items, (uint32_t)pl.tiles, acc_params(p, reduction),
                                    pix ? pix->t_final : nullptr, pix ? pix->n_blend : nullptr, nullptr, nullptr, 1,
                                    ctx->status_dev, ctx->npairs_dev + kQueueWord));
    if (timed) HIPCHECK(ctx, hipEventRecord(ctx->acc_ev[1], ctx->stream));
    ctx->acc_timed = timed;
    if (reduction == FS_RED_DET)
        HIPCHECK(ctx, launch_fix_finish(ctx->stream, (const unsigned long long *)ctx->fix.p, A_hi, A_lo, n_fix));
    return FS_OK;
}

int fs_accumulate_noalloc(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                          const uint8_t *masks, int32_t n_classes, const fs_params *p, float *A_hi, float *A_lo,
                          int32_t reduction, const fs_pixel_out *pix)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_accumulate(ctx, proj, bins, cams, masks, n_classes, p, A_hi, A_lo, &reduction));
    if (reduction == FS_RED_DET)
        return set_err(ctx, FS_ERR_ARG, "FS_RED_DET needs an n x n_classes workspace; use fs_accumulate");
    const int32_t V = proj->n_views;
    if (proj->n == 0 || V == 0) return FS_OK;
    if (V > FS_NOALLOC_MAX_VIEWS)
        return set_err(ctx, FS_ERR_CAPACITY, "%d views in one call, the static scratch holds %d", V,
                       FS_NOALLOC_MAX_VIEWS);
    uint64_t n_tiles = 0;
    for (int v = 0; v < V; ++v)
        n_tiles += (uint64_t)((cams[v].width + p->tile_w - 1) / p->tile_w) *
                   (uint64_t)((cams[v].height + p->tile_h - 1) / p->tile_h);
    if (n_tiles > (uint64_t)FS_NOALLOC_MAX_TILES)
        return set_err(ctx, FS_ERR_CAPACITY, "%llu tiles in one call, the static scratch holds %d",
                       (unsigned long long)n_tiles, FS_NOALLOC_MAX_TILES);
    const uint32_t lblocks = (uint32_t)((n_tiles + kSortTile - 1) / kSortTile);
    if (radix_ws_bytes(lblocks) > kNaWsBytes)
        return set_err(ctx, FS_ERR_CAPACITY, "work-order sort needs %zu bytes of scratch, %zu reserved",
                       radix_ws_bytes(lblocks), kNaWsBytes);
    if (!ctx->scratch || !ctx->na_host) return set_err(ctx, FS_ERR_STATE, "context has no static scratch");
    // the call's tables, built in the pinned host room once its previous copy has completed
    if (ctx->na_pending) {
        HIPCHECK(ctx, hipEventSynchronize(ctx->na_ev));
        ctx->na_pending = false;
    }
    unsigned char *h = (unsigned char *)ctx->na_host;
    *(SceneDev *)(h + kNaSceneOff) = scene_dev(nullptr, proj->n, masks, A_hi, A_lo, n_classes);
    *(SegDev *)(h + kNaSegOff) = SegDev{0, (uint32_t)n_tiles, 0, (uint32_t)n_tiles, 0};
    ViewDev *hv = (ViewDev *)(h + kNaViewsOff);
    uint64_t tb = 0, mo = 0, eo = 0;
    for (int v = 0; v < V; ++v) {
        hv[v] = make_view(cams[v], p, 0, proj->n, tb, mo, eo, mo);
        tb += (uint64_t)hv[v].tiles_x * (uint64_t)hv[v].tiles_y;
        mo += (uint64_t)cams[v].width * (uint64_t)cams[v].height;
        eo += (uint64_t)proj->n;
    }
    unsigned char *d = ctx->scratch;
    hipStream_t s = ctx->stream;
    HIPCHECK(ctx, hipMemcpyAsync(d, h, kNaViewsOff + (size_t)V * sizeof(ViewDev), hipMemcpyHostToDevice, s));
    HIPCHECK(ctx, hipEventRecord(ctx->na_ev, s));
    ctx->na_pending = true;
    const ViewDev *views = (const ViewDev *)(d + kNaViewsOff);
    const SceneDev *scenes = (const SceneDev *)(d + kNaSceneOff);
    uint32_t *it[4];
    for (int i = 0; i < 4; ++i) it[i] = (uint32_t *)(d + kNaItemsOff + (size_t)i * kNaItemBytes);
    const uint32_t *items = nullptr;
    if (p->tile_order == 0) {
        RCHECK(enqueue_lpt(ctx, s, bins->ranges, n_tiles, (const SegDev *)(d + kNaSegOff), it[0], it[1], it[2], it[3],
                           d + kNaWsOff));
        items = it[0];
    } else if (p->tile_order == 2) {
        hipLaunchKernelGGL(k_xcd_items, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, s, it[0],
                           (uint32_t)n_tiles);
        HIPCHECK(ctx, hipGetLastError());
        items = it[0];
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHECK(ctx, hipStreamIsCapturing(s, &cap));
    const bool timed = cap == hipStreamCaptureStatusNone;
    if (timed) HIPCHECK(ctx, hipEventRecord(ctx->acc_ev[0], s));
    HIPCHECK(ctx, launch_accumulate(s, proj->rec, bins->vals, bins->ranges, views, V, scenes, items, (uint32_t)n_tiles,
                                    acc_params(p, reduction), pix ? pix->t_final : nullptr,
                                    pix ? pix->n_blend : nullptr, nullptr, nullptr, 1, ctx->status_dev,
                                    (uint32_t *)(d + kNaQueueOff)));
    if (timed) HIPCHECK(ctx, hipEventRecord(ctx->acc_ev[1], s));
    ctx->acc_timed = timed;
    return FS_OK;
}

int fs_last_accumulate_ms(fs_ctx *ctx, float *ms)
{
    if (!ctx || !ms) return FS_ERR_ARG;
    if (!ctx->acc_timed) return set_err(ctx, FS_ERR_ARG, "no timed compositing launch on this context");
    HIPCHECK(ctx, hipEventSynchronize(ctx->acc_ev[1]));
    HIPCHECK(ctx, hipEventElapsedTime(ms, ctx->acc_ev[0], ctx->acc_ev[1]));
    return FS_OK;
}

int fs_assign(fs_ctx *ctx, const float *A_hi, const float *A_lo, int64_t n, int32_t n_classes, float gamma, uint8_t *S,
              float *margin)
{
    if (!ctx) return FS_ERR_ARG;
    if (n < 0) return set_err(ctx, FS_ERR_ARG, "n < 0");
    if (n_classes < 2 || n_classes > 256) return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, 256]", n_classes);
    if (!finite_f(gamma) || gamma < -1.f || gamma > 1.f) return set_err(ctx, FS_ERR_ARG, "gamma must be finite in [-1, 1]");
    if (n > 0 && (!A_hi || !S)) return set_err(ctx, FS_ERR_ARG, "A_hi or S is NULL");
    HIPCHECK(ctx, launch_assign(ctx->stream, A_hi, A_lo, n, n_classes, gamma, S, margin, ctx->status_dev));
    return FS_OK;
}

int fs_render_masks(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                    const uint8_t *S, int32_t n_classes, const fs_params *p, float tau, int32_t mode,
                    uint8_t *labels, float *rho, float *depth)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_params(ctx, p, true));
    RCHECK(check_proj(ctx, proj));
    if (!bins || !bins->ranges) return set_err(ctx, FS_ERR_ARG, "bins is NULL");
    RCHECK(check_cams(ctx, cams, proj->n_views));
    if (n_classes < 2 || n_classes > 256) return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, 256]", n_classes);
    if (mode != FS_MASK_DEPTH && mode != FS_MASK_ARGMAX) return set_err(ctx, FS_ERR_ARG, "unknown mask mode %d", mode);
    if (!finite_f(tau)) return set_err(ctx, FS_ERR_ARG, "tau must be finite");
    const int32_t V = proj->n_views;
    if (proj->n == 0 || V == 0) return FS_OK;
    if (!S || !labels) return set_err(ctx, FS_ERR_ARG, "S or labels is NULL");
    Plan pl;
    plan_add(pl, p, 0, proj->n, cams, 0, V, 0);
    RCHECK(upload_vec(ctx, ctx->views, pl.views));
    RCHECK(ensure(ctx, ctx->memb, (size_t)render_member_bytes(proj->n, n_classes, mode)));
    HIPCHECK(ctx, launch_render(ctx->stream, proj->rec, bins->vals, bins->ranges, (const ViewDev *)ctx->views.p, V,
                                (uint32_t)pl.tiles, S, proj->n, n_classes, acc_params(p, FS_RED_LDS), tau, mode, labels,
                                rho, depth, (int64_t)pl.pixels, (uint8_t *)ctx->memb.p));
    return FS_OK;
}

int fs_diagnose(fs_ctx *ctx, const float *A_hi, const float *A_lo, const uint8_t *S, const int32_t *gt, int64_t n,
                int32_t n_classes, float rel_eps, uint64_t *contrib_hist, uint64_t *member_hist, uint64_t *overlap)
{
    if (!ctx) return FS_ERR_ARG;
    if (n < 0 || n >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "n out of range");
    if (n_classes < 2 || n_classes > kMaxDiagE)
        return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, %d]", n_classes, kMaxDiagE);
    if (!finite_f(rel_eps) || rel_eps < 0.f || rel_eps >= 1.f) return set_err(ctx, FS_ERR_ARG, "need 0 <= rel_eps < 1");
    const bool want_c = A_hi && contrib_hist, want_m = S && member_hist, want_o = S && gt && overlap;
    if (!want_c && !want_m && !want_o) return set_err(ctx, FS_ERR_ARG, "nothing to compute");
    const size_t E1 = (size_t)n_classes + 1, nw = 2 * E1 + 3 * (size_t)n_classes;
    RCHECK(ensure(ctx, ctx->items_k, nw * 8));
    unsigned long long *d = (unsigned long long *)ctx->items_k.p;
    HIPCHECK(ctx, launch_fill_u32(ctx->stream, (uint32_t *)d, 0u, (int64_t)nw * 2));
    HIPCHECK(ctx, launch_diag_rows(ctx->stream, want_c ? A_hi : nullptr, want_c ? A_lo : nullptr,
                                   (want_m || want_o) ? S : nullptr, want_o ? gt : nullptr, n, n_classes,
                                   (double)rel_eps, d, d + E1, d + 2 * E1));
    std::vector<uint64_t> h(nw);
    HIPCHECK(ctx, hipMemcpyAsync(h.data(), d, nw * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (want_c) memcpy(contrib_hist, h.data(), E1 * 8);
    if (want_m) memcpy(member_hist, h.data() + E1, E1 * 8);
    if (want_o) memcpy(overlap, h.data() + 2 * E1, 3 * (size_t)n_classes * 8);
    return FS_OK;
}

int fs_prompt_propagate(fs_ctx *ctx, const fs_gaussians *g, const fs_camera *cams, int32_t n_views,
                        int32_t ref_view, const float *prompts, int32_t n_prompts, int32_t k, const fs_params *p,
                        int64_t *chosen, int64_t *nearest, float *uv, uint8_t *visible)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_gauss(ctx, g));
    RCHECK(check_params(ctx, p, false));
    RCHECK(check_cams(ctx, cams, n_views));
    if (n_views < 1 || ref_view < 0 || ref_view >= n_views) return set_err(ctx, FS_ERR_ARG, "bad ref_view");
    if (k < 1 || k > prompt_max_k()) return set_err(ctx, FS_ERR_ARG, "k must be in [1, %d]", prompt_max_k());
    if (n_prompts < 0 || n_prompts > 65535) return set_err(ctx, FS_ERR_ARG, "n_prompts must be in [0, 65535]");
    if (n_prompts == 0) return FS_OK;
    if (!prompts || !chosen || !uv || !visible) return set_err(ctx, FS_ERR_ARG, "NULL prompt or output");
    for (int i = 0; i < n_prompts; ++i)
        if (!finite_f(prompts[3 * i]) || !finite_f(prompts[3 * i + 1]) || !finite_f(prompts[3 * i + 2]) ||
            !(prompts[3 * i + 2] > 0.f))
            return set_err(ctx, FS_ERR_ARG, "prompt %d: need a finite pixel and a finite depth > 0", i);
    const size_t P = (size_t)n_prompts, V = (size_t)n_views;
    if (g->n == 0) {
        for (size_t i = 0; i < P; ++i) chosen[i] = -1;
        for (size_t i = 0; nearest && i < P * k; ++i) nearest[i] = -1;
        memset(uv, 0, P * V * 2 * sizeof(float));
        memset(visible, 0, P * V);
        return FS_OK;
    }
    Plan pl;
    plan_add(pl, p, 0, g->n, cams, 0, n_views, 0);
    RCHECK(upload_vec(ctx, ctx->views, pl.views));
    int64_t blocks = (g->n + 255) / 256;
    if (blocks > 512) blocks = 512;
    // device layout: prompts | ids [P][1+k] | uv [P][V][2] | visible [P][V]
    const size_t in_bytes = P * 3 * sizeof(float);
    const size_t ids_off = (in_bytes + 255) & ~(size_t)255;
    const size_t uv_off = ids_off + P * (1 + k) * 8;
    const size_t vis_off = uv_off + P * V * 8;
    const size_t total = vis_off + P * V;
    RCHECK(ensure(ctx, ctx->items_k, P * (size_t)blocks * k * 8));
    RCHECK(ensure(ctx, ctx->items_k2, total));
    char *o = (char *)ctx->items_k2.p;
    HIPCHECK(ctx, hipMemcpyAsync(o, prompts, in_bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, launch_prompt(ctx->stream, gauss_ptrs(g), g->n, (const ViewDev *)ctx->views.p, n_views,
                                pl.views[ref_view], (const float *)o, n_prompts, k, p->znear,
                                (unsigned long long *)ctx->items_k.p, (int32_t)blocks, (long long *)(o + ids_off),
                                (float *)(o + uv_off), (uint8_t *)(o + vis_off)));
    std::vector<char> h(total - ids_off);
    HIPCHECK(ctx, hipMemcpyAsync(h.data(), o + ids_off, total - ids_off, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    const long long *hid = (const long long *)h.data();
    for (size_t i = 0; i < P; ++i) {
        chosen[i] = (int64_t)hid[i * (1 + k)];
        for (int j = 0; nearest && j < k; ++j) nearest[i * k + j] = (int64_t)hid[i * (1 + k) + 1 + j];
    }
    memcpy(uv, h.data() + (uv_off - ids_off), P * V * 8);
    memcpy(visible, h.data() + (vis_off - ids_off), P * V);
    return FS_OK;
}

int fs_assign_sweep(fs_ctx *ctx, const float *A_hi, const float *A_lo, int64_t n, int32_t n_classes,
                    const float *gammas, int32_t n_gamma, uint8_t *S, int64_t *counts)
{
    if (!ctx) return FS_ERR_ARG;
    if (n < 0) return set_err(ctx, FS_ERR_ARG, "n < 0");
    if (n_classes < 2 || n_classes > 256) return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, 256]", n_classes);
    if (!gammas || n_gamma < 1 || n_gamma > sweep_max_gammas(n_classes))
        return set_err(ctx, FS_ERR_ARG, "n_gamma must be in [1, %d]", sweep_max_gammas(n_classes));
    for (int k = 0; k < n_gamma; ++k)
        if (!finite_f(gammas[k]) || gammas[k] < -1.f || gammas[k] > 1.f)
            return set_err(ctx, FS_ERR_ARG, "gamma %d must be finite in [-1, 1]", k);
    if (n > 0 && !A_hi) return set_err(ctx, FS_ERR_ARG, "A_hi is NULL");
    if (!S && !counts) return set_err(ctx, FS_ERR_ARG, "nothing to compute: S and counts are NULL");
    const size_t ncnt = (size_t)n_gamma * n_classes;
    RCHECK(upload(ctx, ctx->items_ws, gammas, sizeof(float) * n_gamma));
    if (counts) {
        RCHECK(ensure(ctx, ctx->items_k, ncnt * 8));
        HIPCHECK(ctx, launch_fill_u32(ctx->stream, (uint32_t *)ctx->items_k.p, 0u, (int64_t)ncnt * 2));
    }
    HIPCHECK(ctx, launch_assign_sweep(ctx->stream, A_hi, A_lo, n, n_classes, (const float *)ctx->items_ws.p, n_gamma,
                                      S, counts ? (unsigned long long *)ctx->items_k.p : nullptr));
    if (counts) {
        HIPCHECK(ctx, hipMemcpyAsync(counts, ctx->items_k.p, ncnt * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return FS_OK;
}

int fs_compact(fs_ctx *ctx, const fs_gaussians *in, const uint8_t *select, int32_t keep_selected,
               const fs_gaussians *out, int64_t *index_map, int64_t *n_out)
{
    if (!ctx) return FS_ERR_ARG;
    RCHECK(check_gauss(ctx, in));
    if (!out || !n_out) return set_err(ctx, FS_ERR_ARG, "out or n_out is NULL");
    if (out->n < 0) return set_err(ctx, FS_ERR_ARG, "out->n < 0");
    if (in->n > 0 && !select) return set_err(ctx, FS_ERR_ARG, "select is NULL");
    const int64_t n = in->n;
    *n_out = 0;
    if (n == 0) return FS_OK;
    RCHECK(ensure(ctx, ctx->counts, (size_t)n * 4));
    RCHECK(ensure(ctx, ctx->offsets, (size_t)n * 4));
    RCHECK(ensure(ctx, ctx->scan_ws, scan_ws_bytes(n)));
    HIPCHECK(ctx, launch_select_flags(ctx->stream, select, n, keep_selected, (uint32_t *)ctx->counts.p));
    HIPCHECK(ctx, scan_exclusive(ctx->stream, (const uint32_t *)ctx->counts.p, (uint32_t *)ctx->offsets.p, n,
                                 ctx->npairs_dev, ctx->scan_ws.p));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->npairs_host, ctx->npairs_dev, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t kept = (int64_t)ctx->npairs_host[0];
    *n_out = kept;
    if (kept > out->n) return set_err(ctx, FS_ERR_CAPACITY, "%lld Gaussians kept, room for %lld", (long long)kept,
                                      (long long)out->n);
    if (kept == 0) return FS_OK;
    const float *src[11] = {in->mx, in->my, in->mz, in->qw, in->qx, in->qy, in->qz, in->sx, in->sy, in->sz,
                            in->opacity};
    // fs_gaussians holds read-only pointers; the output arrays are written here
    float *dst[11] = {const_cast<float *>(out->mx), const_cast<float *>(out->my), const_cast<float *>(out->mz),
                      const_cast<float *>(out->qw), const_cast<float *>(out->qx), const_cast<float *>(out->qy),
                      const_cast<float *>(out->qz), const_cast<float *>(out->sx), const_cast<float *>(out->sy),
                      const_cast<float *>(out->sz), const_cast<float *>(out->opacity)};
    for (int k = 0; k < 11; ++k)
        if (!dst[k]) return set_err(ctx, FS_ERR_ARG, "output Gaussian array %d is NULL", k);
    HIPCHECK(ctx, launch_compact(ctx->stream, src, dst, (const uint32_t *)ctx->counts.p,
                                 (const uint32_t *)ctx->offsets.p, n, index_map));
    return FS_OK;
}

}  // extern "C"

// ===========================================================================
// Batched solve
// ===========================================================================
namespace {

struct SceneIn {
    fs_gaussians g;
    std::vector<fs_camera> cams;
    std::vector<uint64_t> mask_off;  // per view, within the scene's masks
    const uint8_t *masks;
    int32_t E;
    float *A_hi, *A_lo;
    unsigned long long *fix = nullptr;  // FS_RED_DET: this scene's fixed-point totals
    uint8_t *S;
    float *margin;
    float gamma;
};

struct ViewRef {
    uint32_t scene;
    int32_t v;
};

struct Chunk {
    Plan plan;
    std::vector<ViewRef> refs;
    uint64_t pairs = 0;       // planned (exact at creation)
    uint64_t slab_max = 0;    // largest pair count of one depth slab (before culling finished tiles)
    uint32_t pair_cap = 0;    // slots used by this chunk
    uint32_t pblocks = 0;
    int32_t ptpb = 1;         // block tiles per block of the pair sort
    std::vector<uint64_t> vpairs;  // planned pairs of each view
    // packed pair sort: one u32 item (tile in view << gbits | Gaussian) per pair,
    // one sort segment per view; used when both fit in 32 bits (single pass)
    bool packed = false;
    int32_t gbits = 0, tbits = 0;
    int32_t cshift = 0;  // depth-sort values: Gaussian id | listed-tile count << cshift (0: id only)
    uint32_t lblocks = 0;
    int passes = 0;
    DevBuf views, tasks, dsegs, psegs, lsegs;
};

}  // namespace

// Workspace of one lane. Chunks go to the lanes in turn; each lane has its own
// stream, so one chunk's sort can run while another's compositing does.
struct Work {
    DevBuf rec, rect, ntiles, flags, codes, dkeys, dvals, dkeys2, dvals2, counts, offsets;
    DevBuf ptiles, pvals, pk_alt, pv_alt, ranges, items, items_k, items_k2, items_v2;
    DevBuf sort_ws, scan_ws, tscan_ws, view_offs, tstate, tile_done, queue;
    hipStream_t stream = nullptr;  // default priority, created with the batch (lanes > 1)
    hipEvent_t done = nullptr;
};

struct fs_batch {
    fs_ctx *ctx = nullptr;
    fs_params p;
    fs_batch_opts o;
    std::vector<SceneIn> scenes;
    std::vector<Chunk> chunks;
    DevBuf scenes_d;
    DevBuf fix;              // FS_RED_DET: every scene's fixed-point totals
    int64_t fix_words = 0;
    std::vector<Work> work;  // one per lane
    hipEvent_t fork = nullptr;
    DevBuf npairs;
    uint64_t max_elems = 0, max_tiles = 0, max_pairs = 0, max_pixels = 0;
    int n_slabs = 1;
    uint32_t slab_num[9] = {0, 1024};  // depth-slab boundaries, numerators over 1024
    uint32_t max_dblocks = 0, max_pblocks = 0, max_lblocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // without a graph: events right around every compositing launch, [chunk][slab][2]
    std::vector<hipEvent_t> acc_ev;
    bool acc_recorded = false;
    int64_t ws_bytes = 0;
    int64_t total_pairs = 0, total_elems = 0, total_tiles = 0;
};

namespace {

std::vector<DevBuf *> batch_bufs(fs_batch *b)
{
    std::vector<DevBuf *> v = {&b->scenes_d, &b->npairs, &b->fix};
    for (Work &w : b->work)
        for (DevBuf *d : {&w.rec, &w.rect, &w.ntiles, &w.flags, &w.codes, &w.dkeys, &w.dvals, &w.dkeys2, &w.dvals2,
                          &w.counts, &w.offsets, &w.ptiles, &w.pvals, &w.pk_alt, &w.pv_alt, &w.ranges, &w.items, &w.items_k,
                          &w.items_k2, &w.items_v2, &w.sort_ws, &w.scan_ws, &w.tscan_ws, &w.view_offs, &w.tstate,
                          &w.tile_done, &w.queue})
            v.push_back(d);
    for (Chunk &c : b->chunks) {
        v.push_back(&c.views);
        v.push_back(&c.tasks);
        v.push_back(&c.dsegs);
        v.push_back(&c.psegs);
        v.push_back(&c.lsegs);
    }
    return v;
}

void chunk_plan(fs_batch *b, Chunk &c)
{
    c.plan = Plan();
    // consecutive views of one scene form one run of plan_add
    size_t i = 0;
    while (i < c.refs.size()) {
        size_t j = i;
        while (j + 1 < c.refs.size() && c.refs[j + 1].scene == c.refs[i].scene && c.refs[j + 1].v == c.refs[j].v + 1) ++j;
        const SceneIn &s = b->scenes[c.refs[i].scene];
        plan_add(c.plan, &b->p, c.refs[i].scene, s.g.n, s.cams.data(), c.refs[i].v, c.refs[j].v + 1,
                 s.mask_off[c.refs[i].v]);
        i = j + 1;
    }
}

// projection and per-view depth sort of one chunk
int enqueue_front(fs_batch *b, Work &w, Chunk &c, hipStream_t s)
{
    fs_ctx *ctx = b->ctx;
    const Plan &pl = c.plan;
    if (pl.elems == 0) return FS_OK;
    uint32_t *dk = (uint32_t *)w.dkeys.p, *dv = (uint32_t *)w.dvals.p;
    ProjParams pp = proj_params(&b->p);
    pp.cshift = c.cshift;
    HIPCHECK(ctx, launch_project(s, (const ProjTask *)c.tasks.p, (int32_t)pl.tasks.size(), pl.proj_blocks,
                                 (const SceneDev *)b->scenes_d.p, (const ViewDev *)c.views.p, pp,
                                 (float *)w.rec.p, (int16_t *)w.rect.p, (int32_t *)w.ntiles.p, (uint8_t *)w.flags.p,
                                 dk, dv, (uint64_t *)w.codes.p, ctx->status_dev));
    HIPCHECK(ctx, radix_sort(s, dk, dv, (uint32_t *)w.dkeys2.p, (uint32_t *)w.dvals2.p, (const SegDev *)c.dsegs.p,
                             (int32_t)pl.views.size(), pl.dblocks, 32, w.sort_ws.p, nullptr, 1));
    return FS_OK;
}

// pair counts of every element (no slab, no culling) and their exclusive scan; total into *np
int enqueue_full_count(fs_batch *b, Work &w, Chunk &c, uint32_t *np, hipStream_t s)
{
    fs_ctx *ctx = b->ctx;
    const Plan &pl = c.plan;
    const int64_t total = (int64_t)pl.elems;
    if (total == 0) {
        HIPCHECK(ctx, launch_fill_u32(s, np, 0u, 1));
        return FS_OK;
    }
    HIPCHECK(ctx, launch_gather_counts(s, (const uint32_t *)w.dkeys.p, (const uint32_t *)w.dvals.p,
                                       (const int32_t *)w.ntiles.p, (const ViewDev *)c.views.p,
                                       (int32_t)pl.views.size(), total, (uint32_t *)w.counts.p, c.cshift));
    HIPCHECK(ctx, scan_exclusive(s, (const uint32_t *)w.counts.p, (uint32_t *)w.offsets.p, total, np, w.scan_ws.p));
    return FS_OK;
}

// Depth slabs of one chunk, front to back: the pairs of the Gaussians in slab k
// (their depth ranks) are counted, emitted, sorted by tile and composited,
// resuming every pixel's transmittance from the previous slab. Tiles whose
// pixels have all finished are marked by the compositing and get no pairs in
// later slabs, so the long tails of dense tiles are never sorted.
int enqueue_slabs(fs_batch *b, Work &w, Chunk &c, int chunk_idx, hipStream_t s, bool composite = true)
{
    fs_ctx *ctx = b->ctx;
    const Plan &pl = c.plan;
    const int64_t total = (int64_t)pl.elems;
    const int32_t V = (int32_t)pl.views.size();
    if (total == 0 || c.pair_cap == 0 || pl.tiles == 0) return FS_OK;
    const int S = b->n_slabs;
    uint32_t *dk = (uint32_t *)w.dkeys.p, *dv = (uint32_t *)w.dvals.p;
    uint32_t *k0, *v0, *k1, *v1;
    uint32_t *pt = (uint32_t *)w.ptiles.p, *pv = (uint32_t *)w.pvals.p;
    uint32_t *pta = (uint32_t *)w.pk_alt.p, *pva = (uint32_t *)w.pv_alt.p;
    if (c.passes % 2 == 0) {
        k0 = pt; v0 = pv; k1 = pta; v1 = pva;
    } else {
        k0 = pta; v0 = pva; k1 = pt; v1 = pv;
    }
    uint8_t *done = S > 1 ? (uint8_t *)w.tile_done.p : nullptr;
    float *tstate = S > 1 ? (float *)w.tstate.p : nullptr;
    if (done) HIPCHECK(ctx, launch_fill_u32(s, (uint32_t *)done, 0u, (int64_t)((pl.tiles + 3) / 4)));
    for (int k = 0; k < S; ++k) {
        uint32_t *np = (uint32_t *)b->npairs.p + (size_t)chunk_idx * S + k;
        const Slab sl{b->slab_num[k], b->slab_num[k + 1]};
        HIPCHECK(ctx, launch_slab_counts(s, dk, dv, (const float *)w.rec.p, (const int16_t *)w.rect.p,
                                         b->p.fp64_conic ? nullptr : (const uint8_t *)w.flags.p,
                                         (const int32_t *)w.ntiles.p,
                                         (const ViewDev *)c.views.p, V, total, sl, k > 0 ? done : nullptr,
                                         b->p.tile_w, b->p.tile_h, b->p.sigma_k, (const uint64_t *)w.codes.p,
                                         (uint32_t *)w.counts.p, c.cshift));
        HIPCHECK(ctx, scan_exclusive(s, (const uint32_t *)w.counts.p, (uint32_t *)w.offsets.p, total, np,
                                     w.scan_ws.p));
        const uint8_t *fl = b->p.fp64_conic ? nullptr : (const uint8_t *)w.flags.p;
        // tile lists: the sort's last pass counts the pairs of every tile (and
        // skips writing the sorted tile ids, which nothing reads), then the
        // ranges are the exclusive scan of those counts
        uint32_t *tcount = (uint32_t *)w.items_k.p, *tstart = (uint32_t *)w.items_k2.p;
        HIPCHECK(ctx, launch_fill_u32(s, tcount, 0u, (int64_t)pl.tiles));
        if (c.packed) {
            // one u32 item per pair, sorted per view by its tile bits only
            HIPCHECK(ctx, launch_emit(s, dk, dv, (const uint32_t *)w.offsets.p, (const uint32_t *)w.counts.p,
                                      (const float *)w.rec.p, (const int16_t *)w.rect.p, fl,
                                      (const ViewDev *)c.views.p, V, total, c.pair_cap, b->p.tile_w, b->p.tile_h,
                                      b->p.sigma_k, k > 0 ? done : nullptr, pt, nullptr, ctx->status_dev, c.gbits,
                                      (const uint64_t *)w.codes.p, c.cshift));
            HIPCHECK(ctx, launch_pair_segs(s, (const uint32_t *)w.offsets.p, (const ViewDev *)c.views.p, V, total, np,
                                           c.pair_cap, (SegDev *)c.psegs.p, ctx->status_dev));
            HIPCHECK(ctx, radix_sort_packed(s, pt, pta, pv, (const SegDev *)c.psegs.p, V, c.pblocks, c.gbits, c.tbits,
                                            w.sort_ws.p, c.ptpb, tcount));
        } else {
            HIPCHECK(ctx, launch_emit(s, dk, dv, (const uint32_t *)w.offsets.p, (const uint32_t *)w.counts.p,
                                      (const float *)w.rec.p, (const int16_t *)w.rect.p, fl,
                                      (const ViewDev *)c.views.p, V, total, c.pair_cap, b->p.tile_w, b->p.tile_h,
                                      b->p.sigma_k, k > 0 ? done : nullptr, k0, v0, ctx->status_dev, 0,
                                      (const uint64_t *)w.codes.p, c.cshift));
            HIPCHECK(ctx, radix_sort(s, k0, v0, k1, v1, (const SegDev *)c.psegs.p, 1, c.pblocks, c.passes * 8,
                                     w.sort_ws.p, np, c.ptpb, tcount, false));
        }
        HIPCHECK(ctx, scan_exclusive(s, tcount, tstart, (int64_t)pl.tiles, nullptr, w.tscan_ws.p));
        HIPCHECK(ctx, launch_count_ranges(s, tcount, tstart, (int64_t)pl.tiles, (uint32_t *)w.ranges.p));
        if (!composite) continue;
        const uint32_t *items = nullptr;
        if (b->p.tile_order == 0) {
            RCHECK(enqueue_lpt(ctx, s, (const uint32_t *)w.ranges.p, pl.tiles, (const SegDev *)c.lsegs.p,
                               (uint32_t *)w.items.p, (uint32_t *)w.items_k.p, (uint32_t *)w.items_k2.p,
                               (uint32_t *)w.items_v2.p, w.sort_ws.p));
            items = (const uint32_t *)w.items.p;
        }
        hipEvent_t *ev = b->acc_ev.empty() ? nullptr : &b->acc_ev[2 * ((size_t)chunk_idx * S + k)];
        if (ev) HIPCHECK(ctx, hipEventRecord(ev[0], s));
        HIPCHECK(ctx, launch_accumulate(s, (const float *)w.rec.p, pv, (const uint32_t *)w.ranges.p,
                                        (const ViewDev *)c.views.p, V, (const SceneDev *)b->scenes_d.p, items,
                                        (uint32_t)pl.tiles, acc_params(&b->p, b->o.reduction), nullptr, nullptr,
                                        tstate, done, k == 0 ? 1 : 0,
                                        ctx->status_dev, (uint32_t *)w.queue.p));
        if (ev) HIPCHECK(ctx, hipEventRecord(ev[1], s));
    }
    return FS_OK;
}

// the whole solve: optional zeroing, every chunk, every scene's assignment
int enqueue_run(fs_batch *b, hipStream_t s)
{
    fs_ctx *ctx = b->ctx;
    if (b->o.zero_accumulators) {
        for (const SceneIn &sc : b->scenes) {
            const int64_t cnt = (int64_t)sc.g.n * sc.E;
            HIPCHECK(ctx, launch_fill_u32(s, (uint32_t *)sc.A_hi, 0u, cnt));
            if (sc.A_lo) HIPCHECK(ctx, launch_fill_u32(s, (uint32_t *)sc.A_lo, 0u, cnt));
        }
    }
    if (b->o.reduction == FS_RED_DET && b->fix_words > 0)
        HIPCHECK(ctx, launch_fill_u32(s, (uint32_t *)b->fix.p, 0u, 2 * b->fix_words));
    const size_t L = b->work.size();
    if (L > 1) {
        // fork: every lane starts after the zeroing; chunk i runs on lane i % L
        HIPCHECK(ctx, hipEventRecord(b->fork, s));
        for (Work &w : b->work) HIPCHECK(ctx, hipStreamWaitEvent(w.stream, b->fork, 0));
    }
    for (size_t i = 0; i < b->chunks.size(); ++i) {
        Work &w = b->work[i % L];
        hipStream_t ls = L > 1 ? w.stream : s;
        RCHECK(enqueue_front(b, w, b->chunks[i], ls));
        RCHECK(enqueue_slabs(b, w, b->chunks[i], (int)i, ls));
    }
    if (L > 1) {
        // join: the assignment waits for every lane
        for (Work &w : b->work) {
            HIPCHECK(ctx, hipEventRecord(w.done, w.stream));
            HIPCHECK(ctx, hipStreamWaitEvent(s, w.done, 0));
        }
    }
    if (b->o.reduction == FS_RED_DET)
        for (const SceneIn &sc : b->scenes)
            HIPCHECK(ctx, launch_fix_finish(s, sc.fix, sc.A_hi, sc.A_lo, (int64_t)sc.g.n * sc.E));
    for (const SceneIn &sc : b->scenes)
        if (sc.S)
            HIPCHECK(ctx, launch_assign(s, sc.A_hi, sc.A_lo, sc.g.n, sc.E, sc.gamma, sc.S, sc.margin, ctx->status_dev));
    return FS_OK;
}

int batch_alloc(fs_batch *b, DevBuf &buf, size_t bytes)
{
    RCHECK(alloc_buf(b->ctx, buf, bytes < 256 ? 256 : bytes));
    b->ws_bytes += (int64_t)buf.cap;
    return FS_OK;
}

int batch_build(fs_batch *b, const fs_scene *scenes, int32_t n_scenes)
{
    fs_ctx *ctx = b->ctx;
    const int64_t pair_budget = b->o.pair_budget > 0 ? b->o.pair_budget : (int64_t)1 << 28;
    const int64_t elem_budget = b->o.elem_budget > 0 ? b->o.elem_budget : (int64_t)1 << 26;
    // scenes
    std::vector<SceneDev> sd;
    for (int i = 0; i < n_scenes; ++i) {
        const fs_scene &in = scenes[i];
        SceneIn s;
        s.g = in.gauss;
        s.cams.assign(in.cams, in.cams + in.n_views);
        s.mask_off.resize((size_t)in.n_views);
        uint64_t m = 0;
        for (int v = 0; v < in.n_views; ++v) {
            s.mask_off[v] = m;
            m += (uint64_t)in.cams[v].width * in.cams[v].height;
        }
        s.masks = in.masks;
        s.E = in.n_classes;
        s.A_hi = in.A_hi;
        s.A_lo = in.A_lo;
        s.S = in.S;
        s.margin = in.margin;
        s.gamma = in.gamma;
        b->scenes.push_back(s);
        sd.push_back(scene_dev(&in.gauss, in.gauss.n, in.masks, in.A_hi, in.A_lo, in.n_classes));
    }
    if (b->o.reduction == FS_RED_DET) {
        int64_t words = 0;
        for (const SceneIn &s : b->scenes) words += (int64_t)s.g.n * s.E;
        RCHECK(batch_alloc(b, b->fix, (size_t)words * 8));
        b->fix_words = words;
        int64_t off = 0;
        for (size_t i = 0; i < b->scenes.size(); ++i) {
            b->scenes[i].fix = (unsigned long long *)b->fix.p + off;
            sd[i].A_fix = b->scenes[i].fix;
            off += (int64_t)b->scenes[i].g.n * b->scenes[i].E;
        }
    }
    RCHECK(batch_alloc(b, b->scenes_d, sd.size() * sizeof(SceneDev)));
    RCHECK(upload_vec(ctx, b->scenes_d, sd));

    // 1. provisional chunks by element budget, for the exact count
    std::vector<ViewRef> all;
    for (int i = 0; i < n_scenes; ++i)
        for (int v = 0; v < scenes[i].n_views; ++v) all.push_back(ViewRef{(uint32_t)i, v});
    int64_t pb = pair_budget, eb = elem_budget;  // lowered below to give every lane a chunk
    auto chunk_by = [&](const std::vector<int64_t> *pairs) {
        std::vector<Chunk> out;
        Chunk cur;
        int64_t ce = 0, cp = 0;
        uint64_t ct = 0;
        for (size_t k = 0; k < all.size(); ++k) {
            const SceneIn &s = b->scenes[all[k].scene];
            const int64_t e = s.g.n;
            const int64_t p = pairs ? (*pairs)[k] : 0;
            const fs_camera &c = s.cams[all[k].v];
            const uint64_t t = (uint64_t)((c.width + b->p.tile_w - 1) / b->p.tile_w) *
                               (uint64_t)((c.height + b->p.tile_h - 1) / b->p.tile_h);
            if (!cur.refs.empty() && (ce + e > eb || cp + p > pb || ct + t > 0x7FFFFFFFull)) {
                out.push_back(std::move(cur));
                cur = Chunk();
                ce = cp = 0;
                ct = 0;
            }
            cur.refs.push_back(all[k]);
            ce += e;
            cp += p;
            ct += t;
        }
        if (!cur.refs.empty()) out.push_back(std::move(cur));
        return out;
    };
    std::vector<Chunk> prov = chunk_by(nullptr);
    uint64_t max_e = 0;
    uint32_t max_db = 0;
    size_t max_v = 0;
    for (Chunk &c : prov) {
        chunk_plan(b, c);
        max_e = std::max<uint64_t>(max_e, c.plan.elems);
        max_db = std::max(max_db, c.plan.dblocks);
        max_v = std::max(max_v, c.plan.views.size());
    }
    if (max_e >= 0xFFFFFFFFull) return set_err(ctx, FS_ERR_ARG, "a single view holds too many Gaussians");
    // projection and depth-sort workspace (sized for the element budget)
    const size_t E4 = (size_t)std::max<uint64_t>(max_e, 1) * 4;
    b->work.resize(1);
    auto alloc_elem_ws = [&](Work &w) -> int {
        RCHECK(batch_alloc(b, w.rec, E4 * 8));
        RCHECK(batch_alloc(b, w.rect, E4 * 2));
        RCHECK(batch_alloc(b, w.ntiles, E4));
        RCHECK(batch_alloc(b, w.flags, E4 / 4 + 256));
        RCHECK(batch_alloc(b, w.codes, E4 * 8));  // 32-byte emission records
        RCHECK(batch_alloc(b, w.dkeys, E4));
        RCHECK(batch_alloc(b, w.dvals, E4));
        RCHECK(batch_alloc(b, w.dkeys2, E4));
        RCHECK(batch_alloc(b, w.dvals2, E4));
        RCHECK(batch_alloc(b, w.counts, E4));
        RCHECK(batch_alloc(b, w.offsets, E4));
        RCHECK(batch_alloc(b, w.scan_ws, scan_ws_bytes((int64_t)max_e)));
        return FS_OK;
    };
    RCHECK(alloc_elem_ws(b->work[0]));
    const int S = b->n_slabs, NB = S + 1;
    RCHECK(batch_alloc(b, b->npairs, 4 * (all.size() * S + 64)));
    RCHECK(batch_alloc(b, b->work[0].view_offs, 4 * (max_v * NB + 64)));
    SlabBounds nb;
    nb.n = (uint32_t)NB;
    for (int i = 0; i < 9; ++i) nb.num[i] = i < NB ? b->slab_num[i] : 1024u;
    DevBuf tmp_sort;
    RCHECK(alloc_buf(ctx, tmp_sort, radix_ws_bytes(std::max<uint32_t>(max_db, 1))));

    // 2. exact pair count of every view and of each of its depth slabs
    std::vector<int64_t> vpairs(all.size(), 0);
    std::vector<int64_t> vslab(all.size() * S, 0);
    std::vector<uint32_t> hoff;
    size_t k0 = 0;
    int rc = FS_OK;
    for (size_t ci = 0; ci < prov.size() && !rc; ++ci) {
        Chunk &c = prov[ci];
        const int32_t V = (int32_t)c.plan.views.size();
        if ((rc = upload_vec(ctx, c.views, c.plan.views)) || (rc = upload_vec(ctx, c.tasks, c.plan.tasks)) ||
            (rc = upload_vec(ctx, c.dsegs, c.plan.dsegs)))
            break;
        std::swap(b->work[0].sort_ws, tmp_sort);
        rc = enqueue_front(b, b->work[0], c, ctx->stream);
        if (!rc) rc = enqueue_full_count(b, b->work[0], c, (uint32_t *)b->npairs.p, ctx->stream);
        std::swap(b->work[0].sort_ws, tmp_sort);
        if (rc) break;
        hipError_t e = c.plan.elems > 0
                           ? launch_slab_offsets(ctx->stream, (const uint32_t *)b->work[0].offsets.p, (const ViewDev *)c.views.p,
                                                 V, (int64_t)c.plan.elems, (const uint32_t *)b->npairs.p, nb,
                                                 (uint32_t *)b->work[0].view_offs.p)
                           : launch_fill_u32(ctx->stream, (uint32_t *)b->work[0].view_offs.p, 0u, (int64_t)V * NB);
        hoff.assign((size_t)V * NB, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hoff.data(), b->work[0].view_offs.p, 4 * hoff.size(), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            rc = set_err(ctx, FS_ERR_HIP, "batch count failed: %s", hipGetErrorString(e));
            break;
        }
        for (int v = 0; v < V; ++v) {
            const uint32_t *o = &hoff[(size_t)v * NB];
            vpairs[k0 + v] = (int64_t)o[S] - (int64_t)o[0];
            for (int q = 0; q < S; ++q) vslab[(k0 + v) * S + q] = (int64_t)o[q + 1] - (int64_t)o[q];
        }
        k0 += (size_t)V;
        free_buf(c.views);
        free_buf(c.tasks);
        free_buf(c.dsegs);
    }
    for (Chunk &c : prov) {
        free_buf(c.views);
        free_buf(c.tasks);
        free_buf(c.dsegs);
    }
    free_buf(tmp_sort);
    if (rc) return rc;

    // 3. final chunks by elements and pairs; per-chunk tables
    const int lanes_req = b->o.lanes == 0 ? 2 : b->o.lanes;
    if (lanes_req > 1) {
        // a lane's share plus one view, so that the greedy split gives `lanes`
        // chunks of nearly equal work rather than one more small chunk
        int64_t tp = 0, te = 0, mp = 0, me = 0;
        for (size_t q = 0; q < all.size(); ++q) {
            tp += vpairs[q];
            te += b->scenes[all[q].scene].g.n;
            mp = std::max<int64_t>(mp, vpairs[q]);
            me = std::max<int64_t>(me, b->scenes[all[q].scene].g.n);
        }
        pb = std::min<int64_t>(pb, std::max<int64_t>(1, (tp + lanes_req - 1) / lanes_req + mp));
        eb = std::min<int64_t>(eb, std::max<int64_t>(1, (te + lanes_req - 1) / lanes_req + me));
    }
    b->chunks = chunk_by(&vpairs);
    size_t k = 0;
    for (Chunk &c : b->chunks) {
        chunk_plan(b, c);
        for (size_t j = 0; j < c.refs.size(); ++j) {
            c.pairs += (uint64_t)vpairs[k + j];
            c.vpairs.push_back((uint64_t)vpairs[k + j]);
        }
        for (int q = 0; q < S; ++q) {
            uint64_t sum = 0;
            for (size_t j = 0; j < c.refs.size(); ++j) sum += (uint64_t)vslab[(k + j) * S + q];
            c.slab_max = std::max(c.slab_max, sum);
        }
        k += c.refs.size();
        if (c.pairs >= 0xFFFFF000ull) return set_err(ctx, FS_ERR_CAPACITY, "a single view needs too many tile pairs");
        b->max_pairs = std::max<uint64_t>(b->max_pairs, c.slab_max);
        b->max_tiles = std::max<uint64_t>(b->max_tiles, c.plan.tiles);
        b->max_pixels = std::max<uint64_t>(b->max_pixels, c.plan.pixels);
        b->max_elems = std::max<uint64_t>(b->max_elems, c.plan.elems);
        b->max_dblocks = std::max(b->max_dblocks, c.plan.dblocks);
        b->total_pairs += (int64_t)c.pairs;
        b->total_elems += (int64_t)c.plan.elems;
        b->total_tiles += (int64_t)c.plan.tiles;
    }
    const uint64_t cap = std::min<uint64_t>(0xFFFFF000ull, b->max_pairs + b->max_pairs / 64 + 4096);
    for (Chunk &c : b->chunks) {
        c.pair_cap = (uint32_t)std::min<uint64_t>(cap, c.slab_max + c.slab_max / 64 + 4096);
        c.ptpb = radix_tiles_per_block(c.pair_cap);
        c.pblocks = (uint32_t)(((uint64_t)c.pair_cap + (uint64_t)kSortTile * c.ptpb - 1) / ((uint64_t)kSortTile * c.ptpb));
        std::vector<SegDev> ps{SegDev{0, c.pair_cap, 0, c.pair_cap, 0}};
        {
            uint64_t max_n = 1, max_tv = 1;
            for (const ViewDev &vd : c.plan.views) {
                max_n = std::max<uint64_t>(max_n, vd.n);
                max_tv = std::max<uint64_t>(max_tv, (uint64_t)vd.tiles_x * (uint64_t)vd.tiles_y);
            }
            c.gbits = bits_for(max_n);
            c.tbits = bits_for(max_tv);
            c.cshift = c.gbits <= 24 ? c.gbits : 0;  // at least 8 bits for the carried count
            // (with depth slabs every slab's pairs of a view are at most the view's planned
            // pairs, so the per-view capacities below hold for every slab)
            c.packed = c.tbits <= 16 && c.gbits + c.tbits <= 32 && c.vpairs.size() == c.plan.views.size();
            if (c.packed) {
                // per-view capacities (planned count plus slack) and blocks
                uint64_t sum = 0;
                for (uint64_t vp : c.vpairs) sum += vp + vp / 64 + 256;
                c.ptpb = radix_tiles_per_block(sum);
                const uint64_t span = (uint64_t)kSortTile * c.ptpb;
                ps.clear();
                uint32_t blk = 0;
                for (size_t j = 0; j < c.vpairs.size(); ++j) {
                    const uint64_t capj = std::min<uint64_t>(c.vpairs[j] + c.vpairs[j] / 64 + 256, c.pair_cap);
                    ps.push_back(SegDev{0, (uint32_t)capj, blk, 0, c.plan.views[j].tile_base});
                    blk += (uint32_t)std::max<uint64_t>(1, (capj + span - 1) / span);
                }
                c.pblocks = blk;
            }
        }
        c.lblocks = (uint32_t)((c.plan.tiles + kSortTile - 1) / kSortTile);
        c.passes = (bits_for(std::max<uint64_t>(c.plan.tiles, 2)) + 7) / 8;
        b->max_pblocks = std::max(b->max_pblocks, c.pblocks);
        b->max_lblocks = std::max(b->max_lblocks, c.lblocks);
        RCHECK(upload_vec(ctx, c.views, c.plan.views));
        RCHECK(upload_vec(ctx, c.tasks, c.plan.tasks));
        RCHECK(upload_vec(ctx, c.dsegs, c.plan.dsegs));
        RCHECK(upload_vec(ctx, c.psegs, ps));
        std::vector<SegDev> ls{SegDev{0, (uint32_t)c.plan.tiles, 0, (uint32_t)c.plan.tiles, 0}};
        RCHECK(upload_vec(ctx, c.lsegs, ls));
        for (DevBuf *d : {&c.views, &c.tasks, &c.dsegs, &c.psegs, &c.lsegs}) b->ws_bytes += (int64_t)d->cap;
    }
    const size_t n_lanes = std::max<size_t>(1, std::min<size_t>((size_t)lanes_req, b->chunks.size()));
    b->work.resize(n_lanes);
    for (size_t l = 1; l < n_lanes; ++l) RCHECK(alloc_elem_ws(b->work[l]));
    const size_t P4 = (size_t)std::max<uint64_t>(cap, 1) * 4;
    const size_t T4 = (size_t)std::max<uint64_t>(b->max_tiles, 1) * 4;
    const uint32_t sb = std::max(std::max(b->max_dblocks, b->max_pblocks), std::max<uint32_t>(b->max_lblocks, 1));
    for (Work &w : b->work) {
        RCHECK(batch_alloc(b, w.ptiles, P4));
        RCHECK(batch_alloc(b, w.pvals, P4));
        RCHECK(batch_alloc(b, w.pk_alt, P4));
        RCHECK(batch_alloc(b, w.pv_alt, P4));
        RCHECK(batch_alloc(b, w.ranges, T4 * 2));
        RCHECK(batch_alloc(b, w.items, T4));
        RCHECK(batch_alloc(b, w.items_k, T4));
        RCHECK(batch_alloc(b, w.items_k2, T4));
        RCHECK(batch_alloc(b, w.items_v2, T4));
        RCHECK(batch_alloc(b, w.tscan_ws, scan_ws_bytes((int64_t)std::max<uint64_t>(b->max_tiles, 1))));
        RCHECK(batch_alloc(b, w.sort_ws, radix_ws_bytes(sb)));
        RCHECK(batch_alloc(b, w.queue, 256));
        if (S > 1) {
            RCHECK(batch_alloc(b, w.tstate, (size_t)std::max<uint64_t>(b->max_pixels, 1) * 4));
            RCHECK(batch_alloc(b, w.tile_done, ((size_t)b->max_tiles + 3) / 4 * 4 + 4));
        }
    }
    if (n_lanes > 1) {
        HIPCHECK(ctx, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (Work &w : b->work) {
            HIPCHECK(ctx, hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
            HIPCHECK(ctx, hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
        }
    }
    if (!b->o.use_graph) {
        b->acc_ev.assign(2 * b->chunks.size() * (size_t)S, nullptr);
        for (hipEvent_t &e : b->acc_ev) HIPCHECK(ctx, hipEventCreate(&e));
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));

    // 4. capture the whole solve into one graph
    if (b->o.use_graph) {
        hipStream_t s = ctx->stream;
        bool own_stream = false;
        if (s == nullptr) {  // the null stream cannot be captured: record on a private stream
            HIPCHECK(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            own_stream = true;
        }
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            if (own_stream) (void)hipStreamDestroy(s);
            return set_err(ctx, FS_ERR_HIP, "graph capture could not start: %s", hipGetErrorString(e));
        }
        rc = enqueue_run(b, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (own_stream) (void)hipStreamDestroy(s);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_err(ctx, FS_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        b->graph = g;
        HIPCHECK(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    return FS_OK;
}

}  // namespace

extern "C" {

void fs_batch_opts_default(fs_batch_opts *o)
{
    if (!o) return;
    o->pair_budget = 0;
    o->elem_budget = 0;
    o->zero_accumulators = 1;
    o->use_graph = 1;
    o->reduction = FS_RED_AUTO;
    o->depth_slabs = 0;
    o->lanes = 0;
}

int fs_batch_create(fs_ctx *ctx, const fs_scene *scenes, int32_t n_scenes, const fs_params *p,
                    const fs_batch_opts *opts, fs_batch **out)
{
    if (!ctx) return FS_ERR_ARG;
    if (!out) return set_err(ctx, FS_ERR_ARG, "out is NULL");
    *out = nullptr;
    RCHECK(check_params(ctx, p, true));
    if (p->tile_order == 2) return set_err(ctx, FS_ERR_ARG, "batches support tile_order 0 and 1");
    if (n_scenes <= 0 || !scenes) return set_err(ctx, FS_ERR_ARG, "need at least one scene");
    fs_batch_opts o;
    fs_batch_opts_default(&o);
    if (opts) o = *opts;
    if (o.reduction < FS_RED_AUTO || o.reduction > FS_RED_DET) return set_err(ctx, FS_ERR_ARG, "unknown reduction");
    if (o.depth_slabs < 0 || o.depth_slabs > 4) return set_err(ctx, FS_ERR_ARG, "depth_slabs must be in [0, 4]");
    if (o.lanes < 0 || o.lanes > 4) return set_err(ctx, FS_ERR_ARG, "lanes must be in [0, 4]");
    bool all_lo = true;
    for (int i = 0; i < n_scenes; ++i) {
        const fs_scene &s = scenes[i];
        RCHECK(check_gauss(ctx, &s.gauss));
        RCHECK(check_cams(ctx, s.cams, s.n_views));
        if (s.n_classes < 2 || s.n_classes > 256) return set_err(ctx, FS_ERR_ARG, "scene %d: n_classes not in [2, 256]", i);
        if (s.gauss.n > 0 && (!s.A_hi || (s.n_views > 0 && !s.masks)))
            return set_err(ctx, FS_ERR_ARG, "scene %d: A_hi or masks is NULL", i);
        if (s.S && (!finite_f(s.gamma) || s.gamma < -1.f || s.gamma > 1.f))
            return set_err(ctx, FS_ERR_ARG, "scene %d: gamma must be finite in [-1, 1]", i);
        if (o.reduction == FS_RED_DET) {
            uint64_t px = 0;
            for (int v = 0; v < s.n_views; ++v) px += (uint64_t)s.cams[v].width * (uint64_t)s.cams[v].height;
            if (px > kFixMaxPixels)
                return set_err(ctx, FS_ERR_ARG, "scene %d: FS_RED_DET takes at most %llu pixels per scene", i,
                               (unsigned long long)kFixMaxPixels);
        }
        all_lo = all_lo && s.A_lo != nullptr;
    }
    if (o.reduction == FS_RED_AUTO) o.reduction = all_lo ? FS_RED_LDS2SUM : FS_RED_LDS;
    if (o.reduction == FS_RED_LDS2SUM && !all_lo) return set_err(ctx, FS_ERR_ARG, "FS_RED_LDS2SUM needs A_lo in every scene");
    fs_batch *b = new (std::nothrow) fs_batch();
    if (!b) return FS_ERR_ALLOC;
    b->ctx = ctx;
    b->p = *p;
    b->o = o;
    {
        static const uint32_t kSlabNum[5][5] = {
            {0, 1024}, {0, 256, 1024}, {0, 102, 307, 1024}, {0, 51, 154, 410, 1024}, {0}};
        const int S = o.depth_slabs == 0 ? 1 : o.depth_slabs;
        b->n_slabs = S;
        for (int i = 0; i <= S; ++i) b->slab_num[i] = kSlabNum[S - 1][i];
    }
    int rc = batch_build(b, scenes, n_scenes);
    if (rc) {
        fs_batch_destroy(b);
        return rc;
    }
    *out = b;
    return FS_OK;
}

int fs_batch_run(fs_batch *b)
{
    if (!b) return FS_ERR_ARG;
    fs_ctx *ctx = b->ctx;
    if (b->exec) {
        HIPCHECK(ctx, hipGraphLaunch(b->exec, ctx->stream));
        return FS_OK;
    }
    b->acc_recorded = false;
    RCHECK(enqueue_run(b, ctx->stream));
    b->acc_recorded = !b->acc_ev.empty();
    return FS_OK;
}

int fs_batch_accumulate_ms(fs_batch *b, float *total_ms, int32_t *n_launches)
{
    if (!b || !total_ms || !n_launches) return FS_ERR_ARG;
    fs_ctx *ctx = b->ctx;
    if (!b->acc_recorded) return set_err(ctx, FS_ERR_STATE, "no fs_batch_run without a graph has been timed");
    double sum = 0.0;
    int32_t cnt = 0;
    for (size_t i = 0; i < b->chunks.size(); ++i) {
        const Chunk &c = b->chunks[i];
        if (c.plan.elems == 0 || c.pair_cap == 0 || c.plan.tiles == 0) continue;  // nothing was launched
        for (int k = 0; k < b->n_slabs; ++k) {
            hipEvent_t e0 = b->acc_ev[2 * (i * (size_t)b->n_slabs + k)], e1 = b->acc_ev[2 * (i * (size_t)b->n_slabs + k) + 1];
            HIPCHECK(ctx, hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHECK(ctx, hipEventElapsedTime(&ms, e0, e1));
            sum += ms;
            ++cnt;
        }
    }
    *total_ms = (float)sum;
    *n_launches = cnt;
    return FS_OK;
}

int fs_batch_chunk_lists(fs_batch *b, int32_t chunk, uint32_t *vals, int64_t vals_cap, uint32_t *ranges,
                         int64_t ranges_cap, int32_t *view_refs, int32_t refs_cap, fs_chunk_info *info)
{
    if (!b || !info) return FS_ERR_ARG;
    fs_ctx *ctx = b->ctx;
    if (chunk < 0 || chunk >= (int32_t)b->chunks.size())
        return set_err(ctx, FS_ERR_ARG, "chunk %d of %zu", chunk, b->chunks.size());
    if (b->n_slabs != 1) return set_err(ctx, FS_ERR_STATE, "tile lists are per depth slab when depth_slabs > 1");
    Chunk &c = b->chunks[chunk];
    info->n_views = (int32_t)c.refs.size();
    info->n_tiles = (int64_t)c.plan.tiles;
    info->n_pairs = (int64_t)c.pairs;
    info->packed = c.packed ? 1 : 0;
    if (!vals || !ranges || !view_refs) return FS_OK;  // sizes only
    if (vals_cap < (int64_t)c.pairs || ranges_cap < (int64_t)c.plan.tiles || refs_cap < (int32_t)c.refs.size())
        return set_err(ctx, FS_ERR_CAPACITY, "chunk %d needs %llu ids, %llu ranges, %zu view refs", chunk,
                       (unsigned long long)c.pairs, (unsigned long long)c.plan.tiles, c.refs.size());
    for (size_t j = 0; j < c.refs.size(); ++j) {
        view_refs[2 * j] = (int32_t)c.refs[j].scene;
        view_refs[2 * j + 1] = c.refs[j].v;
    }
    // the chunk's binning on lane 0's workspace, as the solve runs it, without the compositing
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    for (Work &w : b->work)
        if (w.stream) HIPCHECK(ctx, hipStreamSynchronize(w.stream));
    Work &w = b->work[0];
    hipStream_t s = ctx->stream;
    RCHECK(enqueue_front(b, w, c, s));
    RCHECK(enqueue_slabs(b, w, c, chunk, s, false));
    if (c.pairs > 0)
        HIPCHECK(ctx, hipMemcpyAsync(vals, w.pvals.p, (size_t)c.pairs * 4, hipMemcpyDeviceToDevice, s));
    if (c.plan.tiles > 0)
        HIPCHECK(ctx, hipMemcpyAsync(ranges, w.ranges.p, (size_t)c.plan.tiles * 8, hipMemcpyDeviceToDevice, s));
    HIPCHECK(ctx, hipStreamSynchronize(s));
    return FS_OK;
}

int fs_batch_get_info(fs_batch *b, fs_batch_info *out)
{
    if (!b || !out) return FS_ERR_ARG;
    out->n_chunks = (int32_t)b->chunks.size();
    int32_t nv = 0;
    for (const SceneIn &s : b->scenes) nv += (int32_t)s.cams.size();
    out->n_views = nv;
    out->pairs = b->total_pairs;
    out->pair_capacity = b->work.empty() ? 0 : (int64_t)(b->work[0].ptiles.cap / 4);
    out->elements = b->total_elems;
    out->tiles = b->total_tiles;
    out->workspace_bytes = b->ws_bytes;
    return FS_OK;
}

int fs_batch_destroy(fs_batch *b)
{
    if (!b) return FS_ERR_ARG;
    if (b->ctx) (void)hipStreamSynchronize(b->ctx->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (Work &w : b->work) {
        if (w.stream) {
            (void)hipStreamSynchronize(w.stream);
            (void)hipStreamDestroy(w.stream);
        }
        if (w.done) (void)hipEventDestroy(w.done);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (hipEvent_t e : b->acc_ev)
        if (e) (void)hipEventDestroy(e);
    for (DevBuf *d : batch_bufs(b)) free_buf(*d);
    delete b;
    return FS_OK;
}

}  // extern "C"
