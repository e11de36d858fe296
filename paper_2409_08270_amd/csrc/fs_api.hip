// C ABI of the library: context, argument validation, workspace and the four
// calls of the splat-and-accumulate path (declared in include/flashsplat.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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

}  // namespace

struct fs_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    unsigned long long *status_dev = nullptr;
    unsigned long long *status_host = nullptr;  // pinned
    uint32_t *npairs_dev = nullptr;
    uint32_t *npairs_host = nullptr;            // pinned
    DevBuf cams;
    DevBuf dkeys, dvals, dkeys2, dvals2, counts, offsets;
    DevBuf pk_alt, pv_alt, sort_ws, scan_ws;
    DevBuf items, items_k, items_k2, items_v2, items_ws;
    uint64_t items_tiles = 0;  // tile count the XCD-run table was built for
    Staging stage[4];
    int stage_next = 0;
    std::string last_error;
};

namespace {

int set_err(fs_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

#define HIPCHECK(ctx, expr)                                                                      \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess)                                                                    \
            return set_err((ctx), FS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));    \
    } while (0)

int ensure(fs_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap) return FS_OK;
    if (b.p) {
        // the stream may still use the old buffer
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
        HIPCHECK(ctx, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4 + 4096;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        return set_err(ctx, FS_ERR_ALLOC, "device allocation of %zu bytes failed", want);
    }
    b.cap = want;
    return FS_OK;
}

// Copies host bytes to a device buffer asynchronously through a ring of
// pinned staging buffers (a slot is reused only after its copy completed).
int upload(fs_ctx *ctx, DevBuf &dst, const void *src, size_t bytes)
{
    int rc = ensure(ctx, dst, bytes);
    if (rc) return rc;
    Staging &st = ctx->stage[ctx->stage_next];
    ctx->stage_next = (ctx->stage_next + 1) % 4;
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

// Device camera table; returns the total number of tiles and pixels.
int build_cams(fs_ctx *ctx, const fs_camera *cams, int32_t n_views, const fs_params *p, uint64_t *tiles_out,
               uint64_t *pixels_out)
{
    std::vector<CamDev> cd((size_t)n_views);
    uint64_t tb = 0, px = 0;
    for (int v = 0; v < n_views; ++v) {
        const fs_camera &c = cams[v];
        CamDev &d = cd[v];
        memcpy(d.R, c.R, sizeof(d.R));
        memcpy(d.t, c.t, sizeof(d.t));
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        d.W = c.width; d.H = c.height;
        d.tiles_x = (c.width + p->tile_w - 1) / p->tile_w;
        d.tiles_y = (c.height + p->tile_h - 1) / p->tile_h;
        d.tile_base = (uint32_t)tb;
        d.pad = 0;
        d.mask_off = px;
        tb += (uint64_t)d.tiles_x * d.tiles_y;
        px += (uint64_t)c.width * c.height;
    }
    if (tb >= 0xFFFFFFFFull) return set_err(ctx, FS_ERR_ARG, "too many tiles in one call (%llu)", (unsigned long long)tb);
    if (tiles_out) *tiles_out = tb;
    if (pixels_out) *pixels_out = px;
    if (n_views == 0) return FS_OK;
    return upload(ctx, ctx->cams, cd.data(), cd.size() * sizeof(CamDev));
}

// Work order of fs_accumulate. Workgroups are handed to the chip's 8 XCDs in
// round-robin order of their index, and every XCD has its own L2. The table
// maps workgroup b to tile (b % 8) * run + b / 8 (with the remainder spread
// over the first XCDs), so XCD x composites one contiguous run of tiles: the
// Gaussian records that neighbouring tiles share stay in one L2.
constexpr int kXcds = 8;

int build_items(fs_ctx *ctx, uint64_t n_tiles)
{
    if (ctx->items_tiles == n_tiles && ctx->items.p) return FS_OK;
    ctx->items_tiles = 0;
    std::vector<uint32_t> it((size_t)n_tiles);
    const uint64_t base = n_tiles / kXcds, rem = n_tiles % kXcds;
    uint64_t start[kXcds];
    uint64_t acc = 0;
    for (int x = 0; x < kXcds; ++x) {
        start[x] = acc;
        acc += base + ((uint64_t)x < rem ? 1 : 0);
    }
    for (uint64_t b = 0; b < n_tiles; ++b) it[b] = (uint32_t)(start[b % kXcds] + b / kXcds);
    int rc = upload(ctx, ctx->items, it.data(), it.size() * sizeof(uint32_t));
    if (rc) return rc;
    ctx->items_tiles = n_tiles;
    return FS_OK;
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
    return q;
}

int check_proj(fs_ctx *ctx, const fs_proj *pr)
{
    if (!pr) return set_err(ctx, FS_ERR_ARG, "proj is NULL");
    if (pr->n < 0 || pr->n_views < 0) return set_err(ctx, FS_ERR_ARG, "proj sizes negative");
    if (pr->n >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "too many Gaussians (%lld)", (long long)pr->n);
    if ((int64_t)pr->n * pr->n_views >= 0x7FFFFFFFll * 2)
        return set_err(ctx, FS_ERR_ARG, "n * n_views too large for one call");
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

}  // namespace

extern "C" {

const char *fs_version(void) { return "flashsplat-gfx950 0.1"; }

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
    if (!rc && hipMalloc((void **)&ctx->status_dev, ST_COUNT * sizeof(unsigned long long)) != hipSuccess) rc = FS_ERR_ALLOC;
    if (!rc && hipMalloc((void **)&ctx->npairs_dev, 64) != hipSuccess) rc = FS_ERR_ALLOC;
    if (!rc && hipHostMalloc((void **)&ctx->status_host, ST_COUNT * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        rc = FS_ERR_ALLOC;
    if (!rc && hipHostMalloc((void **)&ctx->npairs_host, 64, hipHostMallocDefault) != hipSuccess) rc = FS_ERR_ALLOC;
    for (int i = 0; !rc && i < 4; ++i)
        if (hipEventCreateWithFlags(&ctx->stage[i].ev, hipEventDisableTiming) != hipSuccess) rc = FS_ERR_HIP;
    if (!rc && launch_fill_u32(ctx->stream, (uint32_t *)ctx->status_dev, 0u, ST_COUNT * 2) != hipSuccess) rc = FS_ERR_HIP;
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
    DevBuf *bufs[] = {&ctx->cams, &ctx->dkeys, &ctx->dvals, &ctx->dkeys2, &ctx->dvals2, &ctx->counts,
                      &ctx->offsets, &ctx->pk_alt, &ctx->pv_alt, &ctx->sort_ws, &ctx->scan_ws, &ctx->items,
                      &ctx->items_k, &ctx->items_k2, &ctx->items_v2, &ctx->items_ws};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (int i = 0; i < 4; ++i) {
        if (ctx->stage[i].host) (void)hipHostFree(ctx->stage[i].host);
        if (ctx->stage[i].ev) (void)hipEventDestroy(ctx->stage[i].ev);
    }
    if (ctx->status_dev) (void)hipFree(ctx->status_dev);
    if (ctx->npairs_dev) (void)hipFree(ctx->npairs_dev);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    if (ctx->npairs_host) (void)hipHostFree(ctx->npairs_host);
    delete ctx;
    return FS_OK;
}

const char *fs_ctx_last_error(fs_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int fs_status_get(fs_ctx *ctx, fs_status *out, int32_t clear)
{
    if (!ctx || !out) return set_err(ctx, FS_ERR_ARG, "NULL argument");
    HIPCHECK(ctx, hipMemcpyAsync(ctx->status_host, ctx->status_dev, ST_COUNT * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned long long *h = ctx->status_host;
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
    if (clear) {
        HIPCHECK(ctx, launch_fill_u32(ctx->stream, (uint32_t *)ctx->status_dev, 0u, ST_COUNT * 2));
    }
    const uint32_t errbits = FS_DEV_BAD_LABEL | FS_DEV_PAIR_OVERFLOW | FS_DEV_INVALID_GAUSS;
    if (out->flags & errbits) return set_err(ctx, FS_ERR_DEVICE, "device status flags 0x%x", out->flags);
    return FS_OK;
}

int fs_project(fs_ctx *ctx, const fs_gaussians *g, const fs_camera *cams, int32_t n_views, const fs_params *p,
               const fs_proj *out)
{
    if (!ctx) return FS_ERR_ARG;
    if (!g || !out) return set_err(ctx, FS_ERR_ARG, "NULL argument");
    int rc = check_params(ctx, p, false);
    if (rc) return rc;
    if ((rc = check_cams(ctx, cams, n_views))) return rc;
    if ((rc = check_proj(ctx, out))) return rc;
    if (g->n < 0) return set_err(ctx, FS_ERR_ARG, "n < 0");
    if (out->n != g->n || out->n_views != n_views)
        return set_err(ctx, FS_ERR_ARG, "proj sized for n=%lld, views=%d; need n=%lld, views=%d", (long long)out->n,
                       out->n_views, (long long)g->n, n_views);
    if (g->n > 0 && (!g->mx || !g->my || !g->mz || !g->qw || !g->qx || !g->qy || !g->qz || !g->sx || !g->sy ||
                     !g->sz || !g->opacity))
        return set_err(ctx, FS_ERR_ARG, "Gaussian array is NULL");
    if (g->n == 0 || n_views == 0) return FS_OK;
    if ((rc = build_cams(ctx, cams, n_views, p, nullptr, nullptr))) return rc;
    GaussPtrs gp{g->mx, g->my, g->mz, g->qw, g->qx, g->qy, g->qz, g->sx, g->sy, g->sz, g->opacity};
    HIPCHECK(ctx, launch_project(ctx->stream, gp, g->n, (const CamDev *)ctx->cams.p, n_views, proj_params(p), out->rec,
                                 out->rect, out->ntiles, out->flags, ctx->status_dev));
    return FS_OK;
}

int fs_bin_sort(fs_ctx *ctx, const fs_proj *proj, const fs_camera *cams, const fs_params *p, const fs_bins *out,
                int64_t *n_pairs)
{
    if (!ctx) return FS_ERR_ARG;
    int rc = check_params(ctx, p, false);
    if (rc) return rc;
    if ((rc = check_proj(ctx, proj))) return rc;
    if (!out) return set_err(ctx, FS_ERR_ARG, "bins is NULL");
    if ((rc = check_cams(ctx, cams, proj->n_views))) return rc;
    if (out->capacity < 0 || out->capacity >= 0xFFFFFFFFll) return set_err(ctx, FS_ERR_ARG, "bad bins capacity");
    if (!out->ranges || (out->capacity > 0 && (!out->vals || !out->tiles)))
        return set_err(ctx, FS_ERR_ARG, "bins has NULL arrays");
    const int64_t n = proj->n;
    const int32_t V = proj->n_views;
    uint64_t total_tiles = 0;
    if ((rc = build_cams(ctx, cams, V, p, &total_tiles, nullptr))) return rc;
    hipStream_t s = ctx->stream;
    HIPCHECK(ctx, launch_fill_u32(s, out->ranges, 0u, (int64_t)total_tiles * 2));
    const int64_t total = n * V;
    if (total == 0) {
        if (n_pairs) *n_pairs = 0;
        HIPCHECK(ctx, launch_fill_u32(s, ctx->npairs_dev, 0u, 1));
        return FS_OK;
    }
    const size_t tb = (size_t)total * 4;
    if ((rc = ensure(ctx, ctx->dkeys, tb)) || (rc = ensure(ctx, ctx->dvals, tb)) || (rc = ensure(ctx, ctx->dkeys2, tb)) ||
        (rc = ensure(ctx, ctx->dvals2, tb)) || (rc = ensure(ctx, ctx->counts, tb)) || (rc = ensure(ctx, ctx->offsets, tb)))
        return rc;
    size_t ws = radix_ws_bytes(n, V);
    if ((rc = ensure(ctx, ctx->sort_ws, ws))) return rc;
    if ((rc = ensure(ctx, ctx->scan_ws, scan_ws_bytes(total)))) return rc;
    uint32_t *dk = (uint32_t *)ctx->dkeys.p, *dv = (uint32_t *)ctx->dvals.p;
    uint32_t *dk2 = (uint32_t *)ctx->dkeys2.p, *dv2 = (uint32_t *)ctx->dvals2.p;
    // depth order of each view's emitting Gaussians (4 passes: result back in dk/dv)
    HIPCHECK(ctx, launch_depth_keys(s, proj->rec, proj->ntiles, proj->flags, n, V, dk, dv));
    HIPCHECK(ctx, radix_sort(s, dk, dv, dk2, dv2, n, V, 32, ctx->sort_ws.p));
    HIPCHECK(ctx, launch_gather_counts(s, dk, dv, proj->ntiles, n, V, (uint32_t *)ctx->counts.p));
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
    const int bits = bits_for(total_tiles);
    const int passes = (bits + 7) / 8;
    if ((rc = ensure(ctx, ctx->pk_alt, (size_t)sort_len * 4)) || (rc = ensure(ctx, ctx->pv_alt, (size_t)sort_len * 4)))
        return rc;
    ws = radix_ws_bytes(sort_len, 1);
    if ((rc = ensure(ctx, ctx->sort_ws, ws))) return rc;
    uint32_t *k0, *v0, *k1, *v1;
    if (passes % 2 == 0) {
        k0 = out->tiles; v0 = out->vals; k1 = (uint32_t *)ctx->pk_alt.p; v1 = (uint32_t *)ctx->pv_alt.p;
    } else {
        k0 = (uint32_t *)ctx->pk_alt.p; v0 = (uint32_t *)ctx->pv_alt.p; k1 = out->tiles; v1 = out->vals;
    }
    if (!n_pairs) HIPCHECK(ctx, launch_fill_u32(s, k0, 0xFFFFFFFFu, sort_len));  // tail beyond the real count sorts last
    HIPCHECK(ctx, launch_emit(s, dk, dv, (const uint32_t *)ctx->offsets.p, (const uint32_t *)ctx->counts.p, proj->rec,
                              proj->rect, proj->flags, (const CamDev *)ctx->cams.p, n, V, (uint32_t)out->capacity,
                              p->tile_w, p->tile_h, p->sigma_k, k0, v0, ctx->status_dev));
    HIPCHECK(ctx, radix_sort(s, k0, v0, k1, v1, sort_len, 1, passes * 8, ctx->sort_ws.p));
    HIPCHECK(ctx, launch_ranges(s, out->tiles, ctx->npairs_dev, (uint32_t)out->capacity, sort_len, out->ranges));
    return FS_OK;
}

int fs_accumulate(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams, const uint8_t *masks,
                  int32_t n_classes, const fs_params *p, float *A_hi, float *A_lo, int32_t reduction,
                  const fs_pixel_out *pix)
{
    if (!ctx) return FS_ERR_ARG;
    int rc = check_params(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_proj(ctx, proj))) return rc;
    if (!bins || !bins->ranges) return set_err(ctx, FS_ERR_ARG, "bins is NULL");
    if ((rc = check_cams(ctx, cams, proj->n_views))) return rc;
    if (n_classes < 2 || n_classes > 256) return set_err(ctx, FS_ERR_ARG, "n_classes %d not in [2, 256]", n_classes);
    if (reduction < FS_RED_AUTO || reduction > FS_RED_LDS2SUM) return set_err(ctx, FS_ERR_ARG, "unknown reduction %d", reduction);
    if (reduction == FS_RED_AUTO) reduction = A_lo ? FS_RED_LDS2SUM : FS_RED_LDS;
    if (reduction == FS_RED_LDS2SUM && !A_lo) return set_err(ctx, FS_ERR_ARG, "FS_RED_LDS2SUM needs A_lo");
    if (proj->n > 0 && proj->n_views > 0 && (!masks || !A_hi)) return set_err(ctx, FS_ERR_ARG, "masks or A_hi is NULL");
    if (!finite_f(p->alpha_min)) return set_err(ctx, FS_ERR_ARG, "bad alpha_min");
    const int32_t V = proj->n_views;
    if (proj->n == 0 || V == 0) return FS_OK;
    uint64_t total_tiles = 0;
    if ((rc = build_cams(ctx, cams, V, p, &total_tiles, nullptr))) return rc;
    AccParams ap;
    const double LOG2E = 1.4426950408889634;
    ap.cut2 = (float)(-0.5 * (double)p->sigma_k * (double)p->sigma_k * LOG2E);
    ap.alpha_min = p->alpha_min;
    ap.alpha_max = p->alpha_max;
    ap.t_min = p->t_min;
    ap.E = n_classes;
    ap.tile_w = p->tile_w;
    ap.tile_h = p->tile_h;
    ap.reduction = reduction;
    const uint32_t *items = nullptr;
    if (p->tile_order == 0) {
        // longest lists first, so that the longest-running workgroups start early
        const size_t tb = (size_t)total_tiles * 4;
        if ((rc = ensure(ctx, ctx->items, tb)) || (rc = ensure(ctx, ctx->items_k, tb)) ||
            (rc = ensure(ctx, ctx->items_k2, tb)) || (rc = ensure(ctx, ctx->items_v2, tb)) ||
            (rc = ensure(ctx, ctx->items_ws, radix_ws_bytes((int64_t)total_tiles, 1))))
            return rc;
        ctx->items_tiles = 0;  // the XCD-run table (tile_order 2) shares the buffer
        HIPCHECK(ctx, launch_tile_keys(ctx->stream, bins->ranges, (int64_t)total_tiles, (uint32_t *)ctx->items_k.p,
                                       (uint32_t *)ctx->items.p));
        HIPCHECK(ctx, radix_sort(ctx->stream, (uint32_t *)ctx->items_k.p, (uint32_t *)ctx->items.p,
                                 (uint32_t *)ctx->items_k2.p, (uint32_t *)ctx->items_v2.p, (int64_t)total_tiles, 1, 16,
                                 ctx->items_ws.p));
        items = (const uint32_t *)ctx->items.p;
    } else if (p->tile_order == 2) {
        if ((rc = build_items(ctx, total_tiles))) return rc;
        items = (const uint32_t *)ctx->items.p;
    }
    HIPCHECK(ctx, launch_accumulate(ctx->stream, proj->rec, bins->vals, bins->ranges, (const CamDev *)ctx->cams.p, V,
                                    items, (uint32_t)total_tiles, proj->n, masks, ap, A_hi,
                                    reduction == FS_RED_LDS2SUM ? A_lo : nullptr, pix ? pix->t_final : nullptr,
                                    pix ? pix->n_blend : nullptr, ctx->status_dev));
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

}  // extern "C"
