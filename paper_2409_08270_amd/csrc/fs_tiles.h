// Tile-listing rule of the binning.
//
// Conic form. A splat's inverse 2D covariance is kept as its LDL^T factors:
// with the covariance (a, b, c) and det = ac - b^2,
//     q(dx, dy) = p (dx + r dy)^2 + s dy^2,  p = c/det, r = -b/c, s = 1/c,
// which equals (c dx^2 - 2b dx dy + a dy^2)/det. Both terms are non-negative,
// so evaluating q does not cancel, even for needle-like splats. On the float32
// path det comes from Kahan's two-product form (fused multiply-adds), and
// p, r, s are correctly rounded quotients.
//
// Definition (strict binary32, every operation as written). A pixel centre
// (row j, column k) is in the listing support of a splat with mean (u, v) iff
//     dx = (k + 0.5) - u,  dy = (j + 0.5) - v,  e = dx + (r dy),
//     q  = (p e) e + (s dy) dy  <=  L = k^2 (1 + 2^-7).
// The margin 2^-7 lies far above the rounding of q, so no pixel of the
// compositing support (q <= k^2) is missed. Each tile row of the splat's tile
// rectangle lists the tiles from the first to the last one holding a pixel
// centre (inside the image) that passes. Splats that fail the conditioning
// predicate list their whole rectangle.
//
// How it is found in O(boundary) work rather than by testing every pixel.
// The ellipse q <= Lo with Lo slightly above L bounds, in real arithmetic,
// every centre that can pass in binary32 (the relative rounding of q is at
// most about 8 u (1 + sqrt(AC/dt)), u = 2^-24). With A = p, B = pr,
// C = s + pr^2 and dt = AC - B^2 = ps, the ellipse spans |y| <= ye =
// sqrt(Lo A/dt), its left-most point (-xe, yx) has xe = sqrt(Lo C/dt),
// yx = B xe / C, its right-most point is (xe, -yx), and at height y it spans
// x = -ry -/+ sqrt((Lo - s y^2)/p); the left edge is convex in y, the right
// edge concave, so over the band of the tile row's centre rows the least x is
// -xe when yx lies in the band and the left edge at the band end nearer yx
// otherwise (likewise for the greatest x). Those bounds, widened by the
// rounding of this approximate arithmetic, give the candidate columns. Columns are then walked inward from each end; in a column only the
// rows of the chord of the Lo ellipse (widened the same way) can pass, and
// each of those centres is decided by the definition's own test. So the
// listed set is the definition's exactly; the approximations only choose
// which centres to test.
//
// Most walks are skipped. The inner ellipse q <= Li = L (1 - rq), shrunk by
// the same margins, holds only centres whose binary32 q is surely <= L; on
// the band row nearest the ellipse's left-most point its chord gives a column
// that surely holds a passing centre. The first passing column lies between
// the candidate bound and that column, so when both fall in one tile the
// row's first listed tile is known without a test (likewise on the right).
// When those rows hold none, the band row nearest the centre (the widest
// chord) is tried. A walk remains only where a tile boundary falls between
// the two, or where the band holds no surely passing centre (the very top
// and bottom of the ellipse). The count (fs_project) and the emission
// (fs_bin_sort) call the same code on the same record, so they agree. Small
// splats hand their spans from the count to the emission as a span code.
//
// The functions are host-callable too, so that the rule can be checked
// against a brute-force listing on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

// approximate square root and reciprocal (about 1 ulp on the device); they
// only bound which centres are tested, never decide one
__host__ __device__ __forceinline__ float approx_sqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

__host__ __device__ __forceinline__ float approx_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

struct Span32 {
    float u, v, p, r, s, lim;  // the definition's inputs
    float lo, B, C, dt, iC, xe, ye, yx, mx, my;  // candidate bounds (approximate, widened; A = p)
    float li;  // inner level L (1 - rq): centres with exact q <= li pass in binary32
    float ip;  // approximate 1 / p
    bool full, ok;
};

// LDL^T factors (p, r, s) of the inverse of the 2D covariance (a, b, c), float32
// path: det by Kahan's two-product form, then correctly rounded quotients
__host__ __device__ __forceinline__ void ldl32(float a, float b, float c, float &p, float &r, float &s)
{
#pragma clang fp contract(off)
    const float w = b * b;
    const float err = fmaf(-b, b, w);  // w - b^2, exactly
    float det = fmaf(a, c, -w) + err;
    if (!(det > 0.0f)) det = 1e-30f;
    p = c / det;
    r = -b / c;
    s = 1.0f / c;
}

// L = (k * k) * (1 + 2^-7)
__host__ __device__ __forceinline__ float support_limit(float k)
{
#pragma clang fp contract(off)
    return (k * k) * 1.0078125f;
}

// the definition's test of pixel centre (row j, column k)
__host__ __device__ __forceinline__ bool support_pass(const Span32 &sp, int k, int j)
{
#pragma clang fp contract(off)
    const float dx = ((float)k + 0.5f) - sp.u;
    const float dy = ((float)j + 0.5f) - sp.v;
    const float e = dx + (sp.r * dy);
    const float q = ((sp.p * e) * e) + ((sp.s * dy) * dy);
    return q <= sp.lim;
}

__host__ __device__ __forceinline__ Span32 make_span32(float u, float v, float p, float r, float s, bool full,
                                                       float lim)
{
    Span32 sp;
    sp.u = u; sp.v = v; sp.p = p; sp.r = r; sp.s = s; sp.lim = lim;
    sp.full = full;
    sp.ok = false;
    sp.lo = sp.B = sp.C = sp.dt = sp.iC = sp.xe = sp.ye = sp.yx = sp.mx = sp.my = sp.li = sp.ip = 0.0f;
    if (full) return sp;
    sp.B = p * r;
    sp.C = s + sp.B * r;
    sp.dt = p * s;
    // conditioning AC / dt = 1 + p r^2 / s >= 1: scales the rounding of q and of
    // the cancellations in the chord and edge formulas
    const float kap = fmaxf(sp.C * approx_rcp(s), 1.0f);
    const float rq = 0x1p-8f + 0x1p-17f * kap;              // bound on the relative rounding of q, widened
    const float rc = approx_sqrt(0x1p-15f * (kap + 2.0f));  // relative error of the chord and edge half-widths
    sp.lo = lim * (1.0f + rq);
    sp.li = lim * (1.0f - rq);
    sp.iC = approx_rcp(sp.C);
    sp.ip = approx_rcp(p);
    const float iD = approx_rcp(sp.dt);
    sp.xe = approx_sqrt((sp.lo * sp.C) * iD);
    sp.ye = approx_sqrt((sp.lo * p) * iD);
    sp.yx = (sp.B * sp.xe) * sp.iC;
    // margins of the approximate bounds: the relative error of the half-widths
    // (rc; cancellation near an end of a chord costs at most sqrt(3u) of the
    // extent) and the absolute rounding of sums of coordinates, a few ulp of
    // |u| + xe (|v| + ye); the offsets of the rows and columns themselves are
    // the definition's own binary32 values, so they carry no error here
    sp.mx = 0x1p-6f + sp.xe * rc + 0x1p-20f * (fabsf(u) + sp.xe);
    sp.my = 0x1p-6f + sp.ye * rc + 0x1p-20f * (fabsf(v) + sp.ye);
    sp.ok = p > 0.0f && s > 0.0f && rc < 0.25f && __builtin_isfinite(sp.xe) && __builtin_isfinite(sp.ye) &&
            __builtin_isfinite(sp.yx) && __builtin_isfinite(sp.iC) && __builtin_isfinite(sp.B);
    return sp;
}

// x of the widened ellipse's boundary at offset y: left (sgn = -1) or right (+1)
__host__ __device__ __forceinline__ float edge_x(const Span32 &sp, float y, float sgn)
{
    const float h = approx_sqrt(fmaxf((sp.lo - (sp.s * y) * y) * sp.ip, 0.0f));
    return -(sp.r * y) + sgn * h;
}

// float bound -> integer index, clamped to [lo, hi] (NaN -> lo)
__host__ __device__ __forceinline__ int clamp_index(float x, int lo, int hi)
{
    if (!(x >= (float)lo)) return lo;
    if (!(x <= (float)hi)) return hi;
    return (int)x;
}

// Does column k hold a passing centre in pixel rows [j0, j1]?
__host__ __device__ __forceinline__ bool column_hit(const Span32 &sp, int k, int j0, int j1)
{
    int a = j0, b = j1;
    if (sp.ok) {
        const float dx = ((float)k + 0.5f) - sp.u;
        const float clo = sp.C * sp.lo;
        const float hh = clo - (sp.dt * dx) * dx;
        // least q over the column is dt dx^2 / C: clearly above Lo, no row can
        // pass (dt = ps has no cancellation, so dt dx^2 is within a few ulp)
        if (hh < -0x1p-9f * clo) return false;
        const float yc = -(sp.B * dx) * sp.iC;
        const float hy = approx_sqrt(fmaxf(hh, 0.0f)) * sp.iC;
        // rows j whose offset j + 0.5 - v lies in [yc - hy - my, yc + hy + my]
        const float ylo = ((sp.v + yc) - hy) - 0.5f - sp.my;
        const float yhi = ((sp.v + yc) + hy) - 0.5f + sp.my;
        a = clamp_index(ceilf(ylo), j0, j1 + 1);
        b = clamp_index(floorf(yhi), j0 - 1, j1);
    }
    for (int j = a; j <= b; ++j)
        if (support_pass(sp, k, j)) return true;
    return false;
}

// Columns [ka, kb] of pixel row j whose centres lie inside the inner ellipse
// q <= li, shrunk by the edge margin: each of them passes the definition's
// test in binary32. False if the shrunk chord holds no column centre.
__host__ __device__ __forceinline__ bool sure_columns(const Span32 &sp, int j, int &ka, int &kb)
{
    const float y = ((float)j + 0.5f) - sp.v;
    const float h = approx_sqrt(fmaxf((sp.li - (sp.s * y) * y) * sp.ip, 0.0f));
    const float xc = sp.u - (sp.r * y);
    const float lo = ((xc - h) - 0.5f) + sp.mx;
    const float hi = ((xc + h) - 0.5f) - sp.mx;
    if (!(lo <= hi) || !(lo > -1.0e9f) || !(hi < 1.0e9f)) return false;
    ka = (int)ceilf(lo);
    kb = (int)floorf(hi);
    return ka <= kb;
}

// n / t for n >= 0: a shift when the tile size t is a power of two (t is the
// same for every lane, so the choice costs one uniform branch)
__host__ __device__ __forceinline__ int tile_of(int n, int t)
{
    return (t & (t - 1)) == 0 ? (n >> __builtin_ctz((unsigned)t)) : n / t;
}

// listed span [l, r] of tile row ty within tile columns [x0, x1]; false if empty
__host__ __device__ __forceinline__ bool row_span(const Span32 &sp, int ty, int x0, int x1, int tw, int th, int W,
                                                  int H, int &l, int &r)
{
    if (sp.full) {
        l = x0;
        r = x1;
        return true;
    }
    const int j0 = ty * th;
    const int j1 = min(j0 + th, H) - 1;
    const int k0 = x0 * tw;
    const int k1 = min((x1 + 1) * tw, W) - 1;
    if (j0 > j1 || k0 > k1) return false;
    int cl = k0, cr = k1;
    if (sp.ok) {
        // offsets of the band's centre rows, clipped to the ellipse's y-extent
        const float y0 = ((float)j0 + 0.5f) - sp.v;
        const float y1 = ((float)j1 + 0.5f) - sp.v;
        if (y0 > sp.ye + sp.my || y1 < -sp.ye - sp.my) return false;
        float lo = fmaxf(y0, -sp.ye), hi = fminf(y1, sp.ye);
        if (lo > hi) lo = hi = y0 > 0.0f ? sp.ye : -sp.ye;  // band beyond the extent, within the margin
        const float yl = sp.yx, yr = -sp.yx;
        const float xmin = (yl >= lo && yl <= hi) ? -sp.xe : edge_x(sp, yl < lo ? lo : hi, -1.0f);
        const float xmax = (yr >= lo && yr <= hi) ? sp.xe : edge_x(sp, yr < lo ? lo : hi, 1.0f);
        // centre columns k with k + 0.5 - u in [xmin - mx, xmax + mx]
        cl = clamp_index(ceilf(((sp.u + xmin) - 0.5f) - sp.mx), k0, k1 + 1);
        cr = clamp_index(floorf(((sp.u + xmax) - 0.5f) + sp.mx), k0 - 1, k1);
    }
    if (sp.ok && cl <= cr) {
        // a surely passing column near each end, on the band row nearest the
        // ellipse's left-most (right-most) point
        int la, lb, ra, rb, sl = 0, sr = -1;
        const int jl = clamp_index(floorf(sp.v + sp.yx), j0, j1);
        const int jr = clamp_index(floorf(sp.v - sp.yx), j0, j1);
        if (sure_columns(sp, jl, la, lb) && sure_columns(sp, jr, ra, rb) && max(la, k0) <= min(lb, k1) &&
            max(ra, k0) <= min(rb, k1)) {
            sl = max(la, k0);
            sr = min(rb, k1);
        } else {
            // the band row nearest the ellipse's centre, where its chord is widest
            const int jc = clamp_index(floorf(sp.v), j0, j1);
            if (sure_columns(sp, jc, la, lb)) {
                sl = max(la, k0);
                sr = min(lb, k1);
            }
        }
        if (sl <= sr) {
            // first passing column in [cl, sl], last in [sr, cr]
            int kl = cl;
            if (tile_of(cl, tw) != tile_of(sl, tw))
                while (kl < sl && !column_hit(sp, kl, j0, j1)) ++kl;
            int kr = cr;
            if (tile_of(cr, tw) != tile_of(sr, tw))
                while (kr > sr && !column_hit(sp, kr, j0, j1)) --kr;
            l = tile_of(kl, tw);
            r = tile_of(kr, tw);
            return true;
        }
    }
    int kl = cl;
    while (kl <= cr && !column_hit(sp, kl, j0, j1)) ++kl;
    if (kl > cr) return false;
    int kr = cr;
    while (kr > kl && !column_hit(sp, kr, j0, j1)) --kr;
    l = tile_of(kl, tw);
    r = tile_of(kr, tw);
    return true;
}

// Span codes. A splat whose tile rectangle has at most kSpanCodeRows rows and
// 16 columns keeps the spans the count found in 16 bytes: byte k describes row
// y0 + k as (l - x0) | (r - l) << 4, and 0xFF marks an empty (or absent) row;
// 0xFF is never a valid span there, since l - x0 = 15 forces r = l. Any other
// splat gets the code with every byte 0xFF (no_code) and its spans are
// recomputed with row_span; a splat whose rows are all empty has that code
// too, but it lists no tile.
constexpr int kSpanCodeRows = 16;

struct SpanCode {
    uint64_t lo, hi;  // rows 0-7, rows 8-15
};

__device__ __forceinline__ SpanCode no_code() { return SpanCode{~0ull, ~0ull}; }

__device__ __forceinline__ bool has_code(const SpanCode &c) { return (c.lo & c.hi) != ~0ull; }

__device__ __forceinline__ void code_set(SpanCode &c, int row, int l, int r, int x0)
{
    const uint64_t byte = (uint64_t)(uint32_t)(l - x0) | ((uint64_t)(uint32_t)(r - l) << 4);
    const uint32_t sh = 8u * (uint32_t)(row & 7);
    if (row < 8) c.lo = (c.lo & ~(0xFFull << sh)) | (byte << sh);
    else c.hi = (c.hi & ~(0xFFull << sh)) | (byte << sh);
}

__device__ __forceinline__ bool code_span(const SpanCode &c, int row, int x0, int &l, int &r)
{
    const uint32_t byte = (uint32_t)(((row < 8 ? c.lo : c.hi) >> (8u * (uint32_t)(row & 7))) & 0xFFull);
    if (byte == 0xFFu) return false;
    l = x0 + (int)(byte & 15u);
    r = l + (int)(byte >> 4);
    return true;
}

// The batch keeps, per element, a 32-byte emission record: the span code and
// the tile rectangle (x0, y0, x1, y1 as 16-bit fields), so that the emission's
// gather of an element touches one 32-byte block instead of two arrays.
__device__ __forceinline__ unsigned long long pack_rect(short4 rc)
{
    return (unsigned long long)(uint16_t)rc.x | ((unsigned long long)(uint16_t)rc.y << 16) |
           ((unsigned long long)(uint16_t)rc.z << 32) | ((unsigned long long)(uint16_t)rc.w << 48);
}

__device__ __forceinline__ short4 unpack_rect(unsigned long long v)
{
    return make_short4((short)(uint16_t)(v & 0xFFFFull), (short)(uint16_t)((v >> 16) & 0xFFFFull),
                       (short)(uint16_t)((v >> 32) & 0xFFFFull), (short)(uint16_t)(v >> 48));
}

__device__ __forceinline__ void store_emit_record(ulonglong2 *recs, int64_t idx, const SpanCode &c, short4 rc)
{
    recs[2 * idx] = make_ulonglong2(c.lo, c.hi);
    recs[2 * idx + 1] = make_ulonglong2(pack_rect(rc), 0ull);
}

// span code and rectangle of element idx: from the emission records when there
// are any (`recs`), else no code and the rectangle array
__device__ __forceinline__ void load_emit_record(const ulonglong2 *recs, const short4 *rect, int64_t idx,
                                                 SpanCode &code, short4 &rc)
{
    if (recs == nullptr) {
        code = no_code();
        rc = rect[idx];
        return;
    }
    const ulonglong2 a = recs[2 * idx];
    const ulonglong2 b = recs[2 * idx + 1];
    code = SpanCode{a.x, a.y};
    rc = unpack_rect(b.x);
}

}  // namespace fs
