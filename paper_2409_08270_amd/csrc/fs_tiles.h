// Tile-listing rule of the binning (strict binary32, no contraction).
//
// The support of a splat is the ellipse q(d) = A dx^2 + 2B dx dy + C dy^2 <= L
// (A, B, C = the float32 conic c/det, -b/det, a/det; L = k^2 (1 + 2^-7), a
// margin far above the rounding of a float32 conic that passed the
// conditioning predicate, so no pixel inside the support k^2 is lost).
//
// A tile row covers the pixel-centre rows y in [y0, y1] (offsets from the
// mean). The ellipse meets that band in a convex set whose x-extent is found
// in closed form: with dt = AC - B^2, the ellipse spans |y| <= ye = sqrt(LA/dt),
// its left-most point (-xe, yx) has xe = sqrt(LC/dt), yx = B xe / C, and its
// right-most point is (xe, -yx). At height y the ellipse spans
// x = (-By -/+ sqrt(AL - dt y^2)) / A; the left edge is convex in y, the right
// edge concave, so over the band the minimum of x is -xe when yx lies in the
// band and the left edge at the band end nearest yx otherwise (likewise for
// the maximum). The listed tiles of the row are those holding a pixel-centre
// column inside [Xmin, Xmax], within the image and the splat's tile
// rectangle. Splats whose conic was inverted in float64 list their whole
// rectangle. Per row this is O(1) work; the count (fs_project) and the
// emission (fs_bin_sort) share this code, so they agree exactly. Small splats
// hand their spans from the count to the emission as a span code (below).
#pragma once

#include <hip/hip_runtime.h>

namespace fs {

struct Span32 {
    float u, v, A, B, dt, lim, xe, ye, yx;
    bool full;
};

// k2lim = (k * k) * (1 + 2^-7)
__device__ __forceinline__ float support_limit(float k)
{
#pragma clang fp contract(off)
    return (k * k) * 1.0078125f;
}

__device__ __forceinline__ Span32 make_span32(float u, float v, float A, float B, float C, bool full, float lim)
{
#pragma clang fp contract(off)
    Span32 s;
    s.u = u; s.v = v; s.A = A; s.B = B;
    s.full = full;
    s.lim = lim;
    s.dt = full ? 1.0f : A * C - B * B;
    s.xe = full ? 0.0f : sqrtf((lim * C) / s.dt);
    s.ye = full ? 0.0f : sqrtf((lim * A) / s.dt);
    s.yx = full ? 0.0f : (B * s.xe) / C;
    return s;
}

// x of the ellipse boundary at height y: left (sgn = -1) or right (sgn = +1)
__device__ __forceinline__ float edge_x(const Span32 &s, float y, float sgn)
{
#pragma clang fp contract(off)
    const float r = sqrtf(fmaxf((s.A * s.lim) - (s.dt * y) * y, 0.0f));
    return (-(s.B * y) + sgn * r) / s.A;
}

// n / t for n >= 0: a shift when the tile size t is a power of two (t is the
// same for every lane, so the choice costs one uniform branch)
__device__ __forceinline__ int tile_of(int n, int t)
{
    return (t & (t - 1)) == 0 ? (n >> (__ffs(t) - 1)) : n / t;
}

// listed span [l, r] of tile row ty within tile columns [x0, x1]; false if empty
__device__ __forceinline__ bool row_span(const Span32 &s, int ty, int x0, int x1, int tw, int th, int W, int H,
                                         int &l, int &r)
{
#pragma clang fp contract(off)
    if (s.full) {
        l = x0;
        r = x1;
        return true;
    }
    int j1 = ty * th + th - 1;
    if (j1 > H - 1) j1 = H - 1;
    const float y0 = ((float)(ty * th) + 0.5f) - s.v;
    const float y1 = ((float)j1 + 0.5f) - s.v;
    const float lo = fmaxf(y0, -s.ye), hi = fminf(y1, s.ye);
    if (!(lo <= hi)) return false;
    const float yl = s.yx, yr = -s.yx;
    const float xmin = (yl >= lo && yl <= hi) ? -s.xe : edge_x(s, yl < lo ? lo : hi, -1.0f);
    const float xmax = (yr >= lo && yr <= hi) ? s.xe : edge_x(s, yr < lo ? lo : hi, 1.0f);
    // pixel-centre columns k with k + 0.5 - u in [xmin, xmax], clamped to the image
    const float kl = fmaxf(ceilf((s.u + xmin) - 0.5f), 0.0f);
    const float kr = fminf(floorf((s.u + xmax) - 0.5f), (float)(W - 1));
    if (!(kl <= kr)) return false;
    int a = tile_of((int)kl, tw), b = tile_of((int)kr, tw);
    if (a < x0) a = x0;
    if (b > x1) b = x1;
    if (a > b) return false;
    l = a;
    r = b;
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

__device__ __forceinline__ SpanCode load_code(const ulonglong2 *codes, int64_t idx)
{
    if (codes == nullptr) return no_code();
    const ulonglong2 q = codes[idx];
    return SpanCode{q.x, q.y};
}

}  // namespace fs
