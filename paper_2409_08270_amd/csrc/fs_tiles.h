// Tile-overlap rule of the binning (strict binary32, no contraction).
//
// A tile can hold a pixel centre inside a Gaussian's support ellipse
// q(d) = A dx^2 + 2B dx dy + C dy^2 <= k^2 (A, B, C = the float32 conic
// c/det, -b/det, a/det) only if the minimum of q over the bounding box of
// its pixel centres is <= k^2. The minimum is zero when the mean is inside
// the box and otherwise the least of the four edge minima, each at the
// clamped vertex of a 1D parabola; the vertex offsets use the reciprocals
// 1/A and 1/C, rounded once per Gaussian. A tile passes when the minimum is
// <= k^2 (1 + 2^-9), a margin far above the rounding of a float32 conic that
// passed the conditioning predicate, so no pixel inside the support is lost.
// In each tile row the listed tiles are the span from the first to the last
// passing tile (the ellipse meets a row in a convex set), found by scanning in
// from both ends. Splats whose conic was inverted in float64 list their whole
// rectangle. The count (fs_project) and the emission (fs_bin_sort) share this
// code, so they agree exactly.
#pragma once

#include <hip/hip_runtime.h>

namespace fs {

struct Conic32 {
    float u, v, A, B, C, iA, iC;
    bool full;
};

__device__ __forceinline__ Conic32 make_conic32(float u, float v, float A, float B, float C, bool full)
{
#pragma clang fp contract(off)
    Conic32 q;
    q.u = u; q.v = v; q.A = A; q.B = B; q.C = C;
    q.full = full;
    q.iA = full ? 0.0f : 1.0f / A;
    q.iC = full ? 0.0f : 1.0f / C;
    return q;
}

__device__ __forceinline__ bool tile_hit(const Conic32 &q, int tx, int ty, int tw, int th, int W, int H, float lim)
{
#pragma clang fp contract(off)
    int x1 = tx * tw + tw - 1, y1 = ty * th + th - 1;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    const float xl = ((float)(tx * tw) + 0.5f) - q.u, xh = ((float)x1 + 0.5f) - q.u;
    const float yl = ((float)(ty * th) + 0.5f) - q.v, yh = ((float)y1 + 0.5f) - q.v;
    if (xl <= 0.0f && xh >= 0.0f && yl <= 0.0f && yh >= 0.0f) return true;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float x = i ? xh : xl;
        const float y = fminf(fmaxf(-(q.B * x) * q.iC, yl), yh);
        const float e = (q.A * x) * x + (2.0f * (q.B * x)) * y + (q.C * y) * y;
        if (e <= lim) return true;
        const float y2 = i ? yh : yl;
        const float x2 = fminf(fmaxf(-(q.B * y2) * q.iA, xl), xh);
        const float e2 = (q.A * x2) * x2 + (2.0f * (q.B * x2)) * y2 + (q.C * y2) * y2;
        if (e2 <= lim) return true;
    }
    return false;
}

// k2lim = (k * k) * (1 + 2^-9), computed once by the caller in binary32
__device__ __forceinline__ float support_limit(float k)
{
#pragma clang fp contract(off)
    return (k * k) * 1.001953125f;
}

// listed span [l, r] of tile row ty within columns [x0, x1]; false if empty
__device__ __forceinline__ bool row_span(const Conic32 &q, int ty, int x0, int x1, int tw, int th, int W, int H,
                                         float lim, int &l, int &r)
{
    if (q.full) {
        l = x0;
        r = x1;
        return true;
    }
    int a = x0;
    while (a <= x1 && !tile_hit(q, a, ty, tw, th, W, H, lim)) ++a;
    if (a > x1) return false;
    int b = x1;
    while (b > a && !tile_hit(q, b, ty, tw, th, W, H, lim)) --b;
    l = a;
    r = b;
    return true;
}

}  // namespace fs
