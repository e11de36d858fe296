// Host build of the binning's tile-listing rule (the same header the GPU
// kernels include), so that a CPU test can compare it with the oracle's
// pixel-by-pixel definition on many splats. Test infrastructure only.
#include "fs_tiles.h"

extern "C" void tr_row_spans(int64_t n, const float *mean2d, const float *cov, const uint8_t *flags,
                             const int32_t *rect, int32_t tw, int32_t th, int32_t W, int32_t H, float k,
                             int32_t max_rows, int32_t *out)
{
    for (int64_t g = 0; g < n; ++g) {
        const float a = cov[3 * g], b = cov[3 * g + 1], c = cov[3 * g + 2];
        const bool full = (flags[g] & 2u) != 0;
        float p = 0.f, r = 0.f, s = 0.f;
        if (!full) fs::ldl32(a, b, c, p, r, s);
        const fs::Span32 sp = fs::make_span32(mean2d[2 * g], mean2d[2 * g + 1], p, r, s, full, fs::support_limit(k));
        for (int i = 0; i < max_rows; ++i) {
            const int ty = rect[4 * g + 1] + i;
            int l = -1, r = -1;
            if (ty > rect[4 * g + 3] || !fs::row_span(sp, ty, rect[4 * g], rect[4 * g + 2], tw, th, W, H, l, r)) {
                l = -1;
                r = -1;
            }
            out[(g * max_rows + i) * 2] = l;
            out[(g * max_rows + i) * 2 + 1] = r;
        }
    }
}
