// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/flashsplat.h"

namespace fs {

// Camera as the kernels see it (one per view of a call).
struct CamDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    int32_t tiles_x, tiles_y;
    uint32_t tile_base;   // first global tile id of this view
    uint32_t pad;
    uint64_t mask_off;    // offset of this view's mask in the concatenated masks
};

struct ProjParams {
    int32_t tile_w, tile_h;
    float sigma_k, lowpass, znear, guard, fp64_cond;
    int32_t fp64_conic;
};

struct GaussPtrs {
    const float *mx, *my, *mz, *qw, *qx, *qy, *qz, *sx, *sy, *sz, *op;
};

// Device status block (ctx-owned): counters are 64-bit, flags in word 0.
enum StatusIdx {
    ST_FLAGS = 0,
    ST_BAD_LABELS,
    ST_INVALID,
    ST_FP64,
    ST_DROPPED,
    ST_BLENDS,
    ST_UNSEEN,
    ST_MULTI,
    ST_LOWMARGIN,
    ST_PAIRS,       // total pairs of the last bin_sort (device-side count)
    ST_EVALS,
    ST_WSTEPS,      // list entries walked, summed over waves (diagnostic)
    ST_WSTEPS_MAX,  // per tile, the longest walk of its waves, summed over tiles (diagnostic)
    ST_COUNT = 16
};

// ---- launchers (all enqueue on `s`, return hipError_t) ----
hipError_t launch_project(hipStream_t s, const GaussPtrs &g, int64_t n, const CamDev *cams_dev,
                          int32_t n_views, const ProjParams &p, float *rec, int16_t *rect,
                          int32_t *ntiles, uint8_t *flags, unsigned long long *status);

hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t count);

// depth keys for the per-view depth sort: key = float bits of depth for
// Gaussians that emit at least one pair, 0xFFFFFFFF otherwise; val = id.
hipError_t launch_depth_keys(hipStream_t s, const float *rec, const int32_t *ntiles,
                             const uint8_t *flags, int64_t n, int32_t n_views,
                             uint32_t *keys, uint32_t *vals);

// Stable LSD radix sort of (key, val) u32 pairs over `segs` equal segments of
// `seg_len` items, sorting on bits [0, bits). Result in (keys, vals); the
// alt buffers are scratch of the same size. Workspace from radix_ws_bytes.
size_t radix_ws_bytes(int64_t seg_len, int32_t segs);
hipError_t radix_sort(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                      uint32_t *vals_alt, int64_t seg_len, int32_t segs, int32_t bits, void *ws);

// Exclusive scan of u32 -> u32 (device-wide), total written to *total_out.
size_t scan_ws_bytes(int64_t n);
hipError_t scan_exclusive(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n,
                          uint32_t *total_out, void *ws);

// counts[v*n + s] = ntiles of the s-th depth-sorted Gaussian of view v (0 if key invalid)
hipError_t launch_gather_counts(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                                const int32_t *ntiles, int64_t n, int32_t n_views, uint32_t *counts);

// emits, for every depth-sorted item, one (tile, id) pair per tile that passes
// tile_hit, at offsets[i]; pairs at or beyond `capacity` are dropped and latched
hipError_t launch_emit(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                       const uint32_t *offsets, const uint32_t *counts, const float *rec, const int16_t *rect,
                       const uint8_t *flags, const CamDev *cams_dev, int64_t n, int32_t n_views, uint32_t capacity,
                       int32_t tile_w, int32_t tile_h, float sigma_k, uint32_t *tiles_out, uint32_t *vals_out,
                       unsigned long long *status);

// keys[t] = 65535 - min(list length of tile t, 65535), vals[t] = t
hipError_t launch_tile_keys(hipStream_t s, const uint32_t *ranges, int64_t n_tiles, uint32_t *keys, uint32_t *vals);

hipError_t launch_ranges(hipStream_t s, const uint32_t *tiles, const uint32_t *n_pairs_dev,
                         uint32_t capacity, int64_t n_pairs_max, uint32_t *ranges);

struct AccParams {
    float cut2;       // -0.5*k^2*log2(e): support bound on the log2-scaled power
    float alpha_min, alpha_max, t_min;
    int32_t E;
    int32_t tile_w, tile_h;
    int32_t reduction;
};

hipError_t launch_accumulate(hipStream_t s, const float *rec, const uint32_t *vals,
                             const uint32_t *ranges, const CamDev *cams_dev, int32_t n_views,
                             const uint32_t *item_view, uint32_t n_items, int64_t n,
                             const uint8_t *masks, const AccParams &p, float *A_hi, float *A_lo,
                             float *t_final, int32_t *n_blend, unsigned long long *status);

hipError_t launch_assign(hipStream_t s, const float *A_hi, const float *A_lo, int64_t n, int32_t E,
                         float gamma, uint8_t *S, float *margin, unsigned long long *status);

}  // namespace fs
