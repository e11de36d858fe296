// Internal declarations shared by the library's translation units.
//
// Every call works on a set of views that may belong to several scenes. The
// host builds small device tables for it:
//   ViewDev   one per view: camera, tile numbering, where the view's
//             projection plane and mask live, and its scene;
//   SceneDev  one per scene: Gaussian arrays, masks, accumulators, classes;
//   ProjTask / SegDev  work lists of the projection and of the sorts.
// Element (v, g) of the projection planes lives at views[v].elem_off + g.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/flashsplat.h"

namespace fs {

struct GaussPtrs {
    const float *mx, *my, *mz, *qw, *qx, *qy, *qz, *sx, *sy, *sz, *op;
};

struct ViewDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    int32_t tiles_x, tiles_y;
    uint32_t tile_base;   // global id of this view's tile (0, 0)
    uint32_t scene;       // index into the scene table
    uint64_t mask_off;    // offset of this view's mask inside its scene's masks
    uint64_t elem_off;    // first element of this view's projection plane
    uint64_t pix_off;     // first pixel of this view in the call's per-pixel state buffer
    uint32_t n;           // Gaussians in the scene (= plane length)
    uint32_t pad;
    float limx, limy;     // guard-band limits of x/z, y/z: guard * ((0.5 W) / fx), likewise for y
};

struct SceneDev {
    GaussPtrs g;
    const uint8_t *masks;
    float *A_hi;
    float *A_lo;          // NULL: no compensation
    unsigned long long *A_fix;  // FS_RED_DET: the call's fixed-point sums [n][E] (else NULL)
    uint32_t n;
    int32_t E;
};

// FS_RED_DET: a partial x is added as the integer round(x * 2^kFixShift) (two's
// complement in 64 bits); integer addition is exact, so the totals do not
// depend on the order of the additions
constexpr int kFixShift = 34;

// projection work: blocks [blk0, blk0 + ceil(n/256)) project the Gaussians of
// `scene` into views [v0, v0 + nv) (all of that scene)
struct ProjTask {
    uint32_t blk0;
    uint32_t scene;
    uint32_t v0;
    uint32_t nv;
};

// radix-sort segment: elements [off, off + len), block tiles from blk0
// A segment of a radix sort: items [off, off + min(len, alen)); `len` (the
// planned capacity) fixes the segment's blocks, `alen` the items present.
// kbase is added to the key's count index (packed pair sort).
struct SegDev {
    uint64_t off;
    uint32_t len;
    uint32_t blk0;
    uint32_t alen;
    uint32_t kbase;
};

struct ProjParams {
    int32_t tile_w, tile_h;
    float sigma_k, lowpass, znear, guard, fp64_cond;
    int32_t fp64_conic;
    int32_t cshift;  // > 0: depth-sort values carry the listed-tile count (see packed_val)
};

// Depth-sort values. With cshift = 0 a value is the Gaussian id g. With
// cshift > 0 (ids below 2^cshift) it also carries the element's listed-tile
// count above the id, saturated at kCountSat(cshift), so that the count is
// read in sorted order with the value rather than gathered per element.
__host__ __device__ __forceinline__ uint32_t count_sat(int32_t cshift) { return 0xFFFFFFFFu >> cshift; }
__host__ __device__ __forceinline__ uint32_t packed_val(uint32_t g, uint32_t nt, int32_t cshift)
{
    if (cshift == 0) return g;
    const uint32_t c = nt < count_sat(cshift) ? nt : count_sat(cshift);
    return g | (c << cshift);
}
__host__ __device__ __forceinline__ uint32_t val_id(uint32_t v, int32_t cshift)
{
    return cshift == 0 ? v : (v & ((1u << cshift) - 1u));
}

// Device status block (ctx-owned): 64-bit counters, each striped over
// kStatusLanes words (indexed by the updating block) so that many blocks
// adding to one counter do not serialise on a single address; flags live in
// the first word of ST_FLAGS. The host sums the stripes.
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
    ST_PAIRS,       // tile pairs emitted
    ST_EVALS,
    ST_WSTEPS,      // list entries walked, summed over waves (diagnostic)
    ST_WSTEPS_MAX,  // per tile, the longest walk of its waves, summed over tiles (diagnostic)
    ST_STAGED,      // tile-list entries the compositing read (up to each tile's termination)
    ST_COUNT = 16
};

constexpr int kStatusLanes = 64;
constexpr int kStatusWords = ST_COUNT * kStatusLanes;

__device__ __forceinline__ void status_add(unsigned long long *status, int idx, unsigned long long v)
{
    atomicAdd(&status[idx * kStatusLanes + (blockIdx.x & (kStatusLanes - 1))], v);
}

__device__ __forceinline__ void status_flag(unsigned long long *status, unsigned long long bits)
{
    atomicOr(&status[ST_FLAGS * kStatusLanes], bits);
}

constexpr int kSortTile = 4096;  // items per radix-sort block tile
constexpr int kProjViews = 8;    // views projected per Gaussian load

// ---- launchers (all enqueue on `s`, return hipError_t) ----
hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t count);

// a1: projection of every task; optionally also writes the depth-sort keys
// (float bits of depth for elements that emit pairs, 0xFFFFFFFF otherwise) and
// values (Gaussian id within its scene) of every element, and (if `codes` is
// not NULL) every element's 32-byte emission record (span code and tile
// rectangle, fs_tiles.h), four u64 per element.
hipError_t launch_project(hipStream_t s, const ProjTask *tasks, int32_t n_tasks, uint32_t n_blocks,
                          const SceneDev *scenes, const ViewDev *views, const ProjParams &p, float *rec,
                          int16_t *rect, int32_t *ntiles, uint8_t *flags, uint32_t *dkeys, uint32_t *dvals,
                          uint64_t *codes, unsigned long long *status);

// depth-sort keys from existing projection planes (same rule as above)
hipError_t launch_depth_keys(hipStream_t s, const float *rec, const int32_t *ntiles, const uint8_t *flags,
                             const ViewDev *views, int32_t n_views, int64_t total, uint32_t *keys, uint32_t *vals);

// Stable LSD radix sort of (key, val) u32 pairs over segments, on bits
// [0, bits) in 8-bit passes; len_dev (optional, single-segment sorts only)
// caps the length on the device. A block sorts `tpb` block tiles of
// kSortTile items; n_blocks and the segments' blk0 count such blocks. After
// an even number of passes the result is in (keys, vals), after an odd number
// in (keys_alt, vals_alt). key_count (optional, zeroed by the caller, one u32
// per key value) receives the number of items of each key; with
// last_keys = false the last pass writes the values only.
size_t radix_ws_bytes(uint32_t n_blocks);
hipError_t radix_sort(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                      const SegDev *segs, int32_t n_segs, uint32_t n_blocks, int32_t bits, void *ws,
                      const uint32_t *len_dev, int32_t tpb, uint32_t *key_count = nullptr, bool last_keys = true);
// block tiles per block for a single-segment sort of n_items
int32_t radix_tiles_per_block(uint64_t n_items);

// Packed pair sort: items = (local tile << gbits) | Gaussian id, one segment
// per view (segs[j].kbase = the view's first tile id). Stable sort by the
// tbits tile bits (one or two passes); the last pass writes the Gaussian ids
// to ids_out and adds every tile's item count to key_count[kbase + tile]
// (zeroed by the caller). items_alt: scratch of the same size; ws as in
// radix_sort.
hipError_t radix_sort_packed(hipStream_t s, uint32_t *items, uint32_t *items_alt, uint32_t *ids_out,
                             const SegDev *segs, int32_t n_segs, uint32_t n_blocks, int32_t gbits, int32_t tbits,
                             void *ws, int32_t tpb, uint32_t *key_count);

// Per-view segments of the pairs emitted this run: segs[j].off/alen from the
// device offsets (pairs beyond the planned capacity segs[j].len, or beyond
// `capacity`, are dropped and latched); len, blk0 and kbase stay as planned.
hipError_t launch_pair_segs(hipStream_t s, const uint32_t *offsets, const ViewDev *views, int32_t n_views,
                            int64_t total_elems, const uint32_t *total_pairs, uint32_t capacity, SegDev *segs,
                            unsigned long long *status);

// Exclusive scan of u32 -> u32 (device-wide), total written to *total_out.
size_t scan_ws_bytes(int64_t n);
hipError_t scan_exclusive(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_out, void *ws);

// counts[i] = ntiles of depth-sorted element i (0 if its key is the sentinel);
// cshift: how the values are packed (ProjParams)
hipError_t launch_gather_counts(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                                const int32_t *ntiles, const ViewDev *views, int32_t n_views, int64_t total,
                                uint32_t *counts, int32_t cshift = 0);

// Depth slab [lo, hi) of a view holding n Gaussians, as fractions num/1024 of its
// depth-sorted elements: ranks [(n*num_lo) >> 10, (n*num_hi) >> 10).
struct Slab {
    uint32_t num_lo, num_hi;
};

// counts[i] = listed tiles of depth-sorted element i that lie in the slab and
// whose tile is not marked in `done` (NULL: no tile is done); 0 outside the slab.
// `flags` may be NULL when float64 conics are on: rec's float64 mark then
// gives the degenerate flag, and one gather per element is saved. `codes` as
// for launch_emit.
hipError_t launch_slab_counts(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                              const float *rec, const int16_t *rect, const uint8_t *flags, const int32_t *ntiles,
                              const ViewDev *views, int32_t n_views, int64_t total, Slab slab, const uint8_t *done,
                              int32_t tile_w, int32_t tile_h, float sigma_k, const uint64_t *codes,
                              uint32_t *counts, int32_t cshift = 0);

// emits, for every depth-sorted element, one (tile, id) pair per listed tile
// (the row_span rule) at offsets[i]; pairs at or beyond `capacity` are
// dropped and latched
// (tiles marked in `done`, if not NULL, are skipped, as in launch_slab_counts;
// `flags` may be NULL as there). With gbits > 0 each pair is one packed item
// (tile index within its view << gbits) | Gaussian id in tiles_out, and
// vals_out is not used. `codes` (may be NULL) are the projection's emission
// records (span code and rectangle); elements with a code skip the row_span
// recomputation, and the rectangle is read from the record, not from `rect`.
hipError_t launch_emit(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                       const uint32_t *offsets, const uint32_t *counts, const float *rec, const int16_t *rect,
                       const uint8_t *flags, const ViewDev *views, int32_t n_views, int64_t total,
                       uint32_t capacity, int32_t tile_w, int32_t tile_h, float sigma_k, const uint8_t *done,
                       uint32_t *tiles_out, uint32_t *vals_out, unsigned long long *status, int32_t gbits = 0,
                       const uint64_t *codes = nullptr, int32_t cshift = 0);

// ranges[t] = [starts[t], starts[t] + counts[t]), or [0, 0) if counts[t] == 0
hipError_t launch_count_ranges(hipStream_t s, const uint32_t *counts, const uint32_t *starts, int64_t n_tiles,
                               uint32_t *ranges);

hipError_t launch_ranges(hipStream_t s, const uint32_t *tiles, const uint32_t *n_pairs_dev, uint32_t capacity,
                         int64_t n_pairs_max, uint32_t *ranges);



// Pair offsets at depth-slab boundaries: out[v * nb.n + b] = offsets at depth
// rank (n_v * nb.num[b]) >> 10 of view v (total_pairs past the last element).
struct SlabBounds {
    uint32_t n;
    uint32_t num[9];
};
hipError_t launch_slab_offsets(hipStream_t s, const uint32_t *offsets, const ViewDev *views, int32_t n_views,
                               int64_t total_elems, const uint32_t *total_pairs, SlabBounds nb, uint32_t *out);

// keys[t] = 65535 - min(list length of tile t, 65535), vals[t] = t
hipError_t launch_tile_keys(hipStream_t s, const uint32_t *ranges, int64_t n_tiles, uint32_t *keys, uint32_t *vals);

struct AccParams {
    float cut2;       // -0.5*k^2*log2(e): support bound on the log2-scaled power
    float alpha_min, alpha_max, t_min;
    float lmin;       // log2(alpha_min) (-inf for 0): alpha >= alpha_min as a bound on the power
    int32_t tile_w, tile_h;
    int32_t reduction;
    int32_t count;    // 1: count in-support evaluations and blends
    int32_t batch;    // most list entries staged per batch (32..256)
    int32_t persistent;  // 1: resident workgroups pull tiles from a device counter
};

// Resumable compositing (depth slabs): with `tstate` set, each pixel's
// transmittance is read from tstate[views[v].pix_off + y*W + x] (unless
// `first`, which starts from T = 1) and written back at the end, -1 marking a
// pixel whose compositing has ended; with `tile_done` set, tiles already marked
// are skipped and tiles left without a live pixel are marked.
// With p.persistent, `queue` (one u32 of device memory, cleared here by a fill
// kernel before the launch) hands out the items.
hipError_t launch_accumulate(hipStream_t s, const float *rec, const uint32_t *vals, const uint32_t *ranges,
                             const ViewDev *views, int32_t n_views, const SceneDev *scenes, const uint32_t *items,
                             uint32_t n_items, const AccParams &p, float *t_final, int32_t *n_blend,
                             float *tstate, uint8_t *tile_done, int32_t first, unsigned long long *status,
                             uint32_t *queue);

// FS_RED_DET: adds the fixed-point totals fix[i] (i < count) into A_hi (and A_lo),
// once per entry, in a fixed order of operations
hipError_t launch_fix_finish(hipStream_t s, const unsigned long long *fix, float *A_hi, float *A_lo, int64_t count);

hipError_t launch_assign(hipStream_t s, const float *A_hi, const float *A_lo, int64_t n, int32_t E, float gamma,
                         uint8_t *S, float *margin, unsigned long long *status);

// novel-view masks (fs_render.hip); memb is workspace of
// render_member_bytes(n, E, mode) bytes (one byte per group of objects and
// Gaussian, rebuilt from S by the launch)
hipError_t launch_render(hipStream_t s, const float *rec, const uint32_t *vals, const uint32_t *ranges,
                         const ViewDev *views, int32_t n_views, uint32_t n_tiles, const uint8_t *S, int64_t n,
                         int32_t E, const AccParams &p, float tau, int32_t mode, uint8_t *labels, float *rho,
                         float *depth, int64_t n_pixels, uint8_t *memb);
int64_t render_member_bytes(int64_t n, int32_t E, int32_t mode);

// per-Gaussian diagnostics (fs_diag.hip): histograms [E+1] and overlap [E][3],
// zeroed by the caller
constexpr int kMaxDiagE = 256;
hipError_t launch_diag_rows(hipStream_t s, const float *A_hi, const float *A_lo, const uint8_t *S, const int32_t *gt,
                            int64_t n, int32_t E, double rel_eps, unsigned long long *contrib,
                            unsigned long long *member, unsigned long long *overlap);

// point-prompt propagation (fs_prompt.hip). prompts: device [n_prompts][3]
// (px, py, depth); part: n_prompts * n_part_blocks * k keys; per prompt
// out_ids = [chosen, k nearest], out_uv [n_views][2], out_vis [n_views]
int prompt_max_k();
hipError_t launch_prompt(hipStream_t s, const GaussPtrs &g, int64_t n, const ViewDev *views, int32_t n_views,
                         const ViewDev &ref_host, const float *prompts, int32_t n_prompts, int32_t k, float znear,
                         unsigned long long *part, int32_t n_part_blocks, long long *out_ids, float *out_uv,
                         uint8_t *out_vis);

// gamma sweep and stream compaction (fs_select.hip)
int sweep_max_gammas(int32_t E);
hipError_t launch_assign_sweep(hipStream_t s, const float *A_hi, const float *A_lo, int64_t n, int32_t E,
                               const float *gammas_dev, int32_t n_gamma, uint8_t *S, unsigned long long *counts);
hipError_t launch_select_flags(hipStream_t s, const uint8_t *select, int64_t n, int32_t keep_selected, uint32_t *flags);
hipError_t launch_compact(hipStream_t s, const float *const in[11], float *const out[11], const uint32_t *flags,
                          const uint32_t *pos, int64_t n, int64_t *index_map);

// ---- device helpers ------------------------------------------------------
// View holding element i: the wave searches once (scalar) for its first
// lane's element, then each lane steps forward while its element lies beyond
// the view (a wave's 64 consecutive elements span few views).
__device__ __forceinline__ int find_view_of_elem(const ViewDev *__restrict__ views, int32_t n_views, int64_t i)
{
    const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)(i & 0xFFFFFFFFll));
    const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)i >> 32));
    const int64_t i0 = (int64_t)(((uint64_t)hi32 << 32) | lo32);
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)views[mid].elem_off <= i0) lo = mid; else hi = mid - 1;
    }
    int v = lo;
    while (v + 1 < n_views && (int64_t)views[v + 1].elem_off <= i) ++v;
    return v;
}

// View holding global tile id t (views ordered by tile_base).
__device__ __forceinline__ int find_view_of_tile(const ViewDev *__restrict__ views, int32_t n_views, uint32_t t)
{
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace fs
