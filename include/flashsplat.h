/*
 * flashsplat.h -- C ABI of the MI355X (gfx950) splat-and-accumulate library.
 *
 * The library lifts per-view 2D label masks onto a reconstructed 3D Gaussian
 * Splatting scene as described in "FlashSplat: 2D to 3D Gaussian Splatting
 * Segmentation Solved Optimally" (Shen, Yang, Wang, ECCV 2024):
 *
 *   fs_project     3D Gaussians -> 2D Gaussians per view (Sec. 3.1)
 *   fs_bin_sort    16x16 tile lists in depth order (Sec. 3.1)
 *   fs_accumulate  front-to-back alpha compositing (Eq. (1)); every weight
 *                  w = alpha*T is added into A[g][label(pixel)]
 *                  (Eq. (7), Eq. (8), Listing 1 of the supplement)
 *   fs_assign      closed-form, L1-normalised, background-biased argmax per
 *                  object (Sec. 3.2 "Regularized ILP", Eq. (8), Listing 1 of the supplement)
 *
 * Conventions shared by all calls
 *  - Memory: every array argument documented as "device" is device memory
 *    owned by the caller; the library never frees or retains it past the
 *    call's completion on the stream. Arguments documented as "host" are read
 *    during the call only. The library owns only its context workspace.
 *  - Asynchrony: calls enqueue work on the context's stream and return
 *    without waiting, except fs_status_get, fs_bin_sort with a non-NULL
 *    n_pairs argument, and fs_batch_* planning calls, which synchronise the
 *    stream.
 *  - Errors: every call returns FS_OK (0) or a negative FS_ERR_* code and
 *    throws nothing. Argument errors are detected before any work is
 *    enqueued. Conditions found on the device (a mask label >= n_classes, an
 *    overflowing pair buffer, invalid Gaussian parameters) are latched in the
 *    context's status word and reported by fs_status_get.
 *  - Threads: one context per host thread; a context is not thread-safe.
 *  - Layout: Gaussians are structure-of-arrays float32 with post-activation
 *    values (linear scales, opacity in [0,1]); quaternions are (w,x,y,z) and
 *    need not be normalised. Cameras map world to camera with OpenCV axes
 *    (x right, y down, z forward); pixel (row j, column k) is sampled at
 *    (k + 0.5, j + 0.5). Masks are uint8, row-major [H][W] per view, views
 *    concatenated; label 0 is background.
 */
#ifndef FLASHSPLAT_H
#define FLASHSPLAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FS_OK 0
#define FS_ERR_ARG (-1)      /* invalid argument (null pointer, bad size or range) */
#define FS_ERR_ALLOC (-2)    /* device or host allocation failed */
#define FS_ERR_HIP (-3)      /* a HIP runtime call failed */
#define FS_ERR_CAPACITY (-4) /* output buffer too small; required size reported */
#define FS_ERR_DEVICE (-5)   /* a condition latched on the device (see fs_status) */
#define FS_ERR_STATE (-6)    /* call not valid in the current state */

/* status bits latched on the device */
#define FS_DEV_BAD_LABEL 1u      /* a mask pixel had label >= n_classes (pixel skipped) */
#define FS_DEV_PAIR_OVERFLOW 2u  /* more tile pairs than the bins capacity (excess dropped) */
#define FS_DEV_INVALID_GAUSS 4u  /* a Gaussian had non-finite values, a zero quaternion or a
                                    non-positive scale (culled) */
#define FS_DEV_MANY_LABELS 8u    /* a tile held more than 64 distinct labels (the pre-reduction
                                    slots); that tile used per-pixel atomics (informational) */

/* reduction strategies of fs_accumulate */
#define FS_RED_AUTO 0   /* library choice (currently FS_RED_LDS2SUM when A_lo != NULL, else FS_RED_LDS) */
#define FS_RED_PLAIN 1  /* one global atomic per contributing (pixel, Gaussian) */
#define FS_RED_LDS 2    /* per-tile pre-reduction over the tile's pixels, one atomic per (tile, Gaussian, label) */
#define FS_RED_LDS2SUM 3 /* as FS_RED_LDS, plus the rounding error of each atomic (exact two-sum) into A_lo */
#define FS_RED_DET 4     /* bit-reproducible: as FS_RED_LDS, with every label summed across the wave and each
                            partial rounded to a 64-bit fixed-point integer (units of 2^-34) and added exactly;
                            the call's totals then go into A_hi (and A_lo) once per entry */

typedef struct fs_ctx fs_ctx;

/* Gaussians G_i = {m_i, q_i, s_i, o_i} (Sec. 3.1; the colour c_i is not used,
 * Sec. 4.2). device float32 arrays of length n. */
typedef struct {
    const float *mx, *my, *mz;       /* mean, world frame */
    const float *qw, *qx, *qy, *qz;  /* rotation quaternion */
    const float *sx, *sy, *sz;       /* linear scales (> 0) */
    const float *opacity;            /* in [0, 1] */
    int64_t n;
} fs_gaussians;

/* One pinhole view (Sec. 3.2: "L rendered views with associated masks").
 * host memory. R is row-major world->camera rotation, t its translation. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} fs_camera;

/* Rasterisation constants. The paper inherits them from the 3DGS renderer
 * without stating values; fs_params_default gives 3DGS-like ones. */
typedef struct {
    int32_t tile_w, tile_h;  /* tile size in pixels; fs_accumulate needs tile_w*tile_h == 256
                                with tile_w in {8, 16, 32} (default 16x16, Sec. 3.1) */
    float sigma_k;           /* support: pixels with Mahalanobis distance <= sigma_k (3) */
    float lowpass;           /* added to the 2D covariance diagonal, px^2 (0.3) */
    float znear;             /* Gaussians with camera depth <= znear are not visible (0.2) */
    float guard;             /* Jacobian clamp, as a multiple of the half field of view (1.3) */
    float alpha_min;         /* smaller alphas are skipped (1/255) */
    float alpha_max;         /* alphas are clamped to this (0.99) */
    float t_min;             /* compositing stops before T would fall below this (1e-4) */
    float fp64_cond;         /* a splat whose float32 2D covariance has a*c >= fp64_cond*det
                                (or det <= 0) gets its conic inverted in float64 (64) */
    int32_t fp64_conic;      /* 1 (default): use the float64 inversion for such splats */
    int32_t tile_order;      /* fs_accumulate work order: 0 (default) longest tile list first;
                                1 = image order; 2 = each of the chip's 8 XCDs (each with its
                                own L2) gets a contiguous run of tiles */
    int32_t count_ops;       /* 1 (default): compositing counts its in-support evaluations and
                                blends into the status (fs_status_get); 0 leaves those two
                                counters alone and saves two instructions per pixel step
                                (A, S and every other output are the same either way) */
    int32_t persistent;      /* compositing launch: 0 (default) one workgroup per tile; 1 as many
                                workgroups as the chip holds at once, each taking the next tile of
                                the work order from a device counter until none is left */
    int32_t lds_batch;       /* most tile-list entries staged in LDS per compositing batch:
                                32, 64, 128 or 256 (0 = default 256); tiles with more than 8
                                labels stage fewer (128, 64, 32 for 16, 32, 64 labels) */
} fs_params;

/* Projected Gaussians, caller-owned device buffers, one plane per view:
 * element (v, g) lives at index v*n + g. */
typedef struct {
    float *rec;       /* float32 [n_views][n][8]: u, v (pixel), p, r, s, opacity, depth
                         (camera z), mark. (p, r, s) are the LDL^T factors of the inverse
                         2D covariance (a, b, c): p = c/det, r = -b/c, s = 1/c, so that
                         d^T Sigma^-1 d = p (dx + r dy)^2 + s dy^2. mark: 0 = float32
                         factors, tiles listed by the support test; 1 = factors from the
                         float64 inversion, whole rectangle listed; 2 = float32 factors,
                         whole rectangle listed (fp64_conic = 0) */
    int16_t *rect;    /* int16 [n_views][n][4]: tile rectangle x0, y0, x1, y1, inclusive */
    int32_t *ntiles;  /* int32 [n_views][n]: tiles in the rectangle, 0 if not visible */
    uint8_t *flags;   /* uint8 [n_views][n]: bit0 visible, bit1 float64 conic, bit2 invalid input */
    int64_t n;
    int32_t n_views;
} fs_proj;

/* Tile lists. Tiles of the views of one call are numbered globally: view v's
 * tile (tx, ty) has id tile_base(v) + ty*tiles_x(v) + tx, where tile_base is
 * the running sum of tiles_x*tiles_y over the earlier views. */
typedef struct {
    uint32_t *vals;    /* device uint32 [capacity]: Gaussian ids, ordered by (tile, depth, id) */
    uint32_t *tiles;   /* device uint32 [capacity]: tile id of each entry */
    uint32_t *ranges;  /* device uint32 [total tiles][2]: [start, end) into vals; [0,0) if empty */
    int64_t capacity;  /* entries available in vals / tiles */
} fs_bins;

/* Optional per-pixel outputs of fs_accumulate, device, views concatenated
 * like the masks; either pointer may be NULL. */
typedef struct {
    float *t_final;    /* float32: transmittance after the last blended Gaussian */
    int32_t *n_blend;  /* int32: number of Gaussians blended into the pixel */
} fs_pixel_out;

typedef struct {
    uint32_t flags;          /* FS_DEV_* bits latched since the last clear */
    int64_t bad_labels;      /* pixels skipped for label >= n_classes */
    int64_t invalid_gauss;   /* (Gaussian, view) pairs culled for invalid input */
    int64_t fp64_splats;     /* (Gaussian, view) pairs inverted in float64 */
    int64_t pairs_dropped;   /* tile pairs beyond capacity */
    int64_t blends;          /* (pixel, Gaussian) weights added into A */
    int64_t evaluated;       /* (pixel, Gaussian) pairs with the pixel inside the Gaussian's support,
                                evaluated before the pixel's compositing ended */
    int64_t wave_steps;      /* diagnostic: list entries walked by the compositing waves, summed */
    int64_t wave_steps_max;  /* diagnostic: per tile, the longest walk of its waves, summed over tiles */
    int64_t unseen;          /* fs_assign: rows of A that are all zero */
    int64_t multi_member;    /* fs_assign: Gaussians assigned to more than one object */
    int64_t low_margin;      /* fs_assign: (object, Gaussian) entries with margin < 1e-4 */
    int64_t pairs_emitted;   /* tile pairs written by fs_bin_sort and the batched solve */
    int64_t entries_staged;  /* tile-list entries the compositing read, each tile's list up to the
                                batch in which its last pixel finished */
} fs_status;

/* Library and context ---------------------------------------------------- */
const char *fs_version(void);
const char *fs_error_string(int code);
void fs_params_default(fs_params *p);   /* 16x16, k=3, 0.3, 0.2, 1.3, 1/255, 0.99, 1e-4, 64, fp64 on */
void fs_params_exact(fs_params *p);     /* as default but alpha_min=0, alpha_max=1, t_min=0 */

/* Creates a context on the current HIP device that enqueues on `stream`
 * (a hipStream_t; NULL = the null stream). */
int fs_ctx_create(fs_ctx **out, void *stream);
int fs_ctx_set_stream(fs_ctx *ctx, void *stream);
int fs_ctx_destroy(fs_ctx *ctx);
/* Message describing the last error returned on this context ("" if none). */
const char *fs_ctx_last_error(fs_ctx *ctx);
/* Synchronises the stream, copies the latched status and counters to *out
 * (host), and clears them if `clear` is non-zero. Returns FS_ERR_DEVICE if
 * any error bit (not FS_DEV_MANY_LABELS) was set. */
int fs_status_get(fs_ctx *ctx, fs_status *out, int32_t clear);

/* Duration in ms of the last compositing kernel that fs_accumulate launched on
 * this context, from HIP events recorded on the context's stream right before
 * and after that launch (the work-order sort and the host's checks are
 * outside). Waits for the launch to finish. FS_ERR_ARG if no fs_accumulate
 * call has been timed (calls made under stream capture are not). */
int fs_last_accumulate_ms(fs_ctx *ctx, float *ms);

/* a1: projection (Sec. 3.1; EWA splatting of 3DGS, which the paper's renderer
 * inherits). For every view v in cams[0..n_views) and Gaussian g: camera-space
 * mean, 2D covariance J W Sigma3 W^T J^T + lowpass*I, its inverse (conic),
 * pixel mean, depth, the per-axis half extents rx = ceil(sigma_k*sqrt(cov_xx)),
 * ry = ceil(sigma_k*sqrt(cov_yy)) of the support ellipse (its exact bounding
 * box, rounded up to whole pixels) and the tile rectangle of the pixel box
 * mean +- (rx, ry). ntiles counts the listed tiles: in each tile row of the
 * rectangle, the tiles from the first to the last that hold a pixel centre
 * (inside the image) with p (dx + r dy)^2 + s dy^2 <= sigma_k^2 (1 + 2^-7),
 * evaluated in binary32 in the order written; splats selected by fp64_cond
 * list their whole rectangle. Visibility, rectangle and ntiles are computed in
 * strict binary32 in a fixed operation order (the bit-exact contract); the
 * conic factors are float32 (det by Kahan's fused two-product form) except for
 * splats selected by fp64_cond, which are inverted in float64 (Cauchy-Binet
 * determinant) and then rounded. cams: host [n_views];
 * out: caller-owned planes for n_views x g->n elements. */
int fs_project(fs_ctx *ctx, const fs_gaussians *g, const fs_camera *cams, int32_t n_views,
               const fs_params *p, const fs_proj *out);

/* a2-a5: count, scan, emit, sort, ranges (Sec. 3.1: the pixels of a 16x16
 * tile share one subset of Gaussians, blended in depth order). Emits one
 * entry per (visible Gaussian, overlapped tile), ordered by tile, then depth,
 * then Gaussian id (ties), and the [start, end) range of every tile.
 * n_pairs: if non-NULL, the call synchronises, writes the exact number of
 * entries to *n_pairs (host) and returns FS_ERR_CAPACITY without touching
 * `out` when it exceeds out->capacity; if NULL the call stays asynchronous
 * and entries beyond capacity are dropped and latched (FS_DEV_PAIR_OVERFLOW).
 * cams: host [proj->n_views] (the same views as fs_project). */
int fs_bin_sort(fs_ctx *ctx, const fs_proj *proj, const fs_camera *cams, const fs_params *p,
                const fs_bins *out, int64_t *n_pairs);

/* a6: compositing and accumulation (Eq. (1), Eq. (7)-(8), Listing 1 of the supplement).
 * For every pixel of every view, front to back over its tile's list:
 * alpha = min(alpha_max, o*exp(-d^T conic d / 2)) for pixels within the
 * support; Gaussians with alpha < alpha_min are skipped; compositing stops
 * before the Gaussian after which T would drop below t_min; otherwise
 * A[g][label(pixel)] += alpha*T and T *= 1 - alpha.
 * masks: device uint8, views concatenated, each [H][W]. A_hi: device float32
 * [n][n_classes], ADDED INTO (the caller zeroes it once; views may be
 * processed over any number of calls). A_lo: same shape, or NULL; with
 * FS_RED_LDS2SUM it receives the exact rounding error of every addition into
 * A_hi, and the partial sums of labels that no 8x8 pixel block of a tile holds
 * in 4 or more pixels (stray, noise-like labels), which are small; the
 * accumulated result is A_hi + A_lo.
 * FS_RED_DET: the call's weights are summed exactly as 64-bit fixed-point
 * integers in units of 2^-34 (each wave's float sum per (Gaussian, label) is
 * rounded once to that grid, about 3e-11), in a context workspace of
 * n * n_classes * 8 bytes; the totals are then added into A_hi (with A_lo:
 * by an exact two-sum, the error into A_lo) once per entry. A_hi and A_lo
 * come out bit-identical on every run and for every tile_order and
 * persistent setting. Such a call covers at most 2^29 pixels in total
 * (FS_ERR_ARG beyond).
 * n_classes in [2, 256]. pix: optional per-pixel outputs, or NULL. */
int fs_accumulate(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                  const uint8_t *masks, int32_t n_classes, const fs_params *p,
                  float *A_hi, float *A_lo, int32_t reduction, const fs_pixel_out *pix);

/* fs_accumulate for callers that cannot allocate memory: code recorded under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as fs_accumulate; the call itself
 * allocates nothing (no hipMalloc, hipFree or host allocation). Its device
 * workspace (the call's view table, the longest-list-first work order and
 * that order's sort workspace) is one static array of about 17.5 MB per GPU
 * (each GPU the library runs on holds it until the process ends); its host
 * tables go through pinned memory that fs_ctx_create reserves.
 * Limits: at most FS_NOALLOC_MAX_VIEWS views and FS_NOALLOC_MAX_TILES tiles
 * per call; larger calls return FS_ERR_CAPACITY before any work is enqueued.
 * FS_RED_DET, whose workspace grows with n, returns FS_ERR_ARG here.
 * All calls on one GPU share the array: calls that overlap in time on that
 * GPU (other contexts, other streams) race and must be serialised by the
 * caller. A call may wait on the host for the table copy of the context's
 * previous call to finish. */
#define FS_NOALLOC_MAX_VIEWS 4096
#define FS_NOALLOC_MAX_TILES 1048576
int fs_accumulate_noalloc(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                          const uint8_t *masks, int32_t n_classes, const fs_params *p,
                          float *A_hi, float *A_lo, int32_t reduction, const fs_pixel_out *pix);

/* a7: assignment (Sec. 3.2 Eq. (7) and "Regularized ILP"; Sec. 3.3 Eq. (8);
 * Listing 1 of the supplement). For every Gaussian g and object t:
 * a = A[g][t], o = sum_{e != t} A[g][e], formed as the row total minus a
 * (as Listing 1 does; the row total is summed once per Gaussian in float64
 * from A_hi + A_lo, so o is exact to about 1e-16 of the row sum and is
 * clamped at 0), (o_n, a_n) = (o, a) / max(o + a, 1e-12);
 * S[t][g] = a_n > o_n + gamma (ties go to "others"); margin[t][g] =
 * |a_n - o_n - gamma|. Sums are formed in float64 from A_hi + A_lo.
 * A_hi, A_lo (A_lo may be NULL): device float32 [n][n_classes].
 * S: device uint8 [n_classes][n]; margin: device float32 [n_classes][n] or NULL.
 * gamma: finite, in [-1, 1]. */
int fs_assign(fs_ctx *ctx, const float *A_hi, const float *A_lo, int64_t n, int32_t n_classes,
              float gamma, uint8_t *S, float *margin);

/* Interactive follow-ups of the assignment ---------------------------------
 * Once A is known the background bias can be adjusted interactively (Sec. 3.2
 * "Regularized ILP for Noise Reduction", Sec. 4.2), and the Gaussians of an
 * object extracted or removed from the scene (Sec. 4.4 "Object Removal"). */

/* Labels for several biases from one read of A: for k < n_gamma, S[k][t][g]
 * is fs_assign's S[t][g] with gamma = gammas[k].
 * gammas: host float [n_gamma], each finite in [-1, 1]; n_gamma in
 *   [1, min(64, 4096 / n_classes)].
 * S: device uint8 [n_gamma][n_classes][n], or NULL to count only.
 * counts: host int64 [n_gamma][n_classes] (members of each object for each
 *   bias), or NULL; when non-NULL the call synchronises the stream. */
int fs_assign_sweep(fs_ctx *ctx, const float *A_hi, const float *A_lo, int64_t n, int32_t n_classes,
                    const float *gammas, int32_t n_gamma, uint8_t *S, int64_t *counts);

/* Stream compaction of the Gaussians: keeps, in their original order, the
 * Gaussians g with (select[g] != 0) == (keep_selected != 0), i.e. an object's
 * Gaussians (keep_selected = 1, extraction) or the rest of the scene
 * (keep_selected = 0, removal), given select = one row S[t] of fs_assign.
 * in: device arrays of in->n Gaussians. out: device arrays with room for
 * out->n Gaussians (FS_ERR_CAPACITY, with *n_out set, if more are kept).
 * select: device uint8 [in->n]. index_map: device int64 [out->n] receiving the
 * source index of every kept Gaussian, or NULL. n_out: host; the call
 * synchronises the stream to read it. */
int fs_compact(fs_ctx *ctx, const fs_gaussians *in, const uint8_t *select, int32_t keep_selected,
               const fs_gaussians *out, int64_t *index_map, int64_t *n_out);

/* Novel-view masks (Sec. 3.4 "Depth-guided Novel View Mask Rendering"; the
 * supplement's "Quantization in novel view mask"). For every object e the
 * Gaussians with S[e][g] != 0 are composited on their own with the rules of
 * fs_accumulate, giving its alpha mask rho_e = sum alpha*T and its depth
 * D_e = sum alpha*T*z / rho_e (z: camera-space depth of the mean). The label
 * of a pixel is
 *   mode FS_MASK_DEPTH: the object e >= 1 with rho_e > tau and least D_e
 *                       (0 if there is none; ties go to the smaller e);
 *   mode FS_MASK_ARGMAX: argmax over every e >= 0 of rho_e (first maximum).
 * proj, bins: fs_project / fs_bin_sort of the rendered views (256-pixel tiles
 * as for fs_accumulate). S: device uint8 [n_classes][n], e.g. fs_assign's
 * output. labels: device uint8, the views' pixels concatenated [H][W] each.
 * rho, depth: device float32 [n_classes][pixels of all views], or NULL
 * (entries for objects that are not rendered are left untouched; depth is
 * 3e38 where rho_e = 0). tau: finite. The context keeps n bytes of
 * workspace per 8 rendered objects (each Gaussian's membership bits, built
 * from S at the start of the call). */
#define FS_MASK_DEPTH 0
#define FS_MASK_ARGMAX 1
int fs_render_masks(fs_ctx *ctx, const fs_proj *proj, const fs_bins *bins, const fs_camera *cams,
                    const uint8_t *S, int32_t n_classes, const fs_params *p, float tau, int32_t mode,
                    uint8_t *labels, float *rho, float *depth);

/* Per-Gaussian diagnostics of a solved scene: the number of objects each
 * Gaussian contributes to (the supplement's "Scene segmentation extension"
 * counts it to show that Gaussians are shared between objects), how many
 * objects' subsets each Gaussian falls in (more than one only for a negative
 * bias, Sec. 3.3), and the overlap of every subset with given per-Gaussian
 * labels (the fewer-masks ablation of Sec. 4.8 reads it as an IoU).
 * A_hi, A_lo: device float [n][n_classes] as fs_accumulate leaves them
 *   (A_lo may be NULL); A_hi NULL skips contrib_hist.
 * S: device uint8 [n_classes][n] (fs_assign's layout); NULL skips
 *   member_hist and overlap.
 * gt: device int32 [n], a label per Gaussian (values outside
 *   [0, n_classes) belong to no object); NULL skips overlap.
 * rel_eps: finite, in [0, 1). Object e counts for Gaussian g when
 *   a > rel_eps * t, a = (double)A_hi + (double)A_lo and t the row's sum of
 *   those values taken in order e = 0, 1, ... in binary64 (0: A > 0).
 * Outputs (host, overwritten; each may be NULL):
 *   contrib_hist uint64 [n_classes + 1]: Gaussians per count of such objects
 *     (unseen Gaussians count 0);
 *   member_hist  uint64 [n_classes + 1]: Gaussians per number of rows of S
 *     that hold them;
 *   overlap      uint64 [n_classes][3]: |S_e and gt = e|, |S_e|, |gt = e|.
 * Synchronous. n_classes in [2, 256]. */
int fs_diagnose(fs_ctx *ctx, const float *A_hi, const float *A_lo, const uint8_t *S, const int32_t *gt, int64_t n,
                int32_t n_classes, float rel_eps, uint64_t *contrib_hist, uint64_t *member_hist,
                uint64_t *overlap);

/* Point-prompt propagation (Sec. 4.1 "2D mask generation and association";
 * the supplement's "Binary Mask Association"). Each prompt (px, py, depth)
 * is a pixel of view ref_view and a camera depth there (for instance the
 * depth fs_render_masks renders at that pixel with every Gaussian in one
 * object). It is back-projected to the world point
 * R^T (depth * K^-1 [px, py, 1] - t); the k Gaussian centres nearest to that
 * point are found (squared L2 distance in binary32, ties to the smaller
 * index); among them the one of least positive depth in the reference view is
 * chosen (ties to the smaller index; -1 if none lies in front of it), and its
 * centre is projected into every view.
 * g: device Gaussians (n < 2^32 - 1). cams: host [n_views], n_views >= 1.
 * prompts: host float [n_prompts][3], finite, depth > 0; n_prompts in
 * [0, 65535]. k in [1, 32] (the paper uses 10).
 * Outputs, all host memory, written whole:
 *   chosen  int64 [n_prompts]: the chosen Gaussian or -1;
 *   nearest int64 [n_prompts][k] by increasing distance (-1 past n), or NULL;
 *   uv      float [n_prompts][n_views][2], the prompt carried to each view
 *           (0 where the chosen centre is not beyond p->znear in that view);
 *   visible uint8 [n_prompts][n_views], 1 where that projection lies beyond
 *           p->znear and inside the image ([0, W) x [0, H)).
 * Synchronous: returns after the outputs are on the host. */
int fs_prompt_propagate(fs_ctx *ctx, const fs_gaussians *g, const fs_camera *cams, int32_t n_views,
                        int32_t ref_view, const float *prompts, int32_t n_prompts, int32_t k, const fs_params *p,
                        int64_t *chosen, int64_t *nearest, float *uv, uint8_t *visible);

/* Batched solve ------------------------------------------------------------
 * Many scenes of uneven size, all their views, in one graph launch: the
 * splat-and-accumulate pass is a sum over views (Eq. (7)), so views of all
 * scenes are projected, binned and composited together, in chunks that fit a
 * bounded workspace, and every scene's assignment follows (Eq. (8)).
 * fs_batch_create plans the work (one exact counting pass and one read-back of
 * the per-view pair counts), allocates the workspace and captures the whole
 * solve into a hipGraph; fs_batch_run replays it on the context's stream.
 * The buffers named in the scene descriptors are borrowed: they must stay
 * valid and keep their addresses until fs_batch_destroy. If the inputs change
 * so that a chunk needs more pairs than planned, the excess is dropped and
 * FS_DEV_PAIR_OVERFLOW is latched; create a new batch then. */
typedef struct fs_batch fs_batch;

typedef struct {
    fs_gaussians gauss;        /* device */
    const fs_camera *cams;     /* host [n_views] (copied at creation) */
    int32_t n_views;
    const uint8_t *masks;      /* device, this scene's views concatenated */
    int32_t n_classes;         /* [2, 256] */
    float *A_hi;               /* device float32 [n][n_classes] */
    float *A_lo;               /* device float32 [n][n_classes], or NULL */
    uint8_t *S;                /* device uint8 [n_classes][n], or NULL to skip the assignment */
    float *margin;             /* device float32 [n_classes][n], or NULL */
    float gamma;               /* background bias in [-1, 1] */
} fs_scene;

typedef struct {
    int64_t pair_budget;       /* max tile pairs per chunk (0: 2^28) */
    int64_t elem_budget;       /* max (Gaussian, view) elements per chunk (0: 2^26) */
    int32_t zero_accumulators; /* 1: each run starts from A = 0 (default 1) */
    int32_t use_graph;         /* 1 (default): capture into a hipGraph; 0: enqueue the kernels per run */
    int32_t reduction;         /* FS_RED_* for the compositing (default FS_RED_AUTO); FS_RED_DET keeps
                                  n * n_classes 64-bit totals per scene in the batch workspace, adds
                                  them into A after every view of the run (the same bits for any
                                  lanes, chunking, depth_slabs or tile_order) and takes at most 2^29
                                  pixels per scene */
    int32_t depth_slabs;       /* 1..4: the Gaussians of each view are binned and composited in this
                                  many depth slabs, front to back, and tiles whose pixels have all
                                  finished get no pairs from later slabs; 0 (default): 1, one pass
                                  over the full lists */
    int32_t lanes;             /* 1..4 workspaces, each with its own stream: the views are split into
                                  at least this many chunks, which take the lanes in turn, so that
                                  one chunk's binning overlaps another's compositing (each lane
                                  holds its own workspace); 0 (default): 2 */
} fs_batch_opts;

typedef struct {
    int32_t n_chunks;
    int32_t n_views;
    int64_t pairs;             /* tile pairs planned, all chunks */
    int64_t pair_capacity;     /* pair slots of the workspace (largest chunk plus slack) */
    int64_t elements;          /* (Gaussian, view) elements, all chunks */
    int64_t tiles;             /* tiles, all chunks */
    int64_t workspace_bytes;   /* device memory held by the batch */
} fs_batch_info;

void fs_batch_opts_default(fs_batch_opts *o);
int fs_batch_create(fs_ctx *ctx, const fs_scene *scenes, int32_t n_scenes, const fs_params *p,
                    const fs_batch_opts *opts, fs_batch **out);
int fs_batch_run(fs_batch *b);
int fs_batch_get_info(fs_batch *b, fs_batch_info *out);
int fs_batch_destroy(fs_batch *b);

/* Measurement: total duration in ms of the compositing launches (Eq. (1),
 * Eq. (7)-(8)) of the last fs_batch_run of a batch created with
 * use_graph = 0, from HIP events recorded on each lane's stream right before
 * and after every launch; *n_launches receives their number. Waits for the
 * run to finish. FS_ERR_STATE for a graph batch or before a run. */
int fs_batch_accumulate_ms(fs_batch *b, float *total_ms, int32_t *n_launches);

/* Inspection of the tile lists (Sec. 3.1) that the batched solve builds for
 * chunk `chunk` (0 <= chunk < n_chunks; batches with depth_slabs = 1): the
 * chunk's projection, depth sort, pair emission, pair sort and ranges are
 * re-run on the context's stream with the kernels and workspace of
 * fs_batch_run, without compositing, and copied out. vals: device uint32
 * [vals_cap], the Gaussian ids (within their scene) of every tile list, lists
 * in tile order; ranges: device uint32 [ranges_cap][2], every tile's
 * [start, end) into vals ([0, 0) when empty), tiles numbered view by view in
 * chunk order, row-major within a view; view_refs: host int32
 * [refs_cap][2], (scene, view) of the chunk's views in order. With vals,
 * ranges or view_refs NULL only *info is filled. Synchronises the stream;
 * FS_ERR_CAPACITY if an output is too small. */
typedef struct {
    int32_t n_views;
    int32_t packed;            /* 1: the chunk sorts packed (tile, Gaussian) words per view */
    int64_t n_tiles;
    int64_t n_pairs;
} fs_chunk_info;
int fs_batch_chunk_lists(fs_batch *b, int32_t chunk, uint32_t *vals, int64_t vals_cap, uint32_t *ranges,
                         int64_t ranges_cap, int32_t *view_refs, int32_t refs_cap, fs_chunk_info *info);

#ifdef __cplusplus
}
#endif
#endif /* FLASHSPLAT_H */
