/*
 * CPU oracle for the FlashSplat splat-and-accumulate pass.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call this code;
 * it exists so that tests, the smoke check and the CPU baseline of the bench
 * can compare the GPU library against a slow, plainly written reference.
 * It shares no source with the GPU library.
 *
 * What it computes (paper: Sec. 3.1 "Preliminary: Rasterization of 3DGS",
 * Eq. (1); Sec. 3.2 Eq. (7); Sec. 3.3 Eq. (8); Listing 1 of the supplement):
 *
 *   A[g][e] = sum over views v, pixels (j,k) with M^v[j][k] == e of
 *             alpha_g(v,j,k) * T_g(v,j,k)
 *
 * where alpha and T come from front-to-back alpha compositing of the
 * depth-sorted Gaussians that cover the pixel's 16x16 tile.
 *
 * Two precisions, deliberately separate:
 *  - or_project32 / or_bin: strict IEEE binary32 (compiled without FP
 *    contraction), the reference for the bit-exact binning contract
 *    (visibility, tile rectangle, per-tile order by (depth, id)).
 *  - or_project64 / or_composite64 / or_render64: binary64 for everything
 *    that is compared within a tolerance.
 *
 * Conventions the paper leaves open (rasterizer constants inherited from
 * 3DGS, pixel centres at +0.5, OpenCV camera axes, the Gaussian that would
 * push T below T_min is not added, elliptical support |d|_Sigma^2 <= k^2) are
 * passed in through the parameter block below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* parameter block, float32 [12]:
 *  0 tile_w  1 tile_h  2 sigma_k  3 lowpass  4 znear  5 guard
 *  6 alpha_min  7 alpha_max  8 t_min  9 fp64_cond  10 band_eps  11 unused */
enum { P_TW, P_TH, P_K, P_LP, P_ZN, P_GUARD, P_AMIN, P_AMAX, P_TMIN, P_COND, P_EPS };

/* camera row, float32 [18]: R (row-major 9), t (3), fx, fy, cx, cy, W, H */

/* ------------------------------------------------------------------------
 * Which tiles of a Gaussian's rectangle are listed: the plain definition,
 * evaluated pixel by pixel.
 *
 * The inverse 2D covariance is taken in its LDL^T form: with the float32
 * covariance (a, b, c) and det = ac - b^2 (Kahan's two-product form, fused
 * multiply-adds), p = c/det, r = -b/c, s = 1/c, and
 *   q(dx, dy) = p (dx + r dy)^2 + s dy^2 = (c dx^2 - 2b dx dy + a dy^2)/det.
 * A pixel centre (row j, column k) is in the listing support when, in strict
 * binary32 with each operation as written,
 *   dx = (k + 0.5) - u,  dy = (j + 0.5) - v,  e = dx + (r dy),
 *   q  = (p e) e + (s dy) dy  <=  L = k^2 (1 + 2^-7).
 * The margin 2^-7 keeps every centre of the compositing support (q <= k^2) in.
 * In each tile row of the rectangle, the listed tiles run from the first to
 * the last tile holding a passing centre inside the image. Splats that fail
 * the conditioning predicate (flag bit 1) list their whole rectangle.
 * Each pixel row of the tile row is walked from its left end to its first
 * passing centre and from its right end to its last one.
 * ---------------------------------------------------------------------- */
typedef struct { float u, v, p, r, s, L; int full; } supp32_t;

static supp32_t supp32(float u, float v, float a, float b, float c, uint8_t f, float k)
{
    supp32_t sp;
    sp.u = u; sp.v = v;
    sp.full = (f & 2) != 0;
    float w = b * b;
    float det = fmaf(a, c, -w) + fmaf(-b, b, w);
    if (!(det > 0.0f)) det = 1e-30f;
    sp.p = c / det; sp.r = -b / c; sp.s = 1.0f / c;
    sp.L = (k * k) * 1.0078125f;
    return sp;
}

static int supp_pass32(const supp32_t *sp, int k, int j)
{
    float dx = ((float)k + 0.5f) - sp->u;
    float dy = ((float)j + 0.5f) - sp->v;
    float e = dx + sp->r * dy;
    float q = (sp->p * e) * e + (sp->s * dy) * dy;
    return q <= sp->L;
}

/* listed tiles [*l, *r] of tile row ty within tile columns [x0, x1]; 0 if none */
static int row_listed32(const supp32_t *sp, int ty, int x0, int x1, int tw, int th, int W, int H, int *l, int *r)
{
    if (sp->full) { *l = x0; *r = x1; return 1; }
    int j0 = ty * th, j1 = ty * th + th - 1;
    int k0 = x0 * tw, k1 = x1 * tw + tw - 1;
    if (j1 > H - 1) j1 = H - 1;
    if (k1 > W - 1) k1 = W - 1;
    int kl = k1 + 1, kr = k0 - 1; /* first and last passing column so far */
    for (int j = j0; j <= j1; ++j) {
        for (int k = k0; k < kl; ++k)
            if (supp_pass32(sp, k, j)) { kl = k; break; }
        for (int k = k1; k > kr; --k)
            if (supp_pass32(sp, k, j)) { kr = k; break; }
    }
    if (kl > kr) return 0;
    *l = kl / tw; *r = kr / tw;
    return 1;
}

/* The listing of arbitrary splats given by mean, 2D covariance, flag and
 * tile rectangle (used to check the rule on shapes a scene rarely produces).
 * Per splat, up to max_rows tile rows from rect[1]: out [n][max_rows][2] =
 * (l, r), or (-1, -1) for a row that lists nothing. */
void or_listed_rows32(int64_t n, const float *mean2d, const float *cov, const uint8_t *flags, const int32_t *rect,
                      int32_t tw, int32_t th, int32_t W, int32_t H, float k, int32_t max_rows, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t g = 0; g < n; ++g) {
        supp32_t sp = supp32(mean2d[2 * g], mean2d[2 * g + 1], cov[3 * g], cov[3 * g + 1], cov[3 * g + 2], flags[g], k);
        for (int i = 0; i < max_rows; ++i) {
            int ty = rect[4 * g + 1] + i, l = -1, r = -1;
            if (ty > rect[4 * g + 3] || !row_listed32(&sp, ty, rect[4 * g + 0], rect[4 * g + 2], tw, th, W, H, &l, &r)) {
                l = -1;
                r = -1;
            }
            out[(g * max_rows + i) * 2] = l;
            out[(g * max_rows + i) * 2 + 1] = r;
        }
    }
}

/* ------------------------------------------------------------------------
 * Strict binary32 projection of one Gaussian into one view.
 * Follows EWA splatting as used by 3DGS (the paper's Sec. 3.1 projects each
 * 3D Gaussian to a 2D Gaussian (m2D, Sigma2D)); every operation is written
 * out in a fixed order so the GPU can reproduce it bit for bit.
 * Outputs: flags bit0 visible, bit1 fp64-conic predicate, bit2 culled for
 * invalid input; rect = tile rectangle [x0,y0,x1,y1] (inclusive) of the
 * support ellipse's pixel bounding box; ntiles = tiles of the rectangle that
 * row_listed32 lists; depth; cov = (a, b, c) of the 2D covariance incl. low-pass.
 * ---------------------------------------------------------------------- */
static void proj32_one(const float *gin /*11*/, const float *cam, const float *prm,
                       uint8_t *flags, int32_t *rect, int32_t *ntiles, float *depth,
                       float *cov, float *mean2d)
{
    float mx = gin[0], my = gin[1], mz = gin[2];
    float qw = gin[3], qx = gin[4], qy = gin[5], qz = gin[6];
    float sx = gin[7], sy = gin[8], sz = gin[9], op = gin[10];
    const float *R = cam;
    const float *t = cam + 9;
    float fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    float Wf = cam[16], Hf = cam[17];
    int W = (int)Wf, H = (int)Hf;
    *flags = 0;
    *ntiles = 0;
    rect[0] = rect[1] = rect[2] = rect[3] = 0;
    *depth = 0.0f;
    cov[0] = cov[1] = cov[2] = 0.0f;
    mean2d[0] = mean2d[1] = 0.0f;

    for (int i = 0; i < 11; ++i)
        if (!isfinite(gin[i])) { *flags = 4; return; }
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(n2 > 0.0f) || !isfinite(n2) || !(sx > 0.0f) || !(sy > 0.0f) || !(sz > 0.0f)) { *flags = 4; return; }
    (void)op;

    /* camera-space mean */
    float px = ((R[0] * mx + R[1] * my) + R[2] * mz) + t[0];
    float py = ((R[3] * mx + R[4] * my) + R[5] * mz) + t[1];
    float pz = ((R[6] * mx + R[7] * my) + R[8] * mz) + t[2];
    *depth = pz;
    if (!(pz > prm[P_ZN])) return;

    /* unit quaternion -> rotation matrix */
    float nrm = sqrtf(n2);
    float w = qw / nrm, x = qx / nrm, y = qy / nrm, z = qz / nrm;
    float q[9];
    q[0] = 1.0f - 2.0f * (y * y + z * z);
    q[1] = 2.0f * (x * y - w * z);
    q[2] = 2.0f * (x * z + w * y);
    q[3] = 2.0f * (x * y + w * z);
    q[4] = 1.0f - 2.0f * (x * x + z * z);
    q[5] = 2.0f * (y * z - w * x);
    q[6] = 2.0f * (x * z - w * y);
    q[7] = 2.0f * (y * z + w * x);
    q[8] = 1.0f - 2.0f * (x * x + y * y);
    float s[3] = {sx, sy, sz};
    float L[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) L[i * 3 + j] = q[i * 3 + j] * s[j];
    /* world rotation of the camera applied to the Gaussian's frame */
    float Vm[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Vm[i * 3 + j] = (R[i * 3 + 0] * L[0 * 3 + j] + R[i * 3 + 1] * L[1 * 3 + j]) + R[i * 3 + 2] * L[2 * 3 + j];

    /* Jacobian of the pinhole projection, with the guard-band clamp */
    float xr = px / pz, yr = py / pz;
    float limx = prm[P_GUARD] * ((0.5f * Wf) / fx);
    float limy = prm[P_GUARD] * ((0.5f * Hf) / fy);
    float txc = fminf(fmaxf(xr, -limx), limx);
    float tyc = fminf(fmaxf(yr, -limy), limy);
    float j00 = fx / pz, j02 = -((fx * txc) / pz);
    float j11 = fy / pz, j12 = -((fy * tyc) / pz);
    float m0[3], m1[3];
    for (int j = 0; j < 3; ++j) {
        m0[j] = j00 * Vm[0 * 3 + j] + j02 * Vm[2 * 3 + j];
        m1[j] = j11 * Vm[1 * 3 + j] + j12 * Vm[2 * 3 + j];
    }
    float lp = prm[P_LP];
    float a = ((m0[0] * m0[0] + m0[1] * m0[1]) + m0[2] * m0[2]) + lp;
    float b = (m0[0] * m1[0] + m0[1] * m1[1]) + m0[2] * m1[2];
    float c = ((m1[0] * m1[0] + m1[1] * m1[1]) + m1[2] * m1[2]) + lp;
    cov[0] = a; cov[1] = b; cov[2] = c;

    float u = fx * xr + cx;
    float v = fy * yr + cy;
    mean2d[0] = u; mean2d[1] = v;

    /* bounding box of the support ellipse d^T Sigma^-1 d <= k^2: its half
     * extents are k*sqrt(a) and k*sqrt(c), rounded up to whole pixels */
    float rx = ceilf(prm[P_K] * sqrtf(a));
    float ry = ceilf(prm[P_K] * sqrtf(c));
    if (!isfinite(u) || !isfinite(v) || !isfinite(rx) || !isfinite(ry) || !isfinite(a) || !isfinite(b) || !isfinite(c)) return;

    float det = a * c - b * b;
    uint8_t f = 1;
    if (!(det > 0.0f) || (a * c >= prm[P_COND] * det)) f |= 2;
    *flags = f;

    float fk0 = ceilf((u - rx) - 0.5f), fk1 = floorf((u + rx) - 0.5f);
    float fj0 = ceilf((v - ry) - 0.5f), fj1 = floorf((v + ry) - 0.5f);
    if (fk1 < 0.0f || fk0 > (float)(W - 1) || fj1 < 0.0f || fj0 > (float)(H - 1) || fk0 > fk1 || fj0 > fj1)
        return;
    int kmin = (int)fmaxf(fk0, 0.0f), kmax = (int)fminf(fk1, (float)(W - 1));
    int jmin = (int)fmaxf(fj0, 0.0f), jmax = (int)fminf(fj1, (float)(H - 1));
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    rect[0] = kmin / tw; rect[1] = jmin / th; rect[2] = kmax / tw; rect[3] = jmax / th;
    supp32_t sp = supp32(u, v, a, b, c, f, prm[P_K]);
    int nt = 0;
    for (int ty = rect[1]; ty <= rect[3]; ++ty) {
        int l, r;
        if (row_listed32(&sp, ty, rect[0], rect[2], tw, th, W, H, &l, &r)) nt += r - l + 1;
    }
    *ntiles = nt;
}

/* gauss: float32 [11][n] structure of arrays (mx,my,mz,qw,qx,qy,qz,sx,sy,sz,op). */
void or_project32(int64_t n, const float *gauss, const float *cam, const float *prm,
                  uint8_t *flags, int32_t *rect, int32_t *ntiles, float *depth, float *cov, float *mean2d)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t g = 0; g < n; ++g) {
        float gin[11];
        for (int i = 0; i < 11; ++i) gin[i] = gauss[(int64_t)i * n + g];
        proj32_one(gin, cam, prm, flags + g, rect + 4 * g, ntiles + g, depth + g, cov + 3 * g, mean2d + 2 * g);
    }
}

/* ------------------------------------------------------------------------
 * Binning: one (tile, depth, id) record per tile overlapped by a visible
 * Gaussian, ordered by tile, then depth ("blended by their depth order",
 * Sec. 3.1), then Gaussian id for equal depths. The sort is the C library's
 * qsort with a plain lexicographic comparator.
 * ---------------------------------------------------------------------- */
typedef struct { int32_t tile; float depth; uint32_t g; } pair_t;

static int cmp_pair(const void *pa, const void *pb)
{
    const pair_t *a = (const pair_t *)pa, *b = (const pair_t *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    if (a->g != b->g) return a->g < b->g ? -1 : 1;
    return 0;
}

/* Returns the number of pairs (-1 if the rectangle enumeration disagrees with
 * ntiles). out_tile/out_g must hold sum(ntiles) entries;
 * ranges: uint32 [tiles_x*tiles_y][2], empty tiles get [0,0). */
int64_t or_bin(int64_t n, const uint8_t *flags, const int32_t *rect, const int32_t *ntiles,
               const float *depth, const float *cov, const float *mean2d, const float *cam, const float *prm,
               int32_t tiles_x, int32_t tiles_y, int32_t *out_tile, uint32_t *out_g, uint32_t *ranges)
{
    int W = (int)cam[16], H = (int)cam[17];
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    int64_t total = 0;
    for (int64_t g = 0; g < n; ++g)
        if (flags[g] & 1) total += ntiles[g];
    pair_t *p = (pair_t *)malloc(sizeof(pair_t) * (size_t)(total > 0 ? total : 1));
    int64_t k = 0;
    for (int64_t g = 0; g < n; ++g) {
        if (!(flags[g] & 1) || ntiles[g] == 0) continue;
        supp32_t sp = supp32(mean2d[2 * g], mean2d[2 * g + 1], cov[3 * g], cov[3 * g + 1], cov[3 * g + 2], flags[g], prm[P_K]);
        for (int ty = rect[4 * g + 1]; ty <= rect[4 * g + 3]; ++ty) {
            int l, r;
            if (!row_listed32(&sp, ty, rect[4 * g + 0], rect[4 * g + 2], tw, th, W, H, &l, &r)) continue;
            for (int tx = l; tx <= r; ++tx) {
                p[k].tile = ty * tiles_x + tx;
                p[k].depth = depth[g];
                p[k].g = (uint32_t)g;
                ++k;
            }
        }
    }
    if (k != total) { free(p); return -1; }
    qsort(p, (size_t)total, sizeof(pair_t), cmp_pair);
    int64_t T = (int64_t)tiles_x * tiles_y;
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)T);
    for (int64_t i = 0; i < total; ++i) {
        out_tile[i] = p[i].tile;
        out_g[i] = p[i].g;
        if (i == 0 || p[i - 1].tile != p[i].tile) ranges[2 * p[i].tile] = (uint32_t)i;
        if (i == total - 1 || p[i + 1].tile != p[i].tile) ranges[2 * p[i].tile + 1] = (uint32_t)(i + 1);
    }
    free(p);
    return total;
}

/* ------------------------------------------------------------------------
 * binary64 projection: mean2D, conic (inverse 2D covariance), computed from
 * the float32 inputs promoted to double. The determinant uses the
 * Cauchy-Binet expansion det(M M^T + d I) = sum_{i<j} minor_ij(M)^2
 * + d * trace(M M^T) + d^2, which has no cancellation.
 * out: double [n][5] = (u, v, conic_xx, conic_xy, conic_yy).
 * ---------------------------------------------------------------------- */
void or_project64(int64_t n, const float *gauss, const float *cam, const float *prm, double *out)
{
    const double R[9] = {cam[0], cam[1], cam[2], cam[3], cam[4], cam[5], cam[6], cam[7], cam[8]};
    const double t[3] = {cam[9], cam[10], cam[11]};
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15], Wd = cam[16], Hd = cam[17];
    double lp = prm[P_LP], guard = prm[P_GUARD];
    for (int64_t g = 0; g < n; ++g) {
        double gi[11];
        for (int i = 0; i < 11; ++i) gi[i] = (double)gauss[(int64_t)i * n + g];
        double *o = out + 5 * g;
        o[0] = o[1] = o[2] = o[3] = o[4] = 0.0;
        double px = R[0] * gi[0] + R[1] * gi[1] + R[2] * gi[2] + t[0];
        double py = R[3] * gi[0] + R[4] * gi[1] + R[5] * gi[2] + t[1];
        double pz = R[6] * gi[0] + R[7] * gi[1] + R[8] * gi[2] + t[2];
        double qn = sqrt(gi[3] * gi[3] + gi[4] * gi[4] + gi[5] * gi[5] + gi[6] * gi[6]);
        if (!(qn > 0.0) || !(pz != 0.0)) continue;
        double w = gi[3] / qn, x = gi[4] / qn, y = gi[5] / qn, z = gi[6] / qn;
        double q[9] = {
            1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
            2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
            2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        double s[3] = {gi[7], gi[8], gi[9]};
        double Vm[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int l = 0; l < 3; ++l) acc += R[i * 3 + l] * q[l * 3 + j] * s[j];
                Vm[i * 3 + j] = acc;
            }
        double xr = px / pz, yr = py / pz;
        double limx = guard * (0.5 * Wd / fx), limy = guard * (0.5 * Hd / fy);
        double txc = fmin(fmax(xr, -limx), limx), tyc = fmin(fmax(yr, -limy), limy);
        double J[6] = {fx / pz, 0.0, -fx * txc / pz, 0.0, fy / pz, -fy * tyc / pz};
        double M[6];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                M[i * 3 + j] = J[i * 3 + 0] * Vm[0 * 3 + j] + J[i * 3 + 1] * Vm[1 * 3 + j] + J[i * 3 + 2] * Vm[2 * 3 + j];
        double s00 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
        double s01 = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
        double s11 = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
        double m01 = M[0] * M[4] - M[1] * M[3];
        double m02 = M[0] * M[5] - M[2] * M[3];
        double m12 = M[1] * M[5] - M[2] * M[4];
        double det = m01 * m01 + m02 * m02 + m12 * m12 + lp * (s00 + s11) + lp * lp;
        double a = s00 + lp, b = s01, c = s11 + lp;
        o[0] = fx * xr + cx;
        o[1] = fy * yr + cy;
        o[2] = c / det;
        o[3] = -b / det;
        o[4] = a / det;
    }
}

/* ------------------------------------------------------------------------
 * binary64 compositing of one view with accumulation into A (Eq. (1),
 * Eq. (7)-(8), Listing 1 of the supplement). For every pixel, front to back over its
 * tile's list:
 *   d = pixel_centre - mean2D
 *   power = -0.5 (cxx dx^2 + cyy dy^2) - cxy dx dy
 *   skip if power < -k^2/2                  (elliptical support)
 *   alpha = min(alpha_max, o * exp(power)); skip if alpha < alpha_min
 *   T' = T (1 - alpha); stop (without adding) if T' < t_min
 *   A[g][label] += alpha * T; T = T'
 *
 * Decision ambiguity. The GPU makes the three threshold decisions in
 * float32; near a threshold the two precisions may decide differently. When
 * a decision lies within a relative band `band_eps` of its threshold, the
 * oracle adds to slack[g] the largest change that a different decision could
 * make to row g (first order): the flipped Gaussian's own weight, and, for
 * every later Gaussian in that pixel, its weight times the relative change of
 * T (alpha/(1-alpha)), or its whole weight after a possible early stop.
 *
 * Inputs: list (out_g of or_bin) + ranges, p64 from or_project64, mask
 * uint8 [H][W]. Accumulates into A (double [n][E]) and slack (double [n]);
 * writes tfinal (double [H][W]) and nblend (int32 [H][W]) when non-NULL.
 * stats (int64 [4]) += {blends, flagged decisions, bad labels, pairs evaluated
 * inside the support before the pixel's compositing ended}.
 * ---------------------------------------------------------------------- */
void or_composite64(int64_t n, const double *p64, const float *opacity, const float *cam,
                    const float *prm, const uint32_t *list, const uint32_t *ranges,
                    const uint8_t *mask, int32_t E, double *A, double *slack,
                    double *tfinal, int32_t *nblend, int64_t *stats)
{
    int W = (int)cam[16], H = (int)cam[17];
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    double k = prm[P_K], cut = -0.5 * k * k;
    double amin = prm[P_AMIN], amax = prm[P_AMAX], tmin = prm[P_TMIN], eps = prm[P_EPS];
    int64_t s_blend = 0, s_flag = 0, s_bad = 0, s_eval = 0;
    (void)n;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : s_blend, s_flag, s_bad, s_eval)
    for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
        int tx = tile % tiles_x, ty = tile / tiles_x;
        uint32_t rs = ranges[2 * tile], re = ranges[2 * tile + 1];
        for (int jj = 0; jj < th; ++jj)
            for (int kk = 0; kk < tw; ++kk) {
                int j = ty * th + jj, kx = tx * tw + kk;
                if (j >= H || kx >= W) continue;
                int lab = mask[(int64_t)j * W + kx];
                if (lab >= E) {
                    s_bad++;
                    if (tfinal) tfinal[(int64_t)j * W + kx] = 1.0;
                    if (nblend) nblend[(int64_t)j * W + kx] = 0;
                    continue;
                }
                double pxc = kx + 0.5, pyc = j + 0.5;
                double T = 1.0, pert = 0.0;
                int tail = 0, nb = 0;
                for (uint32_t i = rs; i < re; ++i) {
                    uint32_t g = list[i];
                    const double *q = p64 + 5 * (int64_t)g;
                    double dx = pxc - q[0], dy = pyc - q[1];
                    double power = -0.5 * (q[2] * dx * dx + q[4] * dy * dy) - q[3] * dx * dy;
                    double alpha = fmin(amax, (double)opacity[g] * exp(power));
                    if (power >= cut) s_eval++;
                    int f_sup = fabs(power - cut) <= eps * (-cut);
                    int f_amin = amin > 0.0 && fabs(alpha - amin) <= eps * amin;
                    int take = (power >= cut) && (alpha >= amin);
                    /* could a float32 evaluation decide this Gaussian the other way? A taken
                     * one if either test lies in its band; a skipped one only if every test
                     * it fails lies in its band */
                    int flip = take ? (f_sup || f_amin)
                                    : ((power >= cut || f_sup) && (alpha >= amin || f_amin));
                    double rel = alpha < 1.0 ? alpha / (1.0 - alpha) : 1.0;
                    if (!take) {
                        if (flip) {
                            s_flag++;
#pragma omp atomic
                            slack[g] += alpha * T * (1.0 + pert);
                            pert += rel + pert * rel;
                        }
                        continue;
                    }
                    double Tn = T * (1.0 - alpha);
                    int f_tmin = tmin > 0.0 && fabs(Tn - tmin) <= (eps + pert) * tmin;
                    if (Tn < tmin) {
                        if (f_tmin) {
                            /* the alternative does not stop here: this Gaussian and the
                             * next ones it could still add, at most at the raised T */
                            s_flag++;
#pragma omp atomic
                            slack[g] += alpha * T * (1.0 + pert);
                            double Ts = Tn * (1.0 + pert);
                            double Tlow = tmin * (1.0 - (eps + pert));
                            for (uint32_t i2 = i + 1; i2 < re && Ts >= Tlow; ++i2) {
                                uint32_t g2 = list[i2];
                                const double *q2 = p64 + 5 * (int64_t)g2;
                                double dx2 = pxc - q2[0], dy2 = pyc - q2[1];
                                double pw2 = -0.5 * (q2[2] * dx2 * dx2 + q2[4] * dy2 * dy2) - q2[3] * dx2 * dy2;
                                double a2 = fmin(amax, (double)opacity[g2] * exp(pw2));
                                if (pw2 < cut * (1.0 + eps) || a2 < amin * (1.0 - eps)) continue;
#pragma omp atomic
                                slack[g2] += a2 * Ts;
                                Ts *= 1.0 - a2;
                            }
                        }
                        break;
                    }
                    double wgt = alpha * T;
#pragma omp atomic
                    A[(int64_t)g * E + lab] += wgt;
                    double sl;
                    if (tail || flip || f_tmin) sl = wgt;
                    else sl = wgt * pert;
                    if (sl != 0.0) {
#pragma omp atomic
                        slack[g] += sl;
                    }
                    if (flip) { s_flag++; pert += rel + pert * rel; }
                    if (f_tmin) { s_flag++; tail = 1; }
                    T = Tn;
                    nb++;
                }
                s_blend += nb;
                if (tfinal) tfinal[(int64_t)j * W + kx] = T;
                if (nblend) nblend[(int64_t)j * W + kx] = nb;
            }
    }
    stats[0] += s_blend;
    stats[1] += s_flag;
    stats[2] += s_bad;
    stats[3] += s_eval;
}

/* ------------------------------------------------------------------------
 * Eq. (1) rendered literally: X = sum_i x_i alpha_i prod_{j<i} (1 - alpha_j)
 * over the Gaussians that the compositing above adds, with the product of
 * (1 - alpha_j) formed afresh for every term (no running transmittance).
 * x: double [n] per-Gaussian property. Used with x = 1 (accumulated alpha)
 * and with x = P_i (a labelling), and for the objective of Eq. (2).
 * out: double [H][W].
 * ---------------------------------------------------------------------- */
void or_render64(int64_t n, const double *p64, const float *opacity, const float *cam,
                 const float *prm, const uint32_t *list, const uint32_t *ranges,
                 const double *x, double *out)
{
    int W = (int)cam[16], H = (int)cam[17];
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    double k = prm[P_K], cut = -0.5 * k * k;
    double amin = prm[P_AMIN], amax = prm[P_AMAX], tmin = prm[P_TMIN];
    (void)n;
    for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
        int tx = tile % tiles_x, ty = tile / tiles_x;
        uint32_t rs = ranges[2 * tile], re = ranges[2 * tile + 1];
        uint32_t cnt = re - rs;
        double *al = (double *)malloc(sizeof(double) * (cnt ? cnt : 1));
        uint32_t *gs = (uint32_t *)malloc(sizeof(uint32_t) * (cnt ? cnt : 1));
        for (int jj = 0; jj < th; ++jj)
            for (int kk = 0; kk < tw; ++kk) {
                int j = ty * th + jj, kx = tx * tw + kk;
                if (j >= H || kx >= W) continue;
                /* collect the alphas that enter the blend, in depth order */
                uint32_t m = 0;
                for (uint32_t i = rs; i < re; ++i) {
                    uint32_t g = list[i];
                    const double *q = p64 + 5 * (int64_t)g;
                    double dx = (kx + 0.5) - q[0], dy = (j + 0.5) - q[1];
                    double power = -0.5 * (q[2] * dx * dx + q[4] * dy * dy) - q[3] * dx * dy;
                    if (power < cut) continue;
                    double a = fmin(amax, (double)opacity[g] * exp(power));
                    if (a < amin) continue;
                    /* the blend ends before the term whose transmittance after it falls below t_min */
                    double prod = 1.0;
                    for (uint32_t l = 0; l < m; ++l) prod *= (1.0 - al[l]);
                    if (prod * (1.0 - a) < tmin) break;
                    al[m] = a;
                    gs[m] = g;
                    ++m;
                }
                double X = 0.0;
                for (uint32_t i = 0; i < m; ++i) {
                    double prod = 1.0;
                    for (uint32_t l = 0; l < i; ++l) prod *= (1.0 - al[l]);
                    X += x[gs[i]] * al[i] * prod;
                }
                out[(int64_t)j * W + kx] = X;
            }
        free(al);
        free(gs);
    }
}

/* ------------------------------------------------------------------------
 * Dense per-pixel weights for tiny scenes: wout double [H*W][n] receives
 * alpha_i T_i for every Gaussian added at every pixel (same rules as
 * or_composite64). Used by the exhaustive checks of Eq. (2) and Eq. (6).
 * ---------------------------------------------------------------------- */
void or_weights64(int64_t n, const double *p64, const float *opacity, const float *cam,
                  const float *prm, const uint32_t *list, const uint32_t *ranges, double *wout)
{
    int W = (int)cam[16], H = (int)cam[17];
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    double k = prm[P_K], cut = -0.5 * k * k;
    double amin = prm[P_AMIN], amax = prm[P_AMAX], tmin = prm[P_TMIN];
    memset(wout, 0, sizeof(double) * (size_t)W * H * (size_t)n);
    for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
        int tx = tile % tiles_x, ty = tile / tiles_x;
        for (int jj = 0; jj < th; ++jj)
            for (int kk = 0; kk < tw; ++kk) {
                int j = ty * th + jj, kx = tx * tw + kk;
                if (j >= H || kx >= W) continue;
                double T = 1.0;
                for (uint32_t i = ranges[2 * tile]; i < ranges[2 * tile + 1]; ++i) {
                    uint32_t g = list[i];
                    const double *q = p64 + 5 * (int64_t)g;
                    double dx = (kx + 0.5) - q[0], dy = (j + 0.5) - q[1];
                    double power = -0.5 * (q[2] * dx * dx + q[4] * dy * dy) - q[3] * dx * dy;
                    if (power < cut) continue;
                    double a = fmin(amax, (double)opacity[g] * exp(power));
                    if (a < amin) continue;
                    double Tn = T * (1.0 - a);
                    if (Tn < tmin) break;
                    wout[((int64_t)j * W + kx) * n + g] += a * T;
                    T = Tn;
                }
            }
    }
}

/* ------------------------------------------------------------------------
 * Novel-view masks (Sec. 3.4; the supplement's "Quantization in novel view
 * mask"), binary64. For every object e, only its member Gaussians
 * (S[e][g] != 0) are composited, front to back over the tile lists, with the
 * same rules as or_composite64:
 *   rho_e = sum alpha T          (the object's alpha mask)
 *   D_e   = sum alpha T z / rho_e (its depth where visible; +inf if rho_e = 0)
 * label = mode 0: the object e >= 1 with rho_e > tau and least D_e (ties to
 *                 the smaller e), 0 if there is none (depth-guided);
 *         mode 1: argmax over every e >= 0 of rho_e (first maximum).
 * z: double [n] camera-space depth of each Gaussian. S: uint8 [E][n].
 * Outputs: label uint8 [H][W]; rho, depth double [E][H][W] (may be NULL).
 * ---------------------------------------------------------------------- */
void or_render_masks64(int64_t n, const double *p64, const float *opacity, const double *z, const float *cam,
                       const float *prm, const uint32_t *list, const uint32_t *ranges, const uint8_t *S, int32_t E,
                       double tau, int32_t mode, uint8_t *label, double *rho_out, double *depth_out)
{
    int W = (int)cam[16], H = (int)cam[17];
    int tw = (int)prm[P_TW], th = (int)prm[P_TH];
    int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    double k = prm[P_K], cut = -0.5 * k * k;
    double amin = prm[P_AMIN], amax = prm[P_AMAX], tmin = prm[P_TMIN];
    int64_t npix = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
        int tx = tile % tiles_x, ty = tile / tiles_x;
        uint32_t rs = ranges[2 * tile], re = ranges[2 * tile + 1];
        for (int jj = 0; jj < th; ++jj)
            for (int kk = 0; kk < tw; ++kk) {
                int j = ty * th + jj, kx = tx * tw + kk;
                if (j >= H || kx >= W) continue;
                int64_t pix = (int64_t)j * W + kx;
                int best = 0;
                double best_d = INFINITY, best_rho = -1.0;
                for (int e = (mode == 1 ? 0 : 1); e < E; ++e) {
                    const uint8_t *mem = S + (int64_t)e * n;
                    double T = 1.0, rho = 0.0, dz = 0.0;
                    for (uint32_t i = rs; i < re; ++i) {
                        uint32_t g = list[i];
                        if (!mem[g]) continue;
                        const double *q = p64 + 5 * (int64_t)g;
                        double dx = (kx + 0.5) - q[0], dy = (j + 0.5) - q[1];
                        double power = -0.5 * (q[2] * dx * dx + q[4] * dy * dy) - q[3] * dx * dy;
                        if (power < cut) continue;
                        double a = fmin(amax, (double)opacity[g] * exp(power));
                        if (a < amin) continue;
                        double Tn = T * (1.0 - a);
                        if (Tn < tmin) break;
                        rho += a * T;
                        dz += a * T * z[g];
                        T = Tn;
                    }
                    double d = rho > 0.0 ? dz / rho : INFINITY;
                    if (rho_out) rho_out[(int64_t)e * npix + pix] = rho;
                    if (depth_out) depth_out[(int64_t)e * npix + pix] = d;
                    if (mode == 1) {
                        if (rho > best_rho) { best_rho = rho; best = e; }
                    } else if (rho > tau && d < best_d) {
                        best_d = d;
                        best = e;
                    }
                }
                label[pix] = (uint8_t)best;
            }
    }
}
