// a1: projection of 3D Gaussians to 2D Gaussians per view (paper Sec. 3.1,
// which inherits EWA splatting from the 3DGS renderer).
//
// This translation unit is compiled with -ffp-contract=off: the visibility
// decision, the bounding radius and the tile rectangle are part of the
// bit-exact binning contract, so every binary32 operation below is evaluated
// exactly as written, in the order written (products rounded, sums left to
// right, correctly rounded division and square root).
#include "fs_internal.h"
#include "fs_tiles.h"

namespace fs {
namespace {

__device__ __forceinline__ bool finite32(float x) { return __builtin_isfinite(x); }

// rows of a block's list whose splat is looked up in a table rather than by a
// binary search in the row offsets (a multiple of 256, so the choice is the
// same for every lane of a wave)
constexpr uint32_t kRowMap = 2048;

// Inclusive sum over the 256 threads of the block (all threads call it).
__device__ __forceinline__ uint32_t block_incl_sum(uint32_t x, uint32_t *s_wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    for (int k = 0; k < w; ++k) x += s_wsum[k];
    __syncthreads();
    return x;
}

// Block b belongs to the task whose [blk0, next blk0) holds b; the task's
// Gaussians are loaded once and projected into its (up to kProjViews) views.
//
// Listed tiles. The tile rows of a splat's rectangle are listed one by one
// (row_span), and splats differ widely in their number of rows, so each thread
// listing its own splat's rows would leave the wave waiting for its largest
// splat. Instead the block lists the rows of all its 256 splats together:
// every thread takes rows in turn from the block's concatenated row list (a
// binary search in the block's row offsets finds the splat), and the counts
// and span-code bytes are gathered per splat in LDS.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_project(const ProjTask *__restrict__ tasks, int32_t n_tasks,
                                                 const SceneDev *__restrict__ scenes, const ViewDev *__restrict__ views,
                                                 ProjParams P, float4 *__restrict__ rec, short4 *__restrict__ rect,
                                                 int32_t *__restrict__ ntiles, uint8_t *__restrict__ flags,
                                                 uint32_t *__restrict__ dkeys, uint32_t *__restrict__ dvals,
                                                 ulonglong2 *__restrict__ codes, unsigned long long *__restrict__ status)
{
    int lo = 0, hi = n_tasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].blk0 <= blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const ProjTask task = tasks[lo];
    const SceneDev &S = scenes[task.scene];
    const GaussPtrs G = S.g;
    const int64_t n = S.n;
    const int64_t g = (int64_t)(blockIdx.x - task.blk0) * blockDim.x + threadIdx.x;
    const int v0 = (int)task.v0;
    const int v1 = (int)(task.v0 + task.nv);
    const bool live = g < n;

    float mx = 0.f, my = 0.f, mz = 0.f, qw = 1.f, qx = 0.f, qy = 0.f, qz = 0.f, sx = 1.f, sy = 1.f, sz = 1.f, op = 0.f;
    if (live) {
        mx = G.mx[g]; my = G.my[g]; mz = G.mz[g];
        qw = G.qw[g]; qx = G.qx[g]; qy = G.qy[g]; qz = G.qz[g];
        sx = G.sx[g]; sy = G.sy[g]; sz = G.sz[g];
        op = G.op[g];
    }
    // input validity (independent of the view)
    bool valid = finite32(mx) && finite32(my) && finite32(mz) && finite32(qw) && finite32(qx) &&
                 finite32(qy) && finite32(qz) && finite32(sx) && finite32(sy) && finite32(sz) && finite32(op);
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    valid = valid && (n2 > 0.0f) && finite32(n2) && (sx > 0.0f) && (sy > 0.0f) && (sz > 0.0f);

    // rotation of the Gaussian (unit quaternion -> matrix) times its scales
    float L[9];
    {
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
        const float s[3] = {sx, sy, sz};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) L[i * 3 + j] = q[i * 3 + j] * s[j];
    }

    __shared__ Span32 s_span[256];
    __shared__ int4 s_rect[256];        // x0, y0, x1, small (span code kept)
    __shared__ uint32_t s_off[257];     // first row of each splat in the block's row list
    __shared__ uint32_t s_cnt[256];     // listed tiles per splat
    __shared__ __align__(16) uint8_t s_code[256][16];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint8_t s_rowsplat[kRowMap];  // the splat of each of the block's first kRowMap rows
    const int tid = threadIdx.x;

    int n_invalid = 0, n_fp64 = 0;
    for (int v = v0; v < v1; ++v) {
        const ViewDev &C = views[v];
        const float *R = C.R;
        const int64_t idx = (int64_t)C.elem_off + g;
        uint8_t f = 0;
        int nt = 0;
        uint32_t rows = 0;                 // tile rows of this splat to list
        Span32 sp_mine = make_span32(0.f, 0.f, 1.f, 0.f, 1.f, true, 1.0f);
        int4 rect_mine = make_int4(0, 0, -1, 0);
        SpanCode code = no_code();
        short4 rc = make_short4(0, 0, 0, 0);
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live && !valid) {
            f = 4;
            n_invalid++;
        } else if (live) {
            float px = ((R[0] * mx + R[1] * my) + R[2] * mz) + C.t[0];
            float py = ((R[3] * mx + R[4] * my) + R[5] * mz) + C.t[1];
            float pz = ((R[6] * mx + R[7] * my) + R[8] * mz) + C.t[2];
            r1.z = pz;
            if (pz > P.znear) {
                float Vm[9];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        Vm[i * 3 + j] = (R[i * 3 + 0] * L[0 * 3 + j] + R[i * 3 + 1] * L[1 * 3 + j]) + R[i * 3 + 2] * L[2 * 3 + j];
                float xr = px / pz, yr = py / pz;
                const float limx = C.limx, limy = C.limy;  // guard * ((0.5 W) / fx), per view
                float txc = fminf(fmaxf(xr, -limx), limx);
                float tyc = fminf(fmaxf(yr, -limy), limy);
                float j00 = C.fx / pz, j02 = -((C.fx * txc) / pz);
                float j11 = C.fy / pz, j12 = -((C.fy * tyc) / pz);
                float m0[3], m1[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    m0[j] = j00 * Vm[0 * 3 + j] + j02 * Vm[2 * 3 + j];
                    m1[j] = j11 * Vm[1 * 3 + j] + j12 * Vm[2 * 3 + j];
                }
                const float lp = P.lowpass;
                float a = ((m0[0] * m0[0] + m0[1] * m0[1]) + m0[2] * m0[2]) + lp;
                float b = (m0[0] * m1[0] + m0[1] * m1[1]) + m0[2] * m1[2];
                float c = ((m1[0] * m1[0] + m1[1] * m1[1]) + m1[2] * m1[2]) + lp;
                float u = C.fx * xr + C.cx;
                float vv = C.fy * yr + C.cy;
                // pixel bounding box of the support ellipse: half extents k*sqrt(a), k*sqrt(c)
                float rx = ceilf(P.sigma_k * sqrtf(a));
                float ry = ceilf(P.sigma_k * sqrtf(c));
                if (finite32(u) && finite32(vv) && finite32(rx) && finite32(ry) && finite32(a) && finite32(b) && finite32(c)) {
                    float det = a * c - b * b;
                    bool deg = !(det > 0.0f) || (a * c >= P.fp64_cond * det);
                    f = deg ? 3 : 1;
                    // inverse 2D covariance as LDL^T factors: q = p (dx + r dy)^2 + s dy^2
                    float cp, cr, cs;
                    if (deg && P.fp64_conic) {
                        n_fp64++;
                        const double d00 = (double)m0[0], d01 = (double)m0[1], d02 = (double)m0[2];
                        const double d10 = (double)m1[0], d11 = (double)m1[1], d12 = (double)m1[2];
                        const double s00 = d00 * d00 + d01 * d01 + d02 * d02;
                        const double s01 = d00 * d10 + d01 * d11 + d02 * d12;
                        const double s11 = d10 * d10 + d11 * d11 + d12 * d12;
                        const double mn01 = d00 * d11 - d01 * d10;
                        const double mn02 = d00 * d12 - d02 * d10;
                        const double mn12 = d01 * d12 - d02 * d11;
                        const double lpd = (double)lp;
                        // Cauchy-Binet: det(M M^T + lp I), every term non-negative
                        const double det64 = mn01 * mn01 + mn02 * mn02 + mn12 * mn12 + lpd * (s00 + s11) + lpd * lpd;
                        const double c64 = s11 + lpd;
                        cp = (float)(c64 / det64);
                        cr = (float)(-s01 / c64);
                        cs = (float)(1.0 / c64);
                    } else {
                        ldl32(a, b, c, cp, cr, cs);
                    }
                    r0 = make_float4(u, vv, cp, cr);
                    r1.x = cs;
                    r1.y = op;
                    // 0: float32 factors, listed by the support test; 1: float64 factors,
                    // whole rectangle listed; 2: float32 factors, whole rectangle listed
                    r1.w = deg ? (P.fp64_conic ? 1.0f : 2.0f) : 0.0f;
                    float fk0 = ceilf((u - rx) - 0.5f), fk1 = floorf((u + rx) - 0.5f);
                    float fj0 = ceilf((vv - ry) - 0.5f), fj1 = floorf((vv + ry) - 0.5f);
                    if (!(fk1 < 0.0f || fk0 > (float)(C.W - 1) || fj1 < 0.0f || fj0 > (float)(C.H - 1) ||
                          fk0 > fk1 || fj0 > fj1)) {
                        int kmin = (int)fmaxf(fk0, 0.0f), kmax = (int)fminf(fk1, (float)(C.W - 1));
                        int jmin = (int)fmaxf(fj0, 0.0f), jmax = (int)fminf(fj1, (float)(C.H - 1));
                        int x0 = tile_of(kmin, P.tile_w), y0 = tile_of(jmin, P.tile_h);
                        int x1 = tile_of(kmax, P.tile_w), y1 = tile_of(jmax, P.tile_h);
                        rc = make_short4((short)x0, (short)y0, (short)x1, (short)y1);
                        // tiles of the rectangle that the support reaches: listed below, row by row
                        sp_mine = make_span32(u, vv, cp, cr, cs, deg, support_limit(P.sigma_k));
                        const bool small = y1 - y0 < kSpanCodeRows && x1 - x0 < 16;
                        rect_mine = make_int4(x0, y0, x1, small ? 1 : 0);
                        rows = (uint32_t)(y1 - y0 + 1);
                    }
                }
            }
        }
        // the block's splats list their tile rows together
        s_span[tid] = sp_mine;
        s_rect[tid] = rect_mine;
        s_cnt[tid] = 0;
        *reinterpret_cast<uint4 *>(&s_code[tid][0]) = make_uint4(~0u, ~0u, ~0u, ~0u);
        const uint32_t incl = block_incl_sum(rows, s_wsum);  // ends with a barrier
        s_off[tid + 1] = incl;
        if (tid == 0) s_off[0] = 0;
        for (uint32_t r = incl - rows; r < min(incl, kRowMap); ++r) s_rowsplat[r] = (uint8_t)tid;
        __syncthreads();
        const uint32_t n_rows = s_off[256];
        for (uint32_t i = (uint32_t)tid; i < n_rows; i += 256u) {
            // the splat e with s_off[e] <= i < s_off[e + 1]: from the map, or by a
            // binary search past its end (i < kRowMap is the same for the whole wave)
            int e;
            if (i < kRowMap) {
                e = s_rowsplat[i];
            } else {
                int lo_e = 0, hi_e = 255;
                while (lo_e < hi_e) {
                    const int mid = (lo_e + hi_e + 1) >> 1;
                    if (s_off[mid] <= i) lo_e = mid; else hi_e = mid - 1;
                }
                e = lo_e;
            }
            const int4 re = s_rect[e];
            const int row = (int)(i - s_off[e]);
            int l, r;
            if (row_span(s_span[e], re.y + row, re.x, re.z, P.tile_w, P.tile_h, C.W, C.H, l, r)) {
                atomicAdd(&s_cnt[e], (uint32_t)(r - l + 1));
                if (re.w) s_code[e][row] = (uint8_t)((uint32_t)(l - re.x) | ((uint32_t)(r - l) << 4));
            }
        }
        __syncthreads();
        if (rows > 0) {
            nt = (int)s_cnt[tid];
            if (rect_mine.w) {
                const uint4 cw = *reinterpret_cast<const uint4 *>(&s_code[tid][0]);
                code = SpanCode{(uint64_t)cw.x | ((uint64_t)cw.y << 32), (uint64_t)cw.z | ((uint64_t)cw.w << 32)};
            }
        }
        __syncthreads();  // the next view reuses the block's LDS
        if (live) {
            rec[idx * 2 + 0] = r0;
            rec[idx * 2 + 1] = r1;
            rect[idx] = rc;
            ntiles[idx] = nt;
            flags[idx] = f;
            if (codes) store_emit_record(codes, idx, code, rc);
            if (dkeys) {
                // depth-sort key: positive float bits order like the depths; the
                // sentinel puts elements without pairs last
                dkeys[idx] = ((f & 1u) && nt > 0) ? __float_as_uint(r1.z) : 0xFFFFFFFFu;
                dvals[idx] = packed_val((uint32_t)g, (uint32_t)nt, P.cshift);
            }
        }
    }
    // one atomic per wave for the counters
    unsigned long long bi = __ballot(n_invalid != 0);
    unsigned long long bf = __ballot(n_fp64 != 0);
    if (bi | bf) {
        int tot_i = n_invalid, tot_f = n_fp64;
        for (int off = 32; off > 0; off >>= 1) {
            tot_i += __shfl_xor(tot_i, off);
            tot_f += __shfl_xor(tot_f, off);
        }
        if ((threadIdx.x & 63) == 0) {
            if (tot_i) {
                status_add(status, ST_INVALID, (unsigned long long)tot_i);
                status_flag(status, (unsigned long long)FS_DEV_INVALID_GAUSS);
            }
            if (tot_f) status_add(status, ST_FP64, (unsigned long long)tot_f);
        }
    }
}

}  // namespace

hipError_t launch_project(hipStream_t s, const ProjTask *tasks, int32_t n_tasks, uint32_t n_blocks,
                          const SceneDev *scenes, const ViewDev *views, const ProjParams &p, float *rec,
                          int16_t *rect, int32_t *ntiles, uint8_t *flags, uint32_t *dkeys, uint32_t *dvals,
                          uint64_t *codes, unsigned long long *status)
{
    if (n_blocks == 0 || n_tasks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3(n_blocks), dim3(256), 0, s, tasks, n_tasks, scenes, views, p,
                       reinterpret_cast<float4 *>(rec), reinterpret_cast<short4 *>(rect), ntiles, flags, dkeys, dvals,
                       reinterpret_cast<ulonglong2 *>(codes), status);
    return hipGetLastError();
}

}  // namespace fs
