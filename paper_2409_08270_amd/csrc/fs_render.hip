// Novel-view mask rendering (paper Sec. 3.4 "Depth-guided Novel View Mask
// Rendering" and the supplement's "Quantization in novel view mask").
//
// For every object e, the Gaussians labelled e (row e of S) are composited on
// their own, front to back, with the compositing rules of the accumulation
// pass: rho_e = sum of alpha*T (the object's alpha mask) and
// D_e = sum of alpha*T*z / rho_e (its depth where it is visible). The mask
// label is then either
//   depth-guided: the object with rho_e > tau of least D_e (0 if none), or
//   argmax:       argmax over all objects (background included) of rho_e.
//
// One workgroup renders one tile (one pixel per thread). The objects are
// taken kObj at a time: one walk over the tile's depth-ordered list serves all
// of them, since a Gaussian's alpha at a pixel does not depend on the object.
// The list is staged through LDS in batches with each entry's membership bits
// for those objects; entries that belong to none of them are compacted away
// with wave ballots, and every thread walks the rest, updating the
// transmittance, alpha mask and depth sum of each object the entry belongs to
// (a uniform loop over the entry's bits). Each object's arithmetic is the same
// sequence of operations as compositing it alone.
//
// The membership bits come from one byte per (group of kObj objects,
// Gaussian), built from S beforehand with reads that are contiguous along the
// Gaussians, so that staging an entry gathers one byte per group instead of
// one row of S per object.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kRBatch = 256;
constexpr int kObj = 8;  // objects composited in one walk of a tile's list

// memb[q][g], bit k: Gaussian g belongs to object e_first + kObj q + k
__global__ void k_member_bytes(const uint8_t *__restrict__ S, int64_t n, int32_t e_first, int32_t E,
                               uint8_t *__restrict__ memb)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    for (int q = 0, e0 = e_first; e0 < E; ++q, e0 += kObj) {
        uint32_t bits = 0;
        for (int k = 0; k < kObj && e0 + k < E; ++k) bits |= (S[(int64_t)(e0 + k) * n + g] != 0 ? 1u : 0u) << k;
        memb[(int64_t)q * n + g] = (uint8_t)bits;
    }
}

__global__ __launch_bounds__(256) void k_render(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                const uint2 *__restrict__ ranges, const ViewDev *__restrict__ views,
                                                int32_t n_views, const uint8_t *__restrict__ memb, int64_t n, int32_t E,
                                                AccParams P, float tau, int32_t mode, uint8_t *__restrict__ labels,
                                                float *__restrict__ rho_out, float *__restrict__ depth_out,
                                                int64_t n_pixels)
{
    __shared__ float4 s_q[kRBatch];   // u, v, p', r (LDL^T factors, p in log2 units)
    __shared__ float4 s_q2[kRBatch];  // c', lo, thr, z
    __shared__ uint8_t s_member[kRBatch];  // bit k: the entry belongs to object e0 + k
    __shared__ uint16_t s_list[kRBatch];
    __shared__ uint32_t s_wcnt[4];

    const uint32_t tile = blockIdx.x;
    const int view = find_view_of_tile(views, n_views, tile);
    const ViewDev &C = views[view];
    const uint32_t local = tile - C.tile_base;
    const int tx = (int)(local % (uint32_t)C.tiles_x), ty = (int)(local / (uint32_t)C.tiles_x);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int x = tx * P.tile_w + tid % P.tile_w;
    const int y = ty * P.tile_h + tid / P.tile_w;
    const bool inside = x < C.W && y < C.H;
    const int64_t pix = (int64_t)C.mask_off + (int64_t)y * C.W + x;
    const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
    const float LOG2E = 1.4426950408889634f;
    const uint2 rg = ranges[tile];
    const int64_t rec_base = (int64_t)C.elem_off;

    int best = 0;
    float best_d = 3.0e38f, best_rho = -1.0f;
    const int e_first = mode == 1 ? 0 : 1;
    for (int e0 = e_first; e0 < E; e0 += kObj) {
        const uint8_t *__restrict__ mq = memb + (int64_t)((e0 - e_first) / kObj) * n;
        const int ne = min(kObj, E - e0);
        float T[kObj], rho[kObj], dz[kObj];
#pragma unroll
        for (int k = 0; k < kObj; ++k) {
            T[k] = 1.0f;
            rho[k] = 0.0f;
            dz[k] = 0.0f;
        }
        // bit k: this pixel still composites object e0 + k
        uint32_t live = inside ? ((1u << ne) - 1u) : 0u;
        for (uint32_t base = rg.x; base < rg.y; base += kRBatch) {
            const uint32_t cnt = min((uint32_t)kRBatch, rg.y - base);
            __syncthreads();  // previous batch consumed
            uint32_t mbits = 0;
            if ((uint32_t)tid < cnt) {
                const uint32_t g = vals[base + tid];
                mbits = mq[g];
                if (mbits) {
                    const float4 r0 = rec[(rec_base + g) * 2];
                    const float4 r1 = rec[(rec_base + g) * 2 + 1];
                    const float lo = fmaxf(__builtin_amdgcn_logf(r1.y), -200.0f);
                    s_q[tid] = make_float4(r0.x, r0.y, -0.5f * LOG2E * r0.z, r0.w);
                    s_q2[tid] = make_float4(-0.5f * LOG2E * r1.x, lo, P.cut2 + lo, r1.z);
                    s_member[tid] = (uint8_t)mbits;
                }
            }
            // entries of the batch that belong to any of the objects, in list order:
            // per-wave ballots, then wave offsets
            const unsigned long long bm = __ballot(mbits != 0u);
            if (lane == 0) s_wcnt[w] = (uint32_t)__popcll(bm);
            __syncthreads();
            uint32_t before = 0, total = 0;
            for (int i = 0; i < 4; ++i) {
                const uint32_t c = s_wcnt[i];
                if (i < w) before += c;
                total += c;
            }
            if (mbits) s_list[before + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull))] = (uint16_t)tid;
            __syncthreads();
            if (live) {
                for (uint32_t i = 0; i < total; ++i) {
                    const uint32_t j = s_list[i];
                    const uint32_t mem = s_member[j] & live;
                    if (mem == 0u) continue;
                    const float4 q = s_q[j];
                    const float4 q2 = s_q2[j];
                    const float dx = pxc - q.x, dy = pyc - q.y;
                    const float e = fmaf(q.w, dy, dx);
                    const float pw = fmaf(q.z * e, e, fmaf(q2.x * dy, dy, q2.y));
                    if (pw < q2.z) continue;
                    const float alpha = fminf(P.alpha_max, __builtin_amdgcn_exp2f(pw));
                    if (alpha < P.alpha_min) continue;
                    // each object the entry belongs to, as if composited alone
#pragma unroll
                    for (int k = 0; k < kObj; ++k) {
                        if ((mem >> k) & 1u) {
                            const float Tn = fmaf(-T[k], alpha, T[k]);
                            if (Tn < P.t_min) {
                                live &= ~(1u << k);
                            } else {
                                const float wv = alpha * T[k];
                                rho[k] += wv;
                                dz[k] = fmaf(wv, q2.w, dz[k]);
                                T[k] = Tn;
                            }
                        }
                    }
                    if (live == 0u) break;
                }
            }
            if (__syncthreads_or(live != 0u) == 0) break;
        }
#pragma unroll
        for (int k = 0; k < kObj; ++k) {
            if (k >= ne) break;
            const int eo = e0 + k;
            const float d = rho[k] > 0.0f ? dz[k] / rho[k] : 3.0e38f;
            if (inside) {
                const int64_t o = (int64_t)eo * n_pixels + pix;
                if (rho_out) rho_out[o] = rho[k];
                if (depth_out) depth_out[o] = d;
            }
            if (mode == 1) {
                if (rho[k] > best_rho) {
                    best_rho = rho[k];
                    best = eo;
                }
            } else if (rho[k] > tau && d < best_d) {
                best_d = d;
                best = eo;
            }
        }
    }
    if (inside) labels[pix] = (uint8_t)best;
}

}  // namespace

hipError_t launch_render(hipStream_t s, const float *rec, const uint32_t *vals, const uint32_t *ranges,
                         const ViewDev *views, int32_t n_views, uint32_t n_tiles, const uint8_t *S, int64_t n,
                         int32_t E, const AccParams &p, float tau, int32_t mode, uint8_t *labels, float *rho,
                         float *depth, int64_t n_pixels, uint8_t *memb)
{
    if (n_tiles == 0) return hipSuccess;
    if (n > 0) {
        hipLaunchKernelGGL(k_member_bytes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, n,
                           mode == 1 ? 0 : 1, E, memb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_render, dim3(n_tiles), dim3(256), 0, s, reinterpret_cast<const float4 *>(rec), vals,
                       reinterpret_cast<const uint2 *>(ranges), views, n_views, memb, n, E, p, tau, mode, labels, rho,
                       depth, n_pixels);
    return hipGetLastError();
}

int64_t render_member_bytes(int64_t n, int32_t E, int32_t mode)
{
    const int e_first = mode == 1 ? 0 : 1;
    return n * (int64_t)((E - e_first + kObj - 1) / kObj);
}

}  // namespace fs
