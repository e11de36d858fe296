// Point-prompt propagation (paper Sec. 4.1 "2D mask generation and
// association" and the supplement's "Binary Mask Association"): each point
// prompt on a reference view is back-projected to the world at a given depth,
// the k Gaussian centres nearest to it (L2) are found, the one of least
// positive depth in the reference view is chosen, and its centre is projected
// into every view, giving the associated prompt of each view.
//
// One grid row (blockIdx.y) per prompt. The first kernel keeps a sorted
// k-list per thread over a grid-stride share of the Gaussians and reduces the
// block's lists to its k best; the second merges the per-block lists of one
// prompt in one workgroup.
//
// Compiled without floating-point contraction: the distances and depths decide
// which Gaussians are chosen, and they are evaluated in binary32 in a fixed
// order, so an independent implementation with the same order makes the same
// choice.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kMaxK = 32;

struct PromptCam {
    float R[9], t[3], fx, fy, cx, cy;
};

// world point of pixel (px, py) at camera depth d: R^T (d * K^-1 [px, py, 1] - t)
__device__ __forceinline__ void back_project(const PromptCam &c, float px, float py, float d, float &X, float &Y,
                                             float &Z)
{
#pragma clang fp contract(off)
    const float xc = d * ((px - c.cx) / c.fx) - c.t[0];
    const float yc = d * ((py - c.cy) / c.fy) - c.t[1];
    const float zc = d - c.t[2];
    X = (c.R[0] * xc + c.R[3] * yc) + c.R[6] * zc;
    Y = (c.R[1] * xc + c.R[4] * yc) + c.R[7] * zc;
    Z = (c.R[2] * xc + c.R[5] * yc) + c.R[8] * zc;
}

// key = (float bits of the squared distance) << 32 | id: non-negative floats
// order like their bit patterns, ties go to the smaller id
__device__ __forceinline__ unsigned long long dist_key(float X, float Y, float Z, float mx, float my, float mz,
                                                       uint32_t id)
{
#pragma clang fp contract(off)
    const float dx = mx - X, dy = my - Y, dz = mz - Z;
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    return ((unsigned long long)__float_as_uint(d2) << 32) | id;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// k smallest keys of the block's candidates, by k rounds of a block-wide minimum
// (each thread offers the head of its sorted list, the owner of the minimum pops it)
__device__ void block_select(unsigned long long (&list)[kMaxK], int k, unsigned long long *out)
{
    __shared__ unsigned long long s_w[4];
    int head = 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int r = 0; r < k; ++r) {
        const unsigned long long mine = head < k ? list[head] : ~0ull;
        const unsigned long long m = wave_min_u64(mine);
        if (lane == 0) s_w[w] = m;
        __syncthreads();
        unsigned long long best = s_w[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) best = s_w[i] < best ? s_w[i] : best;
        if (mine == best && best != ~0ull) ++head;  // keys are unique (they hold the id)
        if (threadIdx.x == 0) out[r] = best;
        __syncthreads();
    }
}

__device__ __forceinline__ void list_insert(unsigned long long (&list)[kMaxK], int k, unsigned long long key)
{
    if (key >= list[k - 1]) return;
    int i = k - 1;
    while (i > 0 && list[i - 1] > key) {
        list[i] = list[i - 1];
        --i;
    }
    list[i] = key;
}

__global__ __launch_bounds__(256) void k_knn_partial(GaussPtrs g, int64_t n, PromptCam ref,
                                                     const float *__restrict__ prompts, int32_t k,
                                                     unsigned long long *__restrict__ part)
{
    const float *pr = prompts + 3 * (int64_t)blockIdx.y;
    float X, Y, Z;
    back_project(ref, pr[0], pr[1], pr[2], X, Y, Z);
    unsigned long long list[kMaxK];
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) list[i] = ~0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        list_insert(list, k, dist_key(X, Y, Z, g.mx[i], g.my[i], g.mz[i], (uint32_t)i));
    block_select(list, k, part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * k);
}

__global__ __launch_bounds__(256) void k_knn_final(const unsigned long long *__restrict__ part, int32_t n_part,
                                                   GaussPtrs g, PromptCam ref, int32_t k,
                                                   const ViewDev *__restrict__ views, int32_t n_views, float znear,
                                                   long long *__restrict__ out_ids, float *__restrict__ out_uv,
                                                   uint8_t *__restrict__ out_vis)
{
    __shared__ unsigned long long s_top[kMaxK];
    __shared__ long long s_chosen;
    const int64_t prompt = blockIdx.x;
    part += prompt * n_part;
    out_ids += prompt * (1 + k);
    out_uv += prompt * n_views * 2;
    out_vis += prompt * n_views;
    unsigned long long list[kMaxK];
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) list[i] = ~0ull;
    for (int i = threadIdx.x; i < n_part; i += blockDim.x) list_insert(list, k, part[i]);
    block_select(list, k, s_top);
    if (threadIdx.x == 0) {
        // among the k nearest centres, the one of least positive depth in the reference view
        long long best = -1;
        float bz = 0.0f;
        for (int i = 0; i < k; ++i) {
            const unsigned long long key = s_top[i];
            if (key == ~0ull) {
                out_ids[1 + i] = -1;
                continue;
            }
            const uint32_t id = (uint32_t)(key & 0xFFFFFFFFull);
            out_ids[1 + i] = id;
            const float z = ((ref.R[6] * g.mx[id] + ref.R[7] * g.my[id]) + ref.R[8] * g.mz[id]) + ref.t[2];
            if (z > 0.0f && (best < 0 || z < bz || (z == bz && (long long)id < best))) {
                best = id;
                bz = z;
            }
        }
        out_ids[0] = best;
        s_chosen = best;
    }
    __syncthreads();
    const long long c = s_chosen;
    for (int v = threadIdx.x; v < n_views; v += blockDim.x) {
        float u = 0.0f, w = 0.0f;
        uint8_t vis = 0;
        if (c >= 0) {
            const ViewDev &C = views[v];
            const float mx = g.mx[c], my = g.my[c], mz = g.mz[c];
            const float x = ((C.R[0] * mx + C.R[1] * my) + C.R[2] * mz) + C.t[0];
            const float y = ((C.R[3] * mx + C.R[4] * my) + C.R[5] * mz) + C.t[1];
            const float z = ((C.R[6] * mx + C.R[7] * my) + C.R[8] * mz) + C.t[2];
            if (z > znear) {
                u = C.fx * (x / z) + C.cx;
                w = C.fy * (y / z) + C.cy;
                vis = (u >= 0.0f && u < (float)C.W && w >= 0.0f && w < (float)C.H) ? 1 : 0;
            }
        }
        out_uv[2 * v] = u;
        out_uv[2 * v + 1] = w;
        out_vis[v] = vis;
    }
}

}  // namespace

int prompt_max_k() { return kMaxK; }

hipError_t launch_prompt(hipStream_t s, const GaussPtrs &g, int64_t n, const ViewDev *views, int32_t n_views,
                         const ViewDev &ref_host, const float *prompts, int32_t n_prompts, int32_t k, float znear,
                         unsigned long long *part, int32_t n_part_blocks, long long *out_ids, float *out_uv,
                         uint8_t *out_vis)
{
    if (n_prompts == 0) return hipSuccess;
    PromptCam rc;
    for (int i = 0; i < 9; ++i) rc.R[i] = ref_host.R[i];
    for (int i = 0; i < 3; ++i) rc.t[i] = ref_host.t[i];
    rc.fx = ref_host.fx;
    rc.fy = ref_host.fy;
    rc.cx = ref_host.cx;
    rc.cy = ref_host.cy;
    hipLaunchKernelGGL(k_knn_partial, dim3((unsigned)n_part_blocks, (unsigned)n_prompts), dim3(256), 0, s, g, n, rc,
                       prompts, k, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_final, dim3((unsigned)n_prompts), dim3(256), 0, s, part, n_part_blocks * k, g, rc, k,
                       views, n_views, znear, out_ids, out_uv, out_vis);
    return hipGetLastError();
}

}  // namespace fs
