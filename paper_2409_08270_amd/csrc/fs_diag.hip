// Per-Gaussian diagnostics of a solved scene (the supplement's "Scene
// segmentation extension", its count of the objects each Gaussian contributes
// to, and the fewer-masks ablation of Sec. 4.8):
//   contrib[c]  Gaussians with exactly c objects e whose A[g][e] exceeds
//               rel_eps times the row's total (c = 0 also holds unseen rows);
//   member[m]   Gaussians that belong to exactly m rows of S (m > 1 happens
//               only for a negative bias, where the subsets may overlap);
//   overlap[e]  |S_e and gt = e|, |S_e|, |gt = e| against per-Gaussian labels,
//               from which a caller forms the IoU of each object.
// One read of A, S and gt; block histograms in LDS, one global atomic per bin.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kDiagLds = 4096;   // doubles of staged rows

__global__ __launch_bounds__(256) void k_diag_rows(const float *__restrict__ A_hi, const float *__restrict__ A_lo,
                                                   const uint8_t *__restrict__ S, const int32_t *__restrict__ gt,
                                                   int64_t n, int32_t E, int32_t rows_per_block, double rel_eps,
                                                   unsigned long long *__restrict__ contrib,
                                                   unsigned long long *__restrict__ member,
                                                   unsigned long long *__restrict__ overlap)
{
    __shared__ double s_a[kDiagLds];
    __shared__ uint32_t s_c[kMaxDiagE + 1], s_m[kMaxDiagE + 1], s_o[3 * kMaxDiagE];
    const int tid = threadIdx.x;
    for (int i = tid; i <= E; i += 256) s_c[i] = s_m[i] = 0;
    for (int i = tid; i < 3 * E; i += 256) s_o[i] = 0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int R = (int)min((int64_t)rows_per_block, n - r0);
    if (A_hi) {
        const int64_t base = r0 * E;
        for (int i = tid; i < R * E; i += 256) {
            double v = (double)A_hi[base + i];
            if (A_lo) v += (double)A_lo[base + i];
            s_a[i] = v;
        }
    }
    __syncthreads();
    for (int r = tid; r < R; r += 256) {
        const int64_t g = r0 + r;
        if (A_hi) {
            double tot = 0.0;
            for (int e = 0; e < E; ++e) tot += s_a[r * E + e];
            const double thr = rel_eps * tot;
            int c = 0;
            for (int e = 0; e < E; ++e) c += s_a[r * E + e] > thr ? 1 : 0;
            atomicAdd(&s_c[c], 1u);
        }
        if (S) {
            const int32_t truth = gt ? gt[g] : -1;
            int m = 0;
            for (int e = 0; e < E; ++e) {
                const bool in = S[(int64_t)e * n + g] != 0;
                m += in ? 1 : 0;
                if (gt && in) {
                    atomicAdd(&s_o[3 * e + 1], 1u);
                    if (truth == e) atomicAdd(&s_o[3 * e], 1u);
                }
            }
            atomicAdd(&s_m[m], 1u);
            if (gt && truth >= 0 && truth < E) atomicAdd(&s_o[3 * truth + 2], 1u);
        }
    }
    __syncthreads();
    for (int i = tid; i <= E; i += 256) {
        if (contrib && s_c[i]) atomicAdd(&contrib[i], (unsigned long long)s_c[i]);
        if (member && s_m[i]) atomicAdd(&member[i], (unsigned long long)s_m[i]);
    }
    for (int i = tid; i < 3 * E; i += 256)
        if (overlap && s_o[i]) atomicAdd(&overlap[i], (unsigned long long)s_o[i]);
}

}  // namespace

hipError_t launch_diag_rows(hipStream_t s, const float *A_hi, const float *A_lo, const uint8_t *S, const int32_t *gt,
                            int64_t n, int32_t E, double rel_eps, unsigned long long *contrib,
                            unsigned long long *member, unsigned long long *overlap)
{
    if (n == 0) return hipSuccess;
    int rows = kDiagLds / E;
    if (rows > 256) rows = 256;
    const int64_t blocks = (n + rows - 1) / rows;
    hipLaunchKernelGGL(k_diag_rows, dim3((unsigned)blocks), dim3(256), 0, s, A_hi, A_lo, S, gt, n, E, rows, rel_eps,
                       contrib, member, overlap);
    return hipGetLastError();
}

}  // namespace fs
