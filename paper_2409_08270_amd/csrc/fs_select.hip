// Interactive follow-ups of the assignment (paper Sec. 3.2 "Regularized ILP
// for Noise Reduction", Sec. 4.2 and Sec. 4.4 "Object Removal"): once A is
// known, the background bias gamma can be swept at the cost of reading A once,
// and the Gaussians of an object are extracted or removed by stream compaction.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kSweepLds = 4096;     // doubles of staged rows
constexpr int kSweepCounters = 4096;  // n_gamma * E counters per block

// S[k][t][g] = a_n > o_n + gamma_k for every gamma of the sweep, from one read
// of A (same arithmetic as the single assignment); counts[k][t] += members.
__global__ __launch_bounds__(256) void k_assign_sweep(const float *__restrict__ A_hi, const float *__restrict__ A_lo,
                                                      int64_t n, int32_t E, int32_t rows_per_block,
                                                      const float *__restrict__ gammas, int32_t n_gamma,
                                                      uint8_t *__restrict__ S,
                                                      unsigned long long *__restrict__ counts)
{
    __shared__ double s_a[kSweepLds];
    __shared__ double s_tot[256];
    __shared__ uint32_t s_cnt[kSweepCounters];
    __shared__ float s_g[64];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int R = (int)min((int64_t)rows_per_block, n - r0);
    const int tid = threadIdx.x;
    for (int i = tid; i < n_gamma * E; i += 256) s_cnt[i] = 0;
    if (tid < n_gamma) s_g[tid] = gammas[tid];
    const int64_t base = r0 * E;
    for (int i = tid; i < R * E; i += 256) {
        double v = (double)A_hi[base + i];
        if (A_lo) v += (double)A_lo[base + i];
        s_a[i] = v;
    }
    __syncthreads();
    if (tid < R) {
        double tot = 0.0;
        for (int e = 0; e < E; ++e) tot += s_a[tid * E + e];
        s_tot[tid] = tot;
    }
    __syncthreads();
    for (int i = tid; i < R * E; i += 256) {
        const int t = i / R, r = i % R;
        const double a = s_a[r * E + t];
        double o = s_tot[r] - a;
        if (o < 0.0) o = 0.0;
        const double s = fmax(a + o, 1e-12);
        const double an = a / s, on = o / s;
        for (int k = 0; k < n_gamma; ++k) {
            const bool in = an > on + (double)s_g[k];
            if (S) S[((int64_t)k * E + t) * n + r0 + r] = in ? 1 : 0;
            if (in) atomicAdd(&s_cnt[k * E + t], 1u);
        }
    }
    __syncthreads();
    for (int i = tid; i < n_gamma * E; i += 256)
        if (s_cnt[i]) atomicAdd(&counts[i], (unsigned long long)s_cnt[i]);
}

__global__ void k_select_flags(const uint8_t *__restrict__ select, int64_t n, int32_t keep_selected,
                               uint32_t *__restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = ((select[i] != 0) == (keep_selected != 0)) ? 1u : 0u;
}

struct Soa11 {
    const float *in[11];
    float *out[11];
};

__global__ void k_compact(Soa11 a, const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos, int64_t n,
                          int64_t *__restrict__ index_map)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t p = pos[i];
#pragma unroll
    for (int k = 0; k < 11; ++k) a.out[k][p] = a.in[k][i];
    if (index_map) index_map[p] = i;
}

unsigned grid_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int sweep_max_gammas(int32_t E) { return kSweepCounters / E < 64 ? kSweepCounters / E : 64; }

hipError_t launch_assign_sweep(hipStream_t s, const float *A_hi, const float *A_lo, int64_t n, int32_t E,
                               const float *gammas_dev, int32_t n_gamma, uint8_t *S, unsigned long long *counts)
{
    if (n == 0 || n_gamma == 0) return hipSuccess;
    int rows = kSweepLds / E;
    if (rows > 256) rows = 256;
    if (rows < 1) rows = 1;
    const int64_t blocks = (n + rows - 1) / rows;
    hipLaunchKernelGGL(k_assign_sweep, dim3((unsigned)blocks), dim3(256), 0, s, A_hi, A_lo, n, E, rows, gammas_dev,
                       n_gamma, S, counts);
    return hipGetLastError();
}

hipError_t launch_select_flags(hipStream_t s, const uint8_t *select, int64_t n, int32_t keep_selected, uint32_t *flags)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_flags, dim3(grid_of(n, 256)), dim3(256), 0, s, select, n, keep_selected, flags);
    return hipGetLastError();
}

hipError_t launch_compact(hipStream_t s, const float *const in[11], float *const out[11], const uint32_t *flags,
                          const uint32_t *pos, int64_t n, int64_t *index_map)
{
    if (n == 0) return hipSuccess;
    Soa11 a;
    for (int k = 0; k < 11; ++k) {
        a.in[k] = in[k];
        a.out[k] = out[k];
    }
    hipLaunchKernelGGL(k_compact, dim3(grid_of(n, 256)), dim3(256), 0, s, a, flags, pos, n, index_map);
    return hipGetLastError();
}

}  // namespace fs
