// Interactive follow-ups of the assignment (paper Sec. 3.2 "Regularized ILP
// for Noise Reduction", Sec. 4.2 and Sec. 4.4 "Object Removal"): once A is
// known, the background bias gamma can be swept at the cost of reading A once,
// and the Gaussians of an object are extracted or removed by stream compaction.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kSweepLds = 4160;     // doubles of staged rows (64 rows of 65)
constexpr int kSweepCounters = 4096;  // n_gamma * E counters per block

// S[k][t][g] = a_n > o_n + gamma_k for every gamma of the sweep, from one read
// of A (same arithmetic as the single assignment); counts[k][t] += members
// (counts may be NULL). A block stages `rows_per_block` rows; thread i takes
// object t = i / R and row i % R, so with R a multiple of 64 every wave holds
// one object and counts its members with one ballot per gamma (waves that
// straddle two objects fall back to one LDS atomic per member). Staged rows
// are E | 1 doubles apart, so that a wave reading one column of consecutive
// rows spreads over the LDS banks.
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
    const int stride = E | 1;
    const int64_t base = r0 * E;
    {
        // (r, e) of element i advance with i
        int r = tid / E, e = tid - (tid / E) * E;
        const int qd = 256 / E, qm = 256 - qd * E;
        for (int i = tid; i < R * E; i += 256) {
            double v = (double)A_hi[base + i];
            if (A_lo) v += (double)A_lo[base + i];
            s_a[r * stride + e] = v;
            r += qd;
            e += qm;
            if (e >= E) {
                e -= E;
                ++r;
            }
        }
    }
    __syncthreads();
    if (tid < R) {
        double tot = 0.0;
        // in order e = 0, 1, ...; unrolled so that several LDS reads are in flight
#pragma unroll 8
        for (int e = 0; e < E; ++e) tot += s_a[tid * stride + e];
        s_tot[tid] = tot;
    }
    __syncthreads();
    const int lane = tid & 63;
    // element i = t * R + r (object t, row r); (t, r) advance with i
    int ti = tid / R, ri = tid - (tid / R) * R;
    const int qd = 256 / R, qm = 256 - qd * R;
    for (int i0 = tid - lane; i0 < R * E; i0 += 256) {
        const int i = i0 + lane;
        const bool ok = i < R * E;
        const int t = ok ? ti : 0, r = ok ? ri : 0;
        ti += qd;
        ri += qm;
        if (ri >= R) {
            ri -= R;
            ++ti;
        }
        double an = 0.0, on = 1.0;
        if (ok) {
            const double a = s_a[r * stride + t];
            double o = s_tot[r] - a;
            if (o < 0.0) o = 0.0;
            const double s = fmax(a + o, 1e-12);
            an = a / s;
            on = o / s;
        }
        // the wave's lanes in range all hold object t0
        const int t0 = __builtin_amdgcn_readfirstlane(t);
        const bool one_obj = __ballot(ok && t != t0) == 0ull;
        // biases 8 at a time, their LDS reads issued together
        for (int k0 = 0; k0 < n_gamma; k0 += 8) {
            double gk[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) gk[j] = k0 + j < n_gamma ? (double)s_g[k0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k0 + j;
                if (k >= n_gamma) break;
                const bool in = ok && an > on + gk[j];
                if (S && ok) S[((int64_t)k * E + t) * n + r0 + r] = in ? 1 : 0;
                if (counts) {
                    if (one_obj) {
                        const unsigned long long b = __ballot(in);
                        if (lane == 0 && b) atomicAdd(&s_cnt[k * E + t0], (uint32_t)__popcll(b));
                    } else if (in) {
                        atomicAdd(&s_cnt[k * E + t], 1u);
                    }
                }
            }
        }
    }
    if (!counts) return;
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
    int rows = kSweepLds / (E | 1);
    if (rows > 256) rows = 256;
    if (rows >= 64) rows &= ~63;  // whole waves per object (E <= 63)
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
