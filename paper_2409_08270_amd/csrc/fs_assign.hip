// a7: closed-form assignment (paper Sec. 3.2 Eq. (7) and the background
// bias of "Regularized ILP for Noise Reduction"; Sec. 3.3 Eq. (8); Listing 1
// of the supplement). For Gaussian g and object t: a = A[g][t], o = sum of the other
// objects' contributions, (o_n, a_n) = (o, a) / max(o + a, 1e-12);
// S[t][g] = a_n > o_n + gamma (ties go to "others", the first index of the
// argmax); margin = |a_n - o_n - gamma|.
//
// The row total is formed once and reused for every object (the reuse the
// paper calls dynamic programming), in float64 from A_hi + A_lo: o = total - a
// is then exact to about 1e-16 of the row sum.
//
// Memory: A is row-major [n][E] (one row per Gaussian) and S is [E][n]. A
// block stages a tile of rows in LDS with coalesced loads and writes S and
// the margins column-tile by column-tile, so both sides stay coalesced. The
// staged rows are E | 1 doubles apart: consecutive lanes read one column of
// consecutive rows, and an even stride (E = 64: 512 bytes) would send them
// all to the same LDS banks.
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kLdsDoubles = 2080;  // staged rows, 16.25 KiB (eight blocks per CU): 32 rows of 65 doubles at E = 64

__global__ __launch_bounds__(256) void k_assign(const float *__restrict__ A_hi, const float *__restrict__ A_lo,
                                                int64_t n, int32_t E, int32_t rows_per_block, float gamma,
                                                uint8_t *__restrict__ S, float *__restrict__ margin,
                                                unsigned long long *__restrict__ status)
{
    __shared__ double s_a[kLdsDoubles];
    __shared__ double s_tot[256];
    __shared__ uint32_t s_members[256];
    __shared__ uint32_t s_cnt[3];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int R = (int)min((int64_t)rows_per_block, n - r0);
    const int tid = threadIdx.x;
    if (tid < 3) s_cnt[tid] = 0;
    const int stride = E | 1;
    // coalesced load of R rows x E columns; (r, e) of element i advance with i
    const int64_t base = r0 * E;
    {
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
        s_members[tid] = 0;
        if (tot == 0.0) atomicAdd(&s_cnt[0], 1u);
    }
    __syncthreads();
    const double gd = (double)gamma;
    uint32_t low = 0;
    // element i = t * R + r (object t, row r); (t, r) advance with i
    int t = tid / R, r = tid - (tid / R) * R;
    const int qd = 256 / R, qm = 256 - qd * R;
    for (int i = tid; i < R * E; i += 256) {
        const double a = s_a[r * stride + t];
        double o = s_tot[r] - a;
        if (o < 0.0) o = 0.0;
        const double s = fmax(a + o, 1e-12);
        const double an = a / s, on = o / s;
        const bool in = an > on + gd;
        const double m = fabs(an - on - gd);
        S[(int64_t)t * n + r0 + r] = in ? 1 : 0;
        if (margin) margin[(int64_t)t * n + r0 + r] = (float)m;
        if (in) atomicAdd(&s_members[r], 1u);
        if (m < 1e-4) low++;
        t += qd;
        r += qm;
        if (r >= R) {
            r -= R;
            ++t;
        }
    }
    if (low) atomicAdd(&s_cnt[2], low);
    __syncthreads();
    if (tid < R && s_members[tid] > 1) atomicAdd(&s_cnt[1], 1u);
    __syncthreads();
    if (tid == 0) {
        if (s_cnt[0]) status_add(status, ST_UNSEEN, (unsigned long long)s_cnt[0]);
        if (s_cnt[1]) status_add(status, ST_MULTI, (unsigned long long)s_cnt[1]);
        if (s_cnt[2]) status_add(status, ST_LOWMARGIN, (unsigned long long)s_cnt[2]);
    }
}

}  // namespace

hipError_t launch_assign(hipStream_t s, const float *A_hi, const float *A_lo, int64_t n, int32_t E, float gamma,
                         uint8_t *S, float *margin, unsigned long long *status)
{
    if (n == 0) return hipSuccess;
    int rows = kLdsDoubles / (E | 1);
    if (rows > 256) rows = 256;
    if (rows < 1) rows = 1;
    const int64_t blocks = (n + rows - 1) / rows;
    hipLaunchKernelGGL(k_assign, dim3((unsigned)blocks), dim3(256), 0, s, A_hi, A_lo, n, E, rows, gamma, S, margin,
                       status);
    return hipGetLastError();
}

}  // namespace fs
