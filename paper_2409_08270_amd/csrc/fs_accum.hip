// a6: front-to-back alpha compositing with accumulation of every weight
// w = alpha * T into A[g][label(pixel)] (paper Eq. (1), Eq. (7)-(8),
// Listing 1 of the supplement).
//
// One workgroup of 256 threads composites one tile of 256 pixels; each wave
// owns an 8x8 block of the tile. The tile's depth-ordered list is staged
// through LDS in batches of 256 Gaussians (one coalesced gather per thread),
// and every thread walks the batch for its pixel.
//
// Scatter-add. The paper adds alpha*T with one atomic per (pixel, Gaussian).
// Here the distinct labels of the tile are compacted into slots (up to 64);
// a label that many lanes of a wave share is summed over the wave for 8
// Gaussians at once with a cross-lane reduce-scatter, the few lanes whose
// label is rare in their wave add their weights to LDS directly, the four
// waves combine in an LDS partial per (Gaussian, slot), and one global atomic
// per (tile, Gaussian, label) remains. The partials hold 2048 floats: a tile
// with up to 8 labels stages 256 Gaussians per batch, with 16, 32 or 64
// labels 128, 64 or 32. With A_lo, the exact rounding error of the global
// atomic (two-sum on the returned old value) goes to A_lo, so that
// A_hi + A_lo carries the sum to about one rounding; the partials of labels
// that only appear as stray pixels in a tile (relabel noise) are small and go
// to A_lo directly, without waiting for a returned value.
//
// Bit-reproducible sums (FS_RED_DET). Atomic float additions round in whatever
// order they arrive. In this mode every label of a wave is summed by the
// reduce-scatter (a fixed butterfly, so the same bits on every run), each such
// sum is rounded once to a 64-bit fixed-point integer, and from there on all
// additions (the tile's LDS partials, the global totals) are integer additions,
// which are exact and so independent of their order. The call's totals are
// then added into A_hi (and A_lo) once per entry.
#include <algorithm>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kPart = 2048;   // LDS partial sums: staged Gaussians x label slots
constexpr int kMaxSlots = 64; // distinct labels per tile handled by pre-reduction
constexpr int kBatch = 256;   // most Gaussians staged per batch
constexpr int kMajor = 4;     // a label held by this many lanes of a wave is summed across the wave
constexpr int kMinorStage = 4;  // minor lanes per wave whose weights go through the LDS staging area
constexpr float kLoFloor = -200.0f;  // floor of log2(opacity): 2^-200 is zero in float32

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// a 64-bit value that is the same in every lane, kept in scalar registers, so
// that loops over its bits are scalar loops
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// value of lane (lane ^ 8), within each 16-lane row (row rotate by 8)
__device__ __forceinline__ float dpp_xor8(float x) { return dpp_mov<0x128>(x); }

// value of lane (lane ^ 4): lanes in 4-lane banks 0 and 2 of a row take lane + 4
// (row shift left by 4), banks 1 and 3 take lane - 4 (row shift right by 4)
__device__ __forceinline__ float dpp_xor4(float x)
{
    const int xi = __float_as_int(x);
    int r = __builtin_amdgcn_update_dpp(xi, xi, 0x104, 0xF, 0x5, false);
    r = __builtin_amdgcn_update_dpp(r, xi, 0x114, 0xF, 0xA, false);
    return __int_as_float(r);
}

// Butterfly reduce-scatter of 8 per-lane values over the 64 lanes: on return,
// the eight lanes of octet e = lane >> 3 hold the sum over all lanes of x[e].
// Two halvings use the gfx950 lane-swap instructions (v_permlane32_swap:
// upper 32 lanes of the first operand <-> lower 32 lanes of the second;
// v_permlane16_swap: odd 16-lane rows of the first <-> even rows of the
// second), the rest are DPP lane moves (no LDS traffic). About 2.5
// instructions per value, against 11 for a full wave sum.
__device__ __forceinline__ float reduce_scatter8(const float (&x)[8])
{
    const int lane = threadIdx.x & 63;
    float s1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[k]), __float_as_uint(x[k + 4]), false, false);
        s1[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // entry k + 4*bit5(lane)
    }
    float s2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s1[k]), __float_as_uint(s1[k + 2]), false, false);
        s2[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // entry k + 2*bit4 + 4*bit5
    }
    const bool b3 = (lane >> 3) & 1;
    const float keep = b3 ? s2[1] : s2[0];
    const float send = b3 ? s2[0] : s2[1];
    float t = keep + dpp_xor8(send);                             // entry lane >> 3, 8 lanes summed
    t += dpp_xor4(t);
    t += dpp_mov<0xB1>(t);                                       // xor 1
    t += dpp_mov<0x4E>(t);                                       // xor 2
    return t;
}

// x in units of 2^-kFixShift, rounded to nearest (|x| < 2^29)
__device__ __forceinline__ unsigned long long to_fix(float x)
{
    return (unsigned long long)(long long)__builtin_rintf(x * 0x1p34f);
}
static_assert(kFixShift == 34, "to_fix scales by 2^34");

__device__ __forceinline__ void add_global(float *hi, float *lo, int64_t idx, float x)
{
    if (lo == nullptr) {
        unsafeAtomicAdd(hi + idx, x);
        return;
    }
    // exact two-sum of the value the atomic found and x
    const float old = unsafeAtomicAdd(hi + idx, x);
    const float s = old + x;
    const float bp = s - old;
    const float err = (old - (s - bp)) + (x - bp);
    if (err != 0.0f) unsafeAtomicAdd(lo + idx, err);
}

// Can any pixel centre of columns [x0, x1] and rows [y0, y1] of the 8x8 block
// with corner (bx, by) lie inside the ellipse p (dx + r dy)^2 + s dy^2 <= lim
// around (u, v)? Minimum of the quadratic over that box of pixel centres: zero
// if the mean is inside, else the least edge minimum (clamped parabola
// vertex; on a column x the vertex is at y = -p r x / (s + p r^2), on a row y
// at x = -r y). Conservative through the margin folded into lim; used only to
// skip work, never to decide a weight.
__device__ __forceinline__ bool block_hit(float u, float v, float p, float r, float s, float bx, float by, float lim,
                                          float x0, float x1, float y0, float y1)
{
    const float xl = bx + x0 + 0.5f - u, xh = bx + x1 + 0.5f - u;
    const float yl = by + y0 + 0.5f - v, yh = by + y1 + 0.5f - v;
    if (xl <= 0.0f && xh >= 0.0f && yl <= 0.0f && yh >= 0.0f) return true;
    const float pr = p * r;
    const float iC = __builtin_amdgcn_rcpf(fmaf(pr, r, s));
    auto q = [&](float x, float y) {
        const float e = fmaf(r, y, x);
        return fmaf(p * e, e, s * y * y);
    };
    float qmin = 3.4e38f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float x = i ? xh : xl;
        qmin = fminf(qmin, q(x, fminf(fmaxf(-(pr * x) * iC, yl), yh)));
        const float y = i ? yh : yl;
        qmin = fminf(qmin, q(fminf(fmaxf(-(r * y), xl), xh), y));
    }
    return qmin <= lim;
}

// Composites one tile (the whole workgroup); every thread calls it with the same tile.
template <bool PIX, bool COUNT, bool DET>
__device__ __forceinline__ void accum_tile(const uint32_t tile, const float4 *__restrict__ rec,
                                           const uint32_t *__restrict__ vals, const uint2 *__restrict__ ranges,
                                           const ViewDev *__restrict__ views, int32_t n_views,
                                           const SceneDev *__restrict__ scenes, const AccParams &P,
                                           float *__restrict__ t_final, int32_t *__restrict__ n_blend,
                                           float *__restrict__ tstate, uint8_t *__restrict__ tile_done,
                                           int32_t first, unsigned long long *__restrict__ status)
{
    // staged entry e: s_rec[e] = (u, v, p', r), (s', lo, thr, sup), with the LDL^T factors
    // p, s scaled to log2 units, lo = log2(opacity), sup = cut2 + lo (the support bound on the power) and
    // thr = max(sup, log2(alpha_min)): a weight is taken only if the power reaches thr, which
    // is the support test and the alpha_min test in one comparison; entry kBatch is a null record
    __shared__ float4 s_rec[2 * (kBatch + 1)];
    __shared__ uint32_t s_g[kBatch];
    __shared__ __align__(8) float s_part[kPart];  // [entry][stride]: partial sums per staged entry and slot
    // FS_RED_DET: the same memory as [entry][stride] 64-bit fixed-point partials
    unsigned long long *const s_part64 = reinterpret_cast<unsigned long long *>(s_part);
    __shared__ uint8_t s_wmask[kBatch];    // bit w: wave w's 8x8 block can be reached
    __shared__ __align__(16) uint32_t s_list[4][kBatch + 8];  // per-wave compacted entries (byte offsets
                                                               // into s_rec), padded with the null record
    __shared__ uint32_t s_bits[8];
    __shared__ uint8_t s_slot_label[kMaxSlots];  // labels are < n_classes <= 256
    __shared__ unsigned long long s_wslots[4];
    __shared__ unsigned long long s_tmajor;  // slots that are major in at least one wave of the tile
    __shared__ uint32_t s_misc[5];      // bad labels, longest wave walk, blends, evaluations, walked entries
    __shared__ int4 s_wbox[4];          // per wave: columns x0..x1, rows y0..y1 of its live pixels
    __shared__ __align__(16) float s_mstage[4][kMinorStage][8];  // per wave: 8 weights of each minor lane

    if (tile_done && tile_done[tile]) return;  // every pixel of this tile has finished (whole block)
    const int view = find_view_of_tile(views, n_views, tile);
    const ViewDev &C = views[view];
    const SceneDev &SC = scenes[C.scene];
    const uint8_t *__restrict__ masks = SC.masks;
    float *__restrict__ A_hi = SC.A_hi;
    float *__restrict__ A_lo = P.reduction == FS_RED_LDS2SUM ? SC.A_lo : nullptr;
    constexpr bool det = DET;  // P.reduction == FS_RED_DET
    unsigned long long *__restrict__ A_fix = SC.A_fix;
    const int E = SC.E;
    const uint32_t local = tile - C.tile_base;
    const int tx = (int)(local % (uint32_t)C.tiles_x), ty = (int)(local / (uint32_t)C.tiles_x);

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int bpr = P.tile_w >> 3;  // 8x8 blocks per tile row
    const int x = tx * P.tile_w + (w % bpr) * 8 + (lane & 7);
    const int y = ty * P.tile_h + (w / bpr) * 8 + (lane >> 3);
    const bool inside = x < C.W && y < C.H;
    const int64_t pix = (int64_t)C.mask_off + (int64_t)y * C.W + x;  // within the scene's masks
    const int64_t spix = (int64_t)C.pix_off + (int64_t)y * C.W + x;  // within the call's pixel state

    int lab = 0;
    bool active = inside;
    if (inside) {
        lab = masks[pix];
        if (lab >= E) active = false;
    }
    if (tid < 8) s_bits[tid] = 0;
    if (tid < 4) s_wslots[tid] = 0;
    if (tid == 0) s_tmajor = 0;
    if (tid < 5) s_misc[tid] = 0;
    __syncthreads();
    if (inside && !active && (first || tstate == nullptr)) atomicAdd(&s_misc[0], 1u);  // counted once per solve
    if (active) atomicOr(&s_bits[lab >> 5], 1u << (lab & 31));
    __syncthreads();
    int slot = 0, nslot = 0;
    {
        const int word = lab >> 5;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int pc = __popc(s_bits[i]);
            nslot += pc;
            if (i < word) slot += pc;
        }
        slot += __popc(s_bits[word] & ((1u << (lab & 31)) - 1u));
    }
    const bool plain = (P.reduction == FS_RED_PLAIN) || nslot > kMaxSlots;
    // partial layout: `stride` slots per staged entry, `bsz` entries per batch
    const int sh = nslot <= 8 ? 3 : (nslot <= 16 ? 4 : (nslot <= 32 ? 5 : 6));
    const int stride = 1 << sh;
    // (fixed-point partials take two words: half as many entries)
    const uint32_t bsz = min(plain ? (uint32_t)kBatch : (uint32_t)(kPart >> (det ? sh + 1 : sh)), (uint32_t)P.batch);
    if (active && !plain) {
        s_slot_label[slot] = (uint8_t)lab;
        atomicOr(&s_wslots[w], 1ull << slot);
    }
    __syncthreads();
    // labels held by at least kMajor lanes of this wave are summed across the
    // wave; the other lanes (minor) add their weights to LDS themselves
    unsigned long long wmajor = 0;
    {
        unsigned long long sl = uniform64(s_wslots[w]);
        while (sl) {
            const int sidx = __ffsll((long long)sl) - 1;
            sl &= sl - 1ull;
            if (__popcll(__ballot(active && slot == sidx)) >= (det ? 1 : kMajor)) wmajor |= 1ull << sidx;
        }
        wmajor = uniform64(wmajor);
    }
    if (lane == 0 && wmajor) atomicOr(&s_tmajor, wmajor);
    const bool minor = active && !plain && !((wmajor >> slot) & 1ull);
    const unsigned long long mmask = __ballot(minor);
    const bool wminor = mmask != 0ull;
    // Minor weights of a group of 8 entries: with at most kMinorStage minor lanes,
    // each writes its 8 weights to the wave's staging area and the 8 * (minor lanes)
    // lanes of the wave ("carriers": lane = 8 * minor rank + entry) each add one of
    // them to LDS, so one atomic instruction covers them all; with more minor
    // lanes, each adds its own nonzero weights.
    const int n_minor = __popcll(mmask);
    const bool mstage = n_minor <= kMinorStage;
    const int mrank = __popcll(mmask & ((1ull << lane) - 1ull));
    int carrier_slot = 0;
    const bool carrier = mstage && (lane >> 3) < n_minor;
    {
        // lane of the (lane >> 3)-th minor lane, then its slot
        unsigned long long mm = mmask;
        int src = 0;
        for (int m = 0; m < kMinorStage && mm; ++m) {
            const int l = __ffsll((long long)mm) - 1;
            mm &= mm - 1ull;
            if ((lane >> 3) == m) src = l;
        }
        carrier_slot = __shfl(slot, src);
    }
    if (tid == 0) {
        if (s_misc[0]) {
            status_add(status, ST_BAD_LABELS, (unsigned long long)s_misc[0]);
            status_flag(status, (unsigned long long)FS_DEV_BAD_LABEL);
        }
        if (nslot > kMaxSlots && P.reduction != FS_RED_PLAIN) status_flag(status, (unsigned long long)FS_DEV_MANY_LABELS);
    }
    for (int i = tid; i < kPart; i += 256) s_part[i] = 0.0f;
    if (tid == 0) {  // null record: far away, never inside its support, zero opacity
        s_rec[2 * kBatch] = make_float4(-1.0e6f, -1.0e6f, 0.0f, 0.0f);
        s_rec[2 * kBatch + 1] = make_float4(0.0f, kLoFloor, 3.0e38f, 3.0e38f);
    }

    const uint2 rg = ranges[tile];
    const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
    const float LOG2E = 1.4426950408889634f;
    // block-reach margin: 1/64 relative on k^2 (the weights use their own test)
    const float lim = -2.0f * P.cut2 / LOG2E * 1.015625f;
    const float tx0 = (float)(tx * P.tile_w), ty0 = (float)(ty * P.tile_h);
    float T = 1.0f;
    if (tstate && !first && active) {
        const float ts = tstate[spix];
        if (ts < 0.0f) active = false;  // this pixel's compositing ended in an earlier slab
        else T = ts;
    }
    uint32_t nb_l = 0, ne_l = 0;      // this pixel's blends and in-support evaluations
    uint32_t steps_w = 0;             // list entries this wave walked
    uint32_t staged = 0;              // list entries this block read (thread 0)
    bool live = active;
    const bool any_live = __syncthreads_or(live) != 0;
    const int64_t rec_base = (int64_t)C.elem_off;

    for (uint32_t base = any_live ? rg.x : rg.y; base < rg.y; base += bsz) {
        const uint32_t cnt = min(bsz, rg.y - base);
        staged += cnt;
        // the box of this wave's live pixels (lane = 8 * row + column): pixels only
        // ever finish, so entries that cannot reach the box cannot add a weight
        {
            const unsigned long long lm = __ballot(live);
            if (lane == 0) {
                uint32_t cols = 0;
                int r0 = 8, r1 = -1;
                for (int r = 0; r < 8; ++r) {
                    const uint32_t row = (uint32_t)(lm >> (8 * r)) & 0xFFu;
                    if (row) {
                        cols |= row;
                        r0 = min(r0, r);
                        r1 = r;
                    }
                }
                s_wbox[w] = cols ? make_int4(__ffs(cols) - 1, 31 - __clz(cols), r0, r1) : make_int4(1, 0, 1, 0);
            }
        }
        __syncthreads();  // previous batch fully consumed
        if ((uint32_t)tid < cnt) {
            const uint32_t g = vals[base + tid];
            const float4 r0 = rec[(rec_base + g) * 2];
            const float4 r1 = rec[(rec_base + g) * 2 + 1];
            const float lo = fmaxf(__builtin_amdgcn_logf(r1.y), kLoFloor);
            s_rec[2 * tid] = make_float4(r0.x, r0.y, -0.5f * LOG2E * r0.z, r0.w);
            s_rec[2 * tid + 1] = make_float4(-0.5f * LOG2E * r1.x, lo, fmaxf(P.cut2 + lo, P.lmin), P.cut2 + lo);
            s_g[tid] = g;
            // cull the waves whose live pixels the support cannot reach
            uint32_t m = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float bx = tx0 + (float)((b % bpr) * 8), by = ty0 + (float)((b / bpr) * 8);
                const int4 bb = s_wbox[b];
                if (bb.x <= bb.y && block_hit(r0.x, r0.y, r0.z, r0.w, r1.x, bx, by, lim, (float)bb.x,
                                              (float)bb.y, (float)bb.z, (float)bb.w))
                    m |= 1u << b;
            }
            s_wmask[tid] = (uint8_t)m;
        }
        __syncthreads();
        // each wave compacts the batch entries that can reach its block, in order
        int nlist = 0;
#pragma unroll
        for (int c = 0; c < kBatch / 64; ++c) {
            const int e = c * 64 + lane;
            const bool hit = (uint32_t)e < cnt && ((s_wmask[e] >> w) & 1u);
            const unsigned long long bm = __ballot(hit);
            if (hit) s_list[w][nlist + __popcll(bm & ((1ull << lane) - 1ull))] = (uint32_t)e * 32u;
            nlist += __popcll(bm);
        }
        if (lane < 8) s_list[w][nlist + lane] = (uint32_t)kBatch * 32u;  // pad the last group with the null record
        __builtin_amdgcn_wave_barrier();

        // one front-to-back step of this lane's pixel over a staged entry: power in
        // log2 units from the LDL^T factors, -(1/2) log2(e) (p (dx + r dy)^2 + s dy^2),
        // with log2(opacity) folded in, so that alpha = min(alpha_max, 2^(power + lo));
        // support and alpha_min tests against thr. A lane that fails them gets alpha = 0, which leaves T exactly as it is
        // and adds nothing. A pixel stops (Eq. (1)'s transmittance cut) at most once,
        // so the step where some lane does is fixed up under a wave-uniform branch:
        // that lane adds no weight and keeps its T.
        auto step = [&](const float4 q, const float4 q2) -> float {
            const float dx = pxc - q.x, dy = pyc - q.y;
            const float e = fmaf(q.w, dy, dx);
            const float pw = fmaf(q.z * e, e, fmaf(q2.x * dy, dy, q2.y));
            const bool ok = live && pw >= q2.z;
            const float alpha = ok ? fminf(P.alpha_max, __builtin_amdgcn_exp2f(pw)) : 0.0f;
            float wv = alpha * T;
            float Tn = fmaf(-T, alpha, T);
            // only a lane that takes a weight can stop: every other lane keeps a T
            // that is at least t_min (or 1 for pixels outside the image)
            const bool stop = Tn < P.t_min;
            if (__builtin_expect(__ballot(stop) != 0ull, 0)) {
                wv = stop ? 0.0f : wv;
                Tn = stop ? T : Tn;
            }
            if (COUNT) {
                ne_l += (live && pw >= q2.w) ? 1u : 0u;
                nb_l += (ok && !stop) ? 1u : 0u;
            }
            live = live && !stop;
            T = Tn;
            return wv;
        };
        auto rec_at = [&](uint32_t off) -> const float4 * {
            return reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_rec) + off);
        };
        // a wave's sum for (staged entry, slot) cell into the tile's partials
        auto part_add = [&](uint32_t cell, float tot) {
            if (det) atomicAdd(&s_part64[cell], to_fix(tot));
            else atomicAdd(&s_part[cell], tot);
        };

        if (__ballot(live) != 0ull) {
            if (!plain) {
                // the weights of 8 entries are summed at once, per major label of the wave
                const bool one = __popcll(wmajor) == 1 && !wminor;
                const int slot0 = __ffsll((long long)wmajor) - 1;
                for (int g0 = 0; g0 < nlist; g0 += 8) {
                    steps_w += 8;
                    float wr[8];
                    const uint4 o0 = *reinterpret_cast<const uint4 *>(&s_list[w][g0]);
                    const uint4 o1 = *reinterpret_cast<const uint4 *>(&s_list[w][g0 + 4]);
                    const uint32_t jj[8] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
                    // the next entry's record is read from LDS while this one is composited
                    float4 q = rec_at(jj[0])[0];
                    float4 q2 = rec_at(jj[0])[1];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        float4 qn = q;
                        float4 qn2 = q2;
                        if (k + 1 < 8) {
                            qn = rec_at(jj[k + 1])[0];
                            qn2 = rec_at(jj[k + 1])[1];
                        }
                        wr[k] = step(q, q2);
                        q = qn;
                        q2 = qn2;
                    }
                    const int e = lane >> 3;
                    const bool head = (lane & 7) == 0 && g0 + e < nlist;
                    if (one) {
                        const float tot = reduce_scatter8(wr);
                        if (head && tot != 0.0f) part_add(((s_list[w][g0 + e] >> 5) << sh) + slot0, tot);
                    } else {
                        if (wminor) {
                            if (mstage) {
                                // minor lanes stage their weights; carrier lane 8 m + k adds
                                // minor lane m's weight of entry k (padding entries weigh 0)
                                if (minor) {
                                    float4 *dst = reinterpret_cast<float4 *>(&s_mstage[w][mrank][0]);
                                    dst[0] = make_float4(wr[0], wr[1], wr[2], wr[3]);
                                    dst[1] = make_float4(wr[4], wr[5], wr[6], wr[7]);
                                }
                                __builtin_amdgcn_wave_barrier();
                                if (carrier) {
                                    const float val = s_mstage[w][lane >> 3][lane & 7];
                                    if (val != 0.0f)
                                        atomicAdd(&s_part[((s_list[w][g0 + (lane & 7)] >> 5) << sh) + carrier_slot], val);
                                }
                                __builtin_amdgcn_wave_barrier();
                            } else if (minor) {
                                // many rare labels: each lane adds its own nonzero weights
#pragma unroll
                                for (int k = 0; k < 8; ++k)
                                    if (wr[k] != 0.0f) atomicAdd(&s_part[((jj[k] >> 5) << sh) + slot], wr[k]);
                            }
                        }
                        // one reduce-scatter per major label of the wave (minor lanes never
                        // hold a major slot, so the selection leaves them out)
                        unsigned long long sl = wmajor;
                        while (sl) {
                            const int sidx = __ffsll((long long)sl) - 1;
                            sl &= sl - 1ull;
                            float v[8];
#pragma unroll
                            for (int k = 0; k < 8; ++k) v[k] = slot == sidx ? wr[k] : 0.0f;
                            const float tot = reduce_scatter8(v);
                            if (head && tot != 0.0f) part_add(((s_list[w][g0 + e] >> 5) << sh) + sidx, tot);
                        }
                    }
                    if (__ballot(live) == 0ull) break;
                }
            } else {
                // the paper's scheme: one global atomic per (pixel, Gaussian)
                for (int it = 0; it < nlist; ++it) {
                    steps_w += 1;
                    const uint32_t off = s_list[w][it];
                    const uint32_t j = off >> 5;
                    const float wgt = step(rec_at(off)[0], rec_at(off)[1]);
                    if (wgt != 0.0f) {
                        if (det) atomicAdd(A_fix + (int64_t)s_g[j] * E + lab, to_fix(wgt));
                        else add_global(A_hi, A_lo, (int64_t)s_g[j] * E + lab, wgt);
                    }
                    if ((it & 15) == 15 && __ballot(live) == 0ull) break;
                }
            }
        }
        __syncthreads();
        if (!plain) {
            // Partials of a slot that no wave holds in kMajor pixels (relabel noise) are
            // small; with A_lo they go there with a plain atomic (no returned value to
            // wait for), as A_lo only carries small values. The others take the two-sum.
            const unsigned long long tmajor = s_tmajor;
            auto flush = [&](int64_t idx, int sidx, float vpart) {
                if (A_lo != nullptr && !((tmajor >> sidx) & 1ull)) unsafeAtomicAdd(A_lo + idx, vpart);
                else add_global(A_hi, A_lo, idx, vpart);
            };
            if (det) {
                // fixed-point cells: exact integer additions into the call's totals
                for (uint32_t i = (uint32_t)tid; i < (cnt << sh); i += 256u) {
                    const int sidx = (int)(i & (uint32_t)(stride - 1));
                    const unsigned long long vpart = s_part64[i];
                    if (sidx < nslot && vpart != 0ull) {
                        atomicAdd(A_fix + (int64_t)s_g[i >> sh] * E + s_slot_label[sidx], vpart);
                        s_part64[i] = 0ull;
                    }
                }
            } else if (sh == 3) {
                if ((uint32_t)tid < cnt) {
                    const uint32_t g = s_g[tid];
                    for (int sidx = 0; sidx < nslot; ++sidx) {
                        const float vpart = s_part[(tid << 3) + sidx];
                        if (vpart != 0.0f) {
                            flush((int64_t)g * E + s_slot_label[sidx], sidx, vpart);
                            s_part[(tid << 3) + sidx] = 0.0f;
                        }
                    }
                }
            } else {
                // many labels, fewer entries: the block's threads share the (entry, slot) cells
                for (uint32_t i = (uint32_t)tid; i < (cnt << sh); i += 256u) {
                    const int sidx = (int)(i & (uint32_t)(stride - 1));
                    const float vpart = s_part[i];
                    if (sidx < nslot && vpart != 0.0f) {
                        flush((int64_t)s_g[i >> sh] * E + s_slot_label[sidx], sidx, vpart);
                        s_part[i] = 0.0f;
                    }
                }
            }
        }
        if (__syncthreads_or(live) == 0) break;
    }

    if (tile_done) {
        const bool still = __syncthreads_or(live) != 0;
        if (tid == 0 && !still) tile_done[tile] = 1;
    }
    if (inside && tstate) tstate[spix] = live ? T : -1.0f;
    if (inside) {
        if (t_final) t_final[pix] = T;
        if (PIX && n_blend) n_blend[pix] = (int32_t)nb_l;
    }
    // counters: summed over the wave, then the block in LDS, then one striped global atomic each
    uint32_t nb_w = nb_l, ne_w = ne_l;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nb_w += __shfl_xor(nb_w, off);
        ne_w += __shfl_xor(ne_w, off);
    }
    if (lane == 0) {
        atomicAdd(&s_misc[2], nb_w);
        atomicAdd(&s_misc[3], ne_w);
        atomicAdd(&s_misc[4], steps_w);
        atomicMax(&s_misc[1], steps_w);
    }
    __syncthreads();
    if (tid == 0) {
        if (s_misc[2]) status_add(status, ST_BLENDS, (unsigned long long)s_misc[2]);
        if (s_misc[3]) status_add(status, ST_EVALS, (unsigned long long)s_misc[3]);
        if (s_misc[4]) status_add(status, ST_WSTEPS, (unsigned long long)s_misc[4]);
        if (s_misc[1]) status_add(status, ST_WSTEPS_MAX, (unsigned long long)s_misc[1]);
        if (staged) status_add(status, ST_STAGED, (unsigned long long)staged);
    }
}

// One workgroup per work item (tile), or (PERSIST) resident workgroups that
// take the next item from the device counter `queue` until none is left.
template <bool PIX, bool COUNT, bool PERSIST, bool DET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_accum(
    const float4 *__restrict__ rec, const uint32_t *__restrict__ vals, const uint2 *__restrict__ ranges,
    const ViewDev *__restrict__ views, int32_t n_views, const SceneDev *__restrict__ scenes,
    const uint32_t *__restrict__ items, uint32_t n_items, AccParams P, float *__restrict__ t_final,
    int32_t *__restrict__ n_blend, float *__restrict__ tstate, uint8_t *__restrict__ tile_done, int32_t first,
    unsigned long long *__restrict__ status, uint32_t *__restrict__ queue)
{
    if (!PERSIST) {
        accum_tile<PIX, COUNT, DET>(items ? items[blockIdx.x] : blockIdx.x, rec, vals, ranges, views, n_views, scenes, P,
                               t_final, n_blend, tstate, tile_done, first, status);
        return;
    }
    __shared__ uint32_t s_next;
    // Control flow here is kept wave-uniform (scalar branches only): a lane-divergent
    // branch around the fetch (thread 0 alone) let the compiler route that lane and the
    // block's other lanes around the loop by different paths, so that the others passed
    // the barriers again, re-read the old item and never saw a new one.
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) == 0;
    for (;;) {
        // the previous tile's last LDS reads are behind the accum_tile's final barrier
        // or behind the two barriers here
        if (wave0) {
            // every lane of wave 0 takes part (lane 0 adds 1, the others 0); lane 0's
            // returned value is the counter before its own increment: this block's item
            const uint32_t old = atomicAdd(queue, (threadIdx.x & 63u) == 0u ? 1u : 0u);
            s_next = __builtin_amdgcn_readfirstlane(old);
        }
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (it >= n_items) break;
        accum_tile<PIX, COUNT, DET>(items ? items[it] : it, rec, vals, ranges, views, n_views, scenes, P, t_final,
                               n_blend, tstate, tile_done, first, status);
    }
}

// FS_RED_DET: the call's fixed-point totals into A_hi (+ A_lo), one thread per entry
__global__ __launch_bounds__(256) void k_fix_finish(const unsigned long long *__restrict__ fix, float *__restrict__ A_hi,
                                                    float *__restrict__ A_lo, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long q = (long long)fix[i];
    if (q == 0) return;
    const double v = (double)q * 0x1p-34;
    if (A_lo == nullptr) {
        A_hi[i] = (float)((double)A_hi[i] + v);
        return;
    }
    // v = vh + vl to about 2^-48 relative; A_hi + vh by an exact two-sum, the
    // error and vl into A_lo
    const float vh = (float)v;
    const float vl = (float)(v - (double)vh);
    const float a = A_hi[i];
    const float sum = a + vh;
    const float bp = sum - a;
    const float err = (a - (sum - bp)) + (vh - bp);
    A_hi[i] = sum;
    A_lo[i] = A_lo[i] + (err + vl);
}
static_assert(kFixShift == 34, "k_fix_finish scales by 2^-34");

// resident workgroups of a compositing kernel on this device (cached per kernel)
template <class K>
uint32_t resident_blocks(K kern)
{
    static int cached = 0;
    if (cached == 0) {
        int per_cu = 0, cus = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        cached = per_cu * cus;
    }
    return (uint32_t)cached;
}

// one compositing launch: a grid of one workgroup per item, or (p.persistent)
// the resident workgroups pulling items from `queue`
template <bool PIX, bool COUNT, bool DET>
hipError_t launch_k(hipStream_t s, const AccParams &p, uint32_t *queue, uint32_t n_items, const float *rec,
                    const uint32_t *vals, const uint32_t *ranges, const ViewDev *views, int32_t n_views,
                    const SceneDev *scenes, const uint32_t *items, float *t_final, int32_t *n_blend, float *tstate,
                    uint8_t *tile_done, int32_t first, unsigned long long *status)
{
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint2 *rg = reinterpret_cast<const uint2 *>(ranges);
    if (p.persistent) {
        if (!queue) return hipErrorInvalidValue;
        const uint32_t grid = std::min(n_items, resident_blocks(k_accum<PIX, COUNT, true, DET>));
        hipError_t e = launch_fill_u32(s, queue, 0u, 1);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_accum<PIX, COUNT, true, DET>), dim3(grid), dim3(256), 0, s, r4, vals, rg, views, n_views,
                           scenes, items, n_items, p, t_final, n_blend, tstate, tile_done, first, status, queue);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_accum<PIX, COUNT, false, DET>), dim3(n_items), dim3(256), 0, s, r4, vals, rg, views, n_views,
                       scenes, items, n_items, p, t_final, n_blend, tstate, tile_done, first, status, queue);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fix_finish(hipStream_t s, const unsigned long long *fix, float *A_hi, float *A_lo, int64_t count)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fix_finish, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, fix, A_hi, A_lo, count);
    return hipGetLastError();
}

hipError_t launch_accumulate(hipStream_t s, const float *rec, const uint32_t *vals, const uint32_t *ranges,
                             const ViewDev *views, int32_t n_views, const SceneDev *scenes, const uint32_t *items,
                             uint32_t n_items, const AccParams &p, float *t_final, int32_t *n_blend,
                             float *tstate, uint8_t *tile_done, int32_t first, unsigned long long *status,
                             uint32_t *queue)
{
    if (n_items == 0) return hipSuccess;
    const bool pix = t_final || n_blend;
    const bool count = p.count || n_blend;  // per-pixel blend counts need the counters
    if (p.reduction == FS_RED_DET)
        return pix ? (count ? launch_k<true, true, true>(s, p, queue, n_items, rec, vals, ranges, views, n_views,
                                                         scenes, items, t_final, n_blend, tstate, tile_done, first,
                                                         status)
                            : launch_k<true, false, true>(s, p, queue, n_items, rec, vals, ranges, views, n_views,
                                                          scenes, items, t_final, n_blend, tstate, tile_done, first,
                                                          status))
                   : (count ? launch_k<false, true, true>(s, p, queue, n_items, rec, vals, ranges, views, n_views,
                                                          scenes, items, t_final, n_blend, tstate, tile_done, first,
                                                          status)
                            : launch_k<false, false, true>(s, p, queue, n_items, rec, vals, ranges, views, n_views,
                                                           scenes, items, t_final, n_blend, tstate, tile_done, first,
                                                           status));
    return pix ? (count ? launch_k<true, true, false>(s, p, queue, n_items, rec, vals, ranges, views, n_views, scenes,
                                                      items, t_final, n_blend, tstate, tile_done, first, status)
                        : launch_k<true, false, false>(s, p, queue, n_items, rec, vals, ranges, views, n_views, scenes,
                                                       items, t_final, n_blend, tstate, tile_done, first, status))
               : (count ? launch_k<false, true, false>(s, p, queue, n_items, rec, vals, ranges, views, n_views, scenes,
                                                       items, t_final, n_blend, tstate, tile_done, first, status)
                        : launch_k<false, false, false>(s, p, queue, n_items, rec, vals, ranges, views, n_views,
                                                        scenes, items, t_final, n_blend, tstate, tile_done, first,
                                                        status));
}

}  // namespace fs
