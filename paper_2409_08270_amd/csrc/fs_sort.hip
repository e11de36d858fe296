// a2-a5: pair counting, scan, emission, stable sort and tile ranges (paper
// Sec. 3.1: the pixels of a 16x16 tile share one subset of Gaussians, which
// are blended in depth order).
//
// Order contract: within a tile, entries are ordered by depth, then by
// Gaussian id. It is reached in two stable sorts: the visible Gaussians of
// every view are sorted by the float bits of their depth (positive floats
// order like their bit patterns; ties keep id order because the input is in
// id order and the sort is stable), their tile pairs are emitted in that
// order, and the pairs are then sorted stably by tile id. Sorting N depth
// keys plus P 16-bit tile keys moves far fewer bytes than sorting P
// (tile, depth) 48-bit keys.
#include "fs_internal.h"
#include "fs_tiles.h"

namespace fs {
namespace {

constexpr int kThreads = 256;
// rows of an emission block whose element is looked up in a table rather than
// by a binary search in the row offsets (a multiple of 256: one choice per wave)
constexpr uint32_t kRowMap = 2048;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096 items per block tile
constexpr int kWaves = kThreads / 64;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- scan ----
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// exclusive scan of the block's values (one per thread), returns block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *s_wsum, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan_u32(x);
    if (lane == 63) s_wsum[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int i = 0; i < kWaves; ++i) {
        uint32_t s = s_wsum[i];
        if (i < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - x;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                          uint32_t *__restrict__ sums)
{
    __shared__ uint32_t s_wsum[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + k * kThreads + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    block_excl_scan(acc, s_wsum, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of block tile blockIdx.x. The tile's offset is offs[b] or,
// with `raw`, the sum of the block totals offs[0 .. b), added up here (this
// saves scanning the totals in a launch of their own).
__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                        int64_t n, const uint32_t *__restrict__ offs,
                                                        uint32_t *__restrict__ total_out, int32_t raw)
{
    __shared__ uint32_t s_wsum[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    // 16-byte accesses where the thread's 16 elements are whole and aligned
    const bool vec = base + kItems <= n &&
                     ((reinterpret_cast<uintptr_t>(in + base) | reinterpret_cast<uintptr_t>(out + base)) & 15u) == 0;
    uint32_t v[kItems];
    uint32_t acc = 0;
    if (vec) {
#pragma unroll
        for (int q = 0; q < kItems / 4; ++q) {
            const uint4 x = *reinterpret_cast<const uint4 *>(in + base + 4 * q);
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            int64_t i = base + k;
            v[k] = i < n ? in[i] : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) acc += v[k];
    uint32_t pre = 0;
    if (offs && raw) {
        uint32_t part = 0;
        for (int i = threadIdx.x; i < (int)blockIdx.x; i += kThreads) part += offs[i];
        uint32_t all;
        block_excl_scan(part, s_wsum, all);
        pre = all;
    } else if (offs) {
        pre = offs[blockIdx.x];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(acc, s_wsum, tot) + pre;
    if (vec) {
#pragma unroll
        for (int q = 0; q < kItems / 4; ++q) {
            uint4 y;
            y.x = ex;
            ex += v[4 * q];
            y.y = ex;
            ex += v[4 * q + 1];
            y.z = ex;
            ex += v[4 * q + 2];
            y.w = ex;
            ex += v[4 * q + 3];
            *reinterpret_cast<uint4 *>(out + base + 4 * q) = y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            int64_t i = base + k;
            if (i < n) out[i] = ex;
            ex += v[k];
        }
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) *total_out = ex;
}

// ------------------------------------------------------------ radix sort --
// Digit histogram of one block tile. Each thread reads 16 consecutive keys and
// adds runs of equal digits with one LDS atomic per run: keys emitted per
// Gaussian in tile order repeat their high digit, which would otherwise
// serialise the atomics.
// A block handles `tpb` consecutive block tiles of kTile items (a super-tile),
// so that large sorts keep their digit tables small: one histogram row per
// super-tile. Segment of block b: the last segment whose first block is <= b
// (segments' blk0 count super-tiles).
struct SegInfo {
    int64_t base;     // first element of this super-tile
    int nvalid;       // valid items in the super-tile
    uint32_t bps;     // super-tiles of the segment
    uint32_t lb;      // super-tile index inside the segment
    uint32_t blk0;
    uint32_t kbase;   // added to count indexes
};

__device__ __forceinline__ SegInfo seg_of_block(const SegDev *__restrict__ segs, int32_t n_segs, uint32_t b,
                                                const uint32_t *__restrict__ len_dev, int32_t tpb)
{
    int lo = 0, hi = n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
    }
    const SegDev sg = segs[lo];
    const int64_t span = (int64_t)kTile * tpb;
    SegInfo r;
    r.blk0 = sg.blk0;
    r.lb = b - sg.blk0;
    r.bps = (uint32_t)(((int64_t)sg.len + span - 1) / span);
    uint32_t len = min(sg.len, sg.alen);
    if (len_dev) len = min(len, *len_dev);
    r.kbase = sg.kbase;
    const int64_t rem = (int64_t)len - (int64_t)r.lb * span;
    r.nvalid = rem <= 0 ? 0 : (rem < span ? (int)rem : (int)span);
    r.base = (int64_t)sg.off + (int64_t)r.lb * span;
    return r;
}

// Digit histogram of one super-tile. Each thread reads 4 groups of 4
// consecutive keys per block tile (16-byte loads, consecutive lanes on
// consecutive addresses) and adds runs of equal digits with one LDS atomic per
// run: keys emitted per Gaussian in tile order repeat their high digit, which
// would otherwise serialise the atomics. Counts are stored
// [segment][digit][block] so that one exclusive scan over the whole table
// gives every block's output positions.
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                         const SegDev *__restrict__ segs, int32_t n_segs,
                                                         int32_t shift, uint32_t *__restrict__ hist,
                                                         const uint32_t *__restrict__ len_dev, int32_t tpb,
                                                         uint32_t dmask)
{
    __shared__ uint32_t s_h[kWaves][256];
    const SegInfo si = seg_of_block(segs, n_segs, blockIdx.x, len_dev, tpb);
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) (&s_h[0][0])[i] = 0;
    __syncthreads();
    uint32_t run_d = 0xFFFFFFFFu, run_n = 0;
    for (int tb = 0; tb * kTile < si.nvalid; ++tb) {
        const int nvalid = min(kTile, si.nvalid - tb * kTile);
        const uint32_t *k = keys + si.base + (int64_t)tb * kTile;
        if (nvalid == kTile) {
            const bool aligned = ((reinterpret_cast<uintptr_t>(k) & 15u) == 0);
            // all four loads are issued before any is used, so that each thread
            // keeps 64 bytes in flight
            uint4 xq[kItems / 4];
#pragma unroll
            for (int q = 0; q < kItems / 4; ++q) {
                const int i0 = 4 * (q * kThreads + threadIdx.x);
                if (aligned) xq[q] = *reinterpret_cast<const uint4 *>(k + i0);
                else xq[q] = make_uint4(k[i0], k[i0 + 1], k[i0 + 2], k[i0 + 3]);
            }
#pragma unroll
            for (int q = 0; q < kItems / 4; ++q) {
                const uint4 x = xq[q];
                const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t d = (xs[e] >> shift) & dmask;
                    if (d != run_d) {
                        if (run_n) atomicAdd(&s_h[w][run_d], run_n);
                        run_d = d;
                        run_n = 0;
                    }
                    run_n++;
                }
            }
        } else {
            for (int it = 0; it < kItems; ++it) {
                const int i = it * kThreads + threadIdx.x;
                if (i >= nvalid) break;
                const uint32_t d = (k[i] >> shift) & dmask;
                if (d != run_d) {
                    if (run_n) atomicAdd(&s_h[w][run_d], run_n);
                    run_d = d;
                    run_n = 0;
                }
                run_n++;
            }
        }
    }
    if (run_n) atomicAdd(&s_h[w][run_d], run_n);
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) c += s_h[i][d];
    hist[(int64_t)si.blk0 * 256 + (int64_t)d * si.bps + si.lb] = c;
}

// Stable scatter of one super-tile, block tile after block tile: wave w ranks
// the contiguous items [w*1024, (w+1)*1024) of the block tile in 16 rounds of
// 64, equal digits matched with 8 ballots; each digit's output cursor then
// advances by the block tile's count of that digit.
// On the last pass the staged block tile is ordered by the sorted key bits,
// so runs of equal keys (k >> kshift) are contiguous in LDS: with key_count,
// each run adds its length to count[kbase + (k >> kshift)] (+end at its last
// item, -start at its first, which sums to the length whatever the order of
// the atomics). kout and vout may be NULL; without vin (keys only), vout
// receives k & vmask.
// VALS = false: keys only (vin is not read, no value staging in LDS). The
// 128-VGPR budget keeps four blocks on a CU (a tighter one spills and is slower).
template <bool VALS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                            uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            const SegDev *__restrict__ segs, int32_t n_segs,
                                                            int32_t shift, const uint32_t *__restrict__ offs,
                                                            const uint32_t *__restrict__ len_dev, int32_t tpb,
                                                            uint32_t *__restrict__ key_count, uint32_t dmask,
                                                            int32_t kshift, uint32_t vmask)
{
    __shared__ uint32_t s_cnt[kWaves][256];
    __shared__ uint32_t s_dstart[256];
    __shared__ uint32_t s_gofs[256];
    __shared__ uint32_t s_wsum[kWaves];
    __shared__ uint32_t s_k[kTile];
    __shared__ uint32_t s_v[VALS ? kTile : 1];

    const SegInfo si = seg_of_block(segs, n_segs, blockIdx.x, len_dev, tpb);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // s_gofs comes from one exclusive scan over the [segment][digit][block]
    // counts of all segments, so it is already a position in the whole array
    s_gofs[threadIdx.x] = offs[(int64_t)si.blk0 * 256 + (int64_t)threadIdx.x * si.bps + si.lb];
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int dbits = 32 - __clz(dmask);  // digit width (dmask is 2^dbits - 1)

    for (int tb = 0; tb * kTile < si.nvalid; ++tb) {
        const int nvalid = min(kTile, si.nvalid - tb * kTile);
        const uint32_t *kbase = kin + si.base + (int64_t)tb * kTile;
        const uint32_t *vbase = VALS ? vin + si.base + (int64_t)tb * kTile : nullptr;
        for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) (&s_cnt[0][0])[i] = 0;
        __syncthreads();

        uint32_t key[kItems], val[VALS ? kItems : 1], rnk[kItems];
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int li = w * (kItems * 64) + r * 64 + lane;
            const bool ok = li < nvalid;
            key[r] = ok ? kbase[li] : 0xFFFFFFFFu;
            if constexpr (VALS) val[r] = ok ? vbase[li] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const uint32_t d = (key[r] >> shift) & dmask;
            // lanes whose digit equals this lane's: for every bit, the lanes that
            // agree with it are ~(ballot ^ m), m = all ones if the bit is set
            // (one three-input bit operation per half of the 64-bit mask)
            uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                if (bit >= dbits) break;
                const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, (unsigned)bit, 1u);
                const unsigned long long bb = __ballot(m != 0u);
                plo &= ~((uint32_t)bb ^ m);
                phi &= ~((uint32_t)(bb >> 32) ^ m);
            }
            const unsigned long long peers = ((unsigned long long)phi << 32) | plo;
            const uint32_t before = s_cnt[w][d];
            rnk[r] = before + (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if ((peers & lt) == 0ull) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // per-digit totals, wave prefixes and the digit starts inside the block tile
        uint32_t tile_count;
        {
            const int d = threadIdx.x;
            uint32_t run = 0;
#pragma unroll
            for (int i = 0; i < kWaves; ++i) {
                const uint32_t c = s_cnt[i][d];
                s_cnt[i][d] = run;
                run += c;
            }
            uint32_t tot;
            const uint32_t ex = block_excl_scan(run, s_wsum, tot);
            s_dstart[d] = ex;
            tile_count = run;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const uint32_t d = (key[r] >> shift) & dmask;
            const uint32_t pos = s_dstart[d] + s_cnt[w][d] + rnk[r];
            s_k[pos] = key[r];
            if constexpr (VALS) s_v[pos] = val[r];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nvalid; i += kThreads) {
            const uint32_t k = s_k[i];
            const uint32_t d = (k >> shift) & dmask;
            const int64_t p = (int64_t)s_gofs[d] + (i - (int64_t)s_dstart[d]);
            if (kout) kout[p] = k;
            if (vout) {
                if constexpr (VALS) vout[p] = s_v[i];
                else vout[p] = k & vmask;
            }
            if (key_count) {
                const uint32_t kk = k >> kshift;
                uint32_t *cnt = key_count + si.kbase + kk;
                if (i + 1 == nvalid || (s_k[i + 1] >> kshift) != kk) atomicAdd(cnt, (uint32_t)(i + 1));
                if (i > 0 && (s_k[i - 1] >> kshift) != kk) atomicSub(cnt, (uint32_t)i);
            }
        }
        __syncthreads();
        s_gofs[threadIdx.x] += tile_count;
    }
}

// ------------------------------------------------------------- binning ---
__global__ void k_depth_keys(const float4 *__restrict__ rec, const int32_t *__restrict__ ntiles,
                             const uint8_t *__restrict__ flags, const ViewDev *__restrict__ views, int32_t n_views,
                             int64_t total, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int v = find_view_of_elem(views, n_views, i);
    const bool emits = (flags[i] & 1) && ntiles[i] > 0;
    keys[i] = emits ? __float_as_uint(rec[2 * i + 1].z) : 0xFFFFFFFFu;
    vals[i] = (uint32_t)(i - (int64_t)views[v].elem_off);
}

__global__ void k_gather_counts(const uint32_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                                const int32_t *__restrict__ ntiles, const ViewDev *__restrict__ views,
                                int32_t n_views, int64_t total, uint32_t *__restrict__ counts, int32_t cshift)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    if (skeys[i] == 0xFFFFFFFFu) {
        counts[i] = 0u;
        return;
    }
    const uint32_t vv = svals[i];
    if (cshift != 0 && (vv >> cshift) < count_sat(cshift)) {
        counts[i] = vv >> cshift;  // the count travels with the value
        return;
    }
    const int v = find_view_of_elem(views, n_views, i);
    counts[i] = (uint32_t)ntiles[(int64_t)views[v].elem_off + val_id(vv, cshift)];
}

// Depth-slab pair counts. An element outside the slab counts 0; inside, its
// listed tiles (the row_span rule) that are not yet marked done.
__device__ __forceinline__ bool in_slab(const ViewDev &C, int64_t i, Slab sl)
{
    const uint64_t r = (uint64_t)(i - (int64_t)C.elem_off);
    const uint64_t lo = ((uint64_t)C.n * sl.num_lo) >> 10, hi = ((uint64_t)C.n * sl.num_hi) >> 10;
    return r >= lo && r < hi;
}

__global__ void k_slab_counts(const uint32_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                              const float4 *__restrict__ rec, const short4 *__restrict__ rect,
                              const uint8_t *__restrict__ flags, const int32_t *__restrict__ ntiles,
                              const ViewDev *__restrict__ views, int32_t n_views, int64_t total, Slab sl,
                              const uint8_t *__restrict__ done, int32_t tw, int32_t th, float sigma_k,
                              const ulonglong2 *__restrict__ codes, uint32_t *__restrict__ counts, int32_t cshift)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    uint32_t c = 0;
    if (skeys[i] != 0xFFFFFFFFu) {
        const uint32_t vv = svals[i];
        // the count travels with the value unless it saturated
        const bool carried = cshift != 0 && (vv >> cshift) < count_sat(cshift);
        if (done == nullptr && carried && sl.num_lo == 0 && sl.num_hi >= 1024) {
            c = vv >> cshift;  // one slab holds every element: no view lookup
        } else {
            const int v = find_view_of_elem(views, n_views, i);
            const ViewDev &C = views[v];
            if (in_slab(C, i, sl)) {
                const int64_t idx = (int64_t)C.elem_off + val_id(vv, cshift);
                if (done == nullptr) {
                    c = carried ? (vv >> cshift) : (uint32_t)ntiles[idx];
                } else {
                    short4 rc;
                    SpanCode code;
                    load_emit_record(codes, rect, idx, code, rc);
                    Span32 sp = make_span32(0.f, 0.f, 1.f, 0.f, 1.f, true, 1.0f);
                    if (!has_code(code)) {
                        const float4 r0 = rec[2 * idx];
                        const float4 r1 = rec[2 * idx + 1];
                        sp = make_span32(r0.x, r0.y, r0.z, r0.w, r1.x, r1.w != 0.0f, support_limit(sigma_k));
                    }
                    for (int ty = rc.y; ty <= rc.w; ++ty) {
                        int l, r;
                        const bool any = has_code(code) ? code_span(code, ty - rc.y, rc.x, l, r)
                                                        : row_span(sp, ty, rc.x, rc.z, tw, th, C.W, C.H, l, r);
                        if (!any) continue;
                        const uint8_t *d = done + C.tile_base + (uint32_t)ty * (uint32_t)C.tiles_x;
                        for (int t = l; t <= r; ++t) c += d[t] ? 0u : 1u;
                    }
                }
            }
        }
    }
    counts[i] = c;
}

// Inclusive sum of x over the block's threads; *total receives the block sum.
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t x, uint32_t *s_wsum, uint32_t *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    uint32_t t = 0;
    for (int k = 0; k < kWaves; ++k) {
        if (k < w) x += s_wsum[k];
        t += s_wsum[k];
    }
    *total = t;
    __syncthreads();
    return x;
}

// Emission of the (tile, Gaussian) pairs. Block b handles the depth-sorted
// elements [256 b, 256 b + 256), whose outputs form one contiguous range from
// offsets[256 b]. Splats differ widely in their number of tile rows and of
// tiles, so the block lists the rows of its elements together: a block prefix
// sum of the row counts concatenates them, and in rounds of 256 rows every
// thread takes one row (a binary search in LDS finds its element), takes the
// row's span (span code or the row_span rule, as in the count, without the
// tiles already finished), and a block prefix sum of the rows' pair counts
// gives each row its place in the output, where the thread writes its pairs.
__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
                                                   const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ counts,
                                                   const float4 *__restrict__ rec, const short4 *__restrict__ rect,
                                                   const uint8_t *__restrict__ flags, const ViewDev *__restrict__ views,
                                                   int32_t n_views, int64_t total, uint32_t capacity, int32_t tw, int32_t th,
                                                   float sigma_k, const uint8_t *__restrict__ done,
                                                   uint32_t *__restrict__ tiles_out,
                                                   uint32_t *__restrict__ vals_out, unsigned long long *__restrict__ status,
                                                   int32_t gbits, const ulonglong2 *__restrict__ codes, int32_t cshift)
{
    __shared__ Span32 s_span[kThreads];
    __shared__ ulonglong2 s_code[kThreads];
    __shared__ short4 s_rc[kThreads];
    __shared__ uint4 s_vw[kThreads];        // tile base, tiles per row, width, height of the element's view
    __shared__ uint32_t s_g[kThreads];
    __shared__ uint32_t s_roff[kThreads + 1];
    __shared__ uint32_t s_wsum[kWaves];
    __shared__ uint32_t s_lo;
    __shared__ uint8_t s_rowelem[kRowMap];  // the element of each of the block's first kRowMap rows
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kThreads;
    const int64_t i = b0 + tid;
    const bool live = i < total && skeys[i] != 0xFFFFFFFFu;
    const uint32_t cnt = live ? counts[i] : 0u;
    if (tid == 0) s_lo = offsets[b0];

    uint32_t rows = 0;
    if (cnt > 0) {
        const int vw = find_view_of_elem(views, n_views, i);
        const uint32_t g = val_id(svals[i], cshift);
        const ViewDev &C = views[vw];
        const int64_t idx = (int64_t)C.elem_off + g;
        short4 rc;
        SpanCode code;
        load_emit_record(codes, rect, idx, code, rc);
        Span32 sp = make_span32(0.f, 0.f, 1.f, 0.f, 1.f, true, 1.0f);
        if (!has_code(code)) {
            const float4 r0 = rec[2 * idx];
            const float4 r1 = rec[2 * idx + 1];
            // rec's mark: non-zero for splats that list their whole rectangle
            sp = make_span32(r0.x, r0.y, r0.z, r0.w, r1.x, r1.w != 0.0f, support_limit(sigma_k));
        }
        s_span[tid] = sp;
        s_code[tid] = make_ulonglong2(code.lo, code.hi);
        s_rc[tid] = rc;
        s_vw[tid] = make_uint4(C.tile_base, (uint32_t)C.tiles_x, (uint32_t)C.W, (uint32_t)C.H);
        s_g[tid] = g;
        rows = (uint32_t)(rc.w - rc.y + 1);
    }
    uint32_t n_rows = 0;
    const uint32_t incl = block_scan_incl(rows, s_wsum, &n_rows);
    s_roff[tid + 1] = incl;
    if (tid == 0) s_roff[0] = 0;
    for (uint32_t r = incl - rows; r < min(incl, kRowMap); ++r) s_rowelem[r] = (uint8_t)tid;
    __syncthreads();
    const uint32_t lo = s_lo;

    uint32_t dropped = 0, carry = 0;
    for (uint32_t c0 = 0; c0 < n_rows; c0 += kThreads) {
        const uint32_t item = c0 + (uint32_t)tid;
        int e = 0, l = 0, r = -1;
        uint32_t n = 0;
        if (item < n_rows) {
            // the element e with s_roff[e] <= item < s_roff[e + 1]: from the map,
            // or by a binary search past its end (the same choice for the whole wave)
            if (item < kRowMap) {
                e = s_rowelem[item];
            } else {
                int a = 0, b = kThreads - 1;
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (s_roff[mid] <= item) a = mid; else b = mid - 1;
                }
                e = a;
            }
            const short4 rc = s_rc[e];
            const int row = (int)(item - s_roff[e]);
            const ulonglong2 cw = s_code[e];
            const SpanCode code{cw.x, cw.y};
            const uint4 vw = s_vw[e];
            const bool any = has_code(code) ? code_span(code, row, rc.x, l, r)
                                            : row_span(s_span[e], rc.y + row, rc.x, rc.z, tw, th, (int)vw.z, (int)vw.w, l, r);
            if (any) {
                if (done == nullptr) {
                    n = (uint32_t)(r - l + 1);
                } else {
                    const uint8_t *d = done + vw.x + (uint32_t)(rc.y + row) * vw.y;
                    for (int t = l; t <= r; ++t) n += d[t] ? 0u : 1u;
                }
            } else {
                r = l - 1;
            }
        }
        uint32_t round_total = 0;
        const uint32_t ex = block_scan_incl(n, s_wsum, &round_total) - n;
        if (n > 0) {
            const short4 rc = s_rc[e];
            const uint4 vw = s_vw[e];
            const uint32_t g = s_g[e];
            const uint32_t ty = (uint32_t)(rc.y + (int)(item - s_roff[e]));
            const uint32_t rowbase = vw.x + ty * vw.y;
            const uint32_t outbase = gbits ? rowbase - vw.x : rowbase;  // packed: the view's local tile
            uint32_t p = lo + carry + ex;
            for (int t = l; t <= r; ++t) {
                if (done != nullptr && done[rowbase + (uint32_t)t]) continue;
                if (p < capacity) {
                    if (gbits) {
                        tiles_out[p] = ((outbase + (uint32_t)t) << gbits) | g;
                    } else {
                        tiles_out[p] = outbase + (uint32_t)t;
                        vals_out[p] = g;
                    }
                } else {
                    dropped++;
                }
                ++p;
            }
        }
        carry += round_total;
    }
    if (tid == 0 && carry > 0) status_add(status, ST_PAIRS, (unsigned long long)carry);
    if (__ballot(dropped != 0) && dropped) {
        status_add(status, ST_DROPPED, (unsigned long long)dropped);
        status_flag(status, (unsigned long long)FS_DEV_PAIR_OVERFLOW);
    }
}

// Ranges of the sorted tile ids: each thread takes 4 consecutive entries (one
// 16-byte load) plus the neighbours on either side, in a grid-stride loop.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t *__restrict__ tiles,
                                                const uint32_t *__restrict__ n_pairs_dev, uint32_t capacity,
                                                int64_t max_pairs, uint2 *__restrict__ ranges)
{
    int64_t np = (int64_t)*n_pairs_dev;
    if (np > (int64_t)capacity) np = capacity;
    if (np > max_pairs) np = max_pairs;
    const int64_t stride = 4 * (int64_t)gridDim.x * blockDim.x;
    const bool aligned = (reinterpret_cast<uintptr_t>(tiles) & 15u) == 0;
    for (int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i0 < np; i0 += stride) {
        uint32_t t[6];
        t[0] = i0 > 0 ? tiles[i0 - 1] : 0xFFFFFFFFu;
        if (aligned && i0 + 4 <= np) {
            const uint4 q = *reinterpret_cast<const uint4 *>(tiles + i0);
            t[1] = q.x; t[2] = q.y; t[3] = q.z; t[4] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) t[1 + k] = i0 + k < np ? tiles[i0 + k] : 0xFFFFFFFFu;
        }
        t[5] = i0 + 4 < np ? tiles[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = i0 + k;
            if (i >= np) break;
            const uint32_t c = t[1 + k];
            if (c != t[k]) ranges[c].x = (uint32_t)i;
            if (c != t[2 + k]) ranges[c].y = (uint32_t)(i + 1);
        }
    }
}

// Ranges from per-tile counts and their exclusive scan; [0, 0) for empty tiles.
__global__ void k_count_ranges(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ starts,
                               int64_t n_tiles, uint2 *__restrict__ ranges)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t c = counts[t], s0 = starts[t];
    ranges[t] = c ? make_uint2(s0, s0 + c) : make_uint2(0u, 0u);
}

// Work-order keys: tiles with longer lists get smaller keys (lengths clamp
// at 65535), so an ascending stable sort puts the longest lists first.
__global__ void k_tile_keys(const uint2 *__restrict__ ranges, int64_t n_tiles, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    keys[t] = 0xFFFFu - (len < 0xFFFFu ? len : 0xFFFFu);
    vals[t] = (uint32_t)t;
}

// Pair offsets at depth-slab boundaries (used to plan chunks and slab capacities
// from one exact count).
__global__ void k_slab_offsets(const uint32_t *__restrict__ offsets, const ViewDev *__restrict__ views,
                               int32_t n_views, int64_t total_elems, const uint32_t *__restrict__ total_pairs,
                               SlabBounds nb, uint32_t *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_views * (int)nb.n) return;
    const int v = i / (int)nb.n, b = i % (int)nb.n;
    const int64_t e = (int64_t)views[v].elem_off + (int64_t)(((uint64_t)views[v].n * nb.num[b]) >> 10);
    out[i] = e < total_elems ? offsets[e] : *total_pairs;
}

// Segments of the packed pair sort, one per view (see launch_pair_segs).
__global__ void k_pair_segs(const uint32_t *__restrict__ offsets, const ViewDev *__restrict__ views, int32_t n_views,
                            int64_t total_elems, const uint32_t *__restrict__ total_pairs, uint32_t capacity,
                            SegDev *__restrict__ segs, unsigned long long *__restrict__ status)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_views) return;
    const uint32_t np = min(*total_pairs, capacity);
    const int64_t e0 = (int64_t)views[j].elem_off;
    const int64_t e1 = j + 1 < n_views ? (int64_t)views[j + 1].elem_off : total_elems;
    const uint32_t a = min(e0 < total_elems ? offsets[e0] : *total_pairs, np);
    const uint32_t b = min(e1 < total_elems ? offsets[e1] : *total_pairs, np);
    const uint32_t have = b > a ? b - a : 0u;
    SegDev sg = segs[j];
    sg.off = a;
    sg.alen = min(have, sg.len);
    if (have > sg.len) {
        status_add(status, ST_DROPPED, (unsigned long long)(have - sg.len));
        status_flag(status, (unsigned long long)FS_DEV_PAIR_OVERFLOW);
    }
    segs[j] = sg;
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t count)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

// ---- scan ----
static int64_t scan_levels_bytes(int64_t n)
{
    int64_t bytes = 0;
    while (n > kTile) {
        n = (n + kTile - 1) / kTile;
        bytes += (n + 64) * 4;
    }
    return bytes + 256;
}

size_t scan_ws_bytes(int64_t n) { return (size_t)scan_levels_bytes(n); }

hipError_t scan_exclusive(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_out, void *ws)
{
    if (n <= 0) {
        if (total_out) return launch_fill_u32(s, total_out, 0u, 1);
        return hipSuccess;
    }
    const int64_t blocks = (n + kTile - 1) / kTile;
    if (blocks == 1) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kThreads), 0, s, in, out, n, (const uint32_t *)nullptr, total_out,
                           0);
        return hipGetLastError();
    }
    uint32_t *sums = (uint32_t *)ws;
    uint32_t *rest = sums + ((blocks + 64) & ~int64_t(63));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)blocks), dim3(kThreads), 0, s, in, n, sums);
    // up to one tile of block totals: each block adds up the totals before it
    const bool raw = blocks <= kTile;
    if (!raw) {
        hipError_t e = scan_exclusive(s, sums, sums, blocks, nullptr, rest);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)blocks), dim3(kThreads), 0, s, in, out, n, (const uint32_t *)sums,
                       total_out, raw ? 1 : 0);
    return hipGetLastError();
}

// ---- radix sort ----
size_t radix_ws_bytes(uint32_t n_blocks)
{
    const int64_t hist = (int64_t)n_blocks * 256;
    return (size_t)(2 * hist * 4 + scan_levels_bytes(hist) + 512);
}

hipError_t radix_sort(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                      const SegDev *segs, int32_t n_segs, uint32_t n_blocks, int32_t bits, void *ws,
                      const uint32_t *len_dev, int32_t tpb, uint32_t *key_count, bool last_keys)
{
    if (n_blocks == 0 || n_segs == 0) return hipSuccess;
    if (tpb < 1) return hipErrorInvalidValue;
    const int64_t hist_n = (int64_t)n_blocks * 256;
    uint32_t *hist = (uint32_t *)ws;
    uint32_t *offs = hist + hist_n;
    void *scan_ws = offs + hist_n;
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(n_blocks), dim3(kThreads), 0, s, ki, segs, n_segs, shift, hist, len_dev,
                           tpb, 255u);
        hipError_t e = scan_exclusive(s, hist, offs, hist_n, nullptr, scan_ws);
        if (e != hipSuccess) return e;
        const bool last = shift + 8 >= bits;
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3(n_blocks), dim3(kThreads), 0, s, ki, vi,
                           (last && !last_keys) ? nullptr : ko, vo, segs, n_segs, shift, (const uint32_t *)offs,
                           len_dev, tpb, last ? key_count : nullptr, 255u, 0, 0u);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t *tk = ki, *tv = vi;
        ki = ko; vi = vo; ko = tk; vo = tv;
    }
    return hipSuccess;
}

hipError_t radix_sort_packed(hipStream_t s, uint32_t *items, uint32_t *items_alt, uint32_t *ids_out,
                             const SegDev *segs, int32_t n_segs, uint32_t n_blocks, int32_t gbits, int32_t tbits,
                             void *ws, int32_t tpb, uint32_t *key_count)
{
    if (n_blocks == 0 || n_segs == 0) return hipSuccess;
    if (tpb < 1 || gbits < 1 || tbits < 1 || tbits > 16 || gbits + tbits > 32) return hipErrorInvalidValue;
    const int64_t hist_n = (int64_t)n_blocks * 256;
    uint32_t *hist = (uint32_t *)ws;
    uint32_t *offs = hist + hist_n;
    void *scan_ws = offs + hist_n;
    // one pass up to 8 tile bits, else two passes of (nearly) equal width:
    // fewer buckets per pass keep the scattered runs long
    const int passes = tbits <= 8 ? 1 : 2;
    const int d0 = passes == 1 ? tbits : (tbits + 1) / 2;
    const uint32_t vmask = gbits == 32 ? 0xFFFFFFFFu : ((1u << gbits) - 1u);
    const uint32_t *ki = items;
    for (int p = 0; p < passes; ++p) {
        const int shift = gbits + (p == 0 ? 0 : d0);
        const int bits = p == 0 ? d0 : tbits - d0;
        const uint32_t dmask = (1u << bits) - 1u;
        const bool last = p + 1 == passes;
        hipLaunchKernelGGL(k_radix_hist, dim3(n_blocks), dim3(kThreads), 0, s, ki, segs, n_segs, shift, hist,
                           (const uint32_t *)nullptr, tpb, dmask);
        hipError_t e = scan_exclusive(s, hist, offs, hist_n, nullptr, scan_ws);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3(n_blocks), dim3(kThreads), 0, s, ki, (const uint32_t *)nullptr,
                           last ? nullptr : items_alt, last ? ids_out : nullptr, segs, n_segs, shift,
                           (const uint32_t *)offs, (const uint32_t *)nullptr, tpb, last ? key_count : nullptr, dmask,
                           gbits, vmask);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ki = items_alt;
    }
    return hipSuccess;
}

int32_t radix_tiles_per_block(uint64_t n_items)
{
    // about 4096 blocks (16 per CU) once the sort is large enough; tables of
    // 256 counts per block stay a few MB
    const uint64_t tiles = (n_items + kTile - 1) / kTile;
    const uint64_t t = tiles / 4096;
    return (int32_t)(t < 1 ? 1 : (t > 64 ? 64 : t));
}

hipError_t launch_depth_keys(hipStream_t s, const float *rec, const int32_t *ntiles, const uint8_t *flags,
                             const ViewDev *views, int32_t n_views, int64_t total, uint32_t *keys, uint32_t *vals)
{
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_depth_keys, dim3(grid_for(total, 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(rec), ntiles, flags, views, n_views, total, keys, vals);
    return hipGetLastError();
}

hipError_t launch_gather_counts(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                                const int32_t *ntiles, const ViewDev *views, int32_t n_views, int64_t total,
                                uint32_t *counts, int32_t cshift)
{
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_counts, dim3(grid_for(total, 256)), dim3(256), 0, s, sorted_keys, sorted_vals,
                       ntiles, views, n_views, total, counts, cshift);
    return hipGetLastError();
}

hipError_t launch_emit(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                       const uint32_t *offsets, const uint32_t *counts, const float *rec, const int16_t *rect,
                       const uint8_t *flags, const ViewDev *views, int32_t n_views, int64_t total,
                       uint32_t capacity, int32_t tile_w, int32_t tile_h, float sigma_k, const uint8_t *done,
                       uint32_t *tiles_out,
                       uint32_t *vals_out, unsigned long long *status, int32_t gbits, const uint64_t *codes,
                       int32_t cshift)
{
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3(grid_for(total, kThreads)), dim3(kThreads), 0, s, sorted_keys, sorted_vals, offsets,
                       counts, reinterpret_cast<const float4 *>(rec), reinterpret_cast<const short4 *>(rect), flags,
                       views, n_views, total, capacity, tile_w, tile_h, sigma_k, done, tiles_out, vals_out, status,
                       gbits, reinterpret_cast<const ulonglong2 *>(codes), cshift);
    return hipGetLastError();
}

hipError_t launch_pair_segs(hipStream_t s, const uint32_t *offsets, const ViewDev *views, int32_t n_views,
                            int64_t total_elems, const uint32_t *total_pairs, uint32_t capacity, SegDev *segs,
                            unsigned long long *status)
{
    if (n_views <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_segs, dim3(grid_for(n_views, 256)), dim3(256), 0, s, offsets, views, n_views,
                       total_elems, total_pairs, capacity, segs, status);
    return hipGetLastError();
}

hipError_t launch_slab_offsets(hipStream_t s, const uint32_t *offsets, const ViewDev *views, int32_t n_views,
                               int64_t total_elems, const uint32_t *total_pairs, SlabBounds nb, uint32_t *out)
{
    if (n_views <= 0 || nb.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slab_offsets, dim3(grid_for((int64_t)n_views * nb.n, 256)), dim3(256), 0, s, offsets, views,
                       n_views, total_elems, total_pairs, nb, out);
    return hipGetLastError();
}

hipError_t launch_slab_counts(hipStream_t s, const uint32_t *sorted_keys, const uint32_t *sorted_vals,
                              const float *rec, const int16_t *rect, const uint8_t *flags, const int32_t *ntiles,
                              const ViewDev *views, int32_t n_views, int64_t total, Slab slab, const uint8_t *done,
                              int32_t tile_w, int32_t tile_h, float sigma_k, const uint64_t *codes,
                              uint32_t *counts, int32_t cshift)
{
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slab_counts, dim3(grid_for(total, 256)), dim3(256), 0, s, sorted_keys, sorted_vals,
                       reinterpret_cast<const float4 *>(rec), reinterpret_cast<const short4 *>(rect), flags, ntiles,
                       views, n_views, total, slab, done, tile_w, tile_h, sigma_k,
                       reinterpret_cast<const ulonglong2 *>(codes), counts, cshift);
    return hipGetLastError();
}


hipError_t launch_count_ranges(hipStream_t s, const uint32_t *counts, const uint32_t *starts, int64_t n_tiles,
                               uint32_t *ranges)
{
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_ranges, dim3(grid_for(n_tiles, 256)), dim3(256), 0, s, counts, starts, n_tiles,
                       reinterpret_cast<uint2 *>(ranges));
    return hipGetLastError();
}

hipError_t launch_tile_keys(hipStream_t s, const uint32_t *ranges, int64_t n_tiles, uint32_t *keys, uint32_t *vals)
{
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_keys, dim3(grid_for(n_tiles, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint2 *>(ranges), n_tiles, keys, vals);
    return hipGetLastError();
}

hipError_t launch_ranges(hipStream_t s, const uint32_t *tiles, const uint32_t *n_pairs_dev, uint32_t capacity,
                         int64_t n_pairs_max, uint32_t *ranges)
{
    if (n_pairs_max <= 0) return hipSuccess;
    int64_t blocks = (n_pairs_max + 1023) / 1024;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, tiles, n_pairs_dev, capacity, n_pairs_max,
                       reinterpret_cast<uint2 *>(ranges));
    return hipGetLastError();
}

}  // namespace fs
