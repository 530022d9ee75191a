// Gaussian-tile key emission, (tile, depth) ordering and per-tile ranges.
//
// The required order is ascending (tile id, depth bits, splat index). It is
// reached with two stable sorts instead of one sort of 64-bit keys:
//
//   1. the splats that cover at least one tile (splats whose shrunk
//      rectangle is empty emit nothing) are radix-sorted by their 32-bit
//      depth key, so ties keep ascending splat index; the first pass reads
//      the selections in (view, index) order and skips the others, which
//      packs the tile-covering splats as it sorts;
//   2. an exclusive prefix scan of their tile counts, taken in that depth
//      order, gives each splat its output offset, and the splat emits one
//      (tile id, splat index) pair per tile of its rectangle;
//   3. the pairs are radix-sorted by tile id only (ceil(log2 tiles) bits),
//      stably, so pairs of one tile keep the depth order of step 1.
//
// Pair traffic drops from ~6 passes over 12-byte (u64 key, u32 value)
// records to 2 passes over 8-byte records at 1080p.
//
// Radix pass (LSD, one digit of BITS bits, stable), three kernels:
//   k_hist      per 1024-item tile: digit histogram (LDS atomics) -> hist[digit][tile]
//   k_rowscan   one workgroup per digit: exclusive scan over the tiles,
//               digit totals
//   k_scatter   per tile: stable local ranks (wave ballot match on the digit
//               bits for all of a wave's rounds, then one pass per digit over
//               the per-(round, wave) counts in item order), items staged
//               through LDS in locally sorted order, then written out so that
//               consecutive lanes write consecutive addresses.
//
// Block offsets of the emission step are exclusive sums over the per-block
// counts of all earlier blocks. Up to 8192 blocks every block adds them up
// itself (a few thousand L2-resident words), so no scan launch sits between
// counting and writing; larger batches scan the counts in one workgroup
// first.
#include "fg_device.h"

#include <algorithm>

namespace {

constexpr int kThreads = 256;
constexpr int kIPT = 4;
constexpr int kTileItems = kThreads * kIPT;  // 1024
constexpr int kWaves = kThreads / fgd::kWave;
constexpr int kEmitIPT = 4;
constexpr int kEmitItems = kThreads * kEmitIPT;  // 1024
constexpr int kEmitRun = 4;                       // consecutive pairs per thread

__device__ __forceinline__ int64_t count_of(const uint32_t* p, int64_t cap)
{
    const int64_t n = (int64_t)*p;
    return n < cap ? n : cap;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t& total)
{
    const int lane = fgd::lane_id();
    const int wave = threadIdx.x / fgd::kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < fgd::kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, fgd::kWave);
        if (lane >= d) x += y;
    }
    if (lane == fgd::kWave - 1) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        const uint32_t t = s_wave[w];
        if (w < wave) before += t;
        total += t;
    }
    __syncthreads();
    return before + x - v;
}

// Sum of v[0 .. k) over the workgroup (every thread gets it).
__device__ __forceinline__ unsigned long long block_prefix(const uint32_t* __restrict__ v, int64_t k,
                                                           unsigned long long* s_red)
{
    unsigned long long x = 0;
    for (int64_t i0 = threadIdx.x; i0 < k; i0 += 4 * kThreads) {  // 4 independent loads per step
        uint32_t a[4];
#pragma unroll
        for (int u = 0; u < 4; u++) a[u] = i0 + u * kThreads < k ? v[i0 + u * kThreads] : 0u;
#pragma unroll
        for (int u = 0; u < 4; u++) x += a[u];
    }
#pragma unroll
    for (int d = fgd::kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, fgd::kWave);
    if (fgd::lane_id() == 0) s_red[threadIdx.x / fgd::kWave] = x;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) t += s_red[w];
    __syncthreads();
    return t;
}

// Block offsets of the emission kernel: either read from counts
// that k_block_scan turned into exclusive offsets, or, when the blocks are few
// enough (kInlineBlocks), summed by every block from the raw counts of the
// blocks before it (L2-resident words), which saves the scan launch; then
// block 0 also stores the total and flags an overflow of cap.
struct BlockOffsets {
    const uint32_t* cnt;
    bool inline_sum;
    uint32_t* total;
    int64_t cap;
    uint32_t* status;
    uint32_t overflow_bit;
};

__device__ __forceinline__ unsigned long long block_offset(const BlockOffsets& o, int64_t blk,
                                                           unsigned long long* s_red)
{
    return o.inline_sum ? block_prefix(o.cnt, blk, s_red) : (unsigned long long)o.cnt[blk];
}

__device__ __forceinline__ void block_total(const BlockOffsets& o, int64_t nblk, unsigned long long* s_red)
{
    if (!o.inline_sum || blockIdx.x != 0) return;
    const unsigned long long t = block_prefix(o.cnt, nblk, s_red);
    if (threadIdx.x == 0) {
        *o.total = (uint32_t)(t < 0xFFFFFFFFull ? t : 0xFFFFFFFFull);
        if ((long long)t > o.cap) atomicOr(o.status, o.overflow_bit);
    }
}

// The views of one call: their splats lie at stride cap_sel in the splat
// planes (view v's splat j is global splat v * cap_sel + j), and their tiles
// have the consecutive global ids tile_base[v] + ty * Wt[v] + tx.
constexpr int kMaxViews = 64;
struct SortViews {
    int n;
    uint32_t cap_sel;
    uint32_t Wt[kMaxViews];
    uint32_t tile_base[kMaxViews];
};

// s_seg[v] = sum over views u < v of min(n_sel[u], cap_sel) (v = 0 .. n): the
// position of view v's first splat among the concatenated selections. Read by
// the first wave; ends with a barrier.
__device__ __forceinline__ void load_segments(const uint32_t* __restrict__ n_sel, const SortViews& V,
                                              uint32_t* s_seg)
{
    if (threadIdx.x < fgd::kWave) {
        const int lane = fgd::lane_id();
        uint32_t c = 0;
        if (lane < V.n) {
            c = n_sel[lane];
            c = c < V.cap_sel ? c : V.cap_sel;
        }
        uint32_t x = c;
#pragma unroll
        for (int d = 1; d < fgd::kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, fgd::kWave);
            if (lane >= d) x += y;
        }
        if (lane == 0) s_seg[0] = 0u;
        if (lane < V.n) s_seg[lane + 1] = x;
    }
    __syncthreads();
}

// Global splat index of concatenated selection item i (i < s_seg[n]).
__device__ __forceinline__ uint32_t item_splat(uint32_t i, const uint32_t* s_seg, const SortViews& V)
{
    int lo = 0, hi = V.n;  // the last view v with s_seg[v] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_seg[mid] <= i) lo = mid; else hi = mid;
    }
    return (uint32_t)lo * V.cap_sel + (i - s_seg[lo]);
}

template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Input of the first depth pass: the concatenated selections themselves.
// Item i is global splat g = item_splat(i); it takes part when its rectangle
// covers a tile (tiles[g] != 0), with key = the bits of its depth and value
// g. So the pass also packs the tile-covering splats, in (view, index) order
// within each digit. The histogram kernel clears the tile ranges and stores
// the item count; the scatter stores the packed count and flags an overflow
// of cap_out.
struct SelInput {
    const float4* rgb_depth;
    const uint32_t* tiles;
    const uint32_t* n_sel;
    uint32_t* n_items;  // selection items (written by k_hist)
    uint32_t* n_out;    // packed items (written by k_scatter)
    int64_t cap_out;
    uint32_t* status;
    uint32_t* ranges;
    int64_t n_range_words;
};

// Key and value of item idx of a pass (valid: the item takes part).
template <bool SEL>
__device__ __forceinline__ void pass_item(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                          const SelInput& si, const SortViews& V, const uint32_t* s_seg,
                                          int64_t idx, int64_t n, bool want_val, bool& valid, uint32_t& k,
                                          uint32_t& v)
{
    valid = idx < n;
    k = 0xFFFFFFFFu;
    v = 0u;
    if (!valid) return;
    if constexpr (SEL) {
        const uint32_t g = item_splat((uint32_t)idx, s_seg, V);
        valid = si.tiles[g] != 0u;
        if (valid) {
            k = __float_as_uint(si.rgb_depth[g].w);
            v = g;
        }
    } else {
        k = kin[idx];
        if (want_val) v = vin[idx];
    }
}

template <int BITS, int IPT, bool SEL>
__global__ __launch_bounds__(kThreads) void k_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_p,
                                                   int64_t cap, int shift, uint32_t* __restrict__ hist, SelInput si,
                                                   SortViews V)
{
    constexpr int R = 1 << BITS;
    __shared__ uint32_t h[R];
    __shared__ uint32_t s_seg[SEL ? kMaxViews + 1 : 1];
    int64_t n;
    if constexpr (SEL) {
        for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < si.n_range_words;
             t += (int64_t)gridDim.x * kThreads)
            si.ranges[t] = 0u;
        load_segments(si.n_sel, V, s_seg);
        n = s_seg[V.n];
        if (blockIdx.x == 0 && threadIdx.x == 0) *si.n_items = (uint32_t)n;
    } else {
        n = count_of(n_p, cap);
    }
    const int64_t n_tiles = (n + (kThreads * IPT) - 1) / (kThreads * IPT);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        for (int d = threadIdx.x; d < R; d += kThreads) h[d] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const int64_t idx = tile * (kThreads * IPT) + r * kThreads + threadIdx.x;
            bool valid;
            uint32_t k, v;
            pass_item<SEL>(keys, nullptr, si, V, s_seg, idx, n, false, valid, k, v);
            if (valid) atomicAdd(&h[(k >> shift) & (R - 1)], 1u);
        }
        __syncthreads();
        for (int d = threadIdx.x; d < R; d += kThreads) hist[(int64_t)d * n_tiles + tile] = h[d];
        __syncthreads();
    }
}

// One workgroup per digit: exclusive scan of hist[digit][0..n_tiles) in place.
template <int IPT>
__global__ __launch_bounds__(kThreads) void k_rowscan(const uint32_t* __restrict__ n_p, int64_t cap,
                                                      uint32_t* __restrict__ hist, uint32_t* __restrict__ digit_total)
{
    __shared__ uint32_t s_wave[kWaves];
    const int64_t n = count_of(n_p, cap);
    const int64_t n_tiles = (n + (kThreads * IPT) - 1) / (kThreads * IPT);
    uint32_t* row = hist + (int64_t)blockIdx.x * n_tiles;
    const int64_t per = (n_tiles + kThreads - 1) / kThreads;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < n_tiles ? lo + per : n_tiles;
    uint32_t s = 0;
    for (int64_t i0 = lo; i0 < hi; i0 += 4) {  // 4 independent loads per step
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = i0 + u < hi ? row[i0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < 4; u++) s += c[u];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(s, s_wave, total);
    for (int64_t i0 = lo; i0 < hi; i0 += 4) {
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = i0 + u < hi ? row[i0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (i0 + u < hi) row[i0 + u] = run;
            run += c[u];
        }
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = total;
}

template <int BITS, int IPT, bool SEL>
__global__ __launch_bounds__(kThreads) void k_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      const uint32_t* __restrict__ n_p, int64_t cap, int shift,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ digit_total, SelInput si,
                                                      SortViews V)
{
    constexpr int R = 1 << BITS;
    static_assert(R <= kThreads, "one thread per digit");
    __shared__ uint32_t s_base[R];
    __shared__ uint32_t s_start[R];
    // per (round, wave, digit): the group's count, then its exclusive offset
    // among the tile's items of that digit (at most (kThreads * IPT): fits 16 bits)
    __shared__ uint16_t s_cnt[IPT][kWaves][R];
    __shared__ uint32_t s_keys[(kThreads * IPT)];
    __shared__ uint32_t s_vals[(kThreads * IPT)];
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_seg[SEL ? kMaxViews + 1 : 1];
    const int64_t n = count_of(n_p, cap);
    const int64_t n_tiles = (n + (kThreads * IPT) - 1) / (kThreads * IPT);
    const int tid = threadIdx.x;
    const int wave = tid / fgd::kWave;
    if constexpr (SEL) load_segments(si.n_sel, V, s_seg);
    {
        uint32_t tot;
        const uint32_t v = tid < R ? digit_total[tid] : 0u;
        const uint32_t e = block_excl_scan(v, s_wave, tot);
        if (tid < R) s_base[tid] = e;
        if (SEL && blockIdx.x == 0 && tid == 0) {
            *si.n_out = tot;
            if ((int64_t)tot > si.cap_out) atomicOr(si.status, FG_STATUS_ITEM_OVERFLOW);
        }
    }
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        uint32_t k[IPT], v[IPT], below[IPT];
        bool ok[IPT];
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const int64_t idx = tile * (kThreads * IPT) + r * kThreads + tid;
            pass_item<SEL>(kin, vin, si, V, s_seg, idx, n, true, ok[r], k[r], v[r]);
        }
        {
            uint32_t* c32 = reinterpret_cast<uint32_t*>(&s_cnt[0][0][0]);
            for (int i = tid; i < IPT * kWaves * R / 2; i += kThreads) c32[i] = 0u;
        }
        __syncthreads();
        // every wave ranks its items of every round among equal digits
        // (ballot match), with no barrier between rounds
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const uint32_t d = (k[r] >> shift) & (R - 1);
            const uint64_t m = match_digit<BITS>(d, ok[r]);
            below[r] = (uint32_t)__popcll(m & fgd::lanemask_lt());
            if (ok[r] && below[r] == 0) s_cnt[r][wave][d] = (uint16_t)__popcll(m);
        }
        __syncthreads();
        // per digit, groups in item order (round-major, then wave)
        uint32_t run = 0;
        if (tid < R) {
#pragma unroll
            for (int r = 0; r < IPT; r++)
#pragma unroll
                for (int w = 0; w < kWaves; w++) {
                    const uint32_t c = s_cnt[r][w][tid];
                    s_cnt[r][w][tid] = (uint16_t)run;
                    run += c;
                }
        }
        uint32_t cnt;  // items of this tile that take part
        {
            const uint32_t e = block_excl_scan(run, s_wave, cnt);
            if (tid < R) s_start[tid] = e;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            if (ok[r]) {
                const uint32_t d = (k[r] >> shift) & (R - 1);
                const uint32_t pos = s_start[d] + s_cnt[r][wave][d] + below[r];
                s_keys[pos] = k[r];
                s_vals[pos] = v[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const int p = r * kThreads + tid;
            if ((uint32_t)p < cnt) {
                const uint32_t key = s_keys[p];
                const uint32_t d = (key >> shift) & (R - 1);
                const int64_t g = (int64_t)s_base[d] + hist[(int64_t)d * n_tiles + tile] + (p - s_start[d]);
                if (!SEL || g < si.cap_out) {
                    kout[g] = key;
                    vout[g] = s_vals[p];
                }
            }
        }
        __syncthreads();
    }
}

// One workgroup: cnt[0 .. *nblk_items / per) becomes its exclusive prefix sum
// in place, *total the sum (and *total_out, when given, a copy of it clamped
// to 32 bits; overflow of cap sets status bit). The number of blocks is
// derived from the item count that the previous kernel counted over.
__global__ __launch_bounds__(kThreads) void k_block_scan(uint32_t* __restrict__ cnt, const uint32_t* __restrict__ n_items,
                                                         int64_t per, int64_t cap_items, uint32_t* __restrict__ total,
                                                         uint32_t* __restrict__ total_out, int64_t cap_total,
                                                         uint32_t* __restrict__ status, uint32_t overflow_bit)
{
    __shared__ uint32_t s_wave[kWaves];
    const int64_t n = count_of(n_items, cap_items);
    const int64_t nblk = (n + per - 1) / per;
    const int tid = threadIdx.x;
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nblk; base += (int64_t)kThreads * 8) {
        uint32_t c[8];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t i = base + (int64_t)tid * 8 + k;
            c[k] = i < nblk ? cnt[i] : 0u;
            sum += c[k];
        }
        uint32_t tot;
        unsigned long long run = carry + block_excl_scan(sum, s_wave, tot);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t i = base + (int64_t)tid * 8 + k;
            if (i < nblk) cnt[i] = (uint32_t)run;
            run += c[k];
        }
        carry += tot;
    }
    if (tid == 0) {
        const uint32_t t32 = (uint32_t)(carry < 0xFFFFFFFFull ? carry : 0xFFFFFFFFull);
        *total = t32;
        if (total_out) *total_out = t32;
        if ((long long)carry > cap_total) atomicOr(status, overflow_bit);
    }
}

// Per 1024 splats in depth order: the sum of their tile counts (the areas of
// their rectangles). The rectangles are gathered here once and stored in depth
// order, so that the emission reads them contiguously.
__global__ __launch_bounds__(kThreads) void k_count_reduce(const uint32_t* __restrict__ order,
                                                           const ushort4* __restrict__ rect,
                                                           const uint32_t* __restrict__ n_p, int64_t cap,
                                                           uint32_t* __restrict__ bsum, ushort4* __restrict__ rect_d)
{
    __shared__ uint32_t s_wave[kWaves];
    const int64_t n = count_of(n_p, cap);
    const int64_t nblk = (n + kEmitItems - 1) / kEmitItems;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        uint32_t s = 0;
#pragma unroll
        for (int r = 0; r < kEmitIPT; r++) {
            const int64_t j = blk * kEmitItems + r * kThreads + threadIdx.x;
            if (j < n) {
                const ushort4 q = rect[order[j]];
                rect_d[j] = q;
                s += (uint32_t)(q.z - q.x) * (uint32_t)(q.w - q.y);
            }
        }
        uint32_t total;
        block_excl_scan(s, s_wave, total);
        if (threadIdx.x == 0) bsum[blk] = total;
    }
}

// Per 1024 splats in depth order: every splat's output offset (the block's
// offset from the scanned block sums, plus an exclusive scan within the
// block), then the block's pairs are written with thread k taking output
// positions k, k + 256, ...: a binary search over the offsets finds the
// splat, and the position within its rectangle (rows, then columns) gives
// the tile, numbered in its view's global tile ids.
__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t* __restrict__ order,
                                                   const ushort4* __restrict__ rect_d, const uint32_t* __restrict__ n_p,
                                                   int64_t cap, BlockOffsets boff, int64_t cap_pairs,
                                                   SortViews V, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals)
{
    __shared__ uint32_t s_wave[kWaves];
    __shared__ unsigned long long s_red[kWaves];
    __shared__ uint32_t s_off[kEmitItems + 1];
    __shared__ uint32_t s_g[kEmitItems];
    __shared__ ushort4 s_rect[kEmitItems];
    const int64_t n = count_of(n_p, cap);
    const int64_t nblk = (n + kEmitItems - 1) / kEmitItems;
    const int tid = threadIdx.x;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const unsigned long long base = block_offset(boff, blk, s_red);
        const int64_t j0 = blk * kEmitItems + (int64_t)tid * kEmitIPT;
        uint32_t c[kEmitIPT];
        uint32_t sum = 0;
#pragma unroll
        for (int r = 0; r < kEmitIPT; r++) {
            const int64_t j = j0 + r;
            const uint32_t g = j < n ? order[j] : 0u;
            const ushort4 q = j < n ? rect_d[j] : make_ushort4(0, 0, 0, 0);
            c[r] = (uint32_t)(q.z - q.x) * (uint32_t)(q.w - q.y);
            s_g[tid * kEmitIPT + r] = g;
            s_rect[tid * kEmitIPT + r] = q;
            sum += c[r];
        }
        uint32_t total;
        uint32_t run = block_excl_scan(sum, s_wave, total);
#pragma unroll
        for (int r = 0; r < kEmitIPT; r++) {
            s_off[tid * kEmitIPT + r] = run;
            run += c[r];
        }
        if (tid == 0) s_off[kEmitItems] = total;
        __syncthreads();
        // runs of kEmitRun consecutive outputs per thread: one binary search
        // per run (the last splat k with s_off[k] <= o; splats with no tile
        // share their successor's offset and are passed over), then step
        // through the rectangle, rows then columns
        for (uint32_t o0 = (uint32_t)tid * kEmitRun; o0 < total; o0 += (uint32_t)kThreads * kEmitRun) {
            int lo = 0, hi = kEmitItems;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= o0) lo = mid; else hi = mid;
            }
            ushort4 q = s_rect[lo];
            uint32_t w = (uint32_t)(q.z - q.x);
            uint32_t gv = s_g[lo] / V.cap_sel;
            const uint32_t local = o0 - s_off[lo];
            uint32_t ty = q.y + local / w, tx = q.x + local % w;
            const int m = total - o0 < (uint32_t)kEmitRun ? (int)(total - o0) : kEmitRun;
            for (int r = 0; r < m; r++) {
                const unsigned long long dst = base + o0 + (uint32_t)r;
                if (dst < (unsigned long long)cap_pairs) {
                    keys[dst] = V.tile_base[gv] + ty * V.Wt[gv] + tx;
                    vals[dst] = s_g[lo];
                }
                if (r + 1 < m && ++tx == q.z) {
                    tx = q.x;
                    if (++ty == q.w) {  // next splat with a tile (one exists: r + 1 < m)
                        do {
                            ++lo;
                        } while (s_off[lo + 1] == s_off[lo]);
                        q = s_rect[lo];
                        w = (uint32_t)(q.z - q.x);
                        gv = s_g[lo] / V.cap_sel;
                        tx = q.x;
                        ty = q.y;
                    }
                }
            }
        }
        __syncthreads();
    }
    block_total(boff, nblk, s_red);
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_p, int64_t cap,
                         uint32_t tile_base, int64_t n_tiles, uint32_t* __restrict__ ranges)
{
    const int64_t n = count_of(n_p, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[i];
        const uint32_t t = k - tile_base;
        if ((int64_t)t >= n_tiles) continue;
        if (i == 0 || keys[i - 1] != k) ranges[2 * (int64_t)t] = (uint32_t)i;
        if (i == n - 1 || keys[i + 1] != k) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t tiles_for(int64_t n) { return (n + kTileItems - 1) / kTileItems; }

// Depth keys and splat ids ping-pong between buffers 0 and 1; the depth sort
// has an even number of passes and ends in buffer 0, after which buffer 1
// (8 bytes per splat) holds the rectangles in depth order.
struct SortWs {
    uint32_t *dkey0, *dval0, *dkey1, *dval1, *bsum, *kalt, *valt, *hist, *digit_total, *counts;
    ushort4* rect_d;
};
// counts[0]: concatenated selection items, [1]: tile-covering splats packed

size_t carve(void* base, int64_t sel_items, int64_t cap_items, int64_t cap_pairs, SortWs* w)
{
    int64_t most = cap_items > cap_pairs ? cap_items : cap_pairs;
    if (sel_items > most) most = sel_items;
    const int64_t ht = tiles_for(most);
    const size_t nblk_emit = (size_t)((cap_items + kEmitItems - 1) / kEmitItems + 1);
    const size_t sizes[9] = {
        (size_t)cap_items * 4, (size_t)cap_items * 4, (size_t)cap_items * 8, nblk_emit * 4,
        (size_t)cap_pairs * 4, (size_t)cap_pairs * 4,
        (size_t)256 * (size_t)(ht + 1) * 4, (size_t)256 * 4, 16};
    uint32_t** dst[9] = {&w->dkey0, &w->dval0, &w->dkey1, &w->bsum, &w->kalt, &w->valt, &w->hist,
                         &w->digit_total, &w->counts};
    size_t off = 0;
    for (int i = 0; i < 9; i++) {
        if (base) *dst[i] = (uint32_t*)((char*)base + off);
        off += align_up(sizes[i] + 4);
    }
    if (base) {
        w->dval1 = w->dkey1 + cap_items;
        w->rect_d = reinterpret_cast<ushort4*>(w->dkey1);
    }
    return off;
}

// Items per thread of a radix pass: 4 (1024-item tiles) for one view, whose
// counts are a few million; 16 (4096-item tiles) for a batch of views with a
// capacity of tens of millions, where a scatter tile's 256 digit runs would
// otherwise average four items (16-byte writes into 128-byte lines). Chosen
// from the call's shape on the host (the counts stay on the device).
constexpr int64_t kBigSort = (int64_t)4 << 20;

// Block counts up to which the emission kernel sums its block offsets itself
// (see BlockOffsets): up to 8M splats at 1024 per block.
constexpr int64_t kInlineBlocks = 8192;

template <int BITS, int IPT, bool SEL>
void radix_pass_ipt(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const uint32_t* n_p,
                    int64_t cap, int shift, const SortWs& w, const SelInput& si, const SortViews& V, hipStream_t s)
{
    int64_t grid = (cap + kThreads * IPT - 1) / (kThreads * IPT);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_hist<BITS, IPT, SEL>), dim3((unsigned)grid), dim3(kThreads), 0, s, kin, n_p, cap, shift,
                       w.hist, si, V);
    hipLaunchKernelGGL(k_rowscan<IPT>, dim3(1u << BITS), dim3(kThreads), 0, s, n_p, cap, w.hist, w.digit_total);
    hipLaunchKernelGGL((k_scatter<BITS, IPT, SEL>), dim3((unsigned)grid), dim3(kThreads), 0, s, kin, vin, kout, vout,
                       n_p, cap, shift, w.hist, w.digit_total, si, V);
}

template <int BITS, bool SEL = false>
void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const uint32_t* n_p,
                int64_t cap, int shift, bool big, const SortWs& w, const SelInput& si, const SortViews& V,
                hipStream_t s)
{
    if (big) radix_pass_ipt<BITS, 16, SEL>(kin, vin, kout, vout, n_p, cap, shift, w, si, V, s);
    else radix_pass_ipt<BITS, 4, SEL>(kin, vin, kout, vout, n_p, cap, shift, w, si, V, s);
}

void radix_pass_bits(int bits, const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                     const uint32_t* n_p, int64_t cap, int shift, bool big, const SortWs& w, const SelInput& si,
                     const SortViews& V, hipStream_t s)
{
    switch (bits) {
        case 4: radix_pass<4>(kin, vin, kout, vout, n_p, cap, shift, big, w, si, V, s); break;
        case 5: radix_pass<5>(kin, vin, kout, vout, n_p, cap, shift, big, w, si, V, s); break;
        case 6: radix_pass<6>(kin, vin, kout, vout, n_p, cap, shift, big, w, si, V, s); break;
        case 7: radix_pass<7>(kin, vin, kout, vout, n_p, cap, shift, big, w, si, V, s); break;
        default: radix_pass<8>(kin, vin, kout, vout, n_p, cap, shift, big, w, si, V, s); break;
    }
}

// Validates the views of a sort or render call: sizes, consecutive global
// tile ids (view v's first tile follows view v-1's last). Returns the total
// tile count, or -1.
int64_t views_tiles(const fg_camera* cams, int32_t n_views)
{
    if (!cams || n_views < 1 || n_views > kMaxViews) return -1;
    int64_t total = 0;
    for (int v = 0; v < n_views; v++) {
        if (cams[v].width <= 0 || cams[v].height <= 0) return -1;
        const int64_t nt = (int64_t)((cams[v].width + 15) / 16) * ((cams[v].height + 15) / 16);
        if ((int64_t)cams[v].tile_base != (int64_t)cams[0].tile_base + total) return -1;
        total += nt;
    }
    if ((uint64_t)cams[0].tile_base + (uint64_t)total - 1 > 0xFFFFFFFFull) return -1;
    return total;
}

}  // namespace

extern "C" size_t fg_sort_workspace_size(int64_t cap_sel, int32_t n_views, int64_t cap_items, int64_t cap_pairs)
{
    if (cap_sel < 0 || n_views < 1 || cap_items < 0 || cap_pairs < 0) return 0;
    SortWs w;
    return carve(nullptr, cap_sel * n_views, cap_items, cap_pairs, &w);
}

extern "C" int fg_sort(const fg_splats* splats, const uint32_t* n_sel, int64_t cap_sel, const fg_camera* cams,
                       int32_t n_views, int64_t cap_items, uint32_t* tile_keys, uint32_t* vals, int64_t cap_pairs,
                       uint32_t* n_pairs, uint32_t* ranges, uint32_t* status, void* ws, size_t ws_bytes,
                       const fg_tune* tune, void* stream)
{
    if (!splats || !n_sel || !cams || !n_pairs || !ranges || !status || cap_sel < 0 || cap_pairs < 0 ||
        cap_items < 0 || n_views < 1)
        return FG_ERR_INVALID_ARG;
    if (n_views > kMaxViews || cap_sel * n_views >= ((int64_t)1 << 32) || cap_items >= ((int64_t)1 << 31) ||
        cap_pairs >= ((int64_t)1 << 32) - 1)
        return FG_ERR_UNSUPPORTED;
    if (cap_pairs > 0 && (!tile_keys || !vals)) return FG_ERR_INVALID_ARG;
    if (cap_sel > 0 && (!splats->rgb_depth || !splats->rect || !splats->tiles)) return FG_ERR_INVALID_ARG;
    const int64_t n_tiles = views_tiles(cams, n_views);
    if (n_tiles < 0) return FG_ERR_INVALID_ARG;
    int bits = 0;  // 0: the narrowest digit that needs no more passes than 8-bit digits
    if (tune && tune->radix_bits) {
        if (tune->radix_bits < 4 || tune->radix_bits > 8) return FG_ERR_INVALID_ARG;
        bits = tune->radix_bits;
    }
    SortWs w;
    const size_t need = carve(nullptr, cap_sel * n_views, cap_items, cap_pairs, &w);
    if (!ws || ws_bytes < need) return FG_ERR_WORKSPACE;
    carve(ws, cap_sel * n_views, cap_items, cap_pairs, &w);
    SortViews V;
    V.n = n_views;
    V.cap_sel = (uint32_t)cap_sel;
    for (int v = 0; v < kMaxViews; v++) {
        V.Wt[v] = v < n_views ? (uint32_t)((cams[v].width + 15) / 16) : 0u;
        V.tile_base[v] = v < n_views ? cams[v].tile_base : 0u;
    }
    hipStream_t s = (hipStream_t)stream;
    const uint64_t max_tile = (uint64_t)cams[0].tile_base + (uint64_t)n_tiles - 1;

    // 1. the splats that cover a tile, in depth order: the first 8-bit pass
    //    reads the selections and packs them (into buffer 1), three more
    //    passes end in buffer 0
    auto grid_for = [](int64_t items, int64_t per) {
        int64_t g = (items + per - 1) / per;
        return (unsigned)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    };
    const int64_t sel_items = cap_sel * n_views;
    const bool big_depth = n_views > 1 && cap_items >= kBigSort;
    const SelInput sel{(const float4*)splats->rgb_depth, splats->tiles, n_sel, w.counts, w.counts + 1, cap_items,
                       status, ranges, 2 * n_tiles};
    const SelInput none{};
    radix_pass<8, true>(nullptr, nullptr, w.dkey1, w.dval1, w.counts, sel_items, 0, big_depth, w, sel, V, s);
    uint32_t* n_vis = w.counts + 1;
    for (int p = 1; p < 4; p++) {
        const bool even = (p % 2) == 0;
        radix_pass<8>(even ? w.dkey0 : w.dkey1, even ? w.dval0 : w.dval1, even ? w.dkey1 : w.dkey0,
                      even ? w.dval1 : w.dval0, n_vis, cap_items, 8 * p, big_depth, w, none, V, s);
    }
    // 2. tile counts in depth order and key emission
    const unsigned gv = grid_for(cap_items, kEmitItems);
    hipLaunchKernelGGL(k_count_reduce, dim3(gv), dim3(kThreads), 0, s, w.dval0, (const ushort4*)splats->rect, n_vis,
                       cap_items, w.bsum, w.rect_d);
    const BlockOffsets boff{w.bsum, (cap_items + kEmitItems - 1) / kEmitItems <= kInlineBlocks, n_pairs, cap_pairs,
                            status, FG_STATUS_PAIR_OVERFLOW};
    if (!boff.inline_sum)
        hipLaunchKernelGGL(k_block_scan, dim3(1), dim3(kThreads), 0, s, w.bsum, n_vis, (int64_t)kEmitItems, cap_items,
                           n_pairs, (uint32_t*)nullptr, cap_pairs, status, FG_STATUS_PAIR_OVERFLOW);
    int tile_bits = 1;
    while (tile_bits < 32 && (max_tile >> tile_bits) != 0) ++tile_bits;
    if (bits == 0) {
        const int p8 = (tile_bits + 7) / 8;
        bits = (tile_bits + p8 - 1) / p8;  // e.g. 13 bits: two passes of 7
        if (bits < 4) bits = 4;
    }
    const int passes = (tile_bits + bits - 1) / bits;
    // emit into the buffer that the last pass will not write
    uint32_t* ek = cap_pairs == 0 ? nullptr : (passes % 2) ? w.kalt : tile_keys;
    uint32_t* ev = cap_pairs == 0 ? nullptr : (passes % 2) ? w.valt : vals;
    hipLaunchKernelGGL(k_emit, dim3(gv), dim3(kThreads), 0, s, w.dval0, w.rect_d, n_vis, cap_items, boff, cap_pairs,
                       V, ek, ev);
    if (cap_pairs > 0) {
        // 3. stable sort of the pairs by tile id
        uint32_t *ka = ek, *va = ev, *kb = (ek == tile_keys) ? w.kalt : tile_keys, *vb = (ev == vals) ? w.valt : vals;
        for (int p = 0; p < passes; p++) {
            radix_pass_bits(bits, ka, va, kb, vb, n_pairs, cap_pairs, bits * p, n_views > 1 && cap_pairs >= kBigSort,
                            w, none, V, s);
            uint32_t* t;
            t = ka; ka = kb; kb = t;
            t = va; va = vb; vb = t;
        }
        hipLaunchKernelGGL(k_ranges, dim3(grid_for(cap_pairs, 256)), dim3(256), 0, s, tile_keys, n_pairs, cap_pairs,
                           cams[0].tile_base, n_tiles, ranges);
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
