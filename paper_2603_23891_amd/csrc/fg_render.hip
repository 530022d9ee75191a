// Per-tile front-to-back alpha blending, Eq. (2).
//
// In Eq. (2) the per-fragment opacity alpha_i and the skip decisions
// (power > 0, alpha < 1/255) depend only on the splat and the pixel, not on
// the transmittance; only the product T_i = prod (1 - alpha_j), the early
// stop (T < 1e-4) and the colour sum run sequentially. Tiles near a horizon
// can hold ~10^4 splats whose pixels seldom saturate, so one workgroup that
// tests every (pixel, splat) of such a tile would leave the frame waiting on
// it. The blend therefore runs in two main launches:
//
//   k_masks   every chunk of CHUNK splats of a "heavy" tile (more than CHUNK
//             splats) is one work item: per-pixel bit masks of the splats
//             whose alpha passes the skip tests there go to global memory.
//             All chunks run in parallel.
//   k_render  one workgroup per tile, and per half of a heavy tile of 16
//             or more chunks (heavy work first, items claimed from an atomic
//             ticket): each
//             pixel walks the tile's splats in list order, chunk by chunk,
//             visiting only the marked ones and recomputing alpha with the
//             same expressions, so every value and decision is bit-identical
//             to one sequential pass. Light tiles (one lane per pixel)
//             compute their single chunk's masks in place. In a heavy tile
//             each wave walks the chunks for its own pixels at its own pace:
//             64 pixels, or in a split tile 32 with two lanes per pixel
//             sharing the alphas.
//
// Before them, k_schedule counts each tile's chunks and orders the tiles that
// hold splats, and k_tile_prep writes the pixels of the others (background,
// T = 1) and maps mask items to their tiles.
//
// Masks are computed over the (splat, pixel) pairs inside a conservative box
// per splat (the pixels where its skip test can pass), split evenly over the
// threads, so few large splats and many small ones balance alike. The launch
// boundary orders the mask writes before their reads; no workgroup ever
// waits for another.
#include "fg_device.h"
#include "fg_render_ws.h"

namespace {

constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;

// exp(power) <= exp(-5.6) < 1/255 for power < -5.6, so with opacity <= 1 the
// splat is skipped either way: testing this first avoids evaluating the
// exponential without changing any result.
constexpr float kSkipPower = -5.6f;

// Light tiles with fewer splats than this balance their mask work over
// (splat, pixel) pairs; larger ones give each thread whole splats.
constexpr int kPairSplats = 128;

struct RenderWs {
    uint32_t* nch;        // [n_tiles] chunks per tile (0: no splats)
    uint32_t* mfirst;     // [n_tiles] first mask item of a heavy tile
    uint32_t* order;      // [n_tiles] tiles in processing order, heavy first
    uint32_t* mitem;      // [max_mask_items] mask item -> tile
    uint32_t* counters;   // [0] ticket, [1] heavy tiles, [2] mask items (clamped), [3] tiles with splats
    uint32_t* masks;      // [max_mask_items][CHUNK/32][256]
    float* state;         // with save_state: [max_mask_items][4][256] T, C0, C1, C2 after each chunk; else null
    uint32_t* sched;      // [3][tile blocks] block totals of the many-tile schedule
};

struct Frag {
    unsigned n_eval, n_exp, n_pass, n_blend;
};

// The views of one call. Their tiles are numbered consecutively (view v owns
// tiles tile0[v] .. tile0[v+1] of the call, in the order of its global tile
// ids); view v's image is [3][H][W] at image + 3 * pix0[v], its final T and
// contributor counts at + pix0[v].
constexpr int kMaxViews = 64;
struct RenderViews {
    int n;
    uint32_t tile0[kMaxViews + 1];
    int W[kMaxViews], H[kMaxViews], Wt[kMaxViews];
    int64_t pix0[kMaxViews];
};

// One tile's view and geometry.
struct TileGeom {
    int tx, ty, W, H;
    int64_t pix0;
};

__device__ __forceinline__ TileGeom tile_geom(const RenderViews& V, uint32_t t)
{
    int lo = 0, hi = V.n;  // the view v with tile0[v] <= t < tile0[v+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (V.tile0[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t lt = t - V.tile0[lo];
    TileGeom g;
    g.tx = (int)(lt % (uint32_t)V.Wt[lo]);
    g.ty = (int)(lt / (uint32_t)V.Wt[lo]);
    g.W = V.W[lo];
    g.H = V.H[lo];
    g.pix0 = V.pix0[lo];
    return g;
}

// One workgroup per tile, after k_schedule: the final values of an empty
// tile's pixels (background, T = 1, no contributor), so that the blend never
// visits it, and the mask item -> tile map of a heavy tile's chunks.
template <int CHUNK>
__global__ __launch_bounds__(kThreads) void k_tile_prep(int64_t n_tiles, RenderViews V, float bg0,
                                                        float bg1, float bg2, const uint32_t* __restrict__ nch,
                                                        const uint32_t* __restrict__ mfirst, int64_t max_mask_items,
                                                        uint32_t* __restrict__ mitem, float* __restrict__ image,
                                                        float* __restrict__ final_T,
                                                        uint32_t* __restrict__ n_contrib)
{
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint32_t c = nch[t];
        if (c == 0) {
            const TileGeom g = tile_geom(V, (uint32_t)t);
            const int px = g.tx * fgd::kTile + (int)threadIdx.x % fgd::kTile;
            const int py = g.ty * fgd::kTile + (int)threadIdx.x / fgd::kTile;
            if (px < g.W && py < g.H) {
                const size_t o = (size_t)py * g.W + px;
                const size_t plane = (size_t)g.W * g.H;
                float* img = image + 3 * g.pix0;
                img[o] = bg0;
                img[plane + o] = bg1;
                img[2 * plane + o] = bg2;
                final_T[g.pix0 + o] = 1.0f;
                n_contrib[g.pix0 + o] = 0u;
            }
        } else if (c > 1) {
            const uint32_t mf = mfirst[t];
            for (uint32_t i = threadIdx.x; i < c; i += kThreads)
                if ((int64_t)(mf + i) < max_mask_items) mitem[mf + i] = (uint32_t)t;
        }
    }
}

// One workgroup, one pass: each tile's chunk count (0 for a tile with no
// splats); lists the tiles that hold splats, heavy ones from the front of
// order[] in tile order and light ones from its back in reverse tile order;
// numbers the mask items of heavy tiles (first item per tile) and resets the
// ticket.
// With h heavy tiles, work item i of the blend is part i % L of heavy tile
// order[i / L] for i < L h (L = kHeavyLanes; a heavy tile too short to be
// split is walked by its part 0, its other parts are empty), else the light
// tile order[n_tiles - 1 - (i - L h)]. 8 consecutive tiles per thread per
// round (the ranges are read and the chunk counts written with consecutive
// lanes on consecutive tiles, and handed over through LDS); the running
// counts of heavy and light tiles (one 64-bit word) and of mask items are
// scanned together.
template <int CHUNK>
__global__ __launch_bounds__(kScanThreads) void k_schedule(const uint32_t* __restrict__ ranges, int64_t n_tiles,
                                                           int64_t max_mask_items, uint32_t* __restrict__ nch,
                                                           uint32_t* __restrict__ mfirst, uint32_t* __restrict__ order,
                                                           uint32_t* __restrict__ counters)
{
    __shared__ unsigned long long s_wave[kScanThreads / fgd::kWave];
    __shared__ uint32_t s_wave_m[kScanThreads / fgd::kWave];
    __shared__ unsigned long long s_carry;
    __shared__ uint32_t s_carry_m;
    __shared__ uint32_t s_c[8 * kScanThreads];
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    if (tid == 0) {
        s_carry = 0ull;
        s_carry_m = 0u;
    }
    __syncthreads();
    for (int64_t base = 0; base < n_tiles; base += 8 * kScanThreads) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t t = base + (int64_t)k * kScanThreads + tid;
            uint32_t ck = 0u;
            if (t < n_tiles) {
                const uint2 r = reinterpret_cast<const uint2*>(ranges)[t];
                ck = (r.y - r.x + CHUNK - 1) / CHUNK;
                nch[t] = ck;
            }
            s_c[k * kScanThreads + tid] = ck;
        }
        __syncthreads();
        uint32_t c[8];
        unsigned long long sum = 0;  // low 32: heavy tiles, high 32: light tiles
        uint32_t msum = 0;           // mask items
#pragma unroll
        for (int k = 0; k < 8; k++) {
            c[k] = s_c[tid * 8 + k];
            if (c[k] > 1) {
                sum += 1ull;
                msum += c[k];
            } else if (c[k] == 1) {
                sum += 1ull << 32;
            }
        }
        unsigned long long x = sum;
        uint32_t xm = msum;
#pragma unroll
        for (int d = 1; d < fgd::kWave; d <<= 1) {
            const unsigned long long y = __shfl_up(x, d, fgd::kWave);
            const uint32_t ym = __shfl_up(xm, d, fgd::kWave);
            if (lane >= d) {
                x += y;
                xm += ym;
            }
        }
        if (lane == fgd::kWave - 1) {
            s_wave[wave] = x;
            s_wave_m[wave] = xm;
        }
        __syncthreads();
        unsigned long long before = s_carry, total = 0;
        uint32_t before_m = s_carry_m, total_m = 0;
        for (int w = 0; w < kScanThreads / fgd::kWave; w++) {
            if (w < wave) {
                before += s_wave[w];
                before_m += s_wave_m[w];
            }
            total += s_wave[w];
            total_m += s_wave_m[w];
        }
        unsigned long long run = before + x - sum;
        uint32_t mf = before_m + xm - msum;  // mask items before t
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t t = base + (int64_t)tid * 8 + k;
            if (t < n_tiles && c[k] > 0) {
                if (c[k] > 1) {
                    order[(uint32_t)run] = (uint32_t)t;  // heavy tiles before t
                    mfirst[t] = mf;
                    run += 1ull;
                    mf += c[k];
                } else {
                    order[n_tiles - 1 - (int64_t)(run >> 32)] = (uint32_t)t;  // light tiles before t
                    run += 1ull << 32;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            s_carry += total;
            s_carry_m += total_m;
        }
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t items = s_carry_m;
        counters[0] = 0u;
        counters[1] = (uint32_t)s_carry;
        counters[2] = (int64_t)items < max_mask_items ? items : (uint32_t)max_mask_items;
        counters[3] = (uint32_t)s_carry + (uint32_t)(s_carry >> 32);
    }
}

// The same schedule for many tiles (a batch of views), in three launches:
// per block of 8192 tiles the chunk counts and the block's totals (heavy
// tiles, light tiles, mask items); one workgroup scans the block totals; each
// block then writes its part of order[] and mfirst[] from its base. Results
// equal k_schedule's.
constexpr int kSchedTiles = 8 * kScanThreads;

template <int CHUNK>
__global__ __launch_bounds__(kScanThreads) void k_sched_count(const uint32_t* __restrict__ ranges, int64_t n_tiles,
                                                              uint32_t* __restrict__ nch,
                                                              uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t s_h[kScanThreads / fgd::kWave], s_l[kScanThreads / fgd::kWave],
        s_m[kScanThreads / fgd::kWave];
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    const int64_t base = (int64_t)blockIdx.x * kSchedTiles;
    uint32_t h = 0, l = 0, m = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int64_t t = base + (int64_t)tid * 8 + k;
        const uint32_t c = t < n_tiles ? (ranges[2 * t + 1] - ranges[2 * t] + CHUNK - 1) / CHUNK : 0u;
        if (t < n_tiles) nch[t] = c;
        if (c > 1) {
            h += 1u;
            m += c;
        } else if (c == 1) {
            l += 1u;
        }
    }
#pragma unroll
    for (int d = fgd::kWave / 2; d > 0; d >>= 1) {
        h += __shfl_xor(h, d, fgd::kWave);
        l += __shfl_xor(l, d, fgd::kWave);
        m += __shfl_xor(m, d, fgd::kWave);
    }
    if (lane == 0) {
        s_h[wave] = h;
        s_l[wave] = l;
        s_m[wave] = m;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t th = 0, tl = 0, tm = 0;
        for (int w = 0; w < kScanThreads / fgd::kWave; w++) {
            th += s_h[w];
            tl += s_l[w];
            tm += s_m[w];
        }
        bsum[3 * blockIdx.x] = th;
        bsum[3 * blockIdx.x + 1] = tl;
        bsum[3 * blockIdx.x + 2] = tm;
    }
}

// One thread: exclusive scan of the blocks' totals in place, and the counters.
__global__ void k_sched_scan(uint32_t* __restrict__ bsum, int64_t nb, int64_t max_mask_items,
                             uint32_t* __restrict__ counters)
{
    if (threadIdx.x != 0) return;
    uint32_t h = 0, l = 0, m = 0;
    for (int64_t b = 0; b < nb; b++) {
        const uint32_t a0 = bsum[3 * b], a1 = bsum[3 * b + 1], a2 = bsum[3 * b + 2];
        bsum[3 * b] = h;
        bsum[3 * b + 1] = l;
        bsum[3 * b + 2] = m;
        h += a0;
        l += a1;
        m += a2;
    }
    counters[0] = 0u;
    counters[1] = h;
    counters[2] = (int64_t)m < max_mask_items ? m : (uint32_t)max_mask_items;
    counters[3] = h + l;
}

template <int CHUNK>
__global__ __launch_bounds__(kScanThreads) void k_sched_write(int64_t n_tiles, const uint32_t* __restrict__ nch,
                                                              const uint32_t* __restrict__ bsum,
                                                              uint32_t* __restrict__ mfirst,
                                                              uint32_t* __restrict__ order)
{
    __shared__ unsigned long long s_wave[kScanThreads / fgd::kWave];
    __shared__ uint32_t s_wave_m[kScanThreads / fgd::kWave];
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    const int64_t base = (int64_t)blockIdx.x * kSchedTiles;
    uint32_t c[8];
    unsigned long long sum = 0;  // low 32: heavy tiles, high 32: light tiles
    uint32_t msum = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int64_t t = base + (int64_t)tid * 8 + k;
        c[k] = t < n_tiles ? nch[t] : 0u;
        if (c[k] > 1) {
            sum += 1ull;
            msum += c[k];
        } else if (c[k] == 1) {
            sum += 1ull << 32;
        }
    }
    unsigned long long x = sum;
    uint32_t xm = msum;
#pragma unroll
    for (int d = 1; d < fgd::kWave; d <<= 1) {
        const unsigned long long y = __shfl_up(x, d, fgd::kWave);
        const uint32_t ym = __shfl_up(xm, d, fgd::kWave);
        if (lane >= d) {
            x += y;
            xm += ym;
        }
    }
    if (lane == fgd::kWave - 1) {
        s_wave[wave] = x;
        s_wave_m[wave] = xm;
    }
    __syncthreads();
    unsigned long long run = (unsigned long long)bsum[3 * blockIdx.x] |
                             ((unsigned long long)bsum[3 * blockIdx.x + 1] << 32);
    uint32_t mf = bsum[3 * blockIdx.x + 2];
    for (int w = 0; w < wave; w++) {
        run += s_wave[w];
        mf += s_wave_m[w];
    }
    run += x - sum;
    mf += xm - msum;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int64_t t = base + (int64_t)tid * 8 + k;
        if (t < n_tiles && c[k] > 0) {
            if (c[k] > 1) {
                order[(uint32_t)run] = (uint32_t)t;
                mfirst[t] = mf;
                run += 1ull;
                mf += c[k];
            } else {
                order[n_tiles - 1 - (int64_t)(run >> 32)] = (uint32_t)t;
                run += 1ull << 32;
            }
        }
    }
}

using fgd::kNoBox;
using fgd::splat_box;

// Stage splats [start, start + cnt) of the sorted list into LDS, with their
// boxes on this tile.
__device__ __forceinline__ void stage(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                      const float4* __restrict__ rgb_depth, const uint32_t* __restrict__ vals,
                                      uint32_t start, int cnt, int tx, int ty, int W, int H, float2* s_xy,
                                      float4* s_co, float4* s_rgb, uint32_t* s_box)
{
    for (int j = threadIdx.x; j < cnt; j += kThreads) {
        const uint32_t g = vals[start + j];
        const float2 mm = xy[g];
        const float4 co = conic_o[g];
        s_xy[j] = mm;
        s_co[j] = co;
        if (s_rgb) s_rgb[j] = rgb_depth[g];
        s_box[j] = splat_box(mm, co, tx, ty, W, H);
    }
}

// The skip tests of Eq. (2) for one pixel inside the splat's box: false if
// power > 0 or power < -5.6 (then alpha < 1/255 since opacity <= 1) or alpha
// < 1/255; otherwise alpha = min(0.99, opacity exp(power)).
template <bool STATS>
__device__ __forceinline__ bool pixel_alpha(float2 mm, float4 co, float fpx, float fpy, float& alpha, Frag& f)
{
    const float dx = mm.x - fpx;
    const float dy = mm.y - fpy;
    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
    if (STATS) ++f.n_eval;
    if (power > 0.0f || power < kSkipPower) return false;
    if (STATS) ++f.n_exp;
    float a = co.w * fgd::exp_neg_in_range(power);
    a = a < 0.99f ? a : 0.99f;
    if (a < 1.0f / 255.0f) return false;
    if (STATS) ++f.n_pass;
    alpha = a;
    return true;
}

__device__ __forceinline__ uint32_t box_area(uint32_t b)
{
    const int x0 = (int)(b & 255u), x1 = (int)((b >> 8) & 255u);
    const int y0 = (int)((b >> 16) & 255u), y1 = (int)(b >> 24);
    return x0 <= x1 ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
}

// Exclusive prefix of the staged splats' box areas: s_pref[j] = sum of the
// areas of splats [0, j), s_pref[cnt] = their total. One thread per S
// consecutive splats; ends with a barrier.
template <int CHUNK>
__device__ __forceinline__ void area_prefix(const uint32_t* s_box, int cnt, uint32_t* s_pref, uint32_t* s_wave)
{
    constexpr int S = CHUNK >= kThreads ? CHUNK / kThreads : 1;
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    uint32_t a[S], sum = 0;
#pragma unroll
    for (int k = 0; k < S; k++) {
        const int j = tid * S + k;
        a[k] = j < cnt ? box_area(s_box[j]) : 0u;
        sum += a[k];
    }
    uint32_t x = sum;
#pragma unroll
    for (int d = 1; d < fgd::kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, fgd::kWave);
        if (lane >= d) x += y;
    }
    if (lane == fgd::kWave - 1) s_wave[wave] = x;
    __syncthreads();
    uint32_t run = x - sum, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / fgd::kWave; w++) {
        const uint32_t t = s_wave[w];
        if (w < wave) run += t;
        total += t;
    }
#pragma unroll
    for (int k = 0; k < S; k++) {
        const int j = tid * S + k;
        if (j < cnt) s_pref[j] = run;
        run += a[k];
    }
    if (tid == 0) s_pref[cnt] = total;
    __syncthreads();
}

// Pass masks of the staged splats by (splat, pixel) pairs: the pairs inside
// the splats' boxes, in splat order and rows then columns within a box, are
// split into equal runs of consecutive pairs, one per thread, so a few large
// splats and many small ones cost the same per thread. A pair that passes
// the skip tests sets bit j of its pixel's mask word j/32 (s_mask
// [word][pixel], zero on entry). Needs area_prefix first.
template <bool STATS>
__device__ __forceinline__ void pair_masks(const float2* s_xy, const float4* s_co, const uint32_t* s_box,
                                           const uint32_t* s_pref, int cnt, int tx, int ty, uint32_t* s_mask,
                                           Frag& f)
{
    const uint32_t total = s_pref[cnt];
    const uint32_t per = (total + kThreads - 1) / kThreads;
    uint32_t q = (uint32_t)threadIdx.x * per;
    const uint32_t qend = q + per < total ? q + per : total;
    if (q >= qend) return;
    // the splat holding pair q: the last j with s_pref[j] <= q
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pref[mid] <= q) lo = mid; else hi = mid;
    }
    int j = lo;
    uint32_t b = s_box[j];
    int x0 = (int)(b & 255u), x1 = (int)((b >> 8) & 255u), y0 = (int)((b >> 16) & 255u), y1 = (int)(b >> 24);
    const uint32_t local = q - s_pref[j];
    const int w0 = x1 - x0 + 1;
    int ly = y0 + (int)(local / (uint32_t)w0), lx = x0 + (int)(local % (uint32_t)w0);
    float2 mm = s_xy[j];
    float4 co = s_co[j];
    for (;;) {
        float alpha;
        if (pixel_alpha<STATS>(mm, co, (float)(tx * fgd::kTile + lx) + 0.5f, (float)(ty * fgd::kTile + ly) + 0.5f,
                               alpha, f))
            atomicOr(&s_mask[(j >> 5) * kThreads + ly * fgd::kTile + lx], 1u << (j & 31));
        if (++q >= qend) break;
        if (++lx > x1) {
            lx = x0;
            if (++ly > y1) {  // next splat with a non-empty box
                do {
                    ++j;
                } while (s_pref[j + 1] == s_pref[j]);
                b = s_box[j];
                x0 = (int)(b & 255u);
                x1 = (int)((b >> 8) & 255u);
                y0 = (int)((b >> 16) & 255u);
                y1 = (int)(b >> 24);
                lx = x0;
                ly = y0;
                mm = s_xy[j];
                co = s_co[j];
            }
        }
    }
}

// Narrows [a, b], tile-relative columns of one box row, to the pixels whose
// centre can pass the skip test of Eq. (2). power >= -5.6 is the ellipse
// A dx^2 + 2 B dx dy + C dy^2 <= 11.2 (dx, dy: splat centre minus pixel
// centre), so on a row at offset dy the passing pixel centres lie within
// u + (B dy -+ sqrt(11.2 A - det dy^2)) / A, det = AC - B^2. The interval is
// taken for the bound 11.2 * 1.01 and widened by a slack: for a conic with
// B^2 <= 0.98 AC the float test's rounding moves the form by less than 1e-3,
// far below the 0.11 added, which also covers the rounding of det, the
// discriminant, the approximate reciprocal and square root here; so no pixel
// the test keeps is dropped, and each pixel inside is still tested exactly.
// Nearly degenerate or non-finite conics keep the whole row. a > b on return
// when no pixel of the row can pass.
__device__ __forceinline__ void row_span(float2 mm, float4 co, float fy, int tx, int& a, int& b)
{
    const float A = co.x, B = co.y, Cq = co.z;
    if (!(A > 0.0f) || !(B * B <= 0.98f * (A * Cq))) return;
    const float dy = mm.y - fy;
    const float det = A * Cq - B * B;
    const float disc = (11.2f * 1.01f) * A - det * (dy * dy);
    if (disc < 0.0f) {
        b = a - 1;
        return;
    }
    const float inv = __builtin_amdgcn_rcpf(A);
    const float half = __builtin_amdgcn_sqrtf(disc) * inv;
    const float cen = (mm.x - (float)(tx * fgd::kTile) - 0.5f) + (B * dy) * inv;
    const float slack = 0.05f + 1e-4f * (fabsf(cen) + half);
    const float lo = ceilf(cen - half - slack), hi = floorf(cen + half + slack);
    // clipped in float (a NaN bound keeps the box column) before converting
    const float fa = fminf(fmaxf(lo, (float)a), (float)(b + 1));
    const float fb = fmaxf(fminf(hi, (float)b), (float)(a - 1));
    a = (int)fa;
    b = (int)fb;
}

// Pass masks of one splat (index j of the chunk, box b) on its rows: every
// pixel of each row's span that passes the skip tests (pixel_alpha) sets bit
// j of its mask word j/32 (s_mask [word][pixel]).
template <bool STATS>
__device__ __forceinline__ void splat_rows(float2 mm, float4 co, uint32_t b, int j, int tx, int ty,
                                           uint32_t* s_mask, Frag& f)
{
    const int x0 = (int)(b & 255u), x1 = (int)((b >> 8) & 255u);
    const int y0 = (int)((b >> 16) & 255u), y1 = (int)(b >> 24);
    if (x0 > x1) return;
    const uint32_t bit = 1u << (j & 31);
    uint32_t* mrow = s_mask + (j >> 5) * kThreads;
    for (int ly = y0; ly <= y1; ly++) {
        const float fy = (float)(ty * fgd::kTile + ly) + 0.5f;
        int a = x0, e = x1;
        row_span(mm, co, fy, tx, a, e);
        for (int lx = a; lx <= e; lx++) {
            float alpha;
            if (pixel_alpha<STATS>(mm, co, (float)(tx * fgd::kTile + lx) + 0.5f, fy, alpha, f))
                atomicOr(&mrow[ly * fgd::kTile + lx], bit);
        }
    }
}

// Splat-parallel pass masks of staged splats: each thread takes whole splats
// (s_mask zero on entry). Suits many small splats; a few large ones are
// better served by pair_masks.
template <bool STATS>
__device__ __forceinline__ void splat_masks(const float2* s_xy, const float4* s_co, const uint32_t* s_box, int cnt,
                                            int tx, int ty, uint32_t* s_mask, Frag& f)
{
    for (int j = threadIdx.x; j < cnt; j += kThreads) splat_rows<STATS>(s_xy[j], s_co[j], s_box[j], j, tx, ty, s_mask, f);
}

template <bool STATS, int N>
__device__ __forceinline__ void flush_stats(const Frag& f, unsigned long long* frag_stats)
{
    if (!STATS) return;
    const unsigned long long c[4] = {f.n_eval, f.n_exp, f.n_pass, f.n_blend};
#pragma unroll
    for (int k = 0; k < N; k++) {
        unsigned long long v = c[k];
#pragma unroll
        for (int d = fgd::kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, fgd::kWave);
        if (fgd::lane_id() == 0) atomicAdd(&frag_stats[k], v);
    }
}

// alpha of a fragment that passed the skip tests (so -5.6 <= power <= 0):
// the same expressions as pixel_alpha, hence the same value.
__device__ __forceinline__ float passed_alpha(float2 mm, float4 co, float fpx, float fpy)
{
    const float dx = mm.x - fpx;
    const float dy = mm.y - fpy;
    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
    const float alpha = co.w * fgd::exp_neg_in_range(power);
    return alpha < 0.99f ? alpha : 0.99f;
}

// Pass masks of the chunks of heavy tiles, one chunk per work item (their
// splats are mostly small: splat-parallel); masks go to global memory
// [word][pixel].
template <int CHUNK, bool STATS>
__global__ __launch_bounds__(kThreads) void k_masks(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ ranges, RenderViews V,
                                                    RenderWs ws, unsigned long long* __restrict__ frag_stats)
{
    constexpr int kWords = CHUNK / 32;
    __shared__ uint32_t s_mask[kWords * kThreads];
    Frag f = {0, 0, 0, 0};
    const int tid = threadIdx.x;
    const uint32_t n_items = ws.counters[2];
#pragma unroll
    for (int w = 0; w < kWords; w++) s_mask[w * kThreads + tid] = 0u;
    __syncthreads();
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t tile = ws.mitem[item];
        const uint32_t chunk = item - ws.mfirst[tile];
        const uint32_t r0 = ranges[2 * tile], r1 = ranges[2 * tile + 1];
        const uint32_t start = r0 + chunk * CHUNK;
        const int cnt = (int)(r1 - start < (uint32_t)CHUNK ? r1 - start : (uint32_t)CHUNK);
        const TileGeom tg = tile_geom(V, tile);
        // each thread its own splats of the chunk, straight from the splat
        // records (no staging: no other thread reads them)
        for (int j = tid; j < cnt; j += kThreads) {
            const uint32_t g = vals[start + j];
            const float2 mm = xy[g];
            const float4 co = conic_o[g];
            splat_rows<STATS>(mm, co, fgd::splat_box(mm, co, tg.tx, tg.ty, tg.W, tg.H), j, tg.tx, tg.ty, s_mask, f);
        }
        __syncthreads();
        uint32_t* out = ws.masks + (size_t)item * (kWords * kThreads);
#pragma unroll
        for (int w = 0; w < kWords; w++) {
            out[w * kThreads + tid] = s_mask[w * kThreads + tid];
            s_mask[w * kThreads + tid] = 0u;  // this thread's column, for the next item
        }
        __syncthreads();
    }
    flush_stats<STATS, 3>(f, STATS ? frag_stats + 4 : frag_stats);
}

struct PixelState {
    float T, C0, C1, C2;
    uint32_t last;
    bool done;
};

// One blend step of Eq. (2) in list order, for a lane whose step is valid
// and whose pixel has not stopped: stop before a splat that would take T
// below 1e-4, otherwise accumulate its colour and attenuate T. Written with
// selects rather than branches (the kept values are the same expressions),
// so the four steps of a group run without divergent control flow.
template <bool STATS>
__device__ __forceinline__ void blend_step(PixelState& p, bool valid, float alpha, float4 c, uint32_t pos, Frag& f)
{
    const float Tn = p.T * (1.0f - alpha);
    const bool live = valid && !p.done;
    const bool stop = Tn < 1e-4f;
    const bool take = live && !stop;
    const float n0 = p.C0 + (c.x * alpha) * p.T;
    const float n1 = p.C1 + (c.y * alpha) * p.T;
    const float n2 = p.C2 + (c.z * alpha) * p.T;
    p.C0 = take ? n0 : p.C0;
    p.C1 = take ? n1 : p.C1;
    p.C2 = take ? n2 : p.C2;
    p.T = take ? Tn : p.T;
    p.last = take ? pos + 1u : p.last;
    p.done = p.done || (live && stop);
    if (STATS) f.n_blend += take ? 1u : 0u;
}

// Walks the marked splats of one staged chunk for this lane's pixel. mcol
// points at the pixel's first mask word (words STRIDE apart). A summary
// bit per 64-splat pair of words, read first, sends the lane straight to the
// non-empty words. Up to four marked splats of one such word are taken at a
// time and their alphas (independent of T) computed together, so their LDS
// reads and arithmetic overlap; the blend steps then run strictly in list
// order.
//
// With LPP > 1 lanes per pixel (heavy tiles), the LPP lanes of a pixel hold
// the same mask words and state and run the same steps in lockstep; lane
// `sub` of the pixel computes the alphas of group positions sub, sub + LPP,
// ..., and the group's alphas are exchanged across the pixel's lanes (which
// lie 64 / LPP apart) before the blend steps, so each lane evaluates 4 / LPP
// exponentials per group instead of 4. Every lane then applies the same
// steps to the same values, and the results equal the one-lane walk's.
template <int LPP>
__device__ __forceinline__ void group_alphas(const float2* s_xy, const float4* s_co, float fpx, float fpy, int sub,
                                             int j0, int j1, int j2, int j3, float& a0, float& a1, float& a2,
                                             float& a3)
{
    constexpr int P = fgd::kWave / LPP;
    if constexpr (LPP == 1) {
        a0 = passed_alpha(s_xy[j0], s_co[j0], fpx, fpy);
        a1 = passed_alpha(s_xy[j1], s_co[j1], fpx, fpy);
        a2 = passed_alpha(s_xy[j2], s_co[j2], fpx, fpy);
        a3 = passed_alpha(s_xy[j3], s_co[j3], fpx, fpy);
    } else if constexpr (LPP == 2) {
        const int ja = sub ? j1 : j0, jb = sub ? j3 : j2;
        const float ma = passed_alpha(s_xy[ja], s_co[ja], fpx, fpy);
        const float mb = passed_alpha(s_xy[jb], s_co[jb], fpx, fpy);
        const float oa = __shfl_xor(ma, P, fgd::kWave);
        const float ob = __shfl_xor(mb, P, fgd::kWave);
        a0 = sub ? oa : ma;
        a1 = sub ? ma : oa;
        a2 = sub ? ob : mb;
        a3 = sub ? mb : ob;
    } else {
        static_assert(LPP == 4, "1, 2 or 4 lanes per pixel");
        const int jm = sub == 0 ? j0 : sub == 1 ? j1 : sub == 2 ? j2 : j3;
        const float m = passed_alpha(s_xy[jm], s_co[jm], fpx, fpy);
        // the alpha of position k sits on the pixel's lane k, i.e. at lane
        // distance (k ^ sub) * P
        const float x1 = __shfl_xor(m, P, fgd::kWave);
        const float x2 = __shfl_xor(m, 2 * P, fgd::kWave);
        const float x3 = __shfl_xor(m, 3 * P, fgd::kWave);
        const auto pick = [&](int d) { return d == 0 ? m : d == 1 ? x1 : d == 2 ? x2 : x3; };
        a0 = pick(sub);
        a1 = pick(1 ^ sub);
        a2 = pick(2 ^ sub);
        a3 = pick(3 ^ sub);
    }
}

template <int CHUNK, bool STATS, int STRIDE, int LPP = 1>
__device__ __forceinline__ void walk(const uint32_t* mcol, const float2* s_xy, const float4* s_co,
                                     const float4* s_rgb, float fpx, float fpy, uint32_t base, PixelState& p,
                                     Frag& f, int sub = 0)
{
    constexpr int kPairs = CHUNK / 64;
    uint32_t summary = 0;
#pragma unroll
    for (int k = 0; k < kPairs; k++)
        summary |= ((mcol[(2 * k) * STRIDE] | mcol[(2 * k + 1) * STRIDE]) != 0u ? 1u : 0u) << k;
    while (summary != 0u && !p.done) {
        const int k = __builtin_ctz(summary);
        summary &= summary - 1u;
        unsigned long long m = (unsigned long long)mcol[(2 * k) * STRIDE] |
                               ((unsigned long long)mcol[(2 * k + 1) * STRIDE] << 32);
        const int b = k << 6;
        while (m != 0ull && !p.done) {
            const int j0 = b + __builtin_ctzll(m);
            m &= m - 1ull;
            const bool v1 = m != 0ull;
            const int j1 = v1 ? b + __builtin_ctzll(m) : j0;
            m &= m - 1ull;
            const bool v2 = m != 0ull;
            const int j2 = v2 ? b + __builtin_ctzll(m) : j0;
            m &= m - 1ull;
            const bool v3 = m != 0ull;
            const int j3 = v3 ? b + __builtin_ctzll(m) : j0;
            m &= m - 1ull;
            float a0, a1, a2, a3;
            group_alphas<LPP>(s_xy, s_co, fpx, fpy, sub, j0, j1, j2, j3, a0, a1, a2, a3);
            const float4 c0 = s_rgb[j0], c1 = s_rgb[j1], c2 = s_rgb[j2], c3 = s_rgb[j3];
            blend_step<STATS>(p, true, a0, c0, base + (uint32_t)j0, f);
            blend_step<STATS>(p, v1, a1, c1, base + (uint32_t)j1, f);
            blend_step<STATS>(p, v2, a2, c2, base + (uint32_t)j2, f);
            blend_step<STATS>(p, v3, a3, c3, base + (uint32_t)j3, f);
        }
    }
}

// Register copy of one chunk for one wave of a heavy tile: the splat records
// this lane stages (every 64th of the chunk) and the mask words of its pixel
// (zero where the masks are computed in place).
template <int CHUNK>
struct ChunkRegs {
    static constexpr int S = CHUNK / fgd::kWave;
    float2 xy[S];
    float4 co[S];
    float4 rgb[S];
    uint32_t m[CHUNK / 32];
};

template <int CHUNK>
__device__ __forceinline__ int chunk_count(uint32_t r0, uint32_t r1, uint32_t chunk)
{
    const uint32_t start = r0 + chunk * CHUNK;
    return r1 > start ? (int)(r1 - start < (uint32_t)CHUNK ? r1 - start : (uint32_t)CHUNK) : 0;
}

template <int CHUNK>
__device__ __forceinline__ void fetch_vals(const uint32_t* __restrict__ vals, uint32_t r0, uint32_t r1, uint32_t chunk,
                                           uint32_t (&g)[ChunkRegs<CHUNK>::S])
{
    const int cnt = chunk_count<CHUNK>(r0, r1, chunk);
    const uint32_t start = r0 + chunk * CHUNK;
#pragma unroll
    for (int k = 0; k < ChunkRegs<CHUNK>::S; k++) {
        const int j = k * fgd::kWave + fgd::lane_id();
        g[k] = j < cnt ? vals[start + j] : 0u;
    }
}

template <int CHUNK>
__device__ __forceinline__ void fetch_chunk(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                            const float4* __restrict__ rgb_depth, const uint32_t* __restrict__ masks,
                                            uint32_t r0, uint32_t r1, uint32_t chunk,
                                            const uint32_t (&g)[ChunkRegs<CHUNK>::S], uint32_t mf,
                                            uint32_t n_mask_items, int pix, ChunkRegs<CHUNK>& R)
{
    const int cnt = chunk_count<CHUNK>(r0, r1, chunk);
#pragma unroll
    for (int k = 0; k < ChunkRegs<CHUNK>::S; k++) {
        const int j = k * fgd::kWave + fgd::lane_id();
        if (j < cnt) {
            R.xy[k] = xy[g[k]];
            R.co[k] = conic_o[g[k]];
            R.rgb[k] = rgb_depth[g[k]];
        } else {
            R.xy[k] = make_float2(0.0f, 0.0f);
            R.co[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            R.rgb[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    if (mf + chunk < n_mask_items) {
        const uint32_t* src = masks + (size_t)(mf + chunk) * (CHUNK / 32 * kThreads);
#pragma unroll
        for (int w = 0; w < CHUNK / 32; w++) R.m[w] = src[w * kThreads + pix];
    } else {
#pragma unroll
        for (int w = 0; w < CHUNK / 32; w++) R.m[w] = 0u;
    }
}

// Orders this wave's LDS writes before its own later LDS reads (and reads
// before later writes); no other wave takes part.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass masks of a staged chunk for the 64 / LPP pixels of one wave (rows
// y0 .. y0 + 4 / LPP - 1 of the tile), when the chunk's masks were not
// stored: each lane takes every 64th splat and tests the pixels of its box
// in those rows. w_mask [word][64] is zero on entry; a pixel's bits go to
// each of its LPP lanes' columns.
template <bool STATS, int LPP>
__device__ __forceinline__ void wave_masks(const float2* w_xy, const float4* w_co, int cnt, int tx, int ty, int W,
                                           int H, int y0, uint32_t* w_mask, Frag& f)
{
    constexpr int P = fgd::kWave / LPP;
    constexpr int kRows = P / fgd::kTile;
    for (int j = fgd::lane_id(); j < cnt; j += fgd::kWave) {
        const float2 mm = w_xy[j];
        const float4 co = w_co[j];
        const uint32_t b = splat_box(mm, co, tx, ty, W, H);
        const int x0 = (int)(b & 255u), x1 = (int)((b >> 8) & 255u);
        const int by0 = (int)((b >> 16) & 255u), by1 = (int)(b >> 24);
        if (x0 > x1) continue;
        const int ya = by0 > y0 ? by0 : y0, yb = by1 < y0 + kRows - 1 ? by1 : y0 + kRows - 1;
        const uint32_t bit = 1u << (j & 31);
        uint32_t* mrow = w_mask + (j >> 5) * fgd::kWave;
        for (int ly = ya; ly <= yb; ly++) {
            const float fy = (float)(ty * fgd::kTile + ly) + 0.5f;
            int a = x0, b = x1;
            row_span(mm, co, fy, tx, a, b);
            for (int lx = a; lx <= b; lx++) {
                float alpha;
                if (pixel_alpha<STATS>(mm, co, (float)(tx * fgd::kTile + lx) + 0.5f, fy, alpha, f)) {
#pragma unroll
                    for (int c = 0; c < LPP; c++) atomicOr(&mrow[c * P + (ly - y0) * fgd::kTile + lx], bit);
                }
            }
        }
    }
}

// Lanes per pixel in the walk of a long heavy tile: such a tile is
// kHeavyLanes work items of 256 / kHeavyLanes pixels each. Two halve the
// exponentials on the longest tiles' critical path; four cost more in
// staging (every wave stages whole chunks) than they save. Only tiles of at
// least kSplitChunks chunks are split: for shorter ones the doubled staging
// outweighs the shorter walk (the blend was fastest at 16 among 2 to 48).
constexpr int kHeavyLanes = 2;
constexpr int kSplitChunks = 16;

template <int CHUNK, bool STATS, int LPP>
__global__ __launch_bounds__(kThreads) void k_render(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                                     const float4* __restrict__ rgb_depth,
                                                     const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ ranges, int64_t n_tiles,
                                                     RenderViews V, float bg0, float bg1, float bg2, RenderWs ws,
                                                     float* __restrict__ image, float* __restrict__ final_T,
                                                     uint32_t* __restrict__ n_contrib,
                                                     unsigned long long* __restrict__ frag_stats)
{
    constexpr int kWords = CHUNK / 32;
    constexpr int kWaves = kThreads / fgd::kWave;
    // a light tile uses the first CHUNK records; a heavy tile gives each wave
    // its own CHUNK records and its pixels' mask columns
    __shared__ float2 s_xy[kWaves * CHUNK];
    __shared__ float4 s_co[kWaves * CHUNK];
    __shared__ float4 s_rgb[kWaves * CHUNK];
    __shared__ uint32_t s_mask[kWords * kThreads];
    __shared__ uint32_t s_box[CHUNK];
    __shared__ uint32_t s_pref[CHUNK + 1];
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_item;
    constexpr int P = fgd::kWave / LPP;  // pixels per wave in a heavy tile
    const int tid = threadIdx.x;
    const int wave = tid / fgd::kWave, lane = fgd::lane_id();
    const uint32_t n_mask_items = ws.counters[2];
    const uint32_t n_heavy = ws.counters[1];
    // each heavy tile is LPP items (parts of 256 / LPP pixels), each light tile one
    const uint32_t n_work = ws.counters[3] + (uint32_t)(LPP - 1) * n_heavy;
    Frag f = {0, 0, 0, 0};
    if (tid == 0) s_item = atomicAdd(&ws.counters[0], 1u);
    __syncthreads();
    for (;;) {
        const uint32_t item = s_item;
        if (item >= n_work) break;
        const bool heavy_item = item < (uint32_t)LPP * n_heavy;
        const uint32_t tile = ws.order[heavy_item ? (int64_t)(item / LPP)
                                                  : n_tiles - 1 - (int64_t)(item - (uint32_t)LPP * n_heavy)];
        const uint32_t nch = ws.nch[tile];
        // a heavy tile with fewer than kSplitChunks chunks is walked whole by
        // its first item, one lane per pixel; its other items are empty
        const bool split = LPP > 1 && heavy_item && nch >= (uint32_t)kSplitChunks;
        const int part = heavy_item ? (int)(item % LPP) : 0;
        if (heavy_item && !split && part != 0) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(&ws.counters[0], 1u);
            __syncthreads();
            continue;
        }
        const int sub = split ? lane / P : 0;  // this lane's place among its pixel's lanes
        const int pix = split ? part * (kThreads / LPP) + wave * P + lane % P : tid;
        const int lx = pix % fgd::kTile, ly = pix / fgd::kTile;
        const uint32_t r0 = ranges[2 * tile], r1 = ranges[2 * tile + 1];
        // Tiles are ordered heavy first, so a light tile is followed only by
        // light ones: its workgroup claims the next tile now, hiding the
        // atomic's latency. A heavy tile's workgroup does not, so no tile
        // waits behind a long one.
        uint32_t next_item = 0;
        if (tid == 0 && nch <= 1) next_item = atomicAdd(&ws.counters[0], 1u);
        const uint32_t mf = nch > 1 ? ws.mfirst[tile] : 0u;
        const TileGeom tg = tile_geom(V, tile);
        const int tx = tg.tx, ty = tg.ty, W = tg.W, H = tg.H;
        const int px = tx * fgd::kTile + lx;
        const int py = ty * fgd::kTile + ly;
        const bool inside = px < W && py < H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        PixelState p = {1.0f, 0.0f, 0.0f, 0.0f, 0u, !inside};
        if (nch <= 1) {
            // light tile: one chunk, masks computed here
            const int cnt = (int)(r1 - r0);
#pragma unroll
            for (int w = 0; w < kWords; w++) s_mask[w * kThreads + tid] = 0u;
            stage(xy, conic_o, rgb_depth, vals, r0, cnt, tx, ty, W, H, s_xy, s_co, s_rgb, s_box);
            __syncthreads();
            if (cnt < kPairSplats) {
                area_prefix<CHUNK>(s_box, cnt, s_pref, s_wave);
                pair_masks<STATS>(s_xy, s_co, s_box, s_pref, cnt, tx, ty, s_mask, f);
            } else {
                splat_masks<STATS>(s_xy, s_co, s_box, cnt, tx, ty, s_mask, f);
            }
            __syncthreads();
            walk<CHUNK, STATS, kThreads>(s_mask + tid, s_xy, s_co, s_rgb, fpx, fpy, 0u, p, f);
        } else {
            // heavy tile: each wave walks the chunks for its own 64 / LPP
            // pixels at its own pace, with its own staging area, so no wave waits on the
            // others between chunks. While one chunk is walked, the next
            // chunk's splat records and stored masks are loaded into
            // registers, and the indices of the chunk after it.
            float2* w_xy = s_xy + wave * CHUNK;
            float4* w_co = s_co + wave * CHUNK;
            float4* w_rgb = s_rgb + wave * CHUNK;
            uint32_t* w_mask = s_mask + wave * (kWords * fgd::kWave);
            ChunkRegs<CHUNK> R;
            uint32_t gnext[ChunkRegs<CHUNK>::S];
            {
                uint32_t g0[ChunkRegs<CHUNK>::S];
                fetch_vals<CHUNK>(vals, r0, r1, 0u, g0);
                fetch_chunk<CHUNK>(xy, conic_o, rgb_depth, ws.masks, r0, r1, 0u, g0, mf, n_mask_items, pix, R);
                fetch_vals<CHUNK>(vals, r0, r1, 1u, gnext);
            }
            const unsigned n_blend0 = f.n_blend;
            uint32_t chunk = 0;
            for (; chunk < nch; chunk++) {
                // the wave stops once all of its pixels have terminated
                if (__ballot(!p.done) == 0ull) break;
                const int cnt = chunk_count<CHUNK>(r0, r1, chunk);
                const bool stored = mf + chunk < n_mask_items;
                wave_sync();  // the previous chunk's reads are done
#pragma unroll
                for (int k = 0; k < ChunkRegs<CHUNK>::S; k++) {
                    const int j = k * fgd::kWave + lane;
                    if (j < cnt) {
                        w_xy[j] = R.xy[k];
                        w_co[j] = R.co[k];
                        w_rgb[j] = R.rgb[k];
                    }
                }
                // zero where the masks are computed here
#pragma unroll
                for (int w = 0; w < kWords; w++) w_mask[w * fgd::kWave + lane] = R.m[w];
                wave_sync();
                if (chunk + 1 < nch) {
                    fetch_chunk<CHUNK>(xy, conic_o, rgb_depth, ws.masks, r0, r1, chunk + 1, gnext, mf, n_mask_items,
                                       pix, R);
                    if (chunk + 2 < nch) fetch_vals<CHUNK>(vals, r0, r1, chunk + 2, gnext);
                }
                if (!stored) {  // beyond the mask store: masks computed here
                    if (split)
                        wave_masks<STATS, LPP>(w_xy, w_co, cnt, tx, ty, W, H, (pix - lane % P) / fgd::kTile, w_mask,
                                               f);
                    else
                        wave_masks<STATS, 1>(w_xy, w_co, cnt, tx, ty, W, H, wave * (fgd::kWave / fgd::kTile), w_mask,
                                             f);
                    wave_sync();
                }
                if (split)
                    walk<CHUNK, STATS, fgd::kWave, LPP>(w_mask + lane, w_xy, w_co, w_rgb, fpx, fpy, chunk * CHUNK, p,
                                                        f, sub);
                else
                    walk<CHUNK, STATS, fgd::kWave, 1>(w_mask + lane, w_xy, w_co, w_rgb, fpx, fpy, chunk * CHUNK, p, f);
                if (ws.state && stored && sub == 0) {  // per-pixel state after this chunk, for the backward
                    float* st = ws.state + (size_t)(mf + chunk) * (4 * kThreads);
                    st[pix] = p.T;
                    st[kThreads + pix] = p.C0;
                    st[2 * kThreads + pix] = p.C1;
                    st[3 * kThreads + pix] = p.C2;
                }
            }
            // the state after every later chunk equals the final one
            if (ws.state && sub == 0) {
                for (; chunk < nch && mf + chunk < n_mask_items; chunk++) {
                    float* st = ws.state + (size_t)(mf + chunk) * (4 * kThreads);
                    st[pix] = p.T;
                    st[kThreads + pix] = p.C0;
                    st[2 * kThreads + pix] = p.C1;
                    st[3 * kThreads + pix] = p.C2;
                }
            }
            if (STATS && sub != 0) f.n_blend = n_blend0;  // a pixel's blends count on its first lane only
        }
        if (inside && (nch <= 1 || sub == 0)) {
            const size_t o = (size_t)py * W + px;
            const size_t plane = (size_t)W * H;
            float* img = image + 3 * tg.pix0;
            img[o] = p.C0 + p.T * bg0;
            img[plane + o] = p.C1 + p.T * bg1;
            img[2 * plane + o] = p.C2 + p.T * bg2;
            final_T[tg.pix0 + o] = p.T;
            n_contrib[tg.pix0 + o] = p.last;
        }
        __syncthreads();  // LDS and s_item are reused by the next tile
        if (tid == 0) s_item = nch <= 1 ? next_item : atomicAdd(&ws.counters[0], 1u);
        __syncthreads();
    }
    flush_stats<STATS, 4>(f, frag_stats);
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int chunk_of(const fg_tune* tune)
{
    if (!tune || !tune->render_batch) return 256;
    return tune->render_batch;
}

// Mask storage is capped; chunks beyond the cap compute their masks in the
// tile's own workgroup (same results, less parallelism).
constexpr int64_t kMaskStoreBytes = (int64_t)256 << 20;

size_t carve(void* base, int64_t n_tiles, int64_t cap_pairs, int chunk, bool save_state, int mask_items,
             RenderWs* w, int64_t* max_mask_items)
{
    const int64_t mask_bytes = (int64_t)(chunk / 32) * kThreads * 4;
    const int64_t need = 2 * ((cap_pairs + chunk - 1) / chunk) + 1;
    int64_t cap = kMaskStoreBytes / mask_bytes;
    if (mask_items > 0 && mask_items < cap) cap = mask_items;
    *max_mask_items = need < cap ? need : cap;
    const size_t state_bytes = save_state ? (size_t)*max_mask_items * 4 * kThreads * 4 : 0;
    const size_t sched_bytes = (size_t)3 * 4 * (size_t)((n_tiles + kSchedTiles - 1) / kSchedTiles + 1);
    const size_t sizes[8] = {(size_t)n_tiles * 4, (size_t)n_tiles * 4, (size_t)n_tiles * 4,
                             (size_t)*max_mask_items * 4, 64, (size_t)*max_mask_items * (size_t)mask_bytes,
                             state_bytes, sched_bytes};
    void** dst[8] = {(void**)&w->nch, (void**)&w->mfirst, (void**)&w->order, (void**)&w->mitem,
                     (void**)&w->counters, (void**)&w->masks, (void**)&w->state, (void**)&w->sched};
    size_t off = 0;
    for (int i = 0; i < 8; i++) {
        if (base) *dst[i] = (char*)base + off;
        off += align_up(sizes[i] + 4);
    }
    if (base && !save_state) w->state = nullptr;
    return off;
}

bool save_of(const fg_tune* tune) { return tune && tune->save_state; }

int mask_items_of(const fg_tune* tune) { return tune ? tune->mask_items : 0; }

template <int CHUNK>
void launch(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const RenderViews& V,
            const float bg[3], float* image, float* final_T, uint32_t* n_contrib, unsigned long long* frag_stats,
            const RenderWs& w, int64_t n_tiles, int64_t max_mask_items, const fg_tune* tune, hipStream_t s)
{
    if (n_tiles <= 4 * kSchedTiles) {
        hipLaunchKernelGGL(k_schedule<CHUNK>, dim3(1), dim3(kScanThreads), 0, s, ranges, n_tiles, max_mask_items,
                           w.nch, w.mfirst, w.order, w.counters);
    } else {
        const int64_t nb = (n_tiles + kSchedTiles - 1) / kSchedTiles;
        hipLaunchKernelGGL(k_sched_count<CHUNK>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ranges, n_tiles, w.nch,
                           w.sched);
        hipLaunchKernelGGL(k_sched_scan, dim3(1), dim3(64), 0, s, w.sched, nb, max_mask_items, w.counters);
        hipLaunchKernelGGL(k_sched_write<CHUNK>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, n_tiles, w.nch,
                           w.sched, w.mfirst, w.order);
    }
    const unsigned gp = (unsigned)(n_tiles < 65536 ? n_tiles : 65536);
    hipLaunchKernelGGL(k_tile_prep<CHUNK>, dim3(gp), dim3(kThreads), 0, s, n_tiles, V, bg[0], bg[1], bg[2], w.nch,
                       w.mfirst, max_mask_items, w.mitem, image, final_T, n_contrib);
    const float2* xy = (const float2*)splats->xy;
    const float4* co = (const float4*)splats->conic_o;
    const float4* rgb = (const float4*)splats->rgb_depth;
    const unsigned gm = (unsigned)(max_mask_items < 4096 ? (max_mask_items < 1 ? 1 : max_mask_items) : 4096);
    const unsigned gr = (unsigned)(n_tiles < 4096 ? n_tiles : 4096);
    if (frag_stats) {
        hipLaunchKernelGGL((k_masks<CHUNK, true>), dim3(gm), dim3(kThreads), 0, s, xy, co, vals, ranges, V, w,
                           frag_stats);
        hipLaunchKernelGGL((k_render<CHUNK, true, kHeavyLanes>), dim3(gr), dim3(kThreads), 0, s, xy, co, rgb, vals, ranges, n_tiles,
                           V, bg[0], bg[1], bg[2], w, image, final_T, n_contrib, frag_stats);
    } else {
        hipLaunchKernelGGL((k_masks<CHUNK, false>), dim3(gm), dim3(kThreads), 0, s, xy, co, vals, ranges, V, w,
                           frag_stats);
        const bool timed = tune && tune->blend_events[0] && tune->blend_events[1];
        if (timed) (void)hipEventRecord((hipEvent_t)tune->blend_events[0], s);
        hipLaunchKernelGGL((k_render<CHUNK, false, kHeavyLanes>), dim3(gr), dim3(kThreads), 0, s, xy, co, rgb, vals, ranges, n_tiles,
                           V, bg[0], bg[1], bg[2], w, image, final_T, n_contrib, frag_stats);
        if (timed) (void)hipEventRecord((hipEvent_t)tune->blend_events[1], s);
    }
}

}  // namespace

namespace {

// The views' geometry and total tile count (-1: invalid views: sizes, more
// than kMaxViews, or global tile ids that are not consecutive from view to
// view).
int64_t make_views(const fg_camera* cams, int32_t n_views, RenderViews* V)
{
    if (!cams || n_views < 1 || n_views > kMaxViews) return -1;
    int64_t total = 0, pix = 0;
    V->n = n_views;
    for (int v = 0; v < n_views; v++) {
        const fg_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0) return -1;
        if ((int64_t)c.tile_base != (int64_t)cams[0].tile_base + total) return -1;
        V->tile0[v] = (uint32_t)total;
        V->W[v] = c.width;
        V->H[v] = c.height;
        V->Wt[v] = (c.width + 15) / 16;
        V->pix0[v] = pix;
        total += (int64_t)V->Wt[v] * ((c.height + 15) / 16);
        pix += (int64_t)c.width * c.height;
        if (total >= ((int64_t)1 << 31)) return -1;
    }
    V->tile0[n_views] = (uint32_t)total;
    for (int v = n_views; v < kMaxViews; v++) {
        V->tile0[v + 1] = (uint32_t)total;
        V->W[v] = V->H[v] = V->Wt[v] = 1;
        V->pix0[v] = pix;
    }
    return total;
}

}  // namespace

extern "C" size_t fg_render_workspace_size(const fg_camera* cams, int32_t n_views, int64_t cap_pairs,
                                           const fg_tune* tune)
{
    RenderViews V;
    const int64_t n_tiles = make_views(cams, n_views, &V);
    if (n_tiles < 0 || cap_pairs < 0) return 0;
    RenderWs w;
    int64_t mi;
    return carve(nullptr, n_tiles, cap_pairs, chunk_of(tune), save_of(tune), mask_items_of(tune), &w, &mi);
}

extern "C" int fg_render(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges,
                         const fg_camera* cams, int32_t n_views, const float bg[3], float* image, float* final_T,
                         uint32_t* n_contrib, int64_t cap_pairs, unsigned long long* frag_stats, uint32_t* status,
                         void* ws, size_t ws_bytes, const fg_tune* tune, void* stream)
{
    (void)status;
    if (!splats || !ranges || !cams || !bg || !image || !final_T || !n_contrib || cap_pairs < 0)
        return FG_ERR_INVALID_ARG;
    RenderViews V;
    const int64_t n_tiles = make_views(cams, n_views, &V);
    if (n_tiles < 0) return FG_ERR_INVALID_ARG;
    const int chunk = chunk_of(tune);
    if (chunk != 128 && chunk != 256 && chunk != 512) return FG_ERR_INVALID_ARG;
    RenderWs w;
    int64_t max_mask_items;
    const bool save = save_of(tune);
    if (!ws || ws_bytes < carve(nullptr, n_tiles, cap_pairs, chunk, save, mask_items_of(tune), &w, &max_mask_items))
        return FG_ERR_WORKSPACE;
    carve(ws, n_tiles, cap_pairs, chunk, save, mask_items_of(tune), &w, &max_mask_items);
    hipStream_t s = (hipStream_t)stream;
    switch (chunk) {
        case 128: launch<128>(splats, vals, ranges, V, bg, image, final_T, n_contrib, frag_stats, w, n_tiles,
                              max_mask_items, tune, s); break;
        case 512: launch<512>(splats, vals, ranges, V, bg, image, final_T, n_contrib, frag_stats, w, n_tiles,
                              max_mask_items, tune, s); break;
        default: launch<256>(splats, vals, ranges, V, bg, image, final_T, n_contrib, frag_stats, w, n_tiles,
                             max_mask_items, tune, s); break;
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

namespace fgr {

bool render_ws_view(const void* ws, size_t ws_bytes, const fg_camera* cam, int64_t cap_pairs, const fg_tune* tune,
                    RenderWsView* v)
{
    if (!ws || !cam || !v || !save_of(tune) || cam->width <= 0 || cam->height <= 0 || cap_pairs < 0) return false;
    const int chunk = chunk_of(tune);
    if (chunk != 128 && chunk != 256 && chunk != 512) return false;
    const int64_t n_tiles = (int64_t)((cam->width + 15) / 16) * ((cam->height + 15) / 16);
    RenderWs w;
    int64_t mi;
    if (ws_bytes < carve(nullptr, n_tiles, cap_pairs, chunk, true, mask_items_of(tune), &w, &mi)) return false;
    carve(const_cast<void*>(ws), n_tiles, cap_pairs, chunk, true, mask_items_of(tune), &w, &mi);
    v->nch = w.nch;
    v->mfirst = w.mfirst;
    v->mitem = w.mitem;
    v->counters = w.counters + 2;
    v->state = w.state;
    v->chunk = chunk;
    v->max_items = mi;
    return true;
}

}  // namespace fgr

extern "C" const char* fg_status_string(int code)
{
    switch (code) {
        case FG_OK: return "ok";
        case FG_ERR_INVALID_ARG: return "invalid argument";
        case FG_ERR_INVALID_TREE: return "invalid tree";
        case FG_ERR_UNSUPPORTED: return "unsupported configuration";
        case FG_ERR_WORKSPACE: return "workspace too small";
        case FG_ERR_HIP: return "HIP launch or runtime error";
        case FG_ERR_SCRATCH: return "problem larger than the fixed scratch array of fg_filter_noalloc";
        default: return "unknown status";
    }
}
