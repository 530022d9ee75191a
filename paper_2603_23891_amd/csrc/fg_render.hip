// Per-tile front-to-back alpha blending, Eq. (2).
//
// In Eq. (2) the per-fragment opacity alpha_i and the skip decisions
// (power > 0, alpha < 1/255) depend only on the splat and the pixel, not on
// the transmittance; only the product T_i = prod (1 - alpha_j), the early
// stop (T < 1e-4) and the colour sum run sequentially. Tiles near a horizon
// can hold ~10^4 splats whose pixels seldom saturate, so one workgroup per
// tile would leave the frame waiting on a single long chain. Instead each
// tile's sorted range is cut into chunks of CHUNK splats, one work item per
// chunk:
//
//   phase 1  (all chunks in parallel) the chunk's splat records are staged in
//            LDS and every pixel (one thread each, 256 per 16x16 tile) marks
//            in a bit mask the splats whose alpha passes the skip tests;
//   phase 2  (in chunk order) the item takes over the per-pixel state
//            (T, C, last, done) left by the previous chunk of its tile and
//            walks only the marked splats, recomputing alpha with the same
//            function, so every value and decision is bit-identical to one
//            sequential pass. It then hands the state to the next chunk
//            (plain stores, one agent-scope release fence, then a per-tile
//            counter; the receiver polls the counter with relaxed loads and
//            takes one acquire fence) or, for the tile's last chunk, writes
//            the pixels.
//
// Work items are claimed from an atomic ticket in (tile, chunk) order, so an
// item only ever waits for an item claimed before it by a running workgroup.
// Items of a tile with a single chunk never wait.
#include "fg_device.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / fgd::kWave;
constexpr uint32_t kSpinLimit = 1u << 26;

// exp(power) <= exp(-5.6) < 1/255 for power < -5.6, so with opacity <= 1 the
// splat is skipped either way: testing this first avoids evaluating the
// exponential without changing any result.
constexpr float kSkipPower = -5.6f;

struct RenderWs {
    uint32_t* nch;        // [n_tiles] chunks per tile, then its first item (exclusive scan)
    uint32_t* slot;       // [n_tiles] state slot of a multi-chunk tile
    uint32_t* done_cnt;   // [n_tiles] chunks of the tile already handed over
    uint32_t* item_tile;  // [max_items]
    uint32_t* counters;   // [0] ticket, [1] n_items
    float* state;         // [max_slots][6][256] T, C0, C1, C2, last, done
};

__device__ __forceinline__ float splat_alpha(float2 m, float4 co, float fpx, float fpy, float& power)
{
    const float dx = m.x - fpx;
    const float dy = m.y - fpy;
    power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
    float alpha = co.w * fgd::exp_neg(power);
    return alpha < 0.99f ? alpha : 0.99f;
}

template <int CHUNK>
__global__ __launch_bounds__(kThreads) void k_chunk_count(const uint32_t* __restrict__ ranges, int64_t n_tiles,
                                                          uint32_t* __restrict__ nch, uint32_t* __restrict__ done_cnt)
{
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t < n_tiles) {
        const uint32_t L = ranges[2 * t + 1] - ranges[2 * t];
        nch[t] = L == 0 ? 1u : (L + CHUNK - 1) / CHUNK;
        done_cnt[t] = 0u;
    }
}

// One workgroup of 1024 threads: exclusive scan of the chunk counts (first
// item of each tile), state slots of multi-chunk tiles, the item -> tile map,
// n_items, and the ticket reset. 8 consecutive tiles per thread per round.
__global__ __launch_bounds__(1024) void k_chunk_scan(uint32_t* __restrict__ nch, uint32_t* __restrict__ slot,
                                                     uint32_t* __restrict__ item_tile, int64_t n_tiles,
                                                     int64_t max_items, uint32_t* __restrict__ counters)
{
    __shared__ unsigned long long s_wave[1024 / fgd::kWave];
    __shared__ unsigned long long s_carry;
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    if (tid == 0) s_carry = 0ull;
    __syncthreads();
    for (int64_t base = 0; base < n_tiles; base += 8 * 1024) {
        uint32_t c[8];
        unsigned long long sum = 0;  // low 32: items, high 32: multi-chunk tiles
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t t = base + (int64_t)tid * 8 + k;
            c[k] = t < n_tiles ? nch[t] : 0u;
            sum += (unsigned long long)c[k] | ((unsigned long long)(c[k] > 1) << 32);
        }
        unsigned long long x = sum;
#pragma unroll
        for (int d = 1; d < fgd::kWave; d <<= 1) {
            const unsigned long long y = __shfl_up(x, d, fgd::kWave);
            if (lane >= d) x += y;
        }
        if (lane == fgd::kWave - 1) s_wave[wave] = x;
        __syncthreads();
        unsigned long long before = s_carry, total = 0;
        for (int w = 0; w < 1024 / fgd::kWave; w++) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        unsigned long long run = before + x - sum;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int64_t t = base + (int64_t)tid * 8 + k;
            if (t < n_tiles) {
                const uint32_t first = (uint32_t)run;
                nch[t] = first;
                slot[t] = (uint32_t)(run >> 32);
                for (uint32_t i = 0; i < c[k]; i++)
                    if ((int64_t)(first + i) < max_items) item_tile[first + i] = (uint32_t)t;
            }
            run += (unsigned long long)c[k] | ((unsigned long long)(c[k] > 1) << 32);
        }
        __syncthreads();
        if (tid == 0) s_carry += total;
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t items = (uint32_t)s_carry;
        counters[0] = 0u;
        counters[1] = (int64_t)items < max_items ? items : (uint32_t)max_items;
    }
}

template <int CHUNK, bool STATS>
__global__ __launch_bounds__(kThreads) void k_render(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                                     const float4* __restrict__ rgb_depth,
                                                     const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ ranges, int W, int H, int Wt,
                                                     float bg0, float bg1, float bg2, RenderWs ws, int64_t max_slots,
                                                     float* __restrict__ image, float* __restrict__ final_T,
                                                     uint32_t* __restrict__ n_contrib,
                                                     unsigned long long* __restrict__ frag_stats,
                                                     uint32_t* __restrict__ status)
{
    constexpr int kWords = CHUNK / 32;
    __shared__ float2 s_xy[CHUNK];
    __shared__ float4 s_co[CHUNK];
    __shared__ float4 s_rgb[CHUNK];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    const uint32_t n_items = ws.counters[1];
    uint32_t n_eval = 0, n_exp = 0, n_pass = 0, n_blend = 0;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(&ws.counters[0], 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= n_items) break;
        const uint32_t tile = ws.item_tile[item];
        const uint32_t first = ws.nch[tile];
        const uint32_t chunk = item - first;
        const uint32_t r0 = ranges[2 * tile], r1 = ranges[2 * tile + 1];
        const bool last_chunk = (uint64_t)r0 + (uint64_t)(chunk + 1) * CHUNK >= (uint64_t)r1;
        const uint32_t start = r0 + chunk * CHUNK;
        const int cnt = r1 > start ? (int)(r1 - start < (uint32_t)CHUNK ? r1 - start : (uint32_t)CHUNK) : 0;
        const int tx = (int)(tile % (uint32_t)Wt), ty = (int)(tile / (uint32_t)Wt);
        const int px = tx * fgd::kTile + (tid % fgd::kTile);
        const int py = ty * fgd::kTile + (tid / fgd::kTile);
        const bool inside = px < W && py < H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

        // ---- phase 1: stage the chunk and mark the splats whose alpha passes
        for (int j = tid; j < cnt; j += kThreads) {
            const uint32_t g = vals[start + j];
            s_xy[j] = xy[g];
            s_co[j] = conic_o[g];
            s_rgb[j] = rgb_depth[g];
        }
        __syncthreads();
        uint32_t mask[kWords];
#pragma unroll
        for (int w = 0; w < kWords; w++) {
            uint32_t m = 0;
            if (inside) {
                const int jn = cnt - w * 32 < 32 ? cnt - w * 32 : 32;
                for (int b = 0; b < jn; b++) {
                    const int j = w * 32 + b;
                    const float2 mm = s_xy[j];
                    const float4 co = s_co[j];
                    const float dx = mm.x - fpx;
                    const float dy = mm.y - fpy;
                    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
                    if (STATS) ++n_eval;
                    if (power > 0.0f || power < kSkipPower) continue;
                    if (STATS) ++n_exp;
                    float alpha = co.w * fgd::exp_neg(power);
                    alpha = alpha < 0.99f ? alpha : 0.99f;
                    if (alpha < 1.0f / 255.0f) continue;
                    if (STATS) ++n_pass;
                    m |= 1u << b;
                }
            }
            mask[w] = m;
        }

        // ---- phase 2: take over the pixel state and walk the marked splats
        float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
        uint32_t last = 0;
        bool done = !inside;
        const uint32_t sl = ws.slot[tile];
        float* st = ws.state + (size_t)(sl < max_slots ? sl : 0) * (6 * kThreads);
        if (chunk > 0) {
            if (tid == 0) {
                uint32_t spins = 0;
                while (__hip_atomic_load(&ws.done_cnt[tile], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != chunk) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit) {  // never expected: the previous chunk always hands over
                        atomicOr(status, FG_STATUS_LOOKBACK_STALL);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            T = st[0 * kThreads + tid];
            C0 = st[1 * kThreads + tid];
            C1 = st[2 * kThreads + tid];
            C2 = st[3 * kThreads + tid];
            last = __float_as_uint(st[4 * kThreads + tid]);
            done = st[5 * kThreads + tid] != 0.0f;
        }
#pragma unroll
        for (int w = 0; w < kWords; w++) {
            uint32_t m = mask[w];
            while (m != 0u && !done) {
                const int b = __builtin_ctz(m);
                m &= m - 1u;
                const int j = w * 32 + b;
                float power;
                const float alpha = splat_alpha(s_xy[j], s_co[j], fpx, fpy, power);
                const float Tn = T * (1.0f - alpha);
                if (Tn < 1e-4f) {
                    done = true;
                    break;
                }
                const float4 c = s_rgb[j];
                C0 = C0 + (c.x * alpha) * T;
                C1 = C1 + (c.y * alpha) * T;
                C2 = C2 + (c.z * alpha) * T;
                T = Tn;
                last = chunk * CHUNK + (uint32_t)j + 1u;
                if (STATS) ++n_blend;
            }
        }
        if (last_chunk) {
            if (inside) {
                const size_t o = (size_t)py * W + px;
                const size_t plane = (size_t)W * H;
                image[o] = C0 + T * bg0;
                image[plane + o] = C1 + T * bg1;
                image[2 * plane + o] = C2 + T * bg2;
                final_T[o] = T;
                n_contrib[o] = last;
            }
        } else {
            st[0 * kThreads + tid] = T;
            st[1 * kThreads + tid] = C0;
            st[2 * kThreads + tid] = C1;
            st[3 * kThreads + tid] = C2;
            st[4 * kThreads + tid] = __uint_as_float(last);
            st[5 * kThreads + tid] = done ? 1.0f : 0.0f;
            __syncthreads();
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(&ws.done_cnt[tile], chunk + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();  // LDS and s_item are reused by the next item
    }
    if (STATS) {
        unsigned long long c[4] = {n_eval, n_exp, n_pass, n_blend};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            unsigned long long v = c[k];
#pragma unroll
            for (int d = fgd::kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, fgd::kWave);
            if (fgd::lane_id() == 0) atomicAdd(&frag_stats[k], v);
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int chunk_of(const fg_tune* tune)
{
    if (!tune || !tune->render_batch) return 512;
    return tune->render_batch;
}

size_t carve(void* base, int64_t n_tiles, int64_t cap_pairs, int chunk, RenderWs* w, int64_t* max_items,
             int64_t* max_slots)
{
    *max_items = n_tiles + (cap_pairs + chunk - 1) / chunk;
    const int64_t by_pairs = cap_pairs / chunk + 1;
    *max_slots = n_tiles < by_pairs ? n_tiles : by_pairs;
    const size_t sizes[6] = {(size_t)n_tiles * 4, (size_t)n_tiles * 4, (size_t)n_tiles * 4, (size_t)*max_items * 4,
                             64, (size_t)*max_slots * 6 * kThreads * 4};
    void** dst[6] = {(void**)&w->nch, (void**)&w->slot, (void**)&w->done_cnt, (void**)&w->item_tile,
                     (void**)&w->counters, (void**)&w->state};
    size_t off = 0;
    for (int i = 0; i < 6; i++) {
        if (base) *dst[i] = (char*)base + off;
        off += align_up(sizes[i] + 4);
    }
    return off;
}

template <int CHUNK>
void launch(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cam,
            const float bg[3], float* image, float* final_T, uint32_t* n_contrib, unsigned long long* frag_stats,
            uint32_t* status, const RenderWs& w, int64_t n_tiles, int64_t max_items, int64_t max_slots,
            hipStream_t s)
{
    const int Wt = (cam->width + 15) / 16;
    hipLaunchKernelGGL(k_chunk_count<CHUNK>, dim3((unsigned)((n_tiles + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       s, ranges, n_tiles, w.nch, w.done_cnt);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(1024), 0, s, w.nch, w.slot, w.item_tile, n_tiles, max_items,
                       w.counters);
    int64_t grid = max_items < 4096 ? max_items : 4096;
    const float2* xy = (const float2*)splats->xy;
    const float4* co = (const float4*)splats->conic_o;
    const float4* rgb = (const float4*)splats->rgb_depth;
    if (frag_stats)
        hipLaunchKernelGGL((k_render<CHUNK, true>), dim3((unsigned)grid), dim3(kThreads), 0, s, xy, co, rgb, vals,
                           ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], w, max_slots, image, final_T,
                           n_contrib, frag_stats, status);
    else
        hipLaunchKernelGGL((k_render<CHUNK, false>), dim3((unsigned)grid), dim3(kThreads), 0, s, xy, co, rgb, vals,
                           ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], w, max_slots, image, final_T,
                           n_contrib, frag_stats, status);
}

}  // namespace

extern "C" size_t fg_render_workspace_size(const fg_camera* cam, int64_t cap_pairs, const fg_tune* tune)
{
    if (!cam || cam->width <= 0 || cam->height <= 0 || cap_pairs < 0) return 0;
    const int64_t n_tiles = (int64_t)((cam->width + 15) / 16) * ((cam->height + 15) / 16);
    RenderWs w;
    int64_t mi, ms;
    return carve(nullptr, n_tiles, cap_pairs, chunk_of(tune), &w, &mi, &ms);
}

extern "C" int fg_render(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cam,
                         const float bg[3], float* image, float* final_T, uint32_t* n_contrib, int64_t cap_pairs,
                         unsigned long long* frag_stats, uint32_t* status, void* ws, size_t ws_bytes,
                         const fg_tune* tune, void* stream)
{
    if (!splats || !ranges || !cam || !bg || !image || !final_T || !n_contrib || !status || cap_pairs < 0)
        return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    const int chunk = chunk_of(tune);
    if (chunk != 256 && chunk != 512 && chunk != 1024) return FG_ERR_INVALID_ARG;
    const int64_t n_tiles = (int64_t)((cam->width + 15) / 16) * ((cam->height + 15) / 16);
    if (n_tiles >= ((int64_t)1 << 31)) return FG_ERR_UNSUPPORTED;
    RenderWs w;
    int64_t max_items, max_slots;
    if (!ws || ws_bytes < carve(nullptr, n_tiles, cap_pairs, chunk, &w, &max_items, &max_slots))
        return FG_ERR_WORKSPACE;
    carve(ws, n_tiles, cap_pairs, chunk, &w, &max_items, &max_slots);
    hipStream_t s = (hipStream_t)stream;
    switch (chunk) {
        case 256: launch<256>(splats, vals, ranges, cam, bg, image, final_T, n_contrib, frag_stats, status, w, n_tiles, max_items, max_slots, s); break;
        case 1024: launch<1024>(splats, vals, ranges, cam, bg, image, final_T, n_contrib, frag_stats, status, w, n_tiles, max_items, max_slots, s); break;
        default: launch<512>(splats, vals, ranges, cam, bg, image, final_T, n_contrib, frag_stats, status, w, n_tiles, max_items, max_slots, s); break;
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

extern "C" const char* fg_status_string(int code)
{
    switch (code) {
        case FG_OK: return "ok";
        case FG_ERR_INVALID_ARG: return "invalid argument";
        case FG_ERR_INVALID_TREE: return "invalid tree";
        case FG_ERR_UNSUPPORTED: return "unsupported configuration";
        case FG_ERR_WORKSPACE: return "workspace too small";
        case FG_ERR_HIP: return "HIP launch or runtime error";
        default: return "unknown status";
    }
}
