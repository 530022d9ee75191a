// GTC pre-pass (Sec. 3.3, Fig. 2(b)): the key-value pair contribution of every
// Gaussian-tile pair of a rendered view (Eq. (5)), the Gaussian-to-tile
// contribution of every tile (Eq. (6)), the view's mean over its tiles
// (Eq. (7)), and the scene threshold tau = lambda_G / G_bar over several views
// (Eq. (8)).
//
//   k_kpc       one workgroup per tile, one pixel per lane. The tile's sorted
//               splats are staged 256 at a time in LDS; every lane walks them
//               front to back with the blend's own tests (power, alpha skip,
//               termination), and the alpha * T of each blended fragment is
//               summed over the wave (DPP) and added to the splat's LDS slot
//               (one LDS atomic per wave and splat). A wave passes over a
//               splat whose conservative box misses its four pixel rows, and
//               stops once its pixels have all terminated; when the whole
//               tile has terminated the remaining pairs get 0 without being
//               visited. The pair sums go to kpc[], their mean over the
//               tile's pairs to tile_gtc[t] (Eq. (6): pairs with zero
//               contribution count), and tiles with pairs add G_t and 1 to the
//               view's two float64 accumulators.
//   k_kpc_items the same KPC when the view was blended with saved
//               per-chunk state: the chunks of long lists walk in parallel
//               from the saved transmittance, the other tiles whole;
//               k_tile_gtc then forms each tile's GTC from the pairs' KPC.
//   k_gtc_view  turns the accumulators into the view GTC of Eq. (7).
//   k_gtc_tau   mean of the view GTCs over the views that hold pairs, and
//               tau = lambda_G / G_bar.
//
// The transmittance chain is the blend's, in the same binary32 operations, so
// the set of blended fragments and each alpha * T are those of the sequential
// definition; only the summation order of a pair's terms differs.
#include "fg_device.h"
#include "fg_render_ws.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxEdges = 16;
constexpr float kSkipPower = -5.6f;  // exp(-5.6) < 1/255: skipped for any opacity <= 1

struct Edges {
    float e[kMaxEdges];
    int n;
};

template <bool HIST>
__global__ __launch_bounds__(kThreads) void k_kpc(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                                  const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ ranges,
                                                  const uint32_t* __restrict__ n_pairs, int64_t n_tiles,
                                                  int64_t cap_pairs, int W, int H, int Wt,
                                                  float* __restrict__ kpc, float* __restrict__ tile_gtc,
                                                  double* __restrict__ acc, Edges edges,
                                                  uint32_t* __restrict__ hist)
{
    __shared__ float2 s_xy[kThreads];
    __shared__ float4 s_co[kThreads];
    __shared__ uint32_t s_rows[kThreads];  // first and last pixel row (tile-relative) of the splat's box
    __shared__ float s_kpc[kThreads];
    __shared__ double s_red[kThreads / fgd::kWave];
    __shared__ uint32_t s_hist[kMaxEdges + 1];

    const int tid = threadIdx.x;
    const int lane = fgd::lane_id();
    const int wave = tid / fgd::kWave;
    const int wy0 = wave * (fgd::kWave / fgd::kTile);  // first pixel row of this wave
    const int wy1 = wy0 + fgd::kWave / fgd::kTile - 1;

    // the pairs of a sort that overflowed its capacity are incomplete: every
    // tile is then left undefined and the view is marked (acc[1] < 0)
    const bool overflow = (int64_t)*n_pairs > cap_pairs;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int tx = (int)(t % Wt), ty = (int)(t / Wt);
        uint32_t lo = ranges[2 * t], hi = ranges[2 * t + 1];
        if (overflow || (int64_t)hi > cap_pairs || lo > hi) lo = hi = 0;
        const uint32_t n = hi - lo;
        if (n == 0) {
            if (tid == 0) tile_gtc[t] = __int_as_float(0x7fc00000);  // Eq. (6) is 0/0: undefined
            continue;
        }
        if (HIST && tid <= edges.n) s_hist[tid] = 0u;
        const int px = tx * fgd::kTile + (tid % fgd::kTile);
        const int py = ty * fgd::kTile + (tid / fgd::kTile);
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        bool done = !(px < W && py < H);
        float T = 1.0f;
        double my_sum = 0.0;  // this thread's share of the tile's KPC sum
        for (uint32_t b = 0; b < n; b += kThreads) {
            const int cnt = (int)(n - b < (uint32_t)kThreads ? n - b : (uint32_t)kThreads);
            if (tid < cnt) {
                const uint32_t g = vals[lo + b + tid];
                const float2 mm = xy[g];
                const float4 co = conic_o[g];
                s_xy[tid] = mm;
                s_co[tid] = co;
                const uint32_t box = fgd::splat_box(mm, co, tx, ty, W, H);
                s_rows[tid] = box == fgd::kNoBox ? 0xffffu : ((box >> 16) & 255u) | ((box >> 24) << 8);
            }
            s_kpc[tid] = 0.0f;
            __syncthreads();
            for (int j = 0; j < cnt; j++) {
                if (__ballot(!done) == 0ull) break;  // every pixel of this wave has terminated
                const uint32_t rows = s_rows[j];
                const int y0 = (int)(rows & 255u), y1 = (int)(rows >> 8);
                if (y0 > wy1 || y1 < wy0) continue;  // the box misses this wave's rows (or is empty)
                float c = 0.0f;
                if (!done) {
                    const float2 mm = s_xy[j];
                    const float4 co = s_co[j];
                    const float dx = mm.x - fpx;
                    const float dy = mm.y - fpy;
                    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
                    if (!(power > 0.0f || power < kSkipPower)) {
                        float a = co.w * fgd::exp_neg_in_range(power);
                        a = a < 0.99f ? a : 0.99f;
                        if (a >= 1.0f / 255.0f) {
                            const float Tn = T * (1.0f - a);
                            if (Tn < 1e-4f) {
                                done = true;  // stops before this splat (Eq. (2) termination)
                            } else {
                                c = a * T;
                                T = Tn;
                            }
                        }
                    }
                }
                if (__ballot(c != 0.0f) != 0ull) {
                    const float sum = fgd::wave_total(c);
                    if (lane == 0) atomicAdd(&s_kpc[j], sum);
                }
            }
            __syncthreads();
            if (tid < cnt) {
                const float k = s_kpc[tid];
                kpc[lo + b + tid] = k;
                my_sum += (double)k;
                if (HIST) {
                    int bin = 0;
                    while (bin < edges.n && k >= edges.e[bin]) bin++;
                    atomicAdd(&s_hist[bin], 1u);
                }
            }
            const int alive = __syncthreads_count(!done);
            if (alive == 0 && b + kThreads < n) {
                // the whole tile has terminated: the remaining pairs contribute nothing
                for (uint32_t k = b + kThreads + tid; k < n; k += kThreads) kpc[lo + k] = 0.0f;
                if (HIST && tid == 0) {
                    int bin = 0;
                    while (bin < edges.n && 0.0f >= edges.e[bin]) bin++;
                    atomicAdd(&s_hist[bin], n - (b + kThreads));
                }
                break;
            }
        }
        // tile sum in float64: wave sums through LDS, then one thread
        double v = my_sum;
        for (int off = fgd::kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, fgd::kWave);
        if (lane == 0) s_red[wave] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / fgd::kWave; w++) s += s_red[w];
            const double G = s / (double)n;
            tile_gtc[t] = (float)G;
            atomicAdd(&acc[0], G);
            atomicAdd(&acc[1], 1.0);
        }
        if (HIST && tid <= edges.n && s_hist[tid]) atomicAdd(&hist[tid], s_hist[tid]);
        __syncthreads();
    }
}

// The same per-pair KPC from the blend's saved state, with the long ranges
// split into their chunks: work items are the chunk items of the tiles whose
// every chunk has saved state (each walked from the transmittance the blend
// had after the previous chunk) and whole tiles otherwise (walked from
// T = 1). A fragment at list position pos is blended by a pixel exactly when
// pos is below the pixel's contributor count and it passes the skip tests,
// so the walk needs no termination test, and a chunk does not wait for the
// ones before it. The fragments, their alpha * T and the wave sums per splat
// are those of k_kpc, bit for bit (the transmittance chain is the blend's, in
// the same operations); as there, the four waves' sums of a splat meet in an
// LDS float atomic, in either order. Only the per-pair KPC is written here;
// k_tile_gtc then sums each tile's pairs in k_kpc's order.
__global__ __launch_bounds__(kThreads) void k_kpc_items(const float2* __restrict__ xy,
                                                        const float4* __restrict__ conic_o,
                                                        const uint32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ ranges,
                                                        const uint32_t* __restrict__ n_pairs, int64_t n_tiles,
                                                        int64_t cap_pairs, int W, int H, int Wt,
                                                        const uint32_t* __restrict__ n_contrib,
                                                        fgr::RenderWsView view, float* __restrict__ kpc)
{
    __shared__ float2 s_xy[kThreads];
    __shared__ float4 s_co[kThreads];
    __shared__ uint32_t s_rows[kThreads];
    __shared__ float s_kpc[kThreads];
    __shared__ uint32_t s_max;

    const int tid = threadIdx.x;
    const int lane = fgd::lane_id();
    const int wave = tid / fgd::kWave;
    const int wy0 = wave * (fgd::kWave / fgd::kTile);
    const int wy1 = wy0 + fgd::kWave / fgd::kTile - 1;
    if ((int64_t)*n_pairs > cap_pairs) return;  // incomplete pairs: k_tile_gtc marks the view
    int64_t n_chunk_items = (int64_t)*view.counters;
    if (n_chunk_items > view.max_items) n_chunk_items = view.max_items;
    for (int64_t item = blockIdx.x; item < n_chunk_items + n_tiles; item += gridDim.x) {
        uint32_t tile;
        int64_t lo, hi;  // positions in the tile's list
        int64_t citem = -1;
        const uint32_t* rg;
        if (item < n_chunk_items) {
            tile = view.mitem[item];
            if ((int64_t)tile >= n_tiles) continue;  // a map this frame's blend did not write
            if ((int64_t)view.mfirst[tile] + view.nch[tile] > n_chunk_items) continue;  // walked whole
            rg = ranges + 2 * (int64_t)tile;
            lo = (int64_t)(item - view.mfirst[tile]) * view.chunk;
            hi = lo + view.chunk;
            citem = item;
        } else {
            tile = (uint32_t)(item - n_chunk_items);
            if (view.nch[tile] > 1 && (int64_t)view.mfirst[tile] + view.nch[tile] <= n_chunk_items) continue;
            rg = ranges + 2 * (int64_t)tile;
            lo = 0;
            hi = INT64_MAX;
        }
        const uint32_t r0 = rg[0], r1 = rg[1];
        if ((int64_t)r1 > cap_pairs || r0 > r1) continue;
        const int64_t n = (int64_t)(r1 - r0);
        if (hi > n) hi = n;
        if (lo >= hi) continue;
        const int tx = (int)(tile % (uint32_t)Wt), ty = (int)(tile / (uint32_t)Wt);
        const int px = tx * fgd::kTile + (tid % fgd::kTile);
        const int py = ty * fgd::kTile + (tid / fgd::kTile);
        const bool inside = px < W && py < H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const uint32_t last = inside ? n_contrib[(size_t)py * W + px] : 0u;
        // the transmittance after the previous chunk, as the blend saved it
        float T = citem > (int64_t)view.mfirst[tile] ? view.state[(size_t)(citem - 1) * (4 * kThreads) + tid] : 1.0f;
        __syncthreads();  // LDS of the previous item
        if (tid == 0) s_max = 0u;
        __syncthreads();
        atomicMax(&s_max, last);
        __syncthreads();
        // every blended fragment of the tile lies below s_max
        const int64_t end = hi < (int64_t)s_max ? hi : (int64_t)s_max;
        uint32_t wlast = last;
#pragma unroll
        for (int d = fgd::kWave / 2; d > 0; d >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)wlast, d, fgd::kWave);
            wlast = o > wlast ? o : wlast;
        }
        for (int64_t b = lo; b < end; b += kThreads) {
            const int cnt = (int)(end - b < kThreads ? end - b : kThreads);
            if (tid < cnt) {
                const uint32_t g = vals[r0 + b + tid];
                const float2 mm = xy[g];
                const float4 co = conic_o[g];
                s_xy[tid] = mm;
                s_co[tid] = co;
                const uint32_t box = fgd::splat_box(mm, co, tx, ty, W, H);
                s_rows[tid] = box == fgd::kNoBox ? 0xffffu : ((box >> 16) & 255u) | ((box >> 24) << 8);
            }
            s_kpc[tid] = 0.0f;
            __syncthreads();
            for (int j = 0; j < cnt; j++) {
                const uint32_t pos = (uint32_t)(b + j);
                if (pos >= wlast) break;  // no pixel of this wave blends further
                const uint32_t rows = s_rows[j];
                const int y0 = (int)(rows & 255u), y1 = (int)(rows >> 8);
                if (y0 > wy1 || y1 < wy0) continue;
                float c = 0.0f;
                if (pos < last) {
                    const float2 mm = s_xy[j];
                    const float4 co = s_co[j];
                    const float dx = mm.x - fpx;
                    const float dy = mm.y - fpy;
                    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
                    if (!(power > 0.0f || power < kSkipPower)) {
                        float a = co.w * fgd::exp_neg_in_range(power);
                        a = a < 0.99f ? a : 0.99f;
                        if (a >= 1.0f / 255.0f) {
                            c = a * T;
                            T = T * (1.0f - a);
                        }
                    }
                }
                if (__ballot(c != 0.0f) != 0ull) {
                    const float sum = fgd::wave_total(c);
                    if (lane == 0) atomicAdd(&s_kpc[j], sum);
                }
            }
            __syncthreads();
            if (tid < cnt) kpc[r0 + b + tid] = s_kpc[tid];
            __syncthreads();
        }
        // pairs behind every pixel's last blended fragment contribute nothing
        for (int64_t k = (end > lo ? end : lo) + tid; k < hi; k += kThreads) kpc[r0 + k] = 0.0f;
    }
}

// Eq. (6) from the per-pair KPC: one workgroup per tile sums its pairs in
// float64 in k_kpc's order (thread t the pairs t, t + 256, ..., then the
// wave sums through LDS), and adds G_t and 1 to the view's accumulators;
// with edges, the pairs' KPC histogram.
template <bool HIST>
__global__ __launch_bounds__(kThreads) void k_tile_gtc(const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ n_pairs, int64_t n_tiles,
                                                       int64_t cap_pairs, const float* __restrict__ kpc,
                                                       float* __restrict__ tile_gtc, double* __restrict__ acc,
                                                       Edges edges, uint32_t* __restrict__ hist)
{
    __shared__ double s_red[kThreads / fgd::kWave];
    __shared__ uint32_t s_hist[kMaxEdges + 1];
    const int tid = threadIdx.x;
    const int lane = fgd::lane_id();
    const int wave = tid / fgd::kWave;
    const bool overflow = (int64_t)*n_pairs > cap_pairs;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        uint32_t lo = ranges[2 * t], hi = ranges[2 * t + 1];
        if (overflow || (int64_t)hi > cap_pairs || lo > hi) lo = hi = 0;
        const uint32_t n = hi - lo;
        if (n == 0) {
            if (tid == 0) tile_gtc[t] = __int_as_float(0x7fc00000);  // Eq. (6) is 0/0: undefined
            continue;
        }
        if (HIST && tid <= edges.n) s_hist[tid] = 0u;
        __syncthreads();
        double my_sum = 0.0;
        for (uint32_t k = tid; k < n; k += kThreads) {
            const float v = kpc[lo + k];
            my_sum += (double)v;
            if (HIST) {
                int bin = 0;
                while (bin < edges.n && v >= edges.e[bin]) bin++;
                atomicAdd(&s_hist[bin], 1u);
            }
        }
        double v = my_sum;
        for (int off = fgd::kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, fgd::kWave);
        if (lane == 0) s_red[wave] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / fgd::kWave; w++) s += s_red[w];
            const double G = s / (double)n;
            tile_gtc[t] = (float)G;
            atomicAdd(&acc[0], G);
            atomicAdd(&acc[1], 1.0);
        }
        if (HIST && tid <= edges.n && s_hist[tid]) atomicAdd(&hist[tid], s_hist[tid]);
        __syncthreads();
    }
}

__global__ void k_gtc_zero(double* __restrict__ acc)
{
    if (threadIdx.x < 2) acc[threadIdx.x] = 0.0;
}

// Eq. (7): mean of the tile GTCs over the tiles holding pairs; acc[1] keeps
// their number (0: undefined view, acc[0] = 0; -1: the sort overflowed).
__global__ void k_gtc_view(double* __restrict__ acc, const uint32_t* __restrict__ n_pairs, int64_t cap_pairs)
{
    if (threadIdx.x != 0) return;
    if ((int64_t)*n_pairs > cap_pairs) {
        acc[0] = __longlong_as_double(0x7ff8000000000000ll);
        acc[1] = -1.0;
        return;
    }
    acc[0] = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
}

// Eq. (8): G_bar over the views with pairs, tau = lambda_G / G_bar.
__global__ void k_gtc_tau(const double* __restrict__ view_gtc, int n_views, float lambda_G,
                          double* __restrict__ g_bar, float* __restrict__ tau, uint32_t* __restrict__ status)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    int m = 0;
    bool overflow = false;
    for (int v = 0; v < n_views; v++) {
        if (view_gtc[2 * v + 1] < 0.0) overflow = true;
        if (view_gtc[2 * v + 1] > 0.0) {
            s += view_gtc[2 * v];
            m++;
        }
    }
    if (overflow) {
        *g_bar = __longlong_as_double(0x7ff8000000000000ll);
        *tau = __int_as_float(0x7fc00000);
        if (status) atomicOr(status, FG_STATUS_PAIR_OVERFLOW);
        return;
    }
    if (m == 0) {
        *g_bar = 0.0;
        *tau = __int_as_float(0x7fc00000);
        if (status) atomicOr(status, FG_STATUS_GTC_UNDEFINED);
        return;
    }
    const double G = s / (double)m;
    *g_bar = G;
    *tau = (float)((double)lambda_G / G);
}

}  // namespace

extern "C" int fg_gtc(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cam,
                      const uint32_t* n_pairs, int64_t cap_pairs, float* kpc, float* tile_gtc, double* view_gtc, const float* hist_edges,
                      int32_t n_edges, uint32_t* kpc_hist, const uint32_t* n_contrib, const void* render_ws,
                      size_t render_ws_bytes, const fg_tune* tune, void* stream)
{
    if (!splats || !vals || !ranges || !cam || !n_pairs || !kpc || !tile_gtc || !view_gtc || cap_pairs < 0)
        return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    if (n_edges < 0 || n_edges > kMaxEdges || (n_edges > 0 && (!hist_edges || !kpc_hist)) ||
        (kpc_hist && n_edges == 0))
        return FG_ERR_INVALID_ARG;
    Edges e{};
    e.n = n_edges;
    for (int i = 0; i < n_edges; i++) {
        e.e[i] = hist_edges[i];
        if (i > 0 && !(e.e[i] > e.e[i - 1])) return FG_ERR_INVALID_ARG;
    }
    const int Wt = (cam->width + 15) / 16;
    const int64_t n_tiles = (int64_t)Wt * ((cam->height + 15) / 16);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_gtc_zero, dim3(1), dim3(64), 0, s, view_gtc);
    const unsigned grid = (unsigned)(n_tiles < 65536 ? (n_tiles < 1 ? 1 : n_tiles) : 65536);
    const float2* xy = (const float2*)splats->xy;
    const float4* co = (const float4*)splats->conic_o;
    fgr::RenderWsView rv;
    if (render_ws || n_contrib) {
        // from the blend's saved state: chunk items in parallel, then the tiles
        if (!render_ws || !n_contrib || !fgr::render_ws_view(render_ws, render_ws_bytes, cam, cap_pairs, tune, &rv))
            return FG_ERR_INVALID_ARG;
        const int64_t items = rv.max_items + n_tiles;
        const unsigned gi = (unsigned)(items < 8192 ? items : 8192);
        hipLaunchKernelGGL(k_kpc_items, dim3(gi), dim3(kThreads), 0, s, xy, co, vals, ranges, n_pairs, n_tiles,
                           cap_pairs, cam->width, cam->height, Wt, n_contrib, rv, kpc);
        if (kpc_hist)
            hipLaunchKernelGGL(k_tile_gtc<true>, dim3(grid), dim3(kThreads), 0, s, ranges, n_pairs, n_tiles,
                               cap_pairs, (const float*)kpc, tile_gtc, view_gtc, e, kpc_hist);
        else
            hipLaunchKernelGGL(k_tile_gtc<false>, dim3(grid), dim3(kThreads), 0, s, ranges, n_pairs, n_tiles,
                               cap_pairs, (const float*)kpc, tile_gtc, view_gtc, e, kpc_hist);
    } else if (kpc_hist) {
        hipLaunchKernelGGL(k_kpc<true>, dim3(grid), dim3(kThreads), 0, s, xy, co, vals, ranges, n_pairs, n_tiles,
                           cap_pairs, cam->width, cam->height, Wt, kpc, tile_gtc, view_gtc, e, kpc_hist);
    } else {
        hipLaunchKernelGGL(k_kpc<false>, dim3(grid), dim3(kThreads), 0, s, xy, co, vals, ranges, n_pairs, n_tiles,
                           cap_pairs, cam->width, cam->height, Wt, kpc, tile_gtc, view_gtc, e, kpc_hist);
    }
    hipLaunchKernelGGL(k_gtc_view, dim3(1), dim3(64), 0, s, view_gtc, n_pairs, cap_pairs);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

extern "C" int fg_gtc_tau(const double* view_gtc, int32_t n_views, float lambda_G, double* g_bar, float* tau,
                          uint32_t* status, void* stream)
{
    if (!view_gtc || n_views < 1 || !g_bar || !tau) return FG_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_gtc_tau, dim3(1), dim3(64), 0, (hipStream_t)stream, view_gtc, n_views, lambda_G, g_bar, tau,
                       status);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
