// Per-tile front-to-back alpha blending, Eq. (2).
//
// One workgroup of 256 threads (4 waves) per 16x16 tile, one pixel per
// thread. The tile's sorted splats are staged through LDS in batches: each
// thread loads one splat record (2D mean, conic + opacity, colour), then
// every pixel walks the batch, reading the same LDS words as the rest of its
// wave (broadcast, no bank conflicts). A workgroup stops as soon as all of
// its pixels have terminated.
#include "fg_device.h"

namespace {

constexpr int kThreads = 256;

// exp(power) <= exp(-5.6) < 1/255 for power < -5.6, so with opacity <= 1 the
// splat is skipped either way: testing this first avoids evaluating the
// exponential without changing any result.
constexpr float kSkipPower = -5.6f;

template <int B>
__global__ __launch_bounds__(kThreads) void k_render(const float2* __restrict__ xy, const float4* __restrict__ conic_o,
                                                     const float4* __restrict__ rgb_depth,
                                                     const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ ranges, int W, int H, int Wt,
                                                     float bg0, float bg1, float bg2, float* __restrict__ image,
                                                     float* __restrict__ final_T, uint32_t* __restrict__ n_contrib)
{
    __shared__ float2 s_xy[B];
    __shared__ float4 s_co[B];
    __shared__ float4 s_rgb[B];
    const int tile = blockIdx.x;
    const int tx = tile % Wt, ty = tile / Wt;
    const int px = tx * fgd::kTile + (int)(threadIdx.x % fgd::kTile);
    const int py = ty * fgd::kTile + (int)(threadIdx.x / fgd::kTile);
    const bool inside = px < W && py < H;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t base = start; base < end; base += B) {
        if (__syncthreads_count(done) == kThreads) break;
        if (threadIdx.x < B && base + threadIdx.x < end) {
            const uint32_t g = vals[base + threadIdx.x];
            s_xy[threadIdx.x] = xy[g];
            s_co[threadIdx.x] = conic_o[g];
            s_rgb[threadIdx.x] = rgb_depth[g];
        }
        __syncthreads();
        if (!done) {
            const int cnt = (int)(end - base < (uint32_t)B ? end - base : (uint32_t)B);
            for (int j = 0; j < cnt; j++) {
                const float2 m = s_xy[j];
                const float4 co = s_co[j];
                const float dx = m.x - fpx;
                const float dy = m.y - fpy;
                const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
                if (power > 0.0f || power < kSkipPower) continue;
                float alpha = co.w * fgd::exp_neg(power);
                alpha = alpha < 0.99f ? alpha : 0.99f;
                if (alpha < 1.0f / 255.0f) continue;
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
                last = base - start + (uint32_t)j + 1u;
            }
        }
    }
    if (inside) {
        const size_t o = (size_t)py * W + px;
        const size_t plane = (size_t)W * H;
        image[o] = C0 + T * bg0;
        image[plane + o] = C1 + T * bg1;
        image[2 * plane + o] = C2 + T * bg2;
        final_T[o] = T;
        n_contrib[o] = last;
    }
}

}  // namespace

extern "C" int fg_render(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cam,
                         const float bg[3], float* image, float* final_T, uint32_t* n_contrib, const fg_tune* tune,
                         void* stream)
{
    if (!splats || !ranges || !cam || !bg || !image || !final_T || !n_contrib) return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    int B = 256;
    if (tune && tune->render_batch) {
        B = tune->render_batch;
        if (B != 32 && B != 64 && B != 128 && B != 256) return FG_ERR_INVALID_ARG;
    }
    const int Wt = (cam->width + 15) / 16, Ht = (cam->height + 15) / 16;
    const int64_t n_tiles = (int64_t)Wt * Ht;
    if (n_tiles >= ((int64_t)1 << 31)) return FG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((unsigned)n_tiles), b(kThreads);
    const float2* xy = (const float2*)splats->xy;
    const float4* co = (const float4*)splats->conic_o;
    const float4* rgb = (const float4*)splats->rgb_depth;
    switch (B) {
        case 32: hipLaunchKernelGGL(k_render<32>, g, b, 0, s, xy, co, rgb, vals, ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], image, final_T, n_contrib); break;
        case 64: hipLaunchKernelGGL(k_render<64>, g, b, 0, s, xy, co, rgb, vals, ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], image, final_T, n_contrib); break;
        case 128: hipLaunchKernelGGL(k_render<128>, g, b, 0, s, xy, co, rgb, vals, ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], image, final_T, n_contrib); break;
        default: hipLaunchKernelGGL(k_render<256>, g, b, 0, s, xy, co, rgb, vals, ranges, cam->width, cam->height, Wt, bg[0], bg[1], bg[2], image, final_T, n_contrib); break;
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
