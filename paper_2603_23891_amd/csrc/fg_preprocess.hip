// Projection of the selected Gaussians (Sec. 3.1, Eq. (1)) and their tile
// rectangles under the opacity-aware shrink radius (Sec. 3.3).
//
// One thread per selected Gaussian, a grid-stride loop over the device-side
// count; the y dimension of the grid runs over views (up to 8 per launch),
// each with its own selection, count and splat planes at a stride of cap_sel. Node attributes are gathered through sel_idx: the three position
// planes, scale and rotation planes, opacity, and the node's contiguous SH
// block (192 B at degree 3, read as 16-byte vectors).
#include "fg_device.h"

namespace {

constexpr int kBlock = 128;
constexpr int kViewsPerLaunch = 8;

struct CamSet {
    fgd::Cam c[kViewsPerLaunch];
};

// Real spherical harmonics (orthonormal, closed-form Cartesian polynomials of
// the unit direction), coefficient order (l, m = -l..l).
template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y)
{
    Y[0] = 0.28209479177387814f;
    if (D < 1) return;
    Y[1] = 0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = 0.48860251190291992f * x;
    if (D < 2) return;
    Y[4] = 1.0925484305920792f * (x * y);
    Y[5] = 1.0925484305920792f * (y * z);
    Y[6] = 0.31539156525252005f * (3.0f * (z * z) - 1.0f);
    Y[7] = 1.0925484305920792f * (x * z);
    Y[8] = 0.54627421529603959f * (x * x - y * y);
    if (D < 3) return;
    Y[9] = 0.59004358992664352f * (y * (3.0f * (x * x) - y * y));
    Y[10] = 2.8906114426405538f * ((x * y) * z);
    Y[11] = 0.45704579946446572f * (y * (5.0f * (z * z) - 1.0f));
    Y[12] = 0.3731763325901154f * (z * (5.0f * (z * z) - 3.0f));
    Y[13] = 0.45704579946446572f * (x * (5.0f * (z * z) - 1.0f));
    Y[14] = 1.4453057213202769f * (z * (x * x - y * y));
    Y[15] = 0.59004358992664352f * (x * (x * x - 3.0f * (y * y)));
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_preprocess(fg_tree tree, CamSet cams,
                                                       const fg_camera* __restrict__ dcams, float tau,
                                                       const uint32_t* __restrict__ sel_idx_all,
                                                       const uint32_t* __restrict__ n_sel_all, int64_t cap_sel,
                                                       fg_splats out_all)
{
    constexpr int K = (D + 1) * (D + 1);
    const int64_t N = tree.n_nodes;
    const int v = blockIdx.y;  // view within this launch
    fgd::Cam cam = cams.c[0];
#pragma unroll
    for (int u = 1; u < kViewsPerLaunch; u++)
        if (u == v) cam = cams.c[u];
    if (dcams) fgd::pose_from(cam, dcams + v);
    const uint32_t* __restrict__ sel_idx = sel_idx_all + (int64_t)v * cap_sel;
    const int64_t o = (int64_t)v * cap_sel;  // this view's splat entries
    int64_t n_sel = (int64_t)n_sel_all[v];
    if (n_sel > cap_sel) n_sel = cap_sel;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_sel; i += (int64_t)gridDim.x * kBlock) {
        const int64_t g = sel_idx[i];
        float4 xyo = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 rgbd = make_float4(0.f, 0.f, 0.f, 0.f);
        ushort4 rect = make_ushort4(0, 0, 0, 0);
        uint32_t tiles = 0;
        const float mx = tree.mean[g], my = tree.mean[N + g], mz = tree.mean[2 * N + g];
        float x, y, z;
        fgd::to_camera(cam, mx, my, mz, x, y, z);
        float S[6], a, b, c;
        fgd::covariance3d(tree.scale[g], tree.scale[N + g], tree.scale[2 * N + g], tree.quat[g], tree.quat[N + g],
                          tree.quat[2 * N + g], tree.quat[3 * N + g], S);
        fgd::covariance2d(cam, x, y, z, S, a, b, c);
        const float det = a * c - b * b;
        const float op = tree.opacity[g];
        if (det > 0.0f && op > 0.0f && op <= 1.0f) {
            co.x = c / det;
            co.y = -b / det;
            co.z = a / det;
            co.w = op;
            xyo.x = (cam.fx * x) / z + cam.cx;
            xyo.y = (cam.fy * y) / z + cam.cy;
            rgbd.w = z;
            const float lam = fgd::lambda_max(a, b, c);
            // tile-set radius: 3 sigma, shrunk where alpha decays to tau
            const float r3 = 3.0f * sqrtf(lam);
            float r;
            if (tau <= 0.0f) {
                r = r3;
            } else {
                const float qa = op / tau;
                if (qa <= 1.0f) {
                    r = 0.0f;
                } else {
                    const float rs = sqrtf((2.0f * lam) * fgd::log_gt1(qa));
                    r = rs < r3 ? rs : r3;
                }
            }
            if (r > 0.0f) {
                const float fWt = (float)cam.Wt, fHt = (float)cam.Ht;
                float x0 = floorf((xyo.x - r) * 0.0625f);
                float x1 = floorf((xyo.x + r) * 0.0625f) + 1.0f;
                float y0 = floorf((xyo.y - r) * 0.0625f);
                float y1 = floorf((xyo.y + r) * 0.0625f) + 1.0f;
                x0 = x0 < 0.0f ? 0.0f : (x0 > fWt ? fWt : x0);
                x1 = x1 < 0.0f ? 0.0f : (x1 > fWt ? fWt : x1);
                y0 = y0 < 0.0f ? 0.0f : (y0 > fHt ? fHt : y0);
                y1 = y1 < 0.0f ? 0.0f : (y1 > fHt ? fHt : y1);
                if (x0 < x1 && y0 < y1) {
                    rect = make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)x1,
                                        (unsigned short)y1);
                    tiles = (uint32_t)((x1 - x0) * (y1 - y0));
                }
            }
            if (tiles != 0u) {
                // view-dependent colour, only for a splat that reaches a tile (one
                // that reaches none is never blended; its colour stays 0)
                const float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
                const float len = sqrtf((dx * dx + dy * dy) + dz * dz);
                float Y[16];
                sh_basis<D>(dx / len, dy / len, dz / len, Y);
                const float* shp = tree.sh + (size_t)g * (K * 3);
                float coef[K * 3];
                if constexpr ((K * 3) % 4 == 0) {
                    const float4* s4 = reinterpret_cast<const float4*>(shp);
#pragma unroll
                    for (int k = 0; k < K * 3 / 4; k++) {
                        const float4 v = s4[k];
                        coef[4 * k] = v.x; coef[4 * k + 1] = v.y; coef[4 * k + 2] = v.z; coef[4 * k + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < K * 3; k++) coef[k] = shp[k];
                }
                float rgb[3];
#pragma unroll
                for (int ch = 0; ch < 3; ch++) {
                    float acc = Y[0] * coef[ch];
#pragma unroll
                    for (int k = 1; k < K; k++) acc = acc + Y[k] * coef[k * 3 + ch];
                    acc = acc + 0.5f;
                    rgb[ch] = acc < 0.0f ? 0.0f : acc;
                }
                rgbd.x = rgb[0]; rgbd.y = rgb[1]; rgbd.z = rgb[2];
            }
        }
        reinterpret_cast<float2*>(out_all.xy)[o + i] = make_float2(xyo.x, xyo.y);
        reinterpret_cast<float4*>(out_all.conic_o)[o + i] = co;
        reinterpret_cast<float4*>(out_all.rgb_depth)[o + i] = rgbd;
        reinterpret_cast<ushort4*>(out_all.rect)[o + i] = rect;
        out_all.tiles[o + i] = tiles;
    }
}

}  // namespace

extern "C" int fg_preprocess(const fg_tree* tree, const uint32_t* sel_idx, const uint32_t* n_sel, int64_t cap_sel,
                             const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev, float tau,
                             const fg_splats* out, uint32_t* status, void* stream)
{
    (void)status;
    if (!tree || !cams || n_views < 1 || !n_sel || !out || cap_sel < 0) return FG_ERR_INVALID_ARG;
    if (cap_sel == 0) return FG_OK;
    if (!sel_idx || !out->xy || !out->conic_o || !out->rgb_depth || !out->rect || !out->tiles)
        return FG_ERR_INVALID_ARG;
    if (tree->sh_degree < 0 || tree->sh_degree > 3) return FG_ERR_UNSUPPORTED;
    if (tree->n_nodes > 0 && (!tree->mean || !tree->scale || !tree->quat || !tree->opacity || !tree->sh))
        return FG_ERR_INVALID_ARG;
    for (int v = 0; v < n_views; v++)
        if (cams[v].width <= 0 || cams[v].height <= 0 || cams[v].width > 32768 * 16 || cams[v].height > 32768 * 16)
            return FG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    for (int v0 = 0; v0 < n_views; v0 += kViewsPerLaunch) {
        const int nv = n_views - v0 < kViewsPerLaunch ? n_views - v0 : kViewsPerLaunch;
        CamSet cs;
        for (int v = 0; v < kViewsPerLaunch; v++) cs.c[v] = fgd::make_cam(cams[v0 + (v < nv ? v : 0)]);
        int64_t blocks = (cap_sel + kBlock - 1) / kBlock;
        const int64_t max_blocks = 32768 / nv;
        if (blocks > max_blocks) blocks = max_blocks;
        const dim3 g((unsigned)blocks, (unsigned)nv), b(kBlock);
        const fg_camera* dc = cams_dev ? cams_dev + v0 : nullptr;
        const uint32_t* si = sel_idx + (int64_t)v0 * cap_sel;
        const uint32_t* ns = n_sel + v0;
        fg_splats o = *out;
        const int64_t off = (int64_t)v0 * cap_sel;
        o.xy += 2 * off;
        o.conic_o += 4 * off;
        o.rgb_depth += 4 * off;
        o.rect += 4 * off;
        o.tiles += off;
        switch (tree->sh_degree) {
            case 0: hipLaunchKernelGGL(k_preprocess<0>, g, b, 0, s, *tree, cs, dc, tau, si, ns, cap_sel, o); break;
            case 1: hipLaunchKernelGGL(k_preprocess<1>, g, b, 0, s, *tree, cs, dc, tau, si, ns, cap_sel, o); break;
            case 2: hipLaunchKernelGGL(k_preprocess<2>, g, b, 0, s, *tree, cs, dc, tau, si, ns, cap_sel, o); break;
            default: hipLaunchKernelGGL(k_preprocess<3>, g, b, 0, s, *tree, cs, dc, tau, si, ns, cap_sel, o); break;
        }
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
