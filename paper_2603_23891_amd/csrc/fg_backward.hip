// Differentiable form: parameter activation and the backward pass of the
// blend (Eq. (2)) and of the projection (Sec. 3.1, Eq. (1)).
//
//   k_activate     scale = exp(log_scale), opacity = 1 / (1 + exp(-logit)),
//                  with the library's exponential (so the CPU reference sees
//                  the same activated values).
//   k_render_bwd   one pixel per lane, walking splats back to front. A
//                  splat was blended by a pixel exactly when its position is
//                  below the pixel's contributor count and it passes the same
//                  skip tests as in the forward (recomputed bit for bit), so
//                  no per-splat alphas are stored: the transmittance before
//                  splat k is recovered as T_k = T_{k+1} / (1 - alpha_k).
//                  Work items are whole tiles (walked from the final T) and,
//                  when the forward saved its per-chunk state, the chunks of
//                  long ranges, each walked from the (T, colour) the forward
//                  had after that chunk, so a long range no longer runs on
//                  one workgroup. A conservative box per splat (pixels where
//                  its power can reach -5.6) lets a wave pass over splats
//                  that miss its rows. Per splat, the gradients w.r.t. its 2D
//                  mean, conic, opacity and colour are summed over the wave
//                  (DPP permutes) and added with one atomic per value.
//   k_project_bwd  one thread per selected Gaussian: the chain from those
//                  splat gradients to the raw parameters (SH coefficients, the
//                  mean through the 2D mean, the Jacobian and the view
//                  direction, log-scales and the rotation through its
//                  normalisation, opacity logits).
#include "fg_device.h"
#include "fg_render_ws.h"

#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 256;
constexpr int kNG = 9;  // du dv dA dB dC dopacity dr dg db
constexpr float kSkipPower = -5.6f;

// exp for |x| <= 87: the library's Cody & Waite exponential (exp_neg is valid
// for positive arguments up to 88 as well).
__device__ __forceinline__ float exp_any(float x) { return fgd::exp_neg(x); }

__global__ void k_activate(const float* __restrict__ log_scale, const float* __restrict__ logit, int64_t m,
                           float* __restrict__ scale, float* __restrict__ opacity)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * m; i += (int64_t)gridDim.x * blockDim.x) {
        scale[i] = exp_any(log_scale[i]);
        if (i < m) opacity[i] = 1.0f / (1.0f + exp_any(-logit[i]));
    }
}

__global__ void k_zero(float* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Chunk items of long ranges (from the forward's saved state) and whole
// tiles; see the header comment.
struct BwdView {
    const uint32_t* nch;
    const uint32_t* mfirst;
    const uint32_t* mitem;
    const uint32_t* n_items;  // device count of chunk items; null: no saved state
    const float* state;
    int chunk;
    int64_t max_items;        // chunk items the workspace holds (bounds *n_items)
};

// Sums over the 64 lanes of the 9 gradient components, by halving: padded to
// 16, each lane keeps half of its components and adds its partner's half of
// the same ones, across lane bit 5, then 4 (lane shuffles), 3 and 2 (DPP row
// and half-row mirrors, which pair lanes that differ in that bit and hold the
// same set); then the one component left is summed within each quad. Lane l
// returns the total of component ((l >> 2) & 15), the same in all four lanes
// of the quad (components 9..15 are zero). 12 shuffles and 5 DPP adds, where
// nine separate reductions take 54 DPP steps and 9 lane reads.
__device__ __forceinline__ float grad_reduce_scatter(const float (&g)[kNG])
{
    const int lane = fgd::lane_id();
    float v[16];
#pragma unroll
    for (int c = 0; c < 16; c++) v[c] = c < kNG ? g[c] : 0.0f;
    float w8[8];
    {
        const bool hi = (lane & 32) != 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const float keep = hi ? v[i + 8] : v[i];
            const float send = hi ? v[i] : v[i + 8];
            w8[i] = keep + __shfl_xor(send, 32, fgd::kWave);
        }
    }
    float w4[4];
    {
        const bool hi = (lane & 16) != 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float keep = hi ? w8[i + 4] : w8[i];
            const float send = hi ? w8[i] : w8[i + 4];
            w4[i] = keep + __shfl_xor(send, 16, fgd::kWave);
        }
    }
    float w2[2];
    {
        const bool hi = (lane & 8) != 0;  // row mirror: lane i <-> 15 - i of its row
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const float keep = hi ? w4[i + 2] : w4[i];
            const float send = hi ? w4[i] : w4[i + 2];
            w2[i] = keep + fgd::dpp_mov<0x140>(send);
        }
    }
    float w1;
    {
        const bool hi = (lane & 4) != 0;  // half-row mirror: lane i <-> 7 - i of its half row
        const float keep = hi ? w2[1] : w2[0];
        const float send = hi ? w2[0] : w2[1];
        w1 = keep + fgd::dpp_mov<0x141>(send);
    }
    w1 = w1 + fgd::dpp_mov<0xB1>(w1);  // quad_perm [1, 0, 3, 2]
    w1 = w1 + fgd::dpp_mov<0x4E>(w1);  // quad_perm [2, 3, 0, 1]
    return w1;
}

template <bool STATS>
__global__ __launch_bounds__(kThreads) void k_render_bwd(const float2* __restrict__ xy,
                                                         const float4* __restrict__ conic_o,
                                                         const float4* __restrict__ rgb_depth,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ ranges, int W, int H, int Wt,
                                                         int64_t n_tiles, float bg0, float bg1, float bg2,
                                                         const float* __restrict__ final_T,
                                                         const uint32_t* __restrict__ n_contrib,
                                                         const float* __restrict__ image,
                                                         const float* __restrict__ dL_dimage, BwdView view,
                                                         float* __restrict__ gacc,
                                                         unsigned long long* __restrict__ stats)
{
    unsigned long long n_frag = 0, n_instr = 0, n_elem = 0;  // STATS: this lane's counts
    __shared__ float2 s_xy[kBatch];
    __shared__ float4 s_co[kBatch];
    __shared__ float4 s_rgb[kBatch];
    __shared__ uint32_t s_g[kBatch];
    __shared__ uint32_t s_box[kBatch];
    __shared__ uint32_t s_max;
    const int tid = threadIdx.x;
    const int lx = tid % fgd::kTile, ly = tid / fgd::kTile;
    const int lane = fgd::lane_id();
    const int wy0 = (tid / fgd::kWave) * (fgd::kWave / fgd::kTile);  // first pixel row of this wave
    const size_t plane = (size_t)W * H;
    int64_t n_chunk_items = view.n_items ? (int64_t)*view.n_items : 0;
    if (n_chunk_items > view.max_items) n_chunk_items = view.max_items;
    for (int64_t item = blockIdx.x; item < n_chunk_items + n_tiles; item += gridDim.x) {
        // work item: a chunk of a long range, or a whole tile
        uint32_t tile;
        int64_t lo = 0, hi_cap;
        int64_t citem = -1;
        if (item < n_chunk_items) {
            tile = view.mitem[item];
            if ((int64_t)tile >= n_tiles) continue;  // not a map this frame's forward wrote
            const uint32_t nch = view.nch[tile];
            if ((int64_t)view.mfirst[tile] + nch > n_chunk_items) continue;  // tile item walks it whole
            lo = (int64_t)(item - view.mfirst[tile]) * view.chunk;
            hi_cap = lo + view.chunk;
            citem = item;
        } else {
            tile = (uint32_t)(item - n_chunk_items);
            if (view.n_items && view.nch[tile] > 1 &&
                (int64_t)view.mfirst[tile] + view.nch[tile] <= n_chunk_items)
                continue;  // walked by its chunk items
            hi_cap = INT64_MAX;
        }
        const int tx = (int)(tile % (uint32_t)Wt), ty = (int)(tile / (uint32_t)Wt);
        const int px = tx * fgd::kTile + lx;
        const int py = ty * fgd::kTile + ly;
        const bool inside = px < W && py < H;
        const uint32_t r0 = ranges[2 * tile];
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const size_t o = (size_t)py * W + px;
        const uint32_t last = inside ? n_contrib[o] : 0u;
        float G0 = 0.f, G1 = 0.f, G2 = 0.f;
        if (inside) {
            G0 = dL_dimage[o];
            G1 = dL_dimage[plane + o];
            G2 = dL_dimage[2 * plane + o];
        }
        // T after the walked span and the colour behind it (later splats and
        // background): from final_T for a whole tile, from the state saved
        // after the chunk (colour behind = image - colour accumulated so far)
        float T, S0, S1, S2;
        if (citem < 0) {
            T = inside ? final_T[o] : 1.0f;
            S0 = T * bg0; S1 = T * bg1; S2 = T * bg2;
        } else {
            const float* st = view.state + (size_t)citem * (4 * kThreads);
            T = st[tid];
            S0 = inside ? image[o] - st[kThreads + tid] : 0.0f;
            S1 = inside ? image[plane + o] - st[2 * kThreads + tid] : 0.0f;
            S2 = inside ? image[2 * plane + o] - st[3 * kThreads + tid] : 0.0f;
        }
        __syncthreads();  // LDS of the previous item
        if (tid == 0) s_max = 0u;
        __syncthreads();
        atomicMax(&s_max, last);
        __syncthreads();
        // positions [0, s_max) of the range hold every blended splat
        const int64_t hi = hi_cap < (int64_t)s_max ? hi_cap : (int64_t)s_max;
        for (int64_t end = hi; end > lo; end -= kBatch) {
            const int64_t begin = end - kBatch > lo ? end - kBatch : lo;
            const int cnt = (int)(end - begin);
            __syncthreads();
            if (tid < cnt) {
                const uint32_t g = vals[r0 + begin + tid];
                s_g[tid] = g;
                const float2 mm = xy[g];
                const float4 co = conic_o[g];
                s_xy[tid] = mm;
                s_co[tid] = co;
                s_rgb[tid] = rgb_depth[g];
                s_box[tid] = fgd::splat_box(mm, co, tx, ty, W, H);
            }
            __syncthreads();
            uint32_t boxes = fgd::kNoBox;  // lane l: box of splat (window base) + l
            for (int jj = cnt - 1; jj >= 0; jj--) {
                // boxes are read 64 at a time, one per lane, and tested as
                // scalars: a splat whose box misses the wave's rows is passed
                // over (every pixel outside the box has power < -5.6, so it
                // blended nowhere there)
                const int wbase = jj & ~(fgd::kWave - 1);
                if (jj == cnt - 1 || (jj & (fgd::kWave - 1)) == fgd::kWave - 1)
                    boxes = wbase + lane < cnt ? s_box[wbase + lane] : fgd::kNoBox;
                const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)boxes, jj - wbase);
                const int bx0 = (int)(b & 255u), bx1 = (int)((b >> 8) & 255u);
                const int by0 = (int)((b >> 16) & 255u), by1 = (int)(b >> 24);
                if (bx0 > bx1 || by1 < wy0 || by0 > wy0 + 3) continue;
                const uint32_t pos = (uint32_t)(begin + jj);
                float gr[kNG] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                bool hit = false;
                if (pos < last && lx >= bx0 && lx <= bx1 && ly >= by0 && ly <= by1) {
                    const float2 m = s_xy[jj];
                    const float4 co = s_co[jj];
                    const float dx = m.x - fpx;
                    const float dy = m.y - fpy;
                    const float power = -0.5f * ((co.x * dx) * dx + (co.z * dy) * dy) - (co.y * dx) * dy;
                    if (!(power > 0.0f || power < kSkipPower)) {
                        const float e = fgd::exp_neg_in_range(power);  // -5.6 <= power <= 0
                        const float araw = co.w * e;
                        const float alpha = araw < 0.99f ? araw : 0.99f;
                        if (alpha >= 1.0f / 255.0f) {
                            hit = true;
                            const float4 c = s_rgb[jj];
                            // one division, then products: the gradients carry a
                            // tolerance, not the forward's bit-exactness
                            const float inv = 1.0f / (1.0f - alpha);
                            const float Tk = T * inv;
                            const float w = alpha * Tk;
                            gr[6] = G0 * w;
                            gr[7] = G1 * w;
                            gr[8] = G2 * w;
                            const float dLda = (G0 * (c.x * Tk - S0 * inv) + G1 * (c.y * Tk - S1 * inv)) +
                                               G2 * (c.z * Tk - S2 * inv);
                            S0 = S0 + c.x * w;
                            S1 = S1 + c.y * w;
                            S2 = S2 + c.z * w;
                            T = Tk;
                            if (araw < 0.99f) {
                                const float dLdp = dLda * alpha;
                                gr[5] = dLda * e;
                                gr[0] = dLdp * (-(co.x * dx + co.y * dy));
                                gr[1] = dLdp * (-(co.z * dy + co.y * dx));
                                gr[2] = dLdp * (-0.5f * (dx * dx));
                                gr[3] = dLdp * (-(dx * dy));
                                gr[4] = dLdp * (-0.5f * (dy * dy));
                            }
                        }
                    }
                }
                if (__ballot(hit)) {
                    // the 9 wave sums, then one atomic instruction: the first
                    // lane of quad k adds sum k
                    const float tot = grad_reduce_scatter(gr);
                    const int k = lane >> 2;
                    const bool adds = (lane & 3) == 0 && k < kNG && tot != 0.0f;
                    if (adds) atomicAdd(gacc + (size_t)s_g[jj] * kNG + k, tot);
                    if (STATS) {
                        const uint64_t am = __ballot(adds);
                        if (lane == 0 && am != 0ull) {
                            ++n_instr;
                            n_elem += (unsigned long long)__popcll(am);
                        }
                    }
                }
                if (STATS) n_frag += hit ? 1u : 0u;
            }
        }
    }
    if (STATS) {
        const unsigned long long c[3] = {n_instr, n_elem, n_frag};
#pragma unroll
        for (int k = 0; k < 3; k++) {
            unsigned long long v = c[k];
#pragma unroll
            for (int d = fgd::kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, fgd::kWave);
            if (lane == 0) atomicAdd(&stats[k], v);
        }
    }
}

template <int D>
__device__ __forceinline__ void sh_basis_and_grad(float x, float y, float z, float* Y, float* dY)
{
    constexpr float c0 = 0.28209479177387814f, c1 = 0.48860251190291992f, c2a = 1.0925484305920792f,
                    c2b = 0.31539156525252005f, c2c = 0.54627421529603959f, c3a = 0.59004358992664352f,
                    c3b = 2.8906114426405538f, c3c = 0.45704579946446572f, c3d = 0.3731763325901154f,
                    c3e = 1.4453057213202769f;
    constexpr int K = (D + 1) * (D + 1);
#pragma unroll
    for (int i = 0; i < 3 * K; i++) dY[i] = 0.0f;
    Y[0] = c0;
    if (D < 1) return;
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    dY[1 * 3 + 1] = c1; dY[2 * 3 + 2] = c1; dY[3 * 3 + 0] = c1;
    if (D < 2) return;
    Y[4] = c2a * (x * y); Y[5] = c2a * (y * z); Y[6] = c2b * (3.0f * (z * z) - 1.0f); Y[7] = c2a * (x * z);
    Y[8] = c2c * (x * x - y * y);
    dY[4 * 3 + 0] = c2a * y; dY[4 * 3 + 1] = c2a * x;
    dY[5 * 3 + 1] = c2a * z; dY[5 * 3 + 2] = c2a * y;
    dY[6 * 3 + 2] = 6.0f * c2b * z;
    dY[7 * 3 + 0] = c2a * z; dY[7 * 3 + 2] = c2a * x;
    dY[8 * 3 + 0] = 2.0f * c2c * x; dY[8 * 3 + 1] = -2.0f * c2c * y;
    if (D < 3) return;
    Y[9] = c3a * (y * (3.0f * (x * x) - y * y)); Y[10] = c3b * ((x * y) * z);
    Y[11] = c3c * (y * (5.0f * (z * z) - 1.0f)); Y[12] = c3d * (z * (5.0f * (z * z) - 3.0f));
    Y[13] = c3c * (x * (5.0f * (z * z) - 1.0f)); Y[14] = 1.4453057213202769f * (z * (x * x - y * y));
    Y[15] = c3a * (x * (x * x - 3.0f * (y * y)));
    dY[9 * 3 + 0] = 6.0f * c3a * x * y; dY[9 * 3 + 1] = c3a * (3.0f * x * x - 3.0f * y * y);
    dY[10 * 3 + 0] = c3b * y * z; dY[10 * 3 + 1] = c3b * x * z; dY[10 * 3 + 2] = c3b * x * y;
    dY[11 * 3 + 1] = c3c * (5.0f * z * z - 1.0f); dY[11 * 3 + 2] = 10.0f * c3c * y * z;
    dY[12 * 3 + 2] = c3d * (15.0f * z * z - 3.0f);
    dY[13 * 3 + 0] = c3c * (5.0f * z * z - 1.0f); dY[13 * 3 + 2] = 10.0f * c3c * x * z;
    dY[14 * 3 + 0] = 2.0f * c3e * x * z; dY[14 * 3 + 1] = -2.0f * c3e * y * z; dY[14 * 3 + 2] = c3e * (x * x - y * y);
    dY[15 * 3 + 0] = c3a * (3.0f * x * x - 3.0f * y * y); dY[15 * 3 + 1] = -6.0f * c3a * x * y;
}

template <int D>
__global__ __launch_bounds__(256) void k_project_bwd(fg_params prm, fgd::Cam cam, const uint32_t* __restrict__ sel_idx,
                                                     const uint32_t* __restrict__ n_sel_p, int64_t cap_sel,
                                                     const float* __restrict__ gacc, fg_grads out)
{
    constexpr int K = (D + 1) * (D + 1);
    const int64_t m = prm.m;
    int64_t n_sel = (int64_t)*n_sel_p;
    if (n_sel > cap_sel) n_sel = cap_sel;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_sel; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = sel_idx[i];
        const float* gq = gacc + (size_t)i * kNG;
        const float gu = gq[0], gv = gq[1], gA = gq[2], gB = gq[3], gC = gq[4], go = gq[5];
        const float grgb[3] = {gq[6], gq[7], gq[8]};
        const float mx = prm.mean[g], my = prm.mean[m + g], mz = prm.mean[2 * m + g];
        const float* Wm = cam.R;
        float X, Y, Z;
        fgd::to_camera(cam, mx, my, mz, X, Y, Z);
        float s[3];
        for (int a = 0; a < 3; a++) s[a] = exp_any(prm.log_scale[a * m + g]);
        const float q0 = prm.quat[g], q1 = prm.quat[m + g], q2 = prm.quat[2 * m + g], q3 = prm.quat[3 * m + g];
        const float qn = sqrtf(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
        const float w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
        float R[9];
        R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
        R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
        R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
        float M[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) M[3 * a + b] = R[3 * a + b] * s[b];
        float Sg[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Sg[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
        const float j00 = cam.fx / Z, j02 = -(cam.fx * X) / (Z * Z), j11 = cam.fy / Z, j12 = -(cam.fy * Y) / (Z * Z);
        float T[6];
        for (int b = 0; b < 3; b++) {
            T[b] = j00 * Wm[b] + j02 * Wm[6 + b];
            T[3 + b] = j11 * Wm[3 + b] + j12 * Wm[6 + b];
        }
        float U[6];
        for (int r = 0; r < 2; r++)
            for (int b = 0; b < 3; b++) U[3 * r + b] = T[3 * r] * Sg[b] + T[3 * r + 1] * Sg[3 + b] + T[3 * r + 2] * Sg[6 + b];
        const float a2 = (U[0] * T[0] + U[1] * T[1] + U[2] * T[2]) + 0.3f;
        const float b2 = U[0] * T[3] + U[1] * T[4] + U[2] * T[5];
        const float c2 = (U[3] * T[3] + U[4] * T[4] + U[5] * T[5]) + 0.3f;
        const float det = a2 * c2 - b2 * b2;
        const float QA = c2 / det, QB = -b2 / det, QC = a2 / det;
        float dmu[3] = {0.f, 0.f, 0.f}, dpc[3] = {0.f, 0.f, 0.f};
        // colour -> SH coefficients and view direction
        const float dx0 = mx - cam.campos[0], dy0 = my - cam.campos[1], dz0 = mz - cam.campos[2];
        const float len = sqrtf((dx0 * dx0 + dy0 * dy0) + dz0 * dz0);
        const float dir[3] = {dx0 / len, dy0 / len, dz0 / len};
        float Yb[16], dY[48];
        sh_basis_and_grad<D>(dir[0], dir[1], dir[2], Yb, dY);
        // the K x 3 coefficients are read once and the gradients written in
        // memory order, 16 bytes at a time where K x 3 is a multiple of 4
        const float* sh = prm.sh + (size_t)g * (K * 3);
        float* dsh = out.sh + (size_t)g * (K * 3);
        float coef[K * 3];
        if constexpr ((K * 3) % 4 == 0) {
            const float4* s4 = reinterpret_cast<const float4*>(sh);
#pragma unroll
            for (int q = 0; q < K * 3 / 4; q++) {
                const float4 v = s4[q];
                coef[4 * q] = v.x; coef[4 * q + 1] = v.y; coef[4 * q + 2] = v.z; coef[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < K * 3; q++) coef[q] = sh[q];
        }
        float grv[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float acc = 0.5f;
#pragma unroll
            for (int k = 0; k < K; k++) acc += Yb[k] * coef[k * 3 + ch];
            grv[ch] = acc < 0.0f ? 0.0f : grgb[ch];
        }
        if constexpr ((K * 3) % 4 == 0) {
            float4* d4 = reinterpret_cast<float4*>(dsh);
#pragma unroll
            for (int q = 0; q < K * 3 / 4; q++)
                d4[q] = make_float4(grv[(4 * q) % 3] * Yb[(4 * q) / 3], grv[(4 * q + 1) % 3] * Yb[(4 * q + 1) / 3],
                                    grv[(4 * q + 2) % 3] * Yb[(4 * q + 2) / 3], grv[(4 * q + 3) % 3] * Yb[(4 * q + 3) / 3]);
        } else {
#pragma unroll
            for (int q = 0; q < K * 3; q++) dsh[q] = grv[q % 3] * Yb[q / 3];
        }
        float dd[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
#pragma unroll
            for (int k = 0; k < K; k++)
#pragma unroll
                for (int a = 0; a < 3; a++) dd[a] += grv[ch] * coef[k * 3 + ch] * dY[k * 3 + a];
        }
        const float ddot = dd[0] * dir[0] + dd[1] * dir[1] + dd[2] * dir[2];
        for (int a = 0; a < 3; a++) dmu[a] += (dd[a] - dir[a] * ddot) / len;
        // opacity logit
        const float op = 1.0f / (1.0f + exp_any(-prm.logit[g]));
        out.logit[g] = go * op * (1.0f - op);
        // 2D mean
        dpc[0] += gu * cam.fx / Z;
        dpc[1] += gv * cam.fy / Z;
        dpc[2] += -(gu * cam.fx * X + gv * cam.fy * Y) / (Z * Z);
        // conic -> Sigma_2D: dL/dSigma_2D = -Q G Q with G = [[gA, gB/2], [gB/2, gC]]
        const float G01 = 0.5f * gB;
        const float QG00 = QA * gA + QB * G01, QG01 = QA * G01 + QB * gC;
        const float QG10 = QB * gA + QC * G01, QG11 = QB * G01 + QC * gC;
        const float H00 = -(QG00 * QA + QG01 * QB), H01 = -(QG00 * QB + QG01 * QC);
        const float H11 = -(QG10 * QB + QG11 * QC);
        // Sigma_2D = T Sigma T^T: dL/dSigma = T^T H T, dL/dT = 2 H T Sigma
        float dS[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                dS[3 * a + b] = T[a] * (H00 * T[b] + H01 * T[3 + b]) + T[3 + a] * (H01 * T[b] + H11 * T[3 + b]);
        float HT[6];
        for (int b = 0; b < 3; b++) {
            HT[b] = H00 * T[b] + H01 * T[3 + b];
            HT[3 + b] = H01 * T[b] + H11 * T[3 + b];
        }
        float dJ00 = 0.f, dJ02 = 0.f, dJ11 = 0.f, dJ12 = 0.f;
        for (int b = 0; b < 3; b++) {
            const float dT0 = 2.0f * (HT[0] * Sg[b] + HT[1] * Sg[3 + b] + HT[2] * Sg[6 + b]);
            const float dT1 = 2.0f * (HT[3] * Sg[b] + HT[4] * Sg[3 + b] + HT[5] * Sg[6 + b]);
            dJ00 += dT0 * Wm[b];
            dJ02 += dT0 * Wm[6 + b];
            dJ11 += dT1 * Wm[3 + b];
            dJ12 += dT1 * Wm[6 + b];
        }
        const float iz2 = 1.0f / (Z * Z);
        dpc[0] += dJ02 * (-cam.fx * iz2);
        dpc[1] += dJ12 * (-cam.fy * iz2);
        dpc[2] += dJ00 * (-cam.fx * iz2) + dJ11 * (-cam.fy * iz2) + dJ02 * (2.0f * cam.fx * X * iz2 / Z) +
                  dJ12 * (2.0f * cam.fy * Y * iz2 / Z);
        for (int a = 0; a < 3; a++) dmu[a] += Wm[a] * dpc[0] + Wm[3 + a] * dpc[1] + Wm[6 + a] * dpc[2];
        // Sigma = M M^T -> scale and rotation
        float ds[3] = {0.f, 0.f, 0.f}, dR[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                const float dM = 2.0f * (dS[3 * a] * M[b] + dS[3 * a + 1] * M[3 + b] + dS[3 * a + 2] * M[6 + b]);
                ds[b] += dM * R[3 * a + b];
                dR[3 * a + b] = dM * s[b];
            }
        const float dw = 2.0f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        const float dxq = 2.0f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0f * x * dR[4] - w * dR[5] + z * dR[6] +
                                  w * dR[7] - 2.0f * x * dR[8]);
        const float dyq = 2.0f * (-2.0f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                                  z * dR[7] - 2.0f * y * dR[8]);
        const float dzq = 2.0f * (-2.0f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0f * z * dR[4] + y * dR[5] +
                                  x * dR[6] + y * dR[7]);
        const float qd = dw * w + dxq * x + dyq * y + dzq * z;
        out.quat[g] = (dw - w * qd) / qn;
        out.quat[m + g] = (dxq - x * qd) / qn;
        out.quat[2 * m + g] = (dyq - y * qd) / qn;
        out.quat[3 * m + g] = (dzq - z * qd) / qn;
        for (int a = 0; a < 3; a++) {
            out.log_scale[a * m + g] = ds[a] * s[a];
            out.mean[a * m + g] = dmu[a];
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" int fg_activate(const fg_params* p, float* scale, float* opacity, void* stream)
{
    if (!p || !scale || !opacity || p->m < 0 || (p->m > 0 && (!p->log_scale || !p->logit))) return FG_ERR_INVALID_ARG;
    if (p->m == 0) return FG_OK;
    int64_t blocks = (3 * p->m + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_activate, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p->log_scale, p->logit,
                       p->m, scale, opacity);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

extern "C" size_t fg_render_backward_workspace_size(int64_t cap_sel)
{
    if (cap_sel < 0) return 0;
    return align_up((size_t)(cap_sel > 0 ? cap_sel : 1) * kNG * 4);
}

extern "C" int fg_render_backward(const fg_params* p, const fg_camera* cam, const float bg[3], const uint32_t* sel_idx,
                                  const uint32_t* n_sel, int64_t cap_sel, const fg_splats* splats,
                                  const uint32_t* vals, const uint32_t* ranges, const float* final_T,
                                  const uint32_t* n_contrib, const float* image, const void* render_ws,
                                  size_t render_ws_bytes, int64_t cap_pairs, const fg_tune* tune,
                                  const float* dL_dimage, const fg_grads* out, void* ws, size_t ws_bytes,
                                  void* stream)
{
    if (!p || !cam || !bg || !n_sel || !splats || !ranges || !final_T || !n_contrib || !dL_dimage || !out ||
        cap_sel < 0)
        return FG_ERR_INVALID_ARG;
    if (p->sh_degree < 0 || p->sh_degree > 3) return FG_ERR_UNSUPPORTED;
    if (!out->mean || !out->log_scale || !out->quat || !out->logit || !out->sh) return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fg_render_backward_workspace_size(cap_sel)) return FG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = p->m;
    const int K = (p->sh_degree + 1) * (p->sh_degree + 1);
    float* gacc = (float*)ws;
    const unsigned zb = 2048;
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, gacc, (int64_t)(cap_sel > 0 ? cap_sel : 1) * kNG);
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, out->mean, 3 * m);
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, out->log_scale, 3 * m);
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, out->quat, 4 * m);
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, out->logit, m);
    hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, s, out->sh, (int64_t)K * 3 * m);
    if (cap_sel == 0 || m == 0) return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
    const int Wt = (cam->width + 15) / 16, Ht = (cam->height + 15) / 16;
    const int64_t n_tiles = (int64_t)Wt * Ht;
    BwdView view = {nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0};
    fgr::RenderWsView rv;
    if (image && fgr::render_ws_view(render_ws, render_ws_bytes, cam, cap_pairs, tune, &rv))
        view = {rv.nch, rv.mfirst, rv.mitem, rv.counters, rv.state, rv.chunk, rv.max_items};
    int64_t gb = n_tiles + (view.n_items ? rv.max_items : 0);
    if (gb > 8192) gb = 8192;
    unsigned long long* stats = tune ? tune->bwd_stats : nullptr;
    if (stats)
        hipLaunchKernelGGL(k_render_bwd<true>, dim3((unsigned)gb), dim3(kThreads), 0, s, (const float2*)splats->xy,
                           (const float4*)splats->conic_o, (const float4*)splats->rgb_depth, vals, ranges, cam->width,
                           cam->height, Wt, n_tiles, bg[0], bg[1], bg[2], final_T, n_contrib, image, dL_dimage, view,
                           gacc, stats);
    else
        hipLaunchKernelGGL(k_render_bwd<false>, dim3((unsigned)gb), dim3(kThreads), 0, s, (const float2*)splats->xy,
                           (const float4*)splats->conic_o, (const float4*)splats->rgb_depth, vals, ranges, cam->width,
                           cam->height, Wt, n_tiles, bg[0], bg[1], bg[2], final_T, n_contrib, image, dL_dimage, view,
                           gacc, stats);
    const fgd::Cam c = fgd::make_cam(*cam);
    int64_t blocks = (cap_sel + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const dim3 g((unsigned)blocks), b(256);
    switch (p->sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_bwd<0>, g, b, 0, s, *p, c, sel_idx, n_sel, cap_sel, gacc, *out); break;
        case 1: hipLaunchKernelGGL(k_project_bwd<1>, g, b, 0, s, *p, c, sel_idx, n_sel, cap_sel, gacc, *out); break;
        case 2: hipLaunchKernelGGL(k_project_bwd<2>, g, b, 0, s, *p, c, sel_idx, n_sel, cap_sel, gacc, *out); break;
        default: hipLaunchKernelGGL(k_project_bwd<3>, g, b, 0, s, *p, c, sel_idx, n_sel, cap_sel, gacc, *out); break;
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
