// Device-side helpers shared by the libfg kernels (gfx950, wave64).
//
// Numeric contract: every function here evaluates its formula in IEEE
// binary32 in the exact operation order written, with contraction disabled
// at compile time (-ffp-contract=off), so that discrete decisions taken from
// these values (frustum, radius threshold, tile rectangle, alpha skip and
// termination) are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fg.h"

namespace fgd {

constexpr int kWave = 64;
constexpr int kTile = 16;

// exp(x) for -87 <= x <= 0: Cody & Waite reduction x = n ln2 + r (ln2 as a
// 16-bit head plus a tail), Taylor polynomial of degree 7 for e^r in Horner
// form with fused multiply-adds, times 2^n.
__device__ __forceinline__ float exp_neg_in_range(float x)
{
    const float n = rintf(x * 1.44269504f);
    float r = fmaf(-n, 0.693145751953125f, x);
    r = fmaf(-n, 1.42860677e-06f, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)n);
}

// exp(x) for x <= 0, flushed to 0 below -87.
__device__ __forceinline__ float exp_neg(float x)
{
    if (x < -87.0f) return 0.0f;
    return exp_neg_in_range(x);
}

// ln(x) for x > 1: x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s),
// s = (m - 1)/(m + 1) carried with its exact division residual, odd series to
// s^9; e ln2 added as head + tail.
__device__ __forceinline__ float log_gt1(float x)
{
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float f = m - 1.0f;
    const float d = m + 1.0f;
    const float s = f / d;
    const float dlo = m - (d - 1.0f);
    float res = fmaf(-s, d, f);
    res = fmaf(-s, dlo, res);
    const float slo = res / d;
    const float s2 = s * s;
    float q = 1.0f / 9.0f;
    q = fmaf(q, s2, 1.0f / 7.0f);
    q = fmaf(q, s2, 1.0f / 5.0f);
    q = fmaf(q, s2, 1.0f / 3.0f);
    q = q * s2;
    const float s_2 = 2.0f * s;
    const float lm = s_2 + fmaf(s_2, q, 2.0f * slo);
    const float ef = (float)e;
    return fmaf(ef, 0.693145751953125f, fmaf(ef, 1.42860677e-06f, lm));
}

struct Cam {
    float R[9];
    float t[3];
    float campos[3];
    float fx, fy, cx, cy;
    int W, H, Wt, Ht;
    float znear, kx, ky;
    uint32_t tile_base;
};

inline Cam make_cam(const fg_camera& c)
{
    Cam k;
    for (int i = 0; i < 9; i++) k.R[i] = c.R[i];
    for (int i = 0; i < 3; i++) { k.t[i] = c.t[i]; k.campos[i] = c.campos[i]; }
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    k.W = c.width; k.H = c.height;
    k.Wt = (c.width + kTile - 1) / kTile;
    k.Ht = (c.height + kTile - 1) / kTile;
    k.znear = c.znear; k.kx = c.kx; k.ky = c.ky;
    k.tile_base = c.tile_base;
    return k;
}

// The pose (R, t, camera centre) of a camera in device memory replaces c's;
// intrinsics and image size stay those of c.
__device__ __forceinline__ void pose_from(Cam& c, const fg_camera* __restrict__ d)
{
#pragma unroll
    for (int i = 0; i < 9; i++) c.R[i] = d->R[i];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        c.t[i] = d->t[i];
        c.campos[i] = d->campos[i];
    }
}

// x_c = R x_w + t, each row summed left to right.
__device__ __forceinline__ void to_camera(const Cam& c, float mx, float my, float mz, float& x, float& y, float& z)
{
    x = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
    y = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
    z = ((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2];
}

__device__ __forceinline__ bool in_frustum(const Cam& c, float x, float y, float z)
{
    return z > c.znear && fabsf(x) <= c.kx * z && fabsf(y) <= c.ky * z;
}

// Sigma = M M^T, M = R(q / |q|) diag(s); six unique entries (00 01 02 11 12 22).
__device__ __forceinline__ void covariance3d(float s0, float s1, float s2, float qw, float qx, float qy, float qz,
                                             float S[6])
{
    const float norm = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    const float w = qw / norm, x = qx / norm, y = qy / norm, z = qz / norm;
    const float r00 = 1.0f - 2.0f * (y * y + z * z);
    const float r01 = 2.0f * (x * y - w * z);
    const float r02 = 2.0f * (x * z + w * y);
    const float r10 = 2.0f * (x * y + w * z);
    const float r11 = 1.0f - 2.0f * (x * x + z * z);
    const float r12 = 2.0f * (y * z - w * x);
    const float r20 = 2.0f * (x * z - w * y);
    const float r21 = 2.0f * (y * z + w * x);
    const float r22 = 1.0f - 2.0f * (x * x + y * y);
    const float m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const float m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const float m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    S[0] = (m00 * m00 + m01 * m01) + m02 * m02;
    S[1] = (m00 * m10 + m01 * m11) + m02 * m12;
    S[2] = (m00 * m20 + m01 * m21) + m02 * m22;
    S[3] = (m10 * m10 + m11 * m11) + m12 * m12;
    S[4] = (m10 * m20 + m11 * m21) + m12 * m22;
    S[5] = (m20 * m20 + m21 * m21) + m22 * m22;
}

// EWA: Sigma_2D = T Sigma T^T + 0.3 I, T = J W with J the pinhole Jacobian at
// the camera-space centre and W the world->camera rotation.
__device__ __forceinline__ void covariance2d(const Cam& c, float x, float y, float z, const float S[6], float& a,
                                             float& b, float& cc)
{
    const float j00 = c.fx / z;
    const float j02 = -(c.fx * x) / (z * z);
    const float j11 = c.fy / z;
    const float j12 = -(c.fy * y) / (z * z);
    float T0[3], T1[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        T0[j] = j00 * c.R[j] + j02 * c.R[6 + j];
        T1[j] = j11 * c.R[3 + j] + j12 * c.R[6 + j];
    }
    const float S00 = S[0], S01 = S[1], S02 = S[2], S11 = S[3], S12 = S[4], S22 = S[5];
    // U = T Sigma (rows of T times columns of Sigma)
    const float u00 = (T0[0] * S00 + T0[1] * S01) + T0[2] * S02;
    const float u01 = (T0[0] * S01 + T0[1] * S11) + T0[2] * S12;
    const float u02 = (T0[0] * S02 + T0[1] * S12) + T0[2] * S22;
    const float u10 = (T1[0] * S00 + T1[1] * S01) + T1[2] * S02;
    const float u11 = (T1[0] * S01 + T1[1] * S11) + T1[2] * S12;
    const float u12 = (T1[0] * S02 + T1[1] * S12) + T1[2] * S22;
    const float s00 = (u00 * T0[0] + u01 * T0[1]) + u02 * T0[2];
    const float s01 = (u00 * T1[0] + u01 * T1[1]) + u02 * T1[2];
    const float s11 = (u10 * T1[0] + u11 * T1[1]) + u12 * T1[2];
    a = s00 + 0.3f;
    b = s01;
    cc = s11 + 0.3f;
}

__device__ __forceinline__ float lambda_max(float a, float b, float c)
{
    const float h = 0.5f * (a - c);
    return 0.5f * (a + c) + sqrtf(h * h + b * b);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// DPP move within rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Sum over the 64 lanes, returned in every lane: DPP quad permutes and row
// mirrors give every lane of a row of 16 its row's sum; row broadcasts (lane
// 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3) leave
// the total in lane 63, and one lane read returns it.
__device__ __forceinline__ float wave_total(float v)
{
    v = v + dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = v + dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = v + dpp_mov<0x141>(v);  // row_half_mirror
    v = v + dpp_mov<0x140>(v);  // row_mirror
    v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}


__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Conservative box, in tile-relative pixel coordinates (inclusive), of the
// pixels where a splat's power can reach -5.6: d^T Q d <= 11.2 has
// half-widths sqrt(11.2 Sigma_xx) and sqrt(11.2 Sigma_yy) (Sigma = Q^-1),
// widened here by 1% + 1 px and clipped to the tile and the image. Every pixel
// outside it has power < -5.6 and is skipped by the test of Eq. (2) anyway.
// Packed x0 | x1 << 8 | y0 << 16 | y1 << 24; kNoBox (x0 > x1) when empty.
constexpr uint32_t kNoBox = 1u;

__device__ __forceinline__ uint32_t splat_box(float2 mm, float4 co, int tx, int ty, int W, int H)
{
    const float tx0 = (float)(tx * kTile), ty0 = (float)(ty * kTile);
    const float tx1 = fminf(tx0 + 15.0f, (float)(W - 1)), ty1 = fminf(ty0 + 15.0f, (float)(H - 1));
    float bx0 = tx0, bx1 = tx1, by0 = ty0, by1 = ty1;
    const float qdet = co.x * co.z - co.y * co.y;
    if (qdet > 0.0f) {
        const float ex = sqrtf(11.2f * co.z / qdet) * 1.01f + 1.0f;
        const float ey = sqrtf(11.2f * co.x / qdet) * 1.01f + 1.0f;
        bx0 = fmaxf(bx0, floorf(mm.x - ex - 0.5f));
        bx1 = fminf(bx1, ceilf(mm.x + ex - 0.5f));
        by0 = fmaxf(by0, floorf(mm.y - ey - 0.5f));
        by1 = fminf(by1, ceilf(mm.y + ey - 0.5f));
    }
    if (!(bx0 <= bx1 && by0 <= by1)) return kNoBox;
    const uint32_t x0 = (uint32_t)((int)bx0 - tx * kTile), x1 = (uint32_t)((int)bx1 - tx * kTile);
    const uint32_t y0 = (uint32_t)((int)by0 - ty * kTile), y1 = (uint32_t)((int)by1 - ty * kTile);
    return x0 | (x1 << 8) | (y0 << 16) | (y1 << 24);
}

}  // namespace fgd
