// Traversal-free parallel filter (Sec. 3.2) and order-preserving stream
// compaction of the selection, for one or several views per pass over the
// tree.
//
// The paper runs its R&L and Ancestor filters in one kernel over every
// in-frustum node, with no level-by-level walk (Eq. (4)). Here the same
// per-node decision is split so that HBM traffic is minimal, and a pass
// serves up to kMaxViews cameras ("node-major": each node's data is read
// once for all of them):
//
//   k_small    internal nodes (index < n_internal_span): the view-independent
//              3D covariance once, then per view the frustum test, EWA
//              Sigma_2D and small = R_2D = 3 sqrt(lambda_max) <= tau_R.
//              Leaves never need R_2D (the leaf exemption keeps every
//              in-frustum leaf), so their scale and rotation are never read.
//   k_blocked  internal nodes: blocked(a) = small(a) or small(b) for some
//              ancestor b, for every view in one walk up the parent chain
//              (small bits and parent links of internal nodes stay in L2). An
//              internal node passes R&L exactly when it is small, so a node n
//              is removed by the Ancestor filter exactly when blocked(parent).
//   k_select   every node, one pass: RL(n) = small(n) for internal nodes and
//              F(n) for leaves; sel(n) = RL(n) and not blocked(parent(n)).
//              Leaves whose parent is blocked in every view never read their
//              mean. Wave ballots give the selection words and a count per
//              2048-node tile and view.
//   k_tile_scan  exclusive prefix sum of the tile counts (one workgroup per
//              view) and n_sel.
//   k_compact  one wave per tile and view: the selected ids in ascending
//              order at the tile's offset, from the selection words (256
//              bytes per tile).
//
// Stream compaction is thus reduce-then-scan in three launches. A single-pass
// scan with decoupled look-back (Merrill & Garland 2016) was measured first:
// with about a thousand tiles resident, each tile spent a quarter of its time
// walking back through predecessors that had published only aggregates, since
// agent-scope descriptor reads cost a memory round trip per step.
#include "fg_device.h"

#include <mutex>

namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 8;                    // nodes per thread in k_select
constexpr int kTileNodes = kBlock * kRounds;  // nodes per k_select workgroup
constexpr int kWaves = kBlock / fgd::kWave;
constexpr int kMaxViews = 8;                  // views per pass over the tree

constexpr int kScanThreads = 1024;          // k_tile_scan workgroup

struct CamSet {
    fgd::Cam c[kMaxViews];
};

__global__ void k_reset(uint32_t* __restrict__ status, bool reset_status, uint32_t* __restrict__ n_sel, int nv)
{
    const int i = threadIdx.x;
    if (i == 0 && reset_status) *status = 0u;
    if (i < nv) n_sel[i] = 0u;
}

__device__ __forceinline__ bool bit_of(const uint32_t* __restrict__ w, int64_t i)
{
    return (w[i >> 5] >> (i & 31)) & 1u;
}

__device__ __forceinline__ void store_wave_bits(uint32_t* __restrict__ words, int64_t base, int64_t limit,
                                                uint64_t bits)
{
    if (fgd::lane_id() == 0 && base < limit) {
        words[base >> 5] = (uint32_t)bits;
        if (base + 32 < limit) words[(base >> 5) + 1] = (uint32_t)(bits >> 32);
    }
}

// True when every point of the box [lo, hi] is outside the view's frustum
// by more than the rounding of the per-node test: then in_frustum(to_camera)
// is false in float32 for every node mean inside the box. Each frustum plane
// is a linear function L of the world position (the plane's normal from the
// rows of R); the box is outside a plane when the minimum of L over the box
// (centre term minus the half-extents times |normal|) exceeds a margin of
// 1e-5 (1 + k) S, S = |c|_1 + |h|_1 + |t|_1. The rounding of the node's
// float32 transform and comparison is below 8 * 2^-24 (1 + k) S, and that of
// this test is of the same order, so the margin holds them with a factor of
// more than 10. A box with a NaN or infinite bound is never outside.
__device__ __forceinline__ bool box_outside(const fgd::Cam& c, float4 lo, float4 hi)
{
    const float cx = 0.5f * (lo.x + hi.x), cy = 0.5f * (lo.y + hi.y), cz = 0.5f * (lo.z + hi.z);
    const float hx = 0.5f * (hi.x - lo.x), hy = 0.5f * (hi.y - lo.y), hz = 0.5f * (hi.z - lo.z);
    const float S = ((fabsf(cx) + fabsf(cy)) + fabsf(cz)) + ((hx + hy) + hz) +
                    ((fabsf(c.t[0]) + fabsf(c.t[1])) + fabsf(c.t[2]));
    // L_min(a, b) = a . centre + b - |a| . h
    auto lmin = [&](float a0, float a1, float a2, float b) {
        return (((a0 * cx + a1 * cy) + a2 * cz) + b) - ((fabsf(a0) * hx + fabsf(a1) * hy) + fabsf(a2) * hz);
    };
    const float mx = 1e-5f * (1.0f + c.kx) * S, my = 1e-5f * (1.0f + c.ky) * S, mz = 1e-5f * S;
    // behind the near plane: znear - z > margin everywhere
    if (lmin(-c.R[6], -c.R[7], -c.R[8], c.znear - c.t[2]) > mz) return true;
    // x > kx z and x < -kx z
    if (lmin(c.R[0] - c.kx * c.R[6], c.R[1] - c.kx * c.R[7], c.R[2] - c.kx * c.R[8], c.t[0] - c.kx * c.t[2]) > mx)
        return true;
    if (lmin(-c.R[0] - c.kx * c.R[6], -c.R[1] - c.kx * c.R[7], -c.R[2] - c.kx * c.R[8], -c.t[0] - c.kx * c.t[2]) > mx)
        return true;
    // y > ky z and y < -ky z
    if (lmin(c.R[3] - c.ky * c.R[6], c.R[4] - c.ky * c.R[7], c.R[5] - c.ky * c.R[8], c.t[1] - c.ky * c.t[2]) > my)
        return true;
    if (lmin(-c.R[3] - c.ky * c.R[6], -c.R[4] - c.ky * c.R[7], -c.R[5] - c.ky * c.R[8], -c.t[1] - c.ky * c.t[2]) > my)
        return true;
    return false;
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_small(const float* __restrict__ mean, const float* __restrict__ scale,
                                                  const float* __restrict__ quat, const uint8_t* __restrict__ flags,
                                                  int64_t N, int64_t span, CamSet cams,
                                                  const fg_camera* __restrict__ dcams, int nv, float tau_R,
                                                  uint32_t* __restrict__ small_bits, int64_t words,
                                                  const float4* __restrict__ tile_box,
                                                  uint32_t* __restrict__ status, bool reset_status)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n == 0 && reset_status) *status = 0u;  // before any later kernel of the call sets a bit
    // nodes of a k_select tile whose box is outside every view are not in
    // the frustum, so none of them is small
    bool out = false;
    if (tile_box) {
        const int64_t tile = ((int64_t)blockIdx.x * kBlock) / kTileNodes;
        const float4 lo = tile_box[2 * tile], hi = tile_box[2 * tile + 1];
        out = true;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (v >= nv) break;
            fgd::Cam cam = cams.c[v];
            if (dcams) fgd::pose_from(cam, dcams + v);
            out = out && box_outside(cam, lo, hi);
        }
    }
    uint32_t small = 0;  // bit v: small in view v
    if (!out && n < span && !(flags[n] & 1u)) {
        const float mx = mean[n], my = mean[N + n], mz = mean[2 * N + n];
        float S[6];
        bool have_cov = false;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (v >= nv) break;
            fgd::Cam cam = cams.c[v];
            if (dcams) fgd::pose_from(cam, dcams + v);
            float x, y, z;
            fgd::to_camera(cam, mx, my, mz, x, y, z);
            if (fgd::in_frustum(cam, x, y, z)) {
                if (!have_cov) {
                    fgd::covariance3d(scale[n], scale[N + n], scale[2 * N + n], quat[n], quat[N + n],
                                      quat[2 * N + n], quat[3 * N + n], S);
                    have_cov = true;
                }
                float a, b, c;
                fgd::covariance2d(cam, x, y, z, S, a, b, c);
                if (3.0f * sqrtf(fgd::lambda_max(a, b, c)) <= tau_R) small |= 1u << v;
            }
        }
    }
    const int64_t base = n - (int64_t)fgd::lane_id();
#pragma unroll
    for (int v = 0; v < NV; v++) {
        if (v >= nv) break;
        store_wave_bits(small_bits + v * words, base, span, __ballot((small >> v) & 1u));
    }
}

// Whether the ancestor walks of k_blocked workgroup blockIdx.x can be left
// out: blocked(n) is read only by k_select, for the children of n, and a
// child in a tile whose box is outside every view is never selected. So the
// walks are skipped when the children of the workgroup's nodes (index range
// crange, from the tree's boxes) lie in at most 8 such tiles, or when there
// are none. A workgroup whose nodes have a malformed parent chain has the
// range (-1, -1) and is always walked, so its FG_STATUS_BAD_PARENT is kept.
template <int NV>
__device__ __forceinline__ bool skip_walks(const float4* __restrict__ tile_box, const int2* __restrict__ crange,
                                           const CamSet& cams, const fg_camera* __restrict__ dcams, int nv)
{
    if (!tile_box) return false;
    const int2 cr = crange[blockIdx.x];
    if (cr.x < 0) return false;
    if (cr.x > cr.y) return true;
    const int64_t t0 = cr.x / kTileNodes, t1 = cr.y / kTileNodes;
    if (t1 - t0 >= 8) return false;
    bool out = true;
    for (int64_t t = t0; t <= t1 && out; t++) {
        const float4 lo = tile_box[2 * t], hi = tile_box[2 * t + 1];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (v >= nv) break;
            fgd::Cam cam = cams.c[v];
            if (dcams) fgd::pose_from(cam, dcams + v);
            out = out && box_outside(cam, lo, hi);
        }
    }
    return out;
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_blocked(const int32_t* __restrict__ parent, const uint8_t* __restrict__ flags,
                                                    const uint32_t* __restrict__ small_bits, int64_t words,
                                                    int64_t span, int max_depth, int nv,
                                                    uint32_t* __restrict__ blocked_bits, const float4* __restrict__ tile_box,
                                                    const int2* __restrict__ crange, CamSet cams,
                                                    const fg_camera* __restrict__ dcams, uint32_t* __restrict__ status)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (skip_walks<NV>(tile_box, crange, cams, dcams, nv)) {
        const int64_t base = n - (int64_t)fgd::lane_id();
#pragma unroll
        for (int v = 0; v < NV; v++)
            if (v < nv) store_wave_bits(blocked_bits + v * words, base, span, 0ull);
        return;
    }
    const uint32_t all = (1u << nv) - 1u;
    uint32_t blocked = 0;  // bit v: self or an ancestor small in view v
    bool bad = false;
    if (n < span && !(flags[n] & 1u)) {
        int64_t a = n;
        int32_t p = parent[n];
        int hops = 0;
#pragma unroll
        for (int v = 0; v < NV; v++)
            if (v < nv && bit_of(small_bits + v * words, n)) blocked |= 1u << v;
        while (blocked != all && p >= 0) {
            if ((int64_t)p >= a || (int64_t)p >= span || hops >= max_depth) {
                bad = true;
                break;
            }
#pragma unroll
            for (int v = 0; v < NV; v++)
                if (v < nv && bit_of(small_bits + v * words, p)) blocked |= 1u << v;
            a = p;
            p = parent[p];
            ++hops;
        }
    }
    const int64_t base = n - (int64_t)fgd::lane_id();
#pragma unroll
    for (int v = 0; v < NV; v++) {
        if (v >= nv) break;
        store_wave_bits(blocked_bits + v * words, base, span, __ballot((blocked >> v) & 1u));
    }
    if (__ballot(bad) && fgd::lane_id() == 0) atomicOr(status, FG_STATUS_BAD_PARENT);
}

// One workgroup per k_select tile of kTileNodes nodes: the box of the means
// of all its nodes, as two float4 (lo.xyz, hi.xyz); NaN for a tile holding a
// node whose parent link k_select rejects, so that such a tile is never
// culled.
__global__ __launch_bounds__(kBlock) void k_tile_boxes(const float* __restrict__ mean,
                                                       const int32_t* __restrict__ parent, int64_t N, int64_t span,
                                                       float4* __restrict__ box)
{
    __shared__ float s_r[6][kWaves];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * kTileNodes;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = t0 + r * kBlock + tid;
        if (n < N) {
            const int32_t p = parent[n];
            if (p >= 0 && ((int64_t)p >= n || (int64_t)p >= span)) bad = true;
            const float x = mean[n], y = mean[N + n], z = mean[2 * N + n];
            v[0] = fminf(v[0], x); v[1] = fminf(v[1], y); v[2] = fminf(v[2], z);
            v[3] = fmaxf(v[3], x); v[4] = fmaxf(v[4], y); v[5] = fmaxf(v[5], z);
        }
    }
#pragma unroll
    for (int d = fgd::kWave / 2; d > 0; d >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; k++) v[k] = fminf(v[k], __shfl_xor(v[k], d, fgd::kWave));
#pragma unroll
        for (int k = 3; k < 6; k++) v[k] = fmaxf(v[k], __shfl_xor(v[k], d, fgd::kWave));
    }
    if (__ballot(bad) && fgd::lane_id() == 0) s_bad = 1;
    if (fgd::lane_id() == 0)
        for (int k = 0; k < 6; k++) s_r[k][tid / fgd::kWave] = v[k];
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kWaves; w++) {
            for (int k = 0; k < 3; k++) v[k] = fminf(v[k], s_r[k][w]);
            for (int k = 3; k < 6; k++) v[k] = fmaxf(v[k], s_r[k][w]);
        }
        if (s_bad) {
            box[2 * tile] = make_float4(NAN, NAN, NAN, NAN);
            box[2 * tile + 1] = make_float4(NAN, NAN, NAN, NAN);
        } else {
            box[2 * tile] = make_float4(v[0], v[1], v[2], 0.0f);
            box[2 * tile + 1] = make_float4(v[3], v[4], v[5], 0.0f);
        }
    }
}

// Child index ranges per k_blocked workgroup (kBlock consecutive nodes below
// span): (INT32_MAX, -1) before k_child_ranges, which takes every node with
// a well-formed parent link into its parent's range.
__global__ void k_crange_init(int2* __restrict__ crange, int64_t n_blocks)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_blocks) crange[b] = make_int2(INT32_MAX, -1);
}

__global__ __launch_bounds__(kBlock) void k_child_ranges(const int32_t* __restrict__ parent, int64_t N, int64_t span,
                                                         int2* __restrict__ crange)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t p = n < N ? parent[n] : -1;
    if (p < 0 || (int64_t)p >= n || (int64_t)p >= span) p = -1;
    const int32_t b = p >= 0 ? p / kBlock : -1;
    // most waves hold the children of one workgroup's nodes: one atomic pair
    const int32_t b0 = __shfl(b, 0, fgd::kWave);
    const bool same = __ballot(b != b0) == 0ull;
    if (same) {
        if (b0 >= 0) {
            int32_t lo = (int32_t)n, hi = (int32_t)n;
#pragma unroll
            for (int d = fgd::kWave / 2; d > 0; d >>= 1) {
                lo = min(lo, __shfl_xor(lo, d, fgd::kWave));
                hi = max(hi, __shfl_xor(hi, d, fgd::kWave));
            }
            if (fgd::lane_id() == 0) {
                atomicMin(&crange[b0].x, lo);
                atomicMax(&crange[b0].y, hi);
            }
        }
    } else if (b >= 0) {
        atomicMin(&crange[b].x, (int32_t)n);
        atomicMax(&crange[b].y, (int32_t)n);
    }
}

// (-1, -1) for the workgroups holding a node below span whose parent chain
// k_blocked could reject (a link not below its child or not below span, or
// longer than max_depth), so that their walks always run.
__global__ __launch_bounds__(kBlock) void k_chain_check(const int32_t* __restrict__ parent, int64_t span,
                                                        int max_depth, int2* __restrict__ crange)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (n < span) {
        int64_t a = n;
        int32_t p = parent[n];
        int hops = 0;
        while (p >= 0) {
            if ((int64_t)p >= a || (int64_t)p >= span || hops >= max_depth) {
                bad = true;
                break;
            }
            a = p;
            p = parent[p];
            ++hops;
        }
    }
    if (__ballot(bad) && fgd::lane_id() == 0) crange[blockIdx.x] = make_int2(-1, -1);
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_select(const float* __restrict__ mean, const int32_t* __restrict__ parent,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ small_bits,
                                                   const uint32_t* __restrict__ blocked_bits, int64_t words,
                                                   int64_t N, int64_t span, CamSet cams,
                                                   const fg_camera* __restrict__ dcams, int nv,
                                                   uint32_t* __restrict__ sel_bits, int64_t sel_words,
                                                   uint32_t* __restrict__ tile_cnt, int64_t n_tiles,
                                                   const float4* __restrict__ tile_box,
                                                   uint32_t* __restrict__ status)
{
    __shared__ uint32_t s_cnt[NV][kWaves];
    const int tid = threadIdx.x;
    const int wave = tid / fgd::kWave;
    const int64_t tile = blockIdx.x;
    const uint32_t all = (1u << nv) - 1u;
    // A tile whose box lies outside every view's frustum selects nothing
    // (R&L needs F: a leaf in the frustum, an internal node small, which
    // includes being in the frustum): its selection words and count are
    // zero, and none of its nodes is read.
    if (tile_box) {
        const float4 lo = tile_box[2 * tile], hi = tile_box[2 * tile + 1];
        bool out = true;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (v >= nv) break;
            fgd::Cam cam = cams.c[v];
            if (dcams) fgd::pose_from(cam, dcams + v);
            out = out && box_outside(cam, lo, hi);
        }
        if (out) {
#pragma unroll
            for (int r = 0; r < kRounds; r++) {
                const int64_t n = tile * kTileNodes + r * kBlock + tid;
#pragma unroll
                for (int v = 0; v < NV; v++)
                    if (v < nv) store_wave_bits(sel_bits + v * sel_words, n - (int64_t)fgd::lane_id(), N, 0ull);
            }
            if (tid < nv) tile_cnt[(int64_t)tid * n_tiles + tile] = 0u;
            return;
        }
    }
    bool bad = false;
    // Loads are issued phase by phase for all rounds at once (parent links and
    // flags, then the parents' blocked bits, then leaf positions), so a
    // workgroup waits three memory latencies rather than three per round. The
    // streamed parent links and positions are loaded non-temporally, which
    // keeps the small and blocked bits of the internal nodes in the caches.
    int32_t par[kRounds];
    uint32_t fl[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        par[r] = n < N ? __builtin_nontemporal_load(parent + n) : -1;
        fl[r] = (n < N && n < span) ? (uint32_t)flags[n] : 1u;
    }
    uint32_t cull[kRounds];  // bit v: removed by the Ancestor filter in view v
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        const int32_t p = par[r];
        cull[r] = 0u;
        if (n < N && p >= 0) {
            if ((int64_t)p >= n || (int64_t)p >= span) {
                bad = true;
                cull[r] = all;
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++)
                    if (v < nv && bit_of(blocked_bits + v * words, p)) cull[r] |= 1u << v;
            }
        }
    }
    float mx[kRounds], my[kRounds], mz[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        mx[r] = my[r] = mz[r] = 0.0f;
        if (n < N && cull[r] != all && (fl[r] & 1u)) {
            mx[r] = __builtin_nontemporal_load(mean + n);
            my[r] = __builtin_nontemporal_load(mean + N + n);
            mz[r] = __builtin_nontemporal_load(mean + 2 * N + n);
        }
    }
    uint32_t cnt[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) cnt[v] = 0u;
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            if (v >= nv) break;
            bool sel = false;
            if (n < N && !((cull[r] >> v) & 1u)) {
                if (fl[r] & 1u) {  // leaf: RL = in frustum
                    fgd::Cam cam = cams.c[v];
                    if (dcams) fgd::pose_from(cam, dcams + v);
                    float x, y, z;
                    fgd::to_camera(cam, mx[r], my[r], mz[r], x, y, z);
                    sel = fgd::in_frustum(cam, x, y, z);
                } else {  // internal: RL = small
                    sel = bit_of(small_bits + v * words, n);
                }
            }
            const uint64_t ball = __ballot(sel);
            store_wave_bits(sel_bits + v * sel_words, n - (int64_t)fgd::lane_id(), N, ball);
            cnt[v] += (uint32_t)__popcll(ball);
        }
    }
    if (__ballot(bad) && fgd::lane_id() == 0) atomicOr(status, FG_STATUS_BAD_PARENT);
    if (fgd::lane_id() == 0) {
#pragma unroll
        for (int v = 0; v < NV; v++)
            if (v < nv) s_cnt[v][wave] = cnt[v];
    }
    __syncthreads();
    if (tid < nv) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) t += s_cnt[tid][w];
        tile_cnt[(int64_t)tid * n_tiles + tile] = t;
    }
}

// One workgroup per view: tile_cnt[v][0 .. n_tiles) becomes its exclusive
// prefix sum in place; n_sel[v] = the total. Rounds of 8 x 1024 counts: each
// round is loaded and stored with consecutive lanes on consecutive words and
// transposed through LDS, so that every thread scans 8 consecutive counts.
constexpr int kScanPer = 8;
constexpr int kScanRound = kScanPer * kScanThreads;

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint32_t* __restrict__ tile_cnt, int64_t n_tiles,
                                                            uint32_t* __restrict__ n_sel, int64_t cap_sel,
                                                            uint32_t* __restrict__ status)
{
    __shared__ uint32_t s_buf[kScanRound];
    __shared__ uint32_t s_wave[kScanThreads / fgd::kWave];
    uint32_t* row = tile_cnt + (int64_t)blockIdx.x * n_tiles;
    const int tid = threadIdx.x, lane = fgd::lane_id(), wave = tid / fgd::kWave;
    uint32_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += kScanRound) {
#pragma unroll
        for (int k = 0; k < kScanPer; k++) {
            const int64_t i = base + k * kScanThreads + tid;
            s_buf[k * kScanThreads + tid] = i < n_tiles ? row[i] : 0u;
        }
        __syncthreads();
        uint32_t c[kScanPer];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; k++) {
            c[k] = s_buf[tid * kScanPer + k];
            s += c[k];
        }
        uint32_t x = s;
#pragma unroll
        for (int d = 1; d < fgd::kWave; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, fgd::kWave);
            if (lane >= d) x += y;
        }
        if (lane == fgd::kWave - 1) s_wave[wave] = x;
        __syncthreads();
        uint32_t run = carry + x - s, total = 0;
        for (int w = 0; w < kScanThreads / fgd::kWave; w++) {
            if (w < wave) run += s_wave[w];
            total += s_wave[w];
        }
#pragma unroll
        for (int k = 0; k < kScanPer; k++) {
            s_buf[tid * kScanPer + k] = run;
            run += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; k++) {
            const int64_t i = base + k * kScanThreads + tid;
            if (i < n_tiles) row[i] = s_buf[k * kScanThreads + tid];
        }
        carry += total;
        __syncthreads();  // s_buf and s_wave are reused by the next round
    }
    if (tid == 0) {
        n_sel[blockIdx.x] = carry;
        if ((int64_t)carry > cap_sel) atomicOr(status, FG_STATUS_SEL_OVERFLOW);
    }
}

// One wave per (tile, view): the selected ids of the tile's nodes, in
// ascending order, at the tile's offset. Lane g reads the 64-bit selection
// word of the tile's 64-node group g; a wave scan of their popcounts gives
// each group's offset; then group by group the set lanes write their ids.
constexpr int kGroups = kTileNodes / fgd::kWave;  // 64-node groups per tile
static_assert(kGroups <= fgd::kWave, "one lane per group");

__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* __restrict__ sel_bits, int64_t sel_words,
                                                    int64_t N, const uint32_t* __restrict__ tile_off,
                                                    int64_t n_tiles, uint32_t* __restrict__ sel_idx,
                                                    int64_t cap_sel)
{
    const int lane = fgd::lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kWaves + threadIdx.x / fgd::kWave;
    const int v = blockIdx.y;
    if (tile >= n_tiles) return;
    const uint32_t* bits = sel_bits + (int64_t)v * sel_words;
    uint64_t b = 0;
    if (lane < kGroups) {
        const int64_t base = tile * kTileNodes + (int64_t)lane * fgd::kWave;  // multiple of 64
        if (base < N) {
            b = bits[base >> 5];
            if (base + 32 < N) b |= (uint64_t)bits[(base >> 5) + 1] << 32;
        }
    }
    const uint32_t c = (uint32_t)__popcll(b);
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < fgd::kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, fgd::kWave);
        if (lane >= d) x += y;
    }
    const uint32_t excl = tile_off[(int64_t)v * n_tiles + tile] + x - c;
    const uint64_t lt = fgd::lanemask_lt();
    uint32_t* out = sel_idx + (int64_t)v * cap_sel;
    const uint32_t lo = (uint32_t)b, hi = (uint32_t)(b >> 32);
#pragma unroll 4
    for (int g = 0; g < kGroups; g++) {
        const uint64_t gb = (uint64_t)(uint32_t)__shfl((int)lo, g, fgd::kWave) |
                            ((uint64_t)(uint32_t)__shfl((int)hi, g, fgd::kWave) << 32);
        if (gb == 0ull) continue;  // nothing selected in this group (the same for the whole wave)
        const uint32_t off = (uint32_t)__shfl((int)excl, g, fgd::kWave);
        if ((gb >> lane) & 1ull) {
            const uint32_t o = off + (uint32_t)__popcll(gb & lt);
            if ((int64_t)o < cap_sel) out[o] = (uint32_t)(tile * kTileNodes + (int64_t)g * fgd::kWave + lane);
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct FilterWs {
    uint32_t *small_bits, *blocked_bits, *tile_cnt;
    int64_t words;
};

size_t carve(void* base, int64_t N, int64_t span, int n_views, FilterWs* w)
{
    const int nv = n_views < kMaxViews ? n_views : kMaxViews;
    w->words = ((span + 63) / 64) * 2 + 2;
    const size_t n_tiles = (size_t)((N + kTileNodes - 1) / kTileNodes) + 1;
    const size_t sizes[3] = {(size_t)w->words * 4 * nv, (size_t)w->words * 4 * nv, n_tiles * 4 * nv};
    void** dst[3] = {(void**)&w->small_bits, (void**)&w->blocked_bits, (void**)&w->tile_cnt};
    size_t off = 0;
    for (int i = 0; i < 3; i++) {
        if (base) *dst[i] = (char*)base + off;
        off += align_up(sizes[i]);
    }
    return off;
}

template <int NV>
void launch_pass(const fg_tree* tree, const CamSet& cs, const fg_camera* dcams, int nv, float tau_R,
                 uint32_t* sel_bits, int64_t sel_words,
                 uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel, uint32_t* status, bool reset_status,
                 const FilterWs& w, int64_t N, int64_t span, int64_t n_tiles, hipStream_t s)
{
    if (span > 0) {
        const dim3 g((unsigned)((span + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_small<NV>, g, dim3(kBlock), 0, s, tree->mean, tree->scale, tree->quat, tree->flags, N,
                           span, cs, dcams, nv, tau_R, w.small_bits, w.words, (const float4*)tree->tile_box, status,
                           reset_status);
        const float4* box = (const float4*)tree->tile_box;
        const int2* crange = box ? (const int2*)(box + 2 * n_tiles) : nullptr;
        hipLaunchKernelGGL(k_blocked<NV>, g, dim3(kBlock), 0, s, tree->parent, tree->flags, w.small_bits, w.words,
                           span, tree->max_depth, nv, w.blocked_bits, box, crange, cs, dcams, status);
    }
    hipLaunchKernelGGL(k_select<NV>, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, tree->mean, tree->parent,
                       tree->flags, w.small_bits, w.blocked_bits, w.words, N, span, cs, dcams, nv, sel_bits, sel_words,
                       w.tile_cnt, n_tiles, (const float4*)tree->tile_box, status);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nv), dim3(kScanThreads), 0, s, w.tile_cnt, n_tiles, n_sel,
                       cap_sel, status);
    if (cap_sel > 0)
        hipLaunchKernelGGL(k_compact, dim3((unsigned)((n_tiles + kWaves - 1) / kWaves), (unsigned)nv), dim3(kBlock), 0,
                           s, sel_bits, sel_words, N, w.tile_cnt, n_tiles, sel_idx, cap_sel);
}

// Argument checks shared by fg_filter and fg_filter_noalloc (host only).
int check_filter_args(const fg_tree* tree, const fg_camera* cams, int32_t n_views, uint32_t* sel_bits,
                      uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel, uint32_t* status)
{
    if (!tree || !cams || n_views < 1 || !sel_bits || !n_sel || !status || cap_sel < 0 || (cap_sel > 0 && !sel_idx))
        return FG_ERR_INVALID_ARG;
    const int64_t N = tree->n_nodes, span = tree->n_internal_span;
    if (N < 0 || N >= ((int64_t)1 << 31) || span < 0 || span > N || tree->max_depth < 0 || tree->max_depth > 15)
        return FG_ERR_INVALID_TREE;
    if (N > 0 && (!tree->mean || !tree->parent || (span > 0 && (!tree->scale || !tree->quat || !tree->flags))))
        return FG_ERR_INVALID_ARG;
    for (int v = 0; v < n_views; v++)
        if (cams[v].width <= 0 || cams[v].height <= 0) return FG_ERR_INVALID_ARG;
    return FG_OK;
}

// The launches of one filter call on a workspace already checked for size.
int run_filter(const fg_tree* tree, const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev, float tau_R,
               uint32_t* sel_bits, uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel, uint32_t* status, void* ws,
               void* stream)
{
    const int64_t N = tree->n_nodes, span = tree->n_internal_span;
    FilterWs w;
    carve(ws, N, span, n_views, &w);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_tiles = (N + kTileNodes - 1) / kTileNodes;
    const int64_t sel_words = (N + 31) / 32;
    for (int v0 = 0; v0 < n_views; v0 += kMaxViews) {
        const int nv = n_views - v0 < kMaxViews ? n_views - v0 : kMaxViews;
        CamSet cs;
        for (int v = 0; v < kMaxViews; v++) cs.c[v] = fgd::make_cam(cams[v0 + (v < nv ? v : 0)]);
        // the status word is cleared by the first pass: by k_small when the
        // tree has internal nodes, else by k_reset (which also zeroes n_sel
        // for an empty tree)
        const bool first = v0 == 0;
        if (N == 0 || span == 0)
            hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, status, first, n_sel + v0, nv);
        if (N == 0) continue;
        uint32_t* sb = sel_bits + (int64_t)v0 * sel_words;
        uint32_t* si = sel_idx ? sel_idx + (int64_t)v0 * cap_sel : nullptr;
        uint32_t* ns = n_sel + v0;
        const bool rs = first && span > 0;
        const fg_camera* dc = cams_dev ? cams_dev + v0 : nullptr;
        if (nv == 1) launch_pass<1>(tree, cs, dc, nv, tau_R, sb, sel_words, si, cap_sel, ns, status, rs, w, N, span, n_tiles, s);
        else if (nv == 2) launch_pass<2>(tree, cs, dc, nv, tau_R, sb, sel_words, si, cap_sel, ns, status, rs, w, N, span, n_tiles, s);
        else if (nv <= 4) launch_pass<4>(tree, cs, dc, nv, tau_R, sb, sel_words, si, cap_sel, ns, status, rs, w, N, span, n_tiles, s);
        else launch_pass<8>(tree, cs, dc, nv, tau_R, sb, sel_words, si, cap_sel, ns, status, rs, w, N, span, n_tiles, s);
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

}  // namespace

extern "C" int64_t fg_tree_box_floats(int64_t n_nodes, int64_t n_internal_span)
{
    if (n_nodes < 0 || n_internal_span < 0 || n_internal_span > n_nodes) return -1;
    return 8 * ((n_nodes + kTileNodes - 1) / kTileNodes) + 2 * ((n_internal_span + kBlock - 1) / kBlock);
}

extern "C" int fg_tree_boxes(const fg_tree* tree, float* tile_box, void* stream)
{
    if (!tree || !tile_box) return FG_ERR_INVALID_ARG;
    const int64_t N = tree->n_nodes, span = tree->n_internal_span;
    if (N < 0 || N >= ((int64_t)1 << 31) || span < 0 || span > N) return FG_ERR_INVALID_TREE;
    if (N == 0) return FG_OK;
    if (!tree->mean || !tree->parent) return FG_ERR_INVALID_ARG;
    if (span > 0 && tree->max_depth < 0) return FG_ERR_INVALID_TREE;
    const int64_t n_tiles = (N + kTileNodes - 1) / kTileNodes;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_tile_boxes, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, tree->mean, tree->parent, N, span,
                       (float4*)tile_box);
    if (span > 0) {
        int2* crange = (int2*)(tile_box + 8 * n_tiles);
        const int64_t nb = (span + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_crange_init, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, crange, nb);
        hipLaunchKernelGGL(k_child_ranges, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           tree->parent, N, span, crange);
        hipLaunchKernelGGL(k_chain_check, dim3((unsigned)nb), dim3(kBlock), 0, s, tree->parent, span,
                           tree->max_depth, crange);
    }
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

extern "C" size_t fg_filter_workspace_size(int64_t n_nodes, int64_t n_internal_span, int32_t n_views)
{
    if (n_nodes < 0 || n_internal_span < 0 || n_views < 1) return 0;
    FilterWs w;
    return carve(nullptr, n_nodes, n_internal_span, n_views, &w);
}

extern "C" int fg_filter(const fg_tree* tree, const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev,
                         float tau_R, uint32_t* sel_bits, uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel,
                         uint32_t* status, void* ws, size_t ws_bytes, void* stream)
{
    const int rc = check_filter_args(tree, cams, n_views, sel_bits, sel_idx, cap_sel, n_sel, status);
    if (rc != FG_OK) return rc;
    FilterWs w;
    if (!ws || ws_bytes < carve(nullptr, tree->n_nodes, tree->n_internal_span, n_views, &w)) return FG_ERR_WORKSPACE;
    return run_filter(tree, cams, n_views, cams_dev, tau_R, sel_bits, sel_idx, cap_sel, n_sel, status, ws, stream);
}

// ---- fg_filter_noalloc: the same filter on a fixed device array -----------
//
// For callers that cannot allocate (code under graph capture, serving loops):
// the workspace lives in `scratch`, a file-scope device array of
// FG_NOALLOC_SCRATCH_BYTES. Each device holds its own copy at its own
// address; host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol), but the device address that hipGetSymbolAddress
// returns, looked up once per device on that device's first call.
namespace {

static __device__ __align__(256) unsigned char scratch[FG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

}  // namespace

extern "C" int fg_filter_noalloc(const fg_tree* tree, const fg_camera* cams, int32_t n_views,
                                 const fg_camera* cams_dev, float tau_R, uint32_t* sel_bits, uint32_t* sel_idx,
                                 int64_t cap_sel, uint32_t* n_sel, uint32_t* status, void* stream)
{
    const int rc = check_filter_args(tree, cams, n_views, sel_bits, sel_idx, cap_sel, n_sel, status);
    if (rc != FG_OK) return rc;
    FilterWs w;
    if (carve(nullptr, tree->n_nodes, tree->n_internal_span, n_views, &w) > (size_t)FG_NOALLOC_SCRATCH_BYTES)
        return FG_ERR_SCRATCH;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FG_ERR_HIP;
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = p;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) return FG_ERR_HIP;
    return run_filter(tree, cams, n_views, cams_dev, tau_R, sel_bits, sel_idx, cap_sel, n_sel, status,
                      g_scratch_ptr[dev], stream);
}
