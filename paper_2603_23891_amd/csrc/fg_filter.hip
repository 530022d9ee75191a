// Traversal-free parallel filter (Sec. 3.2) and order-preserving stream
// compaction of the selection.
//
// The paper runs its R&L and Ancestor filters in one kernel over every
// in-frustum node, with no level-by-level walk (Eq. (4)). Here the same
// per-node decision is split so that HBM traffic is minimal:
//
//   k_small    internal nodes (index < n_internal_span): frustum test, EWA
//              Sigma_2D, small = R_2D = 3 sqrt(lambda_max) <= tau_R. Leaves
//              never need R_2D (the leaf exemption keeps every in-frustum
//              leaf), so their scale and rotation are never read.
//   k_blocked  internal nodes: blocked(a) = small(a) or small(b) for some
//              ancestor b (a short parent-chain walk over internal nodes whose
//              small bits and parent links stay in L2). An internal node
//              passes R&L exactly when it is small, so a node n is removed by
//              the Ancestor filter exactly when blocked(parent(n)).
//   k_select   every node, one pass: RL(n) = small(n) for internal nodes and
//              F(n) for leaves; sel(n) = RL(n) and not blocked(parent(n)).
//              Leaves of blocked parents never read their mean. Wave ballots
//              give the selection words; the compacted ids are written in
//              ascending order with a single-pass decoupled look-back scan
//              across workgroups (Merrill & Garland 2016), workgroups taking
//              their tile index from an atomic ticket so every predecessor a
//              workgroup waits on has already started. A descriptor packs its
//              state and value in one 64-bit word, so relaxed agent-scope
//              atomics suffice (no cache-wide release/acquire per access).
#include "fg_device.h"

namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 8;                   // nodes per thread in k_select
constexpr int kTileNodes = kBlock * kRounds;  // nodes per k_select workgroup
constexpr int kWaves = kBlock / fgd::kWave;

// look-back descriptor: state in bits 63..62 (0 none, 1 aggregate, 2 prefix), value in bits 31..0
constexpr unsigned long long kAgg = 1ull << 62;
constexpr unsigned long long kPre = 2ull << 62;
constexpr uint32_t kSpinLimit = 1u << 26;

__global__ void k_reset(uint32_t* __restrict__ status, uint32_t* __restrict__ n_sel, uint32_t* __restrict__ ticket,
                        unsigned long long* __restrict__ desc, int64_t n_desc)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        *status = 0u;
        *n_sel = 0u;
        *ticket = 0u;
    }
    for (int64_t i = i0; i < n_desc; i += (int64_t)gridDim.x * blockDim.x) desc[i] = 0ull;
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

__global__ __launch_bounds__(kBlock) void k_small(const float* __restrict__ mean, const float* __restrict__ scale,
                                                  const float* __restrict__ quat, const uint8_t* __restrict__ flags,
                                                  int64_t N, int64_t span, fgd::Cam cam, float tau_R,
                                                  uint32_t* __restrict__ small_bits)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool small = false;
    if (n < span && !(flags[n] & 1u)) {
        float x, y, z;
        fgd::to_camera(cam, mean[n], mean[N + n], mean[2 * N + n], x, y, z);
        if (fgd::in_frustum(cam, x, y, z)) {
            float S[6], a, b, c;
            fgd::covariance3d(scale[n], scale[N + n], scale[2 * N + n], quat[n], quat[N + n], quat[2 * N + n],
                              quat[3 * N + n], S);
            fgd::covariance2d(cam, x, y, z, S, a, b, c);
            small = 3.0f * sqrtf(fgd::lambda_max(a, b, c)) <= tau_R;
        }
    }
    store_wave_bits(small_bits, n - (int64_t)fgd::lane_id(), span, __ballot(small));
}

__global__ __launch_bounds__(kBlock) void k_blocked(const int32_t* __restrict__ parent, const uint8_t* __restrict__ flags,
                                                    const uint32_t* __restrict__ small_bits, int64_t span,
                                                    int max_depth, uint32_t* __restrict__ blocked_bits,
                                                    uint32_t* __restrict__ status)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool blocked = false, bad = false;
    if (n < span && !(flags[n] & 1u)) {
        blocked = bit_of(small_bits, n);
        int64_t a = n;
        int32_t p = parent[n];
        int hops = 0;
        while (!blocked && p >= 0) {
            if ((int64_t)p >= a || (int64_t)p >= span || hops >= max_depth) {
                bad = true;
                break;
            }
            blocked = bit_of(small_bits, p);
            a = p;
            p = parent[p];
            ++hops;
        }
    }
    store_wave_bits(blocked_bits, n - (int64_t)fgd::lane_id(), span, __ballot(blocked));
    if (__ballot(bad) && fgd::lane_id() == 0) atomicOr(status, FG_STATUS_BAD_PARENT);
}

__global__ __launch_bounds__(kBlock) void k_select(const float* __restrict__ mean, const int32_t* __restrict__ parent,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ small_bits,
                                                   const uint32_t* __restrict__ blocked_bits, int64_t N, int64_t span,
                                                   fgd::Cam cam, uint32_t* __restrict__ sel_bits,
                                                   uint32_t* __restrict__ sel_idx, int64_t cap_sel,
                                                   uint32_t* __restrict__ n_sel, uint32_t* __restrict__ ticket,
                                                   unsigned long long* __restrict__ desc,
                                                   uint32_t* __restrict__ status)
{
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_off[kRounds * kWaves];
    __shared__ uint32_t s_excl;
    const int tid = threadIdx.x;
    const int wave = tid / fgd::kWave;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t n_tiles = (N + kTileNodes - 1) / kTileNodes;
    uint64_t ball[kRounds];
    bool bad = false;
    // Loads are issued phase by phase for all rounds at once (parent links and
    // flags, then the parents' blocked bits, then leaf positions), so a
    // workgroup waits three memory latencies rather than three per round.
    int32_t par[kRounds];
    uint32_t fl[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        par[r] = n < N ? parent[n] : -1;
        fl[r] = (n < N && n < span) ? (uint32_t)flags[n] : 1u;
    }
    uint32_t cull[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        const int32_t p = par[r];
        cull[r] = 0u;
        if (n < N && p >= 0) {
            if ((int64_t)p >= n || (int64_t)p >= span) {
                bad = true;
                cull[r] = 1u;
            } else {
                cull[r] = (blocked_bits[p >> 5] >> (p & 31)) & 1u;
            }
        }
    }
    float mx[kRounds], my[kRounds], mz[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        mx[r] = my[r] = mz[r] = 0.0f;
        if (n < N && !cull[r] && (fl[r] & 1u)) {
            mx[r] = mean[n];
            my[r] = mean[N + n];
            mz[r] = mean[2 * N + n];
        }
    }
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        const int64_t n = tile * kTileNodes + r * kBlock + tid;
        bool sel = false;
        if (n < N && !cull[r]) {
            if (fl[r] & 1u) {  // leaf: RL = in frustum
                float x, y, z;
                fgd::to_camera(cam, mx[r], my[r], mz[r], x, y, z);
                sel = fgd::in_frustum(cam, x, y, z);
            } else {  // internal: RL = small
                sel = bit_of(small_bits, n);
            }
        }
        ball[r] = __ballot(sel);
        store_wave_bits(sel_bits, n - (int64_t)fgd::lane_id(), N, ball[r]);
        if (fgd::lane_id() == 0) s_off[r * kWaves + wave] = (uint32_t)__popcll(ball[r]);
    }
    if (__ballot(bad) && fgd::lane_id() == 0) atomicOr(status, FG_STATUS_BAD_PARENT);
    __syncthreads();
    if (tid < fgd::kWave) {
        // wave 0: exclusive offsets of the (round, wave) groups in node order ...
        uint32_t agg = 0;
        if (tid == 0) {
            uint32_t run = 0;
            for (int i = 0; i < kRounds * kWaves; i++) {
                const uint32_t c = s_off[i];
                s_off[i] = run;
                run += c;
            }
            agg = run;
            __hip_atomic_store(&desc[tile], (tile == 0 ? kPre : kAgg) | agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        agg = __shfl(agg, 0, fgd::kWave);
        // ... then the look-back, 64 predecessors per step: lane i reads the
        // descriptor of tile j - i; the nearest "prefix" lane ends the walk
        // once no lane before it is still unpublished.
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t j = tile - 1;
            uint32_t spins = 0;
            const int lane = fgd::lane_id();
            for (;;) {
                const int64_t idx = j - lane;
                const unsigned long long d =
                    idx >= 0 ? __hip_atomic_load(&desc[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kPre;
                const unsigned long long state = d & (3ull << 62);
                const uint64_t pend = __ballot(state == 0ull);
                const uint64_t pre = __ballot(state == kPre);
                const uint64_t upto = pre ? (pre & (~pre + 1ull)) * 2ull - 1ull : ~0ull;  // lanes 0..first prefix
                if (pend & upto) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit) {  // never expected: predecessors always publish
                        if (lane == 0) atomicOr(status, FG_STATUS_LOOKBACK_STALL);
                        break;
                    }
                    continue;
                }
                uint32_t v = ((upto >> lane) & 1ull) ? (uint32_t)d : 0u;
#pragma unroll
                for (int o = fgd::kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, fgd::kWave);
                excl += v;
                if (pre) break;
                j -= fgd::kWave;
            }
            if (tid == 0)
                __hip_atomic_store(&desc[tile], kPre | (unsigned long long)(excl + agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0) {
            s_excl = excl;
            if (tile == n_tiles - 1) {
                const uint32_t total = excl + agg;
                *n_sel = total;
                if ((int64_t)total > cap_sel) atomicOr(status, FG_STATUS_SEL_OVERFLOW);
            }
        }
    }
    __syncthreads();
    const uint32_t base = s_excl;
    const uint64_t lt = fgd::lanemask_lt();
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        if ((ball[r] >> fgd::lane_id()) & 1ull) {
            const uint32_t off = base + s_off[r * kWaves + wave] + (uint32_t)__popcll(ball[r] & lt);
            if ((int64_t)off < cap_sel) sel_idx[off] = (uint32_t)(tile * kTileNodes + r * kBlock + tid);
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct FilterWs {
    uint32_t *small_bits, *blocked_bits, *ticket;
    unsigned long long* desc;
};

size_t carve(void* base, int64_t N, int64_t span, FilterWs* w)
{
    const size_t words = (size_t)((span + 63) / 64) * 2 + 2;
    const size_t n_desc = (size_t)((N + kTileNodes - 1) / kTileNodes) + 1;
    const size_t sizes[4] = {words * 4, words * 4, 64, n_desc * 8};
    void** dst[4] = {(void**)&w->small_bits, (void**)&w->blocked_bits, (void**)&w->ticket, (void**)&w->desc};
    size_t off = 0;
    for (int i = 0; i < 4; i++) {
        if (base) *dst[i] = (char*)base + off;
        off += align_up(sizes[i]);
    }
    return off;
}

}  // namespace

extern "C" size_t fg_filter_workspace_size(int64_t n_nodes, int64_t n_internal_span)
{
    if (n_nodes < 0 || n_internal_span < 0) return 0;
    FilterWs w;
    return carve(nullptr, n_nodes, n_internal_span, &w);
}

extern "C" int fg_filter(const fg_tree* tree, const fg_camera* cam, float tau_R, uint32_t* sel_bits,
                         uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel, uint32_t* status, void* ws,
                         size_t ws_bytes, void* stream)
{
    if (!tree || !cam || !sel_bits || !n_sel || !status || cap_sel < 0 || (cap_sel > 0 && !sel_idx))
        return FG_ERR_INVALID_ARG;
    const int64_t N = tree->n_nodes, span = tree->n_internal_span;
    if (N < 0 || N >= ((int64_t)1 << 31) || span < 0 || span > N || tree->max_depth < 0 || tree->max_depth > 15)
        return FG_ERR_INVALID_TREE;
    if (N > 0 && (!tree->mean || !tree->parent || (span > 0 && (!tree->scale || !tree->quat || !tree->flags))))
        return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    FilterWs w;
    if (!ws || ws_bytes < carve(nullptr, N, span, &w)) return FG_ERR_WORKSPACE;
    carve(ws, N, span, &w);
    hipStream_t s = (hipStream_t)stream;
    const fgd::Cam c = fgd::make_cam(*cam);
    const int64_t n_tiles = (N + kTileNodes - 1) / kTileNodes;
    int64_t rg = (n_tiles + 255) / 256;
    rg = rg < 1 ? 1 : (rg > 1024 ? 1024 : rg);
    hipLaunchKernelGGL(k_reset, dim3((unsigned)rg), dim3(256), 0, s, status, n_sel, w.ticket, w.desc, n_tiles);
    if (N == 0) return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
    if (span > 0) {
        const dim3 g((unsigned)((span + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_small, g, dim3(kBlock), 0, s, tree->mean, tree->scale, tree->quat, tree->flags, N, span, c,
                           tau_R, w.small_bits);
        hipLaunchKernelGGL(k_blocked, g, dim3(kBlock), 0, s, tree->parent, tree->flags, w.small_bits, span,
                           tree->max_depth, w.blocked_bits, status);
    }
    hipLaunchKernelGGL(k_select, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, tree->mean, tree->parent, tree->flags,
                       w.small_bits, w.blocked_bits, N, span, c, sel_bits, sel_idx, cap_sel, n_sel, w.ticket, w.desc,
                       status);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
