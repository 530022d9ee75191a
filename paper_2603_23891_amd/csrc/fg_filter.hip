// Traversal-free parallel filter (Sec. 3.2) and order-preserving stream
// compaction of the selection.
//
// The paper runs its R&L and Ancestor filters in one kernel over every
// in-frustum node, with no level-by-level walk (Eq. (4)). Here the same
// per-node decision is split so that HBM traffic is minimal:
//
//   k_small   internal nodes only (index < n_internal_span): frustum test,
//             EWA Sigma_2D, R_2D = 3 sqrt(lambda_max) <= tau_R -> 1 bit/node.
//             Leaves never need R_2D (the leaf exemption keeps every
//             in-frustum leaf), so their scale/rotation are never read.
//   k_select  every node: chase the parent chain through the small bits
//             (an internal node passes R&L exactly when it is small, so the
//             Ancestor filter only needs those bits, which stay in L2/MALL),
//             then RL(n) = small(n) for internal nodes or F(n) for leaves.
//             Only leaves that survive the chase read their mean. Wave
//             ballots give the selection bits and per-block counts.
//   k_scan    exclusive scan of the block counts (one workgroup), n_sel.
//   k_compact writes the selected ids in ascending order.
#include "fg_device.h"

namespace {

constexpr int kBlock = 256;

__global__ void k_reset(uint32_t* status, uint32_t* n_sel)
{
    if (threadIdx.x == 0) {
        *status = 0u;
        *n_sel = 0u;
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
    const uint64_t bits = __ballot(small);
    const int64_t base = n - (int64_t)fgd::lane_id();
    if (fgd::lane_id() == 0 && base < span) {
        small_bits[base >> 5] = (uint32_t)bits;
        small_bits[(base >> 5) + 1] = (uint32_t)(bits >> 32);
    }
}

__device__ __forceinline__ bool bit_of(const uint32_t* __restrict__ w, int64_t i)
{
    return (w[i >> 5] >> (i & 31)) & 1u;
}

__global__ __launch_bounds__(kBlock) void k_select(const float* __restrict__ mean, const int32_t* __restrict__ parent,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ small_bits, int64_t N, int64_t span,
                                                   int max_depth, fgd::Cam cam, uint32_t* __restrict__ sel_bits,
                                                   uint32_t* __restrict__ block_count, uint32_t* __restrict__ status)
{
    __shared__ uint32_t wave_count[kBlock / fgd::kWave];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool sel = false;
    bool bad = false;
    if (n < N) {
        bool culled = false;
        int32_t a = parent[n];
        int hops = 0;
        while (a >= 0) {
            if ((int64_t)a >= n || (int64_t)a >= span || hops >= max_depth) {
                bad = true;
                break;
            }
            if (bit_of(small_bits, a)) {
                culled = true;
                break;
            }
            a = parent[a];
            ++hops;
        }
        if (!culled && !bad) {
            const bool leaf = n >= span || (flags[n] & 1u);
            if (leaf) {
                float x, y, z;
                fgd::to_camera(cam, mean[n], mean[N + n], mean[2 * N + n], x, y, z);
                sel = fgd::in_frustum(cam, x, y, z);
            } else {
                sel = bit_of(small_bits, n);
            }
        }
    }
    const uint64_t bits = __ballot(sel);
    const uint64_t badw = __ballot(bad);
    const int64_t base = n - (int64_t)fgd::lane_id();
    const int wave = threadIdx.x / fgd::kWave;
    if (fgd::lane_id() == 0) {
        if (base < N) {
            sel_bits[base >> 5] = (uint32_t)bits;
            if (base + 32 < N) sel_bits[(base >> 5) + 1] = (uint32_t)(bits >> 32);
        }
        wave_count[wave] = (uint32_t)__popcll(bits);
        if (badw) atomicOr(status, FG_STATUS_BAD_PARENT);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kBlock / fgd::kWave; w++) s += wave_count[w];
        block_count[blockIdx.x] = s;
    }
}

// Exclusive scan of nb block counts by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(const uint32_t* __restrict__ block_count,
                                               uint32_t* __restrict__ block_off, int64_t nb, int64_t cap_sel,
                                               uint32_t* __restrict__ n_sel, uint32_t* __restrict__ status)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = t * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; i++) s += block_count[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
        uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = lo; i < hi; i++) {
        block_off[i] = run;
        run += block_count[i];
    }
    if (t == 1023) {
        const uint32_t total = part[1023];
        *n_sel = total;
        if ((int64_t)total > cap_sel) atomicOr(status, FG_STATUS_SEL_OVERFLOW);
    }
}

__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* __restrict__ sel_bits,
                                                    const uint32_t* __restrict__ block_count,
                                                    const uint32_t* __restrict__ block_off, int64_t N,
                                                    int64_t cap_sel, uint32_t* __restrict__ sel_idx)
{
    __shared__ uint32_t wave_count[kBlock / fgd::kWave];
    if (block_count[blockIdx.x] == 0) return;  // uniform per block
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool sel = n < N && bit_of(sel_bits, n);
    const uint64_t bits = __ballot(sel);
    const int wave = threadIdx.x / fgd::kWave;
    if (fgd::lane_id() == 0) wave_count[wave] = (uint32_t)__popcll(bits);
    __syncthreads();
    uint32_t off = block_off[blockIdx.x];
    for (int w = 0; w < wave; w++) off += wave_count[w];
    off += (uint32_t)__popcll(bits & fgd::lanemask_lt());
    if (sel && (int64_t)off < cap_sel) sel_idx[off] = (uint32_t)n;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" size_t fg_filter_workspace_size(int64_t n_nodes, int64_t n_internal_span)
{
    if (n_nodes < 0 || n_internal_span < 0) return 0;
    const size_t small_words = (size_t)((n_internal_span + 63) / 64) * 2;
    const size_t nb = (size_t)((n_nodes + kBlock - 1) / kBlock);
    return align_up(small_words * 4 + 8) + 2 * align_up(nb * 4 + 4);
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
    const size_t need = fg_filter_workspace_size(N, span);
    if (!ws || ws_bytes < need) return FG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const fgd::Cam c = fgd::make_cam(*cam);
    char* w = (char*)ws;
    uint32_t* small_bits = (uint32_t*)w;
    w += align_up((size_t)((span + 63) / 64) * 2 * 4 + 8);
    const int64_t nb = (N + kBlock - 1) / kBlock;
    uint32_t* block_count = (uint32_t*)w;
    w += align_up((size_t)nb * 4 + 4);
    uint32_t* block_off = (uint32_t*)w;

    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, status, n_sel);
    if (N == 0) return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
    if (span > 0)
        hipLaunchKernelGGL(k_small, dim3((unsigned)((span + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, tree->mean,
                           tree->scale, tree->quat, tree->flags, N, span, c, tau_R, small_bits);
    hipLaunchKernelGGL(k_select, dim3((unsigned)nb), dim3(kBlock), 0, s, tree->mean, tree->parent, tree->flags,
                       small_bits, N, span, tree->max_depth, c, sel_bits, block_count, status);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, block_count, block_off, nb, cap_sel, n_sel, status);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kBlock), 0, s, sel_bits, block_count, block_off, N,
                       cap_sel, sel_idx);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}
