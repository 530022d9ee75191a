// The serial, level-by-level selection that the traversal-free filter
// replaces (Sec. 3.2, Eq. (3); the serial rows of Table 2): the cut is grown
// from the roots one tree level at a time. Every node of the current frontier
// is tested; a node that passes R&L (in frustum, and a leaf or R_2D <= tau_R)
// is selected and ends its branch, any other internal node hands its children
// to the next frontier. Each level is one kernel launch, and the host reads
// the next frontier's size back before it can launch the next level: the
// synchronisation the paper charges to this scheme (T_synch), beside the
// frontier evaluations themselves (T_calcu).
//
// The scheme walks down from the roots, so it needs each node's children; the
// tree planes hold only parent links. fg_children builds them once per tree
// (a counting sort of the nodes by parent, with a virtual node N whose
// children are the roots).
//
//   k_child_count / k_scan_* / k_child_fill   CSR of children by parent
//   k_lw_level     one frontier level: F, small, select or expand (wave-
//                  aggregated appends to the next frontier)
#include "fg_device.h"

#include <chrono>

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 2048;  // entries per block of the offset scan

__global__ __launch_bounds__(kBlock) void k_child_count(const int32_t* __restrict__ parent, int64_t N,
                                                        uint32_t* __restrict__ cnt, uint32_t* __restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    const int32_t p = parent[i];
    if (p < 0) {
        atomicAdd(&cnt[N], 1u);
    } else if ((int64_t)p >= i) {
        atomicOr(status, FG_STATUS_BAD_PARENT);  // the node stays unreachable
    } else {
        atomicAdd(&cnt[p], 1u);
    }
}

// Sum of each block of kScanItems counts.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ cnt, int64_t n,
                                                        uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t s_w[kBlock / fgd::kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    uint32_t s = 0;
    for (int k = threadIdx.x; k < kScanItems; k += kBlock)
        if (base + k < n) s += cnt[base + k];
    for (int off = fgd::kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, fgd::kWave);
    if (fgd::lane_id() == 0) s_w[threadIdx.x / fgd::kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / fgd::kWave; w++) t += s_w[w];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive scan of the block sums in place (one workgroup, serial runs per thread).
__global__ __launch_bounds__(kBlock) void k_scan_blocks(uint32_t* __restrict__ bsum, int64_t nb)
{
    __shared__ uint32_t s_part[kBlock];
    const int tid = threadIdx.x;
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t lo = tid * per, hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; i++) s += bsum[i];
    s_part[tid] = s;
    __syncthreads();
    uint32_t run = 0;
    for (int w = 0; w < tid; w++) run += s_part[w];
    for (int64_t i = lo; i < hi; i++) {
        const uint32_t c = bsum[i];
        bsum[i] = run;
        run += c;
    }
}

// offs[k] = exclusive prefix of cnt up to k (block base + in-block scan);
// offs[n] = the total. cursor[k] = 0 for the fill.
__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t* __restrict__ cnt, int64_t n,
                                                       const uint32_t* __restrict__ bsum,
                                                       int32_t* __restrict__ offs, uint32_t* __restrict__ cursor)
{
    __shared__ uint32_t s_v[kScanItems];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    for (int k = threadIdx.x; k < kScanItems; k += kBlock) s_v[k] = base + k < n ? cnt[base + k] : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = bsum[blockIdx.x];
        for (int k = 0; k < kScanItems; k++) {
            const uint32_t c = s_v[k];
            s_v[k] = run;
            run += c;
        }
        if (base + kScanItems >= n) offs[n] = (int32_t)run;  // the last block writes the total
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kScanItems; k += kBlock)
        if (base + k < n) {
            offs[base + k] = (int32_t)s_v[k];
            cursor[base + k] = 0u;
        }
}

__global__ __launch_bounds__(kBlock) void k_child_fill(const int32_t* __restrict__ parent, int64_t N,
                                                       const int32_t* __restrict__ offs,
                                                       uint32_t* __restrict__ cursor, int32_t* __restrict__ ids)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    const int32_t p = parent[i];
    if (p >= 0 && (int64_t)p >= i) return;
    const int64_t q = p < 0 ? N : (int64_t)p;
    const uint32_t k = atomicAdd(&cursor[q], 1u);
    ids[offs[q] + k] = (int32_t)i;
}

__global__ void k_lw_status(uint32_t* __restrict__ status)
{
    if (threadIdx.x == 0) atomicOr(status, FG_STATUS_BAD_PARENT);
}

__global__ void k_lw_reset(uint32_t* __restrict__ counters, uint32_t* __restrict__ n_sel)
{
    if (threadIdx.x < 4) counters[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *n_sel = 0u;
}

__global__ __launch_bounds__(kBlock) void k_zero_words(uint32_t* __restrict__ w, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) w[i] = 0u;
}

// One level: frontier[0 .. *count) -> selections and the next frontier.
__global__ __launch_bounds__(kBlock) void k_lw_level(const float* __restrict__ mean, const float* __restrict__ scale,
                                                     const float* __restrict__ quat,
                                                     const int32_t* __restrict__ offs,
                                                     const int32_t* __restrict__ ids, int64_t N, fgd::Cam cam,
                                                     float tau_R, const int32_t* __restrict__ frontier,
                                                     const uint32_t* __restrict__ count, int32_t* __restrict__ next,
                                                     uint32_t* __restrict__ next_count,
                                                     uint32_t* __restrict__ sel_bits, uint32_t* __restrict__ n_sel)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = fgd::lane_id();
    bool sel = false;
    int32_t c0 = 0, nc = 0;  // children to append
    int32_t n = -1;
    if (i < (int64_t)*count) {
        n = frontier[i];
        c0 = offs[n];
        const int32_t c1 = offs[n + 1];
        const bool leaf = c1 == c0;
        float x, y, z;
        fgd::to_camera(cam, mean[n], mean[N + n], mean[2 * N + n], x, y, z);
        bool rl = false;
        if (fgd::in_frustum(cam, x, y, z)) {
            if (leaf) {
                rl = true;
            } else {
                float S[6];
                fgd::covariance3d(scale[n], scale[N + n], scale[2 * N + n], quat[n], quat[N + n], quat[2 * N + n],
                                  quat[3 * N + n], S);
                float a, b, c;
                fgd::covariance2d(cam, x, y, z, S, a, b, c);
                rl = 3.0f * sqrtf(fgd::lambda_max(a, b, c)) <= tau_R;
            }
        }
        if (rl) sel = true;
        else nc = c1 - c0;  // an internal node that fails R&L expands (a leaf has none)
    }
    if (sel) atomicOr(&sel_bits[n >> 5], 1u << (n & 31));
    const uint64_t sb = __ballot(sel);
    if (lane == 0 && sb) atomicAdd(n_sel, (uint32_t)__popcll(sb));
    // wave-aggregated append of the children
    uint32_t x = (uint32_t)nc;
    for (int d = 1; d < fgd::kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, fgd::kWave);
        if (lane >= d) x += y;
    }
    const uint32_t total = __shfl(x, fgd::kWave - 1, fgd::kWave);
    uint32_t base = 0;
    if (total) {
        if (lane == fgd::kWave - 1) base = atomicAdd(next_count, total);
        base = __shfl(base, fgd::kWave - 1, fgd::kWave);
        const uint32_t o = base + x - (uint32_t)nc;
        for (int32_t k = 0; k < nc; k++) next[o + k] = ids[c0 + k];
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" size_t fg_children_workspace_size(int64_t n_nodes)
{
    if (n_nodes < 0) return 0;
    const int64_t n = n_nodes + 1;
    const int64_t nb = (n + kScanItems - 1) / kScanItems;
    return align_up((size_t)n * 4) * 2 + align_up((size_t)nb * 4);
}

extern "C" int fg_children(const int32_t* parent, int64_t n_nodes, int32_t* child_offs, int32_t* child_ids,
                           uint32_t* status, void* ws, size_t ws_bytes, void* stream)
{
    if (n_nodes < 0 || n_nodes >= ((int64_t)1 << 31) - 1) return FG_ERR_INVALID_TREE;
    if ((n_nodes > 0 && (!parent || !child_ids)) || !child_offs || !status) return FG_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fg_children_workspace_size(n_nodes)) return FG_ERR_WORKSPACE;
    const int64_t N = n_nodes, n = N + 1;
    const int64_t nb = (n + kScanItems - 1) / kScanItems;
    uint32_t* cnt = (uint32_t*)ws;
    uint32_t* cursor = (uint32_t*)((char*)ws + align_up((size_t)n * 4));
    uint32_t* bsum = (uint32_t*)((char*)ws + 2 * align_up((size_t)n * 4));
    hipStream_t s = (hipStream_t)stream;
    const unsigned gz = (unsigned)((n + kBlock - 1) / kBlock < 4096 ? (n + kBlock - 1) / kBlock : 4096);
    hipLaunchKernelGGL(k_zero_words, dim3(gz), dim3(kBlock), 0, s, cnt, n);
    const unsigned gn = (unsigned)((N + kBlock - 1) / kBlock > 0 ? (N + kBlock - 1) / kBlock : 1);
    if (N > 0) hipLaunchKernelGGL(k_child_count, dim3(gn), dim3(kBlock), 0, s, parent, N, cnt, status);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, s, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, n, bsum, child_offs, cursor);
    if (N > 0) hipLaunchKernelGGL(k_child_fill, dim3(gn), dim3(kBlock), 0, s, parent, N, child_offs, cursor, child_ids);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_ERR_HIP;
}

extern "C" size_t fg_filter_levelwise_workspace_size(int64_t n_nodes)
{
    if (n_nodes < 0) return 0;
    return 2 * align_up((size_t)(n_nodes > 0 ? n_nodes : 1) * 4) + 256;
}

extern "C" int fg_filter_levelwise(const fg_tree* tree, const int32_t* child_offs, const int32_t* child_ids,
                                   const fg_camera* cam, float tau_R, uint32_t* sel_bits, uint32_t* n_sel,
                                   uint32_t* status, void* ws, size_t ws_bytes, fg_levelwise_stats* stats,
                                   void* stream)
{
    if (!tree || !child_offs || !cam || !sel_bits || !n_sel || !status) return FG_ERR_INVALID_ARG;
    const int64_t N = tree->n_nodes;
    if (N < 0 || N >= ((int64_t)1 << 31) - 1 || tree->max_depth < 0 || tree->max_depth > 15)
        return FG_ERR_INVALID_TREE;
    if (N > 0 && (!tree->mean || !tree->scale || !tree->quat || !child_ids)) return FG_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0) return FG_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fg_filter_levelwise_workspace_size(N)) return FG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t fb = align_up((size_t)(N > 0 ? N : 1) * 4);
    int32_t* fr[2] = {(int32_t*)ws, (int32_t*)((char*)ws + fb)};
    uint32_t* counters = (uint32_t*)((char*)ws + 2 * fb);  // [0], [1]: sizes of the two frontiers
    const int64_t words = (N + 31) / 32;
    hipLaunchKernelGGL(k_lw_reset, dim3(1), dim3(64), 0, s, counters, n_sel);
    if (words > 0) {
        const unsigned gz = (unsigned)((words + kBlock - 1) / kBlock < 4096 ? (words + kBlock - 1) / kBlock : 4096);
        hipLaunchKernelGGL(k_zero_words, dim3(gz), dim3(kBlock), 0, s, sel_bits, words);
    }
    // level 0: the roots are the children of the virtual node N
    int32_t r01[2] = {0, 0};
    if (hipMemcpyAsync(r01, child_offs + N, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FG_ERR_HIP;
    uint32_t count = (uint32_t)(r01[1] - r01[0]);
    if (r01[0] < 0 || r01[1] < r01[0] || (int64_t)r01[1] > N) return FG_ERR_INVALID_TREE;
    if (count > 0 &&
        hipMemcpyAsync(fr[0], child_ids + r01[0], (size_t)count * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return FG_ERR_HIP;
    if (hipMemcpyAsync(counters, &count, 4, hipMemcpyHostToDevice, s) != hipSuccess) return FG_ERR_HIP;
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) return FG_ERR_HIP;
    const fgd::Cam c = fgd::make_cam(*cam);
    double calc_ms = 0.0;
    int levels = 0;
    int64_t visited = 0;
    int rc = FG_OK;
    while (count > 0) {
        if (levels > tree->max_depth) {  // deeper than the tree says: a malformed parent chain
            hipLaunchKernelGGL(k_lw_status, dim3(1), dim3(64), 0, s, status);
            break;
        }
        const int cur = levels & 1;
        uint32_t* cur_count = counters + cur;
        uint32_t* nxt_count = counters + (cur ^ 1);
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(kBlock), 0, s, nxt_count, (int64_t)1);
        visited += count;
        (void)hipEventRecord(ev[0], s);
        hipLaunchKernelGGL(k_lw_level, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tree->mean,
                           tree->scale, tree->quat, child_offs, child_ids, N, c, tau_R, fr[cur], cur_count,
                           fr[cur ^ 1], nxt_count, sel_bits, n_sel);
        (void)hipEventRecord(ev[1], s);
        // the synchronisation of the serial scheme: the next level's size
        if (hipMemcpyAsync(&count, nxt_count, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = FG_ERR_HIP;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        calc_ms += ms;
        levels++;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc == FG_OK && hipStreamSynchronize(s) != hipSuccess) rc = FG_ERR_HIP;
    const auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->levels = levels;
        stats->visited = visited;
        stats->calc_ms = calc_ms;
        stats->wall_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (rc == FG_OK && hipGetLastError() != hipSuccess) rc = FG_ERR_HIP;
    return rc;
}
