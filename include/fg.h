/*
 * fg.h -- C-ABI of libfg.so, the MI355X (gfx950) per-frame hot path of
 * FilterGS, an LoD 3D Gaussian Splatting renderer (Wang et al., CVPR 2026).
 *
 * A frame is four stream-ordered calls:
 *
 *   fg_filter      traversal-free parallel filtering of an LoD Gaussian tree
 *                  (Sec. 3.2: R&L filter + Ancestor filter, every node
 *                  evaluated independently, Eq. (4)) and stream compaction
 *                  of the selection;
 *   fg_preprocess  EWA projection of the selected Gaussians to 2D conics and
 *                  colours (Sec. 3.1, Eq. (1)) and their tile rectangles under
 *                  the opacity-aware shrink radius (Sec. 3.3, threshold tau of
 *                  Eq. (8));
 *   fg_sort        (tile, depth) ordering of the Gaussian-tile pairs (Sec. 3.3)
 *                  by prefix scan, key emission and LDS-staged radix sorts,
 *                  plus per-tile ranges;
 *   fg_render      per-tile front-to-back alpha blending, Eq. (2).
 *
 * and, for training, fg_activate and fg_render_backward (gradients of a loss
 * on the image w.r.t. the raw Gaussian parameters).
 *
 * Conventions shared by every entry point:
 *
 *  - Pointers named in a struct or argument as "device" are device memory on
 *    the current HIP device. Structs themselves (fg_tree, fg_camera,
 *    fg_splats, fg_tune) are passed by host pointer and read during the call
 *    only; the library keeps no reference to them.
 *  - Views: the stages take an array of n_views cameras (host). Per-view
 *    data lie at fixed strides: selections and splats at cap_sel entries per
 *    view, counts n_sel[v]; fg_sort and fg_render treat the views as one
 *    frame whose tiles have consecutive global ids (cams[v].tile_base =
 *    cams[v-1].tile_base + tiles of view v-1), so one pair list, one range
 *    array and one blend launch serve them all. fg_filter and fg_preprocess
 *    also accept cams_dev, a device copy of the cameras whose pose (R, t,
 *    campos) the kernels read at run time, so that a captured graph replays
 *    with poses written into it between replays (intrinsics and sizes are
 *    those of the host array, captured with the graph).
 *  - The caller owns every buffer. The library allocates nothing in these
 *    calls; scratch memory comes in through (ws, ws_bytes), sized by the
 *    matching *_workspace_size function. Workspace contents need no
 *    initialisation and are not preserved between calls.
 *  - `stream` is a hipStream_t (NULL = the null stream). Every call only
 *    enqueues work on it: no host synchronisation, no host reads of device
 *    data, so a sequence of calls can be captured into a HIP graph. Counts
 *    that depend on the data (n_sel, n_pairs) stay in device memory and the
 *    kernels read them there.
 *  - Synchronous errors (bad arguments, launch failures) are returned as a
 *    negative FG_ERR_* code and nothing is enqueued after the failing launch.
 *    Data-dependent problems are reported in the device word *status as
 *    FG_STATUS_* bits: fg_filter stores 0 into it first, later stages OR bits
 *    in. After an overflow bit, the matching count holds the size that was
 *    required, outputs beyond the capacity were not written, the outputs of
 *    that frame are undefined, and the caller retries with larger buffers.
 *  - Floating point follows one numeric contract on CPU and GPU: IEEE
 *    binary32, round to nearest even, no contraction, correctly rounded
 *    division and square root, and exp/log evaluated by fixed published
 *    methods, so selections, tile sets, orders and pixels are reproducible
 *    bit for bit.
 *  - The library keeps no global mutable state; calls on different streams
 *    with disjoint buffers may overlap.
 */
#ifndef FG_H
#define FG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define FG_OK 0
#define FG_ERR_INVALID_ARG (-1)   /* null pointer, negative size, bad enum */
#define FG_ERR_INVALID_TREE (-2)  /* tree fields inconsistent (sizes, depth) */
#define FG_ERR_UNSUPPORTED (-3)   /* e.g. SH degree > 3, image too large */
#define FG_ERR_WORKSPACE (-4)     /* ws_bytes below the *_workspace_size value */
#define FG_ERR_HIP (-5)           /* a HIP launch or runtime call failed */
#define FG_ERR_SCRATCH (-6)       /* fg_filter_noalloc: the problem needs more than
                                     FG_NOALLOC_SCRATCH_BYTES of workspace */

/* ---- device status bits ------------------------------------------------ */
#define FG_STATUS_SEL_OVERFLOW 1u   /* more selected nodes than cap_sel */
#define FG_STATUS_PAIR_OVERFLOW 2u  /* more Gaussian-tile pairs than cap_pairs */
#define FG_STATUS_BAD_PARENT 4u     /* a parent index >= the child's index, a
                                       parent that is a leaf, or an ancestor chain
                                       longer than max_depth */
#define FG_STATUS_GTC_UNDEFINED 8u  /* fg_gtc_tau: no view holds a Gaussian-tile
                                       pair, so G_bar (Eq. (8)) is undefined */
#define FG_STATUS_ITEM_OVERFLOW 16u /* fg_sort: more tile-covering splats than cap_items */

/* ---- inputs ------------------------------------------------------------ */

/* An LoD Gaussian tree (Sec. 3.1 "Hierarchical Gaussian Tree"): every node is
 * a complete Gaussian with mean mu, covariance R(q) diag(s)^2 R(q)^T, opacity
 * and spherical-harmonic colour (Sec. 3.1, Eq. (1)). The ancestor path of a
 * node (Sec. 3.2 "Ancestor Filter") is its chain of parent links.
 * All planes are device memory, structure of arrays. */
typedef struct fg_tree {
    int64_t n_nodes;         /* N, 0 <= N < 2^31 */
    int64_t n_internal_span; /* every internal (non-leaf) node has index < this;
                                nodes at or beyond it are all leaves */
    int32_t sh_degree;       /* D in 0..3; (D+1)^2 coefficients per channel */
    int32_t max_depth;       /* longest root-to-node chain, 0..15 */
    const float* mean;       /* [3][N] x, y, z planes, world units */
    const float* scale;      /* [3][N] linear (activated) scales */
    const float* quat;       /* [4][N] rotation (w, x, y, z), any non-zero norm */
    const float* opacity;    /* [N] activated opacity; nodes outside (0, 1] emit nothing */
    const float* sh;         /* [N][(D+1)^2][3] coefficient-major, RGB-minor;
                                16-byte aligned (read 16 bytes at a time) */
    const int32_t* parent;   /* [N] parent index (< own index), -1 for a root */
    const uint8_t* flags;    /* [N] bit 0: leaf. Read only for index < n_internal_span */
    const float* tile_box;   /* optional (null: unused): the boxes fg_tree_boxes writes
                                for this tree's mean and parent planes; rebuild them
                                whenever those planes change */
} fg_tree;

/* Filter acceleration boxes (not part of the method; they change no result).
 * In the filter's R&L test (Sec. 3.2) a node passes only when its mean is in
 * the frustum (a leaf by F, an internal node through small). The filter reads
 * the nodes in blocks of 2048 consecutive indices; fg_tree_boxes stores the
 * axis-aligned box of each block's means, and the filter skips a block whose
 * box lies outside every view's frustum by a margin above float32 rounding
 * (none of its nodes could pass), reading none of its nodes in the selection
 * pass and no attributes of its internal nodes in the projected-size pass. A
 * block holding a parent link the filter would reject gets a NaN box and is
 * never skipped, so FG_STATUS_BAD_PARENT is reported as without boxes.
 * The same array also holds, per 256 consecutive nodes below n_internal_span,
 * the index range of their children: the filter leaves out the ancestor walks
 * of such a group when all of its children lie in skipped blocks (only those
 * children read the walks' results), unless a node of the group has a parent
 * chain the filter would reject.
 * fg_tree_box_floats: the float count of the array (8 per block: lo.xyz, 0,
 * hi.xyz, 0; then 2 int32 per group), -1 for inconsistent sizes.
 * fg_tree_boxes: writes it (device memory, 16-byte aligned, caller-owned),
 * stream-ordered. Errors: FG_ERR_INVALID_ARG (null pointers),
 * FG_ERR_INVALID_TREE (sizes as in fg_filter), FG_ERR_HIP. */
int64_t fg_tree_box_floats(int64_t n_nodes, int64_t n_internal_span);
int fg_tree_boxes(const fg_tree* tree, float* tile_box, void* stream);

/* Pinhole camera: x_c = R x_w + t, axes x right, y down, z forward.
 * Pixel (i, j) has its centre at (i + 0.5, j + 0.5); u = fx x_c / z_c + cx.
 * A node is in the frustum when z_c > znear, |x_c| <= kx z_c and
 * |y_c| <= ky z_c (a guard band around the image). Tiles are 16 x 16
 * pixels; this view's tiles have the global ids tile_base + ty*Wt + tx with
 * Wt = ceil(width/16). */
typedef struct fg_camera {
    float R[9];       /* row-major world->camera rotation */
    float t[3];
    float campos[3];  /* camera centre in world space (SH view direction) */
    float fx, fy, cx, cy;
    int32_t width, height;  /* 1..32768 */
    float znear, kx, ky;
    uint32_t tile_base;
} fg_camera;

/* Projected Gaussians ("splats"), device planes of capacity cap_sel entries,
 * entry i describing the i-th selected node (sel_idx[i]). */
typedef struct fg_splats {
    float* xy;         /* [cap][2] 2D mean (u, v) in pixels */
    float* conic_o;    /* [cap][4] (A, B, C, opacity): inverse 2D covariance
                          [[A, B], [B, C]] and the node opacity */
    float* rgb_depth;  /* [cap][4] colour (r, g, b) and camera-space depth */
    uint16_t* rect;    /* [cap][4] tile rectangle [x0, x1) x [y0, y1) as
                          (x0, y0, x1, y1); all zero when the splat emits nothing */
    uint32_t* tiles;   /* [cap] (x1 - x0) * (y1 - y0): pairs this splat emits */
} fg_splats;

/* Speed-only knobs; results never depend on them. NULL = defaults. */
typedef struct fg_tune {
    int32_t render_batch;  /* splats per blend work item (chunk): 128, 256 or 512 (default 256) */
    int32_t radix_bits;    /* digit width of the pair sort: 4..8 (default: the narrowest width
                              that needs no more passes than 8-bit digits, e.g. 7 for
                              13-bit tile ids) */
    int32_t save_state;    /* 1: fg_render keeps, for every chunk of a long range, each pixel's
                              (T, C) after that chunk in its workspace (sized for it by
                              fg_render_workspace_size with the same tune), which
                              fg_render_backward reads; 0: not kept (default) */
    int32_t mask_items;    /* at most this many chunks of long ranges get their pass masks
                              stored by the parallel mask kernel; later chunks compute
                              them in the blend itself (0: as many as 256 MiB hold) */
    void* blend_events[2]; /* NULL, NULL: none; else two caller-owned hipEvent_t that fg_render
                              records on its stream right before and right after its blend
                              kernel (k_render), for timing that kernel alone */
    unsigned long long* bwd_stats; /* NULL: none; else 3 device counters that fg_render_backward
                              adds to (the caller zeroes them): [0] gradient atomic
                              instructions of the blend's backward (one per wave and splat
                              with a blended pixel), [1] gradient elements those add,
                              [2] blended fragments walked */
} fg_tune;

/* ---- stage 1: traversal-free parallel filter (Sec. 3.2) ---------------- */

/* Scratch bytes fg_filter needs for a tree of n_nodes nodes and n_views views. */
size_t fg_filter_workspace_size(int64_t n_nodes, int64_t n_internal_span, int32_t n_views);

/* For every view v of cams[0 .. n_views) (a host array) and every node n,
 * independently:
 *   F(n)     in-frustum test of the node centre (fg_camera);
 *   small(n) F(n) and R_2D = 3 sqrt(lambda_max(Sigma_2D)) <= tau_R, with
 *            Sigma_2D the EWA projection plus 0.3 px^2 on the diagonal
 *            (R&L filter, Sec. 3.2; tau_R = 3 in the paper);
 *   RL(n)    F(n) and (leaf(n) or small(n)) (leaf exemption);
 *   sel(n)   RL(n) and no ancestor a of n has RL(a) (Ancestor filter).
 * Up to 8 views share one pass over the tree (each node's data is read once
 * for all of them). Outputs per view v (device): sel_bits + v*ceil(N/32)
 * words, bit n%32 of word n/32 = sel(n); sel_idx + v*cap_sel, the selected
 * node ids in ascending order; n_sel[v] the number selected. *status
 * (device u32) is set to 0, then FG_STATUS_SEL_OVERFLOW / FG_STATUS_BAD_PARENT
 * as they occur. cams_dev: NULL, or the views' poses in device memory (see
 * the conventions above).
 * Errors: FG_ERR_INVALID_ARG for null pointers, n_views < 1 or cap_sel < 0,
 * FG_ERR_INVALID_TREE for n_nodes out of range, n_internal_span outside
 * [0, n_nodes] or max_depth outside 0..15, FG_ERR_WORKSPACE. */
int fg_filter(const fg_tree* tree, const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev, float tau_R,
              uint32_t* sel_bits, uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel, uint32_t* status, void* ws,
              size_t ws_bytes, void* stream);

/* fg_filter without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, outputs, status bits and errors as
 * fg_filter; the scratch space is a fixed device array of
 * FG_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends. The call allocates nothing (its first call on a device only
 * looks up that device's array address). It returns FG_ERR_SCRATCH, before
 * enqueueing anything, when fg_filter_workspace_size(n_nodes,
 * n_internal_span, n_views) exceeds FG_NOALLOC_SCRATCH_BYTES (16 MiB; views
 * are filtered 8 per pass in the same scratch, so a 20M-node tree with 2.5M
 * internal nodes needs 5.1 MiB for any number of views).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams, or host threads, without ordering between them)
 * race on it and give undefined selections. Calls ordered on one stream are
 * safe; no contents carry over from one call to the next. */
#define FG_NOALLOC_SCRATCH_BYTES (16u << 20)
int fg_filter_noalloc(const fg_tree* tree, const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev,
                      float tau_R, uint32_t* sel_bits, uint32_t* sel_idx, int64_t cap_sel, uint32_t* n_sel,
                      uint32_t* status, void* stream);

/* ---- the serial level-wise filter (the scheme Sec. 3.2 replaces) -------- */

/* Children of every node as a CSR built from the parent links, for top-down
 * walks: the children of node n are child_ids[child_offs[n] ..
 * child_offs[n+1]), and a virtual node N holds the roots (child_offs has
 * N + 2 entries, child_ids N; device). Sibling order is unspecified. A node
 * whose parent index is not below its own is left out and
 * FG_STATUS_BAD_PARENT is ORed into *status. Built once per tree.
 * Errors: FG_ERR_INVALID_ARG, FG_ERR_INVALID_TREE, FG_ERR_WORKSPACE. */
size_t fg_children_workspace_size(int64_t n_nodes);
int fg_children(const int32_t* parent, int64_t n_nodes, int32_t* child_offs, int32_t* child_ids, uint32_t* status,
                void* ws, size_t ws_bytes, void* stream);

/* Timing of one fg_filter_levelwise call (host struct). */
typedef struct fg_levelwise_stats {
    int32_t levels;   /* frontier levels evaluated */
    int32_t pad;
    int64_t visited;  /* nodes evaluated over all levels */
    double calc_ms;   /* sum of the level kernels' durations (HIP events): T_calcu */
    double wall_ms;   /* host wall time of the whole call; wall - calc is T_synch */
} fg_levelwise_stats;

/* The same selection as fg_filter for one camera, computed the serial way
 * (Sec. 3.2, Eq. (3)): the cut grows from the roots one level at a time;
 * each frontier node that passes R&L (in frustum, leaf or
 * R_2D = 3 sqrt(lambda_max) <= tau_R) is selected and ends its branch, every
 * other internal node passes its children to the next level. One kernel
 * launch per level, after which the host reads the next frontier's size: the
 * call SYNCHRONISES the stream once per level (it is the baseline the
 * traversal-free filter is measured against, and cannot be graph-captured).
 * Outputs (device): sel_bits [ceil(N/32)] as in fg_filter (order-free: a
 * bitmask), *n_sel. child_offs / child_ids from fg_children. stats (host,
 * may be NULL) receives the level count and the T_calcu / wall split.
 * Errors: FG_ERR_INVALID_ARG, FG_ERR_INVALID_TREE, FG_ERR_WORKSPACE,
 * FG_ERR_HIP; FG_STATUS_BAD_PARENT when the walk goes deeper than max_depth. */
size_t fg_filter_levelwise_workspace_size(int64_t n_nodes);
int fg_filter_levelwise(const fg_tree* tree, const int32_t* child_offs, const int32_t* child_ids,
                        const fg_camera* cam, float tau_R, uint32_t* sel_bits, uint32_t* n_sel, uint32_t* status,
                        void* ws, size_t ws_bytes, fg_levelwise_stats* stats, void* stream);

/* ---- stage 2: projection and shrunk extents (Sec. 3.1, Sec. 3.3) -------- */

/* For each view v (cams[v], pose from cams_dev + v when cams_dev is given) and
 * i < min(n_sel[v], cap_sel), node g = sel_idx[v*cap_sel + i], written to
 * splat entry v*cap_sel + i of out: camera-space centre,
 * Sigma_2D (+0.3 px^2), conic = Sigma_2D^-1 (dropped when det <= 0), 2D mean,
 * depth, colour 0.5 + sum_k sh_k Y_k(d) clamped at 0 with d the unit vector
 * from campos to the mean and Y the orthonormal real SH basis, and the
 * tile-set radius
 *     r = 3 sqrt(lambda_max)                               if tau <= 0,
 *     r = 0                                                if alpha0 <= tau,
 *     r = min(3 sqrt(lambda_max), sqrt(2 lambda_max ln(alpha0 / tau)))  else
 * (Sec. 3.3 "Gaussian Shrinking Strategy"; tau = lambda_G / G_bar, Eq. (8),
 * or 1/255 for a fixed threshold). The rectangle holds every tile whose
 * 16-px square meets [u - r, u + r] x [v - r, v + r]. Only the tile set
 * shrinks; blending still evaluates the full Gaussian. Views are processed
 * 8 per launch.
 * Errors: FG_ERR_INVALID_ARG, FG_ERR_UNSUPPORTED (sh_degree > 3). */
int fg_preprocess(const fg_tree* tree, const uint32_t* sel_idx, const uint32_t* n_sel, int64_t cap_sel,
                  const fg_camera* cams, int32_t n_views, const fg_camera* cams_dev, float tau,
                  const fg_splats* out, uint32_t* status, void* stream);

/* ---- stage 3: key emission, sort, ranges ------------------------------ */

/* Scratch bytes fg_sort needs. */
size_t fg_sort_workspace_size(int64_t cap_sel, int32_t n_views, int64_t cap_items, int64_t cap_pairs);

/* Orders the Gaussian-tile pairs of all views by the key (global tile id,
 * depth bits) and then by splat index: splat j of view v (global splat index
 * v*cap_sel + j, j < n_sel[v]) contributes one pair per tile of its rectangle.
 * Outputs (device): tile_keys [cap_pairs] the sorted global tile ids
 * (tile_base + ty*Wt + tx of the splat's view), vals [cap_pairs] the matching
 * global splat indices (the full 64-bit key of entry k is
 * tile_keys[k] << 32 | bits(depth[vals[k]])); *n_pairs (device u32);
 * ranges [n_tiles][2] over the tiles of all views in global id order
 * (entry t is global tile cams[0].tile_base + t): [start, end) in the sorted
 * list, [0, 0) for an empty tile.
 * Method: the splats that cover a tile are stably radix-sorted by depth (the
 * first pass reads the selections in (view, index) order and leaves out the
 * others); an exclusive prefix scan of their tile counts
 * in that order places their pairs (key emission), and a stable radix sort of
 * the pairs by tile id gives the (tile, depth, index) order (LDS-staged LSD
 * passes throughout). cap_items bounds the tile-covering splats of all views
 * together (cap_sel for one view).
 * Errors: FG_ERR_INVALID_ARG (also for global tile ids that are not
 * consecutive from view to view), FG_ERR_UNSUPPORTED (n_views > 64,
 * n_views*cap_sel >= 2^32), FG_ERR_WORKSPACE; on the device
 * FG_STATUS_PAIR_OVERFLOW when the pairs exceed cap_pairs (n_pairs then holds
 * the required count) and FG_STATUS_ITEM_OVERFLOW when the tile-covering
 * splats exceed cap_items. */
int fg_sort(const fg_splats* splats, const uint32_t* n_sel, int64_t cap_sel, const fg_camera* cams,
            int32_t n_views, int64_t cap_items, uint32_t* tile_keys, uint32_t* vals, int64_t cap_pairs,
            uint32_t* n_pairs, uint32_t* ranges, uint32_t* status, void* ws, size_t ws_bytes, const fg_tune* tune,
            void* stream);

/* ---- stage 4: blending, Eq. (2) --------------------------------------- */

/* Scratch bytes fg_render needs for these views and pair capacity. */
size_t fg_render_workspace_size(const fg_camera* cams, int32_t n_views, int64_t cap_pairs, const fg_tune* tune);

/* For every pixel of tile t, front to back over ranges[t]:
 *   power = -0.5 (A dx^2 + C dy^2) - B dx dy, d = (u, v) - pixel centre;
 *   skip if power > 0; alpha = min(0.99, opacity exp(power)), skip if
 *   alpha < 1/255; stop before a splat that would take T below 1e-4;
 *   C += rgb alpha T; T *= (1 - alpha).
 * Outputs (device), per view v with P_v the pixels of the views before it:
 * image + 3*P_v, [3][H][W] = C + T bg; final_T + P_v, [H][W];
 * n_contrib + P_v, [H][W] = 1 + position (within the tile's range) of the
 * last splat blended, 0 if none. bg is a host array of 3 floats. vals and
 * ranges are fg_sort's for the same views (global splat indices, tiles in
 * global id order). cap_pairs is the capacity the sort ran with (it bounds
 * the range lengths and sizes the workspace). The tiles of all views form
 * one work queue of one persistent blend launch. Long ranges are cut into
 * chunks whose skip tests run in parallel (a first launch writes per-pixel
 * pass masks); the transmittance chain still runs in list order, so results
 * are those of one sequential pass.
 * frag_stats: NULL, or 8 device counters that the call adds to (the caller
 * zeroes them): [0] (pixel, splat) tests evaluated, [1] tests that reach the
 * exponential (-5.6 <= power <= 0), [2] tests with alpha >= 1/255, [3] splats
 * blended, counted in the blend kernel; [4..6] the same three test counts
 * made by the mask kernel for chunks of long ranges ([7] stays 0). Results do
 * not depend on whether counting is on.
 * status is reserved (not written). Errors: FG_ERR_INVALID_ARG,
 * FG_ERR_WORKSPACE. */
int fg_render(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cams,
              int32_t n_views, const float bg[3], float* image, float* final_T, uint32_t* n_contrib,
              int64_t cap_pairs, unsigned long long* frag_stats, uint32_t* status, void* ws, size_t ws_bytes,
              const fg_tune* tune, void* stream);

/* ---- GTC pre-pass and the scene threshold (Sec. 3.3, Fig. 2(b)) -------- */

/* For one view rendered by fg_filter, fg_preprocess (tau <= 0: the 3-sigma
 * extents of the pre-rendering pass) and fg_sort, with the same camera:
 *   kpc [cap_pairs] (device, entries [0, n_pairs) written): the key-value pair
 *       contribution of each sorted pair k, Eq. (5): the sum over the pixels
 *       of its tile of alpha * T for the pixels that blend that splat (the
 *       tests and termination of Eq. (2), as fg_render; fragments skipped or
 *       never reached add nothing). Each pixel's terms are float32 products
 *       identical to the sequential blend's; their sum is float32 in an
 *       unspecified order.
 *   tile_gtc [n_tiles] (device): the tile's GTC, Eq. (6), the mean KPC over
 *       all pairs of the tile, zero contributions included; NaN for a tile
 *       without pairs (0/0).
 *   view_gtc [2] (device float64): [0] the view's GTC, Eq. (7), the mean of
 *       tile_gtc over the tiles that hold pairs (0 if none); [1] the number of
 *       those tiles.
 *   kpc_hist (device, optional): with n_edges ascending host values
 *       hist_edges (1..16), counts are ADDED to kpc_hist[0 .. n_edges]: bin b
 *       holds the pairs with hist_edges[b-1] <= KPC < hist_edges[b] (bin 0
 *       below hist_edges[0], bin n_edges at or above the last edge); the
 *       caller zeroes it. NULL with n_edges = 0: no histogram.
 * n_pairs (device) and cap_pairs are the sort's pair count and capacity:
 * when the sort overflowed (n_pairs > cap_pairs) every tile is left undefined
 * and view_gtc = (NaN, -1), which fg_gtc_tau reports as an overflow.
 * With n_contrib, render_ws, render_ws_bytes and tune all NULL/0, each tile's
 * list is walked front to back by one workgroup. When the view was also
 * rendered by fg_render (same sort, camera and cap_pairs) with a tune that
 * sets save_state, passing that call's n_contrib, ws and tune splits the long
 * lists into their chunks: each chunk is walked from the transmittance the
 * blend saved after the previous one, and a fragment counts exactly when its
 * list position is below the pixel's contributor count and it passes the
 * skip tests, so every alpha * T and every per-pair sum is the same as in
 * the tile walk, with the long tiles no longer on one workgroup.
 * Errors: FG_ERR_INVALID_ARG (null pointers, bad edges, a render workspace
 * that does not match or holds no saved state). */
int fg_gtc(const fg_splats* splats, const uint32_t* vals, const uint32_t* ranges, const fg_camera* cam,
           const uint32_t* n_pairs, int64_t cap_pairs, float* kpc, float* tile_gtc, double* view_gtc, const float* hist_edges,
           int32_t n_edges, uint32_t* kpc_hist, const uint32_t* n_contrib, const void* render_ws,
           size_t render_ws_bytes, const fg_tune* tune, void* stream);

/* Eq. (8) over n_views views: view_gtc [n_views][2] (device float64, each
 * written by fg_gtc); g_bar (device float64) = the mean view GTC over the
 * views that hold pairs; tau (device float32) = lambda_G / g_bar, rounded
 * once from float64 (lambda_G = 0.2 in Sec. 4.1). With no such view, g_bar
 * = 0, tau = NaN and FG_STATUS_GTC_UNDEFINED is ORed into *status (device,
 * may be NULL); if a view's sort overflowed, g_bar = tau = NaN and
 * FG_STATUS_PAIR_OVERFLOW is ORed in. Errors: FG_ERR_INVALID_ARG. */
int fg_gtc_tau(const double* view_gtc, int32_t n_views, float lambda_G, double* g_bar, float* tau,
               uint32_t* status, void* stream);

/* ---- differentiable form (Sec. 3.1: differentiable splatting) ---------- */

/* Raw, unconstrained parameters of M Gaussians (device planes). The activated
 * values are scale = exp(log_scale) and opacity = 1 / (1 + exp(-logit)). */
typedef struct fg_params {
    int64_t m;
    int32_t sh_degree;       /* 0..3 */
    int32_t pad;
    const float* mean;       /* [3][M] */
    const float* log_scale;  /* [3][M] */
    const float* quat;       /* [4][M] (w, x, y, z), any non-zero norm */
    const float* logit;      /* [M] */
    const float* sh;         /* [M][(D+1)^2][3], 16-byte aligned */
} fg_params;

/* Gradients of a scalar loss w.r.t. the raw parameters, same shapes as
 * fg_params (device, overwritten; zero for Gaussians not rendered). */
typedef struct fg_grads {
    float* mean;
    float* log_scale;
    float* quat;
    float* logit;
    float* sh;               /* 16-byte aligned */
} fg_grads;

/* scale [3][M] = exp(log_scale), opacity [M] = 1 / (1 + exp(-logit)), with the
 * library's exponential (|argument| <= 87). The activated planes, with p->mean,
 * p->quat and p->sh, form an fg_tree of M root leaves (parent -1, flags 1)
 * that fg_filter / fg_preprocess / fg_sort / fg_render render.
 * Errors: FG_ERR_INVALID_ARG. */
int fg_activate(const fg_params* p, float* scale, float* opacity, void* stream);

/* Scratch bytes fg_render_backward needs (9 floats per splat). */
size_t fg_render_backward_workspace_size(int64_t cap_sel);

/* Backward pass of a frame rendered from p (after fg_activate) by fg_filter,
 * fg_preprocess, fg_sort and fg_render: given dL/dimage [3][H][W] (device),
 * writes dL/d(raw parameters) into out. Inputs are that frame's sel_idx,
 * n_sel (device), splats, sorted vals, ranges, final_T and n_contrib, the
 * same camera and background. For every pixel the blended splats are the
 * forward's (position below n_contrib and the same skip tests), visited back
 * to front with the transmittance recovered from final_T
 * (T_k = T_{k+1} / (1 - alpha_k)); alpha capped at 0.99 passes no gradient to
 * opacity or position; the tile rectangle and shrink radius are piecewise
 * constant and pass none. Gradients are summed with float32 atomics, so the
 * summation order (and the last bits) vary between runs.
 * image, render_ws (render_ws_bytes), cap_pairs, tune: that frame's image and
 * the workspace, pair capacity and tune its fg_render call used. When tune
 * has save_state, the chunks of long ranges are walked in parallel, each
 * from the state the forward kept after it (T, and the colour behind as image
 * minus the colour accumulated so far); otherwise, or if render_ws or image is
 * NULL, every tile is walked whole from final_T.
 * Errors: FG_ERR_INVALID_ARG, FG_ERR_UNSUPPORTED (sh_degree > 3),
 * FG_ERR_WORKSPACE. */
int fg_render_backward(const fg_params* p, const fg_camera* cam, const float bg[3], const uint32_t* sel_idx,
                       const uint32_t* n_sel, int64_t cap_sel, const fg_splats* splats, const uint32_t* vals,
                       const uint32_t* ranges, const float* final_T, const uint32_t* n_contrib,
                       const float* image, const void* render_ws, size_t render_ws_bytes, int64_t cap_pairs,
                       const fg_tune* tune, const float* dL_dimage, const fg_grads* out, void* ws,
                       size_t ws_bytes, void* stream);

/* Text for an FG_* return code. */
const char* fg_status_string(int code);


#ifdef __cplusplus
}
#endif
#endif /* FG_H */
