"""Seeded synthetic inputs: LoD Gaussian trees, cameras and camera paths.

This module only *builds inputs*. It holds none of the per-frame method's
arithmetic (filtering, projection, shrinking, sorting, blending): both the
HIP path and the CPU oracle consume what it returns, and neither is imported
here. Rotations come from ``scipy.spatial.transform`` and covariance
eigendecompositions from ``numpy.linalg.eigh``; everything is computed in
float64 and rounded once to float32.

Tree layout (the one the C-ABI reads):

* nodes ``0..N-1`` in level order (root level first), Morton order within a
  level, the children of a node contiguous in the next level;
* ``mean[3][N]``, ``scale[3][N]`` (linear), ``quat[4][N]`` as (w, x, y, z),
  ``opacity[N]`` in (0, 1), ``sh[N][(D+1)^2][3]``;
* ``parent[N]`` (int32, -1 for a root, ``parent[i] < i``), ``flags[N]``
  (uint8: bit 0 = leaf, bits 1-4 = depth).

The tree model follows the paper's hierarchical Gaussian tree (Sec. 3.1,
"Hierarchical Gaussian Tree"): every node is a complete Gaussian. The city
trees are built bottom-up (parents are moment-matched merges of their up to 8
children); ``topdown_tree`` builds the paper's own canonical construction top
down (children placed at oriented offsets of the parent, shrunk by gamma,
inheriting rotation, colour and opacity).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy.spatial.transform import Rotation

SH_COEFFS = {0: 1, 1: 4, 2: 9, 3: 16}
Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi)): degree-0 real SH constant


# --------------------------------------------------------------------------
# trees
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Tree:
    mean: np.ndarray      # f32 [3, N]
    scale: np.ndarray     # f32 [3, N]
    quat: np.ndarray      # f32 [4, N]  (w, x, y, z)
    opacity: np.ndarray   # f32 [N]
    sh: np.ndarray        # f32 [N, K, 3]
    parent: np.ndarray    # i32 [N]
    flags: np.ndarray     # u8  [N]
    sh_degree: int
    n_internal_span: int  # every internal node has index < n_internal_span
    max_depth: int
    level_sizes: List[int]

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    @property
    def is_leaf(self) -> np.ndarray:
        return (self.flags & 1).astype(bool)

    @property
    def depth(self) -> np.ndarray:
        return ((self.flags >> 1) & 15).astype(np.int32)


def _part1by2(v: np.ndarray) -> np.ndarray:
    """Spread the low 21 bits of v so that two zero bits separate each bit."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_order(pos: np.ndarray) -> np.ndarray:
    """Permutation sorting points [n, 3] by their 63-bit Morton code."""
    lo = pos.min(axis=0)
    ext = np.maximum(pos.max(axis=0) - lo, 1e-12)
    q = np.floor((pos - lo) / ext * (2 ** 21 - 1)).astype(np.uint64)
    code = _part1by2(q[:, 0]) | (_part1by2(q[:, 1]) << np.uint64(1)) | (_part1by2(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def _cov_from_scale_quat(scale: np.ndarray, quat_wxyz: np.ndarray) -> np.ndarray:
    """Covariance R diag(s^2) R^T in float64 for [n] Gaussians (generator use)."""
    rot = Rotation.from_quat(np.stack([quat_wxyz[1], quat_wxyz[2], quat_wxyz[3], quat_wxyz[0]], axis=1)).as_matrix()
    rs = rot * (scale.T.astype(np.float64) ** 2)[:, None, :]
    return np.matmul(rs, np.transpose(rot, (0, 2, 1)))


def _scale_quat_from_cov(cov: np.ndarray):
    """Eigen-decompose covariances [n,3,3] (f64) into linear scales and (w,x,y,z) quats."""
    lam, vec = np.linalg.eigh(cov)
    det = np.linalg.det(vec)
    vec[det < 0, :, 2] *= -1.0
    scale = np.sqrt(np.maximum(lam, 1e-30)).T  # [3, n]
    q = Rotation.from_matrix(vec).as_quat()    # (x, y, z, w)
    quat = np.stack([q[:, 3], q[:, 0], q[:, 1], q[:, 2]], axis=0)
    return scale, quat


def _group_reduce(x: np.ndarray, starts: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Mean over consecutive groups along axis 0, accumulated in float64."""
    s = np.add.reduceat(x.astype(np.float64, copy=False), starts, axis=0)
    shape = (-1,) + (1,) * (x.ndim - 1)
    return s / counts.reshape(shape)


def lod_tree_from_leaves(pos, log_scale, quat, opacity, sh, sh_degree: int,
                         branching: int = 8, root_max: int = 9, chunk: int = 1 << 21) -> Tree:
    """Build a level-ordered LoD tree over Morton-sorted leaves.

    Leaves are grouped ``branching`` at a time, level by level, until at most
    ``root_max`` nodes remain; one root then takes all of them as children.
    Every parent is the moment-matched, uniformly weighted merge of its
    children: mean of means, mean of (child covariance + outer product of the
    child's offset), mean opacity, mean SH.

    pos [n,3] f64, log_scale [n,3] f64, quat [n,4] (w,x,y,z) f64, opacity [n]
    f64, sh [n,K,3] f32. Leaves must already be in Morton order.
    """
    n = pos.shape[0]
    K = SH_COEFFS[sh_degree]
    # per-level attribute lists, leaves first (reversed at the end)
    lv_mean = [pos.astype(np.float64)]
    lv_scale = [np.exp(log_scale).T.astype(np.float64)]
    lv_quat = [quat.T.astype(np.float64)]
    lv_op = [opacity.astype(np.float64)]
    lv_sh = [sh.astype(np.float32)]
    child_group = []  # per transition: group index of each child
    # leaf covariances, computed in chunks
    cov = np.empty((n, 3, 3), np.float64)
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        cov[s0:s1] = _cov_from_scale_quat(lv_scale[0][:, s0:s1], lv_quat[0][:, s0:s1])
    cur_n = n
    while cur_n > 1:
        if cur_n <= root_max:
            groups = np.zeros(cur_n, np.int64)
            starts = np.array([0])
        else:
            groups = np.arange(cur_n, dtype=np.int64) // branching
            starts = np.arange(0, cur_n, branching)
        counts = np.diff(np.append(starts, cur_n)).astype(np.float64)
        mu_c = lv_mean[-1]
        mu_p = _group_reduce(mu_c, starts, counts)
        d = mu_c - mu_p[groups]
        second = cov + d[:, :, None] * d[:, None, :]
        cov_p = _group_reduce(second, starts, counts)
        del second, d
        op_p = _group_reduce(lv_op[-1], starts, counts)
        sh_p = _group_reduce(lv_sh[-1], starts, counts).astype(np.float32)
        sc_p, q_p = _scale_quat_from_cov(cov_p.copy())
        lv_mean.append(mu_p)
        lv_scale.append(sc_p)
        lv_quat.append(q_p)
        lv_op.append(op_p)
        lv_sh.append(sh_p)
        child_group.append(groups)
        cov = cov_p
        cur_n = mu_p.shape[0]
    n_levels = len(lv_mean)
    # reverse to root-first level order
    lv_mean.reverse(); lv_scale.reverse(); lv_quat.reverse(); lv_op.reverse(); lv_sh.reverse()
    child_group.reverse()
    sizes = [m.shape[0] for m in lv_mean]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    N = int(offs[-1])
    parent = np.full(N, -1, np.int32)
    flags = np.zeros(N, np.uint8)
    for lvl in range(n_levels):
        flags[offs[lvl]:offs[lvl + 1]] = np.uint8(lvl << 1)
        if lvl > 0:
            parent[offs[lvl]:offs[lvl + 1]] = (offs[lvl - 1] + child_group[lvl - 1]).astype(np.int32)
    flags[offs[n_levels - 1]:] |= np.uint8(1)
    mean = np.empty((3, N), np.float32)
    scale = np.empty((3, N), np.float32)
    quatv = np.empty((4, N), np.float32)
    op = np.empty(N, np.float32)
    shv = np.empty((N, K, 3), np.float32)
    for lvl in range(n_levels):
        a, b = offs[lvl], offs[lvl + 1]
        mean[:, a:b] = lv_mean[lvl].T
        scale[:, a:b] = lv_scale[lvl]
        quatv[:, a:b] = lv_quat[lvl]
        op[a:b] = lv_op[lvl]
        shv[a:b] = lv_sh[lvl]
    return Tree(mean=mean, scale=scale, quat=quatv, opacity=op, sh=shv, parent=parent, flags=flags,
                sh_degree=sh_degree, n_internal_span=int(offs[n_levels - 1]), max_depth=n_levels - 1,
                level_sizes=sizes)


def _unit_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def tiny_tree(seed: int = 0) -> Tree:
    """4,096 leaves uniform in [-10,10]^3, branching 8 -> 4,681 nodes, SH degree 0.

    log-scales N(-2, 0.5) per axis, random unit quaternions, opacity logits
    N(0, 1), RGB uniform in [0,1] stored as the degree-0 SH coefficient
    (c - 0.5) / Y00.
    """
    rng = np.random.default_rng(seed)
    n = 4096
    pos = rng.uniform(-10.0, 10.0, (n, 3))
    order = morton_order(pos)
    pos = pos[order]
    log_s = rng.normal(-2.0, 0.5, (n, 3))
    quat = _unit_quats(rng, n)
    op = _sigmoid(rng.normal(0.0, 1.0, n))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh = ((rgb - 0.5) / Y00).astype(np.float32)[:, None, :]
    return lod_tree_from_leaves(pos, log_s, quat, op, sh, sh_degree=0)


@dataclasses.dataclass
class CitySpec:
    """Clustered 'city-like' leaf cloud: Gaussian blobs inside a flat box."""
    n_leaves: int
    box: Sequence[float]          # (x_half, y_half, z_max): x,y in [-h, h], z in [0, z_max]
    n_blobs: int
    blob_sigma: Sequence[float]
    leaf_log_scale_mu: float
    leaf_log_scale_sd: float = 0.5
    logit_sd: float = 1.5
    sh_degree: int = 3
    sh_sd: float = 0.3
    seed: int = 0


def city_leaves(spec: CitySpec):
    rng = np.random.default_rng(spec.seed)
    n, nb = spec.n_leaves, spec.n_blobs
    hx, hy, zmax = spec.box
    lo = np.array([-hx, -hy, 0.0]); hi = np.array([hx, hy, zmax])
    centres = rng.uniform(lo, hi, (nb, 3))
    per = np.full(nb, n // nb); per[: n % nb] += 1
    blob = np.repeat(np.arange(nb), per)
    sig = np.asarray(spec.blob_sigma, np.float64)
    pos = centres[blob] + rng.standard_normal((n, 3)) * sig
    bad = np.nonzero(np.any((pos < lo) | (pos > hi), axis=1))[0]
    while bad.size:
        pos[bad] = centres[blob[bad]] + rng.standard_normal((bad.size, 3)) * sig
        bad = bad[np.any((pos[bad] < lo) | (pos[bad] > hi), axis=1)]
    order = morton_order(pos)
    pos = pos[order]
    log_s = rng.normal(spec.leaf_log_scale_mu, spec.leaf_log_scale_sd, (n, 3))
    quat = _unit_quats(rng, n)
    op = _sigmoid(rng.normal(0.0, spec.logit_sd, n))
    K = SH_COEFFS[spec.sh_degree]
    sh = (rng.standard_normal((n, K, 3), dtype=np.float32) * np.float32(spec.sh_sd))
    return pos, log_s, quat, op, sh


def city_tree(spec: CitySpec) -> Tree:
    pos, log_s, quat, op, sh = city_leaves(spec)
    return lod_tree_from_leaves(pos, log_s, quat, op, sh, sh_degree=spec.sh_degree)


def random_tree(seed: int, n_roots: int = 2, max_depth: int = 4, max_children: int = 8,
                p_leaf: float = 0.25, extent: float = 10.0, sh_degree: int = 0) -> Tree:
    """Small random forest with leaves at varying depths (test input).

    Node attributes are independent draws whose scale shrinks with depth, so
    a child may be larger than its parent; positions stay near the parent's.
    """
    rng = np.random.default_rng(seed)
    levels = [[(-1, rng.uniform(-extent, extent, 3)) for _ in range(n_roots)]]
    leafmask = []
    while True:
        cur = levels[-1]
        depth = len(levels) - 1
        nxt = []
        lm = []
        for i, (_, p) in enumerate(cur):
            if depth >= max_depth or (depth > 0 and rng.random() < p_leaf):
                lm.append(True)
                continue
            k = int(rng.integers(1, max_children + 1))
            lm.append(False)
            spread = extent * 0.5 ** (depth + 1)
            for _ in range(k):
                nxt.append((i, p + rng.normal(0.0, spread, 3)))
        leafmask.append(lm)
        if not nxt:
            break
        levels.append(nxt)
    sizes = [len(l) for l in levels]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    N = int(offs[-1])
    parent = np.full(N, -1, np.int32)
    flags = np.zeros(N, np.uint8)
    pos = np.zeros((N, 3))
    for d, lv in enumerate(levels):
        for j, (pi, p) in enumerate(lv):
            idx = offs[d] + j
            if d > 0:
                parent[idx] = offs[d - 1] + pi
            flags[idx] = np.uint8((d << 1) | (1 if leafmask[d][j] else 0))
            pos[idx] = p
    depth = (flags >> 1).astype(np.float64)
    log_s = rng.normal(0.0, 0.6, (N, 3)) + (np.log(extent) - 1.0 - 0.69 * depth)[:, None]
    quat = _unit_quats(rng, N)
    op = _sigmoid(rng.normal(0.0, 1.0, N))
    K = SH_COEFFS[sh_degree]
    sh = rng.normal(0.0, 0.3, (N, K, 3)).astype(np.float32)
    internal = np.nonzero((flags & 1) == 0)[0]
    span = int(internal.max()) + 1 if internal.size else 0
    return Tree(mean=pos.T.astype(np.float32).copy(), scale=np.exp(log_s).T.astype(np.float32).copy(),
                quat=quat.T.astype(np.float32).copy(), opacity=op.astype(np.float32), sh=sh,
                parent=parent, flags=flags, sh_degree=sh_degree, n_internal_span=span,
                max_depth=len(levels) - 1, level_sizes=sizes)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    """Pinhole camera, world->camera x_c = R x_w + t, OpenCV axes (x right, y down, z forward).

    kx, ky bound the frustum test |x_c| <= kx z_c, |y_c| <= ky z_c: a guard band
    of ``guard`` times the half image extent.
    """
    R: np.ndarray          # f32 [9] row-major
    t: np.ndarray          # f32 [3]
    campos: np.ndarray     # f32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2
    kx: float = 0.0
    ky: float = 0.0
    tile_base: int = 0

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def n_tiles(self) -> int:
        return self.tiles_x * self.tiles_y


def make_camera(rot: np.ndarray, campos: Sequence[float], width: int, height: int,
                fov_x_deg: float = 60.0, znear: float = 0.2, guard: float = 1.3, tile_base: int = 0) -> Camera:
    rot = np.asarray(rot, np.float64)
    c = np.asarray(campos, np.float64)
    t = -rot @ c
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    fy = fx
    f32 = np.float32
    return Camera(R=rot.reshape(9).astype(np.float32), t=t.astype(np.float32), campos=c.astype(np.float32),
                  fx=float(f32(fx)), fy=float(f32(fy)), cx=float(f32(width / 2.0)), cy=float(f32(height / 2.0)),
                  width=int(width), height=int(height), znear=float(f32(znear)),
                  kx=float(f32(guard * (width / 2.0) / fx)), ky=float(f32(guard * (height / 2.0) / fy)),
                  tile_base=int(tile_base))


def yaw_pitch_rotation(yaw: float, pitch: float) -> np.ndarray:
    """World (x east, y north, z up) -> camera rows (right, down, forward); radians."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    d = np.cross(f, r)
    return np.stack([r, d, f])


def tiny_camera(distance: float = 25.0, width: int = 256, height: int = 256) -> Camera:
    """Camera at (0, 0, -distance) looking at the origin (R = I), 60 deg horizontal FOV."""
    return make_camera(np.eye(3), (0.0, 0.0, -distance), width, height)


def catmull_rom_closed(ctrl: np.ndarray, s: np.ndarray):
    """Position and tangent on a closed uniform Catmull-Rom spline, s in [0, len(ctrl))."""
    k = ctrl.shape[0]
    i = np.floor(s).astype(np.int64)
    u = (s - i)[:, None]
    p0, p1, p2, p3 = (ctrl[(i + o) % k] for o in (-1, 0, 1, 2))
    pos = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u ** 2
                 + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
    tan = 0.5 * ((-p0 + p2) + 2 * (2 * p0 - 5 * p1 + 4 * p2 - p3) * u + 3 * (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 2)
    return pos, tan


def flythrough(n_frames: int, seed: int = 1, n_ctrl: int = 8, half_extent: float = 240.0,
               altitude: float = 40.0, pitch_deg: float = -30.0, width: int = 1920, height: int = 1080,
               yaw_jitter_deg: float = 0.0, params: Optional[np.ndarray] = None,
               resolutions: Optional[Sequence] = None) -> List[Camera]:
    """Cameras on a closed seeded Catmull-Rom spline at fixed altitude, yaw along the tangent."""
    rng = np.random.default_rng(seed)
    ctrl = np.concatenate([rng.uniform(-half_extent, half_extent, (n_ctrl, 2)), np.full((n_ctrl, 1), altitude)], 1)
    s = np.arange(n_frames) * (n_ctrl / n_frames) if params is None else np.asarray(params, np.float64)
    pos, tan = catmull_rom_closed(ctrl, s)
    jit = rng.uniform(-yaw_jitter_deg, yaw_jitter_deg, n_frames) if yaw_jitter_deg > 0 else np.zeros(n_frames)
    res = None
    if resolutions is not None:
        res = [resolutions[int(j)] for j in rng.integers(0, len(resolutions), n_frames)]
    cams = []
    base = 0
    for f in range(n_frames):
        yaw = math.atan2(tan[f, 1], tan[f, 0]) + math.radians(jit[f])
        w, h = (width, height) if res is None else res[f]
        cam = make_camera(yaw_pitch_rotation(yaw, math.radians(pitch_deg)), pos[f], w, h, tile_base=base)
        if res is not None:
            base += cam.n_tiles
        cams.append(cam)
    return cams


@dataclasses.dataclass
class TopDownSpec:
    """A tree built top-down by the canonical recursive construction of
    Sec. 3.1: every parent v places 8 children at mu_v + R(q_v) o_k, o_k the
    eight sign combinations of (s_x/2, s_y/2, s_z/2) of the parent's scale;
    each child's scale is gamma * s_v, and its rotation, colour and opacity are
    the parent's."""
    n_roots: int
    depth: int                     # levels below the roots; leaves at this depth
    box: Sequence[float]           # root centres: x, y uniform in [-h, h], z uniform in [0, z_max]
    root_scale: Sequence[float]    # (s_x, s_y, s_z) of every root, world units
    gamma: float = 0.5
    logit_mu: float = 0.0
    logit_sd: float = 1.5
    sh_degree: int = 3
    sh_sd: float = 0.3
    seed: int = 0


def topdown_tree(spec: TopDownSpec) -> Tree:
    """Level order, the 8 children of a node contiguous (in sign order) in the
    next level. Roots: seeded centres in the box, rotations about the vertical
    axis only (uniform yaw), opacity sigmoid(N(logit_mu, logit_sd)), SH
    coefficients N(0, sh_sd)."""
    rng = np.random.default_rng(spec.seed)
    R0 = spec.n_roots
    hx, hy, zmax = spec.box
    mean = np.stack([rng.uniform(-hx, hx, R0), rng.uniform(-hy, hy, R0), rng.uniform(0.0, zmax, R0)], 1)
    yaw = rng.uniform(-math.pi, math.pi, R0)
    quat = np.stack([np.cos(yaw / 2), np.zeros(R0), np.zeros(R0), np.sin(yaw / 2)], 1)  # (w, x, y, z)
    rot = Rotation.from_quat(quat[:, [1, 2, 3, 0]]).as_matrix()                      # [R0, 3, 3]
    scale = np.tile(np.asarray(spec.root_scale, np.float64), (R0, 1))
    op = _sigmoid(rng.normal(spec.logit_mu, spec.logit_sd, R0))
    K = SH_COEFFS[spec.sh_degree]
    sh = rng.normal(0.0, spec.sh_sd, (R0, K, 3))
    signs = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float64)  # [8, 3]
    # R(q_v) o_k for a root's own scale; a node at level l has scale gamma^l s_root
    # and its root's rotation, so its children's offsets are gamma^l times these
    root_off = np.einsum("rij,rkj->rki", rot, signs[None, :, :] * (scale[:, None, :] / 2.0))  # [R0, 8, 3]
    levels = [(mean, scale, np.arange(R0), np.full(R0, -1, np.int64))]  # (means, scales, root id, parent)
    offs = [0, R0]
    for lvl in range(spec.depth):
        pm, ps, proot, _ = levels[-1]
        m = pm.shape[0]
        cm = pm[:, None, :] + (spec.gamma ** lvl) * root_off[proot]         # mu_v + R(q_v) o_k
        cs = np.repeat(ps * spec.gamma, 8, axis=0)
        croot = np.repeat(proot, 8)
        par = offs[-2] + np.repeat(np.arange(m), 8)
        levels.append((cm.reshape(-1, 3), cs, croot, par))
        offs.append(offs[-1] + 8 * m)
    N = offs[-1]
    mean_all = np.concatenate([l[0] for l in levels], 0)
    scale_all = np.concatenate([l[1] for l in levels], 0)
    root_all = np.concatenate([l[2] for l in levels], 0)
    parent = np.concatenate([l[3] for l in levels], 0).astype(np.int32)
    depth = np.concatenate([np.full(l[0].shape[0], d, np.uint8) for d, l in enumerate(levels)])
    flags = ((depth == spec.depth).astype(np.uint8) | (depth << 1)).astype(np.uint8)
    sizes = [int(l[0].shape[0]) for l in levels]
    return Tree(mean=mean_all.T.astype(np.float32).copy(), scale=scale_all.T.astype(np.float32).copy(),
                quat=quat.astype(np.float32).T.copy()[:, root_all], opacity=op.astype(np.float32)[root_all],
                sh=sh.astype(np.float32)[root_all], parent=parent, flags=flags, sh_degree=spec.sh_degree,
                n_internal_span=int(offs[-2]), max_depth=spec.depth, level_sizes=sizes)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
# Leaves of the city trees lie on thin horizontal patches (blob sigma_z =
# 2 cm) at ~290 leaves/m^2, leaf log-scale N(-3.5, 0.5): at 1080p with
# tau_R = 3 px, parents of such leaves pass the radius test beyond ~150 m and
# coarser levels beyond ~300-800 m, so cuts span several levels. Volumetric
# blobs (sigma = 18, 18, 10 m) would make every cut all-leaves at tau_R = 3.
CITY1M = CitySpec(n_leaves=1_000_000, box=(100.0, 100.0, 30.0), n_blobs=64, blob_sigma=(3.0, 3.0, 0.02),
                  leaf_log_scale_mu=-3.5, seed=0)
CITY20M = CitySpec(n_leaves=17_500_000, box=(300.0, 300.0, 50.0), n_blobs=256, blob_sigma=(6.0, 6.0, 0.02),
                   leaf_log_scale_mu=-3.5, seed=0)
# The canonical top-down construction (Sec. 3.1) on the city's footprint:
# 32768 flat roots of 0.7 m half-extent, three levels of 8 children (19.2M
# nodes), leaves 9 cm across, opacity logits N(2.5, 0.5) inherited down each
# tree. The construction stacks children at +-s_z/2, so every level doubles
# the coincident layers: the scene is congested by design, its GTC is low and
# its threshold tau (Eq. (8)) high. With tau_R = 3 px the fly-through's cuts
# keep leaves near the camera and their parents farther away.
TOPDOWN20M = TopDownSpec(n_roots=32768, depth=3, box=(240.0, 240.0, 10.0), root_scale=(0.7, 0.7, 0.05),
                         logit_mu=2.5, logit_sd=0.5, seed=0)
CITY_PITCH_DEG = -20.0
CITY_ALTITUDE = 40.0
LAMBDA_G = 0.2   # Sec. 4.1: shrink aggressiveness used in all experiments
TAU_R = 3.0      # Sec. 3.2: R&L pixel-radius threshold


def city1m_camera() -> Camera:
    """One 1920x1080 view from (0, -120, 30) facing +y, tilted down 30 degrees."""
    return make_camera(yaw_pitch_rotation(math.pi / 2, math.radians(-30.0)), (0.0, -120.0, 30.0), 1920, 1080)


def city20m_frames(n_frames: int = 64) -> List[Camera]:
    """The 64-frame 1080p fly-through at 40 m altitude (closed spline, seed 1)."""
    return flythrough(n_frames, seed=1, altitude=CITY_ALTITUDE, pitch_deg=CITY_PITCH_DEG)


def city20m_training_views(n: int = 8) -> List[Camera]:
    """Views for the GTC pre-pass: the same path, half-way between the frames' spline knots."""
    return flythrough(n, seed=1, altitude=CITY_ALTITUDE, pitch_deg=CITY_PITCH_DEG,
                      params=(np.arange(n) + 0.5) * (8.0 / n))


def city20m_batch_views(n: int = 32) -> List[Camera]:
    """32 views on the path with +-15 deg yaw jitter and mixed resolutions (global tile ids)."""
    res = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
    return flythrough(n, seed=1, altitude=CITY_ALTITUDE, pitch_deg=CITY_PITCH_DEG, yaw_jitter_deg=15.0,
                      params=np.arange(n) * (8.0 / n), resolutions=res)


# --------------------------------------------------------------------------
# differentiable workload: raw Gaussian parameters
# --------------------------------------------------------------------------
@dataclasses.dataclass
class RawGaussians:
    mean: np.ndarray       # f32 [3, M]
    log_scale: np.ndarray  # f32 [3, M]
    quat: np.ndarray       # f32 [4, M]
    logit: np.ndarray      # f32 [M]
    sh: np.ndarray         # f32 [M, K, 3]
    sh_degree: int


def flat_gaussians(n: int = 2_000_000, seed: int = 0) -> RawGaussians:
    """n Gaussians with the city1m leaf law (thin blobs, log-scale N(-3.5, 0.5),
    logits N(0, 1.5), SH degree 3 N(0, 0.3)), kept where their centre projects
    into the city1m camera's image (drawn 3x over in the ground region that view
    sees, x in [-80, 80], y in [-95, 25], z in [0, 8]; the first n kept in
    Morton order), so all n are rendered by that view."""
    spec = CitySpec(n_leaves=3 * n, box=(80.0, 60.0, 8.0), n_blobs=256, blob_sigma=(3.0, 3.0, 0.02),
                    leaf_log_scale_mu=-3.5, seed=seed)
    pos, log_s, quat, op, sh = city_leaves(spec)
    pos[:, 1] -= 35.0
    cam = city1m_camera()
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    pc = pos @ R.T + np.asarray(cam.t, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.fx * pc[:, 0] / pc[:, 2] + cam.cx
        v = cam.fy * pc[:, 1] / pc[:, 2] + cam.cy
    keep = np.nonzero((pc[:, 2] > 1.0) & (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height))[0][:n]
    if keep.size < n:
        raise ValueError("too few candidate Gaussians in view")
    logit = np.log(op[keep]) - np.log1p(-op[keep])
    return RawGaussians(mean=pos[keep].T.astype(np.float32).copy(), log_scale=log_s[keep].T.astype(np.float32).copy(),
                        quat=quat[keep].T.astype(np.float32).copy(), logit=logit.astype(np.float32),
                        sh=np.ascontiguousarray(sh[keep]), sh_degree=spec.sh_degree)


def city1m_yaw_views(yaws_deg=(-14, -10, -6, -2, 2, 6, 10, 14)) -> List[Camera]:
    """The city1m view turned by each yaw offset (a batch of 8 views)."""
    return [make_camera(yaw_pitch_rotation(math.pi / 2 + math.radians(d), math.radians(-30.0)), (0.0, -120.0, 30.0),
                        1920, 1080) for d in yaws_deg]
