"""CPU oracle of the FilterGS per-frame path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. The product path (the HIP
library ``libfg.so`` and its Python binding) never imports it, and the two
share no code: this package wraps ``fg_oracle.c``, a plain C implementation
written from the paper (see the header of that file), single-threaded by
default; ``set_threads(n)`` switches to the OpenMP build of the same source,
used only to time the oracle on all host cores (results are bit-identical).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")  # same source with -fopenmp: for timing on all cores

_libs = {}
_threads = None  # None: the plain single-threaded build; n: the OpenMP build with n threads


def build() -> str:
    """Compile the oracle with IEEE binary32 semantics (no contraction, no fast
    math): the plain build the tests use, and an OpenMP build of the same
    source for the benchmark's timing (bit-identical results)."""
    base = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
            "-fno-finite-math-only", "-Wall"]
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        subprocess.run(base + extra + ["-o", out + ".tmp", SRC, "-lm"], check=True)
        os.replace(out + ".tmp", out)
    return LIB


def set_threads(n=None) -> int:
    """n = None: the plain single-threaded oracle (the default); n >= 1: the
    OpenMP build with n threads. Returns the thread count in use."""
    global _threads
    _threads = n
    L = lib()
    return int(L.fgo_set_threads(int(n))) if n is not None else 1


class _Tree(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("pad", C.c_int32),
                ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("sh", C.c_void_p), ("parent", C.c_void_p), ("flags", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_float), ("kx", C.c_float),
                ("ky", C.c_float), ("tile_base", C.c_uint32)]


SPLAT_DTYPE = np.dtype([("u", "<f4"), ("v", "<f4"), ("A", "<f4"), ("B", "<f4"), ("C", "<f4"),
                        ("opacity", "<f4"), ("r", "<f4"), ("g", "<f4"), ("b", "<f4"), ("depth", "<f4"),
                        ("lam", "<f4"), ("radius", "<f4"), ("x0", "<i4"), ("y0", "<i4"), ("x1", "<i4"),
                        ("y1", "<i4"), ("tiles", "<u4")])


def lib():
    path = LIB if _threads is None else LIB_OMP
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(path)
        vp, i64, f32 = C.c_void_p, C.c_int64, C.c_float
        L.fgo_exp.restype = f32; L.fgo_exp.argtypes = [f32]
        L.fgo_log.restype = f32; L.fgo_log.argtypes = [f32]
        L.fgo_exp_array.argtypes = [vp, vp, i64]
        L.fgo_log_array.argtypes = [vp, vp, i64]
        L.fgo_node_predicates.argtypes = [vp, vp, f32, vp]
        L.fgo_filter.restype = i64; L.fgo_filter.argtypes = [vp, vp, f32, vp, vp]
        L.fgo_filter_nodes.argtypes = [vp, vp, f32, vp, i64, vp]
        L.fgo_sh_basis.argtypes = [C.c_int, f32, f32, f32, vp]
        L.fgo_preprocess.argtypes = [vp, vp, f32, vp, i64, vp]
        L.fgo_count_pairs.restype = i64; L.fgo_count_pairs.argtypes = [vp, i64]
        L.fgo_sort.argtypes = [vp, i64, vp, vp, vp, vp]
        L.fgo_render.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.fgo_render_pixels.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, vp, vp, vp]
        L.fgo_kpc.argtypes = [vp, vp, vp, vp, vp]
        L.fgo_activate.argtypes = [vp, vp, i64, vp, vp]
        L.fgo_replay64.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fgo_set_threads.restype = C.c_int; L.fgo_set_threads.argtypes = [C.c_int]
        assert L.fgo_splat_size() == SPLAT_DTYPE.itemsize
        _libs[path] = L
    return _libs[path]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class TreeRef:
    """ctypes view of a synth.Tree (keeps the contiguous arrays alive)."""

    def __init__(self, tree):
        self.keep = [np.ascontiguousarray(tree.mean, np.float32), np.ascontiguousarray(tree.scale, np.float32),
                     np.ascontiguousarray(tree.quat, np.float32), np.ascontiguousarray(tree.opacity, np.float32),
                     np.ascontiguousarray(tree.sh, np.float32), np.ascontiguousarray(tree.parent, np.int32),
                     np.ascontiguousarray(tree.flags, np.uint8)]
        m, s, q, o, sh, p, f = self.keep
        self.s = _Tree(n=tree.n_nodes, sh_degree=tree.sh_degree, pad=0, mean=m.ctypes.data, scale=s.ctypes.data,
                       quat=q.ctypes.data, opacity=o.ctypes.data, sh=sh.ctypes.data, parent=p.ctypes.data,
                       flags=f.ctypes.data)
        self.n = tree.n_nodes

    @property
    def ptr(self):
        return C.cast(C.pointer(self.s), C.c_void_p)


def camera_struct(cam) -> _Camera:
    c = _Camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32)]
    c.campos[:] = [float(x) for x in np.asarray(cam.campos, np.float32)]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height = cam.width, cam.height
    c.znear, c.kx, c.ky = cam.znear, cam.kx, cam.ky
    c.tile_base = cam.tile_base
    return c


def _cam_ptr(cam):
    cs = camera_struct(cam)
    return cs, C.cast(C.pointer(cs), C.c_void_p)


def _tree_ref(tree):
    return tree if isinstance(tree, TreeRef) else TreeRef(tree)


# ---------------------------------------------------------------------------
def exp(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().fgo_exp_array(_ptr(x), _ptr(y), x.size)
    return y


def log(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().fgo_log_array(_ptr(x), _ptr(y), x.size)
    return y


def sh_basis(degree: int, d) -> np.ndarray:
    d = np.asarray(d, np.float32).reshape(-1, 3)
    out = np.zeros((d.shape[0], 16), np.float32)
    Y = np.zeros(16, np.float32)
    for i in range(d.shape[0]):
        lib().fgo_sh_basis(degree, float(d[i, 0]), float(d[i, 1]), float(d[i, 2]), _ptr(Y))
        out[i] = Y
    return out[:, : (degree + 1) ** 2]


def node_predicates(tree, cam, tau_R: float) -> np.ndarray:
    """Per node: bit0 in frustum, bit1 small, bit2 passes R&L, bit3 selected."""
    t = _tree_ref(tree)
    cs, cp = _cam_ptr(cam)
    out = np.zeros(t.n, np.uint8)
    lib().fgo_node_predicates(t.ptr, cp, C.c_float(tau_R), _ptr(out))
    return out


def filter(tree, cam, tau_R: float):
    """Returns (selection mask u8[N], selected node ids u32 ascending)."""
    t = _tree_ref(tree)
    cs, cp = _cam_ptr(cam)
    mask = np.zeros(t.n, np.uint8)
    idx = np.zeros(max(t.n, 1), np.uint32)
    k = lib().fgo_filter(t.ptr, cp, C.c_float(tau_R), _ptr(mask), _ptr(idx))
    return mask, idx[:k].copy()


def filter_nodes(tree, cam, tau_R: float, nodes) -> np.ndarray:
    t = _tree_ref(tree)
    cs, cp = _cam_ptr(cam)
    nodes = np.ascontiguousarray(nodes, np.int64)
    out = np.zeros(nodes.size, np.uint8)
    lib().fgo_filter_nodes(t.ptr, cp, C.c_float(tau_R), _ptr(nodes), nodes.size, _ptr(out))
    return out


def preprocess(tree, cam, tau: float, sel_idx) -> np.ndarray:
    t = _tree_ref(tree)
    cs, cp = _cam_ptr(cam)
    sel_idx = np.ascontiguousarray(sel_idx, np.uint32)
    out = np.zeros(sel_idx.size, SPLAT_DTYPE)
    lib().fgo_preprocess(t.ptr, cp, C.c_float(tau), _ptr(sel_idx), sel_idx.size, _ptr(out))
    return out


def sort(splats: np.ndarray, cam):
    """Returns (keys u64[n_pairs], vals u32[n_pairs], ranges u32[n_tiles, 2])."""
    splats = np.ascontiguousarray(splats)
    cs, cp = _cam_ptr(cam)
    n_pairs = lib().fgo_count_pairs(_ptr(splats), splats.size)
    keys = np.zeros(max(n_pairs, 1), np.uint64)
    vals = np.zeros(max(n_pairs, 1), np.uint32)
    ranges = np.zeros((cam.n_tiles, 2), np.uint32)
    lib().fgo_sort(_ptr(splats), splats.size, cp, _ptr(keys), _ptr(vals), _ptr(ranges))
    return keys[:n_pairs].copy(), vals[:n_pairs].copy(), ranges


def render(splats, vals, ranges, cam, bg=(0.0, 0.0, 0.0)):
    """Returns (image f32[3,H,W], final_T f32[H,W], n_contrib u32[H,W])."""
    splats = np.ascontiguousarray(splats)
    vals = np.ascontiguousarray(vals, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    cs, cp = _cam_ptr(cam)
    bgv = np.asarray(bg, np.float32)
    H, W = cam.height, cam.width
    img = np.zeros((3, H, W), np.float32)
    T = np.zeros((H, W), np.float32)
    nc = np.zeros((H, W), np.uint32)
    lib().fgo_render(_ptr(splats), _ptr(vals if vals.size else np.zeros(1, np.uint32)), _ptr(ranges), cp,
                     _ptr(bgv), _ptr(img), _ptr(T), _ptr(nc))
    return img, T, nc


def render_pixels(splats, vals, ranges, cam, px, py, bg=(0.0, 0.0, 0.0)):
    splats = np.ascontiguousarray(splats)
    vals = np.ascontiguousarray(vals, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    cs, cp = _cam_ptr(cam)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    bgv = np.asarray(bg, np.float32)
    m = px.size
    rgb = np.zeros((m, 3), np.float32)
    T = np.zeros(m, np.float32)
    nc = np.zeros(m, np.uint32)
    lib().fgo_render_pixels(_ptr(splats), _ptr(vals if vals.size else np.zeros(1, np.uint32)), _ptr(ranges), cp,
                            _ptr(bgv), _ptr(px), _ptr(py), m, _ptr(rgb), _ptr(T), _ptr(nc))
    return rgb, T, nc


def render_frame(tree, cam, tau_R: float = 3.0, tau: float = 0.0, bg=(0.0, 0.0, 0.0)) -> dict:
    """All stages of one frame."""
    t = _tree_ref(tree)
    mask, sel = filter(t, cam, tau_R)
    splats = preprocess(t, cam, tau, sel)
    keys, vals, ranges = sort(splats, cam)
    img, T, nc = render(splats, vals, ranges, cam, bg)
    return dict(sel_mask=mask, sel_idx=sel, splats=splats, keys=keys, vals=vals, ranges=ranges, image=img,
                final_T=T, n_contrib=nc)


def kpc(splats, vals, ranges, cam) -> np.ndarray:
    """Key-value pair contribution (Eq. (5)) of every sorted pair, float64."""
    splats = np.ascontiguousarray(splats)
    vals = np.ascontiguousarray(vals, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    cs, cp = _cam_ptr(cam)
    out = np.zeros(max(vals.size, 1), np.float64)
    lib().fgo_kpc(_ptr(splats), _ptr(vals if vals.size else np.zeros(1, np.uint32)), _ptr(ranges), cp, _ptr(out))
    return out[: vals.size]


def tile_gtc(kpc_pairs, ranges) -> np.ndarray:
    """Tile GTC (Eq. (6)): for every tile, the mean KPC over all of its pairs,
    pairs with zero contribution included; NaN for a tile without pairs (0/0,
    which the paper leaves undefined)."""
    ranges = np.asarray(ranges).reshape(-1, 2).astype(np.int64)
    out = np.full(ranges.shape[0], np.nan)
    for t, (lo, hi) in enumerate(ranges):
        if hi > lo:
            out[t] = kpc_pairs[lo:hi].sum() / (hi - lo)
    return out


def gtc_view(kpc_pairs, ranges):
    """View GTC (Eq. (7)): mean of the tile GTCs over the tiles that hold
    pairs. None for a view without pairs (undefined; such a view is left out
    of the scene mean)."""
    g = tile_gtc(kpc_pairs, ranges)
    g = g[~np.isnan(g)]
    return float(g.mean()) if g.size else None


def scene_tau(tree, cams, lambda_G: float = 0.2, tau_R: float = 3.0) -> dict:
    """Eq. (8): G_bar = mean of the view GTCs over the views that hold pairs
    (3-sigma extents, the filtered cut), tau = lambda_G / G_bar."""
    t = _tree_ref(tree)
    gv = []
    for cam in cams:
        _, sel = filter(t, cam, tau_R)
        sp = preprocess(t, cam, 0.0, sel)
        keys, vals, ranges = sort(sp, cam)
        gv.append(gtc_view(kpc(sp, vals, ranges, cam), ranges))
    defined = [g for g in gv if g is not None]
    if not defined:
        raise ValueError("no view holds a Gaussian-tile pair: G_bar is undefined")
    G = float(np.mean(defined))
    return dict(G_views=gv, G_bar=G, lambda_G=lambda_G, tau=lambda_G / G)


# ---------------------------------------------------------------------------
# differentiable form
# ---------------------------------------------------------------------------
class _Params(C.Structure):
    _fields_ = [("m", C.c_int64), ("sh_degree", C.c_int32), ("pad", C.c_int32), ("mean", C.c_void_p),
                ("log_scale", C.c_void_p), ("quat", C.c_void_p), ("logit", C.c_void_p), ("sh", C.c_void_p)]


class ParamsRef:
    """ctypes view of raw Gaussian parameters (mean [3,M], log_scale [3,M], quat [4,M], logit [M], sh [M,K,3])."""

    def __init__(self, mean, log_scale, quat, logit, sh, sh_degree):
        self.keep = [np.ascontiguousarray(a, np.float32) for a in (mean, log_scale, quat, logit, sh)]
        m, ls, q, lg, s = self.keep
        self.m = int(lg.shape[0])
        self.s = _Params(m=self.m, sh_degree=sh_degree, pad=0, mean=m.ctypes.data, log_scale=ls.ctypes.data,
                         quat=q.ctypes.data, logit=lg.ctypes.data, sh=s.ctypes.data)
        self.sh_degree = sh_degree

    @property
    def ptr(self):
        return C.cast(C.pointer(self.s), C.c_void_p)


def activate(log_scale, logit):
    """float32 scale = exp(log_scale), opacity = sigmoid(logit) with the project's exponential."""
    ls = np.ascontiguousarray(log_scale, np.float32)
    lg = np.ascontiguousarray(logit, np.float32)
    sc = np.empty_like(ls)
    op = np.empty_like(lg)
    lib().fgo_activate(_ptr(ls), _ptr(lg), lg.size, _ptr(sc), _ptr(op))
    return sc, op


def flat_tree_from_params(prm: ParamsRef):
    """A tree whose nodes are the activated Gaussians, every one a root leaf."""
    from types import SimpleNamespace
    mean, log_scale, quat, logit, sh = prm.keep
    sc, op = activate(log_scale, logit)
    m = prm.m
    return SimpleNamespace(mean=mean, scale=sc, quat=quat, opacity=op, sh=sh, parent=np.full(m, -1, np.int32),
                           flags=np.ones(m, np.uint8), sh_degree=prm.sh_degree, n_internal_span=0, max_depth=0,
                           n_nodes=m)


def forward32(prm: ParamsRef, cam, tau: float = 0.0, bg=(0.0, 0.0, 0.0)) -> dict:
    """The float32 frame of the activated Gaussians (all are root leaves)."""
    return render_frame(flat_tree_from_params(prm), cam, 1e30, tau, bg)


def replay64(prm: ParamsRef, cam, fwd: dict, dL_dimage=None, bg=(0.0, 0.0, 0.0), want_image=True):
    """float64 replay of the float32 forward's decisions: image and gradients."""
    cs, cp = _cam_ptr(cam)
    H, W = cam.height, cam.width
    bgv = np.asarray(bg, np.float32)
    sel = np.ascontiguousarray(fwd["sel_idx"], np.uint32)
    splats = np.ascontiguousarray(fwd["splats"])
    vals = np.ascontiguousarray(fwd["vals"], np.uint32)
    ranges = np.ascontiguousarray(fwd["ranges"], np.uint32)
    nc = np.ascontiguousarray(fwd["n_contrib"], np.uint32)
    img = np.zeros((3, H, W), np.float64) if want_image else None
    m, K = prm.m, (prm.sh_degree + 1) ** 2
    grads = None
    dl = None
    if dL_dimage is not None:
        dl = np.ascontiguousarray(dL_dimage, np.float64)
        grads = dict(mean=np.zeros((3, m)), log_scale=np.zeros((3, m)), quat=np.zeros((4, m)), logit=np.zeros(m),
                     sh=np.zeros((m, K, 3)))
    z = lambda a: None if a is None else _ptr(a)
    one = np.zeros(1, np.uint32)
    lib().fgo_replay64(prm.ptr, cp, _ptr(bgv), _ptr(sel if sel.size else one), sel.size, _ptr(splats),
                       _ptr(vals if vals.size else one), _ptr(ranges), _ptr(nc), z(dl), z(img),
                       *(z(grads[k]) if grads else None for k in ("mean", "log_scale", "quat", "logit", "sh")))
    return img, grads
