"""Python binding of libfg.so (include/fg.h): argument marshalling only.

Every entry point of the C-ABI has a function of the same name here that
takes torch CUDA tensors, passes their device pointers and the stream of
torch's current stream, and raises ``FgError`` on a negative return code.
All computation happens in the HIP kernels; this module never computes any
part of the frame itself and has no CPU fallback: without the built library
it raises.

``DeviceTree`` uploads a tree; ``FrameBuffers`` owns the buffers of one view
and ``render_frame`` chains the four stages.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfg.so")

FG_STATUS_SEL_OVERFLOW = 1
FG_STATUS_PAIR_OVERFLOW = 2
FG_STATUS_BAD_PARENT = 4
FG_STATUS_GTC_UNDEFINED = 8
FG_STATUS_ITEM_OVERFLOW = 16


class FgError(RuntimeError):
    pass


class FgTree(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_internal_span", C.c_int64), ("sh_degree", C.c_int32),
                ("max_depth", C.c_int32), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("parent", C.c_void_p), ("flags", C.c_void_p),
                ("tile_box", C.c_void_p)]


class FgCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("znear", C.c_float), ("kx", C.c_float), ("ky", C.c_float),
                ("tile_base", C.c_uint32)]


class FgSplats(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("conic_o", C.c_void_p), ("rgb_depth", C.c_void_p), ("rect", C.c_void_p),
                ("tiles", C.c_void_p)]


class FgParams(C.Structure):
    _fields_ = [("m", C.c_int64), ("sh_degree", C.c_int32), ("pad", C.c_int32), ("mean", C.c_void_p),
                ("log_scale", C.c_void_p), ("quat", C.c_void_p), ("logit", C.c_void_p), ("sh", C.c_void_p)]


class FgGrads(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p), ("logit", C.c_void_p),
                ("sh", C.c_void_p)]


class FgLevelwiseStats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("pad", C.c_int32), ("visited", C.c_int64), ("calc_ms", C.c_double),
                ("wall_ms", C.c_double)]


class FgTune(C.Structure):
    _fields_ = [("render_batch", C.c_int32), ("radix_bits", C.c_int32), ("save_state", C.c_int32),
                ("mask_items", C.c_int32), ("blend_events", C.c_void_p * 2), ("bwd_stats", C.c_void_p)]


EXPORTS = ["fg_tree_box_floats", "fg_tree_boxes", "fg_filter_workspace_size", "fg_filter", "fg_filter_noalloc",
           "fg_children_workspace_size",
           "fg_children", "fg_filter_levelwise_workspace_size", "fg_filter_levelwise", "fg_preprocess", "fg_sort_workspace_size", "fg_sort",
           "fg_render_workspace_size", "fg_render", "fg_gtc", "fg_gtc_tau", "fg_activate", "fg_render_backward_workspace_size",
           "fg_render_backward", "fg_status_string"]

_lib = None


def lib():
    """Load libfg.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FgError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_23891_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, f32, i32 = C.c_void_p, C.c_int64, C.c_float, C.c_int
        L.fg_tree_box_floats.restype = i64
        L.fg_tree_box_floats.argtypes = [i64, i64]
        L.fg_tree_boxes.restype = i32
        L.fg_tree_boxes.argtypes = [vp, vp, vp]
        L.fg_filter_workspace_size.restype = C.c_size_t
        L.fg_filter_workspace_size.argtypes = [i64, i64, C.c_int32]
        L.fg_filter.restype = i32
        L.fg_filter.argtypes = [vp, vp, C.c_int32, vp, f32, vp, vp, i64, vp, vp, vp, C.c_size_t, vp]
        L.fg_filter_noalloc.restype = i32
        L.fg_filter_noalloc.argtypes = [vp, vp, C.c_int32, vp, f32, vp, vp, i64, vp, vp, vp]
        L.fg_children_workspace_size.restype = C.c_size_t
        L.fg_children_workspace_size.argtypes = [i64]
        L.fg_children.restype = i32
        L.fg_children.argtypes = [vp, i64, vp, vp, vp, vp, C.c_size_t, vp]
        L.fg_filter_levelwise_workspace_size.restype = C.c_size_t
        L.fg_filter_levelwise_workspace_size.argtypes = [i64]
        L.fg_filter_levelwise.restype = i32
        L.fg_filter_levelwise.argtypes = [vp, vp, vp, vp, f32, vp, vp, vp, vp, C.c_size_t, vp, vp]
        L.fg_preprocess.restype = i32
        L.fg_preprocess.argtypes = [vp, vp, vp, i64, vp, C.c_int32, vp, f32, vp, vp, vp]
        L.fg_sort_workspace_size.restype = C.c_size_t
        L.fg_sort_workspace_size.argtypes = [i64, C.c_int32, i64, i64]
        L.fg_sort.restype = i32
        L.fg_sort.argtypes = [vp, vp, i64, vp, C.c_int32, i64, vp, vp, i64, vp, vp, vp, vp, C.c_size_t, vp, vp]
        L.fg_render.restype = i32
        L.fg_render_workspace_size.restype = C.c_size_t
        L.fg_render_workspace_size.argtypes = [vp, C.c_int32, i64, vp]
        L.fg_render.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, i64, vp, vp, vp, C.c_size_t, vp, vp]
        L.fg_gtc.restype = i32
        L.fg_gtc.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, C.c_int32, vp, vp, vp, C.c_size_t, vp, vp]
        L.fg_gtc_tau.restype = i32
        L.fg_gtc_tau.argtypes = [vp, C.c_int32, f32, vp, vp, vp, vp]
        L.fg_activate.restype = i32
        L.fg_activate.argtypes = [vp, vp, vp, vp]
        L.fg_render_backward_workspace_size.restype = C.c_size_t
        L.fg_render_backward_workspace_size.argtypes = [i64]
        L.fg_render_backward.restype = i32
        L.fg_render_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, i64, vp,
                                         vp, vp, vp, C.c_size_t, vp]
        L.fg_status_string.restype = C.c_char_p
        L.fg_status_string.argtypes = [i32]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise FgError(f"{what}: {lib().fg_status_string(rc).decode()} ({rc})")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _ref(s):
    return C.cast(C.pointer(s), C.c_void_p)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def camera_array(cams):
    """A single camera or a sequence of cameras as a ctypes FgCamera array."""
    cams = list(cams) if isinstance(cams, (list, tuple)) else [cams]
    return (FgCamera * len(cams))(*[camera_struct(c) for c in cams]), len(cams)


def camera_struct(cam) -> FgCamera:
    c = FgCamera()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32)]
    c.campos[:] = [float(v) for v in np.asarray(cam.campos, np.float32)]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height = cam.width, cam.height
    c.znear, c.kx, c.ky = cam.znear, cam.kx, cam.ky
    c.tile_base = cam.tile_base
    return c


def tune_struct(render_batch: int = 0, radix_bits: int = 0, save_state: bool = False, blend_events=None,
                mask_items: int = 0, bwd_stats: Optional[torch.Tensor] = None) -> FgTune:
    """blend_events: None, or two recorded torch.cuda.Event (timing enabled)
    that fg_render records around its blend kernel. bwd_stats: None, or an
    int64 device tensor of at least 3 entries that fg_render_backward adds its
    counters to (atomic instructions, gradient elements, blended fragments)."""
    t = FgTune(render_batch=render_batch, radix_bits=radix_bits, save_state=1 if save_state else 0,
               mask_items=mask_items)
    if blend_events is not None:
        t.blend_events[0] = blend_events[0].cuda_event
        t.blend_events[1] = blend_events[1].cuda_event
    if bwd_stats is not None:
        if bwd_stats.dtype != torch.int64 or bwd_stats.numel() < 3 or not bwd_stats.is_cuda:
            raise ValueError("bwd_stats: an int64 device tensor of at least 3 entries")
        t.bwd_stats = bwd_stats.data_ptr()
    return t


# ---------------------------------------------------------------------------
# device-resident inputs and outputs
# ---------------------------------------------------------------------------
class DeviceTree:
    """A synth.Tree (or equivalent arrays) uploaded to the GPU as the fg_tree planes.
    boxes: also build the filter's per-block boxes (fg_tree_boxes), which let
    it skip blocks of nodes outside every view without changing any result;
    rebuild them (build_boxes) after changing mean or parent."""

    def __init__(self, tree, device="cuda", boxes: bool = True):
        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)

        self.mean = up(tree.mean.astype(np.float32), np.float32)
        self.scale = up(tree.scale.astype(np.float32), np.float32)
        self.quat = up(tree.quat.astype(np.float32), np.float32)
        self.opacity = up(tree.opacity.astype(np.float32), np.float32)
        self.sh = up(tree.sh.astype(np.float32), np.float32)
        self.parent = up(tree.parent.astype(np.int32), np.int32)
        self.flags = up(tree.flags.astype(np.uint8), np.uint8)
        self.n_nodes = int(tree.parent.shape[0])
        self.n_internal_span = int(tree.n_internal_span)
        self.sh_degree = int(tree.sh_degree)
        self.max_depth = int(tree.max_depth)
        self.tile_box = None
        if boxes:
            self.build_boxes()

    def build_boxes(self, stream=None):
        """(Re)writes the per-block boxes on the stream (default: current)."""
        n = int(lib().fg_tree_box_floats(self.n_nodes, self.n_internal_span))
        if n < 0:
            raise FgError("fg_tree_box_floats: invalid node count")
        box = torch.empty(max(n, 8), dtype=torch.float32, device=self.mean.device)
        self.tile_box = None
        ts = self.struct()
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().fg_tree_boxes(C.byref(ts), C.c_void_p(box.data_ptr()), C.c_void_p(s.cuda_stream)),
               "fg_tree_boxes")
        self.tile_box = box

    def struct(self) -> FgTree:
        return FgTree(n_nodes=self.n_nodes, n_internal_span=self.n_internal_span, sh_degree=self.sh_degree,
                      max_depth=self.max_depth, mean=self.mean.data_ptr(), scale=self.scale.data_ptr(),
                      quat=self.quat.data_ptr(), opacity=self.opacity.data_ptr(), sh=self.sh.data_ptr(),
                      parent=self.parent.data_ptr(), flags=self.flags.data_ptr(),
                      tile_box=self.tile_box.data_ptr() if self.tile_box is not None else None)


class Splats:
    """Device planes of fg_splats with capacity cap."""

    def __init__(self, cap: int, device="cuda"):
        cap = max(int(cap), 1)
        self.cap = cap
        self.xy = torch.empty((cap, 2), dtype=torch.float32, device=device)
        self.conic_o = torch.empty((cap, 4), dtype=torch.float32, device=device)
        self.rgb_depth = torch.empty((cap, 4), dtype=torch.float32, device=device)
        self.rect = torch.empty((cap, 4), dtype=torch.int16, device=device)
        self.tiles = torch.empty((cap,), dtype=torch.int32, device=device)

    def struct(self) -> FgSplats:
        return FgSplats(xy=self.xy.data_ptr(), conic_o=self.conic_o.data_ptr(), rgb_depth=self.rgb_depth.data_ptr(),
                        rect=self.rect.data_ptr(), tiles=self.tiles.data_ptr())


# ---------------------------------------------------------------------------
# the C-ABI, one function per entry point
# ---------------------------------------------------------------------------
def fg_filter_workspace_size(n_nodes: int, n_internal_span: int, n_views: int = 1) -> int:
    return int(lib().fg_filter_workspace_size(n_nodes, n_internal_span, n_views))


def fg_sort_workspace_size(cap_sel: int, n_views: int, cap_items: int, cap_pairs: int) -> int:
    return int(lib().fg_sort_workspace_size(cap_sel, n_views, cap_items, cap_pairs))


def fg_filter(tree: DeviceTree, cams, tau_R: float, sel_bits, sel_idx, cap_sel: int, n_sel, status, ws,
              stream=None, cams_dev=None):
    """cams: one camera or a sequence of cameras (node-major multi-view filter);
    cams_dev: None or a device tensor holding the cameras' fg_camera records
    (their poses are read on the device)."""
    arr, n = camera_array(cams)
    ts = tree.struct()
    _check(lib().fg_filter(_ref(ts), C.cast(arr, C.c_void_p), n, _p(cams_dev), C.c_float(tau_R), _p(sel_bits),
                           _p(sel_idx), cap_sel, _p(n_sel), _p(status), _p(ws), ws.numel() * ws.element_size(),
                           _stream(stream)), "fg_filter")


def fg_filter_noalloc(tree: DeviceTree, cams, tau_R: float, sel_bits, sel_idx, cap_sel: int, n_sel, status,
                      stream=None, cams_dev=None):
    """fg_filter on the library's fixed per-device scratch array (no workspace argument)."""
    arr, n = camera_array(cams)
    ts = tree.struct()
    _check(lib().fg_filter_noalloc(_ref(ts), C.cast(arr, C.c_void_p), n, _p(cams_dev), C.c_float(tau_R),
                                   _p(sel_bits), _p(sel_idx), cap_sel, _p(n_sel), _p(status), _stream(stream)),
           "fg_filter_noalloc")


def fg_children(parent, n_nodes: int, child_offs, child_ids, status, ws, stream=None):
    _check(lib().fg_children(_p(parent), n_nodes, _p(child_offs), _p(child_ids), _p(status), _p(ws),
                             ws.numel() * ws.element_size(), _stream(stream)), "fg_children")


def fg_filter_levelwise(tree: DeviceTree, child_offs, child_ids, cam, tau_R: float, sel_bits, n_sel, status, ws,
                        stream=None) -> FgLevelwiseStats:
    ts, cs = tree.struct(), camera_struct(cam)
    st = FgLevelwiseStats()
    _check(lib().fg_filter_levelwise(_ref(ts), _p(child_offs), _p(child_ids), _ref(cs), C.c_float(tau_R),
                                     _p(sel_bits), _p(n_sel), _p(status), _p(ws), ws.numel() * ws.element_size(),
                                     _ref(st), _stream(stream)), "fg_filter_levelwise")
    return st


class TreeChildren:
    """Children of every node (CSR, built on the device by fg_children), for the
    serial level-wise filter; plus that filter's workspace."""

    def __init__(self, tree: DeviceTree, device="cuda"):
        N = tree.n_nodes
        self.offs = torch.empty(N + 2, dtype=torch.int32, device=device)
        self.ids = torch.empty(max(N, 1), dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        ws = torch.empty(lib().fg_children_workspace_size(N), dtype=torch.uint8, device=device)
        fg_children(tree.parent, N, self.offs, self.ids, self.status, ws)
        self.ws = torch.empty(lib().fg_filter_levelwise_workspace_size(N), dtype=torch.uint8, device=device)


def fg_preprocess(tree: DeviceTree, cams, tau: float, sel_idx, n_sel, cap_sel: int, out: Splats, status,
                  stream=None, cams_dev=None):
    arr, n = camera_array(cams)
    ts, ss = tree.struct(), out.struct()
    _check(lib().fg_preprocess(_ref(ts), _p(sel_idx), _p(n_sel), cap_sel, C.cast(arr, C.c_void_p), n, _p(cams_dev),
                               C.c_float(tau), _ref(ss), _p(status), _stream(stream)), "fg_preprocess")


def fg_sort(splats: Splats, n_sel, cap_sel: int, cams, tile_keys, vals, cap_pairs: int, n_pairs, ranges, status, ws,
            tune: Optional[FgTune] = None, stream=None, cap_items: Optional[int] = None):
    """cap_items: bound on the tile-covering splats of all views (default: cap_sel per view)."""
    arr, n = camera_array(cams)
    ss = splats.struct()
    cap_items = cap_sel * n if cap_items is None else cap_items
    _check(lib().fg_sort(_ref(ss), _p(n_sel), cap_sel, C.cast(arr, C.c_void_p), n, cap_items, _p(tile_keys),
                         _p(vals), cap_pairs, _p(n_pairs), _p(ranges), _p(status), _p(ws),
                         ws.numel() * ws.element_size(), _ref(tune) if tune is not None else None, _stream(stream)),
           "fg_sort")


def fg_render_workspace_size(cams, cap_pairs: int, tune: Optional[FgTune] = None) -> int:
    arr, n = camera_array(cams)
    return int(lib().fg_render_workspace_size(C.cast(arr, C.c_void_p), n, cap_pairs,
                                              _ref(tune) if tune is not None else None))


def fg_render(splats: Splats, vals, ranges, cams, bg: Sequence[float], image, final_T, n_contrib, cap_pairs: int,
              frag_stats, status, ws, tune: Optional[FgTune] = None, stream=None):
    arr, n = camera_array(cams)
    ss = splats.struct()
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    _check(lib().fg_render(_ref(ss), _p(vals), _p(ranges), C.cast(arr, C.c_void_p), n, C.cast(bgv, C.c_void_p),
                           _p(image), _p(final_T), _p(n_contrib), cap_pairs, _p(frag_stats), _p(status), _p(ws),
                           ws.numel() * ws.element_size(), _ref(tune) if tune is not None else None,
                           _stream(stream)), "fg_render")


def fg_gtc(splats: Splats, vals, ranges, cam, n_pairs, cap_pairs: int, kpc, tile_gtc, view_gtc, hist_edges=None,
           kpc_hist=None, stream=None, n_contrib=None, render_ws=None, tune: Optional[FgTune] = None):
    """hist_edges: None or a sequence of ascending floats (host); kpc_hist the
    device counts. n_contrib, render_ws, tune: those of an fg_render of the
    same view with saved state (chunk-parallel walk), or all None."""
    ss, cs = splats.struct(), camera_struct(cam)
    n_e = 0 if hist_edges is None else len(hist_edges)
    ev = (C.c_float * max(n_e, 1))(*([float(e) for e in hist_edges] if n_e else [0.0]))
    ws_bytes = 0 if render_ws is None else render_ws.numel() * render_ws.element_size()
    _check(lib().fg_gtc(_ref(ss), _p(vals), _p(ranges), _ref(cs), _p(n_pairs), cap_pairs, _p(kpc), _p(tile_gtc), _p(view_gtc),
                        C.cast(ev, C.c_void_p) if n_e else None, n_e, _p(kpc_hist), _p(n_contrib), _p(render_ws),
                        ws_bytes, _ref(tune) if tune is not None else None, _stream(stream)), "fg_gtc")


def fg_gtc_tau(view_gtc, n_views: int, lambda_G: float, g_bar, tau, status=None, stream=None):
    _check(lib().fg_gtc_tau(_p(view_gtc), n_views, C.c_float(lambda_G), _p(g_bar), _p(tau), _p(status),
                            _stream(stream)), "fg_gtc_tau")


# ---------------------------------------------------------------------------
# one view's buffers and the four-stage frame
# ---------------------------------------------------------------------------
class FrameBuffers:
    """All buffers of one view; capacities are fixed at construction."""

    def __init__(self, tree: DeviceTree, width: int, height: int, cap_sel: int, cap_pairs: int, device="cuda",
                 save_state: bool = False):
        self.width, self.height = width, height
        self.cap_sel, self.cap_pairs = int(cap_sel), int(cap_pairs)
        N = tree.n_nodes
        i32 = torch.int32
        self.sel_bits = torch.empty(max((N + 31) // 32, 1), dtype=i32, device=device)
        self.sel_idx = torch.empty(max(self.cap_sel, 1), dtype=i32, device=device)
        self.counts = torch.zeros(4, dtype=i32, device=device)  # n_sel, n_pairs, status, spare
        self.filter_ws = torch.empty(fg_filter_workspace_size(N, tree.n_internal_span), dtype=torch.uint8,
                                     device=device)
        self.splats = Splats(self.cap_sel, device)
        n_tiles = ((width + 15) // 16) * ((height + 15) // 16)
        self.tile_keys = torch.empty(max(self.cap_pairs, 1), dtype=i32, device=device)
        self.vals = torch.empty(max(self.cap_pairs, 1), dtype=i32, device=device)
        self.ranges = torch.empty((n_tiles, 2), dtype=i32, device=device)

        class _C:  # camera of this size, only for the workspace query
            R = np.eye(3, dtype=np.float32).reshape(9); t = np.zeros(3, np.float32); campos = t
            fx = fy = cx = cy = 1.0; znear = 0.2; kx = ky = 1.0; tile_base = 0
        _C.width, _C.height = width, height
        self.sort_ws = torch.empty(fg_sort_workspace_size(self.cap_sel, 1, self.cap_sel, self.cap_pairs),
                                   dtype=torch.uint8, device=device)
        rw = max(fg_render_workspace_size(_C, self.cap_pairs, tune_struct(c, save_state=save_state))
                 for c in (128, 256, 512))
        self.render_ws = torch.empty(rw, dtype=torch.uint8, device=device)
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((height, width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((height, width), dtype=i32, device=device)

    @property
    def n_sel(self):
        return self.counts[0:1]

    @property
    def n_pairs(self):
        return self.counts[1:2]

    @property
    def status(self):
        return self.counts[2:3]


def filter_stage(tree, cam, fb: FrameBuffers, tau_R=3.0, stream=None):
    fg_filter(tree, cam, tau_R, fb.sel_bits, fb.sel_idx, fb.cap_sel, fb.n_sel, fb.status, fb.filter_ws, stream)


def preprocess_stage(tree, cam, fb: FrameBuffers, tau=0.0, stream=None):
    fg_preprocess(tree, cam, tau, fb.sel_idx, fb.n_sel, fb.cap_sel, fb.splats, fb.status, stream)


def sort_stage(cam, fb: FrameBuffers, tune=None, stream=None):
    fg_sort(fb.splats, fb.n_sel, fb.cap_sel, cam, fb.tile_keys, fb.vals, fb.cap_pairs, fb.n_pairs, fb.ranges,
            fb.status, fb.sort_ws, tune, stream)


def render_stage(cam, fb: FrameBuffers, bg=(0.0, 0.0, 0.0), tune=None, stream=None, frag_stats=None):
    fg_render(fb.splats, fb.vals, fb.ranges, cam, bg, fb.image, fb.final_T, fb.n_contrib, fb.cap_pairs, frag_stats,
              fb.status, fb.render_ws, tune, stream)


def render_frame(tree: DeviceTree, cam, fb: FrameBuffers, tau_R: float = 3.0, tau: float = 0.0,
                 bg=(0.0, 0.0, 0.0), tune: Optional[FgTune] = None, stream=None):
    """Filter, preprocess, sort and blend one view into fb (asynchronous)."""
    filter_stage(tree, cam, fb, tau_R, stream)
    preprocess_stage(tree, cam, fb, tau, stream)
    sort_stage(cam, fb, tune, stream)
    render_stage(cam, fb, bg, tune, stream)


class GtcBuffers:
    """Outputs of the GTC pre-pass for n_views views of one size: per-pair KPC
    and per-tile GTC of the last view, the view GTCs, G_bar, tau, and one
    status word per view (plus one for fg_gtc_tau)."""

    def __init__(self, fb: FrameBuffers, n_views: int = 1, device="cuda"):
        self.kpc = torch.empty(max(fb.cap_pairs, 1), dtype=torch.float32, device=device)
        # workspace of the blend run with saved state before each view's KPC walk
        self.tune = tune_struct(0, save_state=True)

        class _C:  # camera of this size, only for the workspace query
            R = np.eye(3, dtype=np.float32).reshape(9); t = np.zeros(3, np.float32); campos = t
            fx = fy = cx = cy = 1.0; znear = 0.2; kx = ky = 1.0; tile_base = 0
        _C.width, _C.height = fb.width, fb.height
        self.render_ws = torch.empty(fg_render_workspace_size(_C, fb.cap_pairs, self.tune), dtype=torch.uint8,
                                     device=device)
        self.tile_gtc = torch.empty(fb.ranges.shape[0], dtype=torch.float32, device=device)
        self.view_gtc = torch.zeros((n_views, 2), dtype=torch.float64, device=device)
        self.g_bar = torch.zeros(1, dtype=torch.float64, device=device)
        self.tau = torch.zeros(1, dtype=torch.float32, device=device)
        self.status = torch.zeros(n_views + 1, dtype=torch.int32, device=device)


def gtc_view_stage(cam, fb: FrameBuffers, gb: GtcBuffers, v: int = 0, hist_edges=None, kpc_hist=None,
                   stream=None, chunked: bool = True, status=None):
    """KPC, tile and view GTC of the view sorted into fb. chunked: first blend
    the view with saved state (into fb's image planes) so that the KPC walk
    runs chunk-parallel; else one workgroup walks each tile's whole list."""
    if chunked:
        fg_render(fb.splats, fb.vals, fb.ranges, cam, (0.0, 0.0, 0.0), fb.image, fb.final_T, fb.n_contrib,
                  fb.cap_pairs, None, fb.status if status is None else status, gb.render_ws, gb.tune, stream)
        fg_gtc(fb.splats, fb.vals, fb.ranges, cam, fb.n_pairs, fb.cap_pairs, gb.kpc, gb.tile_gtc, gb.view_gtc[v],
               hist_edges, kpc_hist, stream, fb.n_contrib, gb.render_ws, gb.tune)
    else:
        fg_gtc(fb.splats, fb.vals, fb.ranges, cam, fb.n_pairs, fb.cap_pairs, gb.kpc, gb.tile_gtc, gb.view_gtc[v],
               hist_edges, kpc_hist, stream)


def scene_tau(tree: DeviceTree, cams, fb: FrameBuffers, lambda_G: float = 0.2, tau_R: float = 3.0,
              gb: Optional[GtcBuffers] = None, stream=None) -> GtcBuffers:
    """The GTC pre-pass over training views (Fig. 2(b)): each view filtered,
    projected with 3-sigma extents and sorted, its GTC accumulated; then
    tau = lambda_G / G_bar on the device (gb.tau, gb.g_bar). Asynchronous:
    each view's stages report into their own status word gb.status[v], and
    fg_gtc_tau into gb.status[n_views]; all must read 0."""
    cams = list(cams)
    gb = gb or GtcBuffers(fb, len(cams))
    for v, cam in enumerate(cams):
        st = gb.status[v:v + 1]
        fg_filter(tree, cam, tau_R, fb.sel_bits, fb.sel_idx, fb.cap_sel, fb.n_sel, st, fb.filter_ws, stream)
        fg_preprocess(tree, cam, 0.0, fb.sel_idx, fb.n_sel, fb.cap_sel, fb.splats, st, stream)
        fg_sort(fb.splats, fb.n_sel, fb.cap_sel, cam, fb.tile_keys, fb.vals, fb.cap_pairs, fb.n_pairs, fb.ranges, st,
                fb.sort_ws, None, stream)
        gtc_view_stage(cam, fb, gb, v, stream=stream, status=st)
    n = len(cams)
    fg_gtc_tau(gb.view_gtc, n, lambda_G, gb.g_bar, gb.tau, gb.status[n:n + 1], stream)
    return gb


def read_counts(fb: FrameBuffers):
    """(n_sel, n_pairs, status) copied to the host (synchronises)."""
    c = fb.counts.cpu().numpy().view(np.uint32)
    return int(c[0]), int(c[1]), int(c[2])


# ---------------------------------------------------------------------------
# differentiable form
# ---------------------------------------------------------------------------
def params_struct(mean, log_scale, quat, logit, sh, sh_degree: int) -> FgParams:
    return FgParams(m=int(logit.shape[0]), sh_degree=sh_degree, pad=0, mean=mean.data_ptr(),
                    log_scale=log_scale.data_ptr(), quat=quat.data_ptr(), logit=logit.data_ptr(), sh=sh.data_ptr())


def fg_activate(prm: FgParams, scale, opacity, stream=None):
    _check(lib().fg_activate(_ref(prm), _p(scale), _p(opacity), _stream(stream)), "fg_activate")


def fg_render_backward_workspace_size(cap_sel: int) -> int:
    return int(lib().fg_render_backward_workspace_size(cap_sel))


def fg_render_backward(prm: FgParams, cam, bg, sel_idx, n_sel, cap_sel: int, splats: Splats, vals, ranges, final_T,
                       n_contrib, image, render_ws, cap_pairs: int, tune: Optional[FgTune], dL_dimage,
                       grads: FgGrads, ws, stream=None):
    cs, ss = camera_struct(cam), splats.struct()
    bgv = (C.c_float * 3)(*[float(b) for b in bg])
    rws_bytes = render_ws.numel() * render_ws.element_size() if render_ws is not None else 0
    _check(lib().fg_render_backward(_ref(prm), _ref(cs), C.cast(bgv, C.c_void_p), _p(sel_idx), _p(n_sel), cap_sel,
                                    _ref(ss), _p(vals), _p(ranges), _p(final_T), _p(n_contrib), _p(image),
                                    _p(render_ws), rws_bytes, cap_pairs, _ref(tune) if tune is not None else None,
                                    _p(dL_dimage), _ref(grads), _p(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)),
           "fg_render_backward")
