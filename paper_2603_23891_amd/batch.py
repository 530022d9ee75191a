"""Batched multi-view rendering: V views of one tree as one frame.

The views go through the four stages together: one node-major filter call
(passes of up to eight views), one projection call, one sort of every view's
Gaussian-tile pairs under global tile ids, and one blend whose persistent
workgroups take (view, tile) work items from a single queue. The cameras'
poses live in a device array that the filter and projection kernels read, so a
batch captured in a HIP graph replays with new poses written into that array
(intrinsics and image sizes are fixed at capture). ``autotune`` picks the
speed-only knobs (blend chunk, radix digit width).

Marshalling and scheduling only: every stage runs in libfg's kernels.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import fg

# fields of fg_camera that a replay keeps from capture time (everything but the pose)
_FIXED = ("fx", "fy", "cx", "cy", "width", "height", "znear", "kx", "ky", "tile_base")


class BatchedRenderer:
    """Renders V views of one device-resident tree per call of ``run``.

    cap_sel: selected-node capacity per view; cap_pairs: pair capacity of the
    whole batch; cap_items: capacity for the tile-covering splats of all views
    (default: V * cap_sel). The views' global tile ids must be consecutive
    (cams[v].tile_base = cams[v-1].tile_base + tiles of view v-1)."""

    def __init__(self, tree: fg.DeviceTree, cams: Sequence, cap_sel: int, cap_pairs: int,
                 cap_items: Optional[int] = None, device="cuda"):
        self.tree, self.cams = tree, list(cams)
        V = len(self.cams)
        self.n_views = V
        self.cap_sel = int(cap_sel)
        self.cap_pairs = int(cap_pairs)
        self.cap_items = int(cap_items) if cap_items is not None else V * self.cap_sel
        self.tile0 = np.zeros(V + 1, np.int64)
        self.pix0 = np.zeros(V + 1, np.int64)
        for v, c in enumerate(self.cams):
            nt = ((c.width + 15) // 16) * ((c.height + 15) // 16)
            if c.tile_base != self.cams[0].tile_base + self.tile0[v]:
                raise ValueError("views need consecutive global tile ids")
            self.tile0[v + 1] = self.tile0[v] + nt
            self.pix0[v + 1] = self.pix0[v] + c.width * c.height
        N = tree.n_nodes
        i32 = torch.int32
        self.words = (N + 31) // 32
        self.sel_bits = torch.empty(V * max(self.words, 1), dtype=i32, device=device)
        self.sel_idx = torch.empty(V * max(self.cap_sel, 1), dtype=i32, device=device)
        self.n_sel = torch.zeros(V, dtype=i32, device=device)
        self.status = torch.zeros(1, dtype=i32, device=device)
        self.filter_ws = torch.empty(fg.fg_filter_workspace_size(N, tree.n_internal_span, V), dtype=torch.uint8,
                                     device=device)
        self.splats = fg.Splats(V * max(self.cap_sel, 1), device)
        self.tile_keys = torch.empty(max(self.cap_pairs, 1), dtype=i32, device=device)
        self.vals = torch.empty(max(self.cap_pairs, 1), dtype=i32, device=device)
        self.n_pairs = torch.zeros(1, dtype=i32, device=device)
        self.ranges = torch.empty((int(self.tile0[-1]), 2), dtype=i32, device=device)
        self.sort_ws = torch.empty(fg.fg_sort_workspace_size(self.cap_sel, V, self.cap_items, self.cap_pairs),
                                   dtype=torch.uint8, device=device)
        rw = max(fg.fg_render_workspace_size(self.cams, self.cap_pairs, fg.tune_struct(c)) for c in (128, 256, 512))
        self.render_ws = torch.empty(rw, dtype=torch.uint8, device=device)
        P = int(self.pix0[-1])
        self.image = torch.empty(3 * P, dtype=torch.float32, device=device)
        self.final_T = torch.empty(P, dtype=torch.float32, device=device)
        self.n_contrib = torch.empty(P, dtype=i32, device=device)
        arr, _ = fg.camera_array(self.cams)
        self.cams_dev = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(device)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.tune = fg.tune_struct()

    # -- per-view views of the packed outputs --------------------------------
    def view_image(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        a = int(self.pix0[v])
        return self.image[3 * a:3 * a + 3 * c.width * c.height].view(3, c.height, c.width)

    def view_final_T(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        a = int(self.pix0[v])
        return self.final_T[a:a + c.width * c.height].view(c.height, c.width)

    def view_n_contrib(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        a = int(self.pix0[v])
        return self.n_contrib[a:a + c.width * c.height].view(c.height, c.width)

    def view_ranges(self, v: int) -> torch.Tensor:
        return self.ranges[int(self.tile0[v]):int(self.tile0[v + 1])]

    # -- poses -----------------------------------------------------------------
    def set_poses(self, cams: Sequence, stream=None):
        """Write new poses (R, t, campos) into the device camera array, stream-
        ordered (a later run or graph replay on the same stream uses them).
        Every other camera field must equal the batch's."""
        cams = list(cams)
        if len(cams) != self.n_views:
            raise ValueError("one camera per view")
        for a, b in zip(cams, self.cams):
            for k in _FIXED:
                if getattr(a, k) != getattr(b, k):
                    raise ValueError(f"camera field {k} differs from the batch's; only poses can change")
        arr, _ = fg.camera_array(cams)
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).pin_memory()
        s = stream or torch.cuda.current_stream()
        with torch.cuda.stream(s):
            self.cams_dev.copy_(host, non_blocking=True)
        self._staging = host  # kept alive until the next call (the copy is asynchronous)

    # -- the batch -------------------------------------------------------------
    def run(self, tau_R: float = 3.0, tau: float = 0.0, bg=(0.0, 0.0, 0.0), tune: Optional[fg.FgTune] = None):
        """Enqueue the whole batch on the current stream (no host
        synchronisation): filter, projection, sort and blend of all views."""
        tune = tune or self.tune
        fg.fg_filter(self.tree, self.cams, tau_R, self.sel_bits, self.sel_idx, self.cap_sel, self.n_sel,
                     self.status, self.filter_ws, cams_dev=self.cams_dev)
        fg.fg_preprocess(self.tree, self.cams, tau, self.sel_idx, self.n_sel, self.cap_sel, self.splats,
                         self.status, cams_dev=self.cams_dev)
        fg.fg_sort(self.splats, self.n_sel, self.cap_sel, self.cams, self.tile_keys, self.vals, self.cap_pairs,
                   self.n_pairs, self.ranges, self.status, self.sort_ws, tune, cap_items=self.cap_items)
        fg.fg_render(self.splats, self.vals, self.ranges, self.cams, bg, self.image, self.final_T, self.n_contrib,
                     self.cap_pairs, None, self.status, self.render_ws, tune)

    def capture(self, tau_R: float = 3.0, tau: float = 0.0, bg=(0.0, 0.0, 0.0),
                tune: Optional[fg.FgTune] = None) -> torch.cuda.CUDAGraph:
        """Capture one batch into a HIP graph (replayed by ``replay``)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run(tau_R, tau, bg, tune)  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(tau_R, tau, bg, tune)
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def counts(self) -> Tuple[np.ndarray, np.ndarray, int]:
        """(n_sel per view, pairs per view, status), synchronising. A view's
        pairs are the contiguous run of the sorted list its tiles cover."""
        ns = self.n_sel.cpu().numpy().view(np.uint32).astype(np.int64)
        r = self.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
        per = np.zeros(self.n_views, np.int64)
        for v in range(self.n_views):
            rv = r[int(self.tile0[v]):int(self.tile0[v + 1])]
            per[v] = int((rv[:, 1] - rv[:, 0]).sum())
        return ns, per, int(self.status.cpu().numpy().view(np.uint32)[0])


def _digest(br: BatchedRenderer) -> np.ndarray:
    return np.concatenate([br.image.cpu().numpy().view(np.uint32), br.n_contrib.cpu().numpy().view(np.uint32)])


def autotune(br: BatchedRenderer, tau_R: float = 3.0, tau: float = 0.0, chunks=(128, 256, 512),
             radix_bits=(6, 7, 8), repeats: int = 3, cache_path: Optional[str] = None,
             cache_key: Optional[str] = None) -> Dict:
    """Times every (blend chunk B, radix digit width) candidate on the batch
    and keeps the fastest. Every candidate must give bit-identical images and
    contributor counts (the knobs change speed only)."""
    if cache_path and cache_key and os.path.exists(cache_path):
        with open(cache_path) as f:
            cached = json.load(f).get(cache_key)
        if cached:
            br.tune = fg.tune_struct(cached["render_batch"], cached["radix_bits"])
            return dict(cached, from_cache=True)
    stream = torch.cuda.current_stream()
    ref = None
    results = []
    for c in chunks:
        for b in radix_bits:
            t = fg.tune_struct(c, b)
            br.run(tau_R, tau, tune=t)
            torch.cuda.synchronize()
            dig = _digest(br)
            if ref is None:
                ref = dig
            elif not np.array_equal(dig, ref):
                raise RuntimeError(f"tuning candidate chunk={c} radix_bits={b} changed the output")
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(repeats):
                br.run(tau_R, tau, tune=t)
            ev[1].record(stream)
            torch.cuda.synchronize()
            results.append(dict(render_batch=c, radix_bits=b, ms=ev[0].elapsed_time(ev[1]) / repeats))
    best = min(results, key=lambda r: r["ms"])
    br.tune = fg.tune_struct(best["render_batch"], best["radix_bits"])
    out = dict(best, candidates=results, from_cache=False)
    if cache_path and cache_key:
        data = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                data = json.load(f)
        data[cache_key] = dict(render_batch=best["render_batch"], radix_bits=best["radix_bits"], ms=best["ms"])
        with open(cache_path, "w") as f:
            json.dump(data, f, indent=1)
    return out
