"""Batched multi-view rendering: one node-major filter pass for all views,
per-view projection, sort and blend, the whole batch captured in one HIP graph,
and an autotuner for the speed-only knobs (blend chunk size, radix digit
width).

Marshalling and scheduling only: every stage runs in libfg's kernels.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import fg


class ViewBuffers:
    """Per-view projection / sort / blend buffers (capacities fixed)."""

    def __init__(self, cam, cap_sel: int, cap_pairs: int, device="cuda"):
        width, height = cam.width, cam.height
        self.width, self.height = width, height
        self.cap_sel, self.cap_pairs = cap_sel, cap_pairs
        i32 = torch.int32
        self.splats = fg.Splats(cap_sel, device)
        self.tile_keys = torch.empty(max(cap_pairs, 1), dtype=i32, device=device)
        self.vals = torch.empty(max(cap_pairs, 1), dtype=i32, device=device)
        n_tiles = ((width + 15) // 16) * ((height + 15) // 16)
        self.ranges = torch.empty((n_tiles, 2), dtype=i32, device=device)
        self.n_pairs = torch.zeros(1, dtype=i32, device=device)
        self.sort_ws = torch.empty(fg.fg_sort_workspace_size(cap_sel, cap_pairs, cam), dtype=torch.uint8,
                                   device=device)
        rw = max(fg.fg_render_workspace_size(cam, cap_pairs, fg.tune_struct(c)) for c in (128, 256, 512))
        self.render_ws = torch.empty(rw, dtype=torch.uint8, device=device)
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((height, width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((height, width), dtype=i32, device=device)


class BatchedRenderer:
    """Renders V views of one device-resident tree per call of ``run``."""

    def __init__(self, tree: fg.DeviceTree, cams: Sequence, cap_sel: int, cap_pairs: Sequence[int] | int,
                 device="cuda", n_streams: int = 4):
        self.tree, self.cams = tree, list(cams)
        V = len(self.cams)
        self.cap_sel = int(cap_sel)
        caps = [int(cap_pairs)] * V if isinstance(cap_pairs, int) else [int(c) for c in cap_pairs]
        N = tree.n_nodes
        self.words = (N + 31) // 32
        self.sel_bits = torch.empty(V * max(self.words, 1), dtype=torch.int32, device=device)
        self.sel_idx = torch.empty(V * max(self.cap_sel, 1), dtype=torch.int32, device=device)
        self.n_sel = torch.zeros(V, dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.filter_ws = torch.empty(fg.fg_filter_workspace_size(N, tree.n_internal_span, V), dtype=torch.uint8,
                                     device=device)
        self.views = [ViewBuffers(c, self.cap_sel, caps[i], device) for i, c in enumerate(self.cams)]
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.tune = fg.tune_struct()
        # views run on n_streams streams (default priority) after the shared
        # filter, so one view's long blend tail overlaps other views' work
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, n_streams))]

    def run(self, tau_R: float = 3.0, tau: float = 0.0, bg=(0.0, 0.0, 0.0), tune: Optional[fg.FgTune] = None):
        """Enqueue the whole batch (no host synchronisation): the node-major
        filter on the current stream, then the views' projection, sort and
        blend spread over the batch's streams, which the current stream joins
        at the end. Graph capture records the fork and join."""
        tune = tune or self.tune
        main = torch.cuda.current_stream()
        fg.fg_filter(self.tree, self.cams, tau_R, self.sel_bits, self.sel_idx, self.cap_sel, self.n_sel,
                     self.status, self.filter_ws, stream=main)
        for st in self.streams:
            st.wait_stream(main)
        for v, (cam, vb) in enumerate(zip(self.cams, self.views)):
            st = self.streams[v % len(self.streams)]
            sel = self.sel_idx[v * self.cap_sel:(v + 1) * self.cap_sel]
            nsel = self.n_sel[v:v + 1]
            fg.fg_preprocess(self.tree, cam, tau, sel, nsel, self.cap_sel, vb.splats, self.status, stream=st)
            fg.fg_sort(vb.splats, nsel, self.cap_sel, cam, vb.tile_keys, vb.vals, vb.cap_pairs, vb.n_pairs,
                       vb.ranges, self.status, vb.sort_ws, tune, stream=st)
            fg.fg_render(vb.splats, vb.vals, vb.ranges, cam, bg, vb.image, vb.final_T, vb.n_contrib, vb.cap_pairs,
                         None, self.status, vb.render_ws, tune, stream=st)
        for st in self.streams:
            main.wait_stream(st)

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
        """(n_sel per view, n_pairs per view, status), synchronising."""
        ns = self.n_sel.cpu().numpy().view(np.uint32).astype(np.int64)
        npairs = np.array([int(vb.n_pairs.cpu().numpy().view(np.uint32)[0]) for vb in self.views])
        return ns, npairs, int(self.status.cpu().numpy().view(np.uint32)[0])


def _digest(br: BatchedRenderer) -> List[np.ndarray]:
    return [np.concatenate([vb.image.cpu().numpy().ravel().view(np.uint32),
                            vb.n_contrib.cpu().numpy().ravel().view(np.uint32)]) for vb in br.views]


def autotune(br: BatchedRenderer, tau_R: float = 3.0, tau: float = 0.0, chunks=(128, 256, 512),
             radix_bits=(6, 7, 8), repeats: int = 3, cache_path: Optional[str] = None,
             cache_key: Optional[str] = None) -> Dict:
    """Times every (blend chunk, radix digit width) candidate on the batch and
    keeps the fastest. Every candidate must give bit-identical images and
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
            elif not all(np.array_equal(a, r) for a, r in zip(dig, ref)):
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
