"""Differentiable rendering of raw Gaussians through libfg (torch.autograd).

``GaussianRenderer`` owns the device buffers of one view size; its
``render(mean, log_scale, quat, logit, sh, cam, tau)`` returns the image
[3, H, W] as a torch tensor whose backward calls ``fg_render_backward``.
Layouts follow the C-ABI: mean [3, M], log_scale [3, M], quat [4, M] (w, x, y,
z), logit [M], sh [M, (D+1)^2, 3]. The activation (fg_activate), the four
frame stages and the backward all run in the HIP kernels; this module only
passes pointers and keeps the forward buffers for the backward.

A renderer holds the state of its latest forward only: the backward of a
frame must run before the next forward on the same renderer (and with the
tune that forward used). Each forward is stamped with a generation number
and its tune; a backward whose frame has been overwritten raises instead of
returning the gradients of another frame. Render several views before one
loss.backward() with one renderer per view.
"""
from __future__ import annotations

import torch

from . import fg


class _FlatTree:
    """fg_tree view of M activated Gaussians, each a root leaf."""

    def __init__(self, m: int, sh_degree: int, device):
        self.n_nodes = m
        self.n_internal_span = 0
        self.max_depth = 0
        self.sh_degree = sh_degree
        self.scale = torch.empty((3, m), dtype=torch.float32, device=device)
        self.opacity = torch.empty((m,), dtype=torch.float32, device=device)
        self.parent = torch.full((m,), -1, dtype=torch.int32, device=device)
        self.flags = torch.ones((m,), dtype=torch.uint8, device=device)
        self.mean = self.quat = self.sh = None

    def struct(self) -> fg.FgTree:
        return fg.FgTree(n_nodes=self.n_nodes, n_internal_span=0, sh_degree=self.sh_degree, max_depth=0,
                         mean=self.mean.data_ptr(), scale=self.scale.data_ptr(), quat=self.quat.data_ptr(),
                         opacity=self.opacity.data_ptr(), sh=self.sh.data_ptr(), parent=self.parent.data_ptr(),
                         flags=self.flags.data_ptr())


class GaussianRenderer:
    def __init__(self, m: int, sh_degree: int, width: int, height: int, cap_pairs: int, device="cuda"):
        self.m, self.sh_degree = m, sh_degree
        self.tree = _FlatTree(m, sh_degree, device)
        # the forward keeps per-chunk state for the backward's parallel walk
        self.tune = fg.tune_struct(save_state=True)
        self.fb = fg.FrameBuffers(self.tree, width, height, cap_sel=m, cap_pairs=cap_pairs, device=device,
                                  save_state=True)
        self.bwd_ws = torch.empty(fg.fg_render_backward_workspace_size(m), dtype=torch.uint8, device=device)
        self.generation = 0     # number of forwards run so far
        self._fwd_stamp = None  # (generation, tune fields) of the frame held in self.fb

    def _tune_key(self):
        t = self.tune
        return (t.render_batch, t.radix_bits, t.save_state, t.mask_items)

    def forward(self, mean, log_scale, quat, logit, sh, cam, tau: float = 0.0, bg=(0.0, 0.0, 0.0)):
        t = self.tree
        t.mean, t.quat, t.sh = mean, quat, sh
        prm = fg.params_struct(mean, log_scale, quat, logit, sh, self.sh_degree)
        fg.fg_activate(prm, t.scale, t.opacity)
        fg.render_frame(t, cam, self.fb, tau_R=3.0e38, tau=tau, bg=bg, tune=self.tune)
        self.generation += 1
        self._fwd_stamp = (self.generation, self._tune_key())
        return self.fb.image

    def backward(self, mean, log_scale, quat, logit, sh, cam, grad_image, bg=(0.0, 0.0, 0.0),
                 generation: int = None):
        """generation: the number forward() stamped on the frame (None: the
        latest frame). Raises if that frame's buffers were overwritten by a
        later forward or the tune changed since."""
        if self._fwd_stamp is None:
            raise RuntimeError("GaussianRenderer.backward before any forward")
        gen, key = self._fwd_stamp
        if generation is not None and generation != gen:
            raise RuntimeError(f"the frame of forward #{generation} was overwritten by forward #{gen} on this "
                               "renderer: run each backward before the next forward, or use one renderer per view")
        if key != self._tune_key():
            raise RuntimeError("the renderer's tune changed between forward and backward")
        prm = fg.params_struct(mean, log_scale, quat, logit, sh, self.sh_degree)
        g = [torch.empty_like(x) for x in (mean, log_scale, quat, logit, sh)]
        grads = fg.FgGrads(*[x.data_ptr() for x in g])
        fb = self.fb
        fg.fg_render_backward(prm, cam, bg, fb.sel_idx, fb.n_sel, fb.cap_sel, fb.splats, fb.vals, fb.ranges,
                              fb.final_T, fb.n_contrib, fb.image, fb.render_ws, fb.cap_pairs, self.tune,
                              grad_image.contiguous(), grads, self.bwd_ws)
        return g

    def render(self, mean, log_scale, quat, logit, sh, cam, tau: float = 0.0, bg=(0.0, 0.0, 0.0)):
        return FilterGSRender.apply(mean, log_scale, quat, logit, sh, self, cam, tau, tuple(bg))


class FilterGSRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, logit, sh, renderer: GaussianRenderer, cam, tau, bg):
        args = [x.detach().contiguous() for x in (mean, log_scale, quat, logit, sh)]
        img = renderer.forward(*args, cam, tau, bg).clone()
        n_sel, n_pairs, status = fg.read_counts(renderer.fb)  # synchronises
        if status != 0:
            raise fg.FgError(f"forward status {status:#x} (selected {n_sel} of capacity {renderer.fb.cap_sel}, "
                             f"pairs {n_pairs} of capacity {renderer.fb.cap_pairs})")
        ctx.renderer, ctx.cam, ctx.bg = renderer, cam, bg
        ctx.generation = renderer.generation
        ctx.save_for_backward(*args)
        return img

    @staticmethod
    def backward(ctx, grad_image):
        g = ctx.renderer.backward(*ctx.saved_tensors, ctx.cam, grad_image, ctx.bg, generation=ctx.generation)
        return (*g, None, None, None, None)
