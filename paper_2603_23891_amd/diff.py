"""Differentiable rendering of raw Gaussians through libfg (torch.autograd).

``GaussianRenderer`` owns the device buffers of one view size; its
``render(mean, log_scale, quat, logit, sh, cam, tau)`` returns the image
[3, H, W] as a torch tensor whose backward calls ``fg_render_backward``.
Layouts follow the C-ABI: mean [3, M], log_scale [3, M], quat [4, M] (w, x, y,
z), logit [M], sh [M, (D+1)^2, 3]. The activation (fg_activate), the four
frame stages and the backward all run in the HIP kernels; this module only
passes pointers and keeps the forward buffers for the backward.
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

    def forward(self, mean, log_scale, quat, logit, sh, cam, tau: float = 0.0, bg=(0.0, 0.0, 0.0)):
        t = self.tree
        t.mean, t.quat, t.sh = mean, quat, sh
        prm = fg.params_struct(mean, log_scale, quat, logit, sh, self.sh_degree)
        fg.fg_activate(prm, t.scale, t.opacity)
        fg.render_frame(t, cam, self.fb, tau_R=3.0e38, tau=tau, bg=bg, tune=self.tune)
        return self.fb.image

    def backward(self, mean, log_scale, quat, logit, sh, cam, grad_image, bg=(0.0, 0.0, 0.0)):
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
        ctx.renderer, ctx.cam, ctx.bg = renderer, cam, bg
        ctx.save_for_backward(*args)
        return img

    @staticmethod
    def backward(ctx, grad_image):
        g = ctx.renderer.backward(*ctx.saved_tensors, ctx.cam, grad_image, ctx.bg)
        return (*g, None, None, None, None)
