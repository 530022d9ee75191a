"""Gradient parity of the differentiable form at full size: 2M raw Gaussians,
SH degree 3, 1920x1080, an L1 loss against a seeded uniform target, in the
renderer configuration the benchmark times (GaussianRenderer, 24M pair
capacity, chunk state saved for the parallel backward walk).

dL/dimage is the L1 loss's, restricted to a seeded, tile-aligned 128x128
crop. The oracle evaluates that crop only: a pixel's colour depends only on
the splats whose tile rectangle holds the pixel's tile, and their order in a
tile's list (depth, then index) does not change when the other Gaussians are
removed. So the float32 forward and the float64 replay of the Gaussians whose
rectangle meets the crop (in their original order) give the crop's pixels and
every gradient, and all other Gaussians have gradient exactly 0. On that
subset: the GPU's crop pixels equal the oracle's bit for bit; its gradients
meet the float64 replay within 1e-3 in each group's norm; and 64 central
differences (h = 1e-3) of the replayed crop loss agree with them.

Elementwise, each gradient element is within 1e-3 of the float64 value
plus 1e-4 of its group's largest element (the small tests use 1e-6 there).
The floor follows from the float32 forward itself: at 1080p a pixel offset
dx = u - (i + 0.5) is formed from coordinates up to 1920, whose half-ulp is
6e-5 px, so each pixel's term of a mean gradient carries a relative error of
~1e-4 against its ~1 px footprint scale; under the L1 loss the terms of a
splat's mean gradient have both signs and largely cancel, so that error
stays of the order of the largest terms (the group's scale), not of the sum.

The full-size launch reaches the grid-stride wrap of both backward kernels
(8160 tiles plus chunk items over at most 8192 workgroups; 2M Gaussians over
4096 x 256 threads).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import diff, fg, synth
from tests.test_gpu_backward import GROUPS, check_grads
from tests.test_oracle_backward import perturbed

pytestmark = pytest.mark.gpu
M = 2_000_000
CROP = 128


@pytest.fixture(scope="module")
def workload():
    g = synth.flat_gaussians(M, seed=0)
    cam = synth.city1m_yaw_views()[3]
    target = np.random.default_rng(2).uniform(0, 1, (3, cam.height, cam.width)).astype(np.float32)
    return g, cam, target


def pick_crop(splats, cam, rng):
    """A tile-aligned 128x128 crop (seeded) and the splats whose rectangle meets it."""
    Wt, Ht = (cam.width + 15) // 16, (cam.height + 15) // 16
    n = CROP // 16
    for _ in range(100):
        tx0, ty0 = int(rng.integers(0, Wt - n + 1)), int(rng.integers(0, Ht - n + 1))
        hit = ((splats["tiles"] > 0) & (splats["x0"] < tx0 + n) & (splats["x1"] > tx0) & (splats["y0"] < ty0 + n)
               & (splats["y1"] > ty0))
        if hit.sum() > 2000:
            return tx0 * 16, ty0 * 16, np.nonzero(hit)[0]
    raise AssertionError("no crop with content")


def test_c5_gradients_on_a_crop_at_full_size(workload):
    g, cam, target = workload
    # GPU: the full frame and its backward, as the benchmark runs them
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.mean, g.log_scale, g.quat, g.logit, g.sh)]
    r = diff.GaussianRenderer(M, g.sh_degree, cam.width, cam.height, cap_pairs=24_000_000)
    img = r.forward(*dev, cam).clone()
    torch.cuda.synchronize()
    n_sel, n_pairs, status = fg.read_counts(r.fb)
    assert status == 0 and n_sel == M and n_pairs > 3_000_000

    # oracle: the Gaussians whose rectangle meets the crop
    prm = oracle.ParamsRef(g.mean, g.log_scale, g.quat, g.logit, g.sh, g.sh_degree)
    full = oracle.flat_tree_from_params(prm)
    _, sel = oracle.filter(full, cam, 1e30)
    assert sel.size == M
    sp = oracle.preprocess(full, cam, 0.0, sel)
    rng = np.random.default_rng(3)
    x0, y0, S = pick_crop(sp, cam, rng)
    sub = oracle.ParamsRef(g.mean[:, S], g.log_scale[:, S], g.quat[:, S], g.logit[S], g.sh[S], g.sh_degree)
    fwd = oracle.forward32(sub, cam)
    ys, xs = slice(y0, y0 + CROP), slice(x0, x0 + CROP)
    img_g = img.cpu().numpy()
    assert np.array_equal(img_g[:, ys, xs], fwd["image"][:, ys, xs]), "crop pixels"

    # L1 loss restricted to the crop
    dl = np.zeros((3, cam.height, cam.width), np.float32)
    dl[:, ys, xs] = np.sign(img_g[:, ys, xs] - target[:, ys, xs]) / np.float32(img_g.size)
    grads = r.backward(*dev, cam, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    g_gpu = {k: v.cpu().numpy() for k, v in zip(GROUPS, grads)}
    outside = np.ones(M, bool)
    outside[S] = False
    for k in GROUPS:
        gk = g_gpu[k]
        assert np.all((gk[..., outside] if k != "sh" else gk[outside]) == 0), f"{k}: gradient outside the crop"
    sub_gpu = {k: (g_gpu[k][..., S] if k != "sh" else g_gpu[k][S]).astype(np.float64) for k in GROUPS}
    w = dl.astype(np.float64)
    _, g64 = oracle.replay64(sub, cam, fwd, dL_dimage=w, want_image=False)
    check_grads(sub_gpu, g64, floor=0.1)

    # central differences on 64 parameters of Gaussians that touch the crop
    touch = np.unique(fwd["vals"][np.concatenate([np.arange(a, b) for a, b in fwd["ranges"].reshape(-1, 2)
                                                  [[ty * ((cam.width + 15) // 16) + tx
                                                    for ty in range(y0 // 16, (y0 + CROP) // 16)
                                                    for tx in range(x0 // 16, (x0 + CROP) // 16)]]])])
    frng = np.random.default_rng(3)
    rows = {"mean": 3, "log_scale": 3, "quat": 4}
    scale = {k: np.abs(sub_gpu[k]).max() for k in GROUPS}
    n = 0
    for group in GROUPS:
        for _ in range(13 if group != "logit" else 12):
            j = int(touch[frng.integers(0, touch.size)])
            if group in rows:
                idx = (int(frng.integers(0, rows[group])), j)
            elif group == "logit":
                idx = (j,)
            else:
                idx = (j, int(frng.integers(0, sub_gpu["sh"].shape[1])), int(frng.integers(0, 3)))
            pp, vp = perturbed(sub, group, idx, 1e-3)
            pm, vm = perturbed(sub, group, idx, -1e-3)
            lp = float((oracle.replay64(pp, cam, fwd)[0][:, ys, xs] * w[:, ys, xs]).sum())
            lm = float((oracle.replay64(pm, cam, fwd)[0][:, ys, xs] * w[:, ys, xs]).sum())
            fd = (lp - lm) / (vp - vm)
            a = sub_gpu[group][idx]
            assert abs(a - fd) <= 1e-3 * max(abs(fd), 0.1 * scale[group]), (group, idx, a, fd)
            n += 1
    assert n == 64


def test_two_views_need_their_own_renderers(workload):
    """Two renders on one renderer before one backward: the first frame's
    buffers are overwritten, so its backward raises; with one renderer per
    view both backwards run and each equals a direct backward of its view."""
    g, cam, target = workload
    m = 200_000  # the first 200K Gaussians keep this test short
    dev = [torch.from_numpy(np.ascontiguousarray(a[..., :m] if a.ndim == 2 else a[:m])).cuda()
           for a in (g.mean, g.log_scale, g.quat, g.logit)]
    dev.append(torch.from_numpy(np.ascontiguousarray(g.sh[:m])).cuda())
    args = [a.clone().requires_grad_(True) for a in dev]
    views = synth.city1m_yaw_views()[2:4]
    tgt = torch.from_numpy(target).cuda()
    r = diff.GaussianRenderer(m, g.sh_degree, cam.width, cam.height, cap_pairs=8_000_000)
    imgs = [r.render(*args, v) for v in views]
    loss = sum((im - tgt).abs().mean() for im in imgs)
    with pytest.raises(RuntimeError, match="overwritten"):
        loss.backward()
    args = [a.detach().clone().requires_grad_(True) for a in dev]
    rs = [diff.GaussianRenderer(m, g.sh_degree, cam.width, cam.height, cap_pairs=8_000_000) for _ in views]
    imgs = [rr.render(*args, v) for rr, v in zip(rs, views)]
    loss = sum((im - tgt).abs().mean() for im in imgs)
    loss.backward()
    total = [torch.zeros_like(a) for a in dev]
    for rr, v, im in zip(rs, views, imgs):
        rr.forward(*dev, v)
        dl = (torch.sign(im.detach() - tgt) / im.numel()).contiguous()
        for t, d in zip(total, rr.backward(*dev, v, dl)):
            t += d
    for a, t in zip(args, total):
        assert torch.allclose(a.grad, t, rtol=1e-4, atol=1e-5 * float(t.abs().max()) + 1e-30)
