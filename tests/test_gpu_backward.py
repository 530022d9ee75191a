"""GPU parity of the differentiable form (fg_activate + frame + fg_render_backward).

* forward: the image of the raw Gaussians equals the oracle's float32 frame
  bit for bit (activation included);
* gradients: against the float64 oracle gradient (the exact derivative of the
  float32 forward's smooth piece, itself pinned by finite differences):
  per parameter group ||g_gpu - g64|| / ||g64|| <= 1e-3, and elementwise
  |g_gpu - g64| <= 1e-3 (|g64| + 1e-3 max|g64|) for elements with
  |g64| >= 1e-2 max|g64|. A gradient element is a sum over many pixels of
  float32 terms whose signs differ (always so under an L1 loss); its rounding
  error scales with the terms (of the order of the group's largest gradient),
  not with the cancelled sum, and the transmittance recovered by repeated
  division adds error along long chains, so elements far below the group's
  scale are held by the group-norm bar only. float32 atomics sum in a varying
  order, so the bar is a tolerance, not bit equality;
* central differences (h = 1e-3) of the float64 replayed loss at 64 sampled
  parameters;
* torch.autograd through FilterGSRender equals a direct backward call.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import diff, fg, synth
from tests.test_oracle_backward import make_params, perturbed

pytestmark = pytest.mark.gpu
GROUPS = ("mean", "log_scale", "quat", "logit", "sh")


def to_dev(prm):
    return [torch.from_numpy(a.copy()).cuda() for a in prm.keep]


def gpu_fwd_bwd(prm, cam, w, tau=0.0, bg=(0.0, 0.0, 0.0), tune=None):
    args = to_dev(prm)
    r = diff.GaussianRenderer(prm.m, prm.sh_degree, cam.width, cam.height, cap_pairs=1 << 20)
    if tune is not None:
        r.tune = tune
    img = r.forward(*args, cam, tau, bg).clone()
    g = r.backward(*args, cam, torch.from_numpy(w.astype(np.float32)).cuda(), bg)
    torch.cuda.synchronize()
    return img.cpu().numpy(), {k: v.cpu().numpy().astype(np.float64) for k, v in zip(GROUPS, g)}, r


def check_grads(g_gpu, g64, tol=1e-3, floor=1e-3):
    """Group norm within tol; elements at least 1 % of the group's largest within
    tol * (|g64| + floor * max|g64|)."""
    report = {}
    for k in GROUPS:
        a, b = g_gpu[k], g64[k]
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(nb, 1e-30)
        big = np.abs(b) >= 1e-2 * np.abs(b).max()
        el = (np.abs(a - b)[big] / (np.abs(b)[big] + floor * np.abs(b).max())).max() if big.any() else 0.0
        report[k] = (rel, el)
        assert rel <= tol, (k, rel)
        assert el <= tol, (k, el)
    return report


@pytest.mark.parametrize("seed,m,size,tau", [(1, 300, (128, 96), 0.0), (5, 3000, (128, 128), 0.05),
                                             (9, 1500, (200, 120), 1 / 255)])
def test_backward_matches_float64_oracle(seed, m, size, tau):
    prm, cam, rng = make_params(seed, m=m, width=size[0], height=size[1])
    bg = (0.1, 0.2, 0.3)
    fwd = oracle.forward32(prm, cam, tau, bg)
    w = rng.normal(0, 1, (3, cam.height, cam.width))
    img, g_gpu, _ = gpu_fwd_bwd(prm, cam, w, tau, bg)
    assert np.array_equal(img, fwd["image"])
    _, g64 = oracle.replay64(prm, cam, fwd, dL_dimage=w, bg=bg, want_image=False)
    check_grads(g_gpu, g64)


def test_backward_against_central_differences():
    prm, cam, rng = make_params(11, m=400)
    fwd = oracle.forward32(prm, cam)
    w = rng.normal(0, 1, (3, cam.height, cam.width))
    _, g_gpu, _ = gpu_fwd_bwd(prm, cam, w)
    sel = fwd["sel_idx"]
    rows = {"mean": 3, "log_scale": 3, "quat": 4}
    scale = {k: np.abs(g_gpu[k]).max() for k in GROUPS}
    h = 1e-3
    n = 0
    for group in GROUPS:
        for _ in range(13 if group != "logit" else 12):
            node = int(sel[rng.integers(0, sel.size)])
            if group in rows:
                idx = (int(rng.integers(0, rows[group])), node)
            elif group == "logit":
                idx = (node,)
            else:
                idx = (node, int(rng.integers(0, g_gpu["sh"].shape[1])), int(rng.integers(0, 3)))
            pp, vp = perturbed(prm, group, idx, h)
            pm, vm = perturbed(prm, group, idx, -h)
            lp = float((oracle.replay64(pp, cam, fwd)[0] * w).sum())
            lm = float((oracle.replay64(pm, cam, fwd)[0] * w).sum())
            fd = (lp - lm) / (vp - vm)
            a = g_gpu[group][idx]
            assert abs(a - fd) <= 1e-3 * max(abs(fd), 1e-2 * scale[group]), (group, idx, a, fd)
            n += 1
    assert n == 64


def test_autograd_function_and_l1_loss():
    prm, cam, rng = make_params(3, m=500)
    target = torch.from_numpy(rng.uniform(0, 1, (3, cam.height, cam.width)).astype(np.float32)).cuda()
    args = [a.requires_grad_(True) for a in to_dev(prm)]
    r = diff.GaussianRenderer(prm.m, prm.sh_degree, cam.width, cam.height, cap_pairs=1 << 20)
    img = r.render(*args, cam)
    loss = (img - target).abs().mean()
    loss.backward()
    dl = (torch.sign(img.detach() - target) / img.numel()).contiguous()
    direct = r.backward(*[a.detach() for a in args], cam, dl)
    # two runs of the backward: fp32 atomics add in a different order each
    # time, so elements that cancel differ at the rounding level of the
    # group's largest terms
    for a, d in zip(args, direct):
        assert torch.allclose(a.grad, d, rtol=1e-5, atol=1e-6 * float(d.abs().max()) + 1e-30)
    # and the float64 oracle of the same L1 loss
    fwd = oracle.forward32(prm, cam)
    _, g64 = oracle.replay64(prm, cam, fwd, dL_dimage=dl.cpu().numpy().astype(np.float64), want_image=False)
    check_grads({k: a.grad.cpu().numpy().astype(np.float64) for k, a in zip(GROUPS, args)}, g64)


def heavy_params(seed, m, opacity_logit_mu):
    """m small Gaussians over a 3 x 2 tile block (48 x 32 px) of a 128 x 96
    image: ranges of thousands of splats, so the forward cuts them into chunks
    and the backward walks the chunks in parallel from the saved state."""
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 128, 96)
    z = rng.uniform(8, 14, m)
    px = rng.uniform(40, 88, m)
    py = rng.uniform(32, 64, m)
    mean = np.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z], 1)
    log_scale = rng.normal(-4.6, 0.3, (m, 3)) + np.log(z)[:, None] - np.log(10.0)
    quat = rng.standard_normal((m, 4))
    logit = rng.normal(opacity_logit_mu, 1.0, m)
    sh = rng.normal(0, 0.3, (m, 16, 3))
    return oracle.ParamsRef(mean.T, log_scale.T, quat.T, logit, sh, 3), cam, rng


@pytest.mark.parametrize("mu,chunk,mask_items", [(-3.0, 256, 0), (0.5, 256, 0), (-3.0, 128, 3), (0.5, 512, 2),
                                                  (0.5, 128, 0)])
def test_backward_long_ranges_from_saved_chunk_state(mu, chunk, mask_items):
    """Translucent (pixels never saturate: every chunk blends) and opaque
    (pixels stop inside a later chunk) variants; gradients against the
    float64 oracle at the same bar, forward bit-exact. With mask_items > 0
    only the first chunks have stored masks and saved state: the tiles past
    them are walked whole by the backward. At 128-splat chunks the longest
    tiles have 16 or more chunks, so the forward blends them as two
    half-tile items and each half saves its own pixels' state."""
    prm, cam, rng = heavy_params(21, 9000, mu)
    fwd = oracle.forward32(prm, cam)
    lens = np.diff(fwd["ranges"], axis=1).ravel()
    assert lens.max() > 1024  # several chunks per tile
    if chunk == 128:
        assert lens.max() > 15 * 128 and np.any((lens > 128) & (lens <= 15 * 128))
    w = rng.normal(0, 1, (3, cam.height, cam.width))
    tune = fg.tune_struct(chunk, save_state=True, mask_items=mask_items)
    img, g_gpu, _ = gpu_fwd_bwd(prm, cam, w, tune=tune)
    assert np.array_equal(img, fwd["image"])
    _, g64 = oracle.replay64(prm, cam, fwd, dL_dimage=w, want_image=False)
    check_grads(g_gpu, g64)


def test_backward_counters():
    """The blend backward's counters (fg_tune.bwd_stats): it walks exactly the
    fragments the forward blended (the forward's own counter), issues one
    gradient atomic per wave and splat with a blended pixel (so no more than
    the fragments) adding 1 to 9 elements each, and its gradients still meet
    the float64 bar."""
    prm, cam, rng = make_params(5, m=3000, width=128, height=128)
    fwd = oracle.forward32(prm, cam, 0.05)
    w = rng.normal(0, 1, (3, cam.height, cam.width))
    args = to_dev(prm)
    r = diff.GaussianRenderer(prm.m, prm.sh_degree, cam.width, cam.height, cap_pairs=1 << 20)
    r.forward(*args, cam, 0.05)
    fstats = torch.zeros(8, dtype=torch.int64, device="cuda")
    fg.render_stage(cam, r.fb, tune=r.tune, frag_stats=fstats)
    bstats = torch.zeros(3, dtype=torch.int64, device="cuda")
    r.tune.bwd_stats = bstats.data_ptr()
    g = r.backward(*args, cam, torch.from_numpy(w.astype(np.float32)).cuda())
    r.tune.bwd_stats = None
    torch.cuda.synchronize()
    n_instr, n_elem, n_frag = (int(x) for x in bstats.cpu().tolist())
    assert n_frag == int(fstats[3].item()) > 0
    assert 0 < n_instr <= n_frag
    assert n_instr <= n_elem <= 9 * n_instr
    _, g64 = oracle.replay64(prm, cam, fwd, dL_dimage=w, want_image=False)
    check_grads({k: v.cpu().numpy().astype(np.float64) for k, v in zip(GROUPS, g)}, g64)
