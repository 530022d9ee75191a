"""GPU parity: every stage of libfg against the CPU oracle on the same seeded inputs.

Bar: selection mask, compacted list, splat records, tile rectangles and
counts, sorted (tile, depth) keys with their values, and per-tile ranges
bit-exact; pixel colours within 1e-4 max-abs (final transmittance likewise)
and the per-pixel contributor count exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import fg, synth
from tests.gpu_util import assert_frame_parity, read_frame, run_gpu_frame

pytestmark = pytest.mark.gpu

TINY = synth.tiny_tree(0)


@pytest.fixture(scope="module")
def tiny_dev():
    return fg.DeviceTree(TINY)


@pytest.mark.parametrize("dist,tau_R", [(25.0, 3.0), (25.0, 30.0), (100.0, 10.0), (100.0, 30.0), (400.0, 3.0),
                                        (25.0, 1e9), (400.0, 100.0)])
@pytest.mark.parametrize("tau", [0.0, 1 / 255, 0.05])
def test_tiny_tree(tiny_dev, dist, tau_R, tau):
    cam = synth.tiny_camera(dist)
    g = run_gpu_frame(TINY, cam, tau_R, tau, dtree=tiny_dev)
    o = oracle.render_frame(TINY, cam, tau_R, tau)
    assert_frame_parity(g, o)


@pytest.mark.parametrize("seed", range(8))
def test_random_forests(seed):
    tree = synth.random_tree(seed, n_roots=1 + seed % 4, max_depth=3 + seed % 4, sh_degree=seed % 4)
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2 + rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3)),
                            (rng.uniform(-3, 3), -rng.uniform(10, 60), rng.uniform(-3, 3)),
                            int(rng.integers(40, 400)), int(rng.integers(40, 300)))
    tau_R = float(rng.choice([1.0, 3.0, 10.0, 30.0]))
    tau = float(rng.choice([0.0, 1 / 255, 0.02]))
    g = run_gpu_frame(tree, cam, tau_R, tau, bg=(0.1, 0.2, 0.3))
    o = oracle.render_frame(tree, cam, tau_R, tau, bg=(0.1, 0.2, 0.3))
    assert_frame_parity(g, o)


def test_ragged_image_and_city_block():
    spec = synth.CitySpec(n_leaves=60_000, box=(30, 30, 8), n_blobs=6, blob_sigma=(5, 5, 2),
                          leaf_log_scale_mu=-2.5, seed=5)
    tree = synth.city_tree(spec)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, np.radians(-25)), (0, -45, 15), 1000, 562)
    for tau in (0.0, 0.02):
        g = run_gpu_frame(tree, cam, 3.0, tau)
        o = oracle.render_frame(tree, cam, 3.0, tau)
        assert o["sel_idx"].size > 1000 and o["keys"].size > 1000
        assert_frame_parity(g, o)


# tiles of at least this many chunks are blended as two half-tile items with
# two lanes per pixel; shorter multi-chunk tiles as one item, one lane per pixel
SPLIT_CHUNKS = 16


@pytest.mark.parametrize("n", [12000, 30000])
@pytest.mark.parametrize("opacity_logit_mu", [-3.0, 1.0])
def test_heavy_tiles_chunked_blend(opacity_logit_mu, n):
    """Thousands of small splats on a few tiles: multi-chunk tiles hand the pixel
    state over between work items; translucent (no termination) and opaque
    (termination inside a later chunk) variants. The denser scene has, at
    every chunk size but 512, both tiles long enough to be split over two
    work items and shorter multi-chunk tiles. The counting variant of the
    blend renders the same frame, and its count of blended fragments does not
    depend on the chunk size or on the split."""
    rng = np.random.default_rng(7)
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 200, 120)
    z = rng.uniform(20, 60, n)
    px = rng.uniform(60, 110, n)
    py = rng.uniform(40, 80, n)
    mean = np.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z], 1)
    scale = np.exp(rng.normal(-3.2, 0.4, (n, 3))) * z[:, None] / 40
    q = rng.standard_normal((n, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = 1 / (1 + np.exp(-rng.normal(opacity_logit_mu, 1.0, n)))
    sh = rng.normal(0, 0.3, (n, 1, 3))
    from tests.helpers import flat_tree
    tree = flat_tree(mean, scale, q, op, sh)
    o = oracle.render_frame(tree, cam, 3.0, 0.0)
    L = (o["ranges"][:, 1].astype(np.int64) - o["ranges"][:, 0])
    assert L.max() > 2048
    for chunk in ((128, 256) if n > 12000 else (128,)):
        nch = (L + chunk - 1) // chunk
        assert np.any(nch >= SPLIT_CHUNKS) and np.any((nch > 1) & (nch < SPLIT_CHUNKS)), chunk
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, tree.n_nodes, 1 << 22)
    blended = set()
    # mask_items > 0 caps the stored chunk masks: the chunks past the cap
    # compute their masks inside the blend, wave by wave
    for chunk, mask_items in ((128, 0), (256, 0), (512, 0), (256, 3), (512, 1)):
        tune = fg.tune_struct(chunk, 0, mask_items=mask_items)
        fg.render_frame(dt, cam, fb, 3.0, 0.0, tune=tune)
        torch.cuda.synchronize()
        assert_frame_parity(read_frame(fb, tree.n_nodes), o)
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        fg.render_stage(cam, fb, tune=tune, frag_stats=stats)
        torch.cuda.synchronize()
        assert_frame_parity(read_frame(fb, tree.n_nodes), o)
        blended.add(int(stats[3].item()))
    assert len(blended) == 1 and blended.pop() > 0


def test_heavy_tiles_on_the_ragged_corner():
    """Long tiles on the image's ragged right column and bottom row (200 x 120
    px: the last tile column and row are half outside), the longest on the
    corner tile: split tiles whose lower half item has no pixel inside, and
    split and unsplit tiles with a part of their columns outside."""
    rng = np.random.default_rng(9)
    n = 20000
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 200, 120)
    z = rng.uniform(20, 60, n)
    px = rng.uniform(186, 204, n)
    py = rng.uniform(106, 124, n)
    mean = np.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z], 1)
    scale = np.exp(rng.normal(-3.2, 0.4, (n, 3))) * z[:, None] / 40
    q = rng.standard_normal((n, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = 1 / (1 + np.exp(-rng.normal(-3.0, 1.0, n)))
    from tests.helpers import flat_tree
    tree = flat_tree(mean, scale, q, op, rng.normal(0, 0.3, (n, 1, 3)))
    o = oracle.render_frame(tree, cam, 3.0, 0.0)
    L = o["ranges"][:, 1].astype(np.int64) - o["ranges"][:, 0]
    Wt = (cam.width + 15) // 16
    corner = ((cam.height + 15) // 16 - 1) * Wt + Wt - 1
    assert L[corner] == L.max() and (L[corner] + 255) // 256 >= SPLIT_CHUNKS
    nch = (L + 255) // 256
    assert np.any((nch > 1) & (nch < SPLIT_CHUNKS))
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, tree.n_nodes, 1 << 22)
    blended = set()
    for chunk, mask_items in ((128, 0), (256, 0), (512, 0), (256, 5)):
        tune = fg.tune_struct(chunk, 0, mask_items=mask_items)
        fg.render_frame(dt, cam, fb, 3.0, 0.0, tune=tune)
        torch.cuda.synchronize()
        assert_frame_parity(read_frame(fb, tree.n_nodes), o)
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        fg.render_stage(cam, fb, tune=tune, frag_stats=stats)
        torch.cuda.synchronize()
        blended.add(int(stats[3].item()))
    assert len(blended) == 1 and blended.pop() > 0


def test_empty_view_and_single_node():
    cam = synth.tiny_camera(25)
    away = synth.make_camera(np.diag([1.0, -1.0, -1.0]), (0, 0, -25), 64, 48)  # looking away from the tree
    g = run_gpu_frame(TINY, away, 3.0, 0.0, bg=(0.5, 0.25, 1.0))
    assert g["n_sel"] == 0 and g["n_pairs"] == 0
    assert np.all(g["image"][0] == 0.5) and np.all(g["image"][2] == 1.0) and np.all(g["n_contrib"] == 0)
    one = synth.random_tree(3, n_roots=1, max_depth=0)
    g = run_gpu_frame(one, cam, 3.0, 0.0)
    o = oracle.render_frame(one, cam, 3.0, 0.0)
    assert_frame_parity(g, o)


def test_tune_knobs_do_not_change_results(tiny_dev):
    cam = synth.tiny_camera(25)
    ref = run_gpu_frame(TINY, cam, 3.0, 1 / 255, dtree=tiny_dev)
    for rb in (4, 5, 6, 7, 8):
        for B in (128, 256, 512):
            g = run_gpu_frame(TINY, cam, 3.0, 1 / 255, dtree=tiny_dev, tune=fg.tune_struct(B, rb))
            for k in ("tile_keys", "vals", "ranges", "image", "final_T", "n_contrib"):
                assert np.array_equal(g[k], ref[k]), (rb, B, k)


def test_run_twice_bitwise_identical(tiny_dev):
    cam = synth.tiny_camera(100)
    a = run_gpu_frame(TINY, cam, 10.0, 0.02, dtree=tiny_dev)
    b = run_gpu_frame(TINY, cam, 10.0, 0.02, dtree=tiny_dev)
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_overflow_reports_required_sizes(tiny_dev):
    cam = synth.tiny_camera(25)
    o = oracle.render_frame(TINY, cam, 3.0, 0.0)
    g = run_gpu_frame(TINY, cam, 3.0, 0.0, dtree=tiny_dev, cap_sel=100)
    assert g["status"] & fg.FG_STATUS_SEL_OVERFLOW and g["n_sel"] == o["sel_idx"].size
    assert np.array_equal(g["sel_idx"], o["sel_idx"][:100])
    g = run_gpu_frame(TINY, cam, 3.0, 0.0, dtree=tiny_dev, cap_pairs=1000)
    assert g["status"] == fg.FG_STATUS_PAIR_OVERFLOW and g["n_pairs"] == o["keys"].size


def test_invalid_arguments_are_rejected(tiny_dev):
    cam = synth.tiny_camera(25)
    fb = fg.FrameBuffers(tiny_dev, cam.width, cam.height, 100, 1000)
    with pytest.raises(fg.FgError):
        fg.fg_filter(tiny_dev, cam, 3.0, fb.sel_bits, fb.sel_idx, fb.cap_sel, fb.n_sel, fb.status, fb.filter_ws[:8])
    with pytest.raises(fg.FgError):
        fg.fg_sort(fb.splats, fb.n_sel, fb.cap_sel, cam, fb.tile_keys, fb.vals, fb.cap_pairs, fb.n_pairs, fb.ranges,
                   fb.status, fb.sort_ws, fg.tune_struct(0, 9))
    torch.cuda.synchronize()
