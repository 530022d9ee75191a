"""GPU parity at the benchmark's full size, in the launch configuration the
bench times: the 20,000,003-node city tree at 1920x1080 with the calibrated
GTC threshold and the bench's capacities (frames of the fly-through), two
views of the 32-view batch (720p and 2160p, global tile ids) through the
batched renderer, and the single 1080p view of the 1M-leaf city (1.14M
nodes) with and without the shrink, at every chunk size. Same bar as the
small cases: selection, splats, keys, ranges and contributor counts
bit-exact, colours within 1e-4.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import batch, fg, synth
from tests.gpu_util import assert_frame_parity, read_frame

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def city():
    tree = synth.city_tree(synth.CITY20M)
    with open(os.path.join(ROOT, "tests", "golden", "city_tau.json")) as f:
        tau = float(json.load(f)["city20m"]["tau"])
    return tree, fg.DeviceTree(tree), tau


@pytest.mark.parametrize("frame", [0, 32])
def test_flythrough_frame_full_size(city, frame):
    tree, dtree, tau = city
    cam = synth.city20m_frames(64)[frame]
    fb = fg.FrameBuffers(dtree, cam.width, cam.height, cap_sel=8_000_000, cap_pairs=48_000_000)
    fg.render_frame(dtree, cam, fb, synth.TAU_R, tau)
    torch.cuda.synchronize()
    g = read_frame(fb, tree.n_nodes)
    o = oracle.render_frame(tree, cam, synth.TAU_R, tau)
    assert o["sel_idx"].size > 100_000 and o["keys"].size > 100_000
    assert_frame_parity(g, o)


def test_batch_views_full_size(city):
    """The whole 32-view batch (720p to 2160p, global tile ids) as the bench
    runs it: one filter, projection, sort and blend for all views. Three
    views (the first 720p, 1080p and 2160p ones) against the oracle."""
    from tests.test_gpu_batch import check_view, read_view
    tree, dtree, tau = city
    views = synth.city20m_batch_views(32)
    br = batch.BatchedRenderer(dtree, views, cap_sel=8_000_000, cap_pairs=128_000_000, cap_items=64_000_000)
    br.run(synth.TAU_R, tau)
    torch.cuda.synchronize()
    ns, npairs, status = br.counts()
    assert status == 0
    picks = [next(v for v in range(32) if views[v].width == w) for w in (1280, 1920, 3840)]
    for v in picks:
        o = oracle.render_frame(tree, views[v], synth.TAU_R, tau)
        assert o["keys"].size > 100_000
        check_view(read_view(br, v), o)


@pytest.fixture(scope="module")
def city1m():
    tree = synth.city_tree(synth.CITY1M)
    with open(os.path.join(ROOT, "tests", "golden", "city_tau.json")) as f:
        tau = float(json.load(f)["city1m"]["tau"])
    return tree, fg.DeviceTree(tree), tau


@pytest.mark.parametrize("shrink", [False, True])
def test_city1m_single_view(city1m, shrink):
    tree, dtree, tau = city1m
    tau = tau if shrink else 0.0
    cam = synth.city1m_camera()
    o = oracle.render_frame(tree, cam, synth.TAU_R, tau)
    assert o["sel_idx"].size > 100_000 and o["keys"].size > 100_000
    for chunk in (128, 256, 512):
        fb = fg.FrameBuffers(dtree, cam.width, cam.height, cap_sel=2_000_000, cap_pairs=16_000_000)
        fg.render_frame(dtree, cam, fb, synth.TAU_R, tau, tune=fg.tune_struct(chunk))
        torch.cuda.synchronize()
        assert_frame_parity(read_frame(fb, tree.n_nodes), o)


def test_city20m_scene_tau_on_gpu(city):
    """The GTC pre-pass on the GPU over the 8 training views of the 20M-node
    city reproduces the stored per-view GTCs, G_bar and tau (written by the
    oracle's pre-pass); tolerance as in test_gpu_gtc."""
    tree, dtree, tau = city
    views = synth.city20m_training_views(8)
    fb = fg.FrameBuffers(dtree, views[0].width, views[0].height, cap_sel=8_000_000, cap_pairs=48_000_000)
    gb = fg.scene_tau(dtree, views, fb, synth.LAMBDA_G, synth.TAU_R)
    torch.cuda.synchronize()
    assert not gb.status.any(), gb.status
    with open(os.path.join(ROOT, "tests", "golden", "city_tau.json")) as f:
        ref = json.load(f)["city20m"]
    vg = gb.view_gtc.cpu().numpy()
    assert np.all(vg[:, 1] > 0)
    assert np.allclose(vg[:, 0], ref["G_views"], rtol=2e-6, atol=0)
    assert abs(gb.g_bar.item() - ref["G_bar"]) <= 2e-6 * ref["G_bar"]
    assert abs(gb.tau.item() - tau) <= 5e-6 * tau
