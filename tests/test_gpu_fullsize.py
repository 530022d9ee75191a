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


# ---------------------------------------------------------------------------
# The filter's per-block leaf boxes (fg_tree_boxes): they skip blocks of leaves
# outside every view and must change no selection.
# ---------------------------------------------------------------------------
BLOCK = 2048  # nodes per filter block (one box each)
GROUP = 256   # nodes per ancestor-walk group (one child range each)


def boxes_of(dtree):
    nb = (dtree.n_nodes + BLOCK - 1) // BLOCK
    return dtree.tile_box[:8 * nb].cpu().numpy().reshape(-1, 8)


def cranges_of(dtree):
    nb = (dtree.n_nodes + BLOCK - 1) // BLOCK
    return dtree.tile_box[8 * nb:].cpu().numpy().view(np.int32).reshape(-1, 2)


def host_cranges(tree):
    """Child index ranges per group of 256 nodes below span, by definition:
    min/max index of the nodes whose parent link is well formed (p < n,
    p < span) and points into the group; (INT32_MAX, -1) without children;
    (-1, -1) when a node of the group below span has a parent chain that is
    malformed or longer than max_depth."""
    N, span = tree.n_nodes, tree.n_internal_span
    ng = (span + GROUP - 1) // GROUP
    out = np.empty((ng, 2), np.int64)
    out[:, 0], out[:, 1] = np.iinfo(np.int32).max, -1
    n = np.arange(N)
    p = tree.parent.astype(np.int64)
    ok = (p >= 0) & (p < n) & (p < span)
    g = p[ok] // GROUP
    np.minimum.at(out[:, 0], g, n[ok])
    np.maximum.at(out[:, 1], g, n[ok])
    # chain walk of every node below span, as the filter's ancestor walk
    a = np.arange(span)
    cur = p[:span].copy()
    bad = np.zeros(span, bool)
    live = cur >= 0
    for hops in range(64):
        if not live.any():
            break
        idx = np.nonzero(live)[0]
        c, prev = cur[idx], a[idx]
        b = (c >= prev) | (c >= span) | (hops >= tree.max_depth)
        bad[idx[b]] = True
        live[idx[b]] = False
        go = idx[~b]
        a[go] = cur[go]
        cur[go] = p[cur[go]]
        live[go] = cur[go] >= 0
    out[np.unique(np.nonzero(bad)[0] // GROUP)] = -1
    return out.astype(np.int32)


def host_boxes(tree):
    """The boxes by their definition, in numpy: min/max of the means of a
    block's nodes; NaN for a block holding a parent link the filter rejects
    (p >= n or p >= span)."""
    N, span = tree.n_nodes, tree.n_internal_span
    nb = (N + BLOCK - 1) // BLOCK
    out = np.full((nb, 8), np.nan, np.float32)
    mean = tree.mean.astype(np.float32)
    n = np.arange(N)
    p = tree.parent.astype(np.int64)
    bad = (p >= 0) & ((p >= n) | (p >= span))
    for b in range(nb):
        lo, hi = b * BLOCK, min(N, (b + 1) * BLOCK)
        if bad[lo:hi].any():
            continue
        out[b, 0:3] = mean[:, lo:hi].min(axis=1)
        out[b, 4:7] = mean[:, lo:hi].max(axis=1)
        out[b, 3] = out[b, 7] = 0.0
    return out


def outside64(cam, lo, hi, margin_scale=1e-5):
    """The boxes the filter may skip, in float64 with the filter's margin: every
    point of the box outside one frustum plane by 1e-5 (1 + k) S."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    S = np.abs(c).sum(1) + h.sum(1) + np.abs(t).sum()
    out = np.zeros(len(lo), bool)
    planes = [(-R[2], cam.znear - t[2], 1.0)]
    for row, k, tt in ((0, cam.kx, t[0]), (1, cam.ky, t[1])):
        for sgn in (1.0, -1.0):
            planes.append((sgn * R[row] - k * R[2], sgn * tt - k * t[2], 1.0 + k))
    for a, b, f in planes:
        lmin = c @ a + b - h @ np.abs(a)
        out |= lmin > margin_scale * f * S
    return out & np.isfinite(lo).all(1) & np.isfinite(hi).all(1)


def selection(dtree, cam, use_boxes):
    saved = dtree.tile_box
    if not use_boxes:
        dtree.tile_box = None
    try:
        fb = fg.FrameBuffers(dtree, cam.width, cam.height, cap_sel=8_000_000, cap_pairs=1)
        fg.filter_stage(dtree, cam, fb, synth.TAU_R)
        torch.cuda.synchronize()
    finally:
        dtree.tile_box = saved
    n_sel, _, status = fg.read_counts(fb)
    return fb.sel_bits.cpu().numpy().copy(), fb.sel_idx[:n_sel].cpu().numpy().copy(), status


def test_tile_boxes_match_their_definition(city1m):
    tree, dtree, _ = city1m
    gpu = boxes_of(dtree)
    ref = host_boxes(tree)
    assert gpu.shape == ref.shape
    assert np.array_equal(np.isnan(gpu), np.isnan(ref))
    assert np.array_equal(np.nan_to_num(gpu), np.nan_to_num(ref))
    assert np.isfinite(ref[:, 0]).all()
    assert np.array_equal(cranges_of(dtree), host_cranges(tree))


def test_tile_boxes_change_no_selection_on_the_flythrough(city):
    """Eight frames of the fly-through (single views) and the 8 training views
    in one pass: selection words and lists are identical with and without the
    boxes, and the boxes let the filter skip a large share of the blocks."""
    tree, dtree, _ = city
    frames = synth.city20m_frames(64)
    box = boxes_of(dtree)
    skipped = []
    for k in range(0, 64, 8):
        a = selection(dtree, frames[k], True)
        b = selection(dtree, frames[k], False)
        assert a[2] == 0 and b[2] == 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), k
        skipped.append(outside64(frames[k], box[:, 0:3].astype(np.float64), box[:, 4:7].astype(np.float64)).mean())
    assert min(skipped) > 0.2, skipped
    # eight views in one node-major pass: a block is skipped only when it is
    # outside all of them
    views = synth.city20m_training_views(8)
    got = [multiview_selection(dtree, views, use) for use in (True, False)]
    assert np.array_equal(got[0][0], got[1][0]) and np.array_equal(got[0][1], got[1][1])
    assert got[0][2] == 0


def multiview_selection(dtree, cams, use_boxes):
    nv, N = len(cams), dtree.n_nodes
    words, cap = (N + 31) // 32, 8_000_000
    sel_bits = torch.empty(nv * words, dtype=torch.int32, device="cuda")
    sel_idx = torch.empty(nv * cap, dtype=torch.int32, device="cuda")
    n_sel = torch.zeros(nv, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(fg.fg_filter_workspace_size(N, dtree.n_internal_span, nv), dtype=torch.uint8, device="cuda")
    saved = dtree.tile_box
    if not use_boxes:
        dtree.tile_box = None
    try:
        fg.fg_filter(dtree, cams, synth.TAU_R, sel_bits, sel_idx, cap, n_sel, status, ws)
        torch.cuda.synchronize()
    finally:
        dtree.tile_box = saved
    ns = n_sel.cpu().numpy().view(np.uint32)
    idx = sel_idx.cpu().numpy().view(np.uint32).reshape(nv, cap)
    lists = np.concatenate([idx[v, :min(int(ns[v]), cap)] for v in range(nv)])
    return sel_bits.cpu().numpy(), np.concatenate([ns.astype(np.int64), lists.astype(np.int64)]), int(status.item())


def test_bad_parent_in_a_skipped_leaf_block_is_reported(city1m):
    """A malformed parent link of a leaf in a block of leaves that lies
    outside the view (so only the selection pass would see it): the block
    gets no box, so the filter still reads it and reports
    FG_STATUS_BAD_PARENT."""
    import dataclasses
    tree, dtree, _ = city1m
    cam = synth.city1m_camera()
    box = boxes_of(dtree)
    out = outside64(cam, box[:, 0:3].astype(np.float64), box[:, 4:7].astype(np.float64))
    out &= np.arange(out.size) * BLOCK >= tree.n_internal_span
    assert out.any()
    blk = int(np.nonzero(out)[0][len(np.nonzero(out)[0]) // 2])
    j = blk * BLOCK + 7
    bad = tree.parent.copy()
    bad[j] = j  # a node as its own parent
    t2 = dataclasses.replace(tree, parent=bad)
    d2 = fg.DeviceTree(t2)
    assert np.isnan(boxes_of(d2)[blk]).all()
    fb = fg.FrameBuffers(d2, cam.width, cam.height, cap_sel=2_000_000, cap_pairs=1)
    fg.filter_stage(d2, cam, fb, synth.TAU_R)
    torch.cuda.synchronize()
    assert fg.read_counts(fb)[2] & fg.FG_STATUS_BAD_PARENT
