"""GPU GTC pre-pass (fg_gtc, fg_gtc_tau) against the CPU oracle.

Per sorted pair, the KPC of Eq. (5); per tile, the GTC of Eq. (6) (NaN where a
tile holds no pair); per view, Eq. (7); and tau of Eq. (8). The GPU adds each
pixel's alpha * T (the same float32 products as the oracle, from the same
transmittance chain) in float32 wave sums, the oracle in float64 in pixel
order, so the bar is a tolerance derived from that summation: a sum of at
most 256 terms in float32 trees of depth <= 10 carries a relative error below
10 * 2^-24 ~ 6e-7 of the sum of its terms; the tests use 2e-6 relative plus
1e-7 absolute for KPC and tile GTC, and 2e-6 for view GTC, G_bar and tau.
At full size, tau of the stored scenes (written by the oracle's pre-pass,
tests/golden/make_tau.py) is reproduced on the GPU.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import fg, synth
from tests.helpers import flat_tree

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RTOL, ATOL = 2e-6, 1e-7
EDGES = [1e-4, 1e-3, 0.01, 0.05, 0.1, 1.0, 10.0]


def golden():
    with open(os.path.join(ROOT, "tests", "golden", "city_tau.json")) as f:
        return json.load(f)


def gpu_view(dtree, cam, fb, tau_R, hist=True, chunked=True):
    """One view through filter, 3-sigma preprocess, sort and fg_gtc (by
    default chunk-parallel, after a blend with saved state)."""
    gb = fg.GtcBuffers(fb, 1)
    fg.filter_stage(dtree, cam, fb, tau_R)
    fg.preprocess_stage(dtree, cam, fb, 0.0)
    fg.sort_stage(cam, fb)
    h = torch.zeros(len(EDGES) + 1, dtype=torch.int32, device="cuda") if hist else None
    fg.gtc_view_stage(cam, fb, gb, 0, EDGES if hist else None, h, chunked=chunked)
    torch.cuda.synchronize()
    n_sel, n_pairs, status = fg.read_counts(fb)
    assert status == 0
    return dict(kpc=gb.kpc[:n_pairs].cpu().numpy().astype(np.float64), tile=gb.tile_gtc.cpu().numpy(),
                view=gb.view_gtc[0].cpu().numpy(), hist=None if h is None else h.cpu().numpy(),
                vals=fb.vals[:n_pairs].cpu().numpy().view(np.uint32), n_pairs=n_pairs)


def oracle_view(tree, cam, tau_R):
    _, sel = oracle.filter(tree, cam, tau_R)
    sp = oracle.preprocess(tree, cam, 0.0, sel)
    keys, vals, ranges = oracle.sort(sp, cam)
    k = oracle.kpc(sp, vals, ranges, cam)
    return dict(kpc=k, vals=vals, ranges=ranges, tile=oracle.tile_gtc(k, ranges), view=oracle.gtc_view(k, ranges))


def assert_gtc_parity(g, o):
    assert np.array_equal(g["vals"], o["vals"]), "the pre-pass walks the oracle's pair order"
    k_o = o["kpc"]
    assert np.all(np.abs(g["kpc"] - k_o) <= RTOL * k_o + ATOL), np.abs(g["kpc"] - k_o).max()
    assert np.array_equal(np.isnan(g["tile"]), np.isnan(o["tile"])), "empty tiles are undefined"
    m = ~np.isnan(o["tile"])
    assert np.all(np.abs(g["tile"][m] - o["tile"][m]) <= RTOL * o["tile"][m] + ATOL)
    if o["view"] is None:
        assert g["view"][1] == 0 and g["view"][0] == 0
    else:
        assert g["view"][1] == m.sum()
        assert abs(g["view"][0] - o["view"]) <= RTOL * o["view"]
    if g["hist"] is not None:
        # binning of the oracle's values; a pair within tolerance of an edge may
        # fall on either side of it
        ref = np.bincount(np.searchsorted(np.asarray(EDGES), k_o, side="right"), minlength=len(EDGES) + 1)
        near = sum(int(np.sum(np.abs(k_o - e) <= RTOL * e + ATOL)) for e in EDGES)
        assert int(np.abs(g["hist"] - ref).sum()) <= 2 * near, (g["hist"], ref)
        assert g["hist"].sum() == k_o.size


TINY = synth.tiny_tree(0)


@pytest.mark.parametrize("dist,tau_R", [(25.0, 3.0), (100.0, 10.0), (400.0, 3.0), (100.0, 30.0), (25.0, 1e9)])
def test_tiny_tree_gtc(dist, tau_R):
    cam = synth.tiny_camera(dist)
    dt = fg.DeviceTree(TINY)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, TINY.n_nodes, 1 << 20)
    g = gpu_view(dt, cam, fb, tau_R)
    o = oracle_view(TINY, cam, tau_R)
    assert o["kpc"].size >= 250
    assert_gtc_parity(g, o)


@pytest.mark.parametrize("seed", range(4))
def test_random_forest_gtc(seed):
    tree = synth.random_tree(seed, n_roots=1 + seed, max_depth=3 + seed, sh_degree=seed % 4)
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2 + rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3)),
                            (rng.uniform(-3, 3), -rng.uniform(10, 60), rng.uniform(-3, 3)),
                            int(rng.integers(40, 400)), int(rng.integers(40, 300)))
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, tree.n_nodes, 1 << 22)
    assert_gtc_parity(gpu_view(dt, cam, fb, 3.0), oracle_view(tree, cam, 3.0))


@pytest.mark.parametrize("opacity_logit_mu", [-3.0, 1.0])
@pytest.mark.parametrize("n", [12000, 30000])
def test_heavy_tiles_gtc(opacity_logit_mu, n):
    """Thousands of small splats on a few tiles, translucent (no termination)
    and opaque (whole tiles terminate: their later pairs get 0 unvisited).
    Both walks: chunk-parallel from the blend's saved state, and one
    workgroup per tile; they also agree with each other to float32 rounding
    of the per-splat sums (the four waves' sums meet in an LDS atomic). In
    the denser scene the longest tiles have 16 or more 256-splat chunks, so
    the blend whose state the chunk-parallel walk starts from splits them
    over two half-tile items."""
    rng = np.random.default_rng(7)
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 200, 120)
    z = rng.uniform(20, 60, n)
    px = rng.uniform(60, 110, n)
    py = rng.uniform(40, 80, n)
    mean = np.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z], 1)
    scale = np.exp(rng.normal(-3.2, 0.4, (n, 3))) * z[:, None] / 40
    q = rng.standard_normal((n, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = 1 / (1 + np.exp(-rng.normal(opacity_logit_mu, 1.0, n)))
    tree = flat_tree(mean, scale, q, op, rng.normal(0, 0.3, (n, 1, 3)))
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, n, 1 << 22)
    g = gpu_view(dt, cam, fb, 3.0)
    o = oracle_view(tree, cam, 3.0)
    L = o["ranges"][:, 1].astype(np.int64) - o["ranges"][:, 0]
    assert L.max() > (15 * 256 if n > 12000 else 2048)
    if opacity_logit_mu > 0:
        assert np.sum(o["kpc"] == 0) > 1000  # pairs behind terminated pixels
    assert_gtc_parity(g, o)
    t = gpu_view(dt, cam, fb, 3.0, chunked=False)
    assert_gtc_parity(t, o)
    assert np.all(np.abs(g["kpc"] - t["kpc"]) <= 1e-6 * np.abs(t["kpc"]) + 1e-9)
    m = ~np.isnan(t["tile"])
    assert np.array_equal(np.isnan(g["tile"]), np.isnan(t["tile"]))
    assert np.all(np.abs(g["tile"][m] - t["tile"][m]) <= 1e-6 * np.abs(t["tile"][m]) + 1e-9)
    assert g["view"][1] == t["view"][1] and abs(g["view"][0] - t["view"][0]) <= 1e-6 * abs(t["view"][0])


def test_city_block_ragged_gtc():
    spec = synth.CitySpec(n_leaves=60_000, box=(30, 30, 8), n_blobs=6, blob_sigma=(5, 5, 2),
                          leaf_log_scale_mu=-2.5, seed=5)
    tree = synth.city_tree(spec)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, np.radians(-25)), (0, -45, 15), 1000, 562)
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, tree.n_nodes, 1 << 23)
    assert_gtc_parity(gpu_view(dt, cam, fb, 3.0), oracle_view(tree, cam, 3.0))


def test_empty_view_and_tau_edge_cases():
    """A view without pairs is undefined (count 0) and left out of G_bar; no
    defined view gives tau = NaN and the status bit; an overflowed sort marks
    its view and reports an overflow."""
    away = synth.make_camera(np.diag([1.0, -1.0, -1.0]), (0, 0, -25), 64, 48)
    near = synth.tiny_camera(100.0)
    dt = fg.DeviceTree(TINY)
    fbs = [fg.FrameBuffers(dt, c.width, c.height, TINY.n_nodes, 1 << 20) for c in (away, near)]
    gb = fg.scene_tau(dt, [away], fbs[0], 0.2, 3.0)
    torch.cuda.synchronize()
    st = gb.status.cpu().numpy().view(np.uint32)
    assert st[1] == fg.FG_STATUS_GTC_UNDEFINED and np.isnan(gb.tau.item()) and gb.g_bar.item() == 0
    assert gb.view_gtc[0, 1].item() == 0
    # one undefined view and one defined one: tau from the defined one alone
    vg = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    gb2 = fg.GtcBuffers(fbs[1], 2)
    for v, (cam, fb) in enumerate(zip((away, near), fbs)):
        gb1 = fg.scene_tau(dt, [cam], fb, 0.2, 3.0)
        vg[v] = gb1.view_gtc[0]
    fg.fg_gtc_tau(vg, 2, 0.2, gb2.g_bar, gb2.tau, gb2.status[2:3])
    r = oracle.scene_tau(TINY, [away, near], 0.2, 3.0)
    torch.cuda.synchronize()
    assert r["G_views"][0] is None
    assert abs(gb2.g_bar.item() - r["G_bar"]) <= RTOL * r["G_bar"]
    assert abs(gb2.tau.item() - r["tau"]) <= 5e-6 * r["tau"]
    # a pair capacity too small for the view: overflow, no tau
    small = fg.FrameBuffers(dt, near.width, near.height, TINY.n_nodes, 100)
    gb3 = fg.scene_tau(dt, [near], small, 0.2, 3.0)
    torch.cuda.synchronize()
    st = gb3.status.cpu().numpy().view(np.uint32)
    assert st[0] & fg.FG_STATUS_PAIR_OVERFLOW and st[1] & fg.FG_STATUS_PAIR_OVERFLOW
    assert gb3.view_gtc[0, 1].item() == -1 and np.isnan(gb3.tau.item())


def test_city1m_tau_full_size():
    """The single 1080p view of the 1M-leaf city (1.14M nodes), compared pair by
    pair with the oracle, and its tau against the stored value."""
    tree = synth.city_tree(synth.CITY1M)
    cam = synth.city1m_camera()
    dt = fg.DeviceTree(tree)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, 2_000_000, 24_000_000)
    g = gpu_view(dt, cam, fb, synth.TAU_R)
    o = oracle_view(tree, cam, synth.TAU_R)
    assert o["kpc"].size > 100_000
    assert_gtc_parity(g, o)
    gb = fg.scene_tau(dt, [cam], fb, synth.LAMBDA_G, synth.TAU_R)
    torch.cuda.synchronize()
    assert not gb.status.any()
    ref = golden()["city1m"]
    assert abs(gb.g_bar.item() - ref["G_bar"]) <= RTOL * ref["G_bar"]
    assert abs(gb.tau.item() - ref["tau"]) <= 5e-6 * ref["tau"]
