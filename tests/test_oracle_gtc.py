"""Pins of the oracle's GTC pre-pass (Sec. 3.3, Eqs. (5)-(8)).

* Eq. (5) telescopes: along a pixel's blend chain the sum of alpha_k T_k is
  1 - T_final, up to the float32 rounding of the transmittance products (at
  most 2^-23 T_k per blended splat), so per tile the KPC of its pairs sums to
  the tile's total 1 - final_T. KPC credited to skipped splats (alpha < 1/255)
  or to the splat that would cross the termination threshold breaks this.
* closed forms in float64 for one Gaussian (KPC = sum of alpha over the tile's
  pixels, T = 1), for two overlapping Gaussians (the back one is weighted by
  1 - alpha of the front one) and for an opaque stack whose third splat would
  take T below 1e-4 (it and everything behind it get KPC 0);
* Eq. (6)/(7) on hand-built ranges: zero-KPC pairs count in a tile's mean,
  tiles without pairs are left out of the view mean, a view without pairs is
  undefined;
* Eq. (8): tau = lambda_G / G_bar for a two-view scene, against a float64
  brute force (each tile's Gaussians found by testing every 3-sigma
  rectangle, ordered by depth, blended per pixel).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2603_23891_amd import synth
from tests.helpers import flat_tree

F32 = np.float32


def per_tile(values, ranges):
    r = np.asarray(ranges).reshape(-1, 2).astype(np.int64)
    return np.array([values[lo:hi].sum() for lo, hi in r])


def tile_pixel_sums(img2d, cam):
    H, W = img2d.shape
    out = np.zeros(cam.n_tiles)
    for ty in range(cam.tiles_y):
        for tx in range(cam.tiles_x):
            out[ty * cam.tiles_x + tx] = img2d[ty * 16:min(H, ty * 16 + 16), tx * 16:min(W, tx * 16 + 16)].sum()
    return out


@pytest.mark.parametrize("dist,tau_R", [(25.0, 3.0), (100.0, 10.0), (400.0, 3.0)])
def test_kpc_telescopes_to_one_minus_T_tiny(dist, tau_R):
    tree = synth.tiny_tree(0)
    cam = synth.tiny_camera(dist)
    out = oracle.render_frame(tree, cam, tau_R, 0.0)
    k = oracle.kpc(out["splats"], out["vals"], out["ranges"], cam)
    assert k.size == out["vals"].size and k.min() >= 0.0
    got = per_tile(k, out["ranges"])
    want = tile_pixel_sums(1.0 - out["final_T"].astype(np.float64), cam)
    bound = tile_pixel_sums(out["n_contrib"].astype(np.float64), cam) * 2.0 ** -23 + 1e-12
    assert np.all(np.abs(got - want) <= bound), np.abs(got - want).max()
    assert want.sum() > 100.0  # the frame is not nearly empty


@pytest.mark.parametrize("seed", range(4))
def test_kpc_telescopes_random_forest(seed):
    tree = synth.random_tree(seed, n_roots=2, max_depth=4, sh_degree=0)
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2 + rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2)),
                            (rng.uniform(-2, 2), -rng.uniform(15, 40), rng.uniform(-2, 2)), 200, 136)
    out = oracle.render_frame(tree, cam, 3.0, 0.0)
    k = oracle.kpc(out["splats"], out["vals"], out["ranges"], cam)
    got = per_tile(k, out["ranges"])
    want = tile_pixel_sums(1.0 - out["final_T"].astype(np.float64), cam)
    bound = tile_pixel_sums(out["n_contrib"].astype(np.float64), cam) * 2.0 ** -23 + 1e-12
    assert np.all(np.abs(got - want) <= bound)


# ---------------------------------------------------------------------------
# float64 brute force over isotropic Gaussians (q = identity)
# ---------------------------------------------------------------------------
def brute_kpc64(mean, s, o, cam):
    """{(tile, gaussian): KPC} in float64, and the smallest relative margin of
    any skip / clamp / termination decision (float32 may only be trusted where
    that margin is far above its rounding)."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    pc = mean @ R.T + np.asarray(cam.t, np.float64)
    n = mean.shape[0]
    x, y, z = pc[:, 0], pc[:, 1], pc[:, 2]
    u = cam.fx * x / z + cam.cx
    v = cam.fy * y / z + cam.cy
    rects, Q = [], []
    for i in range(n):
        J = np.array([[cam.fx / z[i], 0.0, -cam.fx * x[i] / z[i] ** 2], [0.0, cam.fy / z[i], -cam.fy * y[i] / z[i] ** 2]])
        S2 = s[i] ** 2 * (J @ J.T) + 0.3 * np.eye(2)
        Q.append(np.linalg.inv(S2))
        r = 3.0 * math.sqrt(np.linalg.eigvalsh(S2).max())
        x0 = max(0, math.floor((u[i] - r) / 16)); x1 = min(cam.tiles_x, math.floor((u[i] + r) / 16) + 1)
        y0 = max(0, math.floor((v[i] - r) / 16)); y1 = min(cam.tiles_y, math.floor((v[i] + r) / 16) + 1)
        rects.append((x0, y0, x1, y1))
    order = sorted(range(n), key=lambda i: (z[i], i))
    kpc, margin = {}, np.inf
    for ty in range(cam.tiles_y):
        for tx in range(cam.tiles_x):
            t = ty * cam.tiles_x + tx
            members = [i for i in order if rects[i][0] <= tx < rects[i][2] and rects[i][1] <= ty < rects[i][3]]
            for i in members:
                kpc[(t, i)] = 0.0
            for py in range(ty * 16, min(cam.height, ty * 16 + 16)):
                for px in range(tx * 16, min(cam.width, tx * 16 + 16)):
                    T = 1.0
                    for i in members:
                        d = np.array([u[i] - (px + 0.5), v[i] - (py + 0.5)])
                        power = -0.5 * d @ Q[i] @ d
                        a = o[i] * math.exp(power)
                        margin = min(margin, abs(a - 0.99) / 0.99, abs(a * 255.0 - 1.0))
                        a = min(0.99, a)
                        if a < 1.0 / 255.0:
                            continue
                        Tn = T * (1.0 - a)
                        margin = min(margin, abs(Tn - 1e-4) / 1e-4)
                        if Tn < 1e-4:
                            break
                        kpc[(t, i)] += a * T
                        T = Tn
    return kpc, margin


def oracle_kpc_pairs(mean, s, o, cam, tau_R=1e30):
    n = mean.shape[0]
    tree = flat_tree(mean, np.repeat(np.asarray(s, np.float64)[:, None], 3, 1), np.tile([1.0, 0, 0, 0], (n, 1)), o,
                     np.zeros((n, 1, 3)))
    out = oracle.render_frame(tree, cam, tau_R, 0.0)
    k = oracle.kpc(out["splats"], out["vals"], out["ranges"], cam)
    pairs = {}
    for t, (lo, hi) in enumerate(out["ranges"].astype(np.int64)):
        for j in range(lo, hi):
            pairs[(t, int(out["sel_idx"][out["vals"][j]]))] = k[j]
    return pairs, out, k


def assert_pairs_match(got, want, rtol=2e-5, atol=1e-6):
    assert set(got) == set(want)
    for key, w in want.items():
        assert abs(got[key] - w) <= atol + rtol * abs(w), (key, got[key], w)


def on_axis_mean(cam, u, v, z):
    """World point (R = identity camera) that projects to pixel position (u, v) at depth z."""
    return np.array([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z]) - np.asarray(cam.t, np.float64)


def test_single_gaussian_kpc_is_sum_of_alpha():
    cam = synth.tiny_camera(25.0)
    mean = on_axis_mean(cam, 58.3, 61.7, 25.0)[None]
    s, o = np.array([0.12]), np.array([0.8])
    want, margin = brute_kpc64(mean, s, o, cam)
    assert margin > 1e-4
    got, out, _ = oracle_kpc_pairs(mean, s, o, cam)
    assert len(want) >= 2  # its 3-sigma rectangle spans several tiles
    assert_pairs_match(got, want)
    # T = 1 for a single splat: its KPC over the frame is the whole 1 - T
    assert abs(sum(got.values()) - (1.0 - out["final_T"].astype(np.float64)).sum()) < 1e-4


def test_two_gaussians_back_one_weighted_by_front():
    cam = synth.tiny_camera(25.0)
    mean = np.stack([on_axis_mean(cam, 100.0, 40.0, 25.0), on_axis_mean(cam, 102.5, 42.0, 27.0)])
    s, o = np.array([0.15, 0.2]), np.array([0.7, 0.9])
    want, margin = brute_kpc64(mean, s, o, cam)
    assert margin > 1e-4
    got, _, _ = oracle_kpc_pairs(mean, s, o, cam)
    assert_pairs_match(got, want)
    # the back splat loses weight to the front one on their shared tile
    t = (40 // 16) * cam.tiles_x + 100 // 16
    front_alone, _ = brute_kpc64(mean[1:], s[1:], o[1:], cam)
    assert got[(t, 1)] < 0.9 * front_alone[(t, 0)]


def test_terminated_splats_get_no_kpc():
    # four huge, nearly opaque Gaussians over tile (3, 3) one behind another:
    # T goes 1 -> ~0.02 -> ~4e-4; the third would take it to ~8e-6 < 1e-4, so
    # it and the fourth are never blended and receive nothing
    cam = synth.tiny_camera(25.0)
    mean = np.stack([on_axis_mean(cam, 56.0, 56.0, 25.0 + i) for i in range(4)])
    s, o = np.full(4, 12.0), np.full(4, 0.98)
    want, margin = brute_kpc64(mean, s, o, cam)
    assert margin > 1e-4
    got, out, _ = oracle_kpc_pairs(mean, s, o, cam)
    assert_pairs_match(got, want)
    t = 3 * cam.tiles_x + 3
    assert got[(t, 2)] == 0.0 and got[(t, 3)] == 0.0
    assert got[(t, 0)] > 0.97 * 256 and 0.01 * 256 < got[(t, 1)] < 0.03 * 256
    assert np.all(out["n_contrib"][48:64, 48:64] == 2)


def test_tile_and_view_gtc_hand_built():
    kpc = np.array([1.0, 0.0, 3.0, 0.0, 0.0, 2.5])
    ranges = np.array([[0, 2], [0, 0], [2, 5], [5, 6]])
    g = oracle.tile_gtc(kpc, ranges)
    assert g[0] == 0.5 and np.isnan(g[1]) and g[2] == 1.0 and g[3] == 2.5
    assert oracle.gtc_view(kpc, ranges) == pytest.approx((0.5 + 1.0 + 2.5) / 3, rel=1e-15)
    assert oracle.gtc_view(np.zeros(0), np.zeros((4, 2))) is None


def two_view_scene():
    rng = np.random.default_rng(5)
    n = 6
    mean = np.concatenate([rng.uniform(-4.0, 4.0, (n, 2)), rng.uniform(-2.0, 2.0, (n, 1))], 1)
    s = rng.uniform(0.08, 0.35, n)
    o = rng.uniform(0.3, 0.95, n)
    front = synth.tiny_camera(25.0)
    back = synth.make_camera(np.diag([-1.0, 1.0, -1.0]), (0.0, 0.0, 25.0), 256, 256)  # from the far side
    return mean, s, o, [front, back]


def test_scene_tau_two_views_against_brute_force():
    mean, s, o, cams = two_view_scene()
    lam = 0.2
    gv = []
    for cam in cams:
        pairs, margin = brute_kpc64(mean, s, o, cam)
        assert margin > 1e-4
        tiles = {}
        for (t, i), k in pairs.items():
            tiles.setdefault(t, []).append(k)
        gv.append(np.mean([np.mean(v) for v in tiles.values()]))
    n = mean.shape[0]
    tree = flat_tree(mean, np.repeat(s[:, None], 3, 1), np.tile([1.0, 0, 0, 0], (n, 1)), o, np.zeros((n, 1, 3)))
    r = oracle.scene_tau(tree, cams, lam, tau_R=1e30)
    assert r["G_views"] == pytest.approx(gv, rel=2e-5)
    assert r["tau"] == pytest.approx(lam / np.mean(gv), rel=2e-5)
    assert gv[0] != pytest.approx(gv[1], rel=1e-2)  # the two views differ (depth order flips)


def test_scene_tau_leaves_out_views_without_pairs():
    mean, s, o, cams = two_view_scene()
    away = synth.make_camera(np.diag([1.0, -1.0, -1.0]), (0.0, 0.0, -25.0), 64, 48)  # sees nothing
    n = mean.shape[0]
    tree = flat_tree(mean, np.repeat(s[:, None], 3, 1), np.tile([1.0, 0, 0, 0], (n, 1)), o, np.zeros((n, 1, 3)))
    a = oracle.scene_tau(tree, cams, 0.2, tau_R=1e30)
    b = oracle.scene_tau(tree, cams + [away], 0.2, tau_R=1e30)
    assert b["G_views"][2] is None and b["tau"] == a["tau"]
    with pytest.raises(ValueError):
        oracle.scene_tau(tree, [away], 0.2, tau_R=1e30)
