"""GPU parity on degenerate node attributes: NaN and infinite positions,
infinite, zero and huge scales, zero and NaN quaternions, opacities of 0,
1.5 and NaN, and NaN or infinite SH coefficients, in leaves and internal
nodes of a random forest. The frame completes with status 0 and matches the
oracle: selections, splat records, keys, ranges and contributor counts bit
for bit; colours and transmittance bit for bit where finite, and NaN in the
same places (the NaN bit patterns of the host and the GPU differ)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2603_23891_amd import synth
from tests.gpu_util import bits, run_gpu_frame

pytestmark = pytest.mark.gpu


def degenerate_tree(seed):
    tree = synth.random_tree(seed, n_roots=2, max_depth=4, sh_degree=3)
    mean, scale, quat, op, sh = (tree.mean.copy(), tree.scale.copy(), tree.quat.copy(), tree.opacity.copy(),
                                 tree.sh.copy())
    rng = np.random.default_rng(seed)
    L = rng.permutation(np.nonzero(tree.flags & 1)[0])[:12]
    mean[:, L[0]] = np.nan
    mean[2, L[1]] = np.inf
    scale[:, L[2]] = np.inf
    scale[:, L[3]] = 0.0
    quat[:, L[4]] = 0.0
    quat[1, L[5]] = np.nan
    op[L[6]] = 0.0
    op[L[7]] = 1.5
    op[L[8]] = np.nan
    sh[L[9]] = np.nan
    sh[L[10]] = np.inf
    scale[0, L[11]] = 1e30
    I = rng.permutation(np.nonzero((tree.flags & 1) == 0)[0])[:3]
    scale[:, I[0]] = np.inf
    mean[:, I[1]] = np.nan
    quat[:, I[2]] = 0.0
    return dataclasses.replace(tree, mean=mean, scale=scale, quat=quat, opacity=op, sh=sh)


def same_or_both_nan(a, b):
    a, b = np.ascontiguousarray(a, np.float32), np.ascontiguousarray(b, np.float32)
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(bits(a)[~na], bits(b)[~nb])


@pytest.mark.parametrize("seed", [2, 5])
@pytest.mark.parametrize("tau", [0.0, 0.02])
def test_degenerate_attributes(seed, tau):
    tree = degenerate_tree(seed)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, -0.2), (0, -30, 4), 320, 240)
    bg = (0.1, 0.2, 0.3)
    g = run_gpu_frame(tree, cam, 3.0, tau, bg=bg)
    o = oracle.render_frame(tree, cam, 3.0, tau, bg=bg)
    assert g["status"] == 0
    assert o["sel_idx"].size > 50 and o["keys"].size > 100
    assert np.array_equal(g["sel_mask"], o["sel_mask"])
    assert np.array_equal(g["sel_idx"], o["sel_idx"])
    sp = o["splats"]
    assert np.array_equal(g["tiles"], sp["tiles"])
    assert np.array_equal(g["rect"].astype(np.int64), np.stack([sp["x0"], sp["y0"], sp["x1"], sp["y1"]], 1))
    assert same_or_both_nan(g["xy"], np.stack([sp["u"], sp["v"]], 1))
    assert same_or_both_nan(g["conic_o"], np.stack([sp["A"], sp["B"], sp["C"], sp["opacity"]], 1))
    assert same_or_both_nan(g["rgb_depth"], np.stack([sp["r"], sp["g"], sp["b"], sp["depth"]], 1))
    assert np.array_equal(g["vals"], o["vals"])
    assert np.array_equal(g["ranges"].reshape(-1, 2), o["ranges"])
    assert np.array_equal(g["n_contrib"], o["n_contrib"])
    assert same_or_both_nan(g["image"], o["image"])
    assert same_or_both_nan(g["final_T"], o["final_T"])
