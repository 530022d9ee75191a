"""The top-down tree generator follows the canonical recursive construction
of Sec. 3.1: a parent v with rotation R(q_v) and scale s_v has 8 children at
mu_v + R(q_v) o_k, o_k the sign combinations of (s_x/2, s_y/2, s_z/2); each
child's scale is gamma * s_v; rotation, colour (SH) and opacity are the
parent's. Checked node by node in float64 against scipy's rotation of the
stored quaternion, plus the layout the C-ABI reads."""
import itertools

import numpy as np
from scipy.spatial.transform import Rotation

from paper_2603_23891_amd import synth


def test_children_follow_the_canonical_construction():
    spec = synth.TopDownSpec(n_roots=5, depth=3, box=(20, 20, 4), root_scale=(2.0, 1.5, 0.3), gamma=0.6, seed=4)
    t = synth.topdown_tree(spec)
    N = t.n_nodes
    assert N == 5 * (1 + 8 + 64 + 512) and t.level_sizes == [5, 40, 320, 2560]
    assert t.max_depth == 3 and t.n_internal_span == 5 + 40 + 320
    assert np.all(t.parent[:5] == -1) and np.all(t.parent[5:] < np.arange(5, N))
    depth = (t.flags >> 1) & 15
    leaf = (t.flags & 1).astype(bool)
    assert np.array_equal(leaf, depth == 3)
    signs = np.array(list(itertools.product((-1, 1), repeat=3)), np.float64)
    for c in range(5, N):
        p = t.parent[c]
        k = (c - t.level_sizes[0] - sum(t.level_sizes[1:depth[c]])) % 8  # rank among its siblings
        assert depth[c] == depth[p] + 1
        R = Rotation.from_quat(np.r_[t.quat[1:, p], t.quat[0, p]].astype(np.float64)).as_matrix()
        s_p = t.scale[:, p].astype(np.float64)
        expect = t.mean[:, p].astype(np.float64) + R @ (signs[k] * s_p / 2)
        assert np.allclose(t.mean[:, c], expect, rtol=0, atol=1e-5 * (1 + np.abs(expect).max())), c
        assert np.allclose(t.scale[:, c], spec.gamma * s_p, rtol=1e-6)
        assert np.array_equal(t.quat[:, c], t.quat[:, p])
        assert t.opacity[c] == t.opacity[p]
        assert np.array_equal(t.sh[c], t.sh[p])
    # rotations about the vertical axis only: the roots stay flat
    assert np.allclose(t.quat[1:3], 0.0)
    assert np.allclose(np.linalg.norm(t.quat, axis=0), 1.0, atol=1e-6)
