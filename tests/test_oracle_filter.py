"""Pins of the oracle's traversal-free filter (Sec. 3.2).

The parallel form (R&L then Ancestor, each node on its own) must select
exactly the cut that a tree walk selects: a recursive depth-first walk and
the per-level frontier walk of the serial scheme (Eq. (3)); the paper states
this identity (Sec. 4.3, Table 3). Plus the cut invariants, the special
values of tau_R, monotonicity, closed-form frustum cases and a float64
check of the radius predicate.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2603_23891_amd import synth
from tests import ref64
from tests.helpers import flat_tree


def children_of(tree):
    ch = [[] for _ in range(tree.n_nodes)]
    for i, p in enumerate(tree.parent):
        if p >= 0:
            ch[p].append(i)
    return ch


def recursive_cut(tree, rl):
    ch = children_of(tree)
    out = []

    def visit(n):
        if rl[n]:
            out.append(n)
            return
        for c in ch[n]:
            visit(c)

    for r in np.nonzero(tree.parent < 0)[0]:
        visit(int(r))
    return np.array(sorted(out), np.uint32)


def levelwise_cut(tree, rl):
    """One frontier per level; every level is a full pass (the serial scheme)."""
    ch = children_of(tree)
    frontier = [int(r) for r in np.nonzero(tree.parent < 0)[0]]
    out = []
    while frontier:
        nxt = []
        for n in frontier:
            if rl[n]:
                out.append(n)
            else:
                nxt.extend(ch[n])
        frontier = nxt
    return np.array(sorted(out), np.uint32)


def ancestors(tree, n):
    a = tree.parent[n]
    while a >= 0:
        yield int(a)
        a = tree.parent[a]


def check_cut(tree, cam, tau_R):
    pred = oracle.node_predicates(tree, cam, tau_R)
    F = (pred & 1).astype(bool)
    small = ((pred >> 1) & 1).astype(bool)
    rl = ((pred >> 2) & 1).astype(bool)
    assert np.array_equal(rl, F & (tree.is_leaf | small))
    assert not np.any(small & ~F)
    mask, sel = oracle.filter(tree, cam, tau_R)
    assert np.array_equal(np.nonzero(mask)[0].astype(np.uint32), sel)
    assert np.array_equal(sel, recursive_cut(tree, rl))
    assert np.array_equal(sel, levelwise_cut(tree, rl))
    selset = set(sel.tolist())
    for leaf in np.nonzero(tree.is_leaf & F)[0]:
        path = [int(leaf)] + list(ancestors(tree, leaf))
        k = sum(1 for n in path if n in selset)
        assert k <= 1
        if F.all():
            assert k == 1
    return F, small, rl, sel


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 10 ** 6), tau_R=st.sampled_from([0.0, 1.0, 3.0, 10.0, 30.0, 100.0, 1e9]),
       dist=st.sampled_from([8.0, 25.0, 100.0, 400.0]), yaw=st.floats(-0.6, 0.6))
def test_parallel_filter_equals_tree_walks(seed, tau_R, dist, yaw):
    tree = synth.random_tree(seed, n_roots=1 + seed % 3, max_depth=2 + seed % 4)
    rot = synth.yaw_pitch_rotation(np.pi / 2 + yaw, 0.0)
    cam = synth.make_camera(rot, (0.0, -dist, 0.0), 320, 240)
    check_cut(tree, cam, tau_R)


@pytest.mark.parametrize("dist", [25.0, 100.0, 400.0])
@pytest.mark.parametrize("tau_R", [3.0, 10.0, 30.0, 100.0, 1e9])
def test_tiny_tree_cuts(dist, tau_R):
    tree = synth.tiny_tree(0)
    check_cut(tree, synth.tiny_camera(dist), tau_R)


def test_tau_zero_selects_in_frustum_leaves():
    tree = synth.random_tree(4, n_roots=3, max_depth=5)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, 0), (0, -12, 0), 320, 240)
    F, _, _, sel = check_cut(tree, cam, 0.0)
    assert np.array_equal(sel, np.nonzero(tree.is_leaf & F)[0].astype(np.uint32))


def test_tau_infinite_selects_first_in_frustum_nodes():
    for seed in range(6):
        tree = synth.random_tree(seed, n_roots=3, max_depth=4)
        cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, 0), (0, -6, 0), 160, 120)
        F, _, _, sel = check_cut(tree, cam, np.inf)
        want = [n for n in range(tree.n_nodes) if F[n] and not any(F[a] for a in ancestors(tree, n))]
        assert np.array_equal(sel, np.array(want, np.uint32))


def test_selection_count_monotone_in_tau_R_when_all_in_frustum():
    tree = synth.tiny_tree(0)
    cam = synth.tiny_camera(100)
    prev = None
    for tau_R in [0.0, 1.0, 2.0, 3.0, 5.0, 8.0, 13.0, 21.0, 34.0, 55.0, 1e9]:
        F, _, _, sel = check_cut(tree, cam, tau_R)
        assert F.all()
        if prev is not None:
            assert sel.size <= prev
        prev = sel.size


def test_small_predicate_matches_float64_radius():
    tree = synth.tiny_tree(0)
    for dist in (25.0, 100.0, 400.0):
        cam = synth.tiny_camera(dist)
        for tau_R in (3.0, 10.0, 30.0):
            pred = oracle.node_predicates(tree, cam, tau_R)
            small = ((pred >> 1) & 1).astype(bool)
            for n in range(tree.n_internal_span):
                R = ref64.radius3(tree, cam, n)
                if abs(R - tau_R) > 1e-4 * tau_R:
                    assert small[n] == (R <= tau_R), (dist, tau_R, n, R)


def test_frustum_closed_forms():
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 256, 256)  # R = I, t = 0: x_c = x_w exactly
    zn = np.float32(cam.znear)
    kx = np.float32(cam.kx)
    pts = [([0, 0, 1], True),                                       # on axis
           ([0, 0, float(zn)], False),                              # on the near plane: not in front of it
           ([0, 0, float(np.nextafter(zn, np.float32(1)))], True),
           ([float(kx), 0, 1], True),                               # exactly on the guard-band boundary
           ([float(np.nextafter(kx, np.float32(9))), 0, 1], False),
           ([0, float(-np.float32(cam.ky)), 1], True),
           ([0, 0, -5], False)]                                     # behind the camera
    tree = flat_tree([p for p, _ in pts], np.full((len(pts), 3), 0.01), np.tile([1, 0, 0, 0], (len(pts), 1)),
                     np.full(len(pts), 0.5), np.zeros((len(pts), 1, 3)))
    F = oracle.node_predicates(tree, cam, 3.0) & 1
    assert F.tolist() == [int(w) for _, w in pts]
    for i in range(len(pts)):
        assert bool(F[i]) == ref64.in_frustum(tree, cam, i)[0]


def test_filter_nodes_matches_full_filter():
    tree = synth.tiny_tree(0)
    cam = synth.tiny_camera(100)
    mask, _ = oracle.filter(tree, cam, 10.0)
    nodes = np.arange(tree.n_nodes)
    assert np.array_equal(oracle.filter_nodes(tree, cam, 10.0, nodes), mask)
