"""The serial level-wise filter (fg_filter_levelwise, Sec. 3.2 Eq. (3)) selects
exactly the set of the traversal-free filter (fg_filter) and of the oracle:
the identity the paper reports in Table 3. Also the children CSR that
fg_children builds from the parent links, and the status bit of malformed
parent links."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_23891_amd import fg, synth

pytestmark = pytest.mark.gpu


def mask_of(words, n):
    w = words.cpu().numpy().view(np.uint32)
    return ((w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)[:n].astype(np.uint8)


def both_filters(tree, cam, tau_R, dt=None, ch=None):
    dt = dt or fg.DeviceTree(tree)
    ch = ch or fg.TreeChildren(dt)
    N = tree.n_nodes
    words = max((N + 31) // 32, 1)
    bits_lw = torch.full((words,), -1, dtype=torch.int32, device="cuda")
    n_lw = torch.zeros(1, dtype=torch.int32, device="cuda")
    st_lw = torch.zeros(1, dtype=torch.int32, device="cuda")
    stats = fg.fg_filter_levelwise(dt, ch.offs, ch.ids, cam, tau_R, bits_lw, n_lw, st_lw, ch.ws)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, N, 1)
    fg.filter_stage(dt, cam, fb, tau_R)
    torch.cuda.synchronize()
    return (mask_of(bits_lw, N), int(n_lw.item()), int(st_lw.item()), stats,
            mask_of(fb.sel_bits, N), fg.read_counts(fb)[0], int(ch.status.item()))


TINY = synth.tiny_tree(0)


def test_children_csr():
    tree = synth.random_tree(4, n_roots=3, max_depth=5)
    dt = fg.DeviceTree(tree)
    ch = fg.TreeChildren(dt)
    torch.cuda.synchronize()
    offs = ch.offs.cpu().numpy()
    ids = ch.ids.cpu().numpy()
    N = tree.n_nodes
    assert ch.status.item() == 0
    assert offs[0] == 0 and offs[N + 1] == N
    for n in list(range(N)) + [N]:
        kids = sorted(ids[offs[n]:offs[n + 1]])
        expect = np.nonzero(tree.parent == (n if n < N else -1))[0]
        assert np.array_equal(kids, expect), n


@pytest.mark.parametrize("dist,tau_R", [(25.0, 3.0), (100.0, 10.0), (400.0, 3.0), (100.0, 30.0), (25.0, 1e9),
                                        (400.0, 100.0)])
def test_tiny_tree_same_set(dist, tau_R):
    cam = synth.tiny_camera(dist)
    m_lw, n_lw, st, stats, m_par, n_par, _ = both_filters(TINY, cam, tau_R)
    mask, sel = oracle.filter(TINY, cam, tau_R)
    assert st == 0
    assert np.array_equal(m_lw, mask) and np.array_equal(m_par, mask)
    assert n_lw == n_par == sel.size
    assert 1 <= stats.levels <= TINY.max_depth + 1 and stats.calc_ms > 0 and stats.wall_ms >= stats.calc_ms


@pytest.mark.parametrize("seed", range(6))
def test_random_forests_same_set(seed):
    tree = synth.random_tree(seed, n_roots=1 + seed % 4, max_depth=3 + seed % 4)
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2 + rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3)),
                            (rng.uniform(-3, 3), -rng.uniform(10, 60), rng.uniform(-3, 3)),
                            int(rng.integers(40, 400)), int(rng.integers(40, 300)))
    tau_R = float(rng.choice([1.0, 3.0, 10.0, 30.0]))
    m_lw, n_lw, st, _, m_par, n_par, _ = both_filters(tree, cam, tau_R)
    mask, sel = oracle.filter(tree, cam, tau_R)
    assert st == 0
    assert np.array_equal(m_lw, mask) and np.array_equal(m_par, mask)
    assert n_lw == n_par == sel.size


def test_city1m_same_set():
    tree = synth.city_tree(synth.CITY1M)
    cam = synth.city1m_camera()
    m_lw, n_lw, st, stats, m_par, n_par, cst = both_filters(tree, cam, synth.TAU_R)
    assert st == 0 and cst == 0
    assert np.array_equal(m_lw, m_par) and n_lw == n_par > 100_000
    assert stats.levels == tree.max_depth + 1


def test_malformed_parent_links_are_reported():
    """A parent index not below its child's (pointing forward, or past the
    end): both filters and the children builder report FG_STATUS_BAD_PARENT
    and finish normally (every parent link is bounds-checked before use)."""
    tree = synth.random_tree(2, n_roots=2, max_depth=4)
    N = tree.n_nodes
    bad = tree.parent.copy()
    leaves = np.nonzero(tree.flags & 1)[0]
    bad[leaves[0]] = N + 5        # past the end
    bad[leaves[1]] = leaves[1]    # itself
    bad[leaves[2]] = N - 1 if leaves[2] < N - 1 else 0  # a later node
    import dataclasses
    t2 = dataclasses.replace(tree, parent=bad)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, 0.0), (0, -40, 0), 160, 120)
    m_lw, n_lw, st, _, m_par, n_par, cst = both_filters(t2, cam, 3.0)
    assert cst & fg.FG_STATUS_BAD_PARENT
    dt = fg.DeviceTree(t2)
    fb = fg.FrameBuffers(dt, cam.width, cam.height, N, 1)
    fg.filter_stage(dt, cam, fb, 3.0)
    torch.cuda.synchronize()
    assert fg.read_counts(fb)[2] & fg.FG_STATUS_BAD_PARENT
