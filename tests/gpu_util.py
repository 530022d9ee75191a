"""Helpers for the GPU parity tests: run a frame through libfg and read it back."""
import numpy as np
import torch

from paper_2603_23891_amd import fg


def run_gpu_frame(tree, cam, tau_R=3.0, tau=0.0, bg=(0.0, 0.0, 0.0), cap_sel=None, cap_pairs=None, tune=None,
                  dtree=None):
    dtree = dtree or fg.DeviceTree(tree)
    cap_sel = tree.n_nodes if cap_sel is None else cap_sel
    cap_pairs = (1 << 22) if cap_pairs is None else cap_pairs
    fb = fg.FrameBuffers(dtree, cam.width, cam.height, cap_sel, cap_pairs)
    fg.render_frame(dtree, cam, fb, tau_R, tau, bg, tune)
    torch.cuda.synchronize()
    return read_frame(fb, tree.n_nodes)


def read_frame(fb, n_nodes):
    n_sel, n_pairs, status = fg.read_counts(fb)
    ns = min(n_sel, fb.cap_sel)
    npairs = min(n_pairs, fb.cap_pairs)
    u32 = lambda t: t.cpu().numpy().view(np.uint32)
    bits = u32(fb.sel_bits)
    mask = ((bits[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)[:n_nodes].astype(np.uint8)
    sp = fb.splats
    return dict(
        n_sel=n_sel, n_pairs=n_pairs, status=status, sel_mask=mask, sel_idx=u32(fb.sel_idx)[:ns],
        xy=sp.xy[:ns].cpu().numpy(), conic_o=sp.conic_o[:ns].cpu().numpy(), rgb_depth=sp.rgb_depth[:ns].cpu().numpy(),
        rect=sp.rect[:ns].cpu().numpy().view(np.uint16), tiles=u32(sp.tiles)[:ns],
        tile_keys=u32(fb.tile_keys)[:npairs], vals=u32(fb.vals)[:npairs], ranges=u32(fb.ranges),
        image=fb.image.cpu().numpy(), final_T=fb.final_T.cpu().numpy(), n_contrib=u32(fb.n_contrib))


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def assert_frame_parity(g, o, check_image=True):
    """Bit-exact selection, splats, keys and ranges; image within 1e-4 (and n_contrib exact)."""
    assert g["status"] == 0, g["status"]
    assert np.array_equal(g["sel_mask"], o["sel_mask"]), "selection mask"
    assert np.array_equal(g["sel_idx"], o["sel_idx"]), "compacted selection"
    sp = o["splats"]
    assert np.array_equal(g["tiles"], sp["tiles"]), "tile counts"
    assert np.array_equal(g["rect"].astype(np.int64),
                          np.stack([sp["x0"], sp["y0"], sp["x1"], sp["y1"]], 1).astype(np.int64)), "tile rects"
    assert np.array_equal(bits(g["xy"]), bits(np.stack([sp["u"], sp["v"]], 1))), "2D means"
    assert np.array_equal(bits(g["conic_o"]), bits(np.stack([sp["A"], sp["B"], sp["C"], sp["opacity"]], 1))), "conics"
    assert np.array_equal(bits(g["rgb_depth"]), bits(np.stack([sp["r"], sp["g"], sp["b"], sp["depth"]], 1))), "rgb/depth"
    assert g["n_pairs"] == o["keys"].size, (g["n_pairs"], o["keys"].size)
    dbits = bits(g["rgb_depth"][:, 3])
    key64 = (g["tile_keys"].astype(np.uint64) << np.uint64(32)) | dbits[g["vals"]].astype(np.uint64)
    assert np.array_equal(key64, o["keys"]), "sorted keys"
    assert np.array_equal(g["vals"], o["vals"]), "sorted values"
    assert np.array_equal(g["ranges"].reshape(-1, 2), o["ranges"]), "tile ranges"
    if check_image:
        err = np.abs(g["image"] - o["image"]).max() if o["image"].size else 0.0
        assert err <= 1e-4, err
        assert np.array_equal(g["n_contrib"], o["n_contrib"]), "n_contrib"
        assert np.abs(g["final_T"] - o["final_T"]).max() <= 1e-4
