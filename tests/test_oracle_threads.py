"""The OpenMP build of the oracle (used only to time it on all host cores)
gives bit-identical results to the plain single-threaded build: every unit
(node, Gaussian, tile) is computed by the same operations in the same order,
only by different threads."""
import numpy as np

import oracle
from paper_2603_23891_amd import synth


def test_threaded_oracle_is_bit_identical():
    spec = synth.CitySpec(n_leaves=40_000, box=(30, 30, 8), n_blobs=6, blob_sigma=(5, 5, 0.05),
                          leaf_log_scale_mu=-3.0, seed=5)
    tree = synth.city_tree(spec)
    cam = synth.make_camera(synth.yaw_pitch_rotation(np.pi / 2, np.radians(-25)), (0, -60, 18), 640, 360)
    try:
        ref = oracle.render_frame(tree, cam, 3.0, 0.02)
        ref_kpc = oracle.kpc(ref["splats"], ref["vals"], ref["ranges"], cam)
        assert oracle.set_threads(8) >= 2
        got = oracle.render_frame(tree, cam, 3.0, 0.02)
        got_kpc = oracle.kpc(got["splats"], got["vals"], got["ranges"], cam)
    finally:
        oracle.set_threads(None)
    assert ref["sel_idx"].size > 1000 and ref["keys"].size > 1000
    for k in ("sel_mask", "sel_idx", "keys", "vals", "ranges", "n_contrib"):
        assert np.array_equal(ref[k], got[k]), k
    assert ref["splats"].tobytes() == got["splats"].tobytes()
    for k in ("image", "final_T"):
        assert ref[k].tobytes() == got[k].tobytes(), k
    assert ref_kpc.tobytes() == got_kpc.tobytes()
