"""Writes tests/golden/city_tau.json: the scene-adaptive shrink threshold
tau = lambda_G / G_bar (Eq. (8), lambda_G = 0.2 per Sec. 4.1) of the synthetic
scenes, from the CPU oracle's GTC pre-pass (Eqs. (5)-(7), 3-sigma extents,
the filtered cut) over their seeded training views.

Calls only the oracle and the input generators.

    python tests/golden/make_tau.py [scene ...]     (default: every scene)

Scenes named on the command line are recomputed and merged into the existing
file; the others keep their stored values.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2603_23891_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "city_tau.json")


def flat2m_tree():
    g = synth.flat_gaussians(2_000_000, seed=0)
    prm = oracle.ParamsRef(g.mean, g.log_scale, g.quat, g.logit, g.sh, g.sh_degree)
    return oracle.flat_tree_from_params(prm)


SCENES = {
    "city1m": (lambda: synth.city_tree(synth.CITY1M), lambda: [synth.city1m_camera()], "city1m_camera()"),
    "city20m": (lambda: synth.city_tree(synth.CITY20M), lambda: synth.city20m_training_views(8),
                "city20m_training_views(8)"),
    "topdown20m": (lambda: synth.topdown_tree(synth.TOPDOWN20M), lambda: synth.city20m_training_views(8),
                   "city20m_training_views(8)"),
    "flat2m": (flat2m_tree, lambda: [synth.city1m_yaw_views()[3]], "city1m_yaw_views()[3]"),
}


def main():
    names = sys.argv[1:] or list(SCENES)
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    oracle.set_threads(os.cpu_count())  # the OpenMP build: bit-identical, faster
    t0 = time.time()
    for name in names:
        make_tree, make_views, views = SCENES[name]
        tree = make_tree()
        r = oracle.scene_tau(tree, make_views(), synth.LAMBDA_G, synth.TAU_R)
        out[name] = dict(r, views=views)
        print(name, r, round(time.time() - t0, 1), flush=True)
        del tree
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
