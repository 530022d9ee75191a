"""Writes tests/golden/city_tau.json: the scene-adaptive shrink threshold
tau = lambda_G / G_bar (Eq. (8), lambda_G = 0.2 per Sec. 4.1) of the synthetic
city scenes, from the CPU oracle's GTC pre-pass (Eqs. (5)-(7), 3-sigma
extents, the filtered cut) over their seeded training views.

Calls only the oracle and the input generators.   python tests/golden/make_tau.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2603_23891_amd import synth  # noqa: E402


def main():
    out = {}
    t0 = time.time()
    tree = synth.city_tree(synth.CITY1M)
    r = oracle.scene_tau(tree, [synth.city1m_camera()], synth.LAMBDA_G, synth.TAU_R)
    out["city1m"] = dict(r, views="city1m_camera()")
    print("city1m", r, round(time.time() - t0, 1), flush=True)
    del tree
    tree = synth.city_tree(synth.CITY20M)
    print("city20m tree built", round(time.time() - t0, 1), flush=True)
    r = oracle.scene_tau(tree, synth.city20m_training_views(8), synth.LAMBDA_G, synth.TAU_R)
    out["city20m"] = dict(r, views="city20m_training_views(8)")
    print("city20m", r, round(time.time() - t0, 1), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "city_tau.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
