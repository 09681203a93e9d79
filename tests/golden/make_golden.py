"""Writes tests/golden/tiny_scene.json from the CPU oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
It records digests of the oracle's basic image, HQ image and shuffled-Morton
permutation for a small building scene, so that a later change to the oracle's
arithmetic shows up as a failing test that has to be justified.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2104_07526_amd import synth  # noqa: E402


def main():
    n, seed, W, H = 20000, 4, 64, 36
    orc = oracle.default()
    pts = synth.buildings(n, seed=seed)
    m = synth.buildings_overview(W, H, seed=seed)
    fb = orc.render_basic(pts, m, W, H)
    basic = orc.resolve_basic(fb, W, H)
    D, RG, BA = orc.render_hq(pts, m, W, H)
    hq = orc.resolve_hq(RG, BA, W, H)
    perm = orc.reorder(pts, oracle.ORDER_MORTON_SHUFFLE, 128, seed)
    out = {
        "what": "building scene (synth.buildings), overview camera; digests of oracle outputs",
        "n": n, "seed": seed, "W": W, "H": H,
        "mvp": [float(v) for v in m],
        "covered_pixels": int(np.count_nonzero(basic)),
        "basic_sha256": hashlib.sha256(basic.tobytes()).hexdigest(),
        "hq_sha256": hashlib.sha256(hq.tobytes()).hexdigest(),
        "morton_shuffle_sha256": hashlib.sha256(perm.tobytes()).hexdigest(),
    }
    with open(os.path.join(ROOT, "tests", "golden", "tiny_scene.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["covered_pixels"], "covered pixels of", W * H)


if __name__ == "__main__":
    main()
