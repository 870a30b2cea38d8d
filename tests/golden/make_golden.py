"""Writes tests/golden/oracle_small_scene.json from the CPU oracle alone.

Regression record of the oracle on a small seeded scene (4 frames with
exposure drift): the pair matrices, flags, quantiles, threshold means and a
digest of every panorama.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd.scenes import small_scene  # noqa: E402


def record():
    s = small_scene(n_cams=3, W=128, H=80, overlap=0.3, drift=0.05)
    o = O.Oracle(s.rig())
    out = []
    for t in range(4):
        pano = o.stitch(s.frames(t))
        out.append(dict(t=t, pano_sha256=hashlib.sha256(pano.tobytes()).hexdigest(),
                        mpair=o.tap("mpair").round(12).tolist(), flags=o.tap("flags").tolist(),
                        quant=o.tap("quant").tolist(), mbar=o.tap("mbar").tolist()))
    return dict(scene="small_scene(n_cams=3, W=128, H=80, overlap=0.3, drift=0.05)", frames=out)


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small_scene.json")
    with open(path, "w") as f:
        json.dump(record(), f, indent=1)
    print("wrote", path)
