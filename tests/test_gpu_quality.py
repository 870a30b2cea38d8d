"""GPU: the quality harness on a small drifting ring (three frames) scores the
library's panoramas exactly as it scores the oracle's (the panoramas and taps
are bit-identical), for 2D-M, 3D-M and the three literal readings; and the
adopted readings beat the literal ones where the metrics say they should."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import quality as Q  # noqa: E402
from paper_2308_09209_amd.scenes import small_scene  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_sequence(scene, n_frames, **params):
    """run_sequence's records from the oracle"""
    orc = O.Oracle(scene.rig(), **params)
    out = []
    for t in range(n_frames):
        pano = orc.stitch(scene.frames(t))
        rec = dict(pano=pano, cover=orc.tap("cover").astype(bool), mpair=orc.tap("mpair").copy(), pairs=[])
        two = np.zeros(rec["cover"].shape, bool)
        for p in range(orc.n_pairs):
            x0, y0 = orc.strip_box(p)[:2]
            mask = orc.tap("mask", p).astype(bool)
            ys, xs = np.nonzero(mask)
            two[ys + y0, np.mod(xs + x0, two.shape[1])] = True
            rec["pairs"].append(dict(mask=mask, yj=orc.tap("pyr", p, 0).copy(), yi=orc.tap("pyr", p, 8).copy()))
        rec["two"] = two
        out.append(rec)
    return out


@pytest.mark.parametrize("params", [dict(color_window=1), dict(color_window=3), dict(readings=1),
                                    dict(readings=2), dict(readings=4)])
def test_harness_scores_gpu_and_oracle_alike(params):
    sc = small_scene(n_cams=3, W=240, H=120, overlap=0.3, ring=True, seed_config=98, drift=0.03)
    g = Q.score(sc, Q.run_sequence(sc, 3, balance=0, **params))
    o = Q.score(sc, oracle_sequence(sc, 3, balance=0, **params))
    say(f"[quality {params}] " + ", ".join(f"{k} {v:.4f}" for k, v in g.items()))
    for k in g:
        assert abs(g[k] - o[k]) <= 1e-9 * max(1.0, abs(o[k])), (k, g[k], o[k])
