"""The oracle against the constants the paper states, and against its own
recorded outputs on a small seeded scene (regression record written by
tests/golden/make_golden.py, which calls only the oracle)."""

import json
import os

import numpy as np

from oracle import oracle as O
from tests.golden.make_golden import record

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_defaults_are_the_papers_constants():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    p = O.default_params()
    assert p.lambda_pct / 100.0 == c["balance_lambda"]["value"]
    assert p.color_window == c["temporal_window"]["value"]


def test_oracle_regression_record():
    want = json.load(open(os.path.join(GOLD, "oracle_small_scene.json")))
    got = record()
    for a, b in zip(want["frames"], got["frames"]):
        assert a["pano_sha256"] == b["pano_sha256"], a["t"]
        np.testing.assert_allclose(np.array(a["mpair"]), np.array(b["mpair"]), rtol=0, atol=1e-11)
        assert a["flags"] == b["flags"] and a["quant"] == b["quant"] and a["mbar"] == b["mbar"]

