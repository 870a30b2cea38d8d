"""GPU parity of the literal readings (VS_READ_* options: overlap-only colour,
eq. (17) as printed, nearest-CDF histogram specification), each alone and all
together, against the oracle with the same readings: small rings over three
frames (the colour state passes through the temporal window) and one full-size
4 x 1080p frame with all three.  Bars as in the default path's parity tests."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import vstitch as V  # noqa: E402
from paper_2308_09209_amd.scenes import scene_for, small_scene  # noqa: E402
from tests.test_gpu_parity import check_steps, dev, lsb  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("readings", [V.READ_OVERLAP_ONLY, V.READ_LITERAL_EQ17, V.READ_NEAREST_CDF, 7])
def test_readings_match_oracle_on_a_small_ring(readings):
    sc = small_scene(n_cams=3, W=200, H=110, overlap=0.35, ring=True, seed_config=96, drift=0.03)
    st = V.Stitcher(sc.rig(), debug_taps=1, readings=readings)
    orc = O.Oracle(sc.rig(), readings=readings)
    for t in range(3):
        frames = sc.frames(t)
        got = st.stitch(dev(frames)).cpu().numpy()
        want = orc.stitch(frames)
        d = lsb(got, want)
        say(f"[readings {readings}] frame {t}: max diff {d} LSB, identical px "
            f"{np.mean(np.all(got == want, -1)):.6f}")
        assert d <= 1
        check_steps(st, orc, f"readings {readings} t={t}")
        np.testing.assert_array_equal(st.tap("pano_pre"), orc.tap("pano_pre"))
        np.testing.assert_allclose(st.tap("mk"), orc.tap("mk"), rtol=1e-4, atol=1e-6)
        if readings & V.READ_OVERLAP_ONLY:
            assert np.abs(st.tap("mk") - np.eye(3)).max() == 0
    st.close()


def test_all_readings_full_size_4x1080p():
    s = scene_for("4x1920x1080_ring")
    st = V.Stitcher(s.rig(), debug_taps=1, readings=7)
    orc = O.Oracle(s.rig(), readings=7)
    frames = s.frames(0)
    got = st.stitch(dev(frames)).cpu().numpy()
    want = orc.stitch(frames)
    d = lsb(got, want)
    say(f"[readings 7, 4x1080p] max diff {d} LSB, identical px {np.mean(np.all(got == want, -1)):.6f}")
    assert d <= 1
    check_steps(st, orc, "readings 7 4x1080p")
    st.close()
