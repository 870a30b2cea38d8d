"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/vstitch.h declares, its structs have the header's layout,
and the host planner's homographies are the oracle's bit for bit."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_09209_amd import vstitch as V
from paper_2308_09209_amd.scenes import small_scene, scene_for
from tests.rigs import crop_rig, smooth_image

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vstitch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    L = V.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(V.EXPORTS) == names
    assert L.vs_abi_version() == 1


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "vstitch.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(vs_color_state),'
                   'sizeof(vs_rig), sizeof(vs_params), sizeof(vs_plan_info), sizeof(vs_frame_info),'
                   'offsetof(vs_color_state, q), offsetof(vs_rig, ring));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [C.sizeof(V.ColorState), C.sizeof(V.Rig), C.sizeof(V.Params), C.sizeof(V.PlanInfo),
            C.sizeof(V.FrameInfo), V.ColorState.q.offset, V.Rig.ring.offset]
    assert got == want


def test_default_params_are_the_papers():
    p = V.default_params()
    assert p.lambda_pct == 5 and p.color_window == 3
    assert (p.lk_levels, p.lk_iters, p.lk_radius, p.lk_lambda) == (4, 5, 4, 256.0)
    assert V.lib().vs_status_str(-2) == b"geometry"


def _strong_perspective_rig():
    from tests.test_oracle_geometry import strong_perspective_rig
    return strong_perspective_rig()[1]


@pytest.mark.parametrize("rigf", [lambda: small_scene(n_cams=3, ring=True, W=120, H=64).rig(),
                                  lambda: scene_for("2x640x360_chain").rig(), _strong_perspective_rig])
def test_host_planner_homographies_match_oracle_bitwise(rigf):
    rig = rigf()
    Hk, Hinv = V.compose_homographies(rig)
    o = O.Oracle(rig)
    n = rig["n_cams"]
    assert np.array_equal(np.array(o.plan.hk)[:n].reshape(n, 3, 3), Hk)
    assert np.array_equal(np.array(o.plan.hinv)[:n].reshape(n, 3, 3), Hinv)
    assert np.all(np.abs(Hinv[:, 2, 2]) == 1.0)


def test_invalid_rigs_rejected_before_any_device_work():
    tex = smooth_image(20, 200, seed=1)
    rig, _ = crop_rig(tex, 100, 20, [(0, 0), (60, 0)])
    bad = []
    r = dict(rig)
    r["n_cams"] = 1
    bad.append(r)
    r = dict(rig)
    r["ring"], r["ring_period"] = 1, 160   # a ring needs >= 3 cameras
    bad.append(r)
    r = dict(rig)
    r["cam_pitch"] = [200, 300]            # pitch below 3 * width
    bad.append(r)
    r = dict(rig)
    r["H_pair"] = [np.eye(3), np.full((3, 3), np.nan)]
    bad.append(r)
    r = dict(rig)
    r["canvas_w"] = 0
    bad.append(r)
    for b in bad:
        with pytest.raises(V.VSError) as e:
            V.Stitcher(b)
        assert e.value.status == -1
    with pytest.raises(V.VSError):
        V.Stitcher(rig, lk_radius=9)
    with pytest.raises(V.VSError):
        V.Stitcher(rig, lambda_pct=60)


class _FakeDeviceFrame:
    """Duck-typed stand-in for a device frame tensor (no GPU on the host)."""

    def __init__(self, shape):
        import torch
        self.dtype = torch.uint8
        self.is_cuda = True
        self.shape = shape
        self.device = torch.device("cuda", 0)

    def is_contiguous(self):
        return True

    def data_ptr(self):
        raise AssertionError("no pointer may be taken before the checks pass")


def test_host_tensor_panorama_is_rejected_before_any_library_call(monkeypatch):
    import torch

    st = object.__new__(V.Stitcher)
    st.n_cams = 2
    st.cam_shape = [(8, 16), (8, 16)]
    st.info = V.PlanInfo()
    st.info.canvas_h, st.info.canvas_w = 8, 24

    def no_lib():
        raise AssertionError("library called")

    monkeypatch.setattr(V, "lib", no_lib)
    frames = [_FakeDeviceFrame((8, 16, 3)) for _ in range(2)]
    with pytest.raises(ValueError, match="device tensor"):
        st.stitch(frames, pano=torch.zeros((8, 24, 3), dtype=torch.uint8))
    with pytest.raises(ValueError, match="device tensor"):
        V._check_pano(torch.zeros((8, 24, 3), dtype=torch.uint8), (8, 24), torch.device("cuda", 0))
    with pytest.raises(ValueError, match="canvas"):
        V._check_pano(torch.zeros((8, 23, 3), dtype=torch.uint8), (8, 24), torch.device("cuda", 0))
    b = object.__new__(V.Batch)
    b.stitchers = [st]
    with pytest.raises(ValueError, match="device tensor"):
        b._ptrs([frames], [torch.zeros((8, 24, 3), dtype=torch.uint8)])


def test_noalloc_flow_rejects_oversized_pairs_on_the_host():
    """vs_flow_run_noalloc refuses a pair whose workspace exceeds its static
    array before any device call (the pointers are never dereferenced), and
    NULL inputs; no GPU needed."""
    L = V.lib()
    fake = C.c_void_p(16)
    assert L.vs_flow_run_noalloc(4000, 3000, None, fake, fake, fake, fake, None) == -1
    assert L.vs_flow_run_noalloc(64, 64, None, None, fake, fake, fake, None) == -1
    assert L.vs_flow_run_noalloc(1, 64, None, fake, fake, fake, fake, None) == -1


def test_flow_only_rejects_bad_arguments_on_the_host():
    """vs_flow_only refuses a null context or strip and empty sizes before any
    device call (the pointers are never dereferenced); no GPU needed."""
    L = V.lib()
    fake = C.c_void_p(16)
    assert L.vs_flow_only(None, fake, fake, 64, 32, fake, fake, None) == -1
    assert L.vs_flow_only(fake, None, fake, 64, 32, fake, fake, None) == -1
    assert L.vs_flow_only(fake, fake, None, 64, 32, fake, fake, None) == -1
    assert L.vs_flow_only(fake, fake, fake, 0, 32, fake, fake, None) == -1
    assert L.vs_flow_only(fake, fake, fake, 64, 0, fake, fake, None) == -1


def test_create_rejects_unknown_readings():
    """vs_params.readings outside the VS_READ_* mask is refused before any
    device work."""
    from paper_2308_09209_amd.scenes import small_scene
    rig = V.make_rig(small_scene().rig())
    p = V.default_params(readings=8)
    h = C.c_void_p()
    assert V.lib().vs_create(C.byref(rig), C.byref(p), C.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_variational_weights():
    """flow = 2 with an odd number of Jacobi steps, a non-positive smoothness
    weight or a negative gradient weight is refused by both contexts before
    any device work; flow outside 0..2 too."""
    from paper_2308_09209_amd.scenes import small_scene
    rig = V.make_rig(small_scene().rig())
    for kw in (dict(var_inner=5), dict(var_alpha=0.0), dict(var_gamma=-1.0), dict(var_outer=-1), dict(flow=3)):
        p = V.default_params(flow=kw.pop("flow", 2), **kw)
        h = C.c_void_p()
        assert V.lib().vs_create(C.byref(rig), C.byref(p), C.byref(h)) == -1, kw
        assert V.lib().vs_flow_create(64, 48, C.byref(p), C.byref(h)) == -1, kw
        assert not h.value


def test_calibration_host_helpers_equal_the_oracle():
    """vs_calib_* (host FP64, eqs. (8), (11), (12), (14)) against the oracle's
    independent implementation, bit for bit."""
    from tests.test_oracle_calib import rot
    args = (0.006, 5e-6, 5.2e-6, 1e-5, -2e-5, 960.0, 540.0)
    K = V.calib_intrinsics(*args)
    np.testing.assert_array_equal(K, O.calib_intrinsics(*args))
    R, t = rot(0.05, -0.3, 0.02), np.array([0.2, -0.1, 5.0])
    Ha = V.calib_plane_homography(K, R, t)
    np.testing.assert_array_equal(Ha, O.calib_plane_homography(K, R, t))
    Hb = V.calib_plane_homography(K, rot(0.0, 0.2, 0.01), np.array([-0.3, 0.0, 5.1]))
    np.testing.assert_array_equal(V.calib_pair(Ha, Hb), O.calib_pair(Ha, Hb))
    p = (2.5, -1.0, 1.01, 0.98)
    np.testing.assert_array_equal(V.calib_refine(Ha, p), O.calib_refine(Ha, p))
    with pytest.raises(V.VSError):
        V.calib_pair(Ha, np.zeros((3, 3)))


def test_tuning_records_round_trip_through_a_file(tmp_path):
    """vs_tune_put / get / save / load / clear (host only): a record file
    written and read back gives the same records; a later record of an equal
    key replaces the earlier; malformed lines, unknown variant codes, 9x9
    codes with another radius and bad tile heights are refused, loading
    nothing."""
    def key(arch=b"gfx950", cams=4, w=6144, h=1080, levels=4, radius=4):
        k = V.TuneKey()
        k.arch, k.n_cams, k.canvas_w, k.canvas_h, k.lk_levels, k.lk_radius = arch, cams, w, h, levels, radius
        return k
    V.tune_clear()
    assert V.tune_get(key()) is None
    V.tune_put(key(), V.tune_entry([12, 12, 25, 25], 16))
    V.tune_put(key(cams=8, w=24576, h=2160), V.tune_entry([12, 12, 11, 27], 8))
    V.tune_put(key(), V.tune_entry([12, 11, 25, 25], 8))          # replaces the first
    path = tmp_path / "tune.txt"
    V.tune_save(path)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("vstune1 gfx950 ") for ln in lines)
    V.tune_clear()
    assert V.tune_get(key()) is None
    V.tune_load(path)
    e = V.tune_get(key())
    assert list(e.flow_variant) == [12, 11, 25, 25, 0, 0] and e.pyr_tile_rows == 8
    e = V.tune_get(key(cams=8, w=24576, h=2160))
    assert list(e.flow_variant)[:4] == [12, 12, 11, 27] and e.pyr_tile_rows == 8
    assert V.tune_get(key(arch=b"gfx942")) is None
    for bad in (V.tune_entry([12, 12, 13, 25]), V.tune_entry([12, 12, 25, 25], 12),
                V.tune_entry([12, 12, 25, 25, 9])):
        with pytest.raises(V.VSError):
            V.tune_put(key(), bad)
    with pytest.raises(V.VSError):
        V.tune_put(key(radius=3), V.tune_entry([12, 0, 0, 0]))
    V.tune_put(key(radius=3), V.tune_entry([0, 0, 0, 0]))
    for text in ("vstune1 gfx950 4 6144 1080 4 4 12 12 25 25 0 0 16 extra\n",
                 "vstune2 gfx950 4 6144 1080 4 4 12 12 25 25 0 0 16\n",
                 "vstune1 gfx950 4 6144 1080 4 4 12 12 25 64 0 0 16\n",
                 "vstune1 gfx950 4 6144 1080 4\n"):
        bad_path = tmp_path / "bad.txt"
        bad_path.write_text("vstune1 gfx950 2 640 360 4 4 9 9 25 25 0 0 8\n" + text)
        with pytest.raises(V.VSError):
            V.tune_load(bad_path)
        k2 = key(cams=2, w=640, h=360)
        assert V.tune_get(k2) is None        # nothing of a refused file is loaded
    V.tune_clear()
