"""Python binding of libvstitch (the C ABI in include/vstitch.h).

Argument marshalling only: every step of the stitching path runs in the HIP
kernels of libvstitch.so.  torch supplies device memory and streams.  There
is no fallback: if the library is missing, importing the binding fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # load torch first so that libvstitch binds to the HIP runtime torch already holds
    import torch
except ImportError:  # pragma: no cover - symbol checks without torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvstitch.so")

MAX_CAMS = 16
MAX_PAIRS = 16
MAX_LEVELS = 6
STATE_VERSION = 1

STATUS = {0: "VS_OK", -1: "VS_E_INVAL", -2: "VS_E_GEOMETRY", -3: "VS_E_NOMEM", -4: "VS_E_DEVICE",
          -5: "VS_E_STATE", -6: "VS_E_UNSUPPORTED"}
TAP = dict(strip=1, mask=2, hist=3, lut=4, mom=5, mpair=6, mk=7, flags=8, pyr=9, flow=10,
           pano_pre=11, pano_hist=12, bal_lut=13, quant=14, mbar=15, cover=16, need=17,
           deferred=18, surr_pred=19, fb=20, surr_ok=21)
FLOW_PLAIN, FLOW_SURROGATE, FLOW_SURROGATE_FALLBACK = 0, 1, 2
FLOW_VARIANTS = 12  # 9x9 flow-kernel variants the autotuner measures
FLOW_VARIANT_CODES = (1, 2, 3, 4, 9, 10, 11, 12, 25, 26, 27, 28)
FLOW_ALT, FLOW_INBLOCK = 8, 16

# every symbol include/vstitch.h declares
EXPORTS = ["vs_abi_version", "vs_status_str", "vs_default_params", "vs_compose_homographies",
           "vs_create", "vs_destroy", "vs_query", "vs_last_error", "vs_stitch", "vs_state_get",
           "vs_state_set", "vs_debug_tap", "vs_set_timing", "vs_get_timing",
           "vs_set_flow_variant", "vs_get_flow_variant", "vs_load_weights", "vs_set_flow_mode",
           "vs_batch_create", "vs_batch_run",
           "vs_batch_destroy", "vs_batch_last_error", "vs_batch_autotune",
           "vs_tune_put", "vs_tune_get", "vs_tune_clear", "vs_tune_save", "vs_tune_load", "vs_tune_key_of",
           "vs_get_tuning",
           "vs_nn_conv3x3", "vs_nn_wgrad_scratch_bytes", "vs_nn_conv3x3_wgrad", "vs_nn_flip_weights",
           "vs_nn_lrelu_bwd", "vs_nn_pack_pair", "vs_nn_epe_loss", "vs_nn_adam", "vs_nn_to_bf16",
           "vs_nn_pool_flow", "vs_nn_create", "vs_nn_destroy", "vs_nn_forward", "vs_nn_loss", "vs_nn_backward",
           "vs_nn_adam_step", "vs_nn_params", "vs_nn_save", "vs_nn_load", "vs_flow_create", "vs_flow_run", "vs_flow_destroy", "vs_flow_level", "vs_flow_only",
           "vs_flow_run_noalloc", "vs_calib_intrinsics", "vs_calib_plane_homography", "vs_calib_pair",
           "vs_calib_refine", "vs_calib_estimate"]


class Rig(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("cam_w", C.c_int32 * MAX_CAMS),
                ("cam_h", C.c_int32 * MAX_CAMS), ("cam_pitch", C.c_int32 * MAX_CAMS),
                ("H_pair", (C.c_double * 9) * MAX_CAMS), ("H_ref", C.c_double * 9),
                ("ring", C.c_int32), ("ring_period", C.c_int32), ("canvas_w", C.c_int32),
                ("canvas_h", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("color_window", C.c_int32), ("ridge", C.c_double), ("min_pixels", C.c_int32),
                ("flow", C.c_int32), ("lk_levels", C.c_int32), ("lk_iters", C.c_int32),
                ("lk_radius", C.c_int32), ("lk_lambda", C.c_float), ("balance", C.c_int32),
                ("lambda_pct", C.c_int32), ("debug_taps", C.c_int32), ("pyr_tile_rows", C.c_int32),
                ("readings", C.c_int32), ("var_alpha", C.c_float), ("var_gamma", C.c_float),
                ("var_outer", C.c_int32), ("var_inner", C.c_int32)]


READ_OVERLAP_ONLY, READ_LITERAL_EQ17, READ_NEAREST_CDF = 1, 2, 4


class Moments(C.Structure):
    _fields_ = [("A", C.c_uint64 * 6), ("B", C.c_uint64 * 9), ("n", C.c_uint64)]


class ColorState(C.Structure):
    _fields_ = [("version", C.c_uint32), ("size", C.c_uint32), ("n_pairs", C.c_uint32),
                ("frames_seen", C.c_uint32), ("mom", (Moments * 2) * MAX_PAIRS),
                ("q", ((C.c_int32 * 2) * 3) * 2)]


class PlanInfo(C.Structure):
    _fields_ = [("canvas_w", C.c_int32), ("canvas_h", C.c_int32), ("pano_pitch", C.c_int32),
                ("n_cams", C.c_int32), ("n_pairs", C.c_int32), ("ring", C.c_int32),
                ("ring_period", C.c_int32), ("lk_levels", C.c_int32),
                ("pair_j", C.c_int32 * MAX_PAIRS), ("pair_i", C.c_int32 * MAX_PAIRS),
                ("pair_si", C.c_int32 * MAX_PAIRS),
                ("strip_x0", C.c_int32 * MAX_PAIRS), ("strip_y0", C.c_int32 * MAX_PAIRS),
                ("strip_w", C.c_int32 * MAX_PAIRS), ("strip_h", C.c_int32 * MAX_PAIRS),
                ("n_covered", C.c_int64), ("workspace_bytes", C.c_uint64),
                ("state_bytes", C.c_uint32), ("pad0", C.c_uint32),
                ("flow_px", (C.c_uint64 * MAX_LEVELS) * MAX_PAIRS),
                ("flow_taps", (C.c_uint64 * MAX_LEVELS) * MAX_PAIRS)]


NN_MAX_IMAGES = 64
CONV_LRELU, CONV_LINEAR, CONV_F32, CONV_FLOW2 = 0, 1, 2, 3


class NNImages(C.Structure):
    _fields_ = [("n", C.c_int32), ("w", C.c_int32 * NN_MAX_IMAGES), ("h", C.c_int32 * NN_MAX_IMAGES)]


def nn_images(sizes):
    """vs_nn_images for a list of (h, w) image sizes stored back to back."""
    t = NNImages()
    t.n = len(sizes)
    for i, (h, w) in enumerate(sizes):
        t.h[i] = h
        t.w[i] = w
    return t


NN_MAX_LAYERS = 8


class TuneKey(C.Structure):
    _fields_ = [("arch", C.c_char * 32), ("n_cams", C.c_int32), ("canvas_w", C.c_int32), ("canvas_h", C.c_int32),
                ("lk_levels", C.c_int32), ("lk_radius", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("flow_variant", C.c_int32 * MAX_LEVELS), ("pyr_tile_rows", C.c_int32)]


def tune_entry(variants, pyr_tile_rows=0) -> TuneEntry:
    e = TuneEntry()
    for i, v in enumerate(variants):
        e.flow_variant[i] = v
    e.pyr_tile_rows = pyr_tile_rows
    return e


def tune_put(key: TuneKey, entry: TuneEntry):
    check(lib().vs_tune_put(C.byref(key), C.byref(entry)), "vs_tune_put")


def tune_get(key: TuneKey):
    """the record for key, or None"""
    e = TuneEntry()
    st = lib().vs_tune_get(C.byref(key), C.byref(e))
    if st == -6:
        return None
    check(st, "vs_tune_get")
    return e


def tune_clear():
    check(lib().vs_tune_clear(), "vs_tune_clear")


def tune_save(path):
    check(lib().vs_tune_save(os.fsencode(path)), "vs_tune_save")


def tune_load(path):
    check(lib().vs_tune_load(os.fsencode(path)), "vs_tune_load")


class NNSpec(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("cin", C.c_int32 * NN_MAX_LAYERS), ("cout", C.c_int32 * NN_MAX_LAYERS),
                ("in_live", C.c_int32), ("alpha", C.c_float), ("max_pixels", C.c_int64)]


def nn_spec(layers, in_live, alpha, max_pixels) -> NNSpec:
    sp = NNSpec()
    sp.n_layers = len(layers)
    for i, (ci, co) in enumerate(layers):
        sp.cin[i], sp.cout[i] = ci, co
    sp.in_live, sp.alpha, sp.max_pixels = in_live, alpha, max_pixels
    return sp


class FrameInfo(C.Structure):
    _fields_ = [("Mk", (C.c_float * 9) * MAX_CAMS), ("Mpair", (C.c_double * 9) * MAX_PAIRS),
                ("flags", C.c_int32 * MAX_PAIRS), ("quant", (C.c_int32 * 2) * 3),
                ("mbar", (C.c_double * 2) * 3), ("frames_seen", C.c_uint32),
                ("surr_ok", C.c_int32 * MAX_PAIRS), ("fb_err", C.c_float * MAX_PAIRS)]


_lib = None


def lib():
    """The loaded libvstitch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.vs_abi_version.restype = C.c_int
        L.vs_status_str.restype = C.c_char_p
        L.vs_status_str.argtypes = [C.c_int]
        L.vs_default_params.argtypes = [C.POINTER(Params)]
        L.vs_compose_homographies.argtypes = [C.POINTER(Rig), C.c_void_p, C.c_void_p]
        L.vs_create.argtypes = [C.POINTER(Rig), C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.vs_destroy.argtypes = [C.c_void_p]
        L.vs_destroy.restype = None
        L.vs_query.argtypes = [C.c_void_p, C.POINTER(PlanInfo)]
        L.vs_last_error.restype = C.c_char_p
        L.vs_last_error.argtypes = [C.c_void_p]
        L.vs_stitch.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(ColorState), C.c_void_p,
                                C.POINTER(ColorState), C.POINTER(FrameInfo), C.c_void_p]
        L.vs_state_get.argtypes = [C.c_void_p, C.POINTER(ColorState)]
        L.vs_state_set.argtypes = [C.c_void_p, C.POINTER(ColorState)]
        L.vs_debug_tap.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_size_t]
        L.vs_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.vs_get_timing.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32)]
        L.vs_set_flow_variant.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.vs_get_flow_variant.argtypes = [C.c_void_p, C.c_void_p]
        L.vs_load_weights.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.vs_set_flow_mode.argtypes = [C.c_void_p, C.c_int, C.c_float]
        L.vs_batch_create.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]
        L.vs_batch_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vs_batch_destroy.argtypes = [C.c_void_p]
        L.vs_batch_last_error.restype = C.c_char_p
        L.vs_batch_last_error.argtypes = [C.c_void_p]
        L.vs_batch_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                        C.c_void_p]
        L.vs_tune_put.argtypes = [C.POINTER(TuneKey), C.POINTER(TuneEntry)]
        L.vs_tune_get.argtypes = [C.POINTER(TuneKey), C.POINTER(TuneEntry)]
        L.vs_tune_clear.argtypes = []
        L.vs_tune_save.argtypes = [C.c_char_p]
        L.vs_tune_load.argtypes = [C.c_char_p]
        L.vs_tune_key_of.argtypes = [C.c_void_p, C.POINTER(TuneKey)]
        L.vs_get_tuning.argtypes = [C.c_void_p, C.POINTER(TuneEntry)]
        vp, i32, i64, f32 = C.c_void_p, C.c_int, C.c_int64, C.c_float
        imgs = C.POINTER(NNImages)
        L.vs_nn_conv3x3.argtypes = [vp, i32, vp, vp, vp, i32, imgs, i32, f32, vp]
        L.vs_nn_wgrad_scratch_bytes.restype = C.c_size_t
        L.vs_nn_wgrad_scratch_bytes.argtypes = [i32, i32, imgs]
        L.vs_nn_conv3x3_wgrad.argtypes = [vp, i32, vp, i32, imgs, vp, C.c_size_t, vp, vp]
        L.vs_nn_flip_weights.argtypes = [vp, vp, i32, i32, vp]
        L.vs_nn_lrelu_bwd.argtypes = [vp, vp, vp, i64, f32, vp]
        L.vs_nn_pack_pair.argtypes = [vp, vp, vp, i64, vp]
        L.vs_nn_epe_loss.argtypes = [vp, vp, vp, vp, i64, vp]
        L.vs_nn_adam.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
        L.vs_nn_to_bf16.argtypes = [vp, vp, i64, vp]
        L.vs_nn_pool_flow.argtypes = [vp, i32, i32, i32, vp, vp]
        L.vs_nn_create.argtypes = [C.POINTER(NNSpec), C.c_uint64, C.POINTER(C.c_void_p)]
        L.vs_nn_destroy.argtypes = [vp]
        L.vs_nn_forward.argtypes = [vp, vp, imgs, vp, vp]
        L.vs_nn_loss.argtypes = [vp, vp, vp, vp]
        L.vs_nn_backward.argtypes = [vp, vp, vp, vp]
        L.vs_nn_adam_step.argtypes = [vp, f32, f32, f32, f32, vp]
        L.vs_nn_params.argtypes = [vp, vp, vp, C.POINTER(C.c_size_t), vp]
        L.vs_nn_save.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.vs_nn_load.argtypes = [vp, vp, C.c_size_t]
        L.vs_flow_create.argtypes = [i32, i32, C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.vs_flow_run.argtypes = [vp, vp, vp, vp, vp, vp]
        L.vs_flow_destroy.argtypes = [vp]
        L.vs_flow_level.argtypes = [vp, i32, vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp]
        L.vs_flow_only.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
        L.vs_flow_run_noalloc.argtypes = [i32, i32, C.POINTER(Params), vp, vp, vp, vp, vp]
        dbl = C.c_double
        L.vs_calib_intrinsics.argtypes = [dbl] * 7 + [vp]
        L.vs_calib_plane_homography.argtypes = [vp, vp, vp, vp]
        L.vs_calib_pair.argtypes = [vp, vp, vp]
        L.vs_calib_refine.argtypes = [vp, vp, vp]
        L.vs_calib_estimate.argtypes = [vp, i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, vp,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp]
        _lib = L
    return _lib


class VSError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def make_rig(rig: dict) -> Rig:
    r = Rig()
    n = rig["n_cams"]
    r.n_cams = n
    for k in range(n):
        w = rig["cam_w"][k] if "cam_w" in rig else rig["W"]
        h = rig["cam_h"][k] if "cam_h" in rig else rig["H"]
        r.cam_w[k] = w
        r.cam_h[k] = h
        r.cam_pitch[k] = rig["cam_pitch"][k] if "cam_pitch" in rig else 3 * w
    for k in range(1, n):
        hp = np.asarray(rig["H_pair"][k], dtype=np.float64).ravel()
        for i in range(9):
            r.H_pair[k][i] = float(hp[i])
    href = np.asarray(rig["H_ref"], dtype=np.float64).ravel()
    for i in range(9):
        r.H_ref[i] = float(href[i])
    r.ring = int(rig.get("ring", 0))
    r.ring_period = int(rig.get("ring_period", 0))
    r.canvas_w = int(rig["canvas_w"])
    r.canvas_h = int(rig["canvas_h"])
    return r


def default_params(**over) -> Params:
    p = Params()
    lib().vs_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def compose_homographies(rig: dict):
    r = make_rig(rig)
    n = rig["n_cams"]
    Hk = np.zeros((n, 9), np.float64)
    Hinv = np.zeros((n, 9), np.float32)
    st = lib().vs_compose_homographies(C.byref(r), Hk.ctypes.data_as(C.c_void_p),
                                       Hinv.ctypes.data_as(C.c_void_p))
    if st != 0:
        raise VSError(st, "compose")
    return Hk.reshape(n, 3, 3), Hinv.reshape(n, 3, 3)


def _stream_handle(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream)


class Stitcher:
    """One stitching context: one camera rig, its workspaces and colour state."""

    def __init__(self, rig: dict, **params):
        self.rig_struct = make_rig(rig)
        self.params = default_params(**params)
        h = C.c_void_p()
        st = lib().vs_create(C.byref(self.rig_struct), C.byref(self.params), C.byref(h))
        if st != 0:
            raise VSError(st, "vs_create")
        self.h = h
        info = PlanInfo()
        lib().vs_query(self.h, C.byref(info))
        self.info = info
        self.n_cams = rig["n_cams"]
        self.cam_shape = [(self.rig_struct.cam_h[k], self.rig_struct.cam_w[k])
                          for k in range(self.n_cams)]

    def close(self):
        if getattr(self, "h", None):
            lib().vs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals already gone
            pass

    @property
    def canvas(self):
        return self.info.canvas_h, self.info.canvas_w

    @property
    def n_pairs(self):
        return self.info.n_pairs

    def strip_box(self, p):
        I = self.info
        return I.strip_x0[p], I.strip_y0[p], I.strip_w[p], I.strip_h[p]

    def _err(self, st, what):
        raise VSError(st, f"{what}: {lib().vs_last_error(self.h).decode()}")

    def new_pano(self, device="cuda"):
        H, W = self.canvas
        return torch.empty((H, W, 3), dtype=torch.uint8, device=device)

    def stitch(self, frames, pano=None, state_in: ColorState | None = None, want_state=False,
               want_info=False, stream=None):
        """Stitch one frame of device tensors (H, W, 3) uint8; returns the panorama
        (and the state / frame info when asked)."""
        if len(frames) != self.n_cams:
            raise ValueError("one frame per camera")
        for k, f in enumerate(frames):
            if (f.dtype != torch.uint8 or not f.is_cuda or tuple(f.shape) != self.cam_shape[k] + (3,)
                    or not f.is_contiguous()):
                raise ValueError(f"frame {k}: need a contiguous cuda uint8 tensor of shape "
                                 f"{self.cam_shape[k] + (3,)}")
        dev = frames[0].device
        if any(f.device != dev for f in frames):
            raise ValueError("frames: all on one device")
        if pano is None:
            pano = self.new_pano(dev)
        _check_pano(pano, self.canvas, dev)
        ptrs = (C.c_void_p * self.n_cams)(*[f.data_ptr() for f in frames])
        out = ColorState() if want_state else None
        info = FrameInfo() if want_info else None
        st = lib().vs_stitch(self.h, ptrs, C.byref(state_in) if state_in is not None else None,
                             C.c_void_p(pano.data_ptr()), C.byref(out) if out is not None else None,
                             C.byref(info) if info is not None else None, _stream_handle(stream))
        if st != 0:
            self._err(st, "vs_stitch")
        if want_state or want_info:
            return pano, out, info
        return pano

    def state_get(self) -> ColorState:
        s = ColorState()
        st = lib().vs_state_get(self.h, C.byref(s))
        if st != 0:
            self._err(st, "vs_state_get")
        return s

    def state_set(self, s: ColorState):
        st = lib().vs_state_set(self.h, C.byref(s))
        if st != 0:
            self._err(st, "vs_state_set")

    def set_timing(self, on=True):
        st = lib().vs_set_timing(self.h, 1 if on else 0)
        if st != 0:
            self._err(st, "vs_set_timing")

    TIMING_STEPS = ("colour", "pyramids", "flow", "blend", "balance", "frame")

    def timing(self):
        """(summed step times in ms over the timed frames, number of frames)"""
        ms = np.zeros(6, np.float64)
        n = C.c_uint32()
        st = lib().vs_get_timing(self.h, ms.ctypes.data_as(C.c_void_p), C.byref(n))
        if st != 0:
            self._err(st, "vs_get_timing")
        return ms, n.value

    def tune_key(self) -> TuneKey:
        k = TuneKey()
        check(lib().vs_tune_key_of(self.h, C.byref(k)), "vs_tune_key_of")
        return k

    def tuning(self) -> TuneEntry:
        """the context's current flow variants and fused-pyramid tile height"""
        e = TuneEntry()
        check(lib().vs_get_tuning(self.h, C.byref(e)), "vs_get_tuning")
        return e

    def flow_variants(self):
        v = np.zeros(MAX_LEVELS, np.int32)
        lib().vs_get_flow_variant(self.h, v.ctypes.data_as(C.c_void_p))
        return v[:self.info.lk_levels].tolist()

    def set_flow_variant(self, level: int, variant: int):
        st = lib().vs_set_flow_variant(self.h, level, variant)
        if st != 0:
            self._err(st, "vs_set_flow_variant")

    def load_weights(self, blob: bytes):
        """Copy a surrogate weight file ("VSNN" v1) into the context."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        st = lib().vs_load_weights(self.h, buf, len(blob))
        if st != 0:
            self._err(st, "vs_load_weights")

    def set_flow_mode(self, mode: int, fb_tau_px: float = 0.0):
        """FLOW_PLAIN, FLOW_SURROGATE or FLOW_SURROGATE_FALLBACK (threshold in px)."""
        st = lib().vs_set_flow_mode(self.h, mode, fb_tau_px)
        if st != 0:
            self._err(st, "vs_set_flow_mode")

    def flow_only(self, strip_i, strip_j, stream=None):
        """The context's plain flow on a caller strip pair: RGB uint8 device
        tensors (h, w, 3), camera i (moving) and camera j (template); returns
        (flow_ij, flow_ji), float32 (h, w, 2)."""
        for t in (strip_i, strip_j):
            if (t.dtype != torch.uint8 or not t.is_cuda or t.dim() != 3 or t.shape[2] != 3
                    or not t.is_contiguous() or t.shape != strip_i.shape):
                raise ValueError("strips: contiguous cuda uint8 (h, w, 3), both the same shape")
        h, w = int(strip_i.shape[0]), int(strip_i.shape[1])
        fij = torch.empty((h, w, 2), dtype=torch.float32, device=strip_i.device)
        fji = torch.empty_like(fij)
        st = lib().vs_flow_only(self.h, _p(strip_i), _p(strip_j), w, h, _p(fij), _p(fji), _stream_handle(stream))
        if st != 0:
            self._err(st, "vs_flow_only")
        return fij, fji

    def tap(self, name: str, pair: int = 0, sub: int = 0) -> np.ndarray:
        I = self.info
        H, W = self.canvas
        sw, sh = (I.strip_w[pair], I.strip_h[pair]) if 0 <= pair < I.n_pairs else (0, 0)
        shapes = dict(strip=((sh, sw, 3), np.uint8), mask=((sh, sw), np.uint8),
                      hist=((2, 3, 256), np.uint32), lut=((3, 256), np.uint8), mom=((16,), np.uint64),
                      mpair=((I.n_pairs, 3, 3), np.float64), mk=((self.n_cams, 3, 3), np.float32),
                      flags=((I.n_pairs,), np.int32), flow=((sh, sw, 2), np.float32),
                      pano_pre=((H, W, 3), np.uint8), pano_hist=((3, 256), np.uint32),
                      bal_lut=((3, 256), np.uint8), quant=((3, 2), np.int32),
                      mbar=((3, 2), np.float64), cover=((H, W), np.uint8),
                      deferred=((1,), np.uint32), fb=((I.n_pairs, 2), np.uint64),
                      surr_ok=((I.n_pairs,), np.int32))
        if name in ("pyr", "need", "surr_pred"):
            w, h = sw, sh
            for _ in range(sub % 8 if name != "surr_pred" else 2):
                w, h = (w + 1) // 2, (h + 1) // 2
            if name == "surr_pred":
                shape, dt = (h, w, 2), np.float32
            else:
                shape, dt = (h, w), (np.float32 if name == "pyr" else np.uint8)
        else:
            shape, dt = shapes[name]
        out = np.zeros(shape, dt)
        st = lib().vs_debug_tap(self.h, TAP[name], pair, sub, out.ctypes.data_as(C.c_void_p),
                                out.nbytes)
        if st != 0:
            self._err(st, f"vs_debug_tap({name})")
        return out


def state_bytes(s: ColorState) -> bytes:
    return bytes(s)


def state_from_bytes(b: bytes) -> ColorState:
    s = ColorState()
    C.memmove(C.addressof(s), b, C.sizeof(s))
    return s


class Batch:
    """Several stitching contexts run by one captured per-frame graph."""

    def __init__(self, stitchers):
        self.stitchers = list(stitchers)
        arr = (C.c_void_p * len(self.stitchers))(*[st.h.value for st in self.stitchers])
        h = C.c_void_p()
        st = lib().vs_batch_create(arr, len(self.stitchers), C.byref(h))
        if st != 0:
            raise VSError(st, "vs_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().vs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals already gone
            pass

    def _ptrs(self, frames, panos):
        n = len(self.stitchers)
        if len(frames) != n or len(panos) != n:
            raise ValueError("one frame list and one panorama per context")
        rows = []
        for st, fr, pano in zip(self.stitchers, frames, panos):
            if len(fr) != st.n_cams:
                raise ValueError("one frame per camera")
            for k, f in enumerate(fr):
                if (f.dtype != torch.uint8 or not f.is_cuda or not f.is_contiguous()
                        or tuple(f.shape) != st.cam_shape[k] + (3,)):
                    raise ValueError("frames: contiguous cuda uint8 (H, W, 3)")
            if any(f.device != fr[0].device for f in fr):
                raise ValueError("frames: all on one device")
            _check_pano(pano, st.canvas, fr[0].device)
            rows.append((C.c_void_p * st.n_cams)(*[f.data_ptr() for f in fr]))
        self._keep = rows
        fr_arr = (C.c_void_p * n)(*[C.cast(r, C.c_void_p).value for r in rows])
        pano_arr = (C.c_void_p * n)(*[p.data_ptr() for p in panos])
        return fr_arr, pano_arr

    def run(self, frames, panos, stream=None):
        fr_arr, pano_arr = self._ptrs(frames, panos)
        st = lib().vs_batch_run(self.h, fr_arr, pano_arr, _stream_handle(stream))
        if st != 0:
            raise VSError(st, lib().vs_batch_last_error(self.h).decode())
        return panos

    def autotune(self, frames, panos, reps=5):
        fr_arr, pano_arr = self._ptrs(frames, panos)
        ms = np.zeros((MAX_LEVELS, FLOW_VARIANTS), np.float32)
        choice = np.zeros(MAX_LEVELS, np.int32)
        st = lib().vs_batch_autotune(self.h, fr_arr, pano_arr, reps, ms.ctypes.data_as(C.c_void_p),
                                     choice.ctypes.data_as(C.c_void_p))
        if st != 0:
            raise VSError(st, lib().vs_batch_last_error(self.h).decode())
        L = self.stitchers[0].info.lk_levels
        return choice[:L].tolist(), ms[:L]


def _check_pano(pano, canvas, device):
    """The panorama is written by the kernels: a contiguous uint8 device tensor
    of the canvas shape on the frames' device (a host tensor's address would
    reach the kernels' stores)."""
    H, W = canvas
    if (not isinstance(pano, torch.Tensor) or pano.dtype != torch.uint8 or tuple(pano.shape) != (H, W, 3)
            or not pano.is_contiguous()):
        raise ValueError("pano: contiguous uint8 (canvas_h, canvas_w, 3)")
    if not pano.is_cuda or pano.device != device:
        raise ValueError(f"pano: must be a device tensor on {device} (the frames' device), got {pano.device}")


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def check(status, what):
    if status != 0:
        raise VSError(status, what)


class PlainFlow:
    """The plain pyramidal flow on caller luma pairs (device float32 [h][w])."""

    def __init__(self, w: int, h: int, **params):
        self.w, self.h = w, h
        prm = default_params(**params)
        hnd = C.c_void_p()
        check(lib().vs_flow_create(w, h, C.byref(prm), C.byref(hnd)), "vs_flow_create")
        self.hnd = hnd

    def close(self):
        if getattr(self, "hnd", None):
            lib().vs_flow_destroy(self.hnd)
            self.hnd = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals already gone
            pass

    def __call__(self, yt, ym, stream=None):
        """(flow of template yt vs moving ym, the reverse flow), float32 [h][w][2]"""
        for t in (yt, ym):
            if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != (self.h, self.w) or not t.is_contiguous():
                raise ValueError("luma: contiguous cuda float32 (h, w)")
        ftm = torch.empty((self.h, self.w, 2), dtype=torch.float32, device=yt.device)
        fmt = torch.empty_like(ftm)
        check(lib().vs_flow_run(self.hnd, _p(yt), _p(ym), _p(ftm), _p(fmt), _stream_handle(stream)), "vs_flow_run")
        return ftm, fmt

    def level(self, level: int, stream=None):
        """(template, moving) luma at a pyramid level of the last run"""
        w, h = C.c_int32(), C.c_int32()
        check(lib().vs_flow_level(self.hnd, level, None, None, C.byref(w), C.byref(h), None), "vs_flow_level")
        yt = torch.empty((h.value, w.value), dtype=torch.float32, device="cuda")
        ym = torch.empty_like(yt)
        check(lib().vs_flow_level(self.hnd, level, _p(yt), _p(ym), None, None, _stream_handle(stream)),
              "vs_flow_level")
        return yt, ym


def flow_run_noalloc(yt, ym, flow_tm=None, flow_mt=None, stream=None, **params):
    """vs_flow_run_noalloc: the plain flow of template yt vs moving ym (device
    float32 [h][w]) in the library's static workspace, into caller tensors
    flow_tm / flow_mt (float32 [h][w][2], created here when None; either may
    be passed as False to skip it).  Returns (flow_tm, flow_mt)."""
    h, w = tuple(yt.shape)
    for t in (yt, ym):
        if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != (h, w) or not t.is_contiguous():
            raise ValueError("luma: contiguous cuda float32 (h, w), both the same shape")
    outs = []
    for f in (flow_tm, flow_mt):
        if f is None:
            f = torch.empty((h, w, 2), dtype=torch.float32, device=yt.device)
        elif f is not False and (f.dtype != torch.float32 or f.device != yt.device or tuple(f.shape) != (h, w, 2)
                                 or not f.is_contiguous()):
            raise ValueError("flow: contiguous float32 (h, w, 2) on the luma's device")
        outs.append(f)
    prm = default_params(**params)
    check(lib().vs_flow_run_noalloc(w, h, C.byref(prm), _p(yt), _p(ym),
                                    _p(outs[0]) if outs[0] is not False else None,
                                    _p(outs[1]) if outs[1] is not False else None, _stream_handle(stream)),
          "vs_flow_run_noalloc")
    return outs[0], outs[1]


# ---- section 3.1 set-up ----------------------------------------------------

def _d(a, n):
    return np.ascontiguousarray(np.asarray(a, np.float64).reshape(n))


def calib_intrinsics(f, dx, dy, cx, cy, u0, v0):
    K = np.zeros(9)
    check(lib().vs_calib_intrinsics(f, dx, dy, cx, cy, u0, v0, K.ctypes.data_as(C.c_void_p)), "vs_calib_intrinsics")
    return K.reshape(3, 3)


def calib_plane_homography(K, R, t):
    H = np.zeros(9)
    k, r, tt = _d(K, 9), _d(R, 9), _d(t, 3)
    check(lib().vs_calib_plane_homography(k.ctypes.data_as(C.c_void_p), r.ctypes.data_as(C.c_void_p),
                                          tt.ctypes.data_as(C.c_void_p), H.ctypes.data_as(C.c_void_p)),
          "vs_calib_plane_homography")
    return H.reshape(3, 3)


def calib_pair(Ha, Hb):
    H = np.zeros(9)
    a, b = _d(Ha, 9), _d(Hb, 9)
    check(lib().vs_calib_pair(a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                              H.ctypes.data_as(C.c_void_p)), "vs_calib_pair")
    return H.reshape(3, 3)


def calib_refine(H, p):
    out = np.zeros(9)
    h, pp = _d(H, 9), _d(p, 4)
    check(lib().vs_calib_refine(h.ctypes.data_as(C.c_void_p), pp.ctypes.data_as(C.c_void_p),
                                out.ctypes.data_as(C.c_void_p)), "vs_calib_refine")
    return out.reshape(3, 3)


def calib_estimate(frame_a, frame_b, H, margin=16, radius=4, stream=None):
    """(p = (tx, ty, sx, sy) or None, matches, inliers) for device frames a, b
    (uint8 HWC) and the pre-warp H (a pixels -> b pixels)"""
    for f in (frame_a, frame_b):
        if f.dtype != torch.uint8 or not f.is_cuda or f.dim() != 3 or f.shape[2] != 3 or not f.is_contiguous():
            raise ValueError("frames: contiguous cuda uint8 (h, w, 3)")
    h = _d(H, 9)
    p = np.zeros(4)
    nm, ni = C.c_int32(), C.c_int32()
    st = lib().vs_calib_estimate(_p(frame_a), frame_a.shape[1] * 3, frame_a.shape[1], frame_a.shape[0], _p(frame_b),
                                 frame_b.shape[1] * 3, frame_b.shape[1], frame_b.shape[0],
                                 h.ctypes.data_as(C.c_void_p), margin, radius, p.ctypes.data_as(C.c_void_p),
                                 C.byref(nm), C.byref(ni), _stream_handle(stream))
    if st not in (0, -1):
        raise VSError(st, "vs_calib_estimate")
    return (p if st == 0 else None), nm.value, ni.value
