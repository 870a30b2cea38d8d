"""ctypes front end of the plain CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the stitching library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "vso_oracle.c")
SRC_CALIB = os.path.join(HERE, "vso_calib.c")
SRC_VAR = os.path.join(HERE, "vso_var.c")

MAX_CAMS = 16
MAX_PAIRS = 16

TAP = dict(strip=1, mask=2, hist=3, lut=4, mom=5, mpair=6, mk=7, flags=8, pyr=9, flow=10,
           pano_pre=11, pano_hist=12, bal_lut=13, quant=14, mbar=15, cover=16, need=17,
           surr_pred=18, fb=19, surr_ok=20)

FLOW_PLAIN, FLOW_SURROGATE, FLOW_FALLBACK = 0, 1, 2


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no FP contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", LIB_PATH + ".tmp", SRC, SRC_CALIB, SRC_VAR, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Rig(C.Structure):
    _fields_ = [("n_cams", C.c_int), ("cam_w", C.c_int * MAX_CAMS), ("cam_h", C.c_int * MAX_CAMS),
                ("H_pair", (C.c_double * 9) * MAX_CAMS), ("H_ref", C.c_double * 9),
                ("ring", C.c_int), ("ring_period", C.c_int), ("canvas_w", C.c_int),
                ("canvas_h", C.c_int)]


class Params(C.Structure):
    _fields_ = [("color_window", C.c_int), ("ridge", C.c_double), ("min_pixels", C.c_int),
                ("flow", C.c_int), ("lk_levels", C.c_int), ("lk_iters", C.c_int),
                ("lk_radius", C.c_int), ("lk_lambda", C.c_float), ("balance", C.c_int),
                ("lambda_pct", C.c_int), ("readings", C.c_int), ("var_alpha", C.c_float),
                ("var_gamma", C.c_float), ("var_outer", C.c_int), ("var_inner", C.c_int)]


READ_OVERLAP_ONLY, READ_LITERAL_EQ17, READ_NEAREST_CDF = 1, 2, 4


class PlanInfo(C.Structure):
    _fields_ = [("canvas_w", C.c_int), ("canvas_h", C.c_int), ("n_pairs", C.c_int),
                ("n_cams", C.c_int), ("ring", C.c_int), ("ring_period", C.c_int),
                ("pair_j", C.c_int * MAX_PAIRS), ("pair_i", C.c_int * MAX_PAIRS),
                ("pair_si", C.c_int * MAX_PAIRS),
                ("strip_x0", C.c_int * MAX_PAIRS), ("strip_y0", C.c_int * MAX_PAIRS),
                ("strip_w", C.c_int * MAX_PAIRS), ("strip_h", C.c_int * MAX_PAIRS),
                ("hinv", (C.c_float * 9) * MAX_CAMS), ("hk", (C.c_double * 9) * MAX_CAMS),
                ("n_covered", C.c_longlong)]


class View(C.Structure):
    _fields_ = [("frame", C.c_void_p), ("pitch", C.c_int), ("W", C.c_int), ("H", C.c_int),
                ("hinv", C.c_void_p), ("M", C.c_void_p), ("X", C.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.vso_create.restype = C.c_void_p
        L.vso_create.argtypes = [C.POINTER(Rig), C.POINTER(Params), C.POINTER(C.c_int)]
        L.vso_destroy.argtypes = [C.c_void_p]
        L.vso_plan_info_get.argtypes = [C.c_void_p, C.POINTER(PlanInfo)]
        L.vso_stitch.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.c_void_p]
        L.vso_reset.argtypes = [C.c_void_p]
        L.vso_frames_seen.argtypes = [C.c_void_p]
        L.vso_step_times.argtypes = [C.c_void_p, C.c_void_p]
        L.vso_get.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_size_t]
        L.vso_default_params.argtypes = [C.POINTER(Params)]
        L.vso_histspec_lut.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.vso_histspec_lut_nearest.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.vso_solve_color.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.vso_quantiles.argtypes = [C.c_void_p, C.c_longlong, C.c_int, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
        L.vso_balance_lut.argtypes = [C.c_double, C.c_double, C.c_int, C.c_void_p]
        L.vso_pyr_down.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.vso_lk_level.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int,
                                   C.c_int, C.c_int, C.c_int, C.c_float, C.c_void_p, C.c_void_p]
        L.vso_lk_level_f64.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                       C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p]
        L.vso_hom_valid.argtypes = [C.c_void_p, C.c_float, C.c_float, C.c_int, C.c_int,
                                    C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.vso_bilinear.restype = C.c_float
        L.vso_bilinear.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float,
                                   C.c_float]
        L.vso_round8.argtypes = [C.c_float]
        L.vso_var_level.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_float, C.c_float,
                                    C.c_int, C.c_int, C.c_void_p]
        L.vso_var_pyramid.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                      C.c_float, C.c_float, C.c_int, C.c_int, C.c_void_p]
        dbl = C.c_double
        L.vso_calib_intrinsics.argtypes = [dbl] * 7 + [C.c_void_p]
        L.vso_calib_plane_homography.argtypes = [C.c_void_p] * 4
        L.vso_calib_pair.argtypes = [C.c_void_p] * 3
        L.vso_calib_refine.argtypes = [C.c_void_p] * 3
        L.vso_calib_harris.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.vso_calib_harris.restype = C.c_float
        L.vso_calib_ncc.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.vso_calib_ncc.restype = C.c_float
        L.vso_calib_estimate.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vso_luma.argtypes = [C.c_int, C.c_int, C.c_int]
        L.vso_chain_colour.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.vso_fuse_pixel.argtypes = [C.POINTER(View), C.POINTER(View), C.c_float, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.vso_fuse_pixel_literal.argtypes = [C.POINTER(View), C.POINTER(View), C.c_float, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        vp, i = C.c_void_p, C.c_int
        L.vso_conv3x3.argtypes = [vp, i, i, i, i, vp, vp, i, vp]
        L.vso_conv3x3_bwd_data.argtypes = [vp, i, i, i, i, vp, i, vp]
        L.vso_conv3x3_bwd_weight.argtypes = [vp, vp, i, i, i, i, i, vp, vp]
        L.vso_set_surrogate.argtypes = [vp, vp, C.c_size_t, i, C.c_float]
        L.vso_surrogate_net.argtypes = [vp, C.c_size_t, vp, vp, i, i, vp]
        L.vso_surr_upsample.argtypes = [vp, i, i, vp, i, i, vp]
        L.vso_fb_check.argtypes = [vp, vp, i, i, vp, i, i, C.POINTER(C.c_ulonglong), C.POINTER(C.c_ulonglong)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_rig(rig: dict) -> Rig:
    r = Rig()
    n = rig["n_cams"]
    r.n_cams = n
    W = rig["W"] if "W" in rig else None
    for k in range(n):
        r.cam_w[k] = rig["cam_w"][k] if "cam_w" in rig else W
        r.cam_h[k] = rig["cam_h"][k] if "cam_h" in rig else rig["H"]
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
    lib().vso_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


class OracleError(RuntimeError):
    pass


class Oracle:
    """One stitching context on the CPU oracle."""

    def __init__(self, rig: dict, **params):
        self.rig_struct = make_rig(rig)
        self.params = default_params(**params)
        st = C.c_int(0)
        self.h = lib().vso_create(C.byref(self.rig_struct), C.byref(self.params), C.byref(st))
        if not self.h:
            raise OracleError(f"vso_create failed: status {st.value}")
        self.status = st.value
        pi = PlanInfo()
        lib().vso_plan_info_get(self.h, C.byref(pi))
        self.plan = pi
        self.n_cams = rig["n_cams"]

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            try:
                _lib.vso_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.h = None

    @property
    def canvas(self):
        return self.plan.canvas_h, self.plan.canvas_w

    @property
    def n_pairs(self):
        return self.plan.n_pairs

    def strip_box(self, p):
        P = self.plan
        return P.strip_x0[p], P.strip_y0[p], P.strip_w[p], P.strip_h[p]

    def stitch(self, frames) -> np.ndarray:
        frames = [np.ascontiguousarray(f, dtype=np.uint8) for f in frames]
        arr = (C.c_void_p * self.n_cams)(*[f.ctypes.data for f in frames])
        pitch = (C.c_int * self.n_cams)(*[f.shape[1] * 3 for f in frames])
        H, W = self.canvas
        pano = np.zeros((H, W, 3), dtype=np.uint8)
        st = lib().vso_stitch(self.h, arr, pitch, _ptr(pano))
        if st != 0:
            raise OracleError(f"vso_stitch failed: {st}")
        return pano

    def set_surrogate(self, blob: bytes | None, mode: int, tau: float = 0.0):
        """Load a surrogate weight file (None keeps the loaded one) and pick the
        flow mode (FLOW_PLAIN / FLOW_SURROGATE / FLOW_FALLBACK, threshold tau px)."""
        if blob is None:
            st = lib().vso_set_surrogate(self.h, None, 0, mode, tau)
        else:
            buf = C.create_string_buffer(bytes(blob), len(blob))
            st = lib().vso_set_surrogate(self.h, buf, len(blob), mode, tau)
        if st != 0:
            raise OracleError(f"vso_set_surrogate failed: {st}")

    def reset(self):
        lib().vso_reset(self.h)

    def frames_seen(self) -> int:
        return lib().vso_frames_seen(self.h)

    STEPS = ("strips", "moments", "solve", "pyramids", "flow", "blend", "balance")

    def step_times(self) -> dict:
        """wall seconds per step, summed over the frames stitched so far"""
        out = np.zeros(7, np.float64)
        lib().vso_step_times(self.h, _ptr(out))
        return dict(zip(self.STEPS, out.tolist()))

    def tap(self, name: str, pair: int = 0, sub: int = 0) -> np.ndarray:
        P = self.plan
        H, W = self.canvas
        sw, sh = (P.strip_w[pair], P.strip_h[pair]) if 0 <= pair < P.n_pairs else (0, 0)
        if name == "strip":
            out = np.zeros((sh, sw, 3), np.uint8)
        elif name == "mask":
            out = np.zeros((sh, sw), np.uint8)
        elif name == "hist":
            out = np.zeros((2, 3, 256), np.uint32)
        elif name == "lut":
            out = np.zeros((3, 256), np.uint8)
        elif name == "mom":
            out = np.zeros(16, np.uint64)
        elif name == "mpair":
            out = np.zeros((P.n_pairs, 3, 3), np.float64)
        elif name == "mk":
            out = np.zeros((self.n_cams, 3, 3), np.float32)
        elif name == "flags":
            out = np.zeros(P.n_pairs, np.int32)
        elif name in ("pyr", "need"):
            lvl = sub % 8
            w, h = sw, sh
            for _ in range(lvl):
                w, h = (w + 1) // 2, (h + 1) // 2
            out = np.zeros((h, w), np.float32 if name == "pyr" else np.uint8)
        elif name == "flow":
            out = np.zeros((sh, sw, 2), np.float32)
        elif name == "surr_pred":
            w, h = sw, sh
            for _ in range(2):
                w, h = (w + 1) // 2, (h + 1) // 2
            out = np.zeros((h, w, 2), np.float32)
        elif name == "fb":
            out = np.zeros((P.n_pairs, 2), np.uint64)
        elif name == "surr_ok":
            out = np.zeros(P.n_pairs, np.int32)
        elif name == "pano_pre":
            out = np.zeros((H, W, 3), np.uint8)
        elif name == "pano_hist":
            out = np.zeros((3, 256), np.uint32)
        elif name == "bal_lut":
            out = np.zeros((3, 256), np.uint8)
        elif name == "quant":
            out = np.zeros((3, 2), np.int32)
        elif name == "mbar":
            out = np.zeros((3, 2), np.float64)
        elif name == "cover":
            out = np.zeros((H, W), np.uint8)
        else:
            raise KeyError(name)
        st = lib().vso_get(self.h, TAP[name], pair, sub, _ptr(out), out.nbytes)
        if st != 0:
            raise OracleError(f"vso_get({name}) failed: {st}")
        return out


# ---- single steps --------------------------------------------------------

def histspec_lut(Gi, Gj, nearest=False) -> np.ndarray:
    Gi = np.ascontiguousarray(Gi, np.uint32)
    Gj = np.ascontiguousarray(Gj, np.uint32)
    out = np.zeros(256, np.uint8)
    (lib().vso_histspec_lut_nearest if nearest else lib().vso_histspec_lut)(_ptr(Gi), _ptr(Gj), _ptr(out))
    return out


def solve_color(A, B, ridge=1e-9):
    A = np.ascontiguousarray(A, np.float64).reshape(9)
    B = np.ascontiguousarray(B, np.float64).reshape(9)
    M = np.zeros(9, np.float64)
    flag = lib().vso_solve_color(_ptr(A), _ptr(B), ridge, _ptr(M))
    return M.reshape(3, 3), flag


def quantiles(hist, n, lambda_pct=5):
    h = np.ascontiguousarray(hist, np.uint32)
    q1, q2 = C.c_int(), C.c_int()
    lib().vso_quantiles(_ptr(h), int(n), lambda_pct, C.byref(q1), C.byref(q2))
    return q1.value, q2.value


def balance_lut(m1, m2, lambda_pct=5) -> np.ndarray:
    out = np.zeros(256, np.uint8)
    lib().vso_balance_lut(float(m1), float(m2), lambda_pct, _ptr(out))
    return out


def pyr_down(img) -> np.ndarray:
    img = np.ascontiguousarray(img, np.float32)
    h, w = img.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2), np.float32)
    lib().vso_pyr_down(_ptr(img), w, h, _ptr(out))
    return out


def lk_level(T, Mv, u_coarse=None, radius=4, iters=5, lam=1.0, need=None) -> np.ndarray:
    T = np.ascontiguousarray(T, np.float32)
    Mv = np.ascontiguousarray(Mv, np.float32)
    h, w = T.shape
    out = np.zeros((h, w, 2), np.float32)
    nd = None if need is None else np.ascontiguousarray(need, np.uint8)
    ndp = None if nd is None else _ptr(nd)
    if u_coarse is not None:
        uc = np.ascontiguousarray(u_coarse, np.float32)
        lib().vso_lk_level(_ptr(T), _ptr(Mv), w, h, _ptr(uc), uc.shape[1], uc.shape[0], radius,
                           iters, lam, ndp, _ptr(out))
    else:
        lib().vso_lk_level(_ptr(T), _ptr(Mv), w, h, None, 0, 0, radius, iters, lam, ndp, _ptr(out))
    return out


def lk_level_f64(T, Mv, u_coarse=None, radius=4, iters=5, lam=1.0) -> np.ndarray:
    T = np.ascontiguousarray(T, np.float64)
    Mv = np.ascontiguousarray(Mv, np.float64)
    h, w = T.shape
    out = np.zeros((h, w, 2), np.float64)
    if u_coarse is not None:
        uc = np.ascontiguousarray(u_coarse, np.float64)
        lib().vso_lk_level_f64(_ptr(T), _ptr(Mv), w, h, _ptr(uc), uc.shape[1], uc.shape[0],
                               radius, iters, lam, _ptr(out))
    else:
        lib().vso_lk_level_f64(_ptr(T), _ptr(Mv), w, h, None, 0, 0, radius, iters, lam, _ptr(out))
    return out


def pyramid_flow(Tpyr, Mpyr, radius=4, iters=5, lam=1.0, f64=False):
    """Coarse-to-fine flow over lists of pyramid levels (finest first)."""
    u = None
    for l in range(len(Tpyr) - 1, -1, -1):
        f = lk_level_f64 if f64 else lk_level
        u = f(Tpyr[l], Mpyr[l], u, radius, iters, lam)
    return u


def hom_valid(h, x, y, W, H):
    h = np.ascontiguousarray(h, np.float32).reshape(9)
    u, v = C.c_float(), C.c_float()
    ok = lib().vso_hom_valid(_ptr(h), float(x), float(y), W, H, C.byref(u), C.byref(v))
    return bool(ok), u.value, v.value


def bilinear(F, ch, u, v) -> float:
    F = np.ascontiguousarray(F, np.uint8)
    return lib().vso_bilinear(_ptr(F), F.shape[1] * 3, F.shape[1], F.shape[0], ch, u, v)


def luma(r, g, b) -> int:
    return int(lib().vso_luma(int(r), int(g), int(b)))


def chain_colour(Mpair) -> np.ndarray:
    """Eq. (4) chained to camera 0: Mpair [n_cams - 1][3][3] -> Mk [n_cams][3][3] (FP64)."""
    Mp = np.ascontiguousarray(Mpair, dtype=np.float64).reshape(-1, 9)
    n = Mp.shape[0] + 1
    out = np.zeros((n, 9), np.float64)
    lib().vso_chain_colour(_ptr(Mp), n, _ptr(out))
    return out.reshape(n, 3, 3)


def fuse_pixel(frame_j, hinv_j, M_j, X_j, frame_i, hinv_i, M_i, X_i, y, f_ij, f_ji, literal=False) -> np.ndarray:
    """Eqs. (16)-(18) at one canvas pixel covered by cameras j (left) and i
    (right); literal: eq. (17) as printed."""
    keep = []

    def view(F, h, M, X):
        F = np.ascontiguousarray(F, dtype=np.uint8)
        h = np.ascontiguousarray(h, dtype=np.float32).ravel()
        M = np.ascontiguousarray(M, dtype=np.float32).ravel()
        keep.extend([F, h, M])
        return View(F.ctypes.data, F.shape[1] * 3, F.shape[1], F.shape[0], h.ctypes.data, M.ctypes.data,
                    float(X))

    vj = view(frame_j, hinv_j, M_j, X_j)
    vi = view(frame_i, hinv_i, M_i, X_i)
    fij = np.asarray(f_ij, np.float32)
    fji = np.asarray(f_ji, np.float32)
    out = np.zeros(3, np.uint8)
    fn = lib().vso_fuse_pixel_literal if literal else lib().vso_fuse_pixel
    fn(C.byref(vj), C.byref(vi), float(y), _ptr(fij), _ptr(fji), _ptr(out))
    return out


def round8(r) -> int:
    return lib().vso_round8(float(r))


# ---- learned surrogate: FP64 convolution references -----------------------

def conv3x3(x, wt, b=None):
    """x (n, h, w, cin), wt (cout, 9, cin), b (cout,) -> (n, h, w, cout), float64"""
    x = np.ascontiguousarray(x, np.float64)
    wt = np.ascontiguousarray(wt, np.float64)
    n, h, w, cin = x.shape
    cout = wt.shape[0]
    y = np.zeros((n, h, w, cout), np.float64)
    bb = None if b is None else np.ascontiguousarray(b, np.float64)
    lib().vso_conv3x3(_ptr(x), n, h, w, cin, _ptr(wt), None if bb is None else _ptr(bb), cout, _ptr(y))
    return y


def conv3x3_bwd_data(dy, wt):
    dy = np.ascontiguousarray(dy, np.float64)
    wt = np.ascontiguousarray(wt, np.float64)
    n, h, w, cout = dy.shape
    cin = wt.shape[2]
    dx = np.zeros((n, h, w, cin), np.float64)
    lib().vso_conv3x3_bwd_data(_ptr(dy), n, h, w, cout, _ptr(wt), cin, _ptr(dx))
    return dx


def conv3x3_bwd_weight(x, dy):
    x = np.ascontiguousarray(x, np.float64)
    dy = np.ascontiguousarray(dy, np.float64)
    n, h, w, cin = x.shape
    cout = dy.shape[3]
    dw = np.zeros((cout, 9, cin), np.float64)
    db = np.zeros(cout, np.float64)
    lib().vso_conv3x3_bwd_weight(_ptr(x), _ptr(dy), n, h, w, cin, cout, _ptr(dw), _ptr(db))
    return dw, db


# ---- learned surrogate inside the frame ------------------------------------

def surrogate_net(blob: bytes, yt, ym) -> np.ndarray:
    """the network on one luma pair (h, w) -> channels 0-1 of its output (h, w, 2)"""
    yt = np.ascontiguousarray(yt, np.float32)
    ym = np.ascontiguousarray(ym, np.float32)
    h, w = yt.shape
    out = np.zeros((h, w, 2), np.float32)
    buf = C.create_string_buffer(bytes(blob), len(blob))
    if lib().vso_surrogate_net(buf, len(blob), _ptr(yt), _ptr(ym), w, h, _ptr(out)) != 0:
        raise OracleError("vso_surrogate_net: bad weight file")
    return out


def surr_upsample(pred, need0) -> np.ndarray:
    pred = np.ascontiguousarray(pred, np.float32)
    need0 = np.ascontiguousarray(need0, np.uint8)
    h0, w0 = need0.shape
    out = np.zeros((h0, w0, 2), np.float32)
    lib().vso_surr_upsample(_ptr(pred), pred.shape[1], pred.shape[0], _ptr(need0), w0, h0, _ptr(out))
    return out


def fb_check(pred_ij, pred_ji, need0):
    """(sum of the per-pixel forward-backward errors in 1/256 px, pixel count)"""
    a = np.ascontiguousarray(pred_ij, np.float32)
    b = np.ascontiguousarray(pred_ji, np.float32)
    need0 = np.ascontiguousarray(need0, np.uint8)
    s, n = C.c_ulonglong(), C.c_ulonglong()
    lib().vso_fb_check(_ptr(a), _ptr(b), a.shape[1], a.shape[0], _ptr(need0), need0.shape[1], need0.shape[0],
                       C.byref(s), C.byref(n))
    return s.value, n.value


# ---- learned surrogate: FP64 training step of the whole network -----------

def nn_train_step(ws, bs, x, label, sizes, alpha):
    """One training step's forward and backward in FP64: a chain of 3x3
    convolutions (weights ws[l] (cout, 9, cin), biases bs[l]) with leaky ReLU
    (slope alpha) after every layer but the last, on the images of `sizes`
    ((h, w) each) stored back to back in x (pixels, cin0); the loss is the mean
    over all pixels of the end-point error sqrt(dx^2 + dy^2 + 1e-6) of output
    channels 0-1 against label (pixels, 2).  Returns (loss, pred (pixels,
    cout), [dL/dw], [dL/db])."""
    x = np.asarray(x, np.float64)
    label = np.asarray(label, np.float64)
    P = x.shape[0]
    offs = np.cumsum([0] + [h * w for h, w in sizes])

    def per_image(a):
        return [a[offs[i]:offs[i + 1]].reshape(1, h, w, a.shape[1]) for i, (h, w) in enumerate(sizes)]

    def join(parts):
        return np.concatenate([p.reshape(-1, p.shape[-1]) for p in parts])

    L = len(ws)
    hs, zs = [x], []
    for li in range(L):
        z = join([conv3x3(a, ws[li], bs[li]) for a in per_image(hs[-1])])
        zs.append(z)
        hs.append(z if li == L - 1 else np.where(z > 0, z, alpha * z))
    pred = hs[-1]
    d = pred[:, :2] - label
    e = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2 + 1e-6)
    loss = float(e.mean())
    dz = np.zeros_like(pred)
    dz[:, :2] = d / e[:, None] / P
    gw, gb = [None] * L, [None] * L
    for li in range(L - 1, -1, -1):
        gw[li] = np.zeros_like(np.asarray(ws[li], np.float64))
        gb[li] = np.zeros(np.asarray(ws[li]).shape[0])
        for a, g in zip(per_image(hs[li]), per_image(dz)):
            dw, db = conv3x3_bwd_weight(a, g)
            gw[li] += dw
            gb[li] += db
        if li == 0:
            break
        dh = join([conv3x3_bwd_data(g, ws[li]) for g in per_image(dz)])
        dz = np.where(zs[li - 1] > 0, dh, alpha * dh)
    return loss, pred, gw, gb


# ---- section 3.1 set-up: calibration homographies and their revision --------

def _d9(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).reshape(9))


def calib_intrinsics(f, dx, dy, cx, cy, u0, v0) -> np.ndarray:
    K = np.zeros(9)
    lib().vso_calib_intrinsics(*(C.c_double(v) for v in (f, dx, dy, cx, cy, u0, v0)), _ptr(K))
    return K.reshape(3, 3)


def calib_plane_homography(K, R, t) -> np.ndarray:
    H = np.zeros(9)
    tt = np.ascontiguousarray(np.asarray(t, np.float64).reshape(3))
    Kd, Rd = _d9(K), _d9(R)
    lib().vso_calib_plane_homography(_ptr(Kd), _ptr(Rd), _ptr(tt), _ptr(H))
    return H.reshape(3, 3)


def calib_pair(Ha, Hb) -> np.ndarray:
    H = np.zeros(9)
    a, b = _d9(Ha), _d9(Hb)
    if lib().vso_calib_pair(_ptr(a), _ptr(b), _ptr(H)) != 0:
        raise OracleError("singular homography")
    return H.reshape(3, 3)


def calib_refine(H, p) -> np.ndarray:
    out = np.zeros(9)
    h = _d9(H)
    pp = np.ascontiguousarray(np.asarray(p, np.float64).reshape(4))
    lib().vso_calib_refine(_ptr(h), _ptr(pp), _ptr(out))
    return out.reshape(3, 3)


def calib_harris(Y, x, y) -> float:
    Y = np.ascontiguousarray(Y, np.float32)
    return float(lib().vso_calib_harris(_ptr(Y), Y.shape[1], x, y))


def calib_ncc(A, xa, ya, B, xb, yb) -> float:
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    return float(lib().vso_calib_ncc(_ptr(A), A.shape[1], xa, ya, _ptr(B), B.shape[1], xb, yb))


def calib_estimate(frame_a, frame_b, H, margin=16, radius=4):
    """((tx, ty, sx, sy), matches, inliers) or None"""
    Fa = np.ascontiguousarray(frame_a, np.uint8)
    Fb = np.ascontiguousarray(frame_b, np.uint8)
    h = _d9(H)
    out = np.zeros(4)
    nm, ni = C.c_int(), C.c_int()
    st = lib().vso_calib_estimate(_ptr(Fa), Fa.shape[1] * 3, Fa.shape[1], Fa.shape[0], _ptr(Fb), Fb.shape[1] * 3,
                                  Fb.shape[1], Fb.shape[0], _ptr(h), margin, radius, _ptr(out), C.byref(nm),
                                  C.byref(ni))
    return (out, nm.value, ni.value) if st == 0 else (None, nm.value, ni.value)


# ---- the variational flow alternative (vso_var.c) ---------------------------

def var_level(T, Mv, flow0=None, need=None, alpha=128.0, gamma=16.0, outer=3, inner=10) -> np.ndarray:
    """one level of the variational estimator from flow0 (zeros if None)"""
    T = np.ascontiguousarray(T, np.float32)
    Mv = np.ascontiguousarray(Mv, np.float32)
    h, w = T.shape
    f = np.zeros((h, w, 2), np.float32) if flow0 is None else np.array(flow0, np.float32, copy=True, order="C")
    nd = None if need is None else np.ascontiguousarray(need, np.uint8)
    lib().vso_var_level(_ptr(T), _ptr(Mv), None if nd is None else _ptr(nd), w, h, alpha, gamma, outer, inner, _ptr(f))
    return f


def var_pyramid(T, Mv, levels=4, alpha=128.0, gamma=16.0, outer=3, inner=10) -> np.ndarray:
    """coarse-to-fine variational flow of template T vs moving Mv (whole images)"""
    Tp, Mp = [np.ascontiguousarray(T, np.float32)], [np.ascontiguousarray(Mv, np.float32)]
    for _ in range(levels - 1):
        Tp.append(pyr_down(Tp[-1]))
        Mp.append(pyr_down(Mp[-1]))
    h, w = Tp[0].shape
    out = np.zeros((h, w, 2), np.float32)
    PA = C.c_void_p * levels
    ws = (C.c_int * levels)(*[t.shape[1] for t in Tp])
    hs = (C.c_int * levels)(*[t.shape[0] for t in Tp])
    lib().vso_var_pyramid(PA(*[t.ctypes.data for t in Tp]), PA(*[m.ctypes.data for m in Mp]), None, ws, hs, levels,
                          alpha, gamma, outer, inner, _ptr(out))
    return out
