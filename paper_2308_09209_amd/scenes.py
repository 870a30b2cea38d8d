"""Seeded synthetic multi-camera scenes: the inputs of the stitching path.

This module only *produces inputs* (camera frames, the rig's homographies and
the ground truth that generated them).  It holds none of the stitching
arithmetic: it never resamples with the stitcher's conventions, never rounds
the way the stitcher does, and is imported by both the GPU tests and the CPU
oracle tests so that the two sides see identical bytes.

Recipe (the paper's own video database is not available, so these scenes stand
in for it, with the shapes of the workloads the stitcher is measured on):

* Texture: 0.5 plus 16 sinusoids (orientation U[0, pi), wavelength
  log-uniform in [8, 128] px, phase U[0, 2 pi), per-channel amplitude
  U[0, 1/16]), min-max normalised per channel to [0, 1] over the texture
  domain, then 40 flat-coloured rectangles (sides U[16, H_tex/4], colour
  U[0,1]^3) painted in order.  In a 360-degree ring the texture is periodic in
  x: every sinusoid's x-frequency is quantised to whole cycles per ring period
  and rectangles wrap.
* Cameras: nominal crop offset x0_k = k * W * (1 - overlap).  The true
  camera-to-canvas homography is that offset composed with a perturbation about
  the frame centre: rotation U[-3, 3] deg, scale U[0.98, 1.02], translation
  U[-10, 10] px, perspective terms U[-1e-4, 1e-4].
* Residual: a smooth displacement per camera (Gaussian-smoothed white noise,
  sigma = 20 px, rescaled to a maximum magnitude of 3 px) added after the
  homography: pixel (u, v) of camera k shows texture(H_k(u, v) + d_k(u, v)).
  The stitcher is told only the homographies; the residual is what its flow
  must absorb.
* Colour: c = clip(g_k(t) * C_k @ rgb, 0, 1) ** gamma_k with C_k diagonal
  U[0.8, 1.2], off-diagonal U[-0.05, 0.05], gamma_k U[0.9, 1.1]; the exposure
  gain g_k starts at 1 and, for drifting scenes, takes a Gaussian random-walk
  step of sigma 0.01 per frame.  Stored as uint8 = floor(255 c + 0.5).
* Moving occluders (optional): flat-coloured ellipses in canvas space
  (semi-axes U[0.02, 0.06] * H, colour U[0, 1]^3) drawn over the texture until
  they cover the given fraction of the canvas, each translating at U[2, 10]
  px per frame in a direction U[0, 2 pi) (wrapping around the canvas); every
  camera sees them where it sees the canvas point, so overlapping views agree.
* Seeds: seed = 1000 * config + 10 * stream + camera (camera-level draws);
  the texture uses seed = 1000 * config + 10 * stream + 9, the occluders
  1000 * config + 10 * stream + 8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter

# Workloads, by what they are.  "frames" is the sequence length the workload is
# quoted on; the generator produces any number of frames.
WORKLOADS = {
    "2x640x360_chain": dict(config=1, n_cams=2, W=640, H=360, overlap=0.30, ring=False,
                            tex_w=1200, tex_h=400, frames=8, drift=0.0, resid=3.0),
    "4x1920x1080_ring": dict(config=2, n_cams=4, W=1920, H=1080, overlap=0.20, ring=True,
                             tex_w=None, tex_h=1200, frames=60, drift=0.01, resid=3.0),
    "8x3840x2160_ring": dict(config=5, n_cams=8, W=3840, H=2160, overlap=0.20, ring=True,
                             tex_w=None, tex_h=2400, frames=30, drift=0.01, resid=3.0, occluders=0.05),
}


def _rot_scale_persp(theta, s, tx, ty, p1, p2):
    c, si = math.cos(theta), math.sin(theta)
    return np.array([[s * c, -s * si, tx],
                     [s * si, s * c, ty],
                     [p1, p2, 1.0]], dtype=np.float64)


def _translate(tx, ty):
    return np.array([[1.0, 0.0, tx], [0.0, 1.0, ty], [0.0, 0.0, 1.0]], dtype=np.float64)


class Texture:
    """Analytic texture: evaluable at any real canvas coordinate."""

    def __init__(self, rng: np.random.Generator, x_lo: float, x_hi: float, y_lo: float,
                 y_hi: float, period: float | None):
        self.period = period
        theta = rng.uniform(0.0, math.pi, 16)
        lam = np.exp(rng.uniform(math.log(8.0), math.log(128.0), 16))
        self.phase = rng.uniform(0.0, 2.0 * math.pi, 16)
        self.amp = rng.uniform(0.0, 1.0 / 16.0, (16, 3))
        kx = 2.0 * math.pi * np.cos(theta) / lam
        ky = 2.0 * math.pi * np.sin(theta) / lam
        if period is not None:
            cycles = np.round(kx * period / (2.0 * math.pi))
            kx = cycles * 2.0 * math.pi / period
        self.kx, self.ky = kx, ky
        # per-channel min-max over the texture domain (2 px grid)
        gx = np.arange(x_lo, x_hi, 2.0)
        gy = np.arange(y_lo, y_hi, 2.0)
        lo = np.full(3, np.inf)
        hi = np.full(3, -np.inf)
        for y0 in range(0, len(gy), 64):
            X, Y = np.meshgrid(gx, gy[y0:y0 + 64])
            v = self._sines(X.ravel(), Y.ravel())
            lo = np.minimum(lo, v.min(axis=0))
            hi = np.maximum(hi, v.max(axis=0))
        self.lo, self.hi = lo, hi
        tex_h = y_hi - y_lo
        self.rects = []
        for _ in range(40):
            w = rng.uniform(16.0, tex_h / 4.0)
            h = rng.uniform(16.0, tex_h / 4.0)
            x0 = rng.uniform(x_lo, x_hi)
            y0 = rng.uniform(y_lo, y_hi)
            col = rng.uniform(0.0, 1.0, 3)
            self.rects.append((x0, y0, w, h, col))

    def _sines(self, X, Y):
        ph = np.outer(X, self.kx) + np.outer(Y, self.ky) + self.phase
        return 0.5 + np.sin(ph) @ self.amp

    def __call__(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        shape = X.shape
        X = X.ravel()
        Y = Y.ravel()
        out = np.clip((self._sines(X, Y) - self.lo) / (self.hi - self.lo), 0.0, 1.0)
        for (x0, y0, w, h, col) in self.rects:
            dx = X - x0
            if self.period is not None:
                dx = np.mod(dx, self.period)
            inside = (dx >= 0.0) & (dx < w) & (Y >= y0) & (Y < y0 + h)
            out[inside] = col
        return out.reshape(shape + (3,))


@dataclass
class Camera:
    H_true: np.ndarray          # camera pixel -> canvas, float64 3x3
    resid: np.ndarray           # (H, W, 2) canvas-unit residual displacement
    C: np.ndarray               # 3x3 colour matrix (column-vector convention)
    gamma: float
    gains: list = field(default_factory=list)   # exposure gain per frame index


class Scene:
    """One camera rig looking at one analytic texture.

    ``rig()`` gives what the stitcher is told (pairwise homographies, camera 0
    to canvas, canvas size, ring period); ``frames(t)`` gives the uint8 HWC
    frames of time step t.
    """

    def __init__(self, n_cams: int, W: int, H: int, overlap: float, ring: bool,
                 tex_h: int, tex_w: int | None = None, drift: float = 0.0,
                 resid: float = 3.0, config: int = 0, stream: int = 0,
                 perturb: bool = True, colour: bool = True, occluders: float = 0.0):
        self.n_cams, self.W, self.H, self.ring = n_cams, W, H, ring
        self.step = int(round(W * (1.0 - overlap)))
        if ring:
            self.canvas_w = n_cams * self.step
            self.period = self.canvas_w
        else:
            self.canvas_w = W + (n_cams - 1) * self.step
            self.period = None
        self.canvas_h = H
        self.drift = drift
        base = 1000 * config + 10 * stream
        trng = np.random.default_rng(base + 9)
        my = (tex_h - H) / 2.0
        if ring:
            x_lo, x_hi = 0.0, float(self.canvas_w)
        else:
            tw = tex_w if tex_w is not None else self.canvas_w
            mx = (tw - self.canvas_w) / 2.0
            x_lo, x_hi = -mx, self.canvas_w + mx
        self.texture = Texture(trng, x_lo, x_hi, -my, H + my, self.period)
        self.cams: list[Camera] = []
        cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
        for k in range(n_cams):
            rng = np.random.default_rng(base + k)
            th = math.radians(rng.uniform(-3.0, 3.0))
            s = rng.uniform(0.98, 1.02)
            tx, ty = rng.uniform(-10.0, 10.0, 2)
            p1, p2 = rng.uniform(-1e-4, 1e-4, 2)
            if not perturb:
                th, s, tx, ty, p1, p2 = 0.0, 1.0, 0.0, 0.0, 0.0, 0.0
            P = _rot_scale_persp(th, s, tx, ty, p1, p2)
            Hk = _translate(k * self.step, 0.0) @ _translate(cx, cy) @ P @ _translate(-cx, -cy)
            Hk = Hk / Hk[2, 2]
            noise = rng.standard_normal((2, H, W))
            d = np.stack([gaussian_filter(noise[0], 20.0, mode="reflect"),
                          gaussian_filter(noise[1], 20.0, mode="reflect")], axis=-1)
            mag = np.sqrt((d ** 2).sum(-1)).max()
            d = d * (resid / mag) if (resid > 0 and mag > 0) else np.zeros_like(d)
            if colour:
                C = np.diag(rng.uniform(0.8, 1.2, 3))
                off = rng.uniform(-0.05, 0.05, (3, 3))
                C = C + off * (1.0 - np.eye(3))
                gamma = float(rng.uniform(0.9, 1.1))
            else:
                C, gamma = np.eye(3), 1.0
            cam = Camera(H_true=Hk, resid=d, C=C, gamma=gamma, gains=[1.0])
            cam._rng = rng  # drift draws continue this camera's stream
            self.cams.append(cam)
        self._base_rgb: list[np.ndarray | None] = [None] * n_cams
        # moving occluders: (cx, cy, a, b, vx, vy, colour) in canvas pixels
        self.occ = []
        if occluders > 0:
            orng = np.random.default_rng(base + 8)
            area, covered = occluders * self.canvas_w * self.canvas_h, 0.0
            while covered < area:
                a, b = orng.uniform(0.02, 0.06, 2) * H
                cxo, cyo = orng.uniform(0.0, self.canvas_w), orng.uniform(0.0, H)
                speed, ang = orng.uniform(2.0, 10.0), orng.uniform(0.0, 2.0 * math.pi)
                col = orng.uniform(0.0, 1.0, 3)
                self.occ.append((cxo, cyo, a, b, speed * math.cos(ang), speed * math.sin(ang), col))
                covered += math.pi * a * b

    # --- what the stitcher is told ---------------------------------------
    def rig(self) -> dict:
        Hs = [c.H_true for c in self.cams]
        H_pair = [np.eye(3)]  # entry 0 unused
        for k in range(1, self.n_cams):
            Hp = np.linalg.inv(Hs[k - 1]) @ Hs[k]
            H_pair.append(Hp / Hp[2, 2])
        return dict(n_cams=self.n_cams, W=self.W, H=self.H, ring=int(self.ring),
                    ring_period=int(self.period or 0), canvas_w=self.canvas_w,
                    canvas_h=self.canvas_h, H_pair=H_pair, H_ref=Hs[0].copy())

    # --- frames -----------------------------------------------------------
    def base_rgb(self, k: int) -> np.ndarray:
        if self._base_rgb[k] is None:
            cam = self.cams[k]
            out = np.empty((self.H, self.W, 3), dtype=np.float64)
            us = np.arange(self.W, dtype=np.float64)
            h = cam.H_true
            for v0 in range(0, self.H, 64):
                vs = np.arange(v0, min(v0 + 64, self.H), dtype=np.float64)
                U, V = np.meshgrid(us, vs)
                w = h[2, 0] * U + h[2, 1] * V + h[2, 2]
                X = (h[0, 0] * U + h[0, 1] * V + h[0, 2]) / w
                Y = (h[1, 0] * U + h[1, 1] * V + h[1, 2]) / w
                d = cam.resid[v0:v0 + len(vs)]
                out[v0:v0 + len(vs)] = self.texture(X + d[..., 0], Y + d[..., 1])
            self._base_rgb[k] = out
        return self._base_rgb[k]

    def gain(self, k: int, t: int) -> float:
        cam = self.cams[k]
        while len(cam.gains) <= t:
            step = cam._rng.normal(0.0, self.drift) if self.drift > 0 else 0.0
            cam.gains.append(cam.gains[-1] + step)
        return cam.gains[t]

    def _paint_occluders(self, k: int, t: int, rgb: np.ndarray) -> None:
        """draw frame t's occluders into camera k's linear RGB image"""
        h = self.cams[k].H_true
        hinv = np.linalg.inv(h)
        d = self.cams[k].resid
        m = 4.0   # margin for the residual displacement (<= 3 px)
        for (cx0, cy0, a, b, vx, vy, col) in self.occ:
            cy = np.mod(cy0 + vy * t, self.canvas_h)
            cx = np.mod(cx0 + vx * t, self.canvas_w)
            for sh in (-self.canvas_w, 0.0, self.canvas_w):   # occluders wrap around the canvas
                ex = cx + sh
                cx_c = np.array([ex - a - m, ex + a + m, ex - a - m, ex + a + m])
                cy_c = np.array([cy - b - m, cy - b - m, cy + b + m, cy + b + m])
                w = hinv[2, 0] * cx_c + hinv[2, 1] * cy_c + hinv[2, 2]
                if np.any(w <= 0):
                    continue
                u = (hinv[0, 0] * cx_c + hinv[0, 1] * cy_c + hinv[0, 2]) / w
                v = (hinv[1, 0] * cx_c + hinv[1, 1] * cy_c + hinv[1, 2]) / w
                u0, u1 = max(0, int(np.floor(u.min())) - 2), min(self.W - 1, int(np.ceil(u.max())) + 2)
                v0, v1 = max(0, int(np.floor(v.min())) - 2), min(self.H - 1, int(np.ceil(v.max())) + 2)
                if u0 > u1 or v0 > v1:
                    continue
                U, V = np.meshgrid(np.arange(u0, u1 + 1, dtype=np.float64), np.arange(v0, v1 + 1, dtype=np.float64))
                ww = h[2, 0] * U + h[2, 1] * V + h[2, 2]
                X = (h[0, 0] * U + h[0, 1] * V + h[0, 2]) / ww + d[v0:v1 + 1, u0:u1 + 1, 0]
                Y = (h[1, 0] * U + h[1, 1] * V + h[1, 2]) / ww + d[v0:v1 + 1, u0:u1 + 1, 1]
                inside = ((X - ex) / a) ** 2 + ((Y - cy) / b) ** 2 <= 1.0
                if inside.any():
                    sub_img = rgb[v0:v1 + 1, u0:u1 + 1]
                    sub_img[inside] = col

    def frame(self, k: int, t: int) -> np.ndarray:
        cam = self.cams[k]
        rgb = self.base_rgb(k)
        if self.occ:
            rgb = rgb.copy()
            self._paint_occluders(k, t, rgb)
        c = np.clip(self.gain(k, t) * (rgb @ cam.C.T), 0.0, 1.0) ** cam.gamma
        return np.floor(255.0 * c + 0.5).astype(np.uint8)

    def frames(self, t: int) -> list[np.ndarray]:
        return [self.frame(k, t) for k in range(self.n_cams)]

    def truth(self, t: int, ref: int = 0) -> np.ndarray:
        """The panorama an ideal stitch would give at time t: the texture at
        every canvas pixel (canvas coordinates are texture coordinates; no
        residual displacement; occluders drawn where they are at t) through
        camera `ref`'s colour response of frame t, as uint8 HWC.  Colour
        correction chained to camera 0 aims at ref = 0."""
        cam = self.cams[ref]
        out = np.empty((self.canvas_h, self.canvas_w, 3), dtype=np.uint8)
        xs = np.arange(self.canvas_w, dtype=np.float64)
        for y0 in range(0, self.canvas_h, 64):
            ys = np.arange(y0, min(y0 + 64, self.canvas_h), dtype=np.float64)
            X, Y = np.meshgrid(xs, ys)
            rgb = self.texture(X, Y)
            for (cx0, cy0, a, b, vx, vy, col) in self.occ:
                cy = np.mod(cy0 + vy * t, self.canvas_h)
                cx = np.mod(cx0 + vx * t, self.canvas_w)
                for sh in (-self.canvas_w, 0.0, self.canvas_w):
                    inside = ((X - (cx + sh)) / a) ** 2 + ((Y - cy) / b) ** 2 <= 1.0
                    rgb[inside] = col
            c = np.clip(self.gain(ref, t) * (rgb @ cam.C.T), 0.0, 1.0) ** cam.gamma
            out[y0:y0 + len(ys)] = np.floor(255.0 * c + 0.5).astype(np.uint8)
        return out


# Six uneven streams stitched together (3 or 4 cameras, 20 % overlap chains).
BATCH_STREAMS = [
    dict(n_cams=3, W=1280, H=720), dict(n_cams=4, W=1280, H=720),
    dict(n_cams=3, W=1920, H=1080), dict(n_cams=4, W=1920, H=1080),
    dict(n_cams=3, W=2560, H=1440), dict(n_cams=4, W=2560, H=1440),
]


def batch_scenes(streams=None, config: int = 3) -> list:
    """The 6-stream batched workload: one Scene per stream (chain, 20 % overlap,
    exposure drift 0.01 per frame), seeds 1000 * config + 10 * stream + camera."""
    out = []
    for i, spec in enumerate(streams or BATCH_STREAMS):
        out.append(Scene(n_cams=spec["n_cams"], W=spec["W"], H=spec["H"], overlap=0.20, ring=False,
                         tex_h=int(round(spec["H"] * 10 / 9)), tex_w=None, drift=0.01, resid=3.0,
                         config=config, stream=i))
    return out


def scene_for(workload: str, stream: int = 0, **over) -> Scene:
    p = dict(WORKLOADS[workload])
    p.update(over)
    p.pop("frames", None)
    return Scene(n_cams=p["n_cams"], W=p["W"], H=p["H"], overlap=p["overlap"], ring=p["ring"],
                 tex_h=p["tex_h"], tex_w=p["tex_w"], drift=p["drift"], resid=p["resid"],
                 config=p["config"], stream=stream,
                 perturb=p.get("perturb", True), colour=p.get("colour", True),
                 occluders=p.get("occluders", 0.0))


def small_scene(n_cams=2, W=96, H=64, overlap=0.35, ring=False, seed_config=90, **kw) -> Scene:
    """A tiny scene with the same recipe, for parity tests that span a few tiles."""
    return Scene(n_cams=n_cams, W=W, H=H, overlap=overlap, ring=ring,
                 tex_h=int(H * 1.2), tex_w=None, config=seed_config, **kw)


# ---- synthetic weights of the learned flow surrogate ------------------------
# Weight file ("VSNN" v1): magic, u32 version, u32 layers, f32 leaky-ReLU
# slope, per layer u32 cin / u32 cout, then per layer int16 w[cout][9][cin]
# (BF16 bit patterns) and f32 bias[cout]; little endian, packed.

SURROGATE_LAYERS = ((16, 32), (32, 32), (32, 32), (32, 32), (32, 16))


def bf16_bits(x) -> np.ndarray:
    """float values -> BF16 bit patterns (round to nearest even), int16"""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def nn_blob(weights, biases, alpha: float = 0.1) -> bytes:
    """weights[l]: float [cout][9][cin] (rounded to BF16 here), biases[l]: [cout]"""
    import struct
    out = [b"VSNN", struct.pack("<IIf", 1, len(weights), alpha)]
    for w in weights:
        out.append(struct.pack("<II", w.shape[2], w.shape[0]))
    for w, b in zip(weights, biases):
        out.append(bf16_bits(w).tobytes())
        out.append(np.ascontiguousarray(b, np.float32).tobytes())
    return b"".join(out)


def random_net(seed: int, layers=SURROGATE_LAYERS, out_scale: float = 0.5, alpha: float = 0.1):
    """Seeded random weights (He-scaled normal, the last layer scaled by
    out_scale, small random biases): (weights, biases) lists."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for li, (ci, co) in enumerate(layers):
        std = math.sqrt(2.0 / (9 * ci)) * (out_scale if li == len(layers) - 1 else 1.0)
        ws.append(rng.normal(size=(co, 9, ci)) * std)
        bs.append(rng.normal(size=co) * 0.05)
    return ws, bs
