"""Small hand-built rigs and images for the tests (inputs only)."""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter


def T(tx, ty):
    return np.array([[1.0, 0, tx], [0, 1.0, ty], [0, 0, 1.0]])


def smooth_image(h, w, seed, sigma=2.0, periodic_x=False):
    """Random smooth RGB uint8 texture with plenty of gradient."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(0, 255, (h, w, 3))
    mode = ("reflect", "wrap") if periodic_x else "reflect"
    out = np.stack([gaussian_filter(base[..., c], sigma, mode=mode) for c in range(3)], -1)
    lo, hi = out.min(), out.max()
    return np.floor((out - lo) / (hi - lo) * 250.0 + 2.5).astype(np.uint8)


def crop_rig(tex, W, H, offsets, ring_period=0):
    """Cameras that are exact integer crops of `tex` at canvas offsets.

    Canvas coordinates are texture coordinates.  For a ring the texture must
    be `ring_period` wide and the crops wrap in x.
    """
    n = len(offsets)
    frames = []
    for (ox, oy) in offsets:
        if ring_period:
            cols = np.mod(np.arange(ox, ox + W), ring_period)
            frames.append(np.ascontiguousarray(tex[oy:oy + H][:, cols]))
        else:
            frames.append(np.ascontiguousarray(tex[oy:oy + H, ox:ox + W]))
    Hk = [T(ox, oy) for (ox, oy) in offsets]
    H_pair = [np.eye(3)] + [np.linalg.inv(Hk[k - 1]) @ Hk[k] for k in range(1, n)]
    if ring_period:
        cw = ring_period
    else:
        cw = max(ox for ox, _ in offsets) + W
    rig = dict(n_cams=n, W=W, H=H, H_pair=H_pair, H_ref=Hk[0], ring=int(bool(ring_period)),
               ring_period=ring_period, canvas_w=cw, canvas_h=H)
    return rig, frames
