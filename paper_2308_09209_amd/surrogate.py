"""Learned flow surrogate (an addition to the paper's method).

A small 3x3 convolution network, BF16 weights and activations with FP32
accumulation, that maps a template / moving luma pair at pyramid level 2 (a
quarter of the strip resolution) to the flow between them.  It is trained on
the GPU, on pairs whose flows the plain estimator of the library computes,
with every forward and backward step running in the library's matrix-core
kernels (vs_nn_* in include/vstitch.h); torch only allocates device memory.

Network: five 3x3 layers, channels 16 -> 32 -> 32 -> 32 -> 32 -> 16, leaky
ReLU (slope 0.1) after the first four; the input carries the two normalised
luma images in channels 0-1 (the other channels are 0) and the output's
channels 0-1 are the flow in level-2 pixels.  Loss: mean end-point error.
Optimiser: Adam on FP32 master weights.
"""
from __future__ import annotations

import ctypes as C
import math
import struct

import numpy as np
import torch

from . import vstitch as V

LAYERS = ((16, 32), (32, 32), (32, 32), (32, 32), (32, 16))
ALPHA = 0.1
LEVEL = 2
MAGIC = b"VSNN"
VERSION = 1


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    def __init__(self, seed: int = 0, device: str = "cuda"):
        self.device = device
        g = torch.Generator().manual_seed(seed)
        self.w, self.b = [], []
        for li, (ci, co) in enumerate(LAYERS):
            fan = 9 * (2 if li == 0 else ci)
            std = math.sqrt(2.0 / fan) * (0.1 if li == len(LAYERS) - 1 else 1.0)
            w = torch.randn(co, 9, ci, generator=g) * std
            if li == 0:
                w[:, :, 2:] = 0.0
            self.w.append(w.to(device).contiguous())
            self.b.append(torch.zeros(co).to(device))
        self.params = [t for pair in zip(self.w, self.b) for t in pair]
        self.m = [torch.zeros_like(t) for t in self.params]
        self.v = [torch.zeros_like(t) for t in self.params]
        self.step_n = 0
        self.w16 = [torch.empty(t.shape, dtype=torch.int16, device=device) for t in self.w]
        self.wf16 = [torch.empty((ci, 9, co), dtype=torch.int16, device=device) for (ci, co) in LAYERS]
        self.refresh()

    def refresh(self):
        """BF16 copies of the master weights and their flipped transposes."""
        for (ci, co), w, w16, wf in zip(LAYERS, self.w, self.w16, self.wf16):
            V.check(V.lib().vs_nn_to_bf16(_p(w), _p(w16), w.numel(), _s()), "to_bf16")
            V.check(V.lib().vs_nn_flip_weights(_p(w16), _p(wf), ci, co, _s()), "flip")

    # ---- forward / backward ------------------------------------------------
    def forward(self, x16, imgs):
        """x16: int16 [P, 16] packed input; returns (activations, FP32 prediction [P, 16])"""
        P = x16.shape[0]
        acts = [x16]
        h = x16
        for li, (ci, co) in enumerate(LAYERS[:-1]):
            out = torch.empty((P, co), dtype=torch.int16, device=self.device)
            V.check(V.lib().vs_nn_conv3x3(_p(h), ci, _p(self.w16[li]), _p(self.b[li]), _p(out), co,
                                          C.byref(imgs), V.CONV_LRELU, ALPHA, _s()), "conv")
            acts.append(out)
            h = out
        ci, co = LAYERS[-1]
        pred = torch.empty((P, co), dtype=torch.float32, device=self.device)
        V.check(V.lib().vs_nn_conv3x3(_p(h), ci, _p(self.w16[-1]), _p(self.b[-1]), _p(pred), co,
                                      C.byref(imgs), V.CONV_F32, ALPHA, _s()), "conv")
        return acts, pred

    def backward(self, acts, dz, imgs):
        """dz: int16 [P, 16] gradient of the loss at the output; returns FP32 grads
        in the order of self.params"""
        grads = [None] * len(self.params)
        P = dz.shape[0]
        for li in range(len(LAYERS) - 1, -1, -1):
            ci, co = LAYERS[li]
            x = acts[li]
            nbytes = V.lib().vs_nn_wgrad_scratch_bytes(ci, co, C.byref(imgs))
            scratch = torch.empty(nbytes // 4 + 1, dtype=torch.float32, device=self.device)
            dwb = torch.empty(co * 9 * ci + co, dtype=torch.float32, device=self.device)
            V.check(V.lib().vs_nn_conv3x3_wgrad(_p(x), ci, _p(dz), co, C.byref(imgs), _p(scratch),
                                                nbytes, _p(dwb), _s()), "wgrad")
            grads[2 * li] = dwb[:co * 9 * ci].view(co, 9, ci)
            grads[2 * li + 1] = dwb[co * 9 * ci:]
            if li == 0:
                break
            dh = torch.empty((P, ci), dtype=torch.int16, device=self.device)
            V.check(V.lib().vs_nn_conv3x3(_p(dz), co, _p(self.wf16[li]), None, _p(dh), ci, C.byref(imgs),
                                          V.CONV_LINEAR, ALPHA, _s()), "conv bwd data")
            dzp = torch.empty_like(dh)
            V.check(V.lib().vs_nn_lrelu_bwd(_p(dh), _p(acts[li]), _p(dzp), dh.numel(), ALPHA, _s()), "lrelu bwd")
            dz = dzp
        return grads

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_n += 1
        for t, m, v, g in zip(self.params, self.m, self.v, grads):
            g = g.contiguous()   # bound to a name: the pointer must outlive the launch
            V.check(V.lib().vs_nn_adam(_p(t), _p(m), _p(v), _p(g), None, t.numel(), lr, b1, b2,
                                       eps, self.step_n, _s()), "adam")
        self.refresh()

    # ---- persistence ---------------------------------------------------------
    def blob(self) -> bytes:
        out = [MAGIC, struct.pack("<IIf", VERSION, len(LAYERS), ALPHA)]
        for (ci, co) in LAYERS:
            out.append(struct.pack("<II", ci, co))
        for w16, b in zip(self.w16, self.b):
            out.append(w16.cpu().numpy().astype(np.int16).tobytes())
            out.append(b.cpu().numpy().astype(np.float32).tobytes())
        return b"".join(out)

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.blob())

    @classmethod
    def from_blob(cls, data: bytes, device="cuda"):
        assert data[:4] == MAGIC, "not a surrogate weight file"
        version, nl, alpha = struct.unpack_from("<IIf", data, 4)
        assert version == VERSION and nl == len(LAYERS) and abs(alpha - ALPHA) < 1e-7
        off = 16
        for (ci, co) in LAYERS:
            assert struct.unpack_from("<II", data, off) == (ci, co)
            off += 8
        net = cls(device=device)
        for li, (ci, co) in enumerate(LAYERS):
            n = co * 9 * ci
            w16 = np.frombuffer(data, np.int16, n, off).reshape(co, 9, ci)
            off += 2 * n
            b = np.frombuffer(data, np.float32, co, off)
            off += 4 * co
            w = (w16.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
            net.w[li].copy_(torch.from_numpy(w.copy()))
            net.b[li].copy_(torch.from_numpy(b.copy()))
        net.refresh()
        return net


def loss_and_grad(pred, label):
    """mean EPE of pred[:, :2] against label [P, 2] and its gradient (int16 BF16 [P, 16])"""
    P = pred.shape[0]
    dz = torch.empty((P, 16), dtype=torch.int16, device=pred.device)
    nb = (P + 255) // 256
    bl = torch.empty(nb, dtype=torch.float32, device=pred.device)
    V.check(V.lib().vs_nn_epe_loss(_p(pred), _p(label), _p(dz), _p(bl), P, _s()), "epe")
    return bl, dz


def pack(yt, ym):
    """template / moving luma (float32, any shape, same numel) -> int16 [P, 16]"""
    P = yt.numel()
    yt, ym = yt.contiguous(), ym.contiguous()   # held while the kernel is enqueued
    x = torch.empty((P, 16), dtype=torch.int16, device=yt.device)
    V.check(V.lib().vs_nn_pack_pair(_p(yt), _p(ym), _p(x), P, _s()), "pack")
    return x
