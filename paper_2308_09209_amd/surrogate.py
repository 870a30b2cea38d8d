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
Optimiser: Adam on FP32 master weights.  The parameters, optimiser state and
workspaces are the library's network object (vs_nn_* in include/vstitch.h).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import vstitch as V

LAYERS = ((16, 32), (32, 32), (32, 32), (32, 32), (32, 16))
ALPHA = 0.1
LEVEL = 2


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    """The network through the library's vs_nn object: parameters, Adam state
    and training workspaces live on the device and every step is a library
    call; this class only marshals arguments."""

    def __init__(self, seed: int = 0, device: str = "cuda", max_pixels: int = 1 << 19):
        self.device = device
        self.max_pixels = max_pixels
        spec = V.nn_spec(LAYERS, in_live=2, alpha=ALPHA, max_pixels=max_pixels)
        h = C.c_void_p()
        V.check(V.lib().vs_nn_create(C.byref(spec), seed, C.byref(h)), "vs_nn_create")
        self.h = h
        self.loss_sum = torch.zeros((), dtype=torch.float32, device=device)

    def close(self):
        if getattr(self, "h", None):
            V.lib().vs_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def forward(self, x16, imgs, pred=None):
        """x16: int16 [P, 16] packed input (kept by the caller until backward);
        returns the FP32 prediction [P, 16]"""
        if pred is None:
            pred = torch.empty((x16.shape[0], 16), dtype=torch.float32, device=self.device)
        V.check(V.lib().vs_nn_forward(self.h, _p(x16), C.byref(imgs), _p(pred), _s()), "vs_nn_forward")
        return pred

    def backward(self, label):
        """gradients of the mean EPE of the last forward against label [P, 2];
        returns the device sum of the pixel errors (a 0-d tensor, valid after
        the stream reaches it)"""
        V.check(V.lib().vs_nn_backward(self.h, _p(label), _p(self.loss_sum), _s()), "vs_nn_backward")
        return self.loss_sum

    def loss(self, label, out=None):
        """device sum of the last forward's pixel errors against label"""
        out = self.loss_sum if out is None else out
        V.check(V.lib().vs_nn_loss(self.h, _p(label), _p(out), _s()), "vs_nn_loss")
        return out

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        V.check(V.lib().vs_nn_adam_step(self.h, lr, b1, b2, eps, _s()), "vs_nn_adam_step")

    def params(self):
        """(FP32 parameters, gradients of the last backward): device copies,
        layer by layer w [cout][9][cin] then b [cout]"""
        n = C.c_size_t()
        V.check(V.lib().vs_nn_params(self.h, None, None, C.byref(n), None), "vs_nn_params")
        p = torch.empty(n.value, dtype=torch.float32, device=self.device)
        g = torch.empty_like(p)
        V.check(V.lib().vs_nn_params(self.h, _p(p), _p(g), None, _s()), "vs_nn_params")
        return p, g

    # ---- persistence ---------------------------------------------------------
    def blob(self) -> bytes:
        n = C.c_size_t()
        V.check(V.lib().vs_nn_save(self.h, None, 0, C.byref(n)), "vs_nn_save")
        buf = C.create_string_buffer(n.value)
        V.check(V.lib().vs_nn_save(self.h, buf, n.value, C.byref(n)), "vs_nn_save")
        return buf.raw[:n.value]

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.blob())

    @classmethod
    def from_blob(cls, data: bytes, device="cuda", max_pixels: int = 1 << 19):
        net = cls(device=device, max_pixels=max_pixels)
        buf = C.create_string_buffer(bytes(data), len(data))
        V.check(V.lib().vs_nn_load(net.h, buf, len(data)), "vs_nn_load: not a weight file of this network")
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
