"""Learned warm start: binding of the convolutional decoder of include/jtfs.h.

The decoder maps the coefficients of one signal (c_in rows of n_frames frames) to a
waveform that seeds the metamer descent. Every step (weight casts, the transposed
convolutions, their gradients, Adam) runs in the library's HIP kernels; this module
marshals arguments, and PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List

import torch

from . import _lib as L
from .jtfs import _ptr, _require, _stream


@dataclass
class DecoderConfig:
    """Decoder shape. The default is the 8-layer decoder from 266 x 128 coefficients of
    the N = 2^16 signals at T = 2^9 (J = 6, Q1 = 8) to 65536 samples."""
    c_in: int = 266
    n_frames: int = 128
    channels: int = 128
    kernel: int = 9
    strides: List[int] = field(default_factory=lambda: [1, 4, 4, 4, 2, 2, 2, 1])
    leak: float = 0.1
    eps: float = 1e-4

    def c(self) -> L.jtfs_dec_config:
        st = (ctypes.c_int32 * L.JTFS_DEC_MAX_LAYERS)(*([0] * L.JTFS_DEC_MAX_LAYERS))
        for i, s in enumerate(self.strides):
            st[i] = s
        return L.jtfs_dec_config(self.c_in, self.n_frames, self.channels, self.kernel, len(self.strides), st,
                                 self.leak, self.eps)

    def layer_shapes(self):
        """(C_out, C_in, stride) per layer, in parameter order."""
        out, c = [], self.c_in
        for i, s in enumerate(self.strides):
            co = 1 if i == len(self.strides) - 1 else self.channels
            out.append((co, c, s))
            c = co
        return out


class Decoder:
    """A decoder description (jtfs_dec_create) sized for up to ``max_batch`` signals."""

    def __init__(self, cfg: DecoderConfig, max_batch: int = 1):
        handle = ctypes.c_void_p()
        c = cfg.c()
        L.check(L.lib().jtfs_dec_create(ctypes.byref(c), max_batch, ctypes.byref(handle)), "jtfs_dec_create")
        self._h = handle
        self._destroy = L.lib().jtfs_dec_destroy
        self.cfg = cfg
        self.max_batch = max_batch
        n_params, out_len, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        L.check(L.lib().jtfs_dec_query(self._h, ctypes.byref(n_params), ctypes.byref(out_len), ctypes.byref(ws)),
                "jtfs_dec_query")
        self.n_params = n_params.value
        self.out_len = out_len.value
        self.ws_bytes = ws.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)

    def forward(self, params: torch.Tensor, S: torch.Tensor, batch: int, y: torch.Tensor = None,
                ws: torch.Tensor = None) -> torch.Tensor:
        _require(params, self.n_params, "params")
        _require(S, batch * self.cfg.c_in * self.cfg.n_frames, "S")
        if y is None:
            y = torch.empty(batch * self.out_len, dtype=torch.float32, device=S.device)
        _require(y, batch * self.out_len, "y")
        if ws is None:
            ws = self.workspace(S.device)
        L.check(L.lib().jtfs_dec_forward(self._h, _ptr(params), _ptr(S), batch, _ptr(y), _ptr(ws), ws.numel(),
                                         _stream(S.device)), "jtfs_dec_forward")
        return y

    def backward(self, params: torch.Tensor, dy: torch.Tensor, batch: int, ws: torch.Tensor,
                 grad: torch.Tensor = None) -> torch.Tensor:
        _require(params, self.n_params, "params")
        _require(dy, batch * self.out_len, "dy")
        if grad is None:
            grad = torch.empty(self.n_params, dtype=torch.float32, device=dy.device)
        _require(grad, self.n_params, "grad")
        L.check(L.lib().jtfs_dec_backward(self._h, _ptr(params), batch, _ptr(dy), _ptr(grad), _ptr(ws), ws.numel(),
                                          _stream(dy.device)), "jtfs_dec_backward")
        return grad

    def ws_region(self, ws: torch.Tensor, layer: int, which: int) -> torch.Tensor:
        """bfloat16 view [max_batch, t_out, 128] of hidden layer `layer`'s activation
        (which = 0) or pre-activation gradient (which = 1) in ws (see jtfs_dec_ws_region)."""
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        L.check(L.lib().jtfs_dec_ws_region(self._h, layer, which, ctypes.byref(off), ctypes.byref(nb)),
                "jtfs_dec_ws_region")
        v = ws[off.value: off.value + nb.value].view(torch.bfloat16)
        return v.view(self.max_batch, -1, 128)

    def adam_step(self, params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                  lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        for t, name in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
            _require(t, self.n_params, name)
        L.check(L.lib().jtfs_dec_adam_step(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1,
                                           beta2, eps, _stream(params.device)), "jtfs_dec_adam_step")
