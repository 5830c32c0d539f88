"""Learned warm start: FP64 reference of the convolutional decoder (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The decoder is an addition to the metamer method, not part of the paper: the paper
starts every descent from noise (Sec. 2.3). It maps the coefficient vector S of a
signal, read as ``c_in`` rows of ``n_frames`` frames (every block of the output
layout holds ``n_frames`` frames per row, Sec. 3.5), to a waveform that seeds the
descent. Its definition, written out here term by term:

  input      a_0[c, f]  = log(1 + S[c, f] / eps)
  layer l    z_l[o, t]  = b_l[o] + sum_i sum_k W_l[o, i, k] * up(a_{l-1})[i, t + k - h]
             with h = (K - 1) / 2, and up() the zero-stuffing by the layer's stride s:
             up(a)[i, s u] = a[i, u], every other sample and every index outside
             [0, s T) is zero (a transposed convolution, "same" padding)
             a_l        = max(z_l, leak * z_l)          for l < L
  output     y[t]       = z_L[0, t]

Storage emulation (``quantize=True``) reproduces the rounding points of the device
path, which keeps weights, activations and activation gradients in bfloat16 and
accumulates in FP32: every weight, the input a_0, every a_l (l < L) and every
activation gradient dz_l (l < L) is rounded to bfloat16 (round to nearest even, from
the FP32 value). Sums are exact FP64 here.

The backward is the exact adjoint of the forward above (same rounding points), the
optimiser is Adam with bias correction. Pins (tests/test_oracle_decoder.py): the layer
against PyTorch's transposed convolution, the whole backward against PyTorch's
reverse mode and against finite differences, Adam against torch.optim.Adam, the
rounding against PyTorch's bfloat16 conversion.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class DecoderConfig:
    c_in: int = 266
    n_frames: int = 128
    channels: int = 128
    kernel: int = 9
    strides: list = field(default_factory=lambda: [1, 4, 4, 4, 2, 2, 2, 1])
    leak: float = 0.1
    eps: float = 1e-4

    @property
    def n_layers(self) -> int:
        return len(self.strides)

    def shapes(self):
        """(C_out, C_in, T_in, T_out) per layer."""
        out, T, c = [], self.n_frames, self.c_in
        for l, s in enumerate(self.strides):
            co = 1 if l == self.n_layers - 1 else self.channels
            out.append((co, c, T, T * s))
            T, c = T * s, co
        return out

    @property
    def out_len(self) -> int:
        return self.shapes()[-1][3]


def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 -> bfloat16 (round to nearest, ties to even) -> FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def upconv(a: np.ndarray, W: np.ndarray, b: np.ndarray, s: int) -> np.ndarray:
    """z[o, t] = b[o] + sum_{i,k} W[o, i, k] up_s(a)[i, t + k - h], t in [0, s T)."""
    C_in, T = a.shape
    K = W.shape[2]
    h = (K - 1) // 2
    xs = np.zeros((C_in, s * T + 2 * h))
    xs[:, h:h + s * T:s] = a
    z = np.repeat(b[:, None], s * T, axis=1).astype(np.float64)
    for k in range(K):
        z += W[:, :, k] @ xs[:, k:k + s * T]
    return z


def upconv_adjoint(dz: np.ndarray, a: np.ndarray, W: np.ndarray, s: int):
    """Adjoint of ``upconv`` at input a: returns (dW, db, da)."""
    C_in, T = a.shape
    K = W.shape[2]
    h = (K - 1) // 2
    xs = np.zeros((C_in, s * T + 2 * h))
    xs[:, h:h + s * T:s] = a
    dW = np.zeros_like(W, dtype=np.float64)
    dxs = np.zeros_like(xs)
    for k in range(K):
        dW[:, :, k] = dz @ xs[:, k:k + s * T].T
        dxs[:, k:k + s * T] += W[:, :, k].T @ dz
    db = dz.sum(axis=1)
    da = dxs[:, h:h + s * T:s]
    return dW, db, da


def lrelu(z: np.ndarray, leak: float) -> np.ndarray:
    return np.where(z > 0, z, leak * z)


def unpack(cfg: DecoderConfig, theta: np.ndarray):
    """Flat parameter vector -> [(W_l [C_out, C_in, K], b_l [C_out])], layer order."""
    out, o = [], 0
    for co, ci, _, _ in cfg.shapes():
        n = co * ci * cfg.kernel
        W = theta[o:o + n].reshape(co, ci, cfg.kernel)
        o += n
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def n_params(cfg: DecoderConfig) -> int:
    return sum(co * ci * cfg.kernel + co for co, ci, _, _ in cfg.shapes())


def forward(cfg: DecoderConfig, theta: np.ndarray, S: np.ndarray, quantize: bool = True):
    """Waveform y (length out_len) from one coefficient vector S; returns (y, cache)."""
    q = bf16_round if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(cfg, np.asarray(theta, dtype=np.float64))
    a = q(np.log1p(np.asarray(S, dtype=np.float64).reshape(cfg.c_in, cfg.n_frames) / cfg.eps))
    acts = [a]
    Ws = []
    for l, ((W, b), s) in enumerate(zip(layers, cfg.strides)):
        Wq = q(W)
        Ws.append(Wq)
        z = upconv(a, Wq, b, s)
        if l < cfg.n_layers - 1:
            a = q(lrelu(z, cfg.leak))
            acts.append(a)
        else:
            y = z[0]
    return y, (acts, Ws)


def backward(cfg: DecoderConfig, theta: np.ndarray, cache, dy: np.ndarray, quantize: bool = True,
             branches=None, dz_out=None):
    """Gradient of <dy, y> with respect to the flat parameter vector.

    ``branches`` (optional) gives, per hidden layer h < n_layers - 1, a boolean array of
    that layer's activation shape: True where the derivative of the leaky ReLU is taken
    as 1, False where it is the leak. By default it is the sign of the activation; a
    caller comparing with another implementation may pass that implementation's
    decisions for entries within rounding of zero. ``dz_out`` (optional list) receives
    the gradient of each hidden layer's pre-activation, index h.
    """
    q = bf16_round if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    acts, Ws = cache
    grads = [None] * cfg.n_layers
    if dz_out is not None:
        dz_out[:] = [None] * (cfg.n_layers - 1)
    dz = np.asarray(dy, dtype=np.float64)[None, :]
    for l in range(cfg.n_layers - 1, -1, -1):
        dW, db, da = upconv_adjoint(dz, acts[l], Ws[l], cfg.strides[l])
        grads[l] = (dW, db)
        if l > 0:
            # acts[l] = lrelu(z) of hidden layer l - 1: its derivative is 1 where the
            # activation is positive and leak elsewhere (a and z share their sign, leak > 0)
            up = acts[l] > 0 if branches is None else np.asarray(branches[l - 1], dtype=bool)
            dz = q(np.where(up, da, cfg.leak * da))
            if dz_out is not None:
                dz_out[l - 1] = dz
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (bias-corrected, step counter starting at 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
