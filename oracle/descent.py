"""Metamer loss and updates (oracle, FP64; Sec. 2.3).

E(y) = ||S(y) - S(x)||^2 over every order-1 and order-2 coefficient; the relative loss
is E(y) / ||S(x)||^2 (the loss relative to its value at y = 0).

Updates (one call per descent step; the loss reported is the pre-update value):
* "gd":        y <- y - lr * grad.
* "adam":      Adam with bias correction, step counter starting at 1.
* "momentum":  the paper's additive update y_{n+1} = y_n + u_n with
               u_n = m u_{n-1} - mu_n grad E(y_n) (momentum m = 0.9, mu_0 = 0.1; Sec. 2.3;
               the paper's gradient is half the negated true gradient, hence the sign) and a
               bold-driver learning rate: if E did not increase, the step is kept and mu grows
               by ``bold_up``; otherwise y returns to the last kept iterate, the momentum is
               cleared, mu shrinks by ``bold_down`` and a fresh step is taken from the kept
               iterate with its stored gradient.
A non-finite loss leaves y and the optimiser state untouched except that the momentum
buffer is cleared; the step reports it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import fftroute


def loss_and_grad_S(S_y: np.ndarray, S_x: np.ndarray, weights: np.ndarray = None):
    """E = sum w (S_y - S_x)^2 and dE/dS_y (w = 1 unless ``weights`` is given)."""
    d = S_y - S_x
    if weights is None:
        return float(np.dot(d, d)), 2.0 * d
    return float(np.dot(weights * d, d)), 2.0 * weights * d


def block_weights(plan, w0: float) -> np.ndarray:
    """Per-coefficient loss weights: w0 on the zeroth-order block, 1 elsewhere (Eqs. 5-7
    hold only the first and second orders, so the default reading is w0 = 0)."""
    w = np.ones(plan.n_coeff)
    for blk in plan.blocks:
        if blk.order == 0:
            w[blk.offset: blk.offset + blk.n_lambda * blk.n_frames] = w0
    return w


def relative_loss(E: float, S_x: np.ndarray) -> float:
    return E / float(np.dot(S_x, S_x))


@dataclass
class OptState:
    kind: str = "gd"
    lr: float = 0.1
    momentum: float = 0.9
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    bold_up: float = 1.1
    bold_down: float = 0.5
    step: int = 0
    m1: np.ndarray = None
    m2: np.ndarray = None
    u: np.ndarray = None
    y_prev: np.ndarray = None
    g_prev: np.ndarray = None
    E_prev: float = math.inf
    mu: float = field(default=None)


def update(y: np.ndarray, grad: np.ndarray, E: float, st: OptState):
    """Return (new y, finite flag). ``st`` is updated in place."""
    if not math.isfinite(E) or not np.all(np.isfinite(grad)):
        if st.u is not None:
            st.u = np.zeros_like(y)
        return y, False
    if st.kind == "gd":
        return y - st.lr * grad, True
    if st.kind == "adam":
        if st.m1 is None:
            st.m1, st.m2 = np.zeros_like(y), np.zeros_like(y)
        st.step += 1
        st.m1 = st.beta1 * st.m1 + (1.0 - st.beta1) * grad
        st.m2 = st.beta2 * st.m2 + (1.0 - st.beta2) * grad * grad
        mhat = st.m1 / (1.0 - st.beta1 ** st.step)
        vhat = st.m2 / (1.0 - st.beta2 ** st.step)
        return y - st.lr * mhat / (np.sqrt(vhat) + st.eps), True
    if st.kind == "momentum":
        if st.mu is None:
            st.mu = st.lr
        if st.u is None:
            st.u = np.zeros_like(y)
        first = st.y_prev is None
        if first or E <= st.E_prev:
            if not first:
                st.mu *= st.bold_up
            st.y_prev, st.g_prev, st.E_prev = y.copy(), grad.copy(), E
            st.u = st.momentum * st.u - st.mu * grad
            return y + st.u, True
        st.mu *= st.bold_down
        st.u = -st.mu * st.g_prev
        return st.y_prev + st.u, True
    raise ValueError(st.kind)


def metamer(plan, S_target: np.ndarray, y0: np.ndarray, st: OptState, steps: int):
    """Run ``steps`` descent steps from y0; returns (y, list of pre-update losses)."""
    y = np.asarray(y0, dtype=np.float64).copy()
    losses = []
    fc = fftroute.FilterCache(plan)
    for _ in range(steps):
        S_y, cache = fftroute.forward(plan, y, fc=fc, return_cache=True)
        E, dS = loss_and_grad_S(S_y, S_target)
        grad = fftroute.backward(plan, y, dS, cache=cache)
        losses.append(E)
        y, _ = update(y, grad, E, st)
    return y, losses
