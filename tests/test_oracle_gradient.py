"""Pins of the oracle's hand-written adjoint and descent updates (CPU)."""
import math

import numpy as np
import pytest

import jtfs_inputs as ji
from oracle import descent, fftroute
from oracle.plan import make_plan

TINY = (512, 4, 4, 1, 2, 1, 5, 2)
TINY_B = (384, 4, 3, 2, 2, 2, 4, 3)
CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4)


def _energy(plan, S_x):
    def E(y):
        d = fftroute.forward(plan, y) - S_x
        return float(np.dot(d, d))
    return E


@pytest.mark.parametrize("args", [TINY, TINY_B])
def test_gradient_matches_central_differences(args):
    p = make_plan(*args)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.N)
    y = rng.standard_normal(p.N)
    S_x = fftroute.forward(p, x)
    S_y, cache = fftroute.forward(p, y, return_cache=True)
    _, dS = descent.loss_and_grad_S(S_y, S_x)
    g = fftroute.backward(p, y, dS, cache=cache)
    E = _energy(p, S_x)
    h = 1e-5 * math.sqrt(np.mean(y * y))
    for i in rng.choice(p.N, size=16, replace=False):
        e = np.zeros(p.N)
        e[i] = h
        fd = (E(y + e) - E(y - e)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(g)))


@pytest.mark.slow
def test_gradient_matches_central_differences_config1():
    p = make_plan(*CFG1)
    x = ji.config1_signal(0)
    y = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(p, x)
    S_y, cache = fftroute.forward(p, y, return_cache=True)
    _, dS = descent.loss_and_grad_S(S_y, S_x)
    g = fftroute.backward(p, y, dS, cache=cache)
    E = _energy(p, S_x)
    h = 1e-5 * math.sqrt(np.mean(y * y))
    rng = np.random.default_rng(4)
    for i in rng.choice(p.N, size=4, replace=False):
        e = np.zeros(p.N)
        e[i] = h
        fd = (E(y + e) - E(y - e)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(g)))


def test_filter_subsample_adjoint_dot_product():
    rng = np.random.default_rng(12)
    for L, k in [(64, 0), (64, 2), (256, 3), (32, 5)]:
        x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        y = rng.standard_normal(L >> k) + 1j * rng.standard_normal(L >> k)
        h = rng.standard_normal(L)
        lhs = np.vdot(fftroute.filt_dec(x, h, k), y)
        rhs = np.vdot(x, fftroute.filt_dec_adj(y, h, k))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # along axis 0 of a 2-D array
    x = rng.standard_normal((64, 5)) + 1j * rng.standard_normal((64, 5))
    y = rng.standard_normal((16, 5)) + 1j * rng.standard_normal((16, 5))
    h = rng.standard_normal(64)
    lhs = np.vdot(fftroute.filt_dec(x, h, 2, axis=0), y)
    rhs = np.vdot(x, fftroute.filt_dec_adj(y, h, 2, axis=0))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradient_vanishes_at_the_target():
    # Sec. 2.3: grad E(y) = 0 when S(y) = S(x); at y = x exactly.
    p = make_plan(*TINY)
    x = np.random.default_rng(13).standard_normal(p.N)
    S_x, cache = fftroute.forward(p, x, return_cache=True)
    _, dS = descent.loss_and_grad_S(S_x, S_x)
    assert np.all(fftroute.backward(p, x, dS, cache=cache) == 0.0)


@pytest.mark.parametrize("args", [TINY, TINY_B, CFG1])
def test_euler_identity(args):
    # S is positively homogeneous of degree 1, so <y, J^T dS> = <S(y), dS>.
    p = make_plan(*args)
    rng = np.random.default_rng(14)
    y = rng.standard_normal(p.N)
    S_y, cache = fftroute.forward(p, y, return_cache=True)
    dS = rng.standard_normal(p.n_coeff)
    g = fftroute.backward(p, y, dS, cache=cache)
    assert np.dot(y, g) == pytest.approx(np.dot(S_y, dS), rel=1e-10)


def test_backward_is_linear_in_dS():
    p = make_plan(*TINY_B)
    rng = np.random.default_rng(15)
    y = rng.standard_normal(p.N)
    _, cache = fftroute.forward(p, y, return_cache=True)
    a, b = rng.standard_normal(p.n_coeff), rng.standard_normal(p.n_coeff)
    ga = fftroute.backward(p, y, a, cache=cache)
    gb = fftroute.backward(p, y, b, cache=cache)
    gab = fftroute.backward(p, y, 2 * a - 3 * b, cache=cache)
    assert np.linalg.norm(gab - (2 * ga - 3 * gb)) <= 1e-12 * np.linalg.norm(gab)


# ---------------------------------------------------------------- descent updates

def test_gd_descent_decreases_loss():
    p = make_plan(*TINY)
    x = ji.config1_signal(0, n=p.N)
    S_x = fftroute.forward(p, x)
    y0 = ji.white_noise_like(x, 1)
    _, losses = descent.metamer(p, S_x, y0, descent.OptState("gd", lr=0.1), 5)
    assert all(b < a for a, b in zip(losses, losses[1:]))


def test_adam_first_step_is_a_sign_step():
    st = descent.OptState("adam", lr=0.1)
    y = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -1e-3, 2.0])
    y1, ok = descent.update(y, g, 1.0, st)
    assert ok
    assert np.allclose(y1, y - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_momentum_bold_driver_accept_and_reject():
    st = descent.OptState("momentum", lr=0.1, momentum=0.9, bold_up=1.1, bold_down=0.5)
    y0 = np.array([1.0])
    g0 = np.array([2.0])
    y1, _ = descent.update(y0, g0, 10.0, st)            # first step: accepted, mu = 0.1
    assert y1[0] == pytest.approx(1.0 - 0.2)
    y2, _ = descent.update(y1, np.array([1.0]), 9.0, st)   # E fell: mu = 0.11, u = 0.9 u - mu g
    assert st.mu == pytest.approx(0.11)
    assert y2[0] == pytest.approx(y1[0] + (0.9 * -0.2 - 0.11 * 1.0))
    y3, _ = descent.update(y2, np.array([5.0]), 12.0, st)  # E rose: back to y2's origin, mu halves
    assert st.mu == pytest.approx(0.055)
    assert y3[0] == pytest.approx(y1[0] - 0.055 * 1.0)
    assert st.E_prev == 9.0


def test_nonfinite_loss_leaves_iterate():
    st = descent.OptState("momentum")
    y = np.array([1.0, 2.0])
    y1, ok = descent.update(y, np.array([np.nan, 1.0]), float("nan"), st)
    assert not ok and np.array_equal(y1, y)


# ---------------------------------------------------------------- config 2, 64 indices

_FD = {}


def _fd_partial_loss(args):
    """E restricted to the order-1 blocks and the listed groups, at y + s h e_i (worker)."""
    from threadpoolctl import threadpool_limits
    i, s = args
    st = _FD
    y = st["y"].copy()
    y[i] += s * st["h"]
    with threadpool_limits(limits=1):
        S = fftroute.forward_partial(st["op"], y, st["n2s"], fc=st["fc"])
    m = st["mask"]
    d = S[m] - st["S_t"][m]
    return float(np.dot(d, d))


@pytest.mark.slow
def test_config2_central_differences_64_indices():
    # BASELINE config 2's gradient check at full size (N = 2^16, J = 12, Q1 = 12) on the
    # oracle: central differences at 64 random sample indices (seed 4), h = 1e-5 rms(y), of
    # E restricted to the order-1 paths and the two coarsest second-order groups (every
    # path of the first layer, order 1 and the second layer's adjoint at this size; a full
    # forward per difference would take hours on the host). A fork pool over the host
    # cores evaluates the 128 partial forwards.
    import multiprocessing as mp
    import os

    import jtfs_inputs as ji
    op = make_plan(65536, 12, 12, 2, 4, 2, 13, 24.0)
    x = ji.config2_signal(2)
    y = ji.white_noise_like(x, 3)
    n2s = [g.n2 for g in op.groups[-2:]]
    fc = fftroute.FilterCache(op)
    S_t = fftroute.forward_partial(op, x, n2s, fc=fc)
    S_y = fftroute.forward_partial(op, y, n2s, fc=fc)
    mask = ~np.isnan(S_y)
    dS = np.where(mask, 2.0 * (np.nan_to_num(S_y) - np.nan_to_num(S_t)), 0.0)
    g = fftroute.backward(op, y, dS, fc=fc)
    idx = np.random.default_rng(4).choice(op.N, 64, replace=False)
    h = 1e-5 * float(np.sqrt(np.mean(y * y)))
    _FD.update(op=op, y=y, n2s=n2s, fc=fc, S_t=S_t, mask=mask, h=h)
    jobs = [(int(i), s) for i in idx for s in (+1, -1)]
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(procs) as pool:
        Es = pool.map(_fd_partial_loss, jobs)
    fd = np.array([(Es[2 * k] - Es[2 * k + 1]) / (2 * h) for k in range(len(idx))])
    gs = g[idx]
    assert np.linalg.norm(fd - gs) <= 1e-6 * np.linalg.norm(gs)
